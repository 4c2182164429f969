// runtime.cpp -- host side of the C-ABI in include/taco.h: index loading,
// device tables, scratch sizing and the stream-ordered launch sequence of a
// search.  No host synchronization happens inside a search: every size the
// kernels need is either known on the host (budgets, shapes) or kept on the
// device (probe lengths, histogram, candidate counts), and scratch is sized
// for the worst case of a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "build.h"
#include "kernels.h"
#include "taco.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(TC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define TC_HIP(call, what)                         \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

}  // namespace

// Scratch of tc_search_noalloc: a file-scope device array, one copy per GPU,
// held from the library's load to the end of the process.  Its name is not a
// device address in host code: each device's copy is looked up once with
// hipGetSymbolAddress (noalloc_setup) and only that pointer is used.
static __device__ __align__(256) unsigned char scratch[TC_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_ptr;  // device ordinal -> its copy of scratch

// Looks up the current device's copy of the scratch array (once per device).
int noalloc_setup(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return TC_OK;
    void *ptr = nullptr;
    TC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "looking up the static scratch array");
    if (!ptr) return fail(TC_EDEVICE, "the static scratch array has no device address");
    g_scratch_ptr[device] = static_cast<unsigned char *>(ptr);
    return TC_OK;
}

unsigned char *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// FNV-1a, 64-bit (offset basis 14695981039346656037, prime 1099511628211).
struct Fnv {
    uint64_t h = 14695981039346656037ULL;
    void add(const void *p, size_t nb) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < nb; i++) {
            h ^= c[i];
            h *= 1099511628211ULL;
        }
    }
};

struct Reader {
    FILE *f = nullptr;
    Fnv sum;
    ~Reader() {
        if (f) fclose(f);
    }
    bool read(void *dst, size_t nb) {
        if (fread(dst, 1, nb, f) != nb) return false;
        sum.add(dst, nb);
        return true;
    }
};

const char *kKernelNames[] = {"transform", "probe", "count", "select", "rerank", "topk", "recheck",
                              "count_select", "graph", "cdist", "stream"};
enum Kern {
    K_TRANSFORM = 0, K_PROBE, K_COUNT, K_SELECT, K_RERANK, K_TOPK, K_RECHECK, K_FUSED, K_GRAPH, K_CDIST,
    K_STREAM, K_COUNT_
};

struct Timing {
    int kernel;
    hipEvent_t start, stop;
    bool stopped;
};

// Everything a captured graph bakes in; a call with another key is captured again.
struct GraphKey {
    const void *Q, *kq, *alpha_dev, *ids, *dists;
    int64_t nq;
    int k, k_max;
    uint64_t alpha_bits, beta_bits;
    int precision, count_mode, W, qpw, rule, rr_blocks, cdist, list_level, count_qpw, count_nt;
    int64_t Qb, pool, slots;
    bool operator==(const GraphKey &o) const { return memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

}  // namespace

struct tc_index {
    int device = 0;
    uint64_t seed = 0;  // build seed recorded in the index file
    uint64_t ident = 0; // FNV-1a of the centroids and cell offsets (autotune cache key)
    bool tune_precision = true;  // TC_OPT_TUNE_PRECISION
    int64_t n = 0;
    int d = 0, Ns = 0, s = 0, h1 = 0, h2 = 0, l = 0, M = 0, K = 0;
    // index on the device
    float *mean = nullptr, *B = nullptr, *C1 = nullptr, *C2 = nullptr, *base = nullptr;
    uint32_t *offs = nullptr, *ids = nullptr, *off2d = nullptr;
    uint32_t *ids_enc = nullptr;  // id lists in padded 4-id groups, encoded for the tile width
    size_t ids_enc_cap = 0;       // elements allocated for ids_enc
    int W = 65536, T = 1;
    int bits = 8;  // packed-count width: 4 when Ns <= 15, else 8
    int max_lds = 65536;
    int num_cu = 1;
    bool coop = false;      // cooperative launches supported
    int fused_groups = 0;   // co-resident groups of T workgroups (0: fused path unavailable)
    int count_mode = TC_COUNT_AUTO;
    int list_level = 0;          // TC_COUNT_LIST level (0: adaptive, in *lvl)
    uint32_t *lvl = nullptr;     // adaptive list level, on the device
    uint32_t *err = nullptr;     // device error word of the fused kernel
    uint32_t *arrive = nullptr;  // [Qb] tile arrivals per query
    uint32_t *qctr = nullptr;    // [T] per-tile work-queue counters of the fused count
    uint16_t *codes = nullptr;   // [n][code_stride] cell of every point per subspace (TC_COUNT_CODES)
    uint32_t *bm = nullptr;      // [Qb][Ns][ceil(K/32)] probed-cell bitmaps (TC_COUNT_CODES)
    int64_t *Aq = nullptr;       // [Qb] per-query collision budgets (batched calls)
    int32_t *kq = nullptr;       // [Qb] per-query k, clamped
    int probe_qpw = 4;           // queries (wavefronts) per probe workgroup
    int count_qpw = 1;           // queries per counting workgroup
    int count_nt = 1024;         // threads per counting workgroup (768 or 1024)
    int rr_blocks = 32;          // re-rank workgroups per query
    // graph capture of whole calls
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    GraphKey graph_key;
    int64_t graph_captures = 0;
    // options
    int rule = TC_RULE_PRINTED;
    int64_t max_batch = 0;  // 0: automatic
    int64_t scratch_budget = int64_t(64) << 30;
    int64_t cand_slots = 0;  // TC_OPT_CANDIDATE_SLOTS (0: automatic)
    bool profile = false;
    // scratch for one batch of Qb queries; pool: candidate slots (cand,
    // cand_dist, lb), shared by the batch's queries at a call's stride
    int64_t Qb = 0;
    int64_t pool = 0;
    int64_t slots = 0;  // candidate slots per query the batches are planned for
    float *qt = nullptr;
    int32_t *cells = nullptr, *ncells = nullptr;
    int64_t *retrieved = nullptr;
    uint32_t *hist = nullptr, *cand_count = nullptr;
    int32_t *cand = nullptr;
    float *cand_dist = nullptr;
    uint32_t *sc = nullptr;  // packed collision counts, [Qb][T*W bytes]
    uint32_t *tcount = nullptr;  // [Qb][T] entries listed per tile (TC_COUNT_LIST)
    uint32_t *toff = nullptr;    // [Qb][T+1] first candidate slot per tile (TC_COUNT_LIST)
    uint32_t *tlev = nullptr;    // [Qb][T][Ns+1] listed ids per tile and level (TC_COUNT_LIST)
    int32_t *perm = nullptr;     // [Qb] order in which the count and re-rank take the queries
    int32_t *flat = nullptr;     // [Qb][Ns*K] probed cells as index rows, subspace after subspace
    uint32_t *ftot = nullptr;    // [Qb] probed cells per query
    // BF16 re-rank form (built when first selected)
    int precision = TC_FP32;
    float *mu = nullptr;         // [d] mean rounded to BF16
    uint16_t *base16 = nullptr;  // [n][d] bf16(x - mu)
    float *rowerr = nullptr;     // [n] norm of each row's BF16 error, rounded up
    uint8_t *base8 = nullptr;    // [n][d] 8-bit codes (re-rank in TC_U8)
    float4 *rmeta = nullptr;     // [n] per-row (offset, step, error bound, 0) of the codes
    bool u8_plain = false;       // every row: offset 0, step 1, error 0
    float *lb = nullptr;         // [Qb][n] lower bounds of the FP32 distances
    uint32_t *rk_count = nullptr;
    uint32_t *exact = nullptr;   // [Qb] the 8-bit bounds are the FP32 distances
    uint32_t *qinfo = nullptr;   // [Qb][d/4 + 4] per-query bytes, integrality, |q|^2
    int64_t *tau_ids = nullptr;  // [Qb][1024] top-k of the upper bounds
    float *tau_d = nullptr;
    std::vector<float> mean_host;
    // reduced-precision centroid distances (built when first selected)
    int cdist = TC_CDIST_FP32;
    int Kp = 0;                  // M rounded up to 32
    void *cT = nullptr;          // [Ns*2*l][Kp] bf16 or e4m3, block-diagonal, transposed
    float *cnorm = nullptr;      // [Ns*2*l] FP32 centroid norms
    float *csc = nullptr;        // [Ns] FP8 centroid scales
    int cT_form = TC_CDIST_FP32; // form cT currently holds
    std::vector<float> C1h, C2h; // host copies of the centroids
    float *qn = nullptr, *qsc = nullptr, *cd = nullptr;  // per-batch scratch
    uint16_t *qa = nullptr;  // [Qb][M rounded up to 32] contraction operand rows (BF16, or e4m3 bytes)
    // SC-Linear (built on first use): transformed base [n][M], subspace
    // distances [scQ][Ns][n] and per-(query, subspace) thresholds
    float *sct = nullptr, *scD = nullptr;
    uint64_t *scthr = nullptr;
    int64_t scQ = 0;
    // profiling
    std::vector<Timing> pending;
    double total_ms[K_COUNT_] = {0};
    int64_t launches[K_COUNT_] = {0};
};

namespace {

void drop_graph(tc_index *x) {
    if (x->graph_exec) (void)hipGraphExecDestroy(x->graph_exec);
    if (x->graph) (void)hipGraphDestroy(x->graph);
    x->graph_exec = nullptr;
    x->graph = nullptr;
}

void free_scratch(tc_index *x) {
    drop_graph(x);
    (void)hipFree(x->Aq);
    (void)hipFree(x->kq);
    x->Aq = nullptr;
    x->kq = nullptr;
    (void)hipFree(x->qt);
    (void)hipFree(x->cells);
    (void)hipFree(x->ncells);
    (void)hipFree(x->retrieved);
    (void)hipFree(x->hist);
    (void)hipFree(x->cand_count);
    (void)hipFree(x->cand);
    (void)hipFree(x->cand_dist);
    (void)hipFree(x->sc);
    (void)hipFree(x->arrive);
    x->arrive = nullptr;
    (void)hipFree(x->qctr);
    x->qctr = nullptr;
    (void)hipFree(x->bm);
    x->bm = nullptr;
    (void)hipFree(x->lb);
    (void)hipFree(x->rk_count);
    (void)hipFree(x->tau_ids);
    (void)hipFree(x->exact);
    x->exact = nullptr;
    (void)hipFree(x->qinfo);
    x->qinfo = nullptr;
    (void)hipFree(x->tau_d);
    (void)hipFree(x->qn);
    (void)hipFree(x->qsc);
    (void)hipFree(x->qa);
    (void)hipFree(x->cd);
    (void)hipFree(x->lvl);
    x->lvl = nullptr;
    (void)hipFree(x->tcount);
    x->tcount = nullptr;
    (void)hipFree(x->toff);
    x->toff = nullptr;
    (void)hipFree(x->tlev);
    x->tlev = nullptr;
    (void)hipFree(x->perm);
    x->perm = nullptr;
    (void)hipFree(x->flat);
    x->flat = nullptr;
    (void)hipFree(x->ftot);
    x->ftot = nullptr;
    x->qn = x->qsc = x->cd = nullptr;
    x->qa = nullptr;
    x->sc = nullptr;
    x->lb = nullptr;
    x->rk_count = nullptr;
    x->tau_ids = nullptr;
    x->tau_d = nullptr;
    x->qt = nullptr;
    x->cells = x->ncells = nullptr;
    x->retrieved = nullptr;
    x->hist = x->cand_count = nullptr;
    x->cand = nullptr;
    x->cand_dist = nullptr;
    x->Qb = 0;
}

template <typename T>
int dmalloc(T **p, size_t count, const char *what) {
    *p = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (count ? count : 1));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(TC_ENOMEM, std::string("hipMalloc failed for ") + what);
    }
    return TC_OK;
}

// Alg 5's budget R = floor(beta*n), in IEEE double, clamped to [0, n].
int64_t budget_R(int64_t n, double beta) {
    double r = std::floor(beta * double(n));
    if (r < 0.0) r = 0.0;
    if (r > double(n)) r = double(n);
    return static_cast<int64_t>(r);
}

// Candidate slots per query of a call with budget R.  Alg 5 keeps the whole
// threshold level, so |C| is about R but can reach R + that level's size
// (up to n); slots for max(slots, CAP_PER_R * R) of them, and a query with
// more is queued for the streamed top-k, whose partial lists need
// STREAM_SPLIT * k_max of them (the fixed-budget rule takes exactly
// min(R, ...)).  On mixtures with Zipf-skewed cells, one query in twenty
// has |C| above 4R at beta = 0.02 and about one in three hundred above 6R;
// the streamed path reads FP32 rows (four times the bytes of U8 codes), so
// the extra slots, which only shrink the batch, are the cheaper side.
constexpr int64_t CAP_PER_R = 8;
int64_t call_cap(int64_t n, int64_t R, int64_t slots, int k_max) {
    return std::min<int64_t>(
        n, std::max<int64_t>(std::max<int64_t>(slots, CAP_PER_R * R), int64_t(taco::STREAM_SPLIT) * k_max));
}

// Candidate slots per query of the allocated scratch (set by alloc_scratch).
int64_t plan_slots(const tc_index *x) { return x->slots; }

// The scratch plan: per query, the packed counts (which the list form also
// uses for its lists), the probed cells and `slots` candidate slots (ids and
// distances, and in the bounded re-ranks the lower bounds, which also hold
// the re-checked ids).  With TC_OPT_CANDIDATE_SLOTS = S, slots = min(S, n)
// and Qb follows from the budget.  Automatically, Qb follows from the budget
// with min(n, 65536) slots per query, up to QB_FILL queries, and the slots
// then take what the budget leaves (at most n): a query streams only when
// its candidates outgrow all of that.  QB_FILL queries already give each
// launch tens of thousands of workgroups, so a larger batch saves next to
// nothing while fewer slots send more queries to the streamed path.  The
// pool holds at least n slots, so that any beta runs (one query per batch
// at worst).
int64_t batch_for(const tc_index *x, int64_t *pool, int64_t *slots) {
    const int64_t fixed = int64_t(x->T) * x->W * x->bits / 8 + 8 * int64_t(x->Ns) * x->K;
    const int64_t bps = x->precision != TC_FP32 ? 12 : 8;  // bytes per candidate slot
    int64_t s = x->cand_slots > 0 ? std::min<int64_t>(x->cand_slots, x->n) : std::min<int64_t>(x->n, 65536);
    int64_t qb = x->scratch_budget / (fixed + bps * s);
    constexpr int64_t QB_FILL = 16384;
    int64_t cap = x->max_batch > 0 ? x->max_batch : 8192;
    if (x->cand_slots <= 0 && cap > QB_FILL) cap = QB_FILL;
    if (qb > cap) qb = cap;
    if (qb < 1) qb = 1;
    if (x->cand_slots <= 0) {
        const int64_t left = x->scratch_budget - qb * fixed;
        if (left > 0) s = std::max<int64_t>(s, std::min<int64_t>(x->n, left / (bps * qb)));
    }
    *slots = s;
    *pool = std::max<int64_t>(qb * s, x->n);
    return qb;
}

int alloc_scratch(tc_index *x) {
    free_scratch(x);
    int64_t pool = 0, slots = 0;
    const int64_t qb = batch_for(x, &pool, &slots);
    int rc;
    if ((rc = dmalloc(&x->qt, size_t(qb) * x->M, "transformed queries"))) return rc;
    if ((rc = dmalloc(&x->cells, size_t(qb) * x->Ns * x->K, "probed cells"))) return rc;
    if ((rc = dmalloc(&x->ncells, size_t(qb) * x->Ns, "probe lengths"))) return rc;
    if ((rc = dmalloc(&x->retrieved, size_t(qb) * x->Ns, "retrieved counts"))) return rc;
    if ((rc = dmalloc(&x->hist, size_t(qb) * (x->Ns + 1), "level histograms"))) return rc;
    // candidate counts [qb]; for the list selection the queue's header
    // (queued, above the level, overflowed lists) and the queue [qb]; the
    // queue of queries with more candidates than slots: length, queue [qb]
    if ((rc = dmalloc(&x->cand_count, size_t(3 * qb + 4), "candidate counts"))) return rc;
    if ((rc = dmalloc(&x->lvl, 1, "list level"))) return rc;
    if ((rc = dmalloc(&x->tcount, size_t(qb) * x->T, "per-tile list lengths"))) return rc;
    if ((rc = dmalloc(&x->toff, size_t(qb) * (x->T + 1), "per-tile candidate offsets"))) return rc;
    if ((rc = dmalloc(&x->tlev, size_t(qb) * x->T * (x->Ns + 1), "per-tile listed levels"))) return rc;
    if ((rc = dmalloc(&x->perm, size_t(qb), "query order"))) return rc;
    if ((rc = dmalloc(&x->flat, size_t(qb) * x->Ns * x->K, "probed cell rows"))) return rc;
    if ((rc = dmalloc(&x->ftot, size_t(qb), "probed cell totals"))) return rc;
    {
        const uint32_t l0 = static_cast<uint32_t>(std::min(2, x->Ns));
        TC_HIP(hipMemcpy(x->lvl, &l0, sizeof(l0), hipMemcpyHostToDevice), "list level");
    }
    if ((rc = dmalloc(&x->arrive, size_t(qb), "tile arrivals"))) return rc;
    if ((rc = dmalloc(&x->qctr, size_t(x->T), "work-queue counters"))) return rc;
    if ((rc = dmalloc(&x->bm, size_t(qb) * x->Ns * ((x->K + 31) / 32), "probed-cell bitmaps"))) return rc;
    if ((rc = dmalloc(&x->Aq, size_t(qb), "per-query budgets"))) return rc;
    if ((rc = dmalloc(&x->kq, size_t(qb), "per-query k"))) return rc;
    if ((rc = dmalloc(&x->cand, size_t(pool), "candidates"))) return rc;
    if ((rc = dmalloc(&x->cand_dist, size_t(pool), "candidate distances"))) return rc;
    if ((rc = dmalloc(&x->sc, size_t(qb) * x->T * (size_t(x->W) * x->bits / 32), "packed counts")))
        return rc;
    if ((rc = dmalloc(&x->qn, size_t(qb) * x->Ns * 2, "query half norms"))) return rc;
    if ((rc = dmalloc(&x->qsc, size_t(qb) * x->Ns, "query scales"))) return rc;
    if ((rc = dmalloc(&x->cd, size_t(qb) * x->Ns * 2 * x->l, "centroid distances"))) return rc;
    if ((rc = dmalloc(&x->qa, size_t(qb) * ((x->M + 31) / 32 * 32), "query operand rows"))) return rc;
    if (x->precision != TC_FP32) {
        if ((rc = dmalloc(&x->lb, size_t(pool), "distance lower bounds"))) return rc;
        if ((rc = dmalloc(&x->rk_count, size_t(qb), "re-check counts"))) return rc;
        if ((rc = dmalloc(&x->tau_ids, size_t(qb) * 1024, "bound top-k ids"))) return rc;
        if ((rc = dmalloc(&x->exact, size_t(qb), "exact-bound flags"))) return rc;
        if ((rc = dmalloc(&x->qinfo, size_t(qb) * (x->d / 4 + 4), "query bytes"))) return rc;
        if ((rc = dmalloc(&x->tau_d, size_t(qb) * 1024, "bound top-k"))) return rc;
    }
    x->Qb = qb;
    x->pool = pool;
    x->slots = slots;
    return TC_OK;
}

// Tiling for the tile width W: the start of every (subspace, cell, tile)
// slice of the id lists, then the padded lists the count walk reads, each
// slice rounded up to whole 4-id groups.
int build_tiles(tc_index *x) {
    x->T = static_cast<int>((x->n + x->W - 1) / x->W);
    (void)hipFree(x->off2d);
    x->off2d = nullptr;
    const size_t entries = size_t(x->Ns) * x->K * (x->T + 1);
    uint32_t *raw = nullptr;
    int rc = dmalloc(&raw, entries, "tile offsets");
    if (rc) return rc;
    std::vector<uint32_t> h(entries);
    hipError_t e = taco::launch_build_off2d(x->ids, x->offs, x->Ns, x->K, x->n, x->T, x->W, raw, nullptr);
    if (e == hipSuccess) e = hipMemcpy(h.data(), raw, entries * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        (void)hipFree(raw);
        return fail(TC_EDEVICE, std::string("building tile offsets: ") + hipGetErrorString(e));
    }
    // (first, end) group of every slice, laid out tile by tile, and the
    // table itself tile-major ([T][Ns][K]): the workgroups of one tile, which
    // the count grid places on one XCD, then read one contiguous part of the
    // lists and of the table
    const size_t slices = size_t(x->Ns) * x->K;
    std::vector<uint32_t> pr(slices * x->T * 2);
    uint64_t groups = 0;
    for (int t = 0; t < x->T; t++) {
        for (size_t jc = 0; jc < slices; jc++) {
            const size_t c = jc * (size_t(x->T) + 1);
            const uint32_t len = h[c + t + 1] - h[c + t];
            const size_t e = (size_t(t) * slices + jc) * 2;
            pr[e] = static_cast<uint32_t>(groups);
            groups += (len + 3u) / 4u;
            pr[e + 1] = static_cast<uint32_t>(groups);
        }
    }
    const size_t padded = size_t(groups) * 4;
    if (padded >= (size_t(1) << 30)) {
        (void)hipFree(raw);
        return fail(TC_EINVAL, "the padded id lists exceed 2^30 entries");
    }
    if ((rc = dmalloc(&x->off2d, pr.size(), "tile offsets"))) {
        (void)hipFree(raw);
        return rc;
    }
    if (x->ids_enc_cap < padded) {
        (void)hipFree(x->ids_enc);
        x->ids_enc = nullptr;
        x->ids_enc_cap = 0;
        if ((rc = dmalloc(&x->ids_enc, padded, "encoded id lists"))) {
            (void)hipFree(raw);
            return rc;
        }
        x->ids_enc_cap = padded;
    }
    e = hipMemcpy(x->off2d, pr.data(), pr.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = taco::launch_encode_ids(x->ids, raw, x->off2d, x->Ns, x->K, x->T, x->n, x->W, x->bits, x->ids_enc,
                                    nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(raw);
    if (e != hipSuccess) return fail(TC_EDEVICE, std::string("encoding the id lists: ") + hipGetErrorString(e));
    TC_HIP(taco::prepare_count_kernels(x->W, x->bits, x->Ns), "setting LDS size of the count kernels");
    TC_HIP(hipDeviceSynchronize(), "building tile offsets");
    // How many groups of T co-resident workgroups the fused kernel can keep:
    // three quarters of what the occupancy figures allow, so that a few
    // workgroup slots taken by anything else cannot leave its waits short
    x->fused_groups = 0;
    if (x->coop && taco::fused_lds_bytes(x->W, x->bits) <= size_t(x->max_lds)) {
        int per_cu = 0;
        TC_HIP(taco::fused_max_blocks(x->W, x->bits, x->Ns, &per_cu), "occupancy of the fused kernel");
        x->fused_groups = per_cu * x->num_cu * 3 / 4 / x->T;
    }
    return TC_OK;
}

void free_all(tc_index *x) {
    free_scratch(x);
    (void)hipFree(x->mean);
    (void)hipFree(x->B);
    (void)hipFree(x->C1);
    (void)hipFree(x->C2);
    (void)hipFree(x->base);
    (void)hipFree(x->offs);
    (void)hipFree(x->ids);
    (void)hipFree(x->off2d);
    (void)hipFree(x->ids_enc);
    (void)hipFree(x->err);
    (void)hipFree(x->mu);
    (void)hipFree(x->base16);
    (void)hipFree(x->rowerr);
    (void)hipFree(x->cT);
    (void)hipFree(x->cnorm);
    (void)hipFree(x->csc);
    (void)hipFree(x->base8);
    (void)hipFree(x->rmeta);
    (void)hipFree(x->codes);
    (void)hipFree(x->sct);
    (void)hipFree(x->scD);
    (void)hipFree(x->scthr);
    for (auto &t : x->pending) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    x->pending.clear();
    if (x->cap_stream) (void)hipStreamDestroy(x->cap_stream);
    x->cap_stream = nullptr;
}

template <typename T>
int upload(T **dst, const std::vector<T> &src, const char *what) {
    int rc = dmalloc(dst, src.size(), what);
    if (rc) return rc;
    TC_HIP(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice), what);
    return TC_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// BF16 form of the base (once): mu = the mean rounded to BF16, then the
// centred BF16 rows and their error norms on the device.
int build_bf16(tc_index *x) {
    if (x->base16) return TC_OK;
    std::vector<float> mu(x->d);
    for (int t = 0; t < x->d; t++) {
        uint32_t b;
        memcpy(&b, &x->mean_host[t], 4);
        b = ((b + 0x7fffu + ((b >> 16) & 1u)) >> 16) << 16;
        memcpy(&mu[t], &b, 4);
    }
    int rc;
    if ((rc = upload(&x->mu, mu, "BF16 centre"))) return rc;
    if ((rc = dmalloc(&x->base16, size_t(x->n) * x->d, "BF16 base"))) return rc;
    if ((rc = dmalloc(&x->rowerr, size_t(x->n), "BF16 row errors"))) return rc;
    TC_HIP(taco::launch_prep_bf16(x->base, x->n, x->d, x->mu, x->base16, x->rowerr, nullptr),
           "building the BF16 base");
    TC_HIP(hipDeviceSynchronize(), "building the BF16 base");
    return TC_OK;
}

int build_u8(tc_index *x) {
    if (x->base8) return TC_OK;
    int rc;
    if ((rc = dmalloc(&x->base8, size_t(x->n) * x->d, "8-bit base"))) return rc;
    if ((rc = dmalloc(&x->rmeta, size_t(x->n), "8-bit row records"))) return rc;
    uint32_t *plain = nullptr;
    if ((rc = dmalloc(&plain, 1, "8-bit plain flag"))) return rc;
    const uint32_t one = 1u;
    TC_HIP(hipMemcpy(plain, &one, sizeof one, hipMemcpyHostToDevice), "8-bit plain flag");
    TC_HIP(taco::launch_prep_u8(x->base, x->n, x->d, x->base8, x->rmeta, plain, nullptr),
           "building the 8-bit base");
    uint32_t got = 0u;
    TC_HIP(hipMemcpy(&got, plain, sizeof got, hipMemcpyDeviceToHost), "8-bit plain flag");
    (void)hipFree(plain);
    x->u8_plain = got != 0u;
    return TC_OK;
}

// The block-diagonal centroid matrix of the reduced-precision centroid
// distances in the given form, with FP32 norms and (FP8) one scale per
// subspace: the largest centroid magnitude of the subspace over 240.
int build_cdist(tc_index *x, int form) {
    if (x->cT && x->cT_form == form) return TC_OK;
    (void)hipFree(x->cT);
    x->cT = nullptr;
    x->Kp = (x->M + 31) / 32 * 32;
    const int ncol = x->Ns * 2 * x->l;
    std::vector<float> csc(x->Ns, 1.0f);
    for (int j = 0; j < x->Ns; j++) {
        float mx = 0.0f;
        for (int c = 0; c < x->l; c++) {
            for (int t = 0; t < x->h1; t++)
                mx = std::max(mx, std::fabs(x->C1h[(size_t(j) * x->l + c) * x->h1 + t]));
            for (int t = 0; t < x->h2; t++)
                mx = std::max(mx, std::fabs(x->C2h[(size_t(j) * x->l + c) * x->h2 + t]));
        }
        csc[j] = mx > 0.0f ? mx / 240.0f : 1.0f;
    }
    int rc;
    if (!x->csc && (rc = upload(&x->csc, csc, "centroid scales"))) return rc;
    if (!x->cnorm && (rc = dmalloc(&x->cnorm, size_t(ncol), "centroid norms"))) return rc;
    const size_t bytes = size_t(ncol) * x->Kp * (form == TC_CDIST_FP8 ? 1 : 2);
    uint8_t *ct = nullptr;
    if ((rc = dmalloc(&ct, bytes, "packed centroids"))) return rc;
    x->cT = ct;
    TC_HIP(taco::launch_prep_centroids(x->C1, x->C2, x->Ns, x->s, x->h1, x->h2, x->l, x->Kp,
                                       form == TC_CDIST_FP8, x->csc, x->cT, x->cnorm, nullptr),
           "packing the centroids");
    TC_HIP(hipDeviceSynchronize(), "packing the centroids");
    x->cT_form = form;
    return TC_OK;
}

// Shape limits the kernels rely on; fills M and K.
int check_shape(tc_index *x, int code) {
    x->M = x->Ns * x->s;
    x->K = x->l * x->l;
    if (x->n <= 0 || x->n >= (int64_t(1) << 31) || x->d <= 0 || x->Ns <= 0 || x->Ns > 16 ||
        int64_t(x->Ns) * x->n >= (int64_t(1) << 30) || x->s < 2 || x->M > x->d || x->l <= 0 ||
        x->l > 64 || x->h1 != x->s / 2 || x->h2 != x->s - x->s / 2)
        return fail(code, "index shape out of range (need n < 2^31, Ns <= 16, Ns*n < 2^30, "
                          "l <= 64, Ns*s <= d, halves s/2 and s - s/2)");
    return TC_OK;
}

// Checks the inverted lists and puts an index on the device: the arrays of
// the file layout on the host, the base rows from the host or the device.
int install(tc_index *x, int device, const std::vector<float> &mean, const std::vector<float> &B,
            const std::vector<float> &C1, const std::vector<float> &C2,
            const std::vector<uint64_t> &off64, const std::vector<uint32_t> &ids,
            const float *base_host, const float *base_dev) {
    const size_t n = size_t(x->n), d = size_t(x->d), Ns = size_t(x->Ns), K = size_t(x->K);
    // The kernels rely on these: offsets partition [0, n), ids are in range
    // and ascending inside each cell, every point appears once per subspace.
    std::vector<uint32_t> offs(Ns * (K + 1));
    std::vector<unsigned char> seen(n);
    for (size_t j = 0; j < Ns; j++) {
        const uint64_t *o = off64.data() + j * (K + 1);
        if (o[0] != 0 || o[K] != n) return fail(TC_EFORMAT, "cell offsets do not span [0, n)");
        std::fill(seen.begin(), seen.end(), 0);
        for (size_t c = 0; c < K; c++) {
            if (o[c + 1] < o[c]) return fail(TC_EFORMAT, "cell offsets decrease");
            for (uint64_t p = o[c]; p < o[c + 1]; p++) {
                const uint32_t id = ids[j * n + p];
                if (id >= n || seen[id]) return fail(TC_EFORMAT, "point id out of range or repeated");
                if (p > o[c] && ids[j * n + p - 1] >= id)
                    return fail(TC_EFORMAT, "ids not ascending inside a cell");
                seen[id] = 1;
            }
        }
        for (size_t c = 0; c <= K; c++) offs[j * (K + 1) + c] = static_cast<uint32_t>(o[c]);
    }
    {
        Fnv f;
        f.add(C1.data(), C1.size() * sizeof(float));
        f.add(C2.data(), C2.size() * sizeof(float));
        f.add(off64.data(), off64.size() * sizeof(uint64_t));
        x->ident = f.h;
    }
    int ndev = 0;
    TC_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(TC_EINVAL, "no such HIP device");
    x->device = device;
    DeviceGuard g(device);
    int rc = noalloc_setup(device);
    if (rc) return rc;
    hipDeviceProp_t prop;
    TC_HIP(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    x->max_lds = static_cast<int>(prop.sharedMemPerBlock);
    x->num_cu = prop.multiProcessorCount;
    int coop = 0;
    TC_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device),
           "hipDeviceGetAttribute");
    x->coop = coop != 0;
    if ((rc = upload(&x->mean, mean, "mean"))) return rc;
    x->mean_host = mean;
    if ((rc = upload(&x->B, B, "transform"))) return rc;
    if ((rc = upload(&x->C1, C1, "half-1 centroids"))) return rc;
    if ((rc = upload(&x->C2, C2, "half-2 centroids"))) return rc;
    x->C1h = C1;
    x->C2h = C2;
    if ((rc = upload(&x->offs, offs, "cell offsets"))) return rc;
    if ((rc = upload(&x->ids, ids, "cell ids"))) return rc;
    if ((rc = dmalloc(&x->base, n * d, "base vectors"))) return rc;
    TC_HIP(hipMemcpy(x->base, base_dev ? base_dev : base_host, sizeof(float) * n * d,
                     base_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice),
           "base vectors");
    if ((rc = dmalloc(&x->err, 1, "error word"))) return rc;
    TC_HIP(hipMemset(x->err, 0, sizeof(uint32_t)), "clearing the error word");
    // Counts are 4-bit when they cannot exceed 15.  Default tile: 64 KB of
    // packed counts (128 Ki ids as nibbles, 64 Ki as bytes), or what the
    // workgroup LDS limit allows.
    x->bits = x->Ns <= 15 ? 4 : 8;
    int W = x->bits == 4 ? 131072 : 65536;
    while (W > 1024 && taco::count_lds_bytes(W, x->bits) > size_t(x->max_lds)) W -= 1024;
    x->W = W;
    if ((rc = build_tiles(x))) return rc;
    if ((rc = alloc_scratch(x))) return rc;
    return TC_OK;
}

int load(const char *path, int device, tc_index *x) {
    Reader r;
    r.f = fopen(path, "rb");
    if (!r.f) return fail(TC_EIO, std::string("cannot open index file ") + path);
    unsigned char hdr[128];
    if (!r.read(hdr, sizeof hdr)) return fail(TC_EFORMAT, "index file shorter than its header");
    uint32_t ver, hb;
    int32_t dims[6];
    memcpy(&ver, hdr + 8, 4);
    memcpy(&hb, hdr + 12, 4);
    memcpy(&x->n, hdr + 16, 8);
    memcpy(dims, hdr + 24, 24);
    memcpy(&x->seed, hdr + 48, 8);
    if (memcmp(hdr, "TACOIDX1", 8) != 0 || ver != 1u || hb != 128u)
        return fail(TC_EFORMAT, "not a version-1 TACOIDX1 index file");
    x->d = dims[0];
    x->Ns = dims[1];
    x->s = dims[2];
    x->h1 = dims[3];
    x->h2 = dims[4];
    x->l = dims[5];
    int rc;
    if ((rc = check_shape(x, TC_EFORMAT))) return rc;
    const size_t n = size_t(x->n), d = size_t(x->d), Ns = size_t(x->Ns), l = size_t(x->l),
                 K = size_t(x->K), M = size_t(x->M);
    std::vector<float> mean(d), B(d * M), C1(Ns * l * x->h1), C2(Ns * l * x->h2);
    std::vector<uint64_t> off64(Ns * (K + 1));
    std::vector<uint32_t> ids(Ns * n);
    std::vector<float> base(n * d);
    if (!r.read(mean.data(), 4 * mean.size()) || !r.read(B.data(), 4 * B.size()) ||
        !r.read(C1.data(), 4 * C1.size()) || !r.read(C2.data(), 4 * C2.size()) ||
        !r.read(off64.data(), 8 * off64.size()) || !r.read(ids.data(), 4 * ids.size()) ||
        !r.read(base.data(), 4 * base.size()))
        return fail(TC_EFORMAT, "index file truncated");
    uint64_t want = 0;
    const uint64_t got = r.sum.h;
    if (fread(&want, 1, 8, r.f) != 8 || want != got)
        return fail(TC_EFORMAT, "index checksum mismatch");
    return install(x, device, mean, B, C1, C2, off64, ids, base.data(), nullptr);
}

void record(tc_index *x, int kern, hipStream_t st, bool begin) {
    if (!x->profile) return;
    if (begin) {
        Timing t{kern, nullptr, nullptr, false};
        if (hipEventCreate(&t.start) != hipSuccess) return;
        if (hipEventCreate(&t.stop) != hipSuccess) {
            (void)hipEventDestroy(t.start);
            return;
        }
        (void)hipEventRecord(t.start, st);
        x->pending.push_back(t);
        return;
    }
    // the latest open interval of this kernel (intervals may nest)
    for (auto it = x->pending.rbegin(); it != x->pending.rend(); ++it) {
        if (it->kernel == kern && !it->stopped) {
            (void)hipEventRecord(it->stop, st);
            it->stopped = true;
            return;
        }
    }
}

int resolve_timings(tc_index *x) {
    int rc = TC_OK;
    for (auto &t : x->pending) {
        // an interval left open (its launch failed) is dropped
        if (t.stopped && rc == TC_OK) {
            float ms = 0.0f;
            if (hipEventSynchronize(t.stop) != hipSuccess || hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess) {
                (void)hipGetLastError();
                rc = fail(TC_EDEVICE, "reading profiling events failed");
            } else {
                x->total_ms[t.kernel] += ms;
                x->launches[t.kernel] += 1;
            }
        }
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    x->pending.clear();
    return rc;
}

// One search call: uniform budgets (alpha, k) or per-query ones (alpha_dev,
// kq_dev, device arrays), results in rows of k_max.
struct Call {
    const float *Q = nullptr;
    int64_t nq = 0;
    int k = 0;
    const int32_t *kq_dev = nullptr;
    int k_max = 0;
    double alpha = 0.0;
    const double *alpha_dev = nullptr;
    double beta = 0.0;
    int64_t *ids = nullptr;
    float *dists = nullptr;
    const tc_stage_dump *dump = nullptr;
    // tc_search_noalloc: the split count form, FP32 re-rank and centroid
    // distances, no timing events, whatever the index's options; scratch
    // from `scratch` instead of the index's buffers
    bool plain = false;
    const struct Scratch *scratch = nullptr;
};

// Per-batch scratch of a call, for Qb queries: the index's own buffers, or
// views into the library's static device array (tc_search_noalloc, which
// sets only what the plain path uses and leaves the rest null).
struct Scratch {
    int64_t Qb = 0;
    int64_t pool = 0;  // candidate slots of cand, cand_dist (and lb)
    float *qt = nullptr;
    int32_t *cells = nullptr, *ncells = nullptr;
    int64_t *retrieved = nullptr;
    uint32_t *hist = nullptr, *cand_count = nullptr;
    int32_t *cand = nullptr;
    float *cand_dist = nullptr;
    uint32_t *sc = nullptr;
    int32_t *perm = nullptr, *flat = nullptr;
    uint32_t *ftot = nullptr;
    // used by the other forms only
    uint32_t *lvl = nullptr, *tcount = nullptr, *toff = nullptr, *tlev = nullptr, *arrive = nullptr;
    uint32_t *qctr = nullptr, *bm = nullptr;
    int64_t *Aq = nullptr;
    int32_t *kq = nullptr;
    float *lb = nullptr;
    uint32_t *rk_count = nullptr, *exact = nullptr, *qinfo = nullptr;
    int64_t *tau_ids = nullptr;
    float *tau_d = nullptr, *qn = nullptr, *qsc = nullptr, *cd = nullptr;
    uint16_t *qa = nullptr;
};

Scratch own_scratch(const tc_index *x) {
    Scratch S;
    S.Qb = x->Qb;
    S.pool = x->pool;
    S.qt = x->qt;
    S.cells = x->cells;
    S.ncells = x->ncells;
    S.retrieved = x->retrieved;
    S.hist = x->hist;
    S.cand_count = x->cand_count;
    S.cand = x->cand;
    S.cand_dist = x->cand_dist;
    S.sc = x->sc;
    S.perm = x->perm;
    S.flat = x->flat;
    S.ftot = x->ftot;
    S.lvl = x->lvl;
    S.tcount = x->tcount;
    S.toff = x->toff;
    S.tlev = x->tlev;
    S.arrive = x->arrive;
    S.qctr = x->qctr;
    S.bm = x->bm;
    S.Aq = x->Aq;
    S.kq = x->kq;
    S.lb = x->lb;
    S.rk_count = x->rk_count;
    S.exact = x->exact;
    S.qinfo = x->qinfo;
    S.tau_ids = x->tau_ids;
    S.tau_d = x->tau_d;
    S.qn = x->qn;
    S.qsc = x->qsc;
    S.cd = x->cd;
    S.qa = x->qa;
    return S;
}

// The launch sequence of a call, batch after batch, on stream st.  Nothing
// here waits on the host, so it can also be captured into a graph.
int enqueue(tc_index *x, const Call &c, hipStream_t st) {
    const tc_stage_dump *dump = c.dump;
    const Scratch S = c.scratch ? *c.scratch : own_scratch(x);
    const int precision = c.plain ? int(TC_FP32) : x->precision;
    const int cdist = c.plain ? int(TC_CDIST_FP32) : x->cdist;
    const int count_mode = c.plain ? int(TC_COUNT_SPLIT) : x->count_mode;
    auto rec = [&](int kern, hipStream_t s_, bool begin) {
        if (!c.plain) record(x, kern, s_, begin);
    };
    // budgets in IEEE double (Alg 4 stop test, Alg 5 budget)
    double a = std::ceil(c.alpha * double(x->n));
    if (a < 1.0) a = 1.0;
    if (a > double(x->n)) a = double(x->n);
    const int64_t A = static_cast<int64_t>(a), R = budget_R(x->n, c.beta);
    // candidate slots per query (all n with stage dumps, which hold every
    // candidate), and the queries per batch they leave
    const int64_t cap = dump ? x->n : call_cap(x->n, R, c.scratch ? S.pool / S.Qb : plan_slots(x), c.k_max);
    const int64_t Qc = std::min<int64_t>(S.Qb, S.pool / cap);
    // queries with more candidates than cap (none possible when cap = n)
    const bool stream = cap < x->n && x->rule != TC_RULE_FIXED;
    uint32_t *ovf = S.cand_count + 2 * S.Qb + 3;
    const int rr_blocks = x->rr_blocks;
    const int k = c.k, k_max = c.k_max;
    // AUTO takes the split launches: on MI355X the ~T*nq independent
    // workgroups of the split form overlap better than the fused groups'
    // lock-step rounds (10.2 vs 17.3 ms per 10k-query step at n = 1M)
    // the fixed-budget rule runs on the packed counts of the split form or
    // on the lists (the fused form takes the split launches for it)
    const bool fixed = x->rule == TC_RULE_FIXED;
    const bool fused = count_mode == TC_COUNT_FUSED && !fixed;
    const bool list = count_mode == TC_COUNT_LIST;
    const bool codes = count_mode == TC_COUNT_CODES;
    for (int64_t b0 = 0; b0 < c.nq; b0 += Qc) {
        const int nb = static_cast<int>(std::min<int64_t>(Qc, c.nq - b0));
        const float *Qb = c.Q + b0 * x->d;
        int64_t *ids = c.ids + b0 * k_max;
        float *dists = c.dists + b0 * k_max;
        const int64_t *Aq = nullptr;
        const int32_t *kq = nullptr;
        if (c.alpha_dev) {
            TC_HIP(taco::launch_budgets(c.alpha_dev + b0, c.kq_dev + b0, nb, x->n, k_max, S.Aq, S.kq,
                                        x->err, st),
                   "budget kernel");
            Aq = S.Aq;
            kq = S.kq;
        }
        TC_HIP(taco::launch_fill_u32(S.hist, int64_t(nb) * (x->Ns + 1), 0u, st), "clearing histograms");
        TC_HIP(taco::launch_fill_u32(S.cand_count, 2 * S.Qb + 4, 0u, st), "clearing candidate counts");

        rec(K_TRANSFORM, st, true);
        TC_HIP(taco::launch_transform(Qb, nb, x->d, x->mean, x->B, x->M, S.qt, st), "transform kernel");
        rec(K_TRANSFORM, st, false);

        float *dcd = dump && dump->cdist ? dump->cdist + b0 * x->Ns * 2 * x->l : nullptr;
        int32_t *dco = dump && dump->corder ? dump->corder + b0 * x->Ns * 2 * x->l : nullptr;
        const float *pre = nullptr;
        if (cdist != TC_CDIST_FP32) {
            rec(K_CDIST, st, true);
            TC_HIP(taco::launch_cdist_mfma(S.qt, nb, x->M, x->Ns, x->s, x->h1, x->h2, x->l, x->Kp,
                                           cdist == TC_CDIST_FP8, x->cT, x->cnorm, x->csc, S.qn,
                                           S.qsc, S.qa, S.cd, st),
                   "centroid distance kernel");
            rec(K_CDIST, st, false);
            pre = S.cd;
        }
        rec(K_PROBE, st, true);
        TC_HIP(taco::launch_probe(S.qt, nb, x->Ns, x->M, x->s, x->h1, x->h2, x->l, x->K, x->C1,
                                  x->C2, x->offs, A, Aq, S.cells, S.ncells, S.retrieved, dcd, dco,
                                  pre, x->probe_qpw, st),
               "probe kernel");
        rec(K_PROBE, st, false);

        // the order in which the count and re-rank take the queries (any order
        // gives the same results)
        const bool order = x->K <= 4096;
        if (order) TC_HIP(taco::launch_query_order(S.cells, nb, x->Ns, x->K, S.perm, st), "query order kernel");
        if (!codes)
            TC_HIP(taco::launch_flatten_cells(S.cells, S.ncells, nb, x->Ns, x->K, S.flat, S.ftot, st),
                   "probed cell list kernel");
        taco::CountLaunch cl{nb, x->Ns, x->K, x->T, x->W, x->bits, x->n, x->ids_enc, x->off2d, S.flat,
                             S.ftot, order ? S.perm : nullptr, c.plain ? 1 : x->count_qpw};
        cl.nt = c.plain ? 1024 : x->count_nt;
        taco::SelectLaunch sl{S.hist, R, x->rule, cap, S.cand, S.cand_count,
                              dump && dump->sc ? dump->sc + b0 * x->n : nullptr,
                              dump && dump->last ? dump->last + b0 : nullptr,
                              dump && dump->hist ? dump->hist + b0 * (x->Ns + 1) : nullptr};
        sl.ovf = ovf;
        if (fused) {
            TC_HIP(taco::launch_fill_u32(S.arrive, nb, 0u, st), "clearing tile arrivals");
            TC_HIP(taco::launch_fill_u32(S.qctr, x->T, 0u, st), "clearing the work queue");
            // per-query budgets: hand the largest walks out first
            if (Aq) TC_HIP(taco::launch_cost_order(S.retrieved, nb, x->Ns, S.perm, st), "cost order kernel");
            rec(K_FUSED, st, true);
            TC_HIP(taco::launch_count_select(cl, sl, std::min(x->fused_groups, nb), S.arrive, x->err,
                                             1u << 24, S.qctr, (Aq || order) ? S.perm : nullptr, S.sc, st),
                   "fused count/select kernel");
            rec(K_FUSED, st, false);
        } else if (list) {
            uint32_t *redo = S.cand_count + S.Qb;
            const bool dsc = dump && dump->sc;
            const bool dh = dump && (dump->hist || dump->last);
            // the lists sit in the packed-count rows, which the list form
            // fills only for the queued queries, after their lists are read
            const taco::ListLaunch ll{x->list_level, S.lvl, cap, int64_t(x->W) * x->bits / 32, S.sc,
                                      S.cand, S.cand_count, S.tcount, redo, 64, R, x->rule, dh,
                                      sl.dump_last, sl.dump_hist, S.toff, S.tlev};
            rec(K_COUNT, st, true);
            TC_HIP(taco::launch_count(cl, S.hist, nullptr, 1, &ll, st), "count kernel (list)");
            rec(K_COUNT, st, false);
            rec(K_SELECT, st, true);
            TC_HIP(taco::launch_list_select(cl, ll, S.hist, st), "list select kernel");
            TC_HIP(taco::launch_count(cl, S.hist, S.sc, 2, &ll, st), "recount kernel");
            taco::SelectLaunch sr = sl;
            sr.dump_sc = nullptr;
            sr.dump_last = nullptr;
            sr.dump_hist = nullptr;
            sr.redo = redo;
            sr.redo_groups = 128;
            TC_HIP(taco::launch_select(cl, sr, S.sc, st), "select kernel (queued)");
            if (fixed)
                TC_HIP(taco::launch_select_level(cl, sr, S.sc, st), "boundary-level select kernel (queued)");
            rec(K_SELECT, st, false);
            if (dsc) {
                // stage dumps: every query's packed counts, over the lists
                // (the level counts it adds go to the spent histograms)
                TC_HIP(taco::launch_count(cl, S.hist, S.sc, 0, nullptr, st), "count kernel (dump)");
                TC_HIP(taco::launch_unpack_counts(S.sc, nb, x->T, x->W, x->bits, x->n, dump->sc + b0 * x->n, st),
                       "dump sc");
            }
        } else {
            rec(K_COUNT, st, true);
            if (codes)
                TC_HIP(taco::launch_count_codes(x->codes, S.cells, S.ncells, nb, x->Ns, x->K, x->n, x->T, x->W,
                                                x->bits, S.bm, S.sc, S.hist, x->num_cu, st),
                       "point-major count kernels");
            else
                TC_HIP(taco::launch_count(cl, S.hist, S.sc, 0, nullptr, st), "count kernel");
            rec(K_COUNT, st, false);
            rec(K_SELECT, st, true);
            TC_HIP(taco::launch_select(cl, sl, S.sc, st), "select kernel");
            if (fixed) TC_HIP(taco::launch_select_level(cl, sl, S.sc, st), "boundary-level select kernel");
            rec(K_SELECT, st, false);
        }

        if (precision != TC_FP32) {
            // bounds from the BF16 or 8-bit rows, the k-th smallest upper bound,
            // then the FP32 path's arithmetic on every row that can still make the top k
            rec(K_RERANK, st, true);
            if (precision == TC_BF16)
                TC_HIP(taco::launch_rerank16(Qb, nb, x->d, x->mu, x->base16, x->rowerr, S.cand,
                                             S.cand_count, cap, S.cand_dist, S.lb, rr_blocks, st),
                       "BF16 rerank kernel");
            else {
                // exact form: plain rows, 16 | d <= 256
                const bool ex = x->u8_plain && x->d % 16 == 0 && x->d <= 256;
                if (ex) TC_HIP(taco::launch_qbytes(Qb, nb, x->d, S.qinfo, st), "query bytes kernel");
                TC_HIP(taco::launch_rerank8(Qb, nb, x->d, x->base8, x->rmeta, x->u8_plain, S.cand,
                                            S.cand_count, cap, S.cand_dist, S.lb, S.exact,
                                            ex ? S.qinfo : nullptr, list ? S.toff : nullptr, x->T,
                                            order ? S.perm : nullptr, rr_blocks, st),
                       "8-bit rerank kernel");
            }
            rec(K_RERANK, st, false);
            rec(K_TOPK, st, true);
            TC_HIP(taco::launch_topk(S.cand, S.cand_dist, S.cand_count, cap, nb, k, kq, k_max,
                                     S.tau_ids, S.tau_d, st),
                   "bound top-k kernel");
            rec(K_TOPK, st, false);
            rec(K_RECHECK, st, true);
            TC_HIP(taco::launch_recheck_topk(Qb, nb, x->d, x->base, S.cand, S.cand_count, S.lb, cap,
                                             S.tau_d, k, kq, k_max, reinterpret_cast<int32_t *>(S.lb),
                                             S.cand_dist, S.rk_count,
                                             ids, dists, precision == TC_U8 ? S.exact : nullptr, S.tau_ids,
                                             st),
                   "re-check and top-k kernel");
            rec(K_RECHECK, st, false);
            if (dump && dump->nrecheck)
                TC_HIP(taco::launch_u32_to_i64(S.rk_count, dump->nrecheck + b0, nb, st), "dump nrecheck");
        } else {
            rec(K_RERANK, st, true);
            TC_HIP(taco::launch_rerank(Qb, nb, x->d, x->base, S.cand, S.cand_count, cap,
                                       S.cand_dist, rr_blocks, st),
                   "rerank kernel");
            rec(K_RERANK, st, false);

            rec(K_TOPK, st, true);
            TC_HIP(taco::launch_topk(S.cand, S.cand_dist, S.cand_count, cap, nb, k, kq, k_max, ids,
                                     dists, st),
                   "top-k kernel");
            rec(K_TOPK, st, false);
        }
        if (stream) {
            rec(K_STREAM, st, true);
            TC_HIP(taco::launch_stream_topk(Qb, nb, x->d, x->base, S.sc, x->T, x->W, x->bits, S.hist, x->Ns, x->n,
                                            R, x->rule, ovf, k, kq, k_max, cap, S.cand, S.cand_dist,
                                            S.cand_count, ids, dists, st),
                   "streamed top-k kernels");
            rec(K_STREAM, st, false);
        }

        if (dump) {
            const hipMemcpyKind dd = hipMemcpyDeviceToDevice;
            if (dump->qt)
                TC_HIP(hipMemcpyAsync(dump->qt + b0 * x->M, S.qt, sizeof(float) * nb * x->M, dd, st), "dump qt");
            if (dump->cells)
                TC_HIP(hipMemcpyAsync(dump->cells + b0 * x->Ns * x->K, S.cells,
                                      sizeof(int32_t) * size_t(nb) * x->Ns * x->K, dd, st), "dump cells");
            if (dump->ncells)
                TC_HIP(hipMemcpyAsync(dump->ncells + b0 * x->Ns, S.ncells, sizeof(int32_t) * nb * x->Ns, dd, st),
                       "dump ncells");
            if (dump->retrieved)
                TC_HIP(hipMemcpyAsync(dump->retrieved + b0 * x->Ns, S.retrieved,
                                      sizeof(int64_t) * nb * x->Ns, dd, st), "dump retrieved");
            if (dump->ncand)
                TC_HIP(taco::launch_u32_to_i64(S.cand_count, dump->ncand + b0, nb, st), "dump ncand");
            // candidates at the call's stride cap, dumped at stride n
            if (dump->cand)
                TC_HIP(hipMemcpy2DAsync(dump->cand + b0 * x->n, sizeof(int32_t) * size_t(x->n), S.cand,
                                        sizeof(int32_t) * size_t(cap), sizeof(int32_t) * size_t(cap), nb, dd, st),
                       "dump cand");
            if (dump->cand_dist && precision == TC_FP32)
                TC_HIP(hipMemcpy2DAsync(dump->cand_dist + b0 * x->n, sizeof(float) * size_t(x->n), S.cand_dist,
                                        sizeof(float) * size_t(cap), sizeof(float) * size_t(cap), nb, dd, st),
                       "dump cand_dist");
        }
    }
    return TC_OK;
}

int run(tc_index *x, const Call &c, void *stream) {
    if (c.nq == 0) return TC_OK;
    DeviceGuard g(x->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (x->count_mode == TC_COUNT_FUSED && x->fused_groups <= 0 && x->rule != TC_RULE_FIXED)
        return fail(TC_EINVAL, "the fused count/select kernel cannot keep all tiles of a query resident");
    if (!x->use_graph || c.dump) return enqueue(x, c, st);
    GraphKey key;
    memset(&key, 0, sizeof key);
    key.Q = c.Q;
    key.kq = c.kq_dev;
    key.alpha_dev = c.alpha_dev;
    key.ids = c.ids;
    key.dists = c.dists;
    key.nq = c.nq;
    key.k = c.k;
    key.k_max = c.k_max;
    memcpy(&key.alpha_bits, &c.alpha, 8);
    memcpy(&key.beta_bits, &c.beta, 8);
    key.precision = x->precision;
    key.count_mode = x->count_mode;
    key.W = x->W;
    key.qpw = x->probe_qpw;
    key.rule = x->rule;
    key.rr_blocks = x->rr_blocks;
    key.cdist = x->cdist;
    key.list_level = x->list_level;
    key.count_qpw = x->count_qpw;
    key.count_nt = x->count_nt;
    key.Qb = x->Qb;
    key.pool = x->pool;
    key.slots = plan_slots(x);
    if (!x->graph_exec || !(key == x->graph_key)) {
        drop_graph(x);
        if (!x->cap_stream)
            TC_HIP(hipStreamCreateWithFlags(&x->cap_stream, hipStreamNonBlocking), "creating the capture stream");
        const bool prof = x->profile;
        x->profile = false;  // no timing events inside a graph
        TC_HIP(hipStreamBeginCapture(x->cap_stream, hipStreamCaptureModeThreadLocal), "beginning capture");
        int rc = enqueue(x, c, x->cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(x->cap_stream, &graph);
        x->profile = prof;
        if (rc != TC_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "ending capture");
        x->graph = graph;
        e = hipGraphInstantiate(&x->graph_exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(x);
            return hip_fail(e, "instantiating the search graph");
        }
        x->graph_key = key;
        x->graph_captures++;
    }
    record(x, K_GRAPH, st, true);
    TC_HIP(hipGraphLaunch(x->graph_exec, st), "launching the search graph");
    record(x, K_GRAPH, st, false);
    return TC_OK;
}

int search(tc_index *x, const float *Q, int64_t nq, int32_t k, double alpha, double beta,
           int64_t *ids, float *dists, void *stream, const tc_stage_dump *dump) {
    if (!x) return fail(TC_EINVAL, "index is NULL");
    if (nq < 0) return fail(TC_EINVAL, "nq < 0");
    if (nq == 0) return TC_OK;
    if (!Q || !ids || !dists) return fail(TC_EINVAL, "queries, ids and dists must be non-NULL");
    if (k < 1 || int64_t(k) > x->n || k > 1024) return fail(TC_EINVAL, "k must be in [1, min(n, 1024)]");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(TC_EINVAL, "alpha must be in (0, 1]");
    if (!(beta >= 0.0 && beta <= 1.0)) return fail(TC_EINVAL, "beta must be in [0, 1]");
    Call c;
    c.Q = Q;
    c.nq = nq;
    c.k = k;
    c.k_max = k;
    c.alpha = alpha;
    c.beta = beta;
    c.ids = ids;
    c.dists = dists;
    c.dump = dump;
    return run(x, c, stream);
}

}  // namespace

extern "C" {

int tc_load_index(const char *path, int device, tc_index **out) {
    if (!out) return fail(TC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!path) return fail(TC_EINVAL, "path is NULL");
    tc_index *x = new (std::nothrow) tc_index();
    if (!x) return fail(TC_ENOMEM, "host allocation failed");
    int rc;
    try {
        rc = load(path, device, x);
    } catch (const std::bad_alloc &) {
        rc = fail(TC_ENOMEM, "host allocation failed while reading the index");
    }
    if (rc != TC_OK) {
        DeviceGuard g(x->device);
        free_all(x);
        delete x;
        return rc;
    }
    *out = x;
    g_err.clear();
    return TC_OK;
}

void tc_free_index(tc_index *x) {
    if (!x) return;
    DeviceGuard g(x->device);
    free_all(x);
    delete x;
}

int tc_index_info(const tc_index *x, int64_t *n, int32_t *d, int32_t *Ns, int32_t *s, int32_t *l) {
    if (!x) return fail(TC_EINVAL, "index is NULL");
    if (n) *n = x->n;
    if (d) *d = x->d;
    if (Ns) *Ns = x->Ns;
    if (s) *s = x->s;
    if (l) *l = x->l;
    return TC_OK;
}

int tc_set_option(tc_index *x, int option, int64_t value) {
    if (!x) return fail(TC_EINVAL, "index is NULL");
    DeviceGuard g(x->device);
    switch (option) {
    case TC_OPT_SELECT_RULE:
        if (value != TC_RULE_PRINTED && value != TC_RULE_PROSE && value != TC_RULE_FIXED)
            return fail(TC_EINVAL, "unknown rule");
        x->rule = static_cast<int>(value);
        return TC_OK;
    case TC_OPT_MAX_BATCH:
        if (value < 1) return fail(TC_EINVAL, "max batch must be >= 1");
        TC_HIP(hipDeviceSynchronize(), "synchronizing before re-sizing scratch");
        x->max_batch = value;
        return alloc_scratch(x);
    case TC_OPT_SCRATCH_BYTES:
        if (value < 1) return fail(TC_EINVAL, "scratch budget must be >= 1 byte");
        TC_HIP(hipDeviceSynchronize(), "synchronizing before re-sizing scratch");
        x->scratch_budget = value;
        return alloc_scratch(x);
    case TC_OPT_CANDIDATE_SLOTS:
        if (value < 0) return fail(TC_EINVAL, "candidate slots must be >= 0 (0: automatic)");
        TC_HIP(hipDeviceSynchronize(), "synchronizing before re-sizing scratch");
        x->cand_slots = value;
        return alloc_scratch(x);
    case TC_OPT_TILE_IDS:
        if (value < 1024 || value % 1024 != 0 || value > (int64_t(1) << 20) ||
            taco::count_lds_bytes(static_cast<int>(value), x->bits) > size_t(x->max_lds))
            return fail(TC_EINVAL, "tile must be a multiple of 1024 ids whose packed counts fit the LDS");
        TC_HIP(hipDeviceSynchronize(), "synchronizing before rebuilding tiles");
        x->W = static_cast<int>(value);
        if (int rc = build_tiles(x)) return rc;
        return alloc_scratch(x);
    case TC_OPT_PRECISION: {
        if (value != TC_FP32 && value != TC_BF16 && value != TC_U8)
            return fail(TC_EINVAL, "precision must be TC_FP32, TC_BF16 or TC_U8");
        TC_HIP(hipDeviceSynchronize(), "synchronizing before re-sizing scratch");
        if (value == TC_BF16) {
            if (int rc = build_bf16(x)) return rc;
        }
        if (value == TC_U8) {
            if (int rc = build_u8(x)) return rc;
        }
        x->precision = static_cast<int>(value);
        return alloc_scratch(x);
    }
    case TC_OPT_CDIST_PRECISION:
        if (value != TC_CDIST_FP32 && value != TC_CDIST_BF16 && value != TC_CDIST_FP8)
            return fail(TC_EINVAL, "centroid-distance precision must be TC_CDIST_FP32, _BF16 or _FP8");
        if (value != TC_CDIST_FP32) {
            TC_HIP(hipDeviceSynchronize(), "synchronizing before packing the centroids");
            if (int rc = build_cdist(x, static_cast<int>(value))) return rc;
        }
        drop_graph(x);
        x->cdist = static_cast<int>(value);
        return TC_OK;
    case TC_OPT_COUNT_MODE:
        if (value != TC_COUNT_AUTO && value != TC_COUNT_SPLIT && value != TC_COUNT_FUSED &&
            value != TC_COUNT_LIST && value != TC_COUNT_CODES)
            return fail(TC_EINVAL, "unknown count mode");
        if (value == TC_COUNT_CODES) {
            if (taco::codes_lds_bytes(x->Ns, x->K) > size_t(x->max_lds))
                return fail(TC_EINVAL, "the probed-cell bitmaps of the point-major form do not fit the LDS");
            if (!x->codes) {
                TC_HIP(hipDeviceSynchronize(), "synchronizing before building the cell codes");
                int rc = dmalloc(&x->codes, size_t(x->n) * taco::code_stride(x->Ns), "cell codes");
                if (rc) return rc;
                TC_HIP(taco::launch_build_codes(x->ids, x->offs, x->Ns, x->K, x->n, x->codes, nullptr),
                       "building the cell codes");
                TC_HIP(hipDeviceSynchronize(), "building the cell codes");
            }
        }
        if (value == TC_COUNT_FUSED && x->fused_groups <= 0)
            return fail(TC_EINVAL, "the fused count/select kernel is unavailable for this index");
        if (value == TC_COUNT_LIST && x->n > (int64_t(1) << taco::list_shift(x->Ns)))
            return fail(TC_EINVAL, "ids and counts do not fit one list word for this index");
        x->count_mode = static_cast<int>(value);
        return TC_OK;
    case TC_OPT_LIST_LEVEL:
        if (value < 0 || value > x->Ns) return fail(TC_EINVAL, "list level must be in [0, Ns]");
        x->list_level = static_cast<int>(value);
        return TC_OK;
    case TC_OPT_GRAPH:
        if (value != 0 && value != 1) return fail(TC_EINVAL, "graph must be 0 or 1");
        x->use_graph = value != 0;
        if (!x->use_graph) drop_graph(x);
        return TC_OK;
    case TC_OPT_PROBE_QPW:
        if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
            return fail(TC_EINVAL, "queries per probe workgroup must be 1, 2, 4, 8 or 16");
        x->probe_qpw = static_cast<int>(value);
        return TC_OK;
    case TC_OPT_RERANK_BLOCKS:
        if (value < 1 || value > 1024) return fail(TC_EINVAL, "re-rank workgroups per query must be in [1, 1024]");
        x->rr_blocks = static_cast<int>(value);
        return TC_OK;
    case TC_OPT_PROFILE:
        if (value != 0 && value != 1) return fail(TC_EINVAL, "profile must be 0 or 1");
        x->profile = value != 0;
        return TC_OK;
    case TC_OPT_TUNE_PRECISION:
        if (value != 0 && value != 1) return fail(TC_EINVAL, "tune precision must be 0 or 1");
        x->tune_precision = value != 0;
        return TC_OK;
    case TC_OPT_COUNT_QPW:
        if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16 && value != 32)
            return fail(TC_EINVAL, "queries per counting workgroup must be 1, 2, 4, 8, 16 or 32");
        x->count_qpw = static_cast<int>(value);
        return TC_OK;
    case TC_OPT_COUNT_BLOCK:
        if (value != 768 && value != 1024)
            return fail(TC_EINVAL, "threads per counting workgroup must be 768 or 1024");
        x->count_nt = static_cast<int>(value);
        return TC_OK;
    default:
        return fail(TC_EINVAL, "unknown option");
    }
}

int tc_search(tc_index *x, const float *queries, int64_t nq, int32_t k, double alpha, double beta,
              int64_t *ids, float *dists, void *stream) {
    return search(x, queries, nq, k, alpha, beta, ids, dists, stream, nullptr);
}

int tc_search_noalloc(tc_index *x, const float *queries, int64_t nq, int32_t k, double alpha, double beta,
                      int64_t *ids, float *dists, void *stream) {
    if (!x) return fail(TC_EINVAL, "index is NULL");
    if (nq < 0) return fail(TC_EINVAL, "nq < 0");
    if (nq == 0) return TC_OK;
    if (!queries || !ids || !dists) return fail(TC_EINVAL, "queries, ids and dists must be non-NULL");
    if (k < 1 || int64_t(k) > x->n || k > 1024) return fail(TC_EINVAL, "k must be in [1, min(n, 1024)]");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(TC_EINVAL, "alpha must be in (0, 1]");
    if (!(beta >= 0.0 && beta <= 1.0)) return fail(TC_EINVAL, "beta must be in [0, 1]");
    unsigned char *base = noalloc_scratch(x->device);
    if (!base) return fail(TC_EDEVICE, "the static scratch array was not set up on this device");
    // per-query bytes of every buffer the plain path touches, each rounded up
    // to the array's 256-byte alignment once per buffer
    const int64_t NsK = int64_t(x->Ns) * x->K;
    const int64_t packed = int64_t(x->T) * (int64_t(x->W) * x->bits / 32);  // u32 words
    // candidate slots per query (queries with more take the streamed top-k)
    const int64_t cap = call_cap(x->n, budget_R(x->n, beta), std::min<int64_t>(plan_slots(x), 16384), k);
    auto up = [](int64_t b) { return (b + 255) & ~int64_t(255); };
    auto need = [&](int64_t qb) {
        return up(4 * qb * x->M) + 2 * up(4 * qb * NsK) + up(4 * qb * x->Ns) + up(8 * qb * x->Ns) +
               up(4 * qb * (x->Ns + 1)) + up(4 * (3 * qb + 4)) + up(4 * qb) + up(4 * qb) +
               2 * up(4 * qb * cap) + up(4 * qb * packed);
    };
    const int64_t limit = static_cast<int64_t>(TC_NOALLOC_SCRATCH_BYTES);
    if (need(1) > limit)
        return fail(TC_EINVAL, "tc_search_noalloc: one query needs " + std::to_string(need(1)) +
                                   " bytes of scratch, more than the " + std::to_string(limit) +
                                   "-byte static array (too many points or too large a beta); use tc_search");
    int64_t qb = std::min<int64_t>(nq, limit / need(1));
    while (qb > 1 && need(qb) > limit) qb--;
    Scratch S;
    S.Qb = qb;
    S.pool = qb * cap;
    int64_t at = 0;
    auto take = [&](int64_t bytes) {
        unsigned char *p = base + at;
        at += up(bytes);
        return p;
    };
    S.qt = reinterpret_cast<float *>(take(4 * qb * x->M));
    S.cells = reinterpret_cast<int32_t *>(take(4 * qb * NsK));
    S.flat = reinterpret_cast<int32_t *>(take(4 * qb * NsK));
    S.ncells = reinterpret_cast<int32_t *>(take(4 * qb * x->Ns));
    S.retrieved = reinterpret_cast<int64_t *>(take(8 * qb * x->Ns));
    S.hist = reinterpret_cast<uint32_t *>(take(4 * qb * (x->Ns + 1)));
    S.cand_count = reinterpret_cast<uint32_t *>(take(4 * (3 * qb + 4)));
    S.perm = reinterpret_cast<int32_t *>(take(4 * qb));
    S.ftot = reinterpret_cast<uint32_t *>(take(4 * qb));
    S.cand = reinterpret_cast<int32_t *>(take(4 * qb * cap));
    S.cand_dist = reinterpret_cast<float *>(take(4 * qb * cap));
    S.sc = reinterpret_cast<uint32_t *>(take(4 * qb * packed));
    if (at > limit) return fail(TC_EINVAL, "tc_search_noalloc: scratch plan exceeds the static array");
    Call c;
    c.Q = queries;
    c.nq = nq;
    c.k = k;
    c.k_max = k;
    c.alpha = alpha;
    c.beta = beta;
    c.ids = ids;
    c.dists = dists;
    c.plain = true;
    c.scratch = &S;
    DeviceGuard g(x->device);
    return enqueue(x, c, static_cast<hipStream_t>(stream));
}

int tc_search_batched(tc_index *x, const float *queries, int64_t nq, const double *alpha,
                      const int32_t *k, int32_t k_max, double beta, int64_t *ids, float *dists,
                      void *stream) {
    if (!x) return fail(TC_EINVAL, "index is NULL");
    if (nq < 0) return fail(TC_EINVAL, "nq < 0");
    if (nq == 0) return TC_OK;
    if (!queries || !alpha || !k || !ids || !dists)
        return fail(TC_EINVAL, "queries, alpha, k, ids and dists must be non-NULL");
    if (k_max < 1 || int64_t(k_max) > x->n || k_max > 1024)
        return fail(TC_EINVAL, "k_max must be in [1, min(n, 1024)]");
    if (!(beta >= 0.0 && beta <= 1.0)) return fail(TC_EINVAL, "beta must be in [0, 1]");
    Call c;
    c.Q = queries;
    c.nq = nq;
    c.k = k_max;
    c.kq_dev = k;
    c.k_max = k_max;
    c.alpha = 0.5;
    c.alpha_dev = alpha;
    c.beta = beta;
    c.ids = ids;
    c.dists = dists;
    return run(x, c, stream);
}

int tc_search_debug(tc_index *x, const float *queries, int64_t nq, int32_t k, double alpha,
                    double beta, int64_t *ids, float *dists, void *stream, const tc_stage_dump *dump) {
    return search(x, queries, nq, k, alpha, beta, ids, dists, stream, dump);
}

int tc_kernel_time(tc_index *x, const char *kernel, double *total_ms, int64_t *launches) {
    if (!x || !kernel) return fail(TC_EINVAL, "index and kernel name must be non-NULL");
    DeviceGuard g(x->device);
    int rc = resolve_timings(x);
    if (rc) return rc;
    for (int i = 0; i < K_COUNT_; i++) {
        if (strcmp(kernel, kKernelNames[i]) == 0) {
            if (total_ms) *total_ms = x->total_ms[i];
            if (launches) *launches = x->launches[i];
            return TC_OK;
        }
    }
    return fail(TC_EINVAL, std::string("unknown kernel name ") + kernel);
}

int tc_profile_reset(tc_index *x) {
    if (!x) return fail(TC_EINVAL, "index is NULL");
    DeviceGuard g(x->device);
    int rc = resolve_timings(x);
    for (int i = 0; i < K_COUNT_; i++) {
        x->total_ms[i] = 0.0;
        x->launches[i] = 0;
    }
    return rc;
}

}  // extern "C"

namespace {

struct TuneConfig {
    int W, mode, qpw, rr, precision, cqpw, nt;
};

// Cache key of a tuning: the GPU, the index (shape, seed, content hash), the
// options that change which kernels run, and the call (`call`).
std::string tune_key(const tc_index *x, const std::string &call) {
    hipDeviceProp_t prop;
    std::string dev = hipGetDeviceProperties(&prop, x->device) == hipSuccess ? prop.gcnArchName : "gpu";
    for (auto &ch : dev)
        if (ch == ' ' || ch == '\t' || ch == '"') ch = '_';
    std::ostringstream os;
    os << dev << "|cu" << x->num_cu << "|n" << x->n << "|d" << x->d << "|Ns" << x->Ns << "|s" << x->s << "|l"
       << x->l << "|seed" << std::hex << x->seed << "|id" << x->ident << std::dec << "|rule" << x->rule
       << "|cdist" << x->cdist << "|lvl" << x->list_level << "|tp"
       << (x->tune_precision ? -1 : x->precision) << "|" << call;
    return os.str();
}

int apply_config(tc_index *x, const TuneConfig &c) {
    int rc;
    if (c.W != x->W && (rc = tc_set_option(x, TC_OPT_TILE_IDS, c.W))) return rc;
    if (c.precision != x->precision && (rc = tc_set_option(x, TC_OPT_PRECISION, c.precision))) return rc;
    if ((rc = tc_set_option(x, TC_OPT_COUNT_MODE, c.mode))) return rc;
    if ((rc = tc_set_option(x, TC_OPT_PROBE_QPW, c.qpw))) return rc;
    if ((rc = tc_set_option(x, TC_OPT_COUNT_QPW, c.cqpw))) return rc;
    if ((rc = tc_set_option(x, TC_OPT_COUNT_BLOCK, c.nt))) return rc;
    return tc_set_option(x, TC_OPT_RERANK_BLOCKS, c.rr);
}

// Coordinate descent over the launch configurations for the call `once`
// (one search on stream st): tile width x count mode, then probe queries per
// workgroup, re-rank precision (if tuned), then re-rank workgroups per query.
int tune(tc_index *x, const std::string &key, const std::function<int()> &once, hipStream_t st,
         const char *cache_path, char *report, size_t report_len) {
    std::ostringstream rep;
    auto finish = [&](int rc) {
        if (report && report_len) {
            std::string s = rep.str();
            size_t m = std::min(s.size(), report_len - 1);
            memcpy(report, s.data(), m);
            report[m] = 0;
        }
        return rc;
    };
    // cache: one JSON object per line {"key": ..., "W": ..., ...}
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
            TuneConfig c{};
            c.nt = 1024;  // (entries written before the workgroup size was tuned have none)
            if (sscanf(line.c_str() + line.find("\"W\""),
                       "\"W\": %d, \"mode\": %d, \"qpw\": %d, \"rr\": %d, \"precision\": %d, \"cqpw\": %d, "
                       "\"nt\": %d",
                       &c.W, &c.mode, &c.qpw, &c.rr, &c.precision, &c.cqpw, &c.nt) >= 6) {
                if (apply_config(x, c) == TC_OK) {
                    rep << "cached " << key << " W=" << c.W << " mode=" << c.mode << " qpw=" << c.qpw
                        << " rr=" << c.rr << " precision=" << c.precision << " cqpw=" << c.cqpw << " nt=" << c.nt
                        << "\n";
                    return finish(TC_OK);
                }
                rep << "cached entry no longer applies (" << g_err << "); measuring\n";
                break;
            }
        }
    }
    hipEvent_t e0, e1;
    TC_HIP(hipEventCreate(&e0), "autotune timing");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return finish(fail(TC_EDEVICE, "autotune timing"));
    }
    const bool graph = x->use_graph, prof = x->profile;
    x->use_graph = false;
    x->profile = false;
    auto measure = [&](const TuneConfig &c, double *ms) -> int {
        int r = apply_config(x, c);
        if (r) return r;
        if ((r = once())) return r;
        TC_HIP(hipEventRecord(e0, st), "autotune timing");
        for (int i = 0; i < 3; i++)
            if ((r = once())) return r;
        TC_HIP(hipEventRecord(e1, st), "autotune timing");
        TC_HIP(hipEventSynchronize(e1), "autotune timing");
        float f = 0.0f;
        TC_HIP(hipEventElapsedTime(&f, e0, e1), "autotune timing");
        *ms = f / 3.0;
        rep << "W=" << c.W << " mode=" << c.mode << " qpw=" << c.qpw << " rr=" << c.rr
            << " precision=" << c.precision << " cqpw=" << c.cqpw << " nt=" << c.nt << " ms=" << *ms << "\n";
        return TC_OK;
    };
    int rc = TC_OK;
    TuneConfig best{x->W, x->count_mode == TC_COUNT_AUTO ? TC_COUNT_SPLIT : x->count_mode, x->probe_qpw,
                    x->rr_blocks, x->precision, x->count_qpw, x->count_nt};
    double best_ms = 1e30;
    std::vector<int> Ws = x->bits == 4 ? std::vector<int>{65536, 131072, 262144}
                                       : std::vector<int>{32768, 65536, 131072};
    for (int W : Ws) {
        if (taco::count_lds_bytes(W, x->bits) > size_t(x->max_lds)) continue;
        for (int mode : {TC_COUNT_SPLIT, TC_COUNT_FUSED, TC_COUNT_LIST}) {
            TuneConfig c = best;
            c.W = W;
            c.mode = mode;
            if (mode == TC_COUNT_FUSED) {
                // the fused form needs its groups resident at this width
                if ((rc = tc_set_option(x, TC_OPT_TILE_IDS, W))) goto done;
                if (x->fused_groups <= 0) continue;
            }
            if (mode == TC_COUNT_LIST && x->n > (int64_t(1) << taco::list_shift(x->Ns))) continue;
            double ms;
            if ((rc = measure(c, &ms))) goto done;
            if (ms < best_ms) best_ms = ms, best = c;
        }
    }
    if (taco::codes_lds_bytes(x->Ns, x->K) <= size_t(x->max_lds)) {
        TuneConfig c = best;
        c.mode = TC_COUNT_CODES;
        double ms;
        if ((rc = measure(c, &ms))) goto done;
        if (ms < best_ms) best_ms = ms, best = c;
    }
    if (best.mode == TC_COUNT_SPLIT || best.mode == TC_COUNT_LIST) {
        for (int cq : {2, 4, 8, 16, 32}) {
            TuneConfig c = best;
            c.cqpw = cq;
            double ms;
            if ((rc = measure(c, &ms))) goto done;
            if (ms < best_ms) best_ms = ms, best = c;
        }
        // the other workgroup size (more registers per wavefront, fewer wavefronts)
        TuneConfig c = best;
        c.nt = best.nt == 768 ? 1024 : 768;
        double ms;
        if ((rc = measure(c, &ms))) goto done;
        if (ms < best_ms) best_ms = ms, best = c;
    }
    for (int qpw : {1, 2, 4, 8, 16}) {
        TuneConfig c = best;
        c.qpw = qpw;
        double ms;
        if ((rc = measure(c, &ms))) goto done;
        if (ms < best_ms) best_ms = ms, best = c;
    }
    if (x->tune_precision) {
        for (int p : {TC_FP32, TC_BF16, TC_U8}) {
            TuneConfig c = best;
            c.precision = p;
            double ms;
            if ((rc = measure(c, &ms))) goto done;
            if (ms < best_ms) best_ms = ms, best = c;
        }
    }
    for (int rr : {8, 16, 32, 64}) {
        TuneConfig c = best;
        c.rr = rr;
        double ms;
        if ((rc = measure(c, &ms))) goto done;
        if (ms < best_ms) best_ms = ms, best = c;
    }
    rc = apply_config(x, best);
    rep << "best W=" << best.W << " mode=" << best.mode << " qpw=" << best.qpw << " rr=" << best.rr
        << " precision=" << best.precision << " cqpw=" << best.cqpw << " nt=" << best.nt << " ms=" << best_ms
        << "\n";
    if (rc == TC_OK && cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        out << "{\"key\": \"" << key << "\", \"W\": " << best.W << ", \"mode\": " << best.mode
            << ", \"qpw\": " << best.qpw << ", \"rr\": " << best.rr << ", \"precision\": " << best.precision
            << ", \"cqpw\": " << best.cqpw << ", \"nt\": " << best.nt << ", \"ms\": " << best_ms << "}\n";
    }
done:
    x->use_graph = graph;
    x->profile = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return finish(rc);
}

}  // namespace

extern "C" {

int tc_autotune(tc_index *x, const float *queries, int64_t nq, int32_t k, double alpha, double beta,
                void *stream, const char *cache_path, char *report, size_t report_len) {
    if (!x || !queries || nq < 1) return fail(TC_EINVAL, "index and a non-empty query batch are required");
    if (k < 1 || int64_t(k) > x->n || k > 1024) return fail(TC_EINVAL, "k must be in [1, min(n, 1024)]");
    if (!(alpha > 0.0 && alpha <= 1.0) || !(beta >= 0.0 && beta <= 1.0))
        return fail(TC_EINVAL, "alpha must be in (0, 1] and beta in [0, 1]");
    DeviceGuard g(x->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::ostringstream call;
    call << "nq" << nq << "|k" << k << "|a" << alpha << "|b" << beta;
    int64_t *ids = nullptr;
    float *dists = nullptr;
    int rc;
    if ((rc = dmalloc(&ids, size_t(nq) * k, "autotune ids"))) return rc;
    if ((rc = dmalloc(&dists, size_t(nq) * k, "autotune dists"))) {
        (void)hipFree(ids);
        return rc;
    }
    rc = tune(x, tune_key(x, call.str()),
              [&]() { return search(x, queries, nq, k, alpha, beta, ids, dists, st, nullptr); }, st,
              cache_path, report, report_len);
    (void)hipFree(ids);
    (void)hipFree(dists);
    return rc;
}

int tc_autotune_batched(tc_index *x, const float *queries, int64_t nq, const double *alpha, const int32_t *k,
                        int32_t k_max, double beta, void *stream, const char *cache_path, char *report,
                        size_t report_len) {
    if (!x || !queries || !alpha || !k || nq < 1)
        return fail(TC_EINVAL, "index, a non-empty query batch and its budgets are required");
    if (k_max < 1 || int64_t(k_max) > x->n || k_max > 1024)
        return fail(TC_EINVAL, "k_max must be in [1, min(n, 1024)]");
    if (!(beta >= 0.0 && beta <= 1.0)) return fail(TC_EINVAL, "beta must be in [0, 1]");
    DeviceGuard g(x->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the budgets enter the key through a hash of their bytes
    std::vector<double> ah(nq);
    std::vector<int32_t> kh(nq);
    TC_HIP(hipMemcpyAsync(ah.data(), alpha, sizeof(double) * nq, hipMemcpyDeviceToHost, st), "reading alpha");
    TC_HIP(hipMemcpyAsync(kh.data(), k, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, st), "reading k");
    TC_HIP(hipStreamSynchronize(st), "reading the budgets");
    Fnv f;
    f.add(ah.data(), ah.size() * sizeof(double));
    f.add(kh.data(), kh.size() * sizeof(int32_t));
    std::ostringstream call;
    call << "batched|nq" << nq << "|kmax" << k_max << "|b" << beta << "|budgets" << std::hex << f.h;
    int64_t *ids = nullptr;
    float *dists = nullptr;
    int rc;
    if ((rc = dmalloc(&ids, size_t(nq) * k_max, "autotune ids"))) return rc;
    if ((rc = dmalloc(&dists, size_t(nq) * k_max, "autotune dists"))) {
        (void)hipFree(ids);
        return rc;
    }
    rc = tune(x, tune_key(x, call.str()),
              [&]() { return tc_search_batched(x, queries, nq, alpha, k, k_max, beta, ids, dists, st); }, st,
              cache_path, report, report_len);
    (void)hipFree(ids);
    (void)hipFree(dists);
    return rc;
}

int tc_device_errors(tc_index *x, uint32_t *flags) {
    if (!x || !flags) return fail(TC_EINVAL, "index and flags must be non-NULL");
    DeviceGuard g(x->device);
    TC_HIP(hipDeviceSynchronize(), "synchronizing before reading the error word");
    TC_HIP(hipMemcpy(flags, x->err, sizeof(uint32_t), hipMemcpyDeviceToHost), "reading the error word");
    TC_HIP(hipMemset(x->err, 0, sizeof(uint32_t)), "clearing the error word");
    return TC_OK;
}

int tc_batch_capacity(const tc_index *x, double beta, int32_t k_max, int64_t *qpb) {
    if (!x || !qpb) return fail(TC_EINVAL, "index and output must be non-NULL");
    if (!(beta >= 0.0 && beta <= 1.0)) return fail(TC_EINVAL, "beta must be in [0, 1]");
    if (k_max < 1 || int64_t(k_max) > x->n || k_max > 1024) return fail(TC_EINVAL, "k must be in [1, min(n, 1024)]");
    *qpb = std::min<int64_t>(x->Qb, x->pool / call_cap(x->n, budget_R(x->n, beta), plan_slots(x), k_max));
    return TC_OK;
}

const char *tc_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Index construction on the GPU (Alg 1-3) and index files.
// ---------------------------------------------------------------------------

namespace {

// Device buffers of one call, freed on every exit path.
struct BuildBuffers {
    std::vector<void *> ptrs;
    ~BuildBuffers() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    int get(T **p, size_t count, const char *what) {
        *p = nullptr;
        void *v = nullptr;
        if (hipMalloc(&v, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess)
            return fail(TC_ENOMEM, std::string("device allocation failed: ") + what);
        ptrs.push_back(v);
        *p = static_cast<T *>(v);
        return TC_OK;
    }
};

struct StreamEvents {
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> ev;
    ~StreamEvents() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        if (st) (void)hipStreamDestroy(st);
    }
};

// Alg 2 (eigensystem allocation).  Eigenvalues are floored at 1e-12 of the
// largest and scaled by the smallest so that all are >= 1; taken in
// descending order (ties keep the lower index), each goes to the bucket with
// the smallest product of eigenvalues among those holding fewer than s, the
// lowest such bucket on ties.  Products are compared as FP64 sums of logs.
// cols = the buckets concatenated, each in append order.
int allocate_eigenpairs(const double *evals, int d, int Ns, int s, int32_t *cols) {
    if (!evals || !cols) return fail(TC_EINVAL, "evals or cols is NULL");
    if (d <= 0 || Ns <= 0 || s <= 0 || int64_t(Ns) * s > d) return fail(TC_EINVAL, "need Ns*s <= d");
    std::vector<double> lam(evals, evals + d);
    double mx = lam[0];
    for (double v : lam) mx = std::max(mx, v);
    for (double &v : lam) v = std::max(v, 1e-12 * mx);
    double mn = lam[0];
    for (double v : lam) mn = std::min(mn, v);
    if (!(mn > 0.0)) return fail(TC_EINVAL, "the covariance has no positive eigenvalue");
    for (double &v : lam) v = v / mn;
    std::vector<int> order(d);
    for (int i = 0; i < d; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] > lam[b]; });
    std::vector<double> logp(Ns, 0.0);
    std::vector<std::vector<int>> bucket(Ns);
    for (int i = 0; i < Ns * s; i++) {
        const int e = order[i];
        int best = -1;
        for (int j = 0; j < Ns; j++)
            if (int(bucket[j].size()) < s && (best < 0 || logp[j] < logp[best])) best = j;
        bucket[best].push_back(e);
        logp[best] += std::log(lam[e]);
    }
    int m = 0;
    for (int j = 0; j < Ns; j++)
        for (int e : bucket[j]) cols[m++] = e;
    return TC_OK;
}

// T = B^T (X - mean) row by row, in launches of at most 2^19 rows.
hipError_t transform_rows(const float *X, int64_t n, int d, const float *mean, const float *B, int M,
                          float *T, hipStream_t st) {
    const int64_t step = int64_t(1) << 19;
    for (int64_t r = 0; r < n; r += step) {
        const int rows = static_cast<int>(std::min(step, n - r));
        hipError_t e = taco::launch_transform(X + r * d, rows, d, mean, B, M, T + r * M, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int check_kmeans_args(int64_t n, int ld, int Ns, int s, int l, int iters, const int64_t *init,
                      const int64_t *train, int64_t nt) {
    if (n <= 0 || Ns <= 0 || s < 2 || int64_t(Ns) * s > ld || l < 1 || l > 64 || iters < 0)
        return fail(TC_EINVAL, "k-means shape out of range (l <= 64, Ns*s <= ld, s >= 2)");
    if (s - s / 2 > taco::bld::KM_HMAX) return fail(TC_EINVAL, "half-subspace wider than 32");
    if (!init) return fail(TC_EINVAL, "init is NULL");
    if (nt < l || nt > n) return fail(TC_EINVAL, "the training sample must hold between l and n points");
    for (int64_t i = 0; i < 2 * int64_t(Ns) * l; i++)
        if (init[i] < 0 || init[i] >= nt) return fail(TC_EINVAL, "seed position outside the training sample");
    if (train)
        for (int64_t p = 0; p < nt; p++)
            if (train[p] < 0 || train[p] >= n) return fail(TC_EINVAL, "training row out of range");
    return TC_OK;
}

// k-means of every half plus the final labels, on stream st.
int run_kmeans(BuildBuffers &bb, const float *T, int64_t n, int ld, int Ns, int s, int l, int iters,
               const int64_t *init, const int64_t *train, int64_t nt, float *cent, int32_t *assign,
               hipStream_t st) {
    int64_t *dinit = nullptr, *dtrain = nullptr;
    int rc;
    const size_t ni = 2 * size_t(Ns) * l;
    if ((rc = bb.get(&dinit, ni, "k-means seeds"))) return rc;
    TC_HIP(hipMemcpyAsync(dinit, init, sizeof(int64_t) * ni, hipMemcpyHostToDevice, st), "k-means seeds");
    if (train) {
        if ((rc = bb.get(&dtrain, size_t(nt), "training rows"))) return rc;
        TC_HIP(hipMemcpyAsync(dtrain, train, sizeof(int64_t) * size_t(nt), hipMemcpyHostToDevice, st),
               "training rows");
    }
    taco::bld::KmArgs a;
    a.T = T;
    a.n = n;
    a.ld = ld;
    a.Ns = Ns;
    a.s = s;
    a.l = l;
    a.iters = iters;
    a.init = dinit;
    a.train = dtrain;
    a.nt = nt;
    unsigned char *scr = nullptr;
    if ((rc = bb.get(&scr, taco::bld::km_scratch_bytes(a), "k-means scratch"))) return rc;
    TC_HIP(taco::bld::launch_kmeans(a, cent, assign, scr, st), "k-means");
    return TC_OK;
}

int run_imi(BuildBuffers &bb, const int32_t *assign, int64_t n, int Ns, int l, uint32_t *offsets,
            uint32_t *ids, hipStream_t st) {
    uint32_t *scr = nullptr;
    int rc;
    if ((rc = bb.get(&scr, taco::bld::imi_scratch_words(n, Ns, l), "IMI scratch"))) return rc;
    TC_HIP(taco::bld::launch_imi(assign, n, Ns, l, offsets, ids, scr, st), "IMI");
    return TC_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0f;
    return ms;
}

int build(const float *X, int64_t n, int d, int Ns, int s, int l, int iters, const int64_t *init,
          const int64_t *train, int64_t n_train, uint64_t seed, const float *mean_in, const float *B_in,
          int device, tc_index *x, double *stage_ms) {
    if (!X) return fail(TC_EINVAL, "base is NULL");
    x->n = n;
    x->d = d;
    x->Ns = Ns;
    x->s = s;
    x->h1 = s / 2;
    x->h2 = s - s / 2;
    x->l = l;
    x->seed = seed;
    int rc;
    if ((rc = check_shape(x, TC_EINVAL))) return rc;
    if (n < 2) return fail(TC_EINVAL, "the covariance needs n >= 2");
    if ((mean_in == nullptr) != (B_in == nullptr)) return fail(TC_EINVAL, "give both mean and B, or neither");
    if (!B_in && d > taco::bld::EIG_MAX_ONE_SIDED)
        return fail(TC_EINVAL, "the GPU eigensolver takes d <= 4096; pass mean and B for a larger d");
    const int64_t nt = train ? n_train : n;
    const int M = Ns * s, K = l * l, G = 2 * Ns, HM = s - s / 2;
    if ((rc = check_kmeans_args(n, M, Ns, s, l, iters, init, train, nt))) return rc;
    int ndev = 0;
    TC_HIP(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(TC_EINVAL, "no such HIP device");
    DeviceGuard g(device);
    StreamEvents se;
    TC_HIP(hipStreamCreateWithFlags(&se.st, hipStreamNonBlocking), "hipStreamCreate");
    se.ev.resize(7);
    for (auto &e : se.ev) TC_HIP(hipEventCreate(&e), "hipEventCreate");
    hipStream_t st = se.st;
    BuildBuffers bb;
    std::vector<float> mean32(d), B32(size_t(d) * M);
    TC_HIP(hipEventRecord(se.ev[0], st), "hipEventRecord");
    if (!B_in) {
        double *mean64, *cov, *sscr, *evals, *evecs, *escr;
        if ((rc = bb.get(&mean64, d, "mean")) || (rc = bb.get(&cov, size_t(d) * d, "covariance")) ||
            (rc = bb.get(&sscr, taco::bld::stats_scratch(n, d), "statistics scratch")) ||
            (rc = bb.get(&evals, d, "eigenvalues")) || (rc = bb.get(&evecs, size_t(d) * d, "eigenvectors")) ||
            (rc = bb.get(&escr, taco::bld::eigen_scratch(d), "rotations")))
            return rc;
        TC_HIP(taco::bld::launch_stats(X, n, d, mean64, cov, sscr, st), "mean and covariance");
        TC_HIP(hipEventRecord(se.ev[1], st), "hipEventRecord");
        TC_HIP(taco::bld::launch_eigen(cov, d, evals, evecs, escr, st), "eigensolver");
        TC_HIP(hipEventRecord(se.ev[2], st), "hipEventRecord");
        std::vector<double> hm(d), hl(d), hv(size_t(d) * d);
        TC_HIP(hipMemcpyAsync(hm.data(), mean64, sizeof(double) * d, hipMemcpyDeviceToHost, st), "mean");
        TC_HIP(hipMemcpyAsync(hl.data(), evals, sizeof(double) * d, hipMemcpyDeviceToHost, st), "eigenvalues");
        TC_HIP(hipMemcpyAsync(hv.data(), evecs, sizeof(double) * d * d, hipMemcpyDeviceToHost, st), "eigenvectors");
        TC_HIP(hipStreamSynchronize(st), "statistics");
        std::vector<int32_t> cols(M);
        if ((rc = allocate_eigenpairs(hl.data(), d, Ns, s, cols.data()))) return rc;
        for (int r = 0; r < d; r++)
            for (int m = 0; m < M; m++) B32[size_t(r) * M + m] = static_cast<float>(hv[size_t(r) * d + cols[m]]);
        for (int t = 0; t < d; t++) mean32[t] = static_cast<float>(hm[t]);
    } else {
        TC_HIP(hipEventRecord(se.ev[1], st), "hipEventRecord");
        TC_HIP(hipEventRecord(se.ev[2], st), "hipEventRecord");
        std::copy(mean_in, mean_in + d, mean32.begin());
        std::copy(B_in, B_in + size_t(d) * M, B32.begin());
    }
    float *dmean, *dB, *T, *cent;
    int32_t *assign;
    uint32_t *offs, *ids;
    if ((rc = bb.get(&dmean, d, "mean")) || (rc = bb.get(&dB, size_t(d) * M, "transform")) ||
        (rc = bb.get(&T, size_t(n) * M, "transformed base")) ||
        (rc = bb.get(&cent, size_t(G) * l * HM, "centroids")) ||
        (rc = bb.get(&assign, size_t(G) * n, "labels")) ||
        (rc = bb.get(&offs, size_t(Ns) * (K + 1), "cell offsets")) || (rc = bb.get(&ids, size_t(Ns) * n, "cell ids")))
        return rc;
    TC_HIP(hipMemcpyAsync(dmean, mean32.data(), sizeof(float) * d, hipMemcpyHostToDevice, st), "mean");
    TC_HIP(hipMemcpyAsync(dB, B32.data(), sizeof(float) * B32.size(), hipMemcpyHostToDevice, st), "transform");
    TC_HIP(hipEventRecord(se.ev[3], st), "hipEventRecord");
    TC_HIP(transform_rows(X, n, d, dmean, dB, M, T, st), "transform");
    TC_HIP(hipEventRecord(se.ev[4], st), "hipEventRecord");
    if ((rc = run_kmeans(bb, T, n, M, Ns, s, l, iters, init, train, nt, cent, assign, st))) return rc;
    TC_HIP(hipEventRecord(se.ev[5], st), "hipEventRecord");
    if ((rc = run_imi(bb, assign, n, Ns, l, offs, ids, st))) return rc;
    TC_HIP(hipEventRecord(se.ev[6], st), "hipEventRecord");
    std::vector<float> hc(size_t(G) * l * HM);
    std::vector<uint32_t> ho(size_t(Ns) * (K + 1)), hids(size_t(Ns) * n);
    TC_HIP(hipMemcpyAsync(hc.data(), cent, sizeof(float) * hc.size(), hipMemcpyDeviceToHost, st), "centroids");
    TC_HIP(hipMemcpyAsync(ho.data(), offs, sizeof(uint32_t) * ho.size(), hipMemcpyDeviceToHost, st), "offsets");
    TC_HIP(hipMemcpyAsync(hids.data(), ids, sizeof(uint32_t) * hids.size(), hipMemcpyDeviceToHost, st), "ids");
    TC_HIP(hipStreamSynchronize(st), "index build");
    if (stage_ms)
        for (int i = 0; i < 6; i++) stage_ms[i] = elapsed(se.ev[i], se.ev[i + 1]);
    const int h1 = s / 2, h2 = s - s / 2;
    std::vector<float> C1(size_t(Ns) * l * h1), C2(size_t(Ns) * l * h2);
    for (int j = 0; j < Ns; j++)
        for (int c = 0; c < l; c++) {
            for (int t = 0; t < h1; t++) C1[(size_t(j) * l + c) * h1 + t] = hc[((size_t(2 * j)) * l + c) * HM + t];
            for (int t = 0; t < h2; t++) C2[(size_t(j) * l + c) * h2 + t] = hc[((size_t(2 * j + 1)) * l + c) * HM + t];
        }
    std::vector<uint64_t> off64(ho.begin(), ho.end());
    return install(x, device, mean32, B32, C1, C2, off64, hids, nullptr, X);
}

int save(const tc_index *x, const char *path) {
    DeviceGuard g(x->device);
    const size_t n = size_t(x->n), d = size_t(x->d), Ns = size_t(x->Ns), K = size_t(x->K), M = size_t(x->M);
    std::vector<float> B(d * M), base(n * d);
    std::vector<uint32_t> offs(Ns * (K + 1)), ids(Ns * n);
    TC_HIP(hipMemcpy(B.data(), x->B, sizeof(float) * B.size(), hipMemcpyDeviceToHost), "transform");
    TC_HIP(hipMemcpy(offs.data(), x->offs, sizeof(uint32_t) * offs.size(), hipMemcpyDeviceToHost), "offsets");
    TC_HIP(hipMemcpy(ids.data(), x->ids, sizeof(uint32_t) * ids.size(), hipMemcpyDeviceToHost), "ids");
    TC_HIP(hipMemcpy(base.data(), x->base, sizeof(float) * base.size(), hipMemcpyDeviceToHost), "base");
    std::vector<uint64_t> off64(offs.begin(), offs.end());
    unsigned char hdr[128];
    memset(hdr, 0, sizeof hdr);
    const uint32_t ver = 1, hb = 128;
    const uint64_t flags = 0;
    const int32_t dims[6] = {x->d, x->Ns, x->s, x->h1, x->h2, x->l};
    memcpy(hdr, "TACOIDX1", 8);
    memcpy(hdr + 8, &ver, 4);
    memcpy(hdr + 12, &hb, 4);
    memcpy(hdr + 16, &x->n, 8);
    memcpy(hdr + 24, dims, 24);
    memcpy(hdr + 48, &x->seed, 8);
    memcpy(hdr + 56, &flags, 8);
    FILE *f = fopen(path, "wb");
    if (!f) return fail(TC_EIO, std::string("cannot create index file ") + path);
    Fnv sum;
    bool ok = true;
    auto put = [&](const void *p, size_t nb) {
        sum.add(p, nb);
        ok = ok && fwrite(p, 1, nb, f) == nb;
    };
    put(hdr, sizeof hdr);
    put(x->mean_host.data(), 4 * d);
    put(B.data(), 4 * B.size());
    put(x->C1h.data(), 4 * x->C1h.size());
    put(x->C2h.data(), 4 * x->C2h.size());
    put(off64.data(), 8 * off64.size());
    put(ids.data(), 4 * ids.size());
    put(base.data(), 4 * base.size());
    ok = ok && fwrite(&sum.h, 1, 8, f) == 8;
    ok = (fclose(f) == 0) && ok;
    return ok ? TC_OK : fail(TC_EIO, std::string("cannot write index file ") + path);
}

// SC-Linear (Section 2.3): exact per-subspace collisions over every point,
// then the fixed-budget selection, the FP32 re-rank and the top-k.
int sclinear(tc_index *x, const float *Q, int64_t nq, int32_t k, double alpha, double beta, int64_t *ids,
             float *dists, hipStream_t st, const tc_stage_dump *dump) {
    if (!x) return fail(TC_EINVAL, "index is NULL");
    if (nq < 0) return fail(TC_EINVAL, "nq < 0");
    if (nq == 0) return TC_OK;
    if (!Q || !ids || !dists) return fail(TC_EINVAL, "queries, ids and dists must be non-NULL");
    if (k < 1 || int64_t(k) > x->n || k > 1024) return fail(TC_EINVAL, "k must be in [1, min(n, 1024)]");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(TC_EINVAL, "alpha must be in (0, 1]");
    if (!(beta >= 0.0 && beta <= 1.0)) return fail(TC_EINVAL, "beta must be in [0, 1]");
    if (size_t(x->M) * 8 * sizeof(float) > 65536) return fail(TC_EINVAL, "SC-Linear needs Ns*s <= 2048");
    DeviceGuard g(x->device);
    int rc;
    const int64_t n = x->n;
    if (!x->sct) {
        if ((rc = dmalloc(&x->sct, size_t(n) * x->M, "SC-Linear transformed base"))) return rc;
        TC_HIP(transform_rows(x->base, n, x->d, x->mean, x->B, x->M, x->sct, nullptr), "transforming the base");
        TC_HIP(hipDeviceSynchronize(), "transforming the base");
    }
    // distances of up to 4 GiB per batch, at most the index's batch size
    const int64_t per_q = int64_t(x->Ns) * n * 4;
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>(x->Qb, (int64_t(4) << 30) / per_q));
    if (x->scQ != want) {
        (void)hipFree(x->scD);
        (void)hipFree(x->scthr);
        x->scD = nullptr;
        x->scthr = nullptr;
        x->scQ = 0;
        if ((rc = dmalloc(&x->scD, size_t(want) * x->Ns * n, "SC-Linear distances"))) return rc;
        if ((rc = dmalloc(&x->scthr, size_t(want) * x->Ns, "SC-Linear thresholds"))) return rc;
        x->scQ = want;
    }
    double a = std::ceil(alpha * double(n));
    a = std::min(std::max(a, 1.0), double(n));
    const int64_t A = static_cast<int64_t>(a), R = budget_R(n, beta);
    // the fixed-budget rule selects min(R, ...) candidates (all n with dumps)
    const int64_t cap = dump ? n : std::max<int64_t>(R, 1);
    const int64_t Qc = std::min<int64_t>(x->scQ, x->pool / cap);
    for (int64_t b0 = 0; b0 < nq; b0 += Qc) {
        const int nb = static_cast<int>(std::min<int64_t>(Qc, nq - b0));
        TC_HIP(taco::launch_fill_u32(x->hist, int64_t(nb) * (x->Ns + 1), 0u, st), "clearing histograms");
        TC_HIP(taco::launch_fill_u32(x->cand_count, 2 * x->Qb + 4, 0u, st), "clearing candidate counts");
        TC_HIP(taco::launch_transform(Q + b0 * x->d, nb, x->d, x->mean, x->B, x->M, x->qt, st), "transform kernel");
        TC_HIP(taco::launch_sub_dist(x->sct, n, x->M, x->Ns, x->s, x->qt, nb, x->scD, st), "subspace distances");
        TC_HIP(taco::launch_sub_select(x->scD, n, x->Ns, nb, A, x->scthr, st), "subspace selection");
        TC_HIP(taco::launch_sub_count(x->scD, n, x->Ns, nb, x->scthr, x->T, x->W, x->bits, x->sc, x->hist, st),
               "SC-Linear counts");
        taco::CountLaunch cl{nb, x->Ns, x->K, x->T, x->W, x->bits, n, x->ids_enc, x->off2d, x->flat, x->ftot,
                             nullptr};
        taco::SelectLaunch sl{x->hist, R, TC_RULE_FIXED, cap, x->cand, x->cand_count,
                              dump && dump->sc ? dump->sc + b0 * n : nullptr,
                              dump && dump->last ? dump->last + b0 : nullptr,
                              dump && dump->hist ? dump->hist + b0 * (x->Ns + 1) : nullptr};
        TC_HIP(taco::launch_select(cl, sl, x->sc, st), "select kernel");
        TC_HIP(taco::launch_select_level(cl, sl, x->sc, st), "boundary-level select kernel");
        TC_HIP(taco::launch_rerank(Q + b0 * x->d, nb, x->d, x->base, x->cand, x->cand_count, cap, x->cand_dist,
                                   x->rr_blocks, st),
               "rerank kernel");
        TC_HIP(taco::launch_topk(x->cand, x->cand_dist, x->cand_count, cap, nb, k, nullptr, k, ids + b0 * k,
                                 dists + b0 * k, st),
               "top-k kernel");
        if (dump && dump->ncand)
            TC_HIP(taco::launch_u32_to_i64(x->cand_count, dump->ncand + b0, nb, st), "dump ncand");
        if (dump && dump->cand)
            TC_HIP(hipMemcpy2DAsync(dump->cand + b0 * n, sizeof(int32_t) * size_t(n), x->cand,
                                    sizeof(int32_t) * size_t(cap), sizeof(int32_t) * size_t(cap), nb,
                                    hipMemcpyDeviceToDevice, st),
                   "dump cand");
    }
    return TC_OK;
}

}  // namespace

extern "C" {

int tc_build_stats(const float *X, int64_t n, int32_t d, double *mean, double *cov, void *stream) {
    if (!X || !mean || !cov) return fail(TC_EINVAL, "NULL buffer");
    if (n < 2 || d < 1) return fail(TC_EINVAL, "need n >= 2 and d >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    BuildBuffers bb;
    double *scr;
    int rc;
    if ((rc = bb.get(&scr, taco::bld::stats_scratch(n, d), "statistics scratch"))) return rc;
    TC_HIP(taco::bld::launch_stats(X, n, d, mean, cov, scr, st), "mean and covariance");
    TC_HIP(hipStreamSynchronize(st), "mean and covariance");
    return TC_OK;
}

int tc_build_eigen(const double *cov, int32_t d, double *evals, double *evecs, void *stream) {
    if (!cov || !evals || !evecs) return fail(TC_EINVAL, "NULL buffer");
    if (d < 1 || d > taco::bld::EIG_MAX_ONE_SIDED)
        return fail(TC_EINVAL, "the GPU eigensolver takes 1 <= d <= 4096");
    hipStream_t st = static_cast<hipStream_t>(stream);
    BuildBuffers bb;
    double *scr;
    int rc;
    if ((rc = bb.get(&scr, taco::bld::eigen_scratch(d), "rotations"))) return rc;
    TC_HIP(taco::bld::launch_eigen(cov, d, evals, evecs, scr, st), "eigensolver");
    TC_HIP(hipStreamSynchronize(st), "eigensolver");
    return TC_OK;
}

int tc_build_allocate(const double *evals, int32_t d, int32_t Ns, int32_t s, int32_t *cols) {
    return allocate_eigenpairs(evals, d, Ns, s, cols);
}

int tc_build_transform(const float *X, int64_t n, int32_t d, const float *mean, const float *B, int32_t M,
                       float *T, void *stream) {
    if (!X || !mean || !B || !T) return fail(TC_EINVAL, "NULL buffer");
    if (n < 0 || d < 1 || M < 1 || M > d) return fail(TC_EINVAL, "need n >= 0 and 1 <= M <= d");
    hipStream_t st = static_cast<hipStream_t>(stream);
    TC_HIP(transform_rows(X, n, d, mean, B, M, T, st), "transform");
    TC_HIP(hipStreamSynchronize(st), "transform");
    return TC_OK;
}

int tc_build_kmeans(const float *T, int64_t n, int32_t ld, int32_t Ns, int32_t s, int32_t l, int32_t iters,
                    const int64_t *init, const int64_t *train, int64_t n_train, float *cent,
                    int32_t *assign, void *stream) {
    if (!T || !cent || !assign) return fail(TC_EINVAL, "NULL buffer");
    const int64_t nt = train ? n_train : n;
    int rc;
    if ((rc = check_kmeans_args(n, ld, Ns, s, l, iters, init, train, nt))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    BuildBuffers bb;
    if ((rc = run_kmeans(bb, T, n, ld, Ns, s, l, iters, init, train, nt, cent, assign, st))) return rc;
    TC_HIP(hipStreamSynchronize(st), "k-means");
    return TC_OK;
}

int tc_build_imi(const int32_t *assign, int64_t n, int32_t Ns, int32_t l, uint32_t *offsets, uint32_t *ids,
                 void *stream) {
    if (!assign || !offsets || !ids) return fail(TC_EINVAL, "NULL buffer");
    if (n <= 0 || n >= (int64_t(1) << 31) || Ns < 1 || l < 1 || l * l > taco::bld::IMI_KMAX)
        return fail(TC_EINVAL, "need 0 < n < 2^31, Ns >= 1 and l*l <= 4096");
    hipStream_t st = static_cast<hipStream_t>(stream);
    BuildBuffers bb;
    int rc;
    if ((rc = run_imi(bb, assign, n, Ns, l, offsets, ids, st))) return rc;
    std::vector<uint32_t> ends(Ns);
    for (int j = 0; j < Ns; j++)
        TC_HIP(hipMemcpyAsync(&ends[j], offsets + (size_t(j) + 1) * (size_t(l) * l + 1) - 1, sizeof(uint32_t),
                              hipMemcpyDeviceToHost, st),
               "offsets");
    TC_HIP(hipStreamSynchronize(st), "IMI");
    for (int j = 0; j < Ns; j++)
        if (ends[j] != uint32_t(n)) return fail(TC_EINVAL, "a label lies outside [0, l)");
    return TC_OK;
}

int tc_build_index(const float *base, int64_t n, int32_t d, int32_t Ns, int32_t s, int32_t l, int32_t iters,
                   const int64_t *init, const int64_t *train, int64_t n_train, uint64_t seed,
                   const float *mean, const float *B, int device, tc_index **out, double *stage_ms) {
    if (!out) return fail(TC_EINVAL, "out is NULL");
    *out = nullptr;
    tc_index *x = new (std::nothrow) tc_index();
    if (!x) return fail(TC_ENOMEM, "host allocation failed");
    int rc;
    try {
        rc = build(base, n, d, Ns, s, l, iters, init, train, n_train, seed, mean, B, device, x, stage_ms);
    } catch (const std::bad_alloc &) {
        rc = fail(TC_ENOMEM, "host allocation failed while building the index");
    }
    if (rc != TC_OK) {
        DeviceGuard g(x->device);
        free_all(x);
        delete x;
        return rc;
    }
    *out = x;
    g_err.clear();
    return TC_OK;
}

int tc_search_sclinear(tc_index *x, const float *queries, int64_t nq, int32_t k, double alpha, double beta,
                       int64_t *ids, float *dists, void *stream, const tc_stage_dump *dump) {
    return sclinear(x, queries, nq, k, alpha, beta, ids, dists, static_cast<hipStream_t>(stream), dump);
}

int tc_save_index(const tc_index *x, const char *path) {
    if (!x || !path) return fail(TC_EINVAL, "index or path is NULL");
    try {
        return save(x, path);
    } catch (const std::bad_alloc &) {
        return fail(TC_ENOMEM, "host allocation failed while writing the index");
    }
}

}  // extern "C"

// kernels.h -- launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace taco {

struct CountLaunch {
    int nq, Ns, K, T, W;
    int bits;               // 4 (nibbles, Ns <= 15) or 8 (bytes) per packed count
    int64_t n;
    const uint32_t *ids;    // the id lists in 4-id groups, every (subspace, cell, tile)
                            // slice padded to whole groups, encoded for the tile width
                            // by launch_encode_ids
    const uint32_t *off2d;  // [T][Ns][K][2] first and end group of each tile's slice of each
                            // cell; slices are laid out tile by tile
    const int32_t *flat;    // [nq][Ns*K] probed cells as rows j*K + cell (launch_flatten_cells)
    const uint32_t *ftot;   // [nq] number of probed cells
    const int32_t *perm = nullptr;  // [nq] order in which the count takes the queries, or null
    int qpw = 1;                    // queries per count workgroup (split and list forms)
    int nt = 1024;                  // threads per count workgroup: 768 or 1024 (not the fused form)
};

struct SelectLaunch {
    const uint32_t *hist;   // [nq][Ns+1] level counts (levels >= 1)
    int64_t R;
    int rule;
    int64_t cap;
    int32_t *cand;
    uint32_t *cand_count;
    uint8_t *dump_sc;
    int32_t *dump_last;
    int64_t *dump_hist;
    const uint32_t *redo = nullptr;  // select the queued queries of a list selection
    int redo_groups = 0;             // workgroups over them (grid y)
    uint32_t *ovf = nullptr;         // [0] queries with more candidates than cap, [1 + i] the
                                     // queue (for launch_stream_topk); null only for the fixed rule
};

// List selection (count form 1): ids with count >= the list level are listed
// while counting and a launch of its own selects from the lists; queries
// whose threshold falls below the level are queued in redo
// ([0] queued, [1] above the level, [2 + i] the queue), recounted (form 2)
// and selected from their packed counts.
struct ListLaunch {
    int fixed;          // list level if > 0, else the adaptive level in *level
    uint32_t *level;    // device word
    int64_t cap;        // candidate slots per query
    int64_t lcap;       // list slots per tile
    uint32_t *list;     // [nq][T][lcap] listed words (count << shift | id), tile after tile
    int32_t *cand;
    uint32_t *count;
    uint32_t *tcount;   // [nq][T] entries listed per tile
    uint32_t *redo;
    int redo_groups;    // workgroups per tile for the recount (grid y)
    int64_t R;
    int rule;
    bool trans;         // the list launch also adds every level count (stage dumps)
    int32_t *dump_last;
    int64_t *dump_hist;
    uint32_t *toff;     // [nq][T+1] first candidate slot of each tile (candidates grouped by
                        // tile), [q][0] = 0xffffffff when query q's are not; or null
    uint32_t *tlev;     // [nq][T][Ns+1] listed ids per tile and level; or null (then no toff)
};

hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t st);
hipError_t launch_u32_to_i64(const uint32_t *src, int64_t *dst, int64_t count, hipStream_t st);
hipError_t launch_build_off2d(const uint32_t *ids, const uint32_t *offs, int Ns, int K, int64_t n,
                              int T, int W, uint32_t *off2d, hipStream_t st);
// raw: [Ns][K][T+1] slice starts in ids[j] (launch_build_off2d); pad:
// [Ns][K][T][2] first and end group of each slice in the padded lists enc.
hipError_t launch_encode_ids(const uint32_t *ids, const uint32_t *raw, const uint32_t *pad, int Ns, int K, int T,
                             int64_t n, int W, int bits, uint32_t *enc, hipStream_t st);
hipError_t launch_transform(const float *Q, int nq, int d, const float *mean, const float *B,
                            int M, float *qt, hipStream_t st);
hipError_t launch_probe(const float *qt, int nq, int Ns, int M, int s, int h1, int h2, int l,
                        int K, const float *C1, const float *C2, const uint32_t *offs, int64_t A,
                        const int64_t *A_q, int32_t *cells, int32_t *ncells, int64_t *retrieved,
                        float *dump_cdist, int32_t *dump_corder, const float *pre, int qpw,
                        hipStream_t st);
// Reduced-precision centroid distances: the block-diagonal centroid matrix
// (transposed, Kp = M rounded up to 32 columns; bf16 or e4m3 with per-
// subspace scales csc) and its FP32 norms, then per batch the distances
// cd[nq][Ns][2][l] (qn [nq][Ns][2], qsc [nq][Ns] and the operand rows qa [nq][Kp] (bytes for
// FP8, 16-bit values for BF16) are scratch).
hipError_t launch_prep_centroids(const float *C1, const float *C2, int Ns, int s, int h1, int h2, int l,
                                 int Kp, bool fp8, const float *csc, void *cT, float *cnorm, hipStream_t st);
hipError_t launch_cdist_mfma(const float *qt, int nq, int M, int Ns, int s, int h1, int h2, int l, int Kp,
                             bool fp8, const void *cT, const float *cnorm, const float *csc, float *qn,
                             float *qsc, void *qa, float *cd, hipStream_t st);
hipError_t launch_budgets(const double *alpha, const int32_t *kq, int nq, int64_t n, int k_max,
                          int64_t *A, int32_t *kc, uint32_t *err, hipStream_t st);
hipError_t prepare_count_kernels(int W, int bits, int Ns);
size_t count_lds_bytes(int W, int bits);
// form 0: store packed counts; 1: list (and store them when sc is given); 2: recount the queue
hipError_t launch_count(const CountLaunch &c, uint32_t *hist, uint32_t *sc, int form, const ListLaunch *l,
                        hipStream_t st);
hipError_t launch_unpack_counts(const uint32_t *sc, int nq, int T, int W, int bits, int64_t n, uint8_t *out,
                                hipStream_t st);
hipError_t launch_list_select(const CountLaunch &c, const ListLaunch &l, uint32_t *hist, hipStream_t st);
int list_shift(int Ns);
// Fixed-budget rule (rule 2), after launch_select: the first points of the
// boundary level in id order, and the final candidate counts (with s.redo,
// of the queued queries of a list selection only).
hipError_t launch_select_level(const CountLaunch &c, const SelectLaunch &s, const uint32_t *sc,
                               hipStream_t st);
hipError_t launch_select(const CountLaunch &c, const SelectLaunch &s, const uint32_t *sc,
                         hipStream_t st);
size_t fused_lds_bytes(int W, int bits);
hipError_t fused_max_blocks(int W, int bits, int Ns, int *blocks_per_cu);
// sc: [nq][T][W*bits/32] words; receives the packed counts of the queries
// whose candidates outgrow s.cap
hipError_t launch_count_select(const CountLaunch &c, const SelectLaunch &s, int NG, uint32_t *arrive,
                               uint32_t *err, uint32_t spin_limit, uint32_t *queue, const int32_t *order,
                               uint32_t *sc, hipStream_t st);
// queries by descending work (sum of retrieved over subspaces), into perm
hipError_t launch_cost_order(const int64_t *retrieved, int nq, int Ns, int32_t *perm, hipStream_t st);
int rerank_lanes_per_row(int d);
hipError_t launch_rerank(const float *Q, int nq, int d, const float *base, const int32_t *cand,
                         const uint32_t *cand_count, int64_t cap, float *cand_dist, int blocks_per_q,
                         hipStream_t st);
hipError_t launch_rerank16(const float *Q, int nq, int d, const float *mu, const uint16_t *base16,
                           const float *rowerr, const int32_t *cand, const uint32_t *cand_count,
                           int64_t cap, float *ub, float *lb, int blocks_per_q, hipStream_t st);
// 8-bit rows with a 16-byte (offset, step, error) record per row (exact for
// integer rows within 255); plain: every record is (0, 1, 0) and none is read.
// exact[q] (optional) is set when both bounds are the FP32 distance.
// qinfo (optional, from launch_qbytes): per-query integrality, |q|^2 and bytes
// toff: [nq][T+1] candidates grouped by tile (k_list_select), or null;
// perm: the order in which the queries are taken (launch_query_order), or null
hipError_t launch_rerank8(const float *Q, int nq, int d, const uint8_t *base8, const float4 *meta, bool plain,
                          const int32_t *cand, const uint32_t *cand_count, int64_t cap, float *ub, float *lb,
                          uint32_t *exact, const uint32_t *qinfo, const uint32_t *toff, int T,
                          const int32_t *perm, int blocks_per_q, hipStream_t st);
// The probed cells (cells [nq][Ns][K], ncells [nq][Ns]) as one list per
// query of rows j*K + cell (flat [nq][Ns*K]) and its length (ftot [nq])
hipError_t launch_flatten_cells(const int32_t *cells, const int32_t *ncells, int nq, int Ns, int K, int32_t *flat,
                                uint32_t *ftot, hipStream_t st);
// perm[i] = the query of rank i when the batch is ordered by the first cell
// probed in subspace 0 (cells: [nq][Ns][K]); K <= 4096
hipError_t launch_query_order(const int32_t *cells, int nq, int Ns, int K, int32_t *perm, hipStream_t st);
// [nq][d/4 + 4]: the values as bytes, an integer-in-[0,255] flag, |q|^2 (16 | d <= 256)
hipError_t launch_qbytes(const float *Q, int nq, int d, uint32_t *info, hipStream_t st);
hipError_t launch_prep_u8(const float *base, int64_t n, int d, uint8_t *base8, float4 *meta, uint32_t *plain,
                          hipStream_t st);
// FP32 re-check of the rows with lb <= tau, then the top-k of those rows;
// queries with exact[q] set (exact may be null) copy the bound top-k rows
hipError_t launch_recheck_topk(const float *Q, int nq, int d, const float *base, const int32_t *cand,
                               const uint32_t *cand_count, const float *lb, int64_t cap, const float *tau_d,
                               int k, const int32_t *kq, int k_max, int32_t *rk_ids, float *rk_dist,
                               uint32_t *rk_count, int64_t *ids_out, float *d_out, const uint32_t *exact,
                               const int64_t *tau_ids, hipStream_t st);
hipError_t launch_prep_bf16(const float *base, int64_t n, int d, const float *mu, uint16_t *base16,
                            float *rowerr, hipStream_t st);
hipError_t launch_topk(const int32_t *cand, const float *cand_dist, const uint32_t *cand_count,
                       int64_t cap, int nq, int k, const int32_t *kq, int k_max, int64_t *ids,
                       float *dists, hipStream_t st);
// Workgroups (id ranges) per query of launch_stream_topk; each leaves up to
// k_max keys in the query's candidate slots, so cap >= STREAM_SPLIT * k_max.
constexpr int STREAM_SPLIT = 32;
// The queued queries of ovf (at most nq): FP32 re-rank and top-k of the ids
// whose packed count in sc reaches Alg 5's threshold (from hist, R, rule),
// into ids/dists [q][k_max], replacing what the top-k wrote for them; their
// candidate slots (cand, cand_dist at stride cap, count 0 before) hold the
// partial top-k lists.  hipErrorInvalidValue if cap < STREAM_SPLIT * k_max.
hipError_t launch_stream_topk(const float *Q, int nq, int d, const float *base, const uint32_t *sc, int T, int W,
                              int bits, const uint32_t *hist, int Ns, int64_t n, int64_t R, int rule,
                              const uint32_t *ovf, int k, const int32_t *kq, int k_max, int64_t cap, int32_t *cand,
                              float *cand_dist, uint32_t *cand_count, int64_t *ids, float *dists,
                              hipStream_t st);

// SC-Linear: per-subspace distances D [nq][Ns][n] of every point (canonical
// FP32 chain on the transformed base T [n][M]), the A-th smallest
// (distance, id) key of each (query, subspace), and the packed SC-scores
// with their level histogram (levels >= 1 added into hist).
hipError_t launch_sub_dist(const float *T, int64_t n, int M, int Ns, int s, const float *qt, int nq, float *D,
                           hipStream_t st);
hipError_t launch_sub_select(const float *D, int64_t n, int Ns, int nq, int64_t A, uint64_t *thr, hipStream_t st);
hipError_t launch_sub_count(const float *D, int64_t n, int Ns, int nq, const uint64_t *thr, int T, int W, int bits,
                            uint32_t *sc, uint32_t *hist, hipStream_t st);

// Point-major counting (TC_COUNT_CODES): codes [n][code_stride(Ns)] u16 of
// every point's cell per subspace (built once from the IMI), then per batch
// the probed-cell bitmaps bm [nq][Ns][ceil(K/32)] and the packed counts and
// level histogram of the split form.
int code_stride(int Ns);
size_t codes_lds_bytes(int Ns, int K);
hipError_t launch_build_codes(const uint32_t *ids, const uint32_t *offs, int Ns, int K, int64_t n, uint16_t *codes,
                              hipStream_t st);
hipError_t launch_count_codes(const uint16_t *codes, const int32_t *cells, const int32_t *ncells, int nq, int Ns,
                              int K, int64_t n, int T, int W, int bits, uint32_t *bm, uint32_t *sc, uint32_t *hist,
                              int num_cu, hipStream_t st);

}  // namespace taco

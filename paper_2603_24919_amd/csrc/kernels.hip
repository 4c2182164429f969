// kernels.hip -- gfx950 kernels of the TaCo query stage (Alg 4-6).
//
// One launch per pipeline step, all stream-ordered on the caller's stream:
//   k_transform   q' = B^T (q - mean)                 (Alg 6 transform step)
//   k_cdist_mfma  (reduced-precision form) half-subspace centroid distances
//                 on the matrix cores
//   k_probe       half distances, their order, and the cell probe of Alg 4
//                 for one (query, subspace) per wavefront
//   k_count       per-point collision counts of a tile of ids, held in LDS,
//                 and the tile's SC level histogram (Alg 6 count step,
//                 Alg 5 histogram)
//   k_select      Alg 5 threshold and candidate compaction from the packed
//                 counts
//   k_rerank      exact FP32 squared distances of the candidates, or
//   k_rerank16/8  intervals from BF16 or 8-bit rows, k_topk on their upper
//                 bounds, then k_recheck_topk: FP32 distances of the rows
//                 that can still make the top k, and their top k
//   k_topk        k smallest (distance, id) pairs by radix select
//
// Integer-deciding arithmetic (transform, half distances, cell keys) uses
// the canonical FP32 chain: one fused multiply-add per term, terms in
// ascending index order, starting from +0; the library is built with
// -ffp-contract=off so no other operation is fused.  That makes probed
// cells, counts and candidates reproducible bit for bit on any CPU that
// evaluates the same chain.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.h"

namespace taco {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / WAVE;

// ---------------------------------------------------------------------------
// wavefront helpers
// ---------------------------------------------------------------------------

// Unsigned minimum over the wavefront with DPP moves (gfx9 row operations):
// quad swaps, half-row and row mirrors leave every lane holding its row's
// minimum; two row broadcasts fold the four rows into lane 63, which is read
// back as a uniform value.
__device__ __forceinline__ uint32_t wave_min_u32_dpp(uint32_t v) {
    int x = static_cast<int>(v);
    // old value = the minimum's identity, so lanes outside row_mask leave x
    // unchanged and each stage can fold into one v_min with a DPP source
#define TACO_DPP_MIN(ctrl, rows)                                                           \
    x = static_cast<int>(min(static_cast<uint32_t>(x),                                     \
                             static_cast<uint32_t>(__builtin_amdgcn_update_dpp(            \
                                 -1, x, ctrl, rows, 0xf, false))))
    TACO_DPP_MIN(0xb1, 0xf);   // quad_perm [1,0,3,2]
    TACO_DPP_MIN(0x4e, 0xf);   // quad_perm [2,3,0,1]
    TACO_DPP_MIN(0x141, 0xf);  // row_half_mirror
    TACO_DPP_MIN(0x140, 0xf);  // row_mirror
    TACO_DPP_MIN(0x142, 0xa);  // row_bcast:15 into rows 1 and 3
    TACO_DPP_MIN(0x143, 0xc);  // row_bcast:31 into rows 2 and 3
#undef TACO_DPP_MIN
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(x, 63));
}

// Inclusive prefix sum over the (fully active) wavefront with DPP moves, no
// LDS: row shifts by 1, 2 and 3 (out-of-row sources read 0) give sums of
// four, shifts by 4 and 8 restricted to the upper banks of each row give the
// row's prefix, and two row broadcasts carry rows 0 and 0-1 into the rows
// above.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v, int lane) {
    (void)lane;
    const int v0 = static_cast<int>(v);
    int x = v0 + __builtin_amdgcn_update_dpp(0, v0, 0x111, 0xf, 0xf, true);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, v0, 0x112, 0xf, 0xf, true);          // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, v0, 0x113, 0xf, 0xf, true);          // row_shr:3
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xe, false);          // row_shr:4, lanes 4-15
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xc, false);          // row_shr:8, lanes 8-15
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);          // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);          // row_bcast:31 into rows 2, 3
    return static_cast<uint32_t>(x);
}

// Sum over the (fully active) wavefront, as a uniform value.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(wave_incl_scan_u32(v, 0)), WAVE - 1));
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint32_t>(v)), m, WAVE));
    const uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint32_t>(v >> 32)), m, WAVE));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Ascending bitonic sort of one value per lane across the wavefront.
__device__ __forceinline__ uint64_t wave_sort_u64(uint64_t v, int lane) {
#pragma unroll
    for (int size = 2; size <= WAVE; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const uint64_t o = shfl_xor_u64(v, stride);
            const bool keep_min = ((lane & stride) == 0) == ((lane & size) == 0);
            v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
        }
    }
    return v;
}

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t *p, int64_t count, uint32_t v) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

// Per-query collision budgets of the batched search: A = ceil(alpha*n) in
// IEEE double (the host's expression), clamped to [1, n]; k clamped to
// [1, k_max].  A value out of range sets bit 1 of *err.
__global__ void k_budgets(const double *alpha, const int32_t *kq, int nq, int64_t n, int k_max,
                          int64_t *A, int32_t *kc, uint32_t *err) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const double a = alpha[q];
    bool bad = !(a > 0.0 && a <= 1.0);
    double v = bad ? static_cast<double>(n) : ceil(a * static_cast<double>(n));
    if (v < 1.0) v = 1.0;
    if (v > static_cast<double>(n)) v = static_cast<double>(n);
    A[q] = static_cast<int64_t>(v);
    int k = kq[q];
    if (k < 1 || k > k_max) {
        bad = true;
        k = k < 1 ? 1 : k_max;
    }
    kc[q] = k;
    if (bad) atomicOr(err, 2u);
}

__global__ void k_u32_to_i64(const uint32_t *src, int64_t *dst, int64_t count) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = static_cast<int64_t>(src[i]);
}

// off2d[(j*K + c)*(T+1) + t] = position in ids[j] of the first id >= t*W among
// cell c's ids (which are ascending).  One thread per (subspace, cell).
__global__ void k_build_off2d(const uint32_t *ids, const uint32_t *offs, int Ns, int K,
                              int64_t n, int T, int W, uint32_t *off2d) {
    int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= static_cast<int64_t>(Ns) * K) return;
    int j = static_cast<int>(g / K), c = static_cast<int>(g % K);
    const uint32_t *idj = ids + static_cast<int64_t>(j) * n;
    uint32_t lo0 = offs[static_cast<int64_t>(j) * (K + 1) + c];
    uint32_t hi0 = offs[static_cast<int64_t>(j) * (K + 1) + c + 1];
    uint32_t *out = off2d + g * (T + 1);
    for (int t = 0; t <= T; t++) {
        uint64_t key = static_cast<uint64_t>(t) * static_cast<uint64_t>(W);
        uint32_t lo = lo0, hi = hi0;
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo) / 2;
            if (static_cast<uint64_t>(idj[mid]) < key) lo = mid + 1;
            else hi = mid;
        }
        out[t] = lo;
    }
}

// The id lists as the count walk reads them for tile width W.  Every slice
// (subspace j, cell c, tile t) of the lists is laid out on its own, padded
// to a whole number of 4-id groups: its first and end group are
// pad[((t*Ns + j)*K + c)*2 + {0, 1}] (the host lays the slices out tile by
// tile), its ids those of the unpadded positions raw[(j*K + c)*(T+1) + t]
// up to [.. + t + 1] of k_build_off2d.  An id's tile-local position
// loc = id mod W becomes (byte offset of its packed word) << 5 | (its bit
// position in the word), so an increment needs no index arithmetic; a pad
// becomes a word of the
// CT_DUMMY-word region that follows the W*bits/8 bytes of counts, spread
// over its words by position.  Offsets stay below 2^17 (the LDS), so codes
// stay below 2^22 and never collide with the walk's 0xffffffff "no id".
// One wavefront per slice.
constexpr uint32_t CT_DUMMY = 64;
__global__ void k_encode_ids(const uint32_t *__restrict__ ids, const uint32_t *__restrict__ raw,
                             const uint32_t *__restrict__ pad, int Ns, int K, int T, int64_t n, int W,
                             int bits, uint32_t *__restrict__ enc) {
    const int64_t sl = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / WAVE;
    if (sl >= static_cast<int64_t>(Ns) * K * T) return;
    const uint32_t lane = threadIdx.x % WAVE;
    const int64_t jc = sl / T;
    const int t = static_cast<int>(sl % T), j = static_cast<int>(jc / K);
    const int64_t b = jc * (T + 1) + t, bp = (static_cast<int64_t>(t) * Ns * K + jc) * 2;
    const uint32_t lo = raw[b], len = raw[b + 1] - lo;
    const uint32_t g0 = pad[bp], m = (pad[bp + 1] - g0) * 4u;
    const uint32_t *src = ids + static_cast<int64_t>(j) * n + lo;
    uint32_t *dst = enc + static_cast<int64_t>(g0) * 4;
    const uint32_t per = 32u / static_cast<uint32_t>(bits);
    const uint32_t cnt_bytes = static_cast<uint32_t>(W) * static_cast<uint32_t>(bits) / 8u;
    for (uint32_t e = lane; e < m; e += WAVE) {
        uint32_t v;
        if (e < len) {
            const uint32_t loc = src[e] % static_cast<uint32_t>(W);
            v = (((loc / per) * 4u) << 5) | ((loc % per) * static_cast<uint32_t>(bits));
        } else {
            v = (cnt_bytes + 4u * ((e + g0 * 4u) % CT_DUMMY)) << 5;
        }
        dst[e] = v;
    }
}

// ---------------------------------------------------------------------------
// transform: qt[q][m] = chain over t of fma(B[t][m], fl32(Q[q][t] - mean[t]))
// block (64, 4): x = output column, y = group of QPT queries.
// ---------------------------------------------------------------------------

constexpr int TR_QPT = 4;
constexpr int TR_Q = 4 * TR_QPT;  // queries per block
constexpr int TR_T = 64;          // t per LDS stage

__global__ __launch_bounds__(256) void k_transform(const float *__restrict__ Q, int nq, int d,
                                                   const float *__restrict__ mean,
                                                   const float *__restrict__ B, int M,
                                                   float *__restrict__ qt) {
    __shared__ float e[TR_Q][TR_T + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int col = blockIdx.x * 64 + tx;
    const int q0 = blockIdx.y * TR_Q;
    float acc[TR_QPT];
#pragma unroll
    for (int r = 0; r < TR_QPT; r++) acc[r] = 0.0f;
    for (int t0 = 0; t0 < d; t0 += TR_T) {
#pragma unroll
        for (int r = 0; r < TR_QPT; r++) {
            int qi = ty * TR_QPT + r, t = t0 + tx;
            float v = 0.0f;
            if (q0 + qi < nq && t < d) v = Q[static_cast<int64_t>(q0 + qi) * d + t] - mean[t];
            e[qi][tx] = v;
        }
        __syncthreads();
        const int tn = min(TR_T, d - t0);
        if (col < M) {
            for (int tt = 0; tt < tn; tt++) {
                float b = B[static_cast<int64_t>(t0 + tt) * M + col];
#pragma unroll
                for (int r = 0; r < TR_QPT; r++) acc[r] = fmaf(b, e[ty * TR_QPT + r][tt], acc[r]);
            }
        }
        __syncthreads();
    }
    if (col < M) {
#pragma unroll
        for (int r = 0; r < TR_QPT; r++) {
            int q = q0 + ty * TR_QPT + r;
            if (q < nq) qt[static_cast<int64_t>(q) * M + col] = acc[r];
        }
    }
}

// ---------------------------------------------------------------------------
// centroid distances on the matrix cores (the reduced-precision form).
// D = |x|^2 + |c|^2 - 2 x.c for each half-subspace centroid c, with x the
// query's half; the norms are FP32 from the FP32 values and only the cross
// term runs on MFMA, with BF16 or FP8 (e4m3) operands and FP32 accumulation.
// All half-subspaces at once form one contraction q' (nq x M) times a block-
// diagonal matrix (M x Ns*2*l): column (j, h, c) holds centroid c of half h
// of subspace j in the rows of that half and zeros elsewhere, so a 16-column
// tile only needs the 32-row blocks its halves cover.  FP8 operands are
// scaled: centroids by one factor per subspace, a query's values by one
// factor per (query, subspace), each mapping the largest magnitude to 240
// (finite in both e4m3 variants), so every product in a column's sum
// carries the same two factors.
// ---------------------------------------------------------------------------

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr float FP8_RANGE = 240.0f;

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Packs four FP32 values (already scaled) into four e4m3 bytes.
__device__ __forceinline__ uint32_t fp8x4(float a, float b, float c, float d) {
    const float lim = FP8_RANGE;
    a = fminf(fmaxf(a, -lim), lim);
    b = fminf(fmaxf(b, -lim), lim);
    c = fminf(fmaxf(c, -lim), lim);
    d = fminf(fmaxf(d, -lim), lim);
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return static_cast<uint32_t>(w);
}

// Per (query, subspace): the two half norms |x_h|^2 (one fma per term,
// ascending) and the FP8 query scale max|x| / 240 (1 when the half values
// are all zero); and the query's operand row of the contraction, qa[q][k]
// for k < Kp (zero from M on): e4m3 of x / scale (FP8) or the BF16 of x.
// grid ceil(nq*Ns/256), block 256.
template <bool FP8>
__global__ __launch_bounds__(256) void k_qstats(const float *__restrict__ qt, int nq, int Ns, int M,
                                                int s, int h1, int Kp, float *__restrict__ qn,
                                                float *__restrict__ qsc, void *__restrict__ qa) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (t >= static_cast<int64_t>(nq) * Ns) return;
    const int64_t q = t / Ns;
    const int j = static_cast<int>(t % Ns);
    const float *x = qt + q * M + static_cast<int64_t>(j) * s;
    float n1 = 0.0f, n2 = 0.0f, mx = 0.0f;
    for (int u = 0; u < s; u++) {
        const float v = x[u];
        if (u < h1)
            n1 = fmaf(v, v, n1);
        else
            n2 = fmaf(v, v, n2);
        mx = fmaxf(mx, fabsf(v));
    }
    qn[t * 2] = n1;
    qn[t * 2 + 1] = n2;
    const float sc = mx > 0.0f ? mx / FP8_RANGE : 1.0f;
    qsc[t] = sc;
    const int k_end = j == Ns - 1 ? Kp : (j + 1) * s;  // the last subspace also writes the zero tail
    for (int k = j * s; k < k_end; k++) {
        const float v = k < M ? qt[q * M + k] : 0.0f;
        if (FP8)
            reinterpret_cast<uint8_t *>(qa)[q * Kp + k] = static_cast<uint8_t>(fp8x4(v / sc, 0.0f, 0.0f, 0.0f));
        else
            reinterpret_cast<uint16_t *>(qa)[q * Kp + k] = bf16_rne(v);
    }
}

// Column col = (j*2 + h)*l + c of the block-diagonal centroid matrix, stored
// transposed: cT[col][k] for k < Kp (bf16 bits or e4m3 bytes), with its
// FP32 norm.  FP8 centroids are divided by csc[j] (max |C| of subspace j
// over 240).  grid Ncol, block 64.
template <bool FP8>
__global__ __launch_bounds__(64) void k_prep_cent(const float *__restrict__ C1, const float *__restrict__ C2,
                                                  int Ns, int s, int h1, int h2, int l, int Kp,
                                                  const float *__restrict__ csc, void *__restrict__ cT,
                                                  float *__restrict__ cnorm) {
    const int col = blockIdx.x;
    const int j = col / (2 * l), h = (col / l) % 2, c = col % l;
    const int hh = h ? h2 : h1;
    const int base = j * s + (h ? h1 : 0);
    const float *src = (h ? C2 + (static_cast<int64_t>(j) * l + c) * h2 : C1 + (static_cast<int64_t>(j) * l + c) * h1);
    const float inv = FP8 ? 1.0f / csc[j] : 1.0f;
    for (int k4 = threadIdx.x * 4; k4 < Kp; k4 += 64 * 4) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int t = k4 + e - base;
            v[e] = (t >= 0 && t < hh) ? src[t] : 0.0f;
        }
        if (FP8) {
            reinterpret_cast<uint32_t *>(cT)[(static_cast<int64_t>(col) * Kp + k4) / 4] =
                fp8x4(v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv);
        } else {
            uint16_t *o = reinterpret_cast<uint16_t *>(cT) + static_cast<int64_t>(col) * Kp + k4;
#pragma unroll
            for (int e = 0; e < 4; e++) o[e] = bf16_rne(v[e]);
        }
    }
    if (threadIdx.x == 0) {
        float nn = 0.0f;
        for (int t = 0; t < hh; t++) nn = fmaf(src[t], src[t], nn);
        cnorm[col] = nn;
    }
}

// One 16 x 16 tile (16 queries x 16 columns) per wavefront, four column
// tiles per workgroup.  Operand layouts of the 16x16x32 MFMA: lane L holds
// row (L % 16) of A and column (L % 16) of B at k = 8*(L / 16) .. +8; the
// result tile gives lane L column (L % 16), rows 4*(L / 16) .. +4.
// grid (ceil(Ncol/64), ceil(nq/16)), block 256.  cd[q][j][h][c] = max(D, 0).
template <bool FP8>
__global__ __launch_bounds__(256) void k_cdist_mfma(const float *__restrict__ qt, int nq, int M, int Ns,
                                                    int s, int h1, int h2, int l, int Kp,
                                                    const void *__restrict__ cT, const float *__restrict__ cnorm,
                                                    const float *__restrict__ csc, const float *__restrict__ qn,
                                                    const float *__restrict__ qsc, const void *__restrict__ qa,
                                                    float *__restrict__ cd) {
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int ncol = Ns * 2 * l;
    const int n0 = (blockIdx.x * 4 + wave) * 16;
    if (n0 >= ncol) return;
    const int q0 = blockIdx.y * 16;
    // rows of the block-diagonal matrix this tile's columns can hold
    const int cl = min(n0 + 15, ncol - 1);
    const int jf = n0 / (2 * l), hf = (n0 / l) % 2, jl = cl / (2 * l), hl = (cl / l) % 2;
    const int k_lo = (jf * s + (hf ? h1 : 0)) / 32 * 32;
    const int k_hi = min(Kp, (jl * s + (hl ? s : h1) + 31) / 32 * 32);
    const int r = lane % 16, kq8 = 8 * (lane / 16);
    const int qrow = q0 + r;                   // this lane's query row of A
    const int colb = min(n0 + r, ncol - 1);    // this lane's column of B
    f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = k_lo; k0 < k_hi; k0 += 32) {
        const int kb = k0 + kq8;
        // A: this lane's 8 operand values of its query row (k_qstats: each
        // value already scaled by its own (query, subspace) factor in FP8)
        if (FP8) {
            const long av = qrow < nq ? *reinterpret_cast<const long *>(reinterpret_cast<const uint8_t *>(qa) +
                                                                       static_cast<int64_t>(qrow) * Kp + kb)
                                      : 0l;
            const long bv = *reinterpret_cast<const long *>(reinterpret_cast<const uint8_t *>(cT) +
                                                            static_cast<int64_t>(colb) * Kp + kb);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc, 0, 0, 0);
        } else {
            bf16x8_t av, bv;
            const uint16_t *bp = reinterpret_cast<const uint16_t *>(cT) + static_cast<int64_t>(colb) * Kp + kb;
            const uint4 braw = *reinterpret_cast<const uint4 *>(bp);
            const uint4 araw = qrow < nq ? *reinterpret_cast<const uint4 *>(reinterpret_cast<const uint16_t *>(qa) +
                                                                           static_cast<int64_t>(qrow) * Kp + kb)
                                         : make_uint4(0u, 0u, 0u, 0u);
            __builtin_memcpy(&av, &araw, 16);
            __builtin_memcpy(&bv, &braw, 16);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
        }
    }
    const int col = n0 + lane % 16;
    if (col >= ncol) return;
    const int j = col / (2 * l), h = (col / l) % 2, c = col % l;
    const float cn = cnorm[col];
    const float cs = FP8 ? csc[j] : 1.0f;
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int q = q0 + 4 * (lane / 16) + v;
        if (q >= nq) continue;
        const int64_t qj = static_cast<int64_t>(q) * Ns + j;
        const float scale = FP8 ? qsc[qj] * cs : 1.0f;
        const float dot = acc[v] * scale;
        const float dd = qn[qj * 2 + h] + cn - 2.0f * dot;
        cd[(qj * 2 + h) * l + c] = fmaxf(dd, 0.0f);
    }
}

// ---------------------------------------------------------------------------
// probe: one wavefront per (query, subspace).  Lane c computes the squared
// distance of each half of q' to centroid c, sorts them across the
// wavefront (stable: ties keep the lower centroid id first), then runs a
// tournament over the l rows of
// the cell grid: lane r holds row r's next unprobed column and its key
// fl32(D1s[r] + D2s[col]); each step takes the lexicographic minimum of
// (key, row) across the wavefront.  Rows are non-decreasing along columns,
// so this visits cells in exactly the order of Alg 4's heap (distance, row)
// and stops at the same cell: the first one that brings the retrieved count
// to at least A.
// grid (ceil(nq/QPW), Ns), block 64*QPW (one query per wavefront); dynamic
// LDS: the K cell sizes of subspace j.  The budget is A_q[q] when A_q is
// given, else A.
// ---------------------------------------------------------------------------

template <int QPW>
__global__ __launch_bounds__(64 * QPW) void k_probe(
    const float *__restrict__ qt, int nq, int M, int s, int h1, int h2, int l, int K,
    const float *__restrict__ C1, const float *__restrict__ C2,
    const uint32_t *__restrict__ offs, int64_t A_all, const int64_t *__restrict__ A_q,
    int32_t *__restrict__ cells, int32_t *__restrict__ ncells, int64_t *__restrict__ retrieved,
    float *__restrict__ dump_cdist, int32_t *__restrict__ dump_corder, const float *__restrict__ pre) {
    extern __shared__ uint32_t sizes[];  // [K]

    const int j = blockIdx.y, Ns = gridDim.y;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int q = blockIdx.x * QPW + wave;
    const uint32_t *off = offs + static_cast<int64_t>(j) * (K + 1);
    // eight cells per thread in flight at a time
    for (int c0 = 0; c0 < K; c0 += 8 * 64 * QPW) {
        uint32_t lo[8], hi[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int c = c0 + threadIdx.x + u * 64 * QPW;
            lo[u] = c < K ? off[c] : 0u;
            hi[u] = c < K ? off[c + 1] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int c = c0 + threadIdx.x + u * 64 * QPW;
            if (c < K) sizes[c] = hi[u] - lo[u];
        }
    }
    __syncthreads();
    if (q >= nq) return;  // no block-wide barrier below this point
    const int64_t A = A_q ? A_q[q] : A_all;

    const float *x = qt + static_cast<int64_t>(q) * M + static_cast<int64_t>(j) * s;
    float d1 = 0.0f, d2 = 0.0f;
    if (pre && lane < l) {
        const int64_t qj0 = static_cast<int64_t>(q) * Ns + j;
        d1 = pre[(qj0 * 2 + 0) * l + lane];
        d2 = pre[(qj0 * 2 + 1) * l + lane];
    } else if (lane < l) {
        // loads of 8 terms are issued together; the sums keep the ascending
        // one-fma-per-term order
        const float *c1 = C1 + (static_cast<int64_t>(j) * l + lane) * h1;
        const float *c2 = C2 + (static_cast<int64_t>(j) * l + lane) * h2;
        for (int t0 = 0; t0 < h1; t0 += 8) {
            float xs[8], cs[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                xs[u] = t0 + u < h1 ? x[t0 + u] : 0.0f;
                cs[u] = t0 + u < h1 ? c1[t0 + u] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                if (t0 + u < h1) {
                    const float v = xs[u] - cs[u];
                    d1 = fmaf(v, v, d1);
                }
            }
        }
        for (int t0 = 0; t0 < h2; t0 += 8) {
            float xs[8], cs[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                xs[u] = t0 + u < h2 ? x[h1 + t0 + u] : 0.0f;
                cs[u] = t0 + u < h2 ? c2[t0 + u] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                if (t0 + u < h2) {
                    const float v = xs[u] - cs[u];
                    d2 = fmaf(v, v, d2);
                }
            }
        }
    }
    // Stable ascending order of each half: a wavefront sort of (distance
    // bits, centroid) keys; distances are >= 0 (adding +0 turns a -0 into
    // +0), so the bits order like the values and equal distances keep the
    // lower centroid first.  Lane r then holds the rank-r distance and its
    // centroid.
    const uint64_t s1 = wave_sort_u64(lane < l ? (static_cast<uint64_t>(__float_as_uint(d1 + 0.0f)) << 32) |
                                                     static_cast<uint32_t>(lane)
                                               : ~0ull,
                                      lane);
    const uint64_t s2 = wave_sort_u64(lane < l ? (static_cast<uint64_t>(__float_as_uint(d2 + 0.0f)) << 32) |
                                                     static_cast<uint32_t>(lane)
                                               : ~0ull,
                                      lane);

    const int64_t qj = static_cast<int64_t>(q) * Ns + j;
    if (dump_cdist && lane < l) {
        dump_cdist[(qj * 2 + 0) * l + lane] = d1;
        dump_cdist[(qj * 2 + 1) * l + lane] = d2;
    }
    if (dump_corder && lane < l) {
        dump_corder[(qj * 2 + 0) * l + lane] = static_cast<int32_t>(static_cast<uint32_t>(s1));
        dump_corder[(qj * 2 + 1) * l + lane] = static_cast<int32_t>(static_cast<uint32_t>(s2));
    }

    // Tournament: lane r holds row r (half-1 rank r) with its next column and
    // key bits (keys are >= +0, so their bit patterns order like the floats).
    // Each step finds the smallest key, then the lowest row holding it.  The
    // sorted half-2 distances sit one per lane, so a step touches no memory;
    // PB steps run before their cells' sizes are read (one LDS read per
    // lane) and scanned for the step that reaches the budget A.  Steps past
    // it are discarded.
    constexpr int PB = 16;
    const float my_d1 = lane < l ? __uint_as_float(static_cast<uint32_t>(s1 >> 32)) : 0.0f;
    const float my_d2 = lane < l ? __uint_as_float(static_cast<uint32_t>(s2 >> 32)) : 0.0f;
    const int my_o1 = lane < l ? static_cast<int>(static_cast<uint32_t>(s1)) : 0;
    const int my_o2 = lane < l ? static_cast<int>(static_cast<uint32_t>(s2)) : 0;
    const float d2_0 = __uint_as_float(static_cast<uint32_t>(
        __builtin_amdgcn_readlane(static_cast<int>(__float_as_uint(my_d2)), 0)));
    int col = 0;
    uint32_t kb = lane < l ? __float_as_uint(my_d1 + d2_0) : 0xffffffffu;
    int32_t *out = cells + qj * K;
    int64_t got = 0;
    int nc = 0;
    bool done = false;
    while (!done) {
        int cellv = 0;  // lane s: the cell of step s of this batch
        int nb = 0;
        // (fully unrolled: the steps' loop control folds away)
#pragma unroll
        for (; nb < PB; nb++) {
            const uint32_t kmin = wave_min_u32_dpp(kb);
            if (kmin == 0xffffffffu) break;
            const int w = static_cast<int>(__builtin_ctzll(__ballot(kb == kmin)));
            const int cw = __builtin_amdgcn_readlane(col, w);
            const int cell = __builtin_amdgcn_readlane(my_o1, w) * l + __builtin_amdgcn_readlane(my_o2, cw);
            if (lane == nb) cellv = cell;
            const int nx = cw + 1 < l ? cw + 1 : 0;
            const uint32_t d2n = static_cast<uint32_t>(
                __builtin_amdgcn_readlane(static_cast<int>(__float_as_uint(my_d2)), nx));
            if (lane == w) {
                col = cw + 1;
                kb = col < l ? __float_as_uint(my_d1 + __uint_as_float(d2n)) : 0xffffffffu;
            }
        }
        if (nb == 0) break;
        // sizes of this batch's cells, their running sum, and the first step
        // whose running total reaches A
        const uint32_t sz = lane < nb ? sizes[cellv] : 0u;
        const uint32_t run = wave_incl_scan_u32(sz, lane);
        const uint64_t hit = __ballot(lane < nb && got + static_cast<int64_t>(run) >= A);
        const int take = hit ? static_cast<int>(__builtin_ctzll(hit)) + 1 : nb;
        if (lane < take) out[nc + lane] = cellv;
        got += static_cast<int64_t>(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(run), take - 1)));
        nc += take;
        done = hit != 0ull || nb < PB;
    }
    if (lane == 0) {
        ncells[qj] = nc;
        retrieved[qj] = got;
    }
}

// ---------------------------------------------------------------------------
// Query order of a batch for the re-rank: one workgroup sorts the queries by
// the first cell they probe in subspace 0 (their nearest cell there) with a
// counting sort over the K cells.  Queries near each other probe the same
// cells and share many candidates; run one after another, they find those
// rows in L2.  Any order gives the same results.  perm[i] is the query of
// rank i; dynamic LDS: K words (K <= 4096).
// ---------------------------------------------------------------------------

// The probed cells of each query as one list in subspace order, as index
// rows j*K + cell (the count kernels' slice lookups take one load), and
// their number.  One wavefront per query; grid ceil(nq/4), block 256.
__global__ __launch_bounds__(256) void k_flatten_cells(const int32_t *__restrict__ cells,
                                                       const int32_t *__restrict__ ncells, int nq, int Ns, int K,
                                                       int32_t *__restrict__ flat, uint32_t *__restrict__ ftot) {
    const int lane = threadIdx.x % WAVE;
    const int q = blockIdx.x * 4 + static_cast<int>(threadIdx.x / WAVE);
    if (q >= nq) return;
    // lane j < Ns: subspace j's count and first slot
    const uint32_t v = lane < Ns ? static_cast<uint32_t>(ncells[static_cast<int64_t>(q) * Ns + lane]) : 0u;
    const uint32_t pre = wave_incl_scan_u32(v, lane) - v;
    int32_t *fq = flat + static_cast<int64_t>(q) * Ns * K;
    for (int j = 0; j < Ns; j++) {
        const int32_t *cj = cells + (static_cast<int64_t>(q) * Ns + j) * K;
        const int n0 = __builtin_amdgcn_readlane(static_cast<int>(pre), j);
        const int nj = __builtin_amdgcn_readlane(static_cast<int>(v), j);
        for (int i = lane; i < nj; i += WAVE) fq[n0 + i] = j * K + cj[i];
    }
    const int tot = __builtin_amdgcn_readlane(static_cast<int>(pre + v), Ns - 1);
    if (lane == 0) ftot[q] = static_cast<uint32_t>(tot);
}

constexpr int ORD_BLOCK = 1024;

__global__ __launch_bounds__(ORD_BLOCK) void k_query_order(const int32_t *__restrict__ cells, int nq, int Ns,
                                                           int K, int32_t *__restrict__ perm) {
    extern __shared__ uint32_t bins[];
    __shared__ uint32_t wsum[ORD_BLOCK / WAVE];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    for (int i = threadIdx.x; i < K; i += ORD_BLOCK) bins[i] = 0u;
    // this thread's keys (queries threadIdx.x + u*ORD_BLOCK), loaded together
    constexpr int KPT = 16;
    int kq[KPT];
#pragma unroll
    for (int u = 0; u < KPT; u++) {
        const int q = static_cast<int>(threadIdx.x) + u * ORD_BLOCK;
        kq[u] = q < nq ? min(max(cells[static_cast<int64_t>(q) * Ns * K], 0), K - 1) : 0;
    }
    auto key = [&](int q) { return min(max(cells[static_cast<int64_t>(q) * Ns * K], 0), K - 1); };
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KPT; u++)
        if (static_cast<int>(threadIdx.x) + u * ORD_BLOCK < nq) atomicAdd(&bins[kq[u]], 1u);
    for (int q = static_cast<int>(threadIdx.x) + KPT * ORD_BLOCK; q < nq; q += ORD_BLOCK) atomicAdd(&bins[key(q)], 1u);
    __syncthreads();
    // exclusive prefix over the bins: a contiguous run of bins per thread
    const int per = (K + ORD_BLOCK - 1) / ORD_BLOCK;
    const int b0 = min(K, static_cast<int>(threadIdx.x) * per), b1 = min(K, b0 + per);
    uint32_t sum = 0u;
    for (int b = b0; b < b1; b++) sum += bins[b];
    const uint32_t inc = wave_incl_scan_u32(sum, lane);
    if (lane == WAVE - 1) wsum[wave] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int w = 0; w < wave; w++) run += wsum[w];
    for (int b = b0; b < b1; b++) {
        const uint32_t c = bins[b];
        bins[b] = run;
        run += c;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KPT; u++) {
        const int q = static_cast<int>(threadIdx.x) + u * ORD_BLOCK;
        if (q < nq) perm[atomicAdd(&bins[kq[u]], 1u)] = q;
    }
    for (int q = static_cast<int>(threadIdx.x) + KPT * ORD_BLOCK; q < nq; q += ORD_BLOCK)
        perm[atomicAdd(&bins[key(q)], 1u)] = q;
}

// Queries by descending work: the sum over subspaces of the points each
// probed (the count's walk), in 64 buckets of its binary logarithm, bucket
// by bucket from the largest (a counting sort; the order inside a bucket is
// arbitrary).  The fused count hands queries out in this order when budgets
// differ per query, so the longest ones start first.  grid 1, block
// ORD_BLOCK.
__global__ __launch_bounds__(ORD_BLOCK) void k_cost_order(const int64_t *__restrict__ retrieved, int nq, int Ns,
                                                          int32_t *__restrict__ perm) {
    __shared__ uint32_t bins[64];
    if (threadIdx.x < 64) bins[threadIdx.x] = 0u;
    __syncthreads();
    auto key = [&](int q) {
        int64_t r = 0;
        for (int j = 0; j < Ns; j++) r += retrieved[static_cast<int64_t>(q) * Ns + j];
        const int lg = r > 0 ? 63 - __clzll(static_cast<unsigned long long>(r)) : 0;
        return 63 - lg;  // larger work, smaller key
    };
    for (int q = threadIdx.x; q < nq; q += ORD_BLOCK) atomicAdd(&bins[key(q)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0u;
        for (int b = 0; b < 64; b++) {
            const uint32_t c = bins[b];
            bins[b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += ORD_BLOCK) perm[atomicAdd(&bins[key(q)], 1u)] = q;
}

// ---------------------------------------------------------------------------
// count / select: workgroup (tile t, query q) owns ids [t*W, t*W + W) and
// keeps their collision counts packed in LDS, BITS bits per id: 4-bit
// nibbles when Ns <= 15, bytes when Ns = 16 (adding 1 << BITS*(id%slot)
// never carries because counts never exceed Ns).  The probed cells of all Ns
// subspaces form one list.  For a chunk of CT_CHUNK of them, every thread
// looks up (index-time table off2d) the slice of one cell's id list that
// falls in the tile; the non-empty slices are compacted and laid end to end
// as one run of "positions" (block-wide prefix sums).  A position is a group
// of four ids: the device lists pad every slice to whole groups, with pads
// that increment a dummy word, so one 16-byte load and one slice lookup serve
// four increments.  Wavefronts then walk that run in windows of 64
// consecutive positions, CT_UNROLL windows in flight, so every lane reads one
// group per window whatever the slice lengths (cell sizes are skewed: a few
// long slices would otherwise serialise their walker).  A window table names the slice holding each window's first
// position and a bitmap marks every position that starts a slice; a lane
// finds its own slice by adding to the window's first slice the number of
// starts at or below its position in the window (one mbcnt over the 64-bit
// word), so no lane loops.  Per tile, the level histogram goes to HBM with
// either the packed counts (streamed back by the select kernel) or the list
// of ids that reached the list level.
// ---------------------------------------------------------------------------

#ifndef TACO_CT_BLOCK
#define TACO_CT_BLOCK 1024
#endif
#ifndef TACO_CT_UNROLL
#define TACO_CT_UNROLL 2
#endif
constexpr int CT_BLOCK = TACO_CT_BLOCK;         // threads of the fused kernel's workgroups and the
                                                // default of k_count's (its NT: 768 or 1024)
constexpr int CT_UNROLL = TACO_CT_UNROLL;       // windows (groups per lane) in flight per wavefront
constexpr int CT_WAVES = CT_BLOCK / WAVE;
constexpr int CT_CHUNK = CT_BLOCK;              // slices staged at a time, one per thread
constexpr int CT_WT = CT_BLOCK / 2;             // windows per position segment
// Functions templated on the workgroup size NT shadow these four with
// NT, NT / WAVE, NT and NT / 2.
constexpr int CT_STAGE = 256;                   // per-wavefront candidate staging slots

struct CountArgs {
    int Ns, K, T, W;
    int64_t n;
    const uint32_t *ids;     // padded 4-id groups encoded for the tile width (see k_encode_ids)
    const uint32_t *off2d;   // [T][Ns][K][2] first and end group of each slice in ids
    const int32_t *flat;     // [nq][Ns*K] probed cells as index rows j*K + cell (k_flatten_cells)
    const uint32_t *ftot;    // [nq] probed cells in all subspaces
    const int32_t *perm;     // [nq] query of each grid row (k_query_order), or null
    int nq;                  // queries of the launch
    int qpw;                 // queries per workgroup: grid row y takes rows y*qpw .. y*qpw+qpw-1
    int xper;                // > 0: one-dimensional grid of 8*xper workgroups in XCD order
};

// LDS carve-up of k_count (dynamic part).  dl and sb are adjacent (the
// fused kernel stages candidates there once counting is done).
struct CountLds {
    uint32_t *cnt;    // W*BITS/32 words of packed counts, then CT_DUMMY words that
                      // the pads of the id lists increment
    uint32_t *dl;     // [CT_CHUNK] (NT) start (group of ids) minus first position, per
                      // non-empty slice: position p of the slice is group dl + p
    uint32_t *sb;     // [2 * CT_WT] of a region of CT_CHUNK + 1 words: bit p - 1 of
                      // the segment is set when a non-empty slice starts at position
                      // p > 0 of the segment
    uint16_t *wt;     // [CT_WT] slice holding the first position of each window
    uint32_t *wsum;   // [2 * CT_WAVES] per-wavefront totals of the prefix sums
    uint32_t *hsum;   // [18] the tile's "count >= v" totals
    uint32_t *lsum;   // [17] levels of the listed ids
    uint32_t *lcnt;   // [1] ids listed by the re-walk (count_tile's XL form)
};

static_assert(2 * CT_WT <= CT_CHUNK + 1, "the start bitmap must fit its region");
static_assert(CT_CHUNK % 2 == 0, "the start bitmap is read in 64-bit words");

// Dynamic LDS of the count kernels with workgroups of nt threads.
__host__ __device__ constexpr size_t count_lds_size(int W, int bits, int nt = CT_BLOCK) {
    return static_cast<size_t>(W) * bits / 8 + CT_DUMMY * 4 + static_cast<size_t>(nt) * 4 +
           static_cast<size_t>(nt + 1) * 4 + static_cast<size_t>(nt / 2) * 2 + 2 * (nt / WAVE) * 4 +
           (18 + 17 + 1) * 4;
}

template <int BITS, int NT = CT_BLOCK>
__device__ __forceinline__ CountLds carve(unsigned char *lds, int W) {
    constexpr int CT_WAVES = NT / WAVE, CT_CHUNK = NT, CT_WT = NT / 2;
    CountLds c;
    c.cnt = reinterpret_cast<uint32_t *>(lds);
    c.dl = c.cnt + W / (32 / BITS) + CT_DUMMY;
    c.sb = c.dl + CT_CHUNK;  // 8-byte aligned: W*BITS/32, CT_DUMMY and CT_CHUNK are even
    c.wt = reinterpret_cast<uint16_t *>(c.sb + CT_CHUNK + 1);
    c.wsum = reinterpret_cast<uint32_t *>(c.wt + CT_WT);
    c.hsum = c.wsum + 2 * CT_WAVES;
    c.lsum = c.hsum + 18;
    c.lcnt = c.lsum + 17;
    return c;
}

// Group g of the padded id lists; the tiling keeps them below 2^30 ids, so
// the byte offset fits 32 bits and the load takes a scalar base.
__device__ __forceinline__ uint4 load_group(const uint32_t *ids, uint32_t g) {
    return *reinterpret_cast<const uint4 *>(reinterpret_cast<const unsigned char *>(ids) + (g << 4));
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

// The packed-count word at byte offset off of the counts.  ZB: the kernel
// has no static LDS, so the dynamic region, and the counts with it, start at
// LDS address 0 and the offset is the address itself (one add less per
// increment; prepare_count_kernels checks that k_count has none).
template <bool ZB>
__device__ __forceinline__ lds_u32 *count_word(uint32_t *cnt, uint32_t off) {
    if (ZB) return (lds_u32 *)static_cast<uintptr_t>(off);
    return (lds_u32 *)(reinterpret_cast<unsigned char *>(cnt) + off);  // an address-space cast
}

// Adds one to the packed count of an id given in its encoded form (byte
// offset of its packed word << 5 | its bit position in the word); returns
// the count it held before.
template <int BITS, bool ZB = false>
__device__ __forceinline__ uint32_t bump(uint32_t *cnt, uint32_t enc) {
    const uint32_t sh = enc & 31u;
    const uint32_t old = __hip_atomic_fetch_add(count_word<ZB>(cnt, enc >> 5), 1u << sh, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
    return (old >> sh) & ((1u << BITS) - 1u);
}

// The same increment when the old count is not needed.
template <int BITS, bool ZB = false>
__device__ __forceinline__ void bump_add(uint32_t *cnt, uint32_t enc) {
    __hip_atomic_fetch_add(count_word<ZB>(cnt, enc >> 5), 1u << (enc & 31u), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Level transitions seen by one lane.  Byte c of lo (c < 8) or of hi (c >=
// 8) counts the bumps that found a count of c.  An id's count rises by one
// per bump, so the ids whose final count is >= v are exactly the bumps that
// found v - 1: the tile's level histogram is the sum of these bytes over
// all lanes, with no pass over the counts.  HI: counts of 8 and more occur
// (Ns > 8).  A byte holds at most 255: the walk flushes before that.
template <bool HI>
struct Trans {
    uint64_t lo, hi;
    __device__ __forceinline__ void add(uint32_t c) {
        const uint64_t inc = 1ull << ((c & 7u) << 3);
        if (!HI || c < 8u)
            lo += inc;
        else
            hi += inc;
    }
};

// Adds the wavefront's transitions to hsum[c + 1] ("ids with count >=
// c + 1") and clears them.  Bytes are spread to 16-bit fields first; a
// field's wavefront sum is at most 64 * 255 and cannot carry.
__device__ __forceinline__ void trans_fold(uint64_t x, int base, uint32_t *hsum, int lane) {
    const uint64_t ev = x & 0x00FF00FF00FF00FFull, od = (x >> 8) & 0x00FF00FF00FF00FFull;
    const uint32_t s0 = wave_sum_u32(static_cast<uint32_t>(ev)), s1 = wave_sum_u32(static_cast<uint32_t>(ev >> 32));
    const uint32_t s2 = wave_sum_u32(static_cast<uint32_t>(od)), s3 = wave_sum_u32(static_cast<uint32_t>(od >> 32));
    if (lane == 0) {
        const uint32_t v[8] = {s0 & 0xffffu, s2 & 0xffffu, s0 >> 16, s2 >> 16,
                               s1 & 0xffffu, s3 & 0xffffu, s1 >> 16, s3 >> 16};
#pragma unroll
        for (int c = 0; c < 8; c++)
            if (v[c]) atomicAdd(&hsum[base + c + 1], v[c]);
    }
}

template <bool HI>
__device__ __forceinline__ void trans_flush(Trans<HI> &T, uint32_t *hsum, int lane) {
    if (__any(T.lo != 0ull)) trans_fold(T.lo, 0, hsum, lane);
    if (HI && __any(T.hi != 0ull)) trans_fold(T.hi, 8, hsum, lane);
    T.lo = T.hi = 0ull;
}

// Byte masks of the counts >= v held in a packed word: bit 7 of byte b of
// m0 (and, for nibbles, of m1) is set when that count is >= v.  For bytes
// b, b >= v exactly when bit 7 of (b | 0x80) - v is set (no borrow: b, v <=
// 16).  Nibbles are first spread into bytes: m0 covers the even nibbles
// (nibble 2b in byte b), m1 the odd ones (nibble 2b+1 in byte b).
template <int BITS>
__device__ __forceinline__ void ge_masks(uint32_t w, uint32_t v, uint32_t &m0, uint32_t &m1) {
    const uint32_t vv = v * 0x01010101u;
    if (BITS == 8) {
        m0 = ((w | 0x80808080u) - vv) & 0x80808080u;
        m1 = 0u;
    } else {
        m0 = (((w & 0x0F0F0F0Fu) | 0x80808080u) - vv) & 0x80808080u;
        m1 = ((((w >> 4) & 0x0F0F0F0Fu) | 0x80808080u) - vv) & 0x80808080u;
    }
}

// One round of a wavefront's walk: windows w0 + u*CT_WAVES (u < CT_UNROLL)
// of the current position segment, one position (group) per lane and
// window; the groups are loaded into id[] (all 0xffffffff where the position
// lies past the segment).  The lane's slice is the window's first slice s0 (window table)
// plus the number of slices starting after the window's first position and
// at or before the lane's: the bits below the lane in the window's 64-bit
// word of the start bitmap (stored one position down), one masked count.  GUARD: some windows or positions of
// the round lie past the segment; otherwise no lane needs a bounds test.
template <bool GUARD, int NT = CT_BLOCK>
__device__ __forceinline__ void walk_load(const CountArgs &a, const CountLds &L, uint32_t seg,
                                          uint32_t seg_end, uint32_t nwin, uint32_t tne, uint32_t w0,
                                          int lane, uint4 (&id)[CT_UNROLL]) {
    constexpr int CT_WAVES = NT / WAVE;
    uint32_t e[CT_UNROLL];
#pragma unroll
    for (int u = 0; u < CT_UNROLL; u++) {
        const uint32_t wi = w0 + u * CT_WAVES;
        uint32_t s0 = 0u, mlo = 0u, mhi = 0u;
        if (!GUARD || wi < nwin) {
            // uniform addresses: every lane reads the same entries
            s0 = L.wt[wi];
            const uint2 m = reinterpret_cast<const uint2 *>(L.sb)[wi];
            mlo = m.x;
            mhi = m.y;
        }
        e[u] = __builtin_amdgcn_mbcnt_hi(mhi, __builtin_amdgcn_mbcnt_lo(mlo, s0));
    }
#pragma unroll
    for (int u = 0; u < CT_UNROLL; u++) e[u] = L.dl[GUARD ? min(e[u], tne - 1u) : e[u]];
#pragma unroll
    for (int u = 0; u < CT_UNROLL; u++) {
        const uint32_t p = seg + (w0 + u * CT_WAVES) * WAVE + static_cast<uint32_t>(lane);
        if (GUARD) {
            id[u] = make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu);
            if (p < seg_end) id[u] = load_group(a.ids, e[u] + p);
        } else {
            id[u] = load_group(a.ids, e[u] + p);
        }
    }
}

// The LDS increments of one round (groups of 0xffffffff skipped when
// GUARD); TR: the old counts feed the level transitions, except those of
// the pads (codes at or above lim, the dummy words).
template <int BITS, bool HI, bool TR, bool ZB>
__device__ __forceinline__ void bump_one(const CountLds &L, uint32_t enc, uint32_t lim, Trans<HI> &tr) {
    if (TR) {
        const uint32_t old = bump<BITS, ZB>(L.cnt, enc);
        if (enc < lim) tr.add(old);
    } else {
        bump_add<BITS, ZB>(L.cnt, enc);
    }
}

template <int BITS, bool HI, bool GUARD, bool TR, bool ZB>
__device__ __forceinline__ void walk_bump(const CountLds &L, const uint4 (&id)[CT_UNROLL], uint32_t lim,
                                          Trans<HI> &tr) {
#pragma unroll
    for (int u = 0; u < CT_UNROLL; u++) {
        if (!GUARD || id[u].x != 0xffffffffu) {
            bump_one<BITS, HI, TR, ZB>(L, id[u].x, lim, tr);
            bump_one<BITS, HI, TR, ZB>(L, id[u].y, lim, tr);
            bump_one<BITS, HI, TR, ZB>(L, id[u].z, lim, tr);
            bump_one<BITS, HI, TR, ZB>(L, id[u].w, lim, tr);
        }
    }
}

// The re-walk of a sparse tile: for each id of the walk once more, an
// atomic AND takes its count and clears it, so only an id's first visit sees
// its final count c; ids with c >= lv are listed as c << shift | id (tile
// base id0) and their levels tallied in L.lsum.  Per window, the four ANDs
// of a lane are issued before any result is used, so their LDS round trips
// overlap (a pad ANDs all ones into a dummy word of its lane: no change; the
// round's windows at or past nwin, all empty, take none), and one
// reservation on L.lcnt per wavefront places the window's listed ids in lane
// order (only the first lcap are stored).  Every lane of the wavefront calls
// it (wr is the round's first window).
template <int BITS, bool ZB, int NT = CT_BLOCK>
__device__ __forceinline__ void walk_take(const CountLds &L, const uint4 (&id)[CT_UNROLL], uint32_t lim,
                                          uint32_t lv, uint32_t *dst, uint32_t lcap, int shift, uint32_t id0,
                                          int lane, uint32_t wr, uint32_t nwin) {
    constexpr int CT_WAVES = NT / WAVE;
    constexpr uint32_t CMASK = (1u << BITS) - 1u;
    const uint32_t dummy = (lim >> 5) + 4u * static_cast<uint32_t>(lane % static_cast<int>(CT_DUMMY));
#pragma unroll
    for (int u = 0; u < CT_UNROLL; u++) {
        if (wr + static_cast<uint32_t>(u * CT_WAVES) >= nwin) break;  // uniform over the wavefront
        const uint32_t e[4] = {id[u].x, id[u].y, id[u].z, id[u].w};
        uint32_t c[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const bool real = e[j] < lim;  // pads and the guard value lie at or above lim
            const uint32_t off = real ? (e[j] >> 5) : dummy;
            const uint32_t keep = real ? ~(CMASK << (e[j] & 31u)) : 0xffffffffu;
            c[j] = __hip_atomic_fetch_and(count_word<ZB>(L.cnt, off), keep, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        uint32_t ne = 0u;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            c[j] = e[j] < lim ? (c[j] >> (e[j] & 31u)) & CMASK : 0u;
            ne += (c[j] >= lv && c[j] != 0u) ? 1u : 0u;
        }
        const uint32_t inc = wave_incl_scan_u32(ne, lane);
        const uint32_t tot = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(inc), WAVE - 1));
        if (tot == 0u) continue;
        uint32_t at = 0u;
        if (lane == 0) at = atomicAdd(L.lcnt, tot);
        uint32_t pos = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(at))) + inc - ne;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (c[j] >= lv && c[j] != 0u) {
                atomicAdd(&L.lsum[c[j]], 1u);
                const uint32_t tid = ((e[j] >> 5) * 8u + (e[j] & 31u)) / BITS;  // id within the tile
                if (pos < lcap) dst[pos] = (c[j] << shift) | (id0 + tid);
                pos++;
            }
        }
    }
}

// Re-walk (XL) only where it reads fewer words than the full scan of the
// tile's counts: positions (groups of four ids) * RW_DENSITY <= 16-byte words.
constexpr uint32_t RW_DENSITY = 4;

// Counts the collisions of tile t of query q into L.cnt and, with TR, adds
// the tile's "count >= v" totals to hsum[v] (hsum zeroed by the caller
// before; complete after the caller's next barrier).  clear: zero the counts
// first (else they are zero already).  XL with xl_dst: when the walk is one
// chunk and one segment and sparse (RW_DENSITY), also lists the ids with
// count >= lv into xl_dst (walk_take; L.lcnt receives their number, L.lsum
// their levels, lsum zeroed by the caller) and leaves every count zero;
// returns whether it did.
template <int BITS, bool HI, bool TR = true, bool XL = false, bool ZB = false, int NT = CT_BLOCK>
__device__ __forceinline__ bool count_tile(const CountArgs &a, int q, int t, const CountLds &L, uint32_t *hsum,
                                           uint32_t *xl_dst = nullptr, uint32_t xl_cap = 0u, int xl_shift = 0,
                                           uint32_t lv = 0u, bool clear = true) {
    constexpr int CT_BLOCK = NT, CT_WAVES = NT / WAVE, CT_CHUNK = NT, CT_WT = NT / 2;
    static_assert(2 * CT_WT <= CT_CHUNK + 1 && CT_CHUNK % 2 == 0, "the start bitmap must fit its region");
    const int vec = a.W * BITS / 128;  // 16-byte words of counts
    if (clear)
        for (int i = threadIdx.x; i < vec; i += CT_BLOCK)
            reinterpret_cast<uint4 *>(L.cnt)[i] = make_uint4(0u, 0u, 0u, 0u);
    if (XL && threadIdx.x == 0) *L.lcnt = 0u;
    // (the counts are cleared before the barriers ahead of the walk)
    bool rw = XL && xl_dst != nullptr;
    const int totalP = static_cast<int>(a.ftot[q]);
    const int32_t *fq = a.flat + static_cast<int64_t>(q) * a.Ns * a.K;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    Trans<HI> tr{0ull, 0ull};
    int held = 0;  // bound on any byte of tr: bumps per lane since the last flush
    constexpr int PER_ROUND = 4 * CT_UNROLL;  // bumps per lane and round
    const uint32_t lim = (static_cast<uint32_t>(a.W) * BITS / 8u) << 5;  // first pad code
    for (int c0 = 0; c0 < totalP; c0 += CT_CHUNK) {
        const int nsl = min(CT_CHUNK, totalP - c0);
        // the start bitmap of the chunk's first segment, cleared ahead of the
        // slice barriers below (its last reader, the previous walk, ended at
        // a barrier)
        for (int i = threadIdx.x; i < 2 * CT_WT; i += CT_BLOCK) L.sb[i] = 0u;
        // this thread's slice
        uint32_t len = 0u, st = 0u;
        if (static_cast<int>(threadIdx.x) < nsl) {
            const int64_t row = fq[c0 + static_cast<int>(threadIdx.x)];
            const uint2 se = reinterpret_cast<const uint2 *>(a.off2d)[static_cast<int64_t>(t) * a.Ns * a.K + row];
            st = se.x;
            len = se.y - se.x;
        }
        // compacted index and first position of each non-empty slice
        const uint32_t ne = len > 0u ? 1u : 0u;
        uint32_t ci, p0, tne, tpos;
        if (nsl <= WAVE) {
            // every slice in wavefront 0: its scans alone, the totals through LDS
            uint32_t ine = 0u, ipos = 0u;
            if (wave == 0) {
                ine = wave_incl_scan_u32(ne, lane);
                ipos = wave_incl_scan_u32(len, lane);
                if (len > 0u) L.dl[ine - ne] = st - (ipos - len);
                if (lane == WAVE - 1) {
                    L.wsum[0] = ine;
                    L.wsum[1] = ipos;
                }
            }
            ci = ine - ne;
            p0 = ipos - len;
            __syncthreads();
            tne = L.wsum[0];
            tpos = L.wsum[1];
        } else {
            const uint32_t ine = wave_incl_scan_u32(ne, lane), ipos = wave_incl_scan_u32(len, lane);
            if (lane == WAVE - 1) {
                L.wsum[wave] = ine;
                L.wsum[CT_WAVES + wave] = ipos;
            }
            __syncthreads();
            // lane w holds wavefront w's totals; sums over the lanes below this
            // wavefront's index give its offsets, over all lanes the chunk's totals
            const uint32_t x1 = lane < CT_WAVES ? L.wsum[lane] : 0u;
            const uint32_t x2 = lane < CT_WAVES ? L.wsum[CT_WAVES + lane] : 0u;
            const uint32_t bne = wave_sum_u32(lane < wave ? x1 : 0u), bpos = wave_sum_u32(lane < wave ? x2 : 0u);
            tne = wave_sum_u32(x1);
            tpos = wave_sum_u32(x2);
            ci = bne + ine - ne;
            p0 = bpos + ipos - len;
            if (len > 0u) L.dl[ci] = st - p0;
            __syncthreads();
        }
        if (XL)
            rw = rw && c0 == 0 && totalP <= CT_CHUNK && tpos <= static_cast<uint32_t>(CT_WT * WAVE) &&
                 tpos * RW_DENSITY <= static_cast<uint32_t>(vec);
        for (uint32_t seg = 0; seg < tpos; seg += CT_WT * WAVE) {
            const uint32_t seg_end = min(tpos, seg + static_cast<uint32_t>(CT_WT * WAVE));
            if (seg != 0u) {  // (the first segment's bitmap was cleared before the slice barriers)
                for (int i = threadIdx.x; i < 2 * CT_WT; i += CT_BLOCK) L.sb[i] = 0u;
                __syncthreads();
            }
            // window table and start bitmap of this segment: every window
            // start (a multiple of 64) lies in exactly one non-empty slice
            if (len > 0u) {
                const uint32_t lo_p = max(p0, seg), hi_p = min(p0 + len, seg_end);
                for (uint32_t wp = (lo_p + WAVE - 1) / WAVE * WAVE; wp < hi_p; wp += WAVE)
                    L.wt[(wp - seg) / WAVE] = static_cast<uint16_t>(ci);
                if (p0 > seg && p0 < seg_end) atomicOr(&L.sb[(p0 - seg - 1) / 32], 1u << ((p0 - seg - 1) % 32));
            }
            __syncthreads();
            const uint32_t nwin = (seg_end - seg + WAVE - 1) / WAVE;
            const uint32_t nfull = (seg_end - seg) / WAVE;  // windows with all 64 positions in range
            constexpr uint32_t STRIDE = CT_WAVES * CT_UNROLL, SPAN = (CT_UNROLL - 1) * CT_WAVES;
            // rounds whose windows all lie in [0, nfull): software-pipelined,
            // the next round's ids are in flight during this round's
            // increments; two buffers take turns (no copies between rounds)
            uint32_t w0 = static_cast<uint32_t>(wave);
            uint4 id[CT_UNROLL], id2[CT_UNROLL];
            bool have = w0 + SPAN < nfull;
            if (have) walk_load<false, NT>(a, L, seg, seg_end, nwin, tne, w0, lane, id);
            while (have) {
                uint32_t wn = w0 + STRIDE;
                bool nhave = wn + SPAN < nfull;
                if (nhave) walk_load<false, NT>(a, L, seg, seg_end, nwin, tne, wn, lane, id2);
                if (TR && held > 255 - PER_ROUND) {
                    trans_flush<HI>(tr, hsum, lane);
                    held = 0;
                }
                held += PER_ROUND;
                walk_bump<BITS, HI, false, TR, ZB>(L, id, lim, tr);
                w0 = wn;
                if (!nhave) break;
                wn = w0 + STRIDE;
                nhave = wn + SPAN < nfull;
                if (nhave) walk_load<false, NT>(a, L, seg, seg_end, nwin, tne, wn, lane, id);
                if (TR && held > 255 - PER_ROUND) {
                    trans_flush<HI>(tr, hsum, lane);
                    held = 0;
                }
                held += PER_ROUND;
                walk_bump<BITS, HI, false, TR, ZB>(L, id2, lim, tr);
                w0 = wn;
                have = nhave;
            }
            // the segment's last round(s), bounds-tested
            for (; w0 < nwin; w0 += STRIDE) {
                if (TR && held > 255 - PER_ROUND) {
                    trans_flush<HI>(tr, hsum, lane);
                    held = 0;
                }
                held += PER_ROUND;
                walk_load<true, NT>(a, L, seg, seg_end, nwin, tne, w0, lane, id);
                walk_bump<BITS, HI, true, TR, ZB>(L, id, lim, tr);
            }
            __syncthreads();
            if (XL && rw) {
                // the only segment: list the tile's ids with count >= lv and
                // clear every count the walk raised
                const uint32_t id0 = static_cast<uint32_t>(t) * static_cast<uint32_t>(a.W);
                for (uint32_t wr = static_cast<uint32_t>(wave); wr < nwin; wr += STRIDE) {
                    walk_load<true, NT>(a, L, seg, seg_end, nwin, tne, wr, lane, id);
                    walk_take<BITS, ZB, NT>(L, id, lim, lv, xl_dst, xl_cap, xl_shift, id0, lane, wr, nwin);
                }
                __syncthreads();
            }
        }
    }
    if (TR) trans_flush<HI>(tr, hsum, lane);
    return rw;
}

// Output of the staged lists: slot j of the query's list receives the
// staged value v (the id itself in the candidate lists).
// Candidate slot writer.  The positions come from an atomic counter; the
// selection decides from the level histogram that |C| <= cap, but a count
// the histogram disagrees with (the fused kernel after a timed-out wait,
// which sets the error word) must not write past the query's cap slots.
struct CandOut {
    int32_t *cq;
    uint32_t cap;
    __device__ __forceinline__ void operator()(uint32_t j, uint32_t v) const {
        if (j < cap) cq[j] = static_cast<int32_t>(v);
    }
};

// A query's candidate count as the later kernels read it: at most its slots.
__device__ __forceinline__ int64_t cand_n(const uint32_t *cand_count, int q, int64_t cap) {
    return min(static_cast<int64_t>(cand_count[q]), cap);
}

// Move a wavefront's staged entries to the query's list: one atomic to
// reserve the range, then coalesced stores.
template <typename Out>
__device__ __forceinline__ void flush_stage(uint32_t *stage, uint32_t &scount, uint32_t *counter,
                                            const Out &out, int lane) {
    wave_sync_lds();
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(counter, scount);
    base = __shfl(base, 0, WAVE);
    for (uint32_t i = lane; i < scount; i += WAVE) out(base + i, stage[i]);
    wave_sync_lds();
    scount = 0;
}

// Appends the entries flagged in a lane's NM masks (bit 8b+7 of mask i
// flags entry id_of(i, b)) to the query's list, in lane order: an exclusive
// prefix sum over the wavefront places each lane's entries, which go to the
// wavefront's LDS stage of CAP slots, or straight to the list (one
// reservation) when they outnumber the stage.
template <int CAP, int NM, typename IdOf, typename Out>
__device__ __forceinline__ void append_flagged(const uint32_t (&m)[NM], IdOf id_of, uint32_t *stage,
                                               uint32_t &scount, uint32_t *counter, const Out &out,
                                               int lane) {
    uint32_t cnt = 0u;
#pragma unroll
    for (int i = 0; i < NM; i++) cnt += static_cast<uint32_t>(__popc(m[i]));
    const uint32_t inc = wave_incl_scan_u32(cnt, lane);
    const uint32_t total = static_cast<uint32_t>(__builtin_amdgcn_readlane(inc, WAVE - 1));
    if (total == 0u) return;
    uint32_t j = inc - cnt;
    if (scount + total > static_cast<uint32_t>(CAP)) flush_stage(stage, scount, counter, out, lane);
    if (total <= static_cast<uint32_t>(CAP)) {
        j += scount;
#pragma unroll
        for (int i = 0; i < NM; i++) {
            uint32_t mm = m[i];
            while (mm != 0u) {
                const int bit = __builtin_ctz(mm);
                mm &= mm - 1u;
                stage[j++] = id_of(i, bit >> 3);
            }
        }
        scount += total;
        wave_sync_lds();
    } else {
        uint32_t base = 0u;
        if (lane == 0) base = atomicAdd(counter, total);
        base = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(base));
        j += base;
#pragma unroll
        for (int i = 0; i < NM; i++) {
            uint32_t mm = m[i];
            while (mm != 0u) {
                const int bit = __builtin_ctz(mm);
                mm &= mm - 1u;
                out(j++, id_of(i, bit >> 3));
            }
        }
    }
}

struct SelectArgs {
    const uint32_t *hist;    // [nq][Ns+1], levels >= 1 filled by k_count
    int64_t R;               // floor(beta*n)
    int rule;                // 0 printed, 1 prose
    int64_t cap;             // candidate slots per query
    int32_t *cand;           // [nq][cap]
    uint32_t *cand_count;    // [nq]
    uint8_t *dump_sc;        // [nq][n] or null
    int32_t *dump_last;      // [nq] or null
    int64_t *dump_hist;      // [nq][Ns+1] or null
    const uint32_t *redo;    // null: query blockIdx.y; else the queue of ListArgs::redo
    uint32_t *ovf;           // [0] queries whose candidates outgrow cap, [1 + i] the queue
};

// Ids scoring at least `last` (every id when last <= 0).
__device__ __forceinline__ int64_t count_at_least(const uint32_t *h, int Ns, int64_t n, int last) {
    if (last <= 0) return n;
    int64_t c = 0;
    for (int v = last; v <= Ns; v++) c += h[v];
    return c;
}

// Alg 5 keeps the whole threshold level, so |C| = S(last) can exceed R and
// the call's cap slots: such a query is queued for k_stream_topk, which
// needs no slots.  The fixed-budget rule takes exactly min(R, ...) <= cap.
__device__ __forceinline__ bool outgrows(const SelectArgs &sa, const uint32_t *h, int Ns, int64_t n, int last) {
    return sa.rule != 2 && count_at_least(h, Ns, n, last) > sa.cap;
}

// Alg 5's threshold (Section 4.3) from the level histogram (level 0 = n
// minus the others).  With S(v) the number of points scoring at least v,
// the threshold is the highest level at which the re-rank budget R is
// exceeded: h[v] + S(v) > R as the algorithm prints its test (rule 0), or
// S(v) > R as the text states it (rule 1); -1 when no level exceeds it.
// Rule 2, the fixed budget (the R highest SC-scores, ties by lower id):
// the boundary level L is the highest level with S(L) >= R; the result is
// L + 1, every point above L is a candidate, and k_select_level adds the
// first R - S(L + 1) points of level L in id order.
__device__ int select_threshold(const uint32_t *h, int Ns, int64_t n, int64_t R, int rule) {
    int64_t above0 = 0;
    for (int v = 1; v <= Ns; v++) above0 += h[v];
    int64_t S = 0;  // S(v), built from the top level down
    for (int v = Ns; v >= 0; v--) {
        const int64_t hv = v == 0 ? n - above0 : static_cast<int64_t>(h[v]);
        S += hv;
        if (rule == 2) {
            if (S >= R) return v + 1;
        } else if ((rule == 1 ? S : hv + S) > R) {
            return v;
        }
    }
    return rule == 2 ? 0 : -1;
}

__device__ __forceinline__ void dump_threshold(int32_t *dump_last, int64_t *dump_hist, int q, int Ns,
                                               int64_t n, const uint32_t *h, int last) {
    if (dump_last) dump_last[q] = last;
    if (dump_hist) {
        int64_t above0 = 0;
        for (int v = 1; v <= Ns; v++) above0 += h[v];
        dump_hist[static_cast<int64_t>(q) * (Ns + 1)] = n - above0;
        for (int v = 1; v <= Ns; v++) dump_hist[static_cast<int64_t>(q) * (Ns + 1) + v] = h[v];
    }
}

// List selection.  With a list level Lv, counting also lists every id of
// the tile whose count reaches Lv in the tile's own lcap slots of the
// query's list (the query's packed-count row, idle in this form: lcap =
// W*BITS/32 words per tile), as one word count << shift | id (shift = 31 -
// bit width of Ns; the loader's bound Ns*n < 2^30 leaves room for both),
// the number of such ids in tcount[q][t] (also past lcap), and adds the
// levels of the listed ids to hist[q] (exact for every level >= Lv).
// Alg 5's threshold `last` follows from the level histogram alone, in a
// launch of its own once every tile is counted: when last >= Lv and no
// tile's list overflowed, the candidates are exactly the listed ids with
// count >= last; other queries are queued, counted again with their packed
// counts stored (CT_REDO) and take the streaming selection.  The level is
// fixed, or adapted on the device from batch to batch: up when more than
// 1/16 of a batch overflowed a tile's list, else down when more than 1/64
// was queued for last < Lv, up when at least 255/256 had last > Lv.
// Results never depend on it.
enum CountForm { CT_STORE = 0, CT_LIST = 1, CT_REDO = 2 };

struct ListArgs {
    int fixed;          // list level if > 0, else the adaptive level *level
    uint32_t *level;    // adaptive level, kept on the device across batches
    int shift;          // a listed word is count << shift | id
    int nq;             // queries in the batch
    int64_t cap;        // candidate slots per query (>= floor(beta*n) or n)
    int64_t lcap;       // list slots per tile
    uint32_t *list;     // [nq][T][lcap] the lists, tile after tile
    int32_t *cand;      // [nq][cap] the candidates
    uint32_t *count;    // [nq] candidate counts
    uint32_t *tcount;   // [nq][T] ids with count >= the list level in each tile
    int T, W;           // tiles per query, ids per tile
    uint32_t *redo;     // [0] queued queries, [1] queries with last > level, [2] queued
                        // because a tile's list overflowed, [3 + i] the queue
    int64_t R;          // floor(beta*n)
    int rule;           // Alg 5 reading
    int redo_hist;      // the recount adds the queued queries' level counts
    int32_t *dump_last; // [nq] or null
    int64_t *dump_hist; // [nq][Ns+1] or null
    uint32_t *toff;     // [nq][T+1] first candidate of each tile, or null (see k_list_select)
    uint32_t *tlev;     // [nq][T][Ns+1] listed ids per tile and level (levels >= the list
                        // level; 0 below), or null
};

__device__ __forceinline__ uint32_t list_level(const ListArgs &la) {
    return la.fixed > 0 ? static_cast<uint32_t>(la.fixed) : *la.level;
}

// Flags of the packed counts >= lv (1 <= lv <= Ns) in one word: the top bit
// of each nibble or byte.  Nibbles of counts <= 8 take one add (v + 8 - lv
// stays below 16); with counts up to 15 the low three bits are tested apart
// from the 8s bit; bytes take the borrow-free subtraction.
template <int BITS, bool HI>
__device__ __forceinline__ uint32_t flag_counts(uint32_t w, uint32_t lv) {
    if (BITS == 8) return ((w | 0x80808080u) - lv * 0x01010101u) & 0x80808080u;
    if (!HI) return (w + (8u - lv) * 0x11111111u) & 0x88888888u;
    const uint32_t h = w & 0x88888888u, t = w & 0x77777777u;
    return lv <= 8u ? (h | ((t + (8u - lv) * 0x11111111u) & 0x88888888u))
                    : (h & ((t + (16u - lv) * 0x11111111u) & 0x88888888u));
}

// Lists the tile's ids with count >= lv in the tile's lcap slots of the
// query's list, and tallies their levels in lsum; tcount receives how many
// there are, also when more than lcap (then only the first lcap are stored
// and the selection queues the query for the recount).  Each thread tests the 16 packed
// words it owns per pass (four
// 16-byte words), keeping only the number of flagged ids and a 16-bit mask
// of the words holding any; a prefix sum over the workgroup places them (no
// atomics: the T tiles of a query write disjoint ranges), and only the
// flagged words are read again from LDS to extract their ids.  Ids past n
// hold 0 and lv >= 1, so none is listed.  wsum: CT_WAVES words of LDS.
template <int BITS, bool HI, int NT = CT_BLOCK>
__device__ __forceinline__ void list_tile(const ListArgs &la, const uint32_t *cnt, uint32_t *wsum, uint32_t *lsum,
                                          int vec, int q, int t, int W, uint32_t lv, int wave, int lane) {
    constexpr int CT_BLOCK = NT, CT_WAVES = NT / WAVE;
    constexpr int PER_WORD = 32 / BITS;
    constexpr uint32_t CMASK = (1u << BITS) - 1u;
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 *c4v = reinterpret_cast<const u32x4 *>(cnt);
    uint32_t *dst = la.list + (static_cast<int64_t>(q) * la.T + t) * la.lcap;
    const uint32_t base = static_cast<uint32_t>(t) * static_cast<uint32_t>(W);
    const uint32_t lim = static_cast<uint32_t>(la.lcap);
    uint32_t run = 0u;  // entries of this tile placed so far
    for (int i0 = 0; i0 < vec; i0 += 4 * CT_BLOCK) {
        uint32_t c = 0u, nz = 0u;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int i = i0 + k * CT_BLOCK + static_cast<int>(threadIdx.x);
            u32x4 v = {0u, 0u, 0u, 0u};
            if (i < vec) v = c4v[i];
            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t f = flag_counts<BITS, HI>(wv[e], lv);
                c += static_cast<uint32_t>(__popc(f));
                nz |= min(f, 1u) << (4 * k + e);
            }
        }
        const uint32_t inc = wave_incl_scan_u32(c, lane);
        if (lane == WAVE - 1) wsum[wave] = inc;
        __syncthreads();
        // lane x holds wavefront x's total: the sum below this wavefront is
        // its offset, the sum of all the pass's total
        const uint32_t xt = lane < CT_WAVES ? wsum[lane] : 0u;
        const uint32_t before = wave_sum_u32(lane < wave ? xt : 0u), tot = wave_sum_u32(xt);
        uint32_t j = run + before + inc - c;
        run += tot;
        while (nz != 0u) {
            const int x = __builtin_ctz(nz);
            nz &= nz - 1u;
            // 32-bit word e of 16-byte word k of this thread
            const int word = (i0 + (x >> 2) * CT_BLOCK + static_cast<int>(threadIdx.x)) * 4 + (x & 3);
            const uint32_t wv = cnt[word];
            uint32_t mm = flag_counts<BITS, HI>(wv, lv);
            const uint32_t id0 = base + static_cast<uint32_t>(word * PER_WORD);
            do {
                const int sub = __builtin_ctz(mm) / BITS;
                mm &= mm - 1u;
                const uint32_t cv = (wv >> (BITS * sub)) & CMASK;
                atomicAdd(&lsum[cv], 1u);
                if (j < lim) dst[j] = (cv << la.shift) | (id0 + static_cast<uint32_t>(sub));
                j++;
            } while (mm != 0u);
        }
        if (i0 + 4 * CT_BLOCK < vec) __syncthreads();  // wsum is rewritten by the next pass
    }
    if (threadIdx.x == 0) la.tcount[static_cast<int64_t>(q) * la.T + t] = run;
}

// grid (T, nq) (CT_REDO: (T, any)), block CT_BLOCK, dynamic LDS
// count_lds_size(W, BITS).  CT_STORE: adds the tile's level counts to
// hist[q] and stores the packed counts to sc[q][t] (W*BITS/8 bytes).
// CT_LIST: lists the ids with count >= the list level, and with TR adds the
// level counts (stage dumps; the list selection needs only the levels >=
// the list level, which the list holds); the packed counts are stored too
// when sc is given.  CT_REDO: for each queued query, stores the packed
// counts and, with la.redo_hist, adds its level counts; workgroup (0, 0)
// also moves the adaptive level.
// NT threads per workgroup: 1024 (eight waves per SIMD, 64 VGPRs) or 768
// (six, 80 VGPRs: the multi-query list form then spills nothing).
template <int BITS, bool HI, int MODE, bool TR, bool MULTI, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 768 ? 6 : 8))) void k_count(
    CountArgs a, uint32_t *__restrict__ hist, uint4 *__restrict__ sc, ListArgs la) {
    constexpr int CT_BLOCK = NT;
    // no static LDS: the packed counts start at address 0, so an increment's
    // byte offset is its address
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const CountLds L = carve<BITS, NT>(lds_raw, a.W);
    uint32_t *hsum = L.hsum, *lsum = L.lsum;
    // (tile t, query row group gy).  In XCD order (a.xper > 0) the T x G units
    // are numbered tile-major and cut into 8 runs of xper, one per XCD: the
    // dispatcher deals consecutive workgroups to the 8 XCDs in turn, so
    // workgroup b runs on XCD b % 8 and takes unit (b % 8)*xper + b/8.  The
    // workgroups an XCD holds at once then share one or two tiles, whose
    // lists and slice table stay in that XCD's L2.
    int t = static_cast<int>(blockIdx.x), gy = static_cast<int>(blockIdx.y);
    if (MODE != CT_REDO && a.xper > 0) {
        const uint32_t groups = static_cast<uint32_t>(MULTI ? (a.nq + a.qpw - 1) / a.qpw : a.nq);
        const uint32_t u = (blockIdx.x % 8u) * static_cast<uint32_t>(a.xper) + blockIdx.x / 8u;
        if (u >= groups * static_cast<uint32_t>(a.T)) return;  // the padding of the last run
        t = static_cast<int>(u / groups);
        gy = static_cast<int>(u % groups);
    }
    const int lane = threadIdx.x % WAVE;
    const int vec = a.W * BITS / 128;  // 16-byte words per tile
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 *c4v = reinterpret_cast<const u32x4 *>(L.cnt);
    // MULTI: a.qpw queries per workgroup, one after the other (fewer,
    // longer-lived workgroups where tiles hold few ids each); otherwise one
    uint32_t nrun = MULTI ? static_cast<uint32_t>(a.qpw) : 1u, f0 = 0u, fstep = 1u;
    if (MODE == CT_REDO) {
        nrun = la.redo[0];
        f0 = blockIdx.y;
        fstep = gridDim.y;
        if (la.fixed == 0 && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
            const uint32_t lv = *la.level, nf = la.redo[0], na = la.redo[1], no = la.redo[2];
            const uint32_t nq = static_cast<uint32_t>(la.nq);
            uint32_t nl = lv;
            // lists overflowing: list fewer ids; thresholds below the level:
            // list more (a recount costs far more than longer lists); almost
            // all thresholds above it: list fewer
            if (no * 16u > nq && lv < static_cast<uint32_t>(a.Ns))
                nl = lv + 1u;
            else if ((nf - no) * 64u > nq && lv > 1u)
                nl = lv - 1u;
            else if (na * 256u >= nq * 255u && lv < static_cast<uint32_t>(a.Ns))
                nl = lv + 1u;
            if (nl != lv) *la.level = nl;
        }
    }
    // the list form lists sparse tiles during a re-walk that also clears the
    // counts (then the next query of this workgroup skips the clear); with
    // the packed counts stored (stage dumps) it scans instead
    constexpr bool XL = MODE == CT_LIST;
    const bool xl = XL && sc == nullptr;
    bool clean = false;
    for (uint32_t f = f0; f < nrun; f += fstep) {
        const int row = MULTI ? gy * a.qpw + static_cast<int>(f) : gy;
        if (MULTI && row >= a.nq) break;
        const int q = MODE == CT_REDO ? static_cast<int>(la.redo[3 + f]) : (a.perm ? a.perm[row] : row);
        if (threadIdx.x < 18) hsum[threadIdx.x] = 0u;
        if (MODE == CT_LIST && threadIdx.x < 17) lsum[threadIdx.x] = 0u;
        uint32_t *xl_dst = xl ? la.list + (static_cast<int64_t>(q) * la.T + t) * la.lcap : nullptr;
        const bool listed = count_tile<BITS, HI, TR, XL, true, NT>(a, q, t, L, hsum, xl_dst,
                                                                   static_cast<uint32_t>(la.lcap), la.shift,
                                                                   XL ? list_level(la) : 0u, !clean);
        clean = listed;
        // count_tile ends at a barrier after its last LDS count access; the
        // level transitions (TR) add to hsum after it
        if (TR || !listed) __syncthreads();

        // Level histogram of the tile: hsum[v] = ids with count >= v, so level v
        // holds hsum[v] - hsum[v+1].  Ids past n hold 0 and count nowhere.
        if (TR && (MODE != CT_REDO || la.redo_hist) && threadIdx.x >= 1 && threadIdx.x <= a.Ns) {
            const uint32_t hv = hsum[threadIdx.x] - hsum[threadIdx.x + 1];
            if (hv) atomicAdd(&hist[static_cast<int64_t>(q) * (a.Ns + 1) + threadIdx.x], hv);
        }
        if (MODE != CT_LIST || sc) {
            // streamed past the caches: the id lists should stay resident there
            u32x4 *dstv = reinterpret_cast<u32x4 *>(sc + (static_cast<int64_t>(q) * a.T + t) * vec);
            for (int i = threadIdx.x; i < vec; i += CT_BLOCK) __builtin_nontemporal_store(c4v[i], &dstv[i]);
        }
        if (MODE == CT_LIST) {
            if (listed) {
                if (threadIdx.x == 0) la.tcount[static_cast<int64_t>(q) * la.T + t] = *L.lcnt;
            } else {
                list_tile<BITS, HI, NT>(la, L.cnt, L.wsum, lsum, vec, q, t, a.W, list_level(la),
                                        threadIdx.x / WAVE, lane);
            }
            // a re-walk's level tallies are complete at count_tile's last barrier
            if (!listed) __syncthreads();
            if (threadIdx.x <= static_cast<unsigned>(a.Ns)) {
                const uint32_t c = lsum[threadIdx.x];
                if (la.tlev) la.tlev[(static_cast<int64_t>(q) * a.T + t) * (a.Ns + 1) + threadIdx.x] = c;
                // levels >= the list level: the listed ids are all of them
                if (!TR && threadIdx.x >= 1 && c)
                    atomicAdd(&hist[static_cast<int64_t>(q) * (a.Ns + 1) + threadIdx.x], c);
            }
        }
        // the next query clears the counts and sums read above.  After a
        // re-walk (counts left zero) without transitions, nothing read here
        // is written before the next query's own barriers: lcnt and lsum[v]
        // are cleared by the threads that read them, the rest by count_tile
        // ahead of its barriers
        if (MODE == CT_REDO || (MULTI && (TR || !listed))) __syncthreads();
    }
}


// Streaming pass over the packed counts of one query: Alg 5's threshold from
// the level histogram, then compaction of C = {id : SC[id] >= last} through
// per-wavefront LDS staging.  grid (blocks per query, nq), block SEL_BLOCK;
// each thread reads SEL_UNROLL 16-byte words (128/BITS ids each) per step.
constexpr int SEL_BLOCK = 512;
constexpr int SEL_WAVES = SEL_BLOCK / WAVE;
constexpr int SEL_UNROLL = 4;


template <int BITS>
__device__ __forceinline__ void select_query(const SelectArgs &sa, int Ns, int64_t n, int64_t words4,
                                             const uint4 *__restrict__ sc, int q, uint32_t *stage_all);

// With sa.redo, the queued queries instead (grid (blocks per query, any)).
template <int BITS>
__global__ __launch_bounds__(SEL_BLOCK) void k_select(SelectArgs sa, int Ns, int64_t n,
                                                     int64_t words4, const uint4 *__restrict__ sc) {
    __shared__ uint32_t stage_all[SEL_WAVES * CT_STAGE];
    if (!sa.redo) {
        select_query<BITS>(sa, Ns, n, words4, sc, blockIdx.y, stage_all);
        return;
    }
    const uint32_t nrun = sa.redo[0];
    for (uint32_t f = blockIdx.y; f < nrun; f += gridDim.y)
        select_query<BITS>(sa, Ns, n, words4, sc, static_cast<int>(sa.redo[3 + f]), stage_all);
}

template <int BITS>
__device__ __forceinline__ void select_query(const SelectArgs &sa, int Ns, int64_t n, int64_t words4,
                                             const uint4 *__restrict__ sc, int q, uint32_t *stage_all) {
    constexpr int PER_WORD = 32 / BITS;   // ids per 32-bit word
    constexpr int PER_VEC = 128 / BITS;   // ids per 16-byte word
    const uint32_t *h = sa.hist + static_cast<int64_t>(q) * (Ns + 1);
    const int last = select_threshold(h, Ns, n, sa.R, sa.rule);
    const bool over = outgrows(sa, h, Ns, n, last);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        dump_threshold(sa.dump_last, sa.dump_hist, q, Ns, n, h, last);
        if (over) sa.ovf[1 + atomicAdd(&sa.ovf[0], 1u)] = static_cast<uint32_t>(q);
    }
    if (over && !sa.dump_sc) return;  // (with stage dumps the pass still dumps the counts)
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    int32_t *cq = sa.cand + static_cast<int64_t>(q) * sa.cap;
    uint32_t *stage = stage_all + wave * CT_STAGE;
    uint32_t *counter = sa.cand_count + q;
    uint32_t scount = 0;
    // with last <= 0 every id below n is a candidate: compare against 0
    const uint32_t lv = static_cast<uint32_t>(last > 0 ? last : 0);
    const uint4 *src = sc + static_cast<int64_t>(q) * words4;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * SEL_BLOCK;
    for (int64_t i0 = static_cast<int64_t>(blockIdx.x) * SEL_BLOCK; i0 < words4;
         i0 += stride * SEL_UNROLL) {
        uint4 v[SEL_UNROLL];
#pragma unroll
        for (int u = 0; u < SEL_UNROLL; u++) {
            const int64_t i = i0 + u * stride + threadIdx.x;
            typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
            u32x4 t = {0u, 0u, 0u, 0u};
            if (i < words4) t = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(src) + i);
            v[u] = make_uint4(t.x, t.y, t.z, t.w);
        }
#pragma unroll
        for (int u = 0; u < SEL_UNROLL; u++) {
            const int64_t i = i0 + u * stride + threadIdx.x;
            const bool in = i < words4;
            const int64_t id0 = i * PER_VEC;  // first id held by this 16-byte word
            const uint32_t wv[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
            if (sa.dump_sc && in) {
                for (int b = 0; b < PER_VEC; b++) {
                    if (id0 + b < n)
                        sa.dump_sc[static_cast<int64_t>(q) * n + id0 + b] = static_cast<uint8_t>(
                            (wv[b / PER_WORD] >> (BITS * (b % PER_WORD))) & ((1u << BITS) - 1u));
                }
            }
            // masks 2c+h: word c, even (h = 0) or odd (h = 1) nibbles; bytes: h = 0 only
            uint32_t m[8];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                ge_masks<BITS>(wv[c], lv, m[2 * c], m[2 * c + 1]);
                if (!in || over) m[2 * c] = m[2 * c + 1] = 0u;
            }
            if (in && id0 + PER_VEC > n) {
                // the last word of the last tile: ids past n are padding
#pragma unroll
                for (int i = 0; i < 8; i++)
                    for (int b = 0; b < 4; b++) {
                        const int c = i / 2, hh = i % 2;
                        const int64_t id = id0 + c * PER_WORD + (BITS == 8 ? b : 2 * b + hh);
                        if (id >= n) m[i] &= ~(0x80u << (8 * b));
                    }
            }
            append_flagged<CT_STAGE, 8>(
                m,
                [&](int i, int b) {
                    return static_cast<uint32_t>(id0 + (i / 2) * PER_WORD + (BITS == 8 ? b : 2 * b + (i % 2)));
                },
                stage, scount, counter, CandOut{cq, static_cast<uint32_t>(sa.cap)}, lane);
        }
    }
    if (__any(scount != 0u)) flush_stage(stage, scount, counter, CandOut{cq, static_cast<uint32_t>(sa.cap)}, lane);
}

// Fixed-budget rule, second part: after k_select has listed the points
// above the boundary level L, append the first R - (their number) points of
// level L in id order (ids below n), and set the candidate count.  One
// workgroup per query walks the packed counts in id order, 256 words at a
// time, ranking matches by a workgroup prefix sum; it stops once enough are
// found.  grid nq, block SL_BLOCK; with sa.redo, the queued queries of a
// list selection instead (grid any).
constexpr int SL_BLOCK = 256;
constexpr int SL_VEC = 4;  // 16-byte words per thread and round

template <int BITS>
__device__ __forceinline__ void select_level_query(const SelectArgs &sa, int Ns, int64_t n, int64_t words,
                                                   const uint32_t *__restrict__ sc32, int q, uint32_t *wtot,
                                                   uint32_t &base_s) {
    constexpr int PER_WORD = 32 / BITS;
    constexpr uint32_t MASK = (1u << BITS) - 1u;
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const uint32_t *h = sa.hist + static_cast<int64_t>(q) * (Ns + 1);
    int64_t above0 = 0;
    for (int v = 1; v <= Ns; v++) above0 += h[v];
    int64_t above = 0, need = 0;
    int L = -1;
    for (int v = Ns; v >= 0; v--) {
        const int64_t hv = v == 0 ? n - above0 : static_cast<int64_t>(h[v]);
        if (above + hv >= sa.R) {
            L = v;
            need = sa.R - above;
            break;
        }
        above += hv;
    }
    if (L < 0 || need <= 0) return;  // uniform: nothing to add at the boundary level
    uint32_t *counter = sa.cand_count + q;
    int32_t *cq = sa.cand + static_cast<int64_t>(q) * sa.cap;
    if (tid == 0) base_s = *counter;
    __syncthreads();
    const int64_t base = base_s;
    // words is a multiple of 4 (tiles hold a multiple of 1024 ids): each
    // thread takes SL_VEC consecutive 16-byte words per round, so one
    // workgroup prefix sum ranks SL_VEC * SL_BLOCK words in id order
    const uint4 *src = reinterpret_cast<const uint4 *>(sc32 + static_cast<int64_t>(q) * words);
    const int64_t words4 = words / 4;
    const uint32_t lv = static_cast<uint32_t>(L);
    int64_t taken = 0;
    for (int64_t w0 = 0; w0 < words4 && taken < need; w0 += SL_VEC * SL_BLOCK) {
        const int64_t wt = w0 + static_cast<int64_t>(tid) * SL_VEC;  // this thread's first word
        uint4 v4[SL_VEC];
#pragma unroll
        for (int u = 0; u < SL_VEC; u++) v4[u] = wt + u < words4 ? src[wt + u] : make_uint4(0u, 0u, 0u, 0u);
        uint32_t mb[SL_VEC][4];
        uint32_t cnt = 0u;
#pragma unroll
        for (int u = 0; u < SL_VEC; u++) {
            const uint32_t wv[4] = {v4[u].x, v4[u].y, v4[u].z, v4[u].w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                mb[u][j] = 0u;
#pragma unroll
                for (int k = 0; k < PER_WORD; k++) {
                    const int64_t id = ((wt + u) * 4 + j) * PER_WORD + k;
                    if (wt + u < words4 && id < n && ((wv[j] >> (BITS * k)) & MASK) == lv) mb[u][j] |= 1u << k;
                }
                cnt += static_cast<uint32_t>(__popc(mb[u][j]));
            }
        }
        const uint32_t incl = wave_incl_scan_u32(cnt, lane);
        if (lane == WAVE - 1) wtot[w] = incl;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int i = 0; i < SL_BLOCK / WAVE; i++) {
            before += i < w ? wtot[i] : 0u;
            total += wtot[i];
        }
        int64_t r = taken + before + incl - cnt;
        if (cnt != 0u && r < need) {
#pragma unroll
            for (int u = 0; u < SL_VEC; u++)
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    uint32_t mbits = mb[u][j];
                    while (mbits) {
                        const int k = __ffs(mbits) - 1;
                        mbits &= mbits - 1u;
                        if (r < need && base + r < sa.cap)
                            cq[base + r] = static_cast<int32_t>(((wt + u) * 4 + j) * PER_WORD + k);
                        r++;
                    }
                }
        }
        taken += total;
        __syncthreads();  // wtot is rewritten by the next round
    }
    if (tid == 0) {
        const int64_t end = base + (taken < need ? taken : need);
        *counter = static_cast<uint32_t>(end < sa.cap ? end : sa.cap);
    }
    __syncthreads();  // base_s is rewritten for the next query
}

template <int BITS>
__global__ __launch_bounds__(SL_BLOCK) void k_select_level(SelectArgs sa, int Ns, int64_t n, int64_t words,
                                                           const uint32_t *__restrict__ sc32) {
    __shared__ uint32_t wtot[SL_BLOCK / WAVE];
    __shared__ uint32_t base_s;
    if (!sa.redo) {
        select_level_query<BITS>(sa, Ns, n, words, sc32, blockIdx.x, wtot, base_s);
        return;
    }
    const uint32_t nrun = sa.redo[0];
    for (uint32_t f = blockIdx.x; f < nrun; f += gridDim.x)
        select_level_query<BITS>(sa, Ns, n, words, sc32, static_cast<int>(sa.redo[3 + f]), wtot, base_s);
}

// Alg 5 on a query's lists: the threshold from the histogram's levels >=
// the list level, scanned from the top (where this scan stops, the full
// scan stops; if it passes the list level, last < it), then either the
// queue (last < list level, or a tile listed more ids than its lcap slots;
// with redo_hist its histogram row is cleared for the recount) or the
// candidates: the listed ids with count >= last, moved from the tiles' list
// ranges to the candidate slots.  Each wavefront takes
// whole tiles.  With toff and tlev (and at most LS_TMAX tiles) the
// candidates are grouped by tile, in list order inside a tile: each tile's
// count is the sum of its listed ids' levels >= last (tlev, from the count
// kernel), and toff[q][t] receives the first slot of tile t
// (toff[q][T] = their number), so the re-rank can hand all candidates of a
// tile, i.e. of one id range, to workgroups on one XCD.  Without toff, or
// with more tiles, a wavefront reserves its slots with one LDS add per 256
// entries and toff[q][0] (if given) is TOFF_NONE, as for a queued query.
// The fixed-budget rule (rule 2) takes the same scan to the boundary level
// L, the highest listed level with S(L) >= R (queued when it lies below the
// list level).  Its candidates are the listed ids above L and the first
// need = R - S(L + 1) listed ids of level L in id order, i.e. those of
// level L below an id bound tau.  Tiles are consecutive id ranges: the
// tile where the running count of level-L entries reaches need holds tau,
// which a binary search over that tile's ids finds (the number of its
// level-L entries below a trial bound, counted by the workgroup).  These
// candidates are never grouped by tile.
// grid nq, block LS_BLOCK.
constexpr int LS_BLOCK = 256;
constexpr int LS_UNROLL = 4;
constexpr int LS_TMAX = 128;
constexpr uint32_t TOFF_NONE = 0xffffffffu;

__global__ __launch_bounds__(LS_BLOCK) void k_list_select(ListArgs la, uint32_t *__restrict__ hist, int Ns,
                                                          int64_t n) {
    __shared__ int s_last, s_tile;
    __shared__ uint32_t s_out, s_over, s_need, s_acc;
    __shared__ uint32_t s_tc[LS_TMAX + 1];
    __shared__ uint32_t s_red[LS_BLOCK / WAVE];
    const int q = blockIdx.x;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int lv = static_cast<int>(list_level(la));
    const bool fixed = la.rule == 2;
    const bool grouped = !fixed && la.toff != nullptr && la.tlev != nullptr && la.T <= LS_TMAX;
    uint32_t *tq = la.toff ? la.toff + static_cast<int64_t>(q) * (la.T + 1) : nullptr;
    uint32_t *h = hist + static_cast<int64_t>(q) * (Ns + 1);
    if (threadIdx.x == 0) s_over = 0u;
    __syncthreads();
    {
        uint32_t over = 0u;
        for (int t = threadIdx.x; t < la.T; t += LS_BLOCK)
            over |= la.tcount[static_cast<int64_t>(q) * la.T + t] > static_cast<uint64_t>(la.lcap) ? 1u : 0u;
        if (over) s_over = 1u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the highest listed level (>= lv) exceeding the budget, as in
        // select_threshold; lv - 1 when none does (the threshold is lower).
        // Rule 2: the boundary level, with S(last) >= R
        int last = lv - 1;
        int64_t S = 0;  // S(last) at the break
        uint32_t need = 0u;
        for (int v = Ns; v >= lv; v--) {
            const int64_t hv = h[v];
            if (fixed && S + hv >= la.R) {
                last = v;
                need = static_cast<uint32_t>(la.R - S);
                S = la.R;
                break;
            }
            S += hv;
            if (!fixed && (la.rule == 1 ? S : hv + S) > la.R) {
                last = v;
                break;
            }
        }
        if (la.dump_last || la.dump_hist)
            // stage dumps: the histogram is complete here; the threshold is
            // the full scan's (equal to last whenever last >= lv; rule 2
            // reports the boundary level plus one)
            dump_threshold(la.dump_last, la.dump_hist, q, Ns, n, h, select_threshold(h, Ns, n, la.R, la.rule));
        if (last > lv) atomicAdd(&la.redo[1], 1u);
        // a tile's list overflowed, or more candidates than slots (the
        // recount's selection queues those for k_stream_topk)
        const bool lover = last >= lv && s_over != 0u;
        const bool over = lover || (last >= lv && S > la.cap);
        if (lover) atomicAdd(&la.redo[2], 1u);  // (moves the adaptive level up)
        if (last < lv || over) {
            const uint32_t f = atomicAdd(&la.redo[0], 1u);
            la.redo[3 + f] = static_cast<uint32_t>(q);
            la.count[q] = 0u;
            if (la.redo_hist)
                for (int v = 1; v <= Ns; v++) h[v] = 0u;
            last = -1;  // queued
        }
        if (tq && (last < lv || !grouped)) tq[0] = TOFF_NONE;
        s_last = last;
        s_out = 0u;
        s_need = need;
        s_tile = -1;
        s_acc = 0u;
    }
    __syncthreads();
    const int last = s_last;
    if (last < lv) return;
    const uint32_t *ls = la.list + static_cast<int64_t>(q) * la.T * la.lcap;
    int32_t *cq = la.cand + static_cast<int64_t>(q) * la.cap;
    const uint32_t idmask = (1u << la.shift) - 1u, lu = static_cast<uint32_t>(last);
    const uint64_t below = lanes_below(lane);
    // ids of level `last` are taken below tau (all of them for Alg 5)
    uint32_t tau = 0xffffffffu;
    if (fixed) {
        const uint32_t need = s_need;
        tau = 0u;  // R = 0: none
        if (need > 0u) {
            // the tile where the level-L entries reach need, LS_TMAX tiles a pass
            for (int t0 = 0; t0 < la.T && s_tile < 0; t0 += LS_TMAX) {
                const int tn = min(LS_TMAX, la.T - t0);
                for (int t = t0 + wave; t < t0 + tn; t += LS_BLOCK / WAVE) {
                    const uint32_t nt = min(la.tcount[static_cast<int64_t>(q) * la.T + t],
                                            static_cast<uint32_t>(la.lcap));
                    const uint32_t *et = ls + static_cast<int64_t>(t) * la.lcap;
                    uint32_t c = 0u;
                    for (uint32_t i = lane; i < nt; i += WAVE) c += (et[i] >> la.shift) == lu ? 1u : 0u;
                    c = wave_sum_u32(c);
                    if (lane == 0) s_tc[t - t0] = c;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    uint32_t acc = s_acc;
                    for (int i = 0; i < tn; i++) {
                        if (acc + s_tc[i] >= need) {
                            s_tile = t0 + i;
                            break;
                        }
                        acc += s_tc[i];
                    }
                    s_acc = acc;  // the entries of level L in the tiles before s_tile
                }
                __syncthreads();
            }
            const int tc = s_tile;
            if (tc < 0) {
                tau = 0xffffffffu;  // (fewer entries than the histogram says: take them all)
            } else {
                // the smallest bound with `want` entries below it: the level-L
                // ids below it are the first `want` of the tile
                const uint32_t want = need - s_acc;
                const uint32_t nt = min(la.tcount[static_cast<int64_t>(q) * la.T + tc],
                                        static_cast<uint32_t>(la.lcap));
                const uint32_t *et = ls + static_cast<int64_t>(tc) * la.lcap;
                uint32_t lo = static_cast<uint32_t>(tc) * static_cast<uint32_t>(la.W);
                uint32_t hi = lo + static_cast<uint32_t>(la.W);  // below lo: none; below hi: >= want
                while (hi - lo > 1u) {
                    const uint32_t mid = lo + (hi - lo) / 2u;
                    uint32_t c = 0u;
                    for (uint32_t i = threadIdx.x; i < nt; i += LS_BLOCK) {
                        const uint32_t v = et[i];
                        c += ((v >> la.shift) == lu && (v & idmask) < mid) ? 1u : 0u;
                    }
                    c = wave_sum_u32(c);
                    if (lane == 0) s_red[wave] = c;
                    __syncthreads();
                    uint32_t tot = 0u;
#pragma unroll
                    for (int i = 0; i < LS_BLOCK / WAVE; i++) tot += s_red[i];
                    __syncthreads();  // s_red is rewritten by the next step
                    if (tot >= want)
                        hi = mid;
                    else
                        lo = mid;
                }
                tau = hi;
            }
        }
    }
    if (grouped) {
        // candidates per tile: its listed ids at levels >= last
        for (int t = threadIdx.x; t < la.T; t += LS_BLOCK) {
            const uint32_t *lt = la.tlev + (static_cast<int64_t>(q) * la.T + t) * (Ns + 1);
            uint32_t c = 0u;
#pragma unroll
            for (int v = 1; v <= 16; v++)
                if (v >= last && v <= Ns) c += lt[v];
            s_tc[t] = c;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t acc = 0u;
            for (int t = 0; t < la.T; t++) {
                const uint32_t c = s_tc[t];
                s_tc[t] = acc;
                tq[t] = acc;
                acc += c;
            }
            tq[la.T] = acc;
            s_out = acc;
        }
        __syncthreads();
        // pass 2: each tile's candidates from its first slot, in list order
        for (int t = wave; t < la.T; t += LS_BLOCK / WAVE) {
            const uint32_t nt = la.tcount[static_cast<int64_t>(q) * la.T + t];
            const uint32_t *et = ls + static_cast<int64_t>(t) * la.lcap;
            uint32_t base = s_tc[t];
            for (uint32_t b0 = 0; b0 < nt; b0 += WAVE * LS_UNROLL) {
                uint32_t v[LS_UNROLL];
#pragma unroll
                for (int u = 0; u < LS_UNROLL; u++) {
                    const uint32_t i = b0 + u * WAVE + lane;
                    v[u] = i < nt ? et[i] : 0u;
                }
#pragma unroll
                for (int u = 0; u < LS_UNROLL; u++) {
                    const uint64_t m = __ballot(v[u] != 0u && (v[u] >> la.shift) >= lu);
                    const uint32_t j = base + static_cast<uint32_t>(__popcll(m & below));
                    if (((m >> lane) & 1u) && j < static_cast<uint32_t>(la.cap)) cq[j] = static_cast<int32_t>(v[u] & idmask);
                    base += static_cast<uint32_t>(__popcll(m));
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) la.count[q] = s_out;
        return;
    }
    for (int t = wave; t < la.T; t += LS_BLOCK / WAVE) {
        const uint32_t nt = la.tcount[static_cast<int64_t>(q) * la.T + t];
        const uint32_t *et = ls + static_cast<int64_t>(t) * la.lcap;
        for (uint32_t b0 = 0; b0 < nt; b0 += WAVE * LS_UNROLL) {
            uint32_t v[LS_UNROLL];
#pragma unroll
            for (int u = 0; u < LS_UNROLL; u++) {
                const uint32_t i = b0 + u * WAVE + lane;
                v[u] = i < nt ? et[i] : 0u;
            }
            uint64_t m[LS_UNROLL];
            uint32_t tot = 0u;
#pragma unroll
            for (int u = 0; u < LS_UNROLL; u++) {
                // listed words hold a count >= 1; 0 marks an empty slot
                const uint32_t lev = v[u] >> la.shift;
                m[u] = __ballot(v[u] != 0u && (lev > lu || (lev == lu && (v[u] & idmask) < tau)));
                tot += static_cast<uint32_t>(__popcll(m[u]));
            }
            if (tot == 0u) continue;
            uint32_t base = 0u;
            if (lane == 0) base = atomicAdd(&s_out, tot);
            base = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(base));
#pragma unroll
            for (int u = 0; u < LS_UNROLL; u++) {
                const uint32_t j = base + static_cast<uint32_t>(__popcll(m[u] & below));
                if (((m[u] >> lane) & 1u) && j < static_cast<uint32_t>(la.cap)) cq[j] = static_cast<int32_t>(v[u] & idmask);
                base += static_cast<uint32_t>(__popcll(m[u]));
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) la.count[q] = s_out;
}

// Packed counts [nq][T*W] to one byte per id [nq][n] (stage dumps).
template <int BITS>
__global__ void k_unpack_counts(const uint32_t *__restrict__ sc, int64_t words_q, int64_t n,
                                uint8_t *__restrict__ out) {
    constexpr int PER_WORD = 32 / BITS;
    const int q = blockIdx.y;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < words_q;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint32_t w = sc[q * words_q + i];
        for (int b = 0; b < PER_WORD; b++) {
            const int64_t id = i * PER_WORD + b;
            if (id < n) out[q * n + id] = static_cast<uint8_t>((w >> (BITS * b)) & ((1u << BITS) - 1u));
        }
    }
}

// ---------------------------------------------------------------------------
// count + select fused in one cooperative, persistent launch.  The grid is
// exactly as large as the GPU can hold at once (cooperative launch): NG
// workgroups per tile.  A workgroup of tile t takes its next query from an
// atomic work queue, the tile's own counter into the query order (queries
// of larger budgets first when budgets differ per query, so the longest
// work starts early and the tail is short).  After counting its tile and
// adding the tile's level counts to hist[q], it arrives on arrive[q] and
// waits until all T tiles of q have arrived.  Every tile hands out the same
// order, and every workgroup is resident, so the earliest unfinished query
// always has each of its tiles counted or being counted and the wait ends;
// it is also bounded (spin_limit polls), setting *err and going on if ever
// exceeded.  Then the threshold comes from the complete histogram and
// candidates are compacted straight from LDS: no packed counts go to HBM.
// ---------------------------------------------------------------------------

struct FuseArgs {
    int nq, NG;
    uint32_t *hist;       // [nq][Ns+1], zero before the launch
    uint32_t *arrive;     // [nq], zero before the launch
    uint32_t *err;        // set to 1 if a wait timed out
    uint32_t spin_limit;
    uint32_t *queue;      // [T] per-tile dequeue counters, zero before the launch
    const int32_t *order; // [nq] the order queries are handed out in, or null (0, 1, ...)
    uint4 *sc;            // [nq][T][W*BITS/128] packed counts of queries that outgrow cap
};

template <int BITS, bool HI>
__global__ __launch_bounds__(CT_BLOCK, 8) void k_count_select(CountArgs a, SelectArgs sa, FuseArgs f) {
    constexpr int PER_WORD = 32 / BITS;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const CountLds L = carve<BITS>(lds_raw, a.W);
    __shared__ uint32_t hsum[18];
    __shared__ uint32_t hq[17];
    __shared__ int s_last, s_over;
    // candidate staging reuses the slice table (idle during compaction):
    // CT_FSTAGE slots per wavefront
    constexpr int CT_FSTAGE = 2 * CT_CHUNK / CT_WAVES >= 128 ? 128 : 64;
    static_assert(CT_FSTAGE * CT_WAVES <= 2 * CT_CHUNK, "staging must fit the slice table");
    __shared__ int s_q;
    const int t = blockIdx.x % a.T;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int words = a.W / PER_WORD;
    const int64_t tile_lo = static_cast<int64_t>(t) * a.W;
    const int tile_n = static_cast<int>(min<int64_t>(a.W, a.n - tile_lo));
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t i = atomicAdd(&f.queue[t], 1u);
            s_q = i < static_cast<uint32_t>(f.nq) ? (f.order ? f.order[i] : static_cast<int>(i)) : -1;
        }
        __syncthreads();
        const int q = s_q;
        if (q < 0) break;
        if (threadIdx.x < 18) hsum[threadIdx.x] = 0u;
        count_tile<BITS, HI>(a, q, t, L, hsum);
        __syncthreads();
        uint32_t *hg = f.hist + static_cast<int64_t>(q) * (a.Ns + 1);
        if (threadIdx.x >= 1 && threadIdx.x <= a.Ns) {
            const uint32_t hv = hsum[threadIdx.x] - hsum[threadIdx.x + 1];
            if (hv) atomicAdd(&hg[threadIdx.x], hv);
            __threadfence();
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(&f.arrive[q], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t polls = 0;
            while (__hip_atomic_load(&f.arrive[q], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
                   static_cast<uint32_t>(a.T)) {
                if (++polls > f.spin_limit) {
                    atomicOr(f.err, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            for (int v = 1; v <= a.Ns; v++)
                hq[v] = __hip_atomic_load(&hg[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_last = select_threshold(hq, a.Ns, a.n, sa.R, sa.rule);
            s_over = outgrows(sa, hq, a.Ns, a.n, s_last) ? 1 : 0;
            if (t == 0) {
                if (s_over) sa.ovf[1 + atomicAdd(&sa.ovf[0], 1u)] = static_cast<uint32_t>(q);
                if (sa.dump_last) sa.dump_last[q] = s_last;
                if (sa.dump_hist) {
                    int64_t above0 = 0;
                    for (int v = 1; v <= a.Ns; v++) above0 += hq[v];
                    sa.dump_hist[static_cast<int64_t>(q) * (a.Ns + 1)] = a.n - above0;
                    for (int v = 1; v <= a.Ns; v++)
                        sa.dump_hist[static_cast<int64_t>(q) * (a.Ns + 1) + v] = hq[v];
                }
            }
        }
        __syncthreads();
        const int last = s_last;
        const bool over = s_over != 0;
        if (over) {
            // the tile's counts go to HBM for k_stream_topk
            const int vec = a.W * BITS / 128;
            uint4 *dst = f.sc + (static_cast<int64_t>(q) * a.T + t) * vec;
            for (int i = threadIdx.x; i < vec; i += CT_BLOCK) dst[i] = reinterpret_cast<const uint4 *>(L.cnt)[i];
            if (!sa.dump_sc) {
                __syncthreads();  // the next query's counting rewrites L.cnt
                continue;
            }
        }
        const uint32_t lv = static_cast<uint32_t>(last > 0 ? last : 0);
        int32_t *cq = sa.cand + static_cast<int64_t>(q) * sa.cap;
        uint32_t *stage = L.dl + wave * CT_FSTAGE;
        uint32_t scount = 0;
        for (int i0 = 0; i0 < words; i0 += CT_BLOCK) {
            const int i = i0 + threadIdx.x;
            const bool in = i < words;
            const uint32_t w = in ? L.cnt[i] : 0u;
            if (sa.dump_sc && in) {
                for (int b = 0; b < PER_WORD; b++) {
                    const int loc = i * PER_WORD + b;
                    if (loc < tile_n)
                        sa.dump_sc[static_cast<int64_t>(q) * a.n + tile_lo + loc] =
                            static_cast<uint8_t>((w >> (BITS * b)) & ((1u << BITS) - 1u));
                }
            }
            uint32_t m[2];
            ge_masks<BITS>(w, lv, m[0], m[1]);
            if (!in || over) m[0] = m[1] = 0u;
            if (in && i * PER_WORD + PER_WORD > tile_n) {
                // ids past n in the last tile are padding
                for (int i2 = 0; i2 < 2; i2++)
                    for (int b = 0; b < 4; b++)
                        if (i * PER_WORD + (BITS == 8 ? b : 2 * b + i2) >= tile_n) m[i2] &= ~(0x80u << (8 * b));
            }
            append_flagged<CT_FSTAGE, 2>(
                m,
                [&](int i2, int b) {
                    return static_cast<uint32_t>(tile_lo + i * PER_WORD + (BITS == 8 ? b : 2 * b + i2));
                },
                stage, scount, sa.cand_count + q, CandOut{cq, static_cast<uint32_t>(sa.cap)}, lane);
        }
        if (__any(scount != 0u))
            flush_stage(stage, scount, sa.cand_count + q, CandOut{cq, static_cast<uint32_t>(sa.cap)}, lane);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// re-rank: squared L2 distance of each candidate row to its query, FP32.
// LPR lanes cooperate on a row with 16-byte loads; the query sits in LDS.
// The per-lane partial sums and the xor tree inside each LPR-lane group are
// shared with k_recheck_topk, so a row's FP32 distance is the same bits wherever
// it is computed.  grid (G, nq), block 256, dynamic LDS d floats.
// ---------------------------------------------------------------------------

template <int LPR, bool VEC4>
__device__ __forceinline__ float row_partial32(const float *qs, const float *row, int d, int li) {
    float acc = 0.0f;
    if (VEC4) {
        const float4 *r4 = reinterpret_cast<const float4 *>(row);
        const float4 *q4 = reinterpret_cast<const float4 *>(qs);
        for (int f = li; f < d / 4; f += LPR) {
            const float4 xv = r4[f], qv = q4[f];
            float u = qv.x - xv.x;
            acc = fmaf(u, u, acc);
            u = qv.y - xv.y;
            acc = fmaf(u, u, acc);
            u = qv.z - xv.z;
            acc = fmaf(u, u, acc);
            u = qv.w - xv.w;
            acc = fmaf(u, u, acc);
        }
    } else {
        for (int f = li; f < d; f += LPR) {
            const float u = qs[f] - row[f];
            acc = fmaf(u, u, acc);
        }
    }
    return acc;
}

// Sum over the LPR lanes of a row group; every lane of the group must call.
template <int LPR>
__device__ __forceinline__ float group_sum(float acc) {
#pragma unroll
    for (int m = LPR / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m, WAVE);
    return acc;
}

// Integer sum over groups of LPR lanes (4, 8 or 16; wider groups use
// shuffles), every lane of a group receiving it, with DPP moves: quad swaps,
// then half-row and row mirrors, each pairing a lane with one in the other
// half of its group.  Exact, so the pairing order does not matter.
template <int LPR>
__device__ __forceinline__ int group_sum_i32(int a) {
    if (LPR > 16) {
#pragma unroll
        for (int m = LPR / 2; m > 0; m >>= 1) a += __shfl_xor(a, m, WAVE);
        return a;
    }
    a += __builtin_amdgcn_update_dpp(0, a, 0xb1, 0xf, 0xf, false);  // quad_perm [1,0,3,2]
    a += __builtin_amdgcn_update_dpp(0, a, 0x4e, 0xf, 0xf, false);  // quad_perm [2,3,0,1]
    if (LPR >= 8) a += __builtin_amdgcn_update_dpp(0, a, 0x141, 0xf, 0xf, false);  // row_half_mirror
    if (LPR >= 16) a += __builtin_amdgcn_update_dpp(0, a, 0x140, 0xf, 0xf, false);  // row_mirror
    return a;
}

// Rows handled at once by a lane group of the re-rank kernels: the chunk
// loop runs outside and the rows inside, so the loads of RU rows are in
// flight together, while each row's terms keep the order of row_partial32.
#ifndef TACO_RU
#define TACO_RU 4
#endif
constexpr int RU = TACO_RU;

template <int LPR, bool VEC4>
__global__ __launch_bounds__(256) void k_rerank(const float *__restrict__ Q, int d,
                                                const float *__restrict__ base,
                                                const int32_t *__restrict__ cand,
                                                const uint32_t *__restrict__ cand_count,
                                                int64_t cap, float *__restrict__ cand_dist) {
    extern __shared__ float qs[];
    const int q = blockIdx.y;
    for (int t = threadIdx.x; t < d; t += BLOCK) qs[t] = Q[static_cast<int64_t>(q) * d + t];
    __syncthreads();
    const int64_t nc = cand_n(cand_count, q, cap);
    constexpr int RPW = WAVE / LPR;  // rows per wavefront per step
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int sub = lane / LPR, li = lane % LPR;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * WAVES * RPW;
    const int32_t *cq = cand + static_cast<int64_t>(q) * cap;
    float *dq = cand_dist + static_cast<int64_t>(q) * cap;
    for (int64_t i0 = (static_cast<int64_t>(blockIdx.x) * WAVES + wave) * RPW; i0 < nc;
         i0 += stride * RU) {
        int64_t row[RU];
        float acc[RU];
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const int64_t i = i0 + u * stride + sub;
            row[u] = i < nc ? static_cast<int64_t>(cq[i]) * d : -1;
            acc[u] = 0.0f;
        }
        if (VEC4) {
            const float4 *q4 = reinterpret_cast<const float4 *>(qs);
            for (int f = li; f < d / 4; f += LPR) {
                float4 xv[RU];
#pragma unroll
                for (int u = 0; u < RU; u++)
                    xv[u] = row[u] >= 0 ? reinterpret_cast<const float4 *>(base + row[u])[f]
                                        : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                const float4 qv = q4[f];
#pragma unroll
                for (int u = 0; u < RU; u++) {
                    float v = qv.x - xv[u].x;
                    acc[u] = fmaf(v, v, acc[u]);
                    v = qv.y - xv[u].y;
                    acc[u] = fmaf(v, v, acc[u]);
                    v = qv.z - xv[u].z;
                    acc[u] = fmaf(v, v, acc[u]);
                    v = qv.w - xv[u].w;
                    acc[u] = fmaf(v, v, acc[u]);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < RU; u++)
                if (row[u] >= 0) acc[u] = row_partial32<LPR, false>(qs, base + row[u], d, li);
        }
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const float a = group_sum<LPR>(acc[u]);
            const int64_t i = i0 + u * stride + sub;
            if (li == 0 && i < nc) dq[i] = a;
        }
    }
}

// ---------------------------------------------------------------------------
// BF16 re-rank with an exact FP32 boundary re-check.
//
// The library keeps xb = bf16(fl32(x - mu)) for every base row, mu being the
// mean rounded to BF16 (so integer-valued data stay exact), and e(x) = the
// FP64 norm of xb - (x - mu), rounded up.  With qc = fl32(q - mu) and
// u~ = fl32(qc - xb), the exact difference u = q - x satisfies
//   ||u~ - u|| <= E = e(x) + 2^-24 (||q - mu|| + ||u~||)   (two FP32 roundings),
// and the FP32 sums of d squares (this kernel's and the FP32 path's) are
// within a relative 2(d+2)2^-24 of their exact values.  So the FP32 path's
// distance d32 of the row lies in [lb, ub] with
//   s = sqrt(d~),  ub = (s(1+g) + E)^2 (1+g),  lb = max(0, s(1-g) - E)^2 (1-g),
// g = 2(d+2)2^-24 + 2^-18: the extra 2^-18 covers the few FP32 roundings of
// evaluating these bounds (each <= 2^-24 relative, sqrt within 2 ulp).  If
// tau is the k-th smallest ub, every row of the FP32 path's top-k has
// lb <= tau; k_recheck_topk recomputes exactly those rows with the FP32 path's
// own arithmetic.
// ---------------------------------------------------------------------------

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ float f32_round_up(double v) {
    float f = static_cast<float>(v);
    if (static_cast<double>(f) < v) f = nextafterf(f, __uint_as_float(0x7f800000u));
    return f;
}


template <int LPR, bool VEC8>
__global__ __launch_bounds__(256) void k_rerank16(const float *__restrict__ Q, int d,
                                                  const float *__restrict__ mu,
                                                  const uint16_t *__restrict__ base16,
                                                  const float *__restrict__ rowerr,
                                                  const int32_t *__restrict__ cand,
                                                  const uint32_t *__restrict__ cand_count,
                                                  int64_t cap, float *__restrict__ ub_out,
                                                  float *__restrict__ lb_out) {
    extern __shared__ float qs[];
    __shared__ float rq_part[WAVES];
    const int q = blockIdx.y;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    float sq = 0.0f;
    for (int t = threadIdx.x; t < d; t += BLOCK) {
        const float v = Q[static_cast<int64_t>(q) * d + t] - mu[t];
        qs[t] = v;
        sq = fmaf(v, v, sq);
    }
#pragma unroll
    for (int m = WAVE / 2; m > 0; m >>= 1) sq += __shfl_xor(sq, m, WAVE);
    if (lane == 0) rq_part[wave] = sq;
    __syncthreads();
    float rq2 = 0.0f;
    for (int w = 0; w < WAVES; w++) rq2 += rq_part[w];
    // ||q - mu||, inflated for the FP32 roundings of q - mu and of the sum
    const float rq = sqrtf(rq2) * (1.0f + (d + 8) * 0x1p-23f);
    const int64_t nc = cand_n(cand_count, q, cap);
    constexpr int RPW = WAVE / LPR;
    const int sub = lane / LPR, li = lane % LPR;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * WAVES * RPW;
    const int32_t *cq = cand + static_cast<int64_t>(q) * cap;
    const float g = 2.0f * (d + 2) * 0x1p-24f + 0x1p-18f;
    for (int64_t i0 = (static_cast<int64_t>(blockIdx.x) * WAVES + wave) * RPW; i0 < nc;
         i0 += stride * RU) {
        int64_t id[RU];
        float acc[RU];
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const int64_t i = i0 + u * stride + sub;
            id[u] = i < nc ? static_cast<int64_t>(cq[i]) : -1;
            acc[u] = 0.0f;
        }
        if (VEC8) {
            for (int f = li; f < d / 8; f += LPR) {
                uint4 v[RU];
#pragma unroll
                for (int u = 0; u < RU; u++)
                    v[u] = id[u] >= 0 ? reinterpret_cast<const uint4 *>(base16 + id[u] * d)[f]
                                      : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
                for (int u = 0; u < RU; u++) {
                    const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                    for (int c = 0; c < 4; c++) {
                        float x = qs[8 * f + 2 * c] - bf16_bits_to_f32(w[c] & 0xffffu);
                        acc[u] = fmaf(x, x, acc[u]);
                        x = qs[8 * f + 2 * c + 1] - bf16_bits_to_f32(w[c] >> 16);
                        acc[u] = fmaf(x, x, acc[u]);
                    }
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < RU; u++) {
                if (id[u] < 0) continue;
                const uint16_t *row = base16 + id[u] * d;
                for (int f = li; f < d; f += LPR) {
                    const float x = qs[f] - bf16_bits_to_f32(row[f]);
                    acc[u] = fmaf(x, x, acc[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const float sum = group_sum<LPR>(acc[u]);
            const int64_t i = i0 + u * stride + sub;
            if (li == 0 && i < nc) {
                const float s = sqrtf(sum > 0.0f ? sum : 0.0f);
                const float su = s * (1.0f + g);
                const float E = rowerr[id[u]] + 0x1p-22f * (rq + su + 1.0f);
                const float hs = su + E;
                const float ls = s * (1.0f - g) - E;
                ub_out[static_cast<int64_t>(q) * cap + i] = hs * hs * (1.0f + g);
                lb_out[static_cast<int64_t>(q) * cap + i] = ls > 0.0f ? ls * ls * (1.0f - g) : 0.0f;
            }
        }
    }
}

// Per query of a batch, for the exact 8-bit re-rank, in rows of d/4 + 4
// words (16-byte aligned for d % 16 == 0): words w < d/4 hold values
// 4w..4w+3 as bytes, word d/4 is 1 when every value is an integer in
// [0, 255] (else 0), word d/4 + 1 is |q|^2 (exact then: integers below 2^24
// for d <= 256).  One wavefront per query; d % 16 == 0, d <= 256.
__global__ __launch_bounds__(256) void k_qbytes(const float *__restrict__ Q, int nq, int d,
                                                uint32_t *__restrict__ info) {
    const int q = blockIdx.x * WAVES + threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    if (q >= nq) return;
    const float *qv = Q + static_cast<int64_t>(q) * d;
    uint32_t *out = info + static_cast<int64_t>(q) * (d / 4 + 4);
    bool ok = true;
    float sq = 0.0f;
    for (int w = lane; w < d / 4; w += WAVE) {
        uint32_t word = 0u;
        for (int b = 0; b < 4; b++) {
            const float v = qv[4 * w + b];
            ok = ok && v >= 0.0f && v <= 255.0f && v == rintf(v);
            sq = fmaf(v, v, sq);
            word |= (ok ? static_cast<uint32_t>(v) : 0u) << (8 * b);
        }
        out[w] = word;
    }
#pragma unroll
    for (int m = WAVE / 2; m > 0; m >>= 1) sq += __shfl_xor(sq, m, WAVE);
    const bool all = __all(ok);
    if (lane == 0) {
        out[d / 4] = all ? 1u : 0u;
        out[d / 4 + 1] = all ? static_cast<uint32_t>(sq) : 0u;
    }
}

// The same bounds from 8-bit rows: row i is stored as codes c_t with its
// own offset lo_i and step sc_i, x^_t = fl(lo_i + fl(c_t * sc_i)); the
// preparation kernel computes the row's error bound against exactly these
// values and keeps (lo, sc, error) in one 16-byte record per row, read
// with one load.  PLAIN: every row has offset 0, step 1 and error 0 (integer
// data in [0, 255]), and no record is read.  The query is used as is (no
// centring), so its only rounding is inside the distance.
// PLAIN with 16 | d <= 256 and a query of integers in [0, 255] (qinfo, from
// k_qbytes; null: never): every term
// (q_t - x_t)^2 <= 255^2 and every partial sum <= d * 255^2 < 2^24 are
// integers that FP32 holds exactly, so the FP32 path's distance is the
// exact integer |q|^2 + |x|^2 - 2 q.x whatever its summation order; that is
// computed with byte dot products and written as the upper bound, and
// exact[q] says so: the top k of the upper bounds is then the result itself
// and the lower bounds are not written (nor read).  Without exact the
// bounded form runs for every query.
// grid (G, nq), block 256, dynamic LDS d floats.
template <int LPR, bool VEC16, bool PLAIN>
__global__ __launch_bounds__(256, PLAIN ? 8 : 1) void k_rerank8(const float *__restrict__ Q, int d,
                                                 const uint8_t *__restrict__ base8,
                                                 const float4 *__restrict__ meta,
                                                 const int32_t *__restrict__ cand,
                                                 const uint32_t *__restrict__ cand_count,
                                                 int64_t cap, float *__restrict__ ub_out,
                                                 float *__restrict__ lb_out, uint32_t *__restrict__ exact,
                                                 const uint32_t *__restrict__ qinfo,
                                                 const uint32_t *__restrict__ toff, int T,
                                                 const int32_t *__restrict__ perm) {
    extern __shared__ float qs[];
    __shared__ float rq_part[WAVES];
    const int q = perm ? perm[blockIdx.y] : static_cast<int>(blockIdx.y), chunk = blockIdx.x;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t nc = cand_n(cand_count, q, cap);
    constexpr int RPW = WAVE / LPR;
    const int sub = lane / LPR, li = lane % LPR;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * WAVES * RPW;
    const int32_t *cq = cand + static_cast<int64_t>(q) * cap;
    const uint32_t *info = qinfo ? qinfo + static_cast<int64_t>(q) * (d / 4 + 4) : nullptr;
    const bool integral = PLAIN && VEC16 && info && info[d / 4] != 0u;
    if (exact && chunk == 0 && threadIdx.x == 0) exact[q] = integral ? 1u : 0u;
    if (PLAIN && VEC16 && integral) {
        const int qq = static_cast<int>(info[d / 4 + 1]);
        const uint4 *qb4 = reinterpret_cast<const uint4 *>(info);
        // RU rows per lane group at slots i0 + u*step + sub below end
        auto pass = [&](int64_t i0, int64_t step, int64_t end) {
            int64_t id[RU];
            int acc[RU];
#pragma unroll
            for (int u = 0; u < RU; u++) {
                const int64_t i = i0 + u * step + sub;
                id[u] = i < end ? static_cast<int64_t>(cq[i]) : -1;
                acc[u] = 0;
            }
            for (int f = li; f < d / 16; f += LPR) {
                const uint4 qv = qb4[f];
                uint4 v[RU];
#pragma unroll
                for (int u = 0; u < RU; u++)
                    v[u] = id[u] >= 0 ? reinterpret_cast<const uint4 *>(base8 + id[u] * d)[f]
                                      : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
                for (int u = 0; u < RU; u++) {
                    // |x|^2 - 2 q.x over these 16 bytes
                    uint32_t xx = __builtin_amdgcn_udot4(v[u].x, v[u].x, 0u, false);
                    xx = __builtin_amdgcn_udot4(v[u].y, v[u].y, xx, false);
                    xx = __builtin_amdgcn_udot4(v[u].z, v[u].z, xx, false);
                    xx = __builtin_amdgcn_udot4(v[u].w, v[u].w, xx, false);
                    uint32_t qx = __builtin_amdgcn_udot4(v[u].x, qv.x, 0u, false);
                    qx = __builtin_amdgcn_udot4(v[u].y, qv.y, qx, false);
                    qx = __builtin_amdgcn_udot4(v[u].z, qv.z, qx, false);
                    qx = __builtin_amdgcn_udot4(v[u].w, qv.w, qx, false);
                    acc[u] += static_cast<int>(xx) - 2 * static_cast<int>(qx);
                }
            }
#pragma unroll
            for (int u = 0; u < RU; u++) {
                const int a = group_sum_i32<LPR>(acc[u]);
                const int64_t i = i0 + u * step + sub;
                // the lower bound is not needed: the re-check takes the bound
                // top k as it is for a flagged query
                if (li == 0 && i < end) ub_out[static_cast<int64_t>(q) * cap + i] = static_cast<float>(qq + a);
            }
        };
        const uint32_t *tq = toff ? toff + static_cast<int64_t>(q) * (T + 1) : nullptr;
        if (tq && tq[0] != 0xffffffffu && gridDim.x % 8 == 0) {
            // candidates grouped by tile (id range): workgroup chunk takes the
            // tiles t = chunk (mod 8), each split between the gridDim.x / 8
            // workgroups of that residue.  Workgroup (q, chunk) has linear id
            // q*gridDim.x + chunk, and the dispatcher deals linear ids to the
            // 8 XCDs in turn, so one XCD serves one id range of the rows (more
            // hits in its L2).  Any placement gives the same results.
            const int nparts = gridDim.x / 8, part = chunk / 8;
            const int64_t lstride = static_cast<int64_t>(WAVES) * RPW;
            for (int t = chunk % 8; t < T; t += 8) {
                const int64_t a0 = tq[t], a1 = tq[t + 1];
                const int64_t per = (a1 - a0 + nparts - 1) / nparts;
                const int64_t r0 = a0 + per * part, r1 = min(a1, r0 + per);
                for (int64_t i0 = r0 + static_cast<int64_t>(wave) * RPW; i0 < r1; i0 += lstride * RU)
                    pass(i0, lstride, r1);
            }
        } else {
            for (int64_t i0 = (static_cast<int64_t>(chunk) * WAVES + wave) * RPW; i0 < nc; i0 += stride * RU)
                pass(i0, stride, nc);
        }
        return;
    }
    float sq = 0.0f;
    for (int t = threadIdx.x; t < d; t += BLOCK) {
        const float v = Q[static_cast<int64_t>(q) * d + t];
        qs[t] = v;
        sq = fmaf(v, v, sq);
    }
#pragma unroll
    for (int m = WAVE / 2; m > 0; m >>= 1) sq += __shfl_xor(sq, m, WAVE);
    if (lane == 0) rq_part[wave] = sq;
    __syncthreads();
    float rq2 = 0.0f;
    for (int w = 0; w < WAVES; w++) rq2 += rq_part[w];
    const float rq = sqrtf(rq2) * (1.0f + (d + 8) * 0x1p-23f);
    const float g = 2.0f * (d + 2) * 0x1p-24f + 0x1p-18f;
    for (int64_t i0 = (static_cast<int64_t>(chunk) * WAVES + wave) * RPW; i0 < nc;
         i0 += stride * RU) {
        int64_t id[RU];
        float acc[RU], lo[RU], sc[RU], er[RU];
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const int64_t i = i0 + u * stride + sub;
            id[u] = i < nc ? static_cast<int64_t>(cq[i]) : -1;
            acc[u] = 0.0f;
        }
#pragma unroll
        for (int u = 0; u < RU; u++) {
            // plain rows: offset 0, step 1, error 0 (the codes are the values)
            const float4 m = (PLAIN || id[u] < 0) ? make_float4(0.0f, 1.0f, 0.0f, 0.0f) : meta[id[u]];
            lo[u] = m.x;
            sc[u] = m.y;
            er[u] = m.z;
        }
        if (VEC16) {
            for (int f = li; f < d / 16; f += LPR) {
                uint4 v[RU];
#pragma unroll
                for (int u = 0; u < RU; u++)
                    v[u] = id[u] >= 0 ? reinterpret_cast<const uint4 *>(base8 + id[u] * d)[f]
                                      : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
                for (int u = 0; u < RU; u++) {
                    const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                    for (int c = 0; c < 4; c++) {
#pragma unroll
                        for (int b = 0; b < 4; b++) {
                            const float xh = lo[u] + static_cast<float>((w[c] >> (8 * b)) & 0xffu) * sc[u];
                            const float x = qs[16 * f + 4 * c + b] - xh;
                            acc[u] = fmaf(x, x, acc[u]);
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < RU; u++) {
                if (id[u] < 0) continue;
                const uint8_t *row = base8 + id[u] * d;
                for (int f = li; f < d; f += LPR) {
                    const float xh = lo[u] + static_cast<float>(row[f]) * sc[u];
                    const float x = qs[f] - xh;
                    acc[u] = fmaf(x, x, acc[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RU; u++) {
            const float sum = group_sum<LPR>(acc[u]);
            const int64_t i = i0 + u * stride + sub;
            if (li == 0 && i < nc) {
                const float s = sqrtf(sum > 0.0f ? sum : 0.0f);
                const float su = s * (1.0f + g);
                const float E = er[u] + 0x1p-22f * (rq + su + 1.0f);
                const float hs = su + E;
                const float ls = s * (1.0f - g) - E;
                ub_out[static_cast<int64_t>(q) * cap + i] = hs * hs * (1.0f + g);
                lb_out[static_cast<int64_t>(q) * cap + i] = ls > 0.0f ? ls * ls * (1.0f - g) : 0.0f;
            }
        }
    }
}

constexpr int RC_CHUNK = 2048;  // candidates tested per round of the re-check

// BF16 copy of the base centred at mu, and each row's exact quantization
// error norm (FP64, rounded up).  One wavefront per row.
__global__ __launch_bounds__(256) void k_prep_bf16(const float *__restrict__ base, int64_t n, int d,
                                                   const float *__restrict__ mu,
                                                   uint16_t *__restrict__ base16,
                                                   float *__restrict__ rowerr) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * WAVES + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (row >= n) return;
    double e2 = 0.0;
    for (int t = lane; t < d; t += WAVE) {
        const float x = base[row * d + t];
        const float c = x - mu[t];
        const uint32_t b = __float_as_uint(c);
        const uint32_t h = (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;  // round to nearest even
        base16[row * d + t] = static_cast<uint16_t>(h);
        const double err = static_cast<double>(bf16_bits_to_f32(h)) -
                           (static_cast<double>(x) - static_cast<double>(mu[t]));
        e2 += err * err;
    }
#pragma unroll
    for (int m = WAVE / 2; m > 0; m >>= 1) e2 += __shfl_xor(e2, m, WAVE);
    if (lane == 0) rowerr[row] = f32_round_up(sqrt(e2) * (1.0 + 0x1p-50));
}

// 8-bit copy of the base: per row an offset, a step, the codes, and the
// exact FP64 norm of the row's quantization error against the values the
// re-rank reconstructs, rounded up; (offset, step, error, 0) form one 16-byte
// record per row.  Rows of integers in [0, 255] get offset 0 and step 1 (the
// codes are the values, error 0); other rows of integers spanning at most
// 255 get their minimum and step 1 (exact); the rest their minimum and
// (max - min)/255.  *plain is cleared unless every row is of the first kind.
// One wavefront per row.
__global__ __launch_bounds__(256) void k_prep_u8(const float *__restrict__ base, int64_t n, int d,
                                                 uint8_t *__restrict__ base8, float4 *__restrict__ meta,
                                                 uint32_t *__restrict__ plain) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * WAVES + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (row >= n) return;
    float mn = __uint_as_float(0x7f800000u), mx = -mn;
    bool integral = true;
    for (int t = lane; t < d; t += WAVE) {
        const float x = base[row * d + t];
        mn = fminf(mn, x);
        mx = fmaxf(mx, x);
        integral = integral && x == rintf(x);
    }
#pragma unroll
    for (int m = WAVE / 2; m > 0; m >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, m, WAVE));
        mx = fmaxf(mx, __shfl_xor(mx, m, WAVE));
    }
    integral = __all(integral);
    float lo = mn, sc = (mx - mn) / 255.0f;
    if (integral && mn >= 0.0f && mx <= 255.0f) {
        lo = 0.0f;
        sc = 1.0f;
    } else if (integral && mx - mn <= 255.0f) {
        sc = 1.0f;
    }
    if (!(sc > 0.0f)) sc = 1.0f;
    double e2 = 0.0;
    for (int t = lane; t < d; t += WAVE) {
        const float x = base[row * d + t];
        const float c = fminf(fmaxf(rintf((x - lo) / sc), 0.0f), 255.0f);
        const uint32_t code = static_cast<uint32_t>(c);
        base8[row * d + t] = static_cast<uint8_t>(code);
        const float xh = lo + static_cast<float>(code) * sc;
        const double err = static_cast<double>(xh) - static_cast<double>(x);
        e2 += err * err;
    }
#pragma unroll
    for (int m = WAVE / 2; m > 0; m >>= 1) e2 += __shfl_xor(e2, m, WAVE);
    if (lane == 0) {
        const float err = f32_round_up(sqrt(e2) * (1.0 + 0x1p-50));
        meta[row] = make_float4(lo, sc, err, 0.0f);
        if (!(lo == 0.0f && sc == 1.0f && err == 0.0f)) atomicAnd(plain, 0u);
    }
}

// ---------------------------------------------------------------------------
// top-k: one workgroup per query.  Keys (distance bits << 32 | id) are unique
// and order like (distance, id) because distances are >= +0.  An MSB-first
// radix select over 8-bit digits finds the smallest prefix whose bucket is
// taken whole; exactly k keys fall at or below it.  They are gathered to LDS
// and bitonic-sorted.  The digits start below the bits all keys share (from
// the block's minimum and maximum key), so the first pass already splits
// the candidates; each pass picks its digit with a block prefix sum over the
// 256 buckets.
// ---------------------------------------------------------------------------

constexpr int TOPK_MAX = 1024;

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int m = WAVE / 2; m > 0; m >>= 1) {
        const uint64_t o = __shfl_xor(v, m, WAVE);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int m = WAVE / 2; m > 0; m >>= 1) {
        const uint64_t o = __shfl_xor(v, m, WAVE);
        v = o > v ? o : v;
    }
    return v;
}

constexpr int TK_KPT = 32;  // keys per thread kept in registers (|C| <= 256 * TK_KPT)

// Calls f(key) for every candidate key of the query: from registers when
// they all fit, else streamed from memory eight loads per thread at a time.
template <typename F>
__device__ __forceinline__ void for_keys(bool reg, const uint64_t (&kr)[TK_KPT], int64_t nc,
                                         const int32_t *cq, const float *dq, F f) {
    if (reg) {
#pragma unroll
        for (int u = 0; u < TK_KPT; u++)
            if (static_cast<int64_t>(threadIdx.x) + u * BLOCK < nc) f(kr[u]);
    } else {
        for (int64_t i0 = threadIdx.x; i0 < nc; i0 += 8 * BLOCK) {
            uint64_t kk[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int64_t i = i0 + u * BLOCK;
                kk[u] = i < nc ? (static_cast<uint64_t>(__float_as_uint(dq[i])) << 32) |
                                     static_cast<uint32_t>(cq[i])
                               : 0ull;
            }
#pragma unroll
            for (int u = 0; u < 8; u++)
                if (i0 + u * BLOCK < nc) f(kk[u]);
        }
    }
}

// The k smallest of the nc keys (dq[i] bits << 32 | cq[i]) of query q, by
// the whole workgroup (256 threads, all must call); results go to row q of
// (ids_out, d_out), k_max entries, padded with (-1, +inf) past k or past nc.
__device__ __forceinline__ void topk_select(int q, const int32_t *__restrict__ cq, const float *__restrict__ dq, int64_t nc,
                            int k, int k_max, int64_t *__restrict__ ids_out, float *__restrict__ d_out) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t wtot[WAVES];
    __shared__ uint64_t wred[2 * WAVES];
    __shared__ uint64_t sel[TOPK_MAX];
    __shared__ uint32_t nsel;
    __shared__ uint32_t s_digit, s_need, s_full;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const bool reg = nc <= static_cast<int64_t>(BLOCK) * TK_KPT;
    uint64_t kr[TK_KPT];
    if (reg) {
#pragma unroll
        for (int u = 0; u < TK_KPT; u++) {
            const int64_t i = threadIdx.x + u * BLOCK;
            kr[u] = i < nc ? (static_cast<uint64_t>(__float_as_uint(dq[i])) << 32) | static_cast<uint32_t>(cq[i])
                           : 0ull;
        }
    }
    if (threadIdx.x == 0) nsel = 0u;
    bool gathered = false;
    if (nc > k && k <= WAVE) {
        // Each wavefront's k-th smallest lane minimum is >= the k-th
        // smallest key (those k minima are k distinct keys); the smallest
        // such bound over the wavefronts usually leaves a few dozen keys.
        // Two passes over the keys, also when they are streamed.
        uint64_t tmin = ~0ull;
        for_keys(reg, kr, nc, cq, dq, [&](uint64_t kk) { tmin = kk < tmin ? kk : tmin; });
        const uint64_t srt = wave_sort_u64(tmin, lane);
        const uint32_t tlo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(srt)), k - 1));
        const uint32_t thi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(srt >> 32)), k - 1));
        if (lane == 0) wred[wave] = (static_cast<uint64_t>(thi) << 32) | tlo;
        __syncthreads();
        uint64_t bound = wred[0];
        for (int w = 1; w < WAVES; w++) bound = wred[w] < bound ? wred[w] : bound;
        for_keys(reg, kr, nc, cq, dq, [&](uint64_t kk) {
            if (kk <= bound) {
                const uint32_t p = atomicAdd(&nsel, 1u);
                if (p < TOPK_MAX) sel[p] = kk;
            }
        });
        __syncthreads();
        gathered = nsel <= static_cast<uint32_t>(TOPK_MAX);
        __syncthreads();
        if (!gathered && threadIdx.x == 0) nsel = 0u;
    }
    int shift = 64;
    uint64_t prefix = 0;
    if (!gathered && nc > k) {
        // bits above `shift` are common to all keys: prefix holds them
        uint64_t mn = ~0ull, mx = 0ull;
        for_keys(reg, kr, nc, cq, dq, [&](uint64_t kk) {
            mn = kk < mn ? kk : mn;
            mx = kk > mx ? kk : mx;
        });
        mn = wave_min_u64(mn);
        mx = wave_max_u64(mx);
        if (lane == 0) {
            wred[wave] = mn;
            wred[WAVES + wave] = mx;
        }
        __syncthreads();
        mn = wred[0];
        mx = wred[WAVES];
        for (int w = 1; w < WAVES; w++) {
            mn = wred[w] < mn ? wred[w] : mn;
            mx = wred[WAVES + w] > mx ? wred[WAVES + w] : mx;
        }
        shift = 64 - __clzll(static_cast<long long>(mn ^ mx));  // mn != mx: keys are unique
        prefix = shift == 64 ? 0ull : mn >> shift;
        uint32_t need = static_cast<uint32_t>(k);
        bool done = false;
        while (!done && shift > 0) {
            const int sh2 = shift > 8 ? shift - 8 : 0;
            const uint32_t dmask = (1u << (shift - sh2)) - 1u;
            hist[threadIdx.x] = 0u;
            __syncthreads();
            for_keys(reg, kr, nc, cq, dq, [&](uint64_t kk) {
                if (shift == 64 || (kk >> shift) == prefix)
                    atomicAdd(&hist[static_cast<uint32_t>(kk >> sh2) & dmask], 1u);
            });
            __syncthreads();
            // the bucket where the running count reaches `need`
            const uint32_t hv = hist[threadIdx.x];
            const uint32_t inc = wave_incl_scan_u32(hv, lane);
            if (lane == WAVE - 1) wtot[wave] = inc;
            __syncthreads();
            uint32_t before = 0u;
            for (int w = 0; w < wave; w++) before += wtot[w];
            const uint32_t incl = before + inc, excl = incl - hv;
            if (excl < need && need <= incl) {
                s_digit = threadIdx.x;
                s_need = need - excl;
                s_full = hv == need - excl;
            }
            __syncthreads();
            prefix = (prefix << (shift - sh2)) | s_digit;
            need = s_need;
            done = s_full != 0u;
            shift = sh2;
            __syncthreads();
        }
    }
    __syncthreads();
    // gather: every key (|C| <= k) or the keys whose top (64-shift) bits <= prefix
    if (!gathered) {
        for_keys(reg, kr, nc, cq, dq, [&](uint64_t kk) {
            if (nc <= k || (kk >> shift) <= prefix) {
                const uint32_t p = atomicAdd(&nsel, 1u);
                if (p < TOPK_MAX) sel[p] = kk;
            }
        });
        __syncthreads();
    }
    // sort the gathered keys (exactly min(|C|, k) of them after the radix
    // select; at least k after the bound) and keep the first k
    const int ns = static_cast<int>(min<uint32_t>(nsel, static_cast<uint32_t>(TOPK_MAX)));
    const int m = min(ns, k);
    if (ns <= WAVE && k_max <= WAVE) {
        // one wavefront sorts them in registers (no workgroup barriers)
        if (wave == 0) {
            const uint64_t v = wave_sort_u64(lane < ns ? sel[lane] : ~0ull, lane);
            if (lane < k_max) {
                const int64_t o = static_cast<int64_t>(q) * k_max + lane;
                ids_out[o] = lane < m ? static_cast<int64_t>(static_cast<uint32_t>(v & 0xffffffffu)) : -1;
                d_out[o] = lane < m ? __uint_as_float(static_cast<uint32_t>(v >> 32)) : __uint_as_float(0x7f800000u);
            }
        }
        return;
    }
    int P = 1;
    while (P < ns) P <<= 1;
    for (int i = ns + threadIdx.x; i < P; i += BLOCK) sel[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P; i += BLOCK) {
                const int pj = i ^ stride;
                if (pj > i) {
                    const bool up = (i & size) == 0;
                    const uint64_t a = sel[i], b = sel[pj];
                    if ((a > b) == up) {
                        sel[i] = b;
                        sel[pj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < k_max; i += BLOCK) {
        const int64_t o = static_cast<int64_t>(q) * k_max + i;
        if (i < m) {
            ids_out[o] = static_cast<int64_t>(static_cast<uint32_t>(sel[i] & 0xffffffffu));
            d_out[o] = __uint_as_float(static_cast<uint32_t>(sel[i] >> 32));
        } else {
            ids_out[o] = -1;
            d_out[o] = __uint_as_float(0x7f800000u);
        }
    }
}

// k is kq[q] when kq is given (else k_all).  grid nq, block 256.
__global__ __launch_bounds__(256) void k_topk(const int32_t *__restrict__ cand,
                                              const float *__restrict__ cand_dist,
                                              const uint32_t *__restrict__ cand_count,
                                              int64_t cap, int k_all, const int32_t *__restrict__ kq,
                                              int k_max, int64_t *__restrict__ ids_out,
                                              float *__restrict__ d_out) {
    const int q = blockIdx.x;
    topk_select(q, cand + static_cast<int64_t>(q) * cap, cand_dist + static_cast<int64_t>(q) * cap,
                cand_n(cand_count, q, cap), kq ? kq[q] : k_all, k_max, ids_out, d_out);
}

// ---------------------------------------------------------------------------
// Queries whose candidate set outgrows the call's slots (Alg 5 keeps the
// whole threshold level, so |C| = S(last) can exceed R): the FP32 re-rank
// straight from the packed counts, and the top-k in two steps, with no more
// than ST_SPLIT * k_max slots per query (which the call's cap leaves).  The
// ids of each queued query are split into ST_SPLIT ranges, one workgroup
// each.  A workgroup scans its range ST_WORDS count words at a time, lists
// the chunk's candidates (count >= last, id < n) in LDS, computes their
// distances with the re-rank's lane groups (row_partial32 and group_sum: the
// bits of k_rerank and k_recheck_topk), and keeps every key (distance bits,
// id) below the running k-th smallest in a buffer that a bitonic sort cuts
// back to k keys whenever it holds more than TOPK_MAX.  Its k smallest go to
// the query's candidate slots (positions reserved on cand_count[q]); the
// top-k of those (k_topk_queued) replaces the query's results, written
// before from its empty candidate list.  grid (ST_SPLIT, any), block BLOCK,
// dynamic LDS d floats; ovf: [0] queued queries, [1 + i] the queue.
// ---------------------------------------------------------------------------
constexpr int ST_SPLIT = STREAM_SPLIT; // workgroups (id ranges) per queued query
constexpr int ST_WORDS = BLOCK;        // 32-bit count words per chunk, one per thread
constexpr int ST_LIST = BLOCK * 8;     // candidates per chunk, at most
constexpr int ST_BUF = 4096;           // >= TOPK_MAX + ST_LIST, a power of two
static_assert(TOPK_MAX + ST_LIST <= ST_BUF, "the key buffer must hold a cut plus a chunk");

// Ascending bitonic sort of a[0, P) in LDS, P a power of two; every thread
// of the workgroup calls it.
__device__ __forceinline__ void lds_bitonic_u64(uint64_t *a, int P) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P; i += BLOCK) {
                const int pj = i ^ stride;
                if (pj > i) {
                    const bool up = (i & size) == 0;
                    const uint64_t x = a[i], y = a[pj];
                    if ((x > y) == up) {
                        a[i] = y;
                        a[pj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Sorts the nb keys of buf (padding to a power of two with ~0) and keeps
// the first min(nb, k); returns how many are kept.
__device__ __forceinline__ uint32_t cut_keys(uint64_t *buf, uint32_t nb, int k) {
    int P = 1;
    while (P < static_cast<int>(nb)) P <<= 1;
    for (int i = static_cast<int>(nb) + threadIdx.x; i < P; i += BLOCK) buf[i] = ~0ull;
    __syncthreads();
    lds_bitonic_u64(buf, P);
    return min(nb, static_cast<uint32_t>(k));
}

template <int LPR, bool VEC4, int BITS>
__global__ __launch_bounds__(BLOCK) void k_stream_topk(const float *__restrict__ Q, int d,
                                                       const float *__restrict__ base,
                                                       const uint32_t *__restrict__ sc, int64_t row_words,
                                                       const uint32_t *__restrict__ hist, int Ns, int64_t n,
                                                       int64_t R, int rule, const uint32_t *__restrict__ ovf,
                                                       int k_all, const int32_t *__restrict__ kq, int64_t cap,
                                                       int32_t *__restrict__ cand, float *__restrict__ cand_dist,
                                                       uint32_t *__restrict__ cand_count) {
    extern __shared__ float qs[];
    __shared__ uint32_t list[ST_LIST];
    __shared__ uint64_t buf[ST_BUF];
    __shared__ uint32_t s_nl, s_nb, s_at;
    __shared__ int s_last;
    constexpr int PER_WORD = 32 / BITS;
    constexpr uint32_t CMASK = (1u << BITS) - 1u;
    constexpr int RPW = WAVE / LPR;  // rows per wavefront per step
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int sub = lane / LPR, li = lane % LPR;
    const int64_t nwords = (n + PER_WORD - 1) / PER_WORD;
    const int64_t span = (nwords + gridDim.x - 1) / gridDim.x;
    const int64_t w_lo = static_cast<int64_t>(blockIdx.x) * span;
    const int64_t w_hi = min(nwords, w_lo + span);
    const uint32_t nov = ovf[0];
    for (uint32_t f = blockIdx.y; f < nov; f += gridDim.y) {
        const int q = static_cast<int>(ovf[1 + f]);
        const int k = kq ? kq[q] : k_all;
        for (int t = threadIdx.x; t < d; t += BLOCK) qs[t] = Q[static_cast<int64_t>(q) * d + t];
        if (threadIdx.x == 0) {
            s_last = select_threshold(hist + static_cast<int64_t>(q) * (Ns + 1), Ns, n, R, rule);
            s_nb = 0u;
        }
        __syncthreads();
        const uint32_t lv = static_cast<uint32_t>(s_last > 0 ? s_last : 0);  // level 0: every id
        const uint32_t *row = sc + static_cast<int64_t>(q) * row_words;
        uint64_t bound = ~0ull;  // the k-th smallest key kept so far (after a cut)
        for (int64_t g0 = w_lo; g0 < w_hi; g0 += ST_WORDS) {
            if (threadIdx.x == 0) s_nl = 0u;
            __syncthreads();
            const int64_t g = g0 + threadIdx.x;
            if (g < w_hi) {
                const uint32_t w = row[g];
#pragma unroll
                for (int j = 0; j < PER_WORD; j++) {
                    const int64_t id = g * PER_WORD + j;
                    if (id < n && ((w >> (BITS * j)) & CMASK) >= lv)
                        list[atomicAdd(&s_nl, 1u)] = static_cast<uint32_t>(id);
                }
            }
            __syncthreads();
            const uint32_t nl = s_nl;
            // every lane of a row group runs the same iterations (group_sum)
            for (uint32_t i0 = static_cast<uint32_t>(wave * RPW); i0 < nl; i0 += WAVES * RPW) {
                const uint32_t i = i0 + static_cast<uint32_t>(sub);
                const bool ok = i < nl;
                const int64_t id = ok ? static_cast<int64_t>(list[i]) : 0;
                const float acc = group_sum<LPR>(row_partial32<LPR, VEC4>(qs, base + id * d, d, li));
                if (ok && li == 0) {
                    const uint64_t key = (static_cast<uint64_t>(__float_as_uint(acc)) << 32) |
                                         static_cast<uint32_t>(id);
                    if (key < bound) buf[atomicAdd(&s_nb, 1u)] = key;
                }
            }
            __syncthreads();
            const uint32_t nb = s_nb;
            if (nb > static_cast<uint32_t>(TOPK_MAX)) {
                const uint32_t kept = cut_keys(buf, nb, k);
                bound = kept == static_cast<uint32_t>(k) ? buf[k - 1] : ~0ull;
                __syncthreads();
                if (threadIdx.x == 0) s_nb = kept;
            }
        }
        __syncthreads();
        const uint32_t m = cut_keys(buf, s_nb, k);
        if (threadIdx.x == 0) s_at = m ? atomicAdd(&cand_count[q], m) : 0u;
        __syncthreads();
        int32_t *cq = cand + static_cast<int64_t>(q) * cap + s_at;
        float *dq = cand_dist + static_cast<int64_t>(q) * cap + s_at;
        for (uint32_t i = threadIdx.x; i < m && s_at + i < cap; i += BLOCK) {
            cq[i] = static_cast<int32_t>(static_cast<uint32_t>(buf[i] & 0xffffffffu));
            dq[i] = __uint_as_float(static_cast<uint32_t>(buf[i] >> 32));
        }
        __syncthreads();  // qs, buf, s_nb and s_at are rewritten for the next query
    }
}

// The top-k of the queued queries of ovf from their candidate slots (the
// workgroups' partial top-k of k_stream_topk).  grid (any), block 256.
__global__ __launch_bounds__(256) void k_topk_queued(const int32_t *__restrict__ cand,
                                                     const float *__restrict__ cand_dist,
                                                     const uint32_t *__restrict__ cand_count, int64_t cap,
                                                     const uint32_t *__restrict__ ovf, int k_all,
                                                     const int32_t *__restrict__ kq, int k_max,
                                                     int64_t *__restrict__ ids_out, float *__restrict__ d_out) {
    const uint32_t nov = ovf[0];
    for (uint32_t f = blockIdx.x; f < nov; f += gridDim.x) {
        const int q = static_cast<int>(ovf[1 + f]);
        topk_select(q, cand + static_cast<int64_t>(q) * cap, cand_dist + static_cast<int64_t>(q) * cap,
                    cand_n(cand_count, q, cap), kq ? kq[q] : k_all, k_max, ids_out, d_out);
        __syncthreads();  // topk_select's shared state is reused for the next query
    }
}

// FP32 re-check of the rows whose lower bound reaches the query's tau (the
// k-th smallest upper bound), then the top-k of those rows, one workgroup per
// query.  Chunks of RC_CHUNK candidates are tested (eight loads per thread in
// flight), the kept ones compacted into LDS and re-ranked by row groups with
// the FP32 path's own arithmetic (row_partial32 and group_sum with the same
// lanes per row); the kept (id, distance) pairs go to (rk_ids, rk_dist), and
// their top k to the output rows.  rk_ids may share memory with lb: a
// chunk's lower bounds are read before its kept rows are written, and kept
// rows land below the chunk's end.  A query with exact[q] set (its bounds are
// the FP32 distances) takes the top k of the bounds as they are.  grid nq,
// block 256, dynamic LDS d floats.
template <int LPR, bool VEC4>
__global__ __launch_bounds__(256) void k_recheck_topk(const float *__restrict__ Q, int d,
                                                      const float *__restrict__ base,
                                                      const int32_t *__restrict__ cand,
                                                      const uint32_t *__restrict__ cand_count,
                                                      const float *lb, int64_t cap,
                                                      const float *__restrict__ tau_d, int k_all,
                                                      const int32_t *__restrict__ kq, int k_max,
                                                      int32_t *rk_ids, float *__restrict__ rk_dist,
                                                      uint32_t *__restrict__ rk_count,
                                                      int64_t *__restrict__ ids_out, float *__restrict__ d_out,
                                                      const uint32_t *__restrict__ exact,
                                                      const int64_t *__restrict__ tau_ids) {
    extern __shared__ float qs[];
    __shared__ int32_t kept[RC_CHUNK];
    __shared__ uint32_t nkept, nrk;
    const int q = blockIdx.x;
    if (exact && exact[q]) {
        for (int i = threadIdx.x; i < k_max; i += BLOCK) {
            const int64_t o = static_cast<int64_t>(q) * k_max + i;
            ids_out[o] = tau_ids[o];
            d_out[o] = tau_d[o];
        }
        if (threadIdx.x == 0) rk_count[q] = 0u;
        return;
    }
    for (int t = threadIdx.x; t < d; t += BLOCK) qs[t] = Q[static_cast<int64_t>(q) * d + t];
    const int64_t nc = cand_n(cand_count, q, cap);
    const int k = kq ? kq[q] : k_all;
    const float tau = tau_d[static_cast<int64_t>(q) * k_max + (k - 1)];  // +inf when |C| < k
    constexpr int RPW = WAVE / LPR;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int sub = lane / LPR, li = lane % LPR;
    const int32_t *cq = cand + static_cast<int64_t>(q) * cap;
    const float *lq = lb + static_cast<int64_t>(q) * cap;
    int32_t *rq_ids = rk_ids + static_cast<int64_t>(q) * cap;
    float *rq_d = rk_dist + static_cast<int64_t>(q) * cap;
    if (threadIdx.x == 0) nrk = 0u;
    for (int64_t c0 = 0; c0 < nc; c0 += RC_CHUNK) {
        if (threadIdx.x == 0) nkept = 0u;
        __syncthreads();
        constexpr int PER = RC_CHUNK / BLOCK;
        float lv[PER];
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int64_t i = c0 + threadIdx.x + u * BLOCK;
            lv[u] = i < nc ? lq[i] : __uint_as_float(0x7f800000u);
        }
#pragma unroll
        for (int u = 0; u < PER; u++) {
            const int64_t i = c0 + threadIdx.x + u * BLOCK;
            if (i < nc && lv[u] <= tau) kept[atomicAdd(&nkept, 1u)] = cq[i];
        }
        __syncthreads();
        const int m = static_cast<int>(nkept);
        for (int r0 = wave * RPW; r0 < m; r0 += WAVES * RPW) {
            const int r = r0 + sub;
            float acc = 0.0f;
            if (r < m) acc = row_partial32<LPR, VEC4>(qs, base + static_cast<int64_t>(kept[r]) * d, d, li);
            acc = group_sum<LPR>(acc);
            if (r < m && li == 0) {
                const uint32_t p = atomicAdd(&nrk, 1u);
                rq_ids[p] = kept[r];
                rq_d[p] = acc;
            }
        }
        __syncthreads();
    }
    const int64_t m_all = nrk;
    if (threadIdx.x == 0) rk_count[q] = static_cast<uint32_t>(m_all);
    topk_select(q, rq_ids, rq_d, m_all, k, k_max, ids_out, d_out);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    k_fill_u32<<<static_cast<unsigned>(blocks), 256, 0, st>>>(p, count, v);
    return hipGetLastError();
}

hipError_t launch_u32_to_i64(const uint32_t *src, int64_t *dst, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_u32_to_i64<<<static_cast<unsigned>((count + 255) / 256), 256, 0, st>>>(src, dst, count);
    return hipGetLastError();
}

hipError_t launch_build_off2d(const uint32_t *ids, const uint32_t *offs, int Ns, int K, int64_t n,
                              int T, int W, uint32_t *off2d, hipStream_t st) {
    int64_t work = static_cast<int64_t>(Ns) * K;
    k_build_off2d<<<static_cast<unsigned>((work + 255) / 256), 256, 0, st>>>(ids, offs, Ns, K, n,
                                                                             T, W, off2d);
    return hipGetLastError();
}

hipError_t launch_encode_ids(const uint32_t *ids, const uint32_t *raw, const uint32_t *pad, int Ns, int K, int T,
                             int64_t n, int W, int bits, uint32_t *enc, hipStream_t st) {
    const int64_t slices = static_cast<int64_t>(Ns) * K * T;
    k_encode_ids<<<static_cast<unsigned>((slices + 3) / 4), 256, 0, st>>>(ids, raw, pad, Ns, K, T, n, W, bits, enc);
    return hipGetLastError();
}

hipError_t launch_flatten_cells(const int32_t *cells, const int32_t *ncells, int nq, int Ns, int K, int32_t *flat,
                                uint32_t *ftot, hipStream_t st) {
    if (nq > 0) k_flatten_cells<<<(nq + 3) / 4, 256, 0, st>>>(cells, ncells, nq, Ns, K, flat, ftot);
    return hipGetLastError();
}

hipError_t launch_query_order(const int32_t *cells, int nq, int Ns, int K, int32_t *perm, hipStream_t st) {
    if (K > 4096) return hipErrorInvalidValue;
    k_query_order<<<1, ORD_BLOCK, sizeof(uint32_t) * static_cast<size_t>(K), st>>>(cells, nq, Ns, K, perm);
    return hipGetLastError();
}

hipError_t launch_transform(const float *Q, int nq, int d, const float *mean, const float *B,
                            int M, float *qt, hipStream_t st) {
    dim3 grid((M + 63) / 64, (nq + TR_Q - 1) / TR_Q), block(64, 4);
    k_transform<<<grid, block, 0, st>>>(Q, nq, d, mean, B, M, qt);
    return hipGetLastError();
}

hipError_t launch_probe(const float *qt, int nq, int Ns, int M, int s, int h1, int h2, int l,
                        int K, const float *C1, const float *C2, const uint32_t *offs, int64_t A,
                        const int64_t *A_q, int32_t *cells, int32_t *ncells, int64_t *retrieved,
                        float *dump_cdist, int32_t *dump_corder, const float *pre, int qpw,
                        hipStream_t st) {
    size_t lds = sizeof(uint32_t) * static_cast<size_t>(K);
#define TACO_PROBE(Q)                                                                          \
    k_probe<Q><<<dim3((nq + Q - 1) / Q, Ns), 64 * Q, lds, st>>>(                               \
        qt, nq, M, s, h1, h2, l, K, C1, C2, offs, A, A_q, cells, ncells, retrieved, dump_cdist, \
        dump_corder, pre)
    switch (qpw) {
    case 1: TACO_PROBE(1); break;
    case 2: TACO_PROBE(2); break;
    case 8: TACO_PROBE(8); break;
    case 16: TACO_PROBE(16); break;
    default: TACO_PROBE(4); break;
    }
#undef TACO_PROBE
    return hipGetLastError();
}

hipError_t launch_prep_centroids(const float *C1, const float *C2, int Ns, int s, int h1, int h2, int l,
                                 int Kp, bool fp8, const float *csc, void *cT, float *cnorm, hipStream_t st) {
    const int ncol = Ns * 2 * l;
    if (fp8)
        k_prep_cent<true><<<ncol, 64, 0, st>>>(C1, C2, Ns, s, h1, h2, l, Kp, csc, cT, cnorm);
    else
        k_prep_cent<false><<<ncol, 64, 0, st>>>(C1, C2, Ns, s, h1, h2, l, Kp, csc, cT, cnorm);
    return hipGetLastError();
}

hipError_t launch_cdist_mfma(const float *qt, int nq, int M, int Ns, int s, int h1, int h2, int l, int Kp,
                             bool fp8, const void *cT, const float *cnorm, const float *csc, float *qn,
                             float *qsc, void *qa, float *cd, hipStream_t st) {
    if (nq <= 0) return hipSuccess;
    const int64_t pairs = static_cast<int64_t>(nq) * Ns;
    const unsigned qblocks = static_cast<unsigned>((pairs + 255) / 256);
    if (fp8)
        k_qstats<true><<<qblocks, 256, 0, st>>>(qt, nq, Ns, M, s, h1, Kp, qn, qsc, qa);
    else
        k_qstats<false><<<qblocks, 256, 0, st>>>(qt, nq, Ns, M, s, h1, Kp, qn, qsc, qa);
    const int ncol = Ns * 2 * l;
    dim3 grid((ncol + 63) / 64, (nq + 15) / 16);
    if (fp8)
        k_cdist_mfma<true><<<grid, 256, 0, st>>>(qt, nq, M, Ns, s, h1, h2, l, Kp, cT, cnorm, csc, qn, qsc, qa, cd);
    else
        k_cdist_mfma<false><<<grid, 256, 0, st>>>(qt, nq, M, Ns, s, h1, h2, l, Kp, cT, cnorm, csc, qn, qsc, qa, cd);
    return hipGetLastError();
}

hipError_t launch_budgets(const double *alpha, const int32_t *kq, int nq, int64_t n, int k_max,
                          int64_t *A, int32_t *kc, uint32_t *err, hipStream_t st) {
    k_budgets<<<(nq + 255) / 256, 256, 0, st>>>(alpha, kq, nq, n, k_max, A, kc, err);
    return hipGetLastError();
}

size_t count_lds_bytes(int W, int bits) { return count_lds_size(W, bits); }

// Instances: nibble counts up to 8 levels (Ns <= 8), nibbles with up to
// 15, bytes (Ns = 16).
template <int MODE, bool TR, bool MULTI, int NT>
static const void *count_kernel_form(int bits, int Ns) {
    if (bits == 8) return reinterpret_cast<const void *>(k_count<8, true, MODE, TR, MULTI, NT>);
    return Ns > 8 ? reinterpret_cast<const void *>(k_count<4, true, MODE, TR, MULTI, NT>)
                  : reinterpret_cast<const void *>(k_count<4, false, MODE, TR, MULTI, NT>);
}

// form 3: the list form with the level transitions; 4 and 5: the list and
// store forms taking several queries per workgroup
template <int NT>
static const void *count_kernel_nt(int bits, int Ns, int form) {
    if (form == CT_LIST) return count_kernel_form<CT_LIST, false, false, NT>(bits, Ns);
    if (form == 3) return count_kernel_form<CT_LIST, true, false, NT>(bits, Ns);
    if (form == 4) return count_kernel_form<CT_LIST, false, true, NT>(bits, Ns);
    if (form == 5) return count_kernel_form<CT_STORE, true, true, NT>(bits, Ns);
    if (form == CT_REDO) return count_kernel_form<CT_REDO, true, false, NT>(bits, Ns);
    return count_kernel_form<CT_STORE, true, false, NT>(bits, Ns);
}

static const void *count_kernel(int bits, int Ns, int form, int nt) {
    return nt == 768 ? count_kernel_nt<768>(bits, Ns, form) : count_kernel_nt<1024>(bits, Ns, form);
}

static const void *count_select_kernel(int bits, int Ns) {
    if (bits == 8) return reinterpret_cast<const void *>(k_count_select<8, true>);
    return Ns > 8 ? reinterpret_cast<const void *>(k_count_select<4, true>)
                  : reinterpret_cast<const void *>(k_count_select<4, false>);
}

hipError_t prepare_count_kernels(int W, int bits, int Ns) {
    for (int nt : {768, 1024}) {
        const int bytes = static_cast<int>(count_lds_size(W, bits, nt));
        for (int form : {0, 1, 2, 3, 4, 5}) {
            const void *k = count_kernel(bits, Ns, form, nt);
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            if (e != hipSuccess) return e;
            // k_count addresses its counts from LDS address 0 (count_word<true>)
            hipFuncAttributes fa{};
            if ((e = hipFuncGetAttributes(&fa, k)) != hipSuccess) return e;
            if (fa.sharedSizeBytes != 0) return hipErrorInvalidDeviceFunction;
        }
    }
    return hipSuccess;
}

int list_shift(int Ns) {
    int b = 0;
    while ((1 << b) <= Ns) b++;
    return 31 - b;
}

static ListArgs list_args(const CountLaunch &c, const ListLaunch *l) {
    ListArgs la{};
    la.nq = c.nq;
    if (l)
        la = ListArgs{l->fixed, l->level, list_shift(c.Ns), c.nq, l->cap, l->lcap, l->list, l->cand, l->count,
                      l->tcount,
                      c.T, c.W, l->redo, l->R, l->rule, l->trans ? 0 : 1, l->dump_last, l->dump_hist,
                      l->toff, l->tlev};
    return la;
}

hipError_t launch_list_select(const CountLaunch &c, const ListLaunch &l, uint32_t *hist, hipStream_t st) {
    k_list_select<<<c.nq, LS_BLOCK, 0, st>>>(list_args(c, &l), hist, c.Ns, c.n);
    return hipGetLastError();
}

hipError_t launch_count(const CountLaunch &c, uint32_t *hist, uint32_t *sc, int form, const ListLaunch *l,
                        hipStream_t st) {
    if (form != CT_STORE && !l) return hipErrorInvalidValue;
    // several queries per workgroup for the list and split forms (not with
    // the list form's level transitions, a stage-dump variant)
    const int qpw = (form == CT_REDO || (form == CT_LIST && l->trans)) ? 1 : std::max(1, c.qpw);
    CountArgs a{c.Ns, c.K, c.T, c.W, c.n, c.ids, c.off2d, c.flat, c.ftot, c.perm, c.nq, qpw, 0};
    const ListArgs la = list_args(c, l);
    dim3 grid(c.T, form == CT_REDO ? l->redo_groups : (c.nq + qpw - 1) / qpw);
    if (form != CT_REDO) {
        // XCD order (k_count): T x groups units in 8 runs
        const int64_t units = static_cast<int64_t>(c.T) * ((c.nq + qpw - 1) / qpw);
        a.xper = static_cast<int>((units + 7) / 8);
        grid = dim3(static_cast<unsigned>(8 * a.xper), 1);
    }
    uint4 *s4 = reinterpret_cast<uint4 *>(sc);
    if (c.nt != 768 && c.nt != 1024) return hipErrorInvalidValue;
    const size_t lds = count_lds_size(c.W, c.bits, c.nt);
#define TACO_COUNT_NT(MODE, TR, MULTI, NT)                                                     \
    do {                                                                                    \
        if (c.bits == 8)                                                                    \
            k_count<8, true, MODE, TR, MULTI, NT><<<grid, NT, lds, st>>>(a, hist, s4, la);  \
        else if (c.Ns > 8)                                                                  \
            k_count<4, true, MODE, TR, MULTI, NT><<<grid, NT, lds, st>>>(a, hist, s4, la);  \
        else                                                                                \
            k_count<4, false, MODE, TR, MULTI, NT><<<grid, NT, lds, st>>>(a, hist, s4, la); \
    } while (0)
#define TACO_COUNT(MODE, TR, MULTI)                 \
    do {                                            \
        if (c.nt == 768)                            \
            TACO_COUNT_NT(MODE, TR, MULTI, 768);    \
        else                                        \
            TACO_COUNT_NT(MODE, TR, MULTI, 1024);   \
    } while (0)
    // several queries per workgroup: instances of their own, so that the
    // one-query forms keep their registers
    const bool multi = qpw > 1;
    if (form == CT_LIST && l->trans)
        TACO_COUNT(CT_LIST, true, false);
    else if (form == CT_LIST && multi)
        TACO_COUNT(CT_LIST, false, true);
    else if (form == CT_LIST)
        TACO_COUNT(CT_LIST, false, false);
    else if (form == CT_REDO)
        TACO_COUNT(CT_REDO, true, false);
    else if (multi)
        TACO_COUNT(CT_STORE, true, true);
    else
        TACO_COUNT(CT_STORE, true, false);
#undef TACO_COUNT
#undef TACO_COUNT_NT
    return hipGetLastError();
}


hipError_t launch_unpack_counts(const uint32_t *sc, int nq, int T, int W, int bits, int64_t n, uint8_t *out,
                                hipStream_t st) {
    const int64_t words_q = static_cast<int64_t>(T) * W * bits / 32;
    int64_t blocks = (words_q + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    dim3 grid(static_cast<unsigned>(blocks), nq);
    if (bits == 4)
        k_unpack_counts<4><<<grid, 256, 0, st>>>(sc, words_q, n, out);
    else
        k_unpack_counts<8><<<grid, 256, 0, st>>>(sc, words_q, n, out);
    return hipGetLastError();
}

hipError_t launch_select_level(const CountLaunch &c, const SelectLaunch &s, const uint32_t *sc,
                               hipStream_t st) {
    SelectArgs sa{s.hist, s.R, s.rule, s.cap, s.cand, s.cand_count, nullptr, nullptr, nullptr, s.redo, nullptr};
    const int64_t words = static_cast<int64_t>(c.T) * c.W * c.bits / 32;
    const unsigned grid = static_cast<unsigned>(s.redo ? s.redo_groups : c.nq);
    if (grid == 0u) return hipErrorInvalidValue;
    if (c.bits == 4)
        k_select_level<4><<<grid, SL_BLOCK, 0, st>>>(sa, c.Ns, c.n, words, sc);
    else
        k_select_level<8><<<grid, SL_BLOCK, 0, st>>>(sa, c.Ns, c.n, words, sc);
    return hipGetLastError();
}

hipError_t launch_select(const CountLaunch &c, const SelectLaunch &s, const uint32_t *sc,
                         hipStream_t st) {
    SelectArgs sa{s.hist, s.R, s.rule, s.cap, s.cand, s.cand_count, s.dump_sc, s.dump_last,
                  s.dump_hist, s.redo, s.ovf};
    const int64_t words4 = static_cast<int64_t>(c.T) * c.W * c.bits / 128;
    // about 16 sixteen-byte words per thread; the few queued queries of a
    // list selection get four (one pass of SEL_UNROLL loads)
    const int64_t per = s.redo ? 4 : 16;
    int64_t blocks = (words4 + SEL_BLOCK * per - 1) / (SEL_BLOCK * per);
    if (blocks > (s.redo ? 256 : 64)) blocks = s.redo ? 256 : 64;
    if (blocks < 1) blocks = 1;
    dim3 grid(static_cast<unsigned>(blocks), s.redo ? s.redo_groups : c.nq);
    const uint4 *s4 = reinterpret_cast<const uint4 *>(sc);
    if (c.bits == 4)
        k_select<4><<<grid, SEL_BLOCK, 0, st>>>(sa, c.Ns, c.n, words4, s4);
    else
        k_select<8><<<grid, SEL_BLOCK, 0, st>>>(sa, c.Ns, c.n, words4, s4);
    return hipGetLastError();
}

size_t fused_lds_bytes(int W, int bits) {
    return count_lds_size(W, bits) + (18 + 17 + 3) * sizeof(uint32_t);
}

hipError_t fused_max_blocks(int W, int bits, int Ns, int *blocks_per_cu) {
    const int bytes = static_cast<int>(count_lds_size(W, bits));
    const void *k = count_select_kernel(bits, Ns);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, CT_BLOCK, bytes);
}

hipError_t launch_cost_order(const int64_t *retrieved, int nq, int Ns, int32_t *perm, hipStream_t st) {
    k_cost_order<<<1, ORD_BLOCK, 0, st>>>(retrieved, nq, Ns, perm);
    return hipGetLastError();
}

hipError_t launch_count_select(const CountLaunch &c, const SelectLaunch &s, int NG, uint32_t *arrive,
                               uint32_t *err, uint32_t spin_limit, uint32_t *queue, const int32_t *order,
                               uint32_t *sc, hipStream_t st) {
    CountArgs a{c.Ns, c.K, c.T, c.W, c.n, c.ids, c.off2d, c.flat, c.ftot, c.perm, c.nq, 1};
    SelectArgs sa{s.hist, s.R, s.rule, s.cap, s.cand, s.cand_count, s.dump_sc, s.dump_last,
                  s.dump_hist, nullptr, s.ovf};
    FuseArgs f{c.nq, NG, const_cast<uint32_t *>(s.hist), arrive, err, spin_limit, queue, order,
               reinterpret_cast<uint4 *>(sc)};
    void *args[] = {&a, &sa, &f};
    const void *k = count_select_kernel(c.bits, c.Ns);
    return hipLaunchCooperativeKernel(k, dim3(static_cast<unsigned>(NG) * c.T), dim3(CT_BLOCK), args,
                                      static_cast<unsigned>(count_lds_size(c.W, c.bits)), st);
}

int rerank_lanes_per_row(int d) {
    if (d % 4 != 0) return 64;
    int chunks = d / 4, lpr = 4;
    while (lpr < 64 && lpr * 4 <= chunks) lpr <<= 1;
    return lpr;
}

hipError_t launch_rerank(const float *Q, int nq, int d, const float *base, const int32_t *cand,
                         const uint32_t *cand_count, int64_t cap, float *cand_dist, int blocks_per_q,
                         hipStream_t st) {
    dim3 grid(blocks_per_q, nq);
    size_t lds = sizeof(float) * static_cast<size_t>(d);
#define TACO_RR(L, V) k_rerank<L, V><<<grid, BLOCK, lds, st>>>(Q, d, base, cand, cand_count, cap, cand_dist)
    if (d % 4 != 0) {
        TACO_RR(64, false);
    } else {
        switch (rerank_lanes_per_row(d)) {
        case 4: TACO_RR(4, true); break;
        case 8: TACO_RR(8, true); break;
        case 16: TACO_RR(16, true); break;
        case 32: TACO_RR(32, true); break;
        default: TACO_RR(64, true); break;
        }
    }
#undef TACO_RR
    return hipGetLastError();
}

hipError_t launch_rerank16(const float *Q, int nq, int d, const float *mu, const uint16_t *base16,
                           const float *rowerr, const int32_t *cand, const uint32_t *cand_count,
                           int64_t cap, float *ub, float *lb, int blocks_per_q, hipStream_t st) {
    dim3 grid(blocks_per_q, nq);
    size_t lds = sizeof(float) * static_cast<size_t>(d);
#define TACO_RR16(L, V) \
    k_rerank16<L, V><<<grid, BLOCK, lds, st>>>(Q, d, mu, base16, rowerr, cand, cand_count, cap, ub, lb)
    if (d % 8 != 0) {
        TACO_RR16(64, false);
    } else {
        // same lanes per row as the FP32 kernel, each lane reading 16 bytes = 8 values
        switch (rerank_lanes_per_row(d) / 2 < 4 ? 4 : rerank_lanes_per_row(d) / 2) {
        case 4: TACO_RR16(4, true); break;
        case 8: TACO_RR16(8, true); break;
        case 16: TACO_RR16(16, true); break;
        default: TACO_RR16(32, true); break;
        }
    }
#undef TACO_RR16
    return hipGetLastError();
}

hipError_t launch_qbytes(const float *Q, int nq, int d, uint32_t *info, hipStream_t st) {
    if (d % 16 != 0 || d > 256) return hipErrorInvalidValue;
    k_qbytes<<<(nq + WAVES - 1) / WAVES, BLOCK, 0, st>>>(Q, nq, d, info);
    return hipGetLastError();
}

hipError_t launch_rerank8(const float *Q, int nq, int d, const uint8_t *base8, const float4 *meta, bool plain,
                          const int32_t *cand, const uint32_t *cand_count, int64_t cap, float *ub, float *lb,
                          uint32_t *exact, const uint32_t *qinfo, const uint32_t *toff, int T,
                          const int32_t *perm, int blocks_per_q, hipStream_t st) {
    dim3 grid(blocks_per_q, nq);
    size_t lds = sizeof(float) * static_cast<size_t>(d);
#define TACO_RR8(L, V)                                                                                    \
    do {                                                                                                  \
        if (plain)                                                                                        \
            k_rerank8<L, V, true><<<grid, BLOCK, lds, st>>>(Q, d, base8, meta, cand, cand_count, cap, ub, lb, \
                                                            exact, qinfo, toff, T, perm);                     \
        else                                                                                              \
            k_rerank8<L, V, false><<<grid, BLOCK, lds, st>>>(Q, d, base8, meta, cand, cand_count, cap, ub, lb, \
                                                             exact, qinfo, toff, T, perm);                    \
    } while (0)
    if (d % 16 != 0) {
        TACO_RR8(64, false);
    } else {
        // each lane reads 16 bytes = 16 codes; a row's chunks spread over LPR lanes
        const int chunks = d / 16;
        int lpr = 4;
        while (lpr < 32 && lpr * 2 <= chunks) lpr <<= 1;
        switch (lpr) {
        case 4: TACO_RR8(4, true); break;
        case 8: TACO_RR8(8, true); break;
        case 16: TACO_RR8(16, true); break;
        default: TACO_RR8(32, true); break;
        }
    }
#undef TACO_RR8
    return hipGetLastError();
}

hipError_t launch_prep_u8(const float *base, int64_t n, int d, uint8_t *base8, float4 *meta, uint32_t *plain,
                          hipStream_t st) {
    const int64_t blocks = (n + WAVES - 1) / WAVES;
    k_prep_u8<<<static_cast<unsigned>(blocks), BLOCK, 0, st>>>(base, n, d, base8, meta, plain);
    return hipGetLastError();
}

hipError_t launch_recheck_topk(const float *Q, int nq, int d, const float *base, const int32_t *cand,
                               const uint32_t *cand_count, const float *lb, int64_t cap, const float *tau_d,
                               int k, const int32_t *kq, int k_max, int32_t *rk_ids, float *rk_dist,
                               uint32_t *rk_count, int64_t *ids_out, float *d_out, const uint32_t *exact,
                               const int64_t *tau_ids, hipStream_t st) {
    size_t lds = sizeof(float) * static_cast<size_t>(d);
#define TACO_RC(L, V)                                                                                 \
    k_recheck_topk<L, V><<<nq, BLOCK, lds, st>>>(Q, d, base, cand, cand_count, lb, cap, tau_d, k, kq, \
                                                 k_max, rk_ids, rk_dist, rk_count, ids_out, d_out, exact, tau_ids)
    if (d % 4 != 0) {
        TACO_RC(64, false);
    } else {
        switch (rerank_lanes_per_row(d)) {
        case 4: TACO_RC(4, true); break;
        case 8: TACO_RC(8, true); break;
        case 16: TACO_RC(16, true); break;
        case 32: TACO_RC(32, true); break;
        default: TACO_RC(64, true); break;
        }
    }
#undef TACO_RC
    return hipGetLastError();
}

hipError_t launch_prep_bf16(const float *base, int64_t n, int d, const float *mu, uint16_t *base16,
                            float *rowerr, hipStream_t st) {
    k_prep_bf16<<<static_cast<unsigned>((n + WAVES - 1) / WAVES), BLOCK, 0, st>>>(base, n, d, mu,
                                                                                 base16, rowerr);
    return hipGetLastError();
}

hipError_t launch_topk(const int32_t *cand, const float *cand_dist, const uint32_t *cand_count,
                       int64_t cap, int nq, int k, const int32_t *kq, int k_max, int64_t *ids,
                       float *dists, hipStream_t st) {
    k_topk<<<nq, BLOCK, 0, st>>>(cand, cand_dist, cand_count, cap, k, kq, k_max, ids, dists);
    return hipGetLastError();
}

hipError_t launch_stream_topk(const float *Q, int nq, int d, const float *base, const uint32_t *sc, int T, int W,
                              int bits, const uint32_t *hist, int Ns, int64_t n, int64_t R, int rule,
                              const uint32_t *ovf, int k, const int32_t *kq, int k_max, int64_t cap, int32_t *cand,
                              float *cand_dist, uint32_t *cand_count, int64_t *ids, float *dists,
                              hipStream_t st) {
    if (static_cast<int64_t>(ST_SPLIT) * k_max > cap) return hipErrorInvalidValue;
    // ST_SPLIT workgroups per queued query, up to 32 queries at a time (each
    // group of them takes queued queries in turn; none when nothing is queued)
    const dim3 grid(ST_SPLIT, static_cast<unsigned>(std::max(1, std::min(nq, 32))));
    const int64_t row_words = static_cast<int64_t>(T) * W * bits / 32;
    const size_t lds = sizeof(float) * static_cast<size_t>(d);
#define TACO_ST(L, V)                                                                                    \
    do {                                                                                                 \
        if (bits == 4)                                                                                   \
            k_stream_topk<L, V, 4><<<grid, BLOCK, lds, st>>>(Q, d, base, sc, row_words, hist, Ns, n, R,  \
                                                            rule, ovf, k, kq, cap, cand, cand_dist,      \
                                                            cand_count);                                 \
        else                                                                                             \
            k_stream_topk<L, V, 8><<<grid, BLOCK, lds, st>>>(Q, d, base, sc, row_words, hist, Ns, n, R,  \
                                                            rule, ovf, k, kq, cap, cand, cand_dist,      \
                                                            cand_count);                                 \
    } while (0)
    if (d % 4 != 0) {
        TACO_ST(64, false);
    } else {
        switch (rerank_lanes_per_row(d)) {
        case 4: TACO_ST(4, true); break;
        case 8: TACO_ST(8, true); break;
        case 16: TACO_ST(16, true); break;
        case 32: TACO_ST(32, true); break;
        default: TACO_ST(64, true); break;
        }
    }
#undef TACO_ST
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_topk_queued<<<static_cast<unsigned>(std::max(1, std::min(nq, 256))), BLOCK, 0, st>>>(
        cand, cand_dist, cand_count, cap, ovf, k, kq, k_max, ids, dists);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// SC-Linear (Section 2.3; Definitions 5 and 6): exact collisions, no index.
// A point collides with the query in subspace j when its key (distance bits
// << 32 | id) is among the A smallest of that subspace; distances use the
// canonical FP32 chain over the subspace's columns of the transformed base.
// ---------------------------------------------------------------------------

// D[q][j][i] = sum_c fmaf(u, u) with u = qt[q][j*s+c] - T[i][j*s+c], c
// ascending (T row-major [n][M]).  grid (ceil(n/256), ceil(nq/SD_Q)), block
// 256: one point per thread, SD_Q queries per block from LDS.
constexpr int SD_Q = 8;

__global__ __launch_bounds__(256) void k_sub_dist(const float *__restrict__ T, int64_t n, int M, int Ns, int s,
                                                  const float *__restrict__ qt, int nq, float *__restrict__ D) {
    extern __shared__ float sq[];  // [SD_Q][M]
    const int q0 = blockIdx.y * SD_Q;
    const int nqb = min(SD_Q, nq - q0);
    for (int i = threadIdx.x; i < nqb * M; i += blockDim.x) sq[i] = qt[static_cast<int64_t>(q0) * M + i];
    __syncthreads();
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *row = T + i * M;
    for (int j = 0; j < Ns; j++) {
        float acc[SD_Q];
#pragma unroll
        for (int b = 0; b < SD_Q; b++) acc[b] = 0.0f;
        for (int c = 0; c < s; c++) {
            const float x = row[j * s + c];
#pragma unroll
            for (int b = 0; b < SD_Q; b++) {
                const float u = sq[b * M + j * s + c] - x;
                acc[b] = fmaf(u, u, acc[b]);
            }
        }
#pragma unroll
        for (int b = 0; b < SD_Q; b++)
            if (b < nqb) D[(static_cast<int64_t>(q0 + b) * Ns + j) * n + i] = acc[b];
    }
}

// Adds one to bin `b` of the LDS histogram for every active lane, one LDS
// add per distinct bin of the wavefront: lanes holding the first active
// lane's bin are folded into a single add (distances share their top bits,
// so most lanes of a pass agree).
__device__ __forceinline__ void wave_hist_add(uint32_t *hist, uint32_t b, bool active) {
    uint64_t pend = __ballot(active);
    while (pend) {
        const int lead = __ffsll(static_cast<unsigned long long>(pend)) - 1;
        const uint32_t lb = static_cast<uint32_t>(__shfl(static_cast<int>(b), lead, WAVE));
        const uint64_t same = __ballot(active && b == lb) & pend;
        if ((threadIdx.x % WAVE) == lead) atomicAdd(&hist[lb], static_cast<uint32_t>(__popcll(same)));
        pend &= ~same;
    }
}

// The A-th smallest key (distance bits << 32 | id) of each (query,
// subspace): an MSB-first radix select on the distance bits, 8 bits per pass
// over the keys whose higher bits match the digits chosen so far, then the
// r-th smallest id among the keys with that distance, by a pass in id
// order with workgroup prefix counts.  grid (Ns, nq), block SS_BLOCK.
constexpr int SS_BLOCK = 1024;

__global__ __launch_bounds__(SS_BLOCK) void k_sub_select(const float *__restrict__ D, int64_t n, int Ns, int64_t A,
                                                         uint64_t *__restrict__ thr) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_digit, s_rank, s_wsum[SS_BLOCK / WAVE];
    __shared__ uint32_t s_id;
    const int j = blockIdx.x, q = blockIdx.y;
    const uint32_t *key = reinterpret_cast<const uint32_t *>(D + (static_cast<int64_t>(q) * Ns + j) * n);
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    uint32_t prefix = 0u, pmask = 0u;
    uint32_t rank = static_cast<uint32_t>(A);  // 1-based rank among the keys matching the prefix
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += SS_BLOCK) hist[b] = 0u;
        __syncthreads();
        for (int64_t i0 = 0; i0 < n; i0 += SS_BLOCK) {
            const int64_t i = i0 + tid;
            const uint32_t k = i < n ? key[i] : 0u;
            const bool in = i < n && (k & pmask) == prefix;
            wave_hist_add(hist, (k >> shift) & 0xffu, in);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t cum = 0u, d = 0u;
            for (; d < 255u; d++) {
                if (cum + hist[d] >= rank) break;
                cum += hist[d];
            }
            s_digit = d;
            s_rank = rank - cum;
        }
        __syncthreads();
        prefix |= s_digit << shift;
        pmask |= 0xffu << shift;
        rank = s_rank;
        __syncthreads();
    }
    // the rank-th id (ascending) among the keys equal to `prefix`
    uint32_t seen = 0u;
    if (tid == 0) s_id = 0xffffffffu;
    __syncthreads();
    for (int64_t i0 = 0; i0 < n; i0 += SS_BLOCK) {
        const int64_t i = i0 + tid;
        const uint32_t f = (i < n && key[i] == prefix) ? 1u : 0u;
        const uint32_t incl = wave_incl_scan_u32(f, lane);
        if (lane == WAVE - 1) s_wsum[wv] = incl;
        __syncthreads();
        uint32_t before = seen;
        for (int w = 0; w < wv; w++) before += s_wsum[w];
        if (f && before + incl == rank) s_id = static_cast<uint32_t>(i);
        uint32_t tot = 0u;
        for (int w = 0; w < SS_BLOCK / WAVE; w++) tot += s_wsum[w];
        seen += tot;
        __syncthreads();
        if (s_id != 0xffffffffu) break;
    }
    if (tid == 0) thr[static_cast<int64_t>(q) * Ns + j] = (static_cast<uint64_t>(prefix) << 32) | s_id;
}

// SC-scores from the thresholds, packed BITS per id (ids past n score 0),
// and the level histogram (levels >= 1, atomically into hist[q]).  grid
// (ceil(words / 256), nq), block 256: one 32-bit word of counts per thread.
template <int BITS>
__global__ __launch_bounds__(256) void k_sub_count(const float *__restrict__ D, int64_t n, int Ns,
                                                   const uint64_t *__restrict__ thr, int64_t words,
                                                   uint32_t *__restrict__ sc, uint32_t *__restrict__ hist) {
    constexpr int PER_WORD = 32 / BITS;
    __shared__ uint32_t lh[17];
    const int q = blockIdx.y;
    if (threadIdx.x <= 16) lh[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (w < words) {
        uint32_t word = 0u;
        for (int b = 0; b < PER_WORD; b++) {
            const int64_t id = w * PER_WORD + b;
            if (id >= n) break;
            uint32_t c = 0u;
            for (int j = 0; j < Ns; j++) {
                const uint32_t kb = __float_as_uint(D[(static_cast<int64_t>(q) * Ns + j) * n + id]);
                const uint64_t key = (static_cast<uint64_t>(kb) << 32) | static_cast<uint64_t>(id);
                c += key <= thr[static_cast<int64_t>(q) * Ns + j] ? 1u : 0u;
            }
            word |= c << (BITS * b);
            if (c) atomicAdd(&lh[c], 1u);
        }
        sc[static_cast<int64_t>(q) * words + w] = word;
    }
    __syncthreads();
    if (threadIdx.x >= 1 && threadIdx.x <= Ns && lh[threadIdx.x])
        atomicAdd(&hist[static_cast<int64_t>(q) * (Ns + 1) + threadIdx.x], lh[threadIdx.x]);
}

hipError_t launch_sub_dist(const float *T, int64_t n, int M, int Ns, int s, const float *qt, int nq, float *D,
                           hipStream_t st) {
    dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>((nq + SD_Q - 1) / SD_Q));
    k_sub_dist<<<grid, 256, sizeof(float) * SD_Q * M, st>>>(T, n, M, Ns, s, qt, nq, D);
    return hipGetLastError();
}

hipError_t launch_sub_select(const float *D, int64_t n, int Ns, int nq, int64_t A, uint64_t *thr, hipStream_t st) {
    k_sub_select<<<dim3(Ns, nq), SS_BLOCK, 0, st>>>(D, n, Ns, A, thr);
    return hipGetLastError();
}

hipError_t launch_sub_count(const float *D, int64_t n, int Ns, int nq, const uint64_t *thr, int T, int W, int bits,
                            uint32_t *sc, uint32_t *hist, hipStream_t st) {
    const int64_t words = static_cast<int64_t>(T) * W * bits / 32;
    dim3 grid(static_cast<unsigned>((words + 255) / 256), static_cast<unsigned>(nq));
    if (bits == 4)
        k_sub_count<4><<<grid, 256, 0, st>>>(D, n, Ns, thr, words, sc, hist);
    else
        k_sub_count<8><<<grid, 256, 0, st>>>(D, n, Ns, thr, words, sc, hist);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Point-major counting ("code scan", TC_COUNT_CODES).  Instead of walking the
// probed cells' id lists, every point's Ns cell codes are tested against
// bitmaps of each query's probed cells held in LDS, for CC_G queries per
// pass over the codes.  The work is n * Ns bitmap reads per query whatever
// the budget, against sum_j R_j increments for the list walk: the form for
// large collision ratios.  Output as k_count's split form: packed counts and
// the level histogram (levels >= 1).
// ---------------------------------------------------------------------------

// codes[i][j] (row stride cs u16) = the cell of point i in subspace j; rows
// padded past Ns with 0.  grid over the Ns*n list entries, block 256.
__global__ void k_build_codes(const uint32_t *__restrict__ ids, const uint32_t *__restrict__ offs, int Ns, int K,
                              int64_t n, int cs, uint16_t *__restrict__ codes) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= static_cast<int64_t>(Ns) * n) return;
    const int j = static_cast<int>(e / n);
    const uint32_t p = static_cast<uint32_t>(e - static_cast<int64_t>(j) * n);
    const uint32_t *o = offs + static_cast<int64_t>(j) * (K + 1);
    int lo = 0, hi = K;  // the cell c with o[c] <= p < o[c+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (o[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    codes[static_cast<int64_t>(ids[e]) * cs + j] = static_cast<uint16_t>(lo);
}

// bm[q][j][KW] = bit c set when query q probed cell c of subspace j.  grid
// nq, block 256, LDS Ns*KW words.
__global__ __launch_bounds__(256) void k_cell_bitmap(const int32_t *__restrict__ cells,
                                                     const int32_t *__restrict__ ncells, int Ns, int K, int KW,
                                                     uint32_t *__restrict__ bm) {
    extern __shared__ uint32_t b[];
    const int q = blockIdx.x;
    for (int i = threadIdx.x; i < Ns * KW; i += blockDim.x) b[i] = 0u;
    __syncthreads();
    for (int j = 0; j < Ns; j++) {
        const int nc = ncells[static_cast<int64_t>(q) * Ns + j];
        const int32_t *cj = cells + (static_cast<int64_t>(q) * Ns + j) * K;
        for (int i = threadIdx.x; i < nc; i += blockDim.x) {
            const int c = cj[i];
            atomicOr(&b[j * KW + (c >> 5)], 1u << (c & 31));
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Ns * KW; i += blockDim.x) bm[static_cast<int64_t>(q) * Ns * KW + i] = b[i];
}

constexpr int CC_G = 16;     // queries per pass over the codes
constexpr int CC_PTS = 8;    // points per thread and chunk (one nibble word, two byte words)

// Adds the per-lane level counts of `lo` (byte c: points of count c < 8),
// `hi` (byte c - 8: 8 <= c < 16) and `top` (count 16) of the wavefront to
// h[1..Ns].  Each byte is at most CC_PTS; the 16-bit sums cannot carry.
__device__ __forceinline__ void code_hist_fold(uint64_t lo, uint64_t hi, uint32_t top, int Ns, uint32_t *h,
                                               int lane) {
    uint64_t xs[2] = {lo, hi};
#pragma unroll
    for (int part = 0; part < 2; part++) {
        if (part == 1 && Ns < 8) break;
        const uint64_t x = xs[part];
        if (!__any(x != 0ull)) continue;
        const uint64_t ev = x & 0x00FF00FF00FF00FFull, od = (x >> 8) & 0x00FF00FF00FF00FFull;
        const uint32_t s0 = wave_sum_u32(static_cast<uint32_t>(ev)), s1 = wave_sum_u32(static_cast<uint32_t>(ev >> 32));
        const uint32_t s2 = wave_sum_u32(static_cast<uint32_t>(od)), s3 = wave_sum_u32(static_cast<uint32_t>(od >> 32));
        if (lane == 0) {
            const uint32_t v[8] = {s0 & 0xffffu, s2 & 0xffffu, s0 >> 16, s2 >> 16,
                                   s1 & 0xffffu, s3 & 0xffffu, s1 >> 16, s3 >> 16};
#pragma unroll
            for (int c = 0; c < 8; c++) {
                const int lv = part * 8 + c;
                if (lv >= 1 && lv <= Ns && v[c]) atomicAdd(&h[lv], v[c]);
            }
        }
    }
    if (Ns >= 16) {
        const uint32_t t = wave_sum_u32(top);
        if (lane == 0 && t) atomicAdd(&h[16], t);
    }
}

// grid (chunk workers, ceil(nq / CC_G)), block 256; LDS: the group's bitmaps
// (CC_G * Ns * KW words) and its histograms (CC_G * 17 words).  Each thread
// takes CC_PTS consecutive points per chunk, keeps their codes in registers
// and, query by query, sums the Ns bitmap bits of each point.
template <int BITS, int CS>
__global__ __launch_bounds__(256) void k_count_codes(const uint16_t *__restrict__ codes, int64_t n, int Ns, int KW,
                                                     const uint32_t *__restrict__ bm, int nq, int64_t words,
                                                     uint32_t *__restrict__ sc, uint32_t *__restrict__ hist) {
    constexpr int PER_WORD = 32 / BITS;
    constexpr int WPT = CC_PTS / PER_WORD;  // output words per thread and chunk
    extern __shared__ uint32_t lds[];
    const int q0 = blockIdx.y * CC_G;
    const int G = min(CC_G, nq - q0);
    uint32_t *bl = lds;                         // [CC_G][Ns][KW]
    uint32_t *hl = lds + CC_G * Ns * KW;        // [CC_G][17]
    for (int i = threadIdx.x; i < G * Ns * KW; i += blockDim.x) bl[i] = bm[static_cast<int64_t>(q0) * Ns * KW + i];
    for (int i = threadIdx.x; i < CC_G * 17; i += blockDim.x) hl[i] = 0u;
    __syncthreads();
    const int lane = threadIdx.x % WAVE;
    const int64_t chunk = static_cast<int64_t>(blockDim.x) * CC_PTS;
    for (int64_t c0 = static_cast<int64_t>(blockIdx.x) * chunk; c0 < n; c0 += static_cast<int64_t>(gridDim.x) * chunk) {
        const int64_t p0 = c0 + static_cast<int64_t>(threadIdx.x) * CC_PTS;
        // the codes of this thread's points (CS/8 16-byte loads per point)
        uint4 cw[CC_PTS][CS / 8];
#pragma unroll
        for (int p = 0; p < CC_PTS; p++)
#pragma unroll
            for (int v = 0; v < CS / 8; v++)
                cw[p][v] = p0 + p < n ? reinterpret_cast<const uint4 *>(codes + (p0 + p) * CS)[v]
                                      : make_uint4(0u, 0u, 0u, 0u);
        for (int g = 0; g < G; g++) {
            const uint32_t *bg = bl + g * Ns * KW;
            uint32_t out[WPT] = {};
            uint64_t lo = 0ull, hi = 0ull;
            uint32_t top = 0u;
#pragma unroll
            for (int p = 0; p < CC_PTS; p++) {
                uint32_t c = 0u;
#pragma unroll
                for (int j = 0; j < CS; j++) {
                    if (j < Ns) {
                        const uint4 v4 = cw[p][j / 8];
                        const uint32_t w32 = (j % 8) < 2 ? v4.x : (j % 8) < 4 ? v4.y : (j % 8) < 6 ? v4.z : v4.w;
                        const uint32_t code = (j % 2) ? (w32 >> 16) : (w32 & 0xffffu);
                        c += (bg[j * KW + (code >> 5)] >> (code & 31u)) & 1u;
                    }
                }
                if (p0 + p >= n) c = 0u;
                out[p / PER_WORD] |= c << (BITS * (p % PER_WORD));
                const uint64_t inc = 1ull << ((c & 7u) << 3);
                if (c < 8u)
                    lo += c ? inc : 0ull;
                else if (c < 16u)
                    hi += inc;
                else
                    top += 1u;
            }
            const int64_t w0 = p0 / PER_WORD;
#pragma unroll
            for (int u = 0; u < WPT; u++)
                if (w0 + u < words) sc[static_cast<int64_t>(q0 + g) * words + w0 + u] = out[u];
            code_hist_fold(lo, hi, top, Ns, hl + g * 17, lane);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < G * 17; i += blockDim.x) {
        const int g = i / 17, v = i % 17;
        if (v >= 1 && v <= Ns && hl[i]) atomicAdd(&hist[static_cast<int64_t>(q0 + g) * (Ns + 1) + v], hl[i]);
    }
}

int code_stride(int Ns) { return Ns <= 8 ? 8 : 16; }

hipError_t launch_build_codes(const uint32_t *ids, const uint32_t *offs, int Ns, int K, int64_t n, uint16_t *codes,
                              hipStream_t st) {
    const int64_t e = static_cast<int64_t>(Ns) * n;
    hipError_t r = hipMemsetAsync(codes, 0, sizeof(uint16_t) * static_cast<size_t>(n) * code_stride(Ns), st);
    if (r != hipSuccess) return r;
    k_build_codes<<<static_cast<unsigned>((e + 255) / 256), 256, 0, st>>>(ids, offs, Ns, K, n, code_stride(Ns), codes);
    return hipGetLastError();
}

size_t codes_lds_bytes(int Ns, int K) {
    const int KW = (K + 31) / 32;
    return sizeof(uint32_t) * (static_cast<size_t>(CC_G) * Ns * KW + CC_G * 17);
}

hipError_t launch_count_codes(const uint16_t *codes, const int32_t *cells, const int32_t *ncells, int nq, int Ns,
                              int K, int64_t n, int T, int W, int bits, uint32_t *bm, uint32_t *sc, uint32_t *hist,
                              int num_cu, hipStream_t st) {
    const int KW = (K + 31) / 32;
    k_cell_bitmap<<<nq, 256, sizeof(uint32_t) * Ns * KW, st>>>(cells, ncells, Ns, K, KW, bm);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    const int64_t words = static_cast<int64_t>(T) * W * bits / 32;
    const int64_t chunks = (n + 256 * CC_PTS - 1) / (256 * CC_PTS);
    const int groups = (nq + CC_G - 1) / CC_G;
    // enough workgroups to fill the GPU a few times over, each taking whole
    // chunks of points (every query group re-reads the codes)
    int64_t gx = (int64_t(num_cu) * 8 + groups - 1) / groups;
    gx = std::max<int64_t>(1, std::min<int64_t>(gx, chunks));
    dim3 grid(static_cast<unsigned>(gx), static_cast<unsigned>(groups));
    const size_t lds = codes_lds_bytes(Ns, K);
    if (bits == 4) {
        if (code_stride(Ns) == 8)
            k_count_codes<4, 8><<<grid, 256, lds, st>>>(codes, n, Ns, KW, bm, nq, words, sc, hist);
        else
            k_count_codes<4, 16><<<grid, 256, lds, st>>>(codes, n, Ns, KW, bm, nq, words, sc, hist);
    } else {
        k_count_codes<8, 16><<<grid, 256, lds, st>>>(codes, n, Ns, KW, bm, nq, words, sc, hist);
    }
    return hipGetLastError();
}

}  // namespace taco

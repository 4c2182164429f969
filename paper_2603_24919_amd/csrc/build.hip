// Index construction on the GPU: the statistics and spectral decomposition
// of Alg 1, the per-half k-means and the inverted multi-index of Alg 3.
//
// Arithmetic that decides integers (k-means labels, cell membership) follows
// one fixed order so that results are reproducible bit for bit:
//   * k-means training runs in FP64: a point's distance to a centroid is
//     s <- s + u*u over u = x_t - c_t, t ascending, each operation rounded
//     (no fused multiply-add; the library is built with contraction off);
//     the nearest centroid wins, ties to the lower id;
//   * centroid sums are formed per block of KM_BLOCK sample positions, each
//     in ascending position order, and the blocks are then added in order;
//   * the final label of every row uses the FP32 chain of the query side:
//     acc <- fmaf(u, u, acc), u = fl32(x_t - c_t), t ascending.
// Mean and covariance are FP64 sums over fixed row chunks, added in chunk
// order.
#include "build.h"

#include <algorithm>

namespace taco {
namespace bld {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Sum over the workgroup, same order every call; every thread gets it.
template <int BLOCK>
__device__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if ((threadIdx.x % WAVE) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < BLOCK / WAVE; i++) s += red[i];
    return s;
}

// ---------------------------------------------------------------------------
// Mean and covariance.
// ---------------------------------------------------------------------------

constexpr int ST_CHUNKS = 1024;   // row chunks of the column sums
constexpr int CV_TILE = 64;       // covariance output tile
constexpr int CV_ROWS = 16;       // rows staged per step
constexpr int CV_CHUNKS = 256;    // row chunks of the covariance

int64_t chunk_rows(int64_t n, int chunks) { return (n + chunks - 1) / chunks; }

// part[c][t] = sum of X[r][t] over the rows r of chunk c, ascending.
__global__ __launch_bounds__(256) void k_colsum(const float *__restrict__ X, int64_t n, int d,
                                                int64_t rows, double *__restrict__ part) {
    const int64_t lo = blockIdx.x * rows;
    const int64_t hi = min(lo + rows, n);
    for (int t = threadIdx.x; t < d; t += 256) {
        double s = 0.0;
        for (int64_t r = lo; r < hi; r++) s += static_cast<double>(X[r * d + t]);
        part[static_cast<int64_t>(blockIdx.x) * d + t] = s;
    }
}

__global__ __launch_bounds__(256) void k_mean(const double *__restrict__ part, int chunks, int64_t n,
                                              int d, double *__restrict__ mean) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= d) return;
    double s = 0.0;
    for (int c = 0; c < chunks; c++) s += part[static_cast<int64_t>(c) * d + t];
    mean[t] = s / static_cast<double>(n);
}

// Upper-triangle tile u -> (bi, bj), bi <= bj, row-major over the triangle.
__device__ __forceinline__ void tile_of(int u, int nb, int &bi, int &bj) {
    int i = 0;
    while (u >= nb - i) {
        u -= nb - i;
        i++;
    }
    bi = i;
    bj = i + u;
}

// part[chunk][u][64][64]: sum over the chunk's rows of (x - m)_a (x - m)_b for
// a in tile row bi, b in tile column bj.  block (16, 16), 4x4 outputs each.
__global__ __launch_bounds__(256) void k_cov_part(const float *__restrict__ X, int64_t n, int d,
                                                  const double *__restrict__ mean, int64_t rows,
                                                  int nb, double *__restrict__ part) {
    __shared__ double A[CV_ROWS][CV_TILE];
    __shared__ double Bs[CV_ROWS][CV_TILE];
    int bi, bj;
    tile_of(blockIdx.x, nb, bi, bj);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t lo = blockIdx.y * rows;
    const int64_t hi = min(lo + rows, n);
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc[u][v] = 0.0;
    for (int64_t r0 = lo; r0 < hi; r0 += CV_ROWS) {
        for (int i = threadIdx.x; i < CV_ROWS * CV_TILE; i += 256) {
            const int rr = i / CV_TILE, cc = i % CV_TILE;
            const int64_t r = r0 + rr;
            const int ca = bi * CV_TILE + cc, cb = bj * CV_TILE + cc;
            double va = 0.0, vb = 0.0;
            if (r < hi) {
                if (ca < d) va = static_cast<double>(X[r * d + ca]) - mean[ca];
                if (cb < d) vb = static_cast<double>(X[r * d + cb]) - mean[cb];
            }
            A[rr][cc] = va;
            Bs[rr][cc] = vb;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < CV_ROWS; rr++) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; u++) a[u] = A[rr][ty * 4 + u];
#pragma unroll
            for (int v = 0; v < 4; v++) b[v] = Bs[rr][tx * 4 + v];
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int v = 0; v < 4; v++) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
    double *out = part + (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * CV_TILE * CV_TILE;
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
        for (int v = 0; v < 4; v++) out[(ty * 4 + u) * CV_TILE + tx * 4 + v] = acc[u][v];
}

// cov[a][b] = cov[b][a] = (sum over chunks of the (min, max) entry) / (n - 1).
__global__ __launch_bounds__(256) void k_cov_final(const double *__restrict__ part, int chunks,
                                                   int ntile, int nb, int64_t n, int d,
                                                   double *__restrict__ cov) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= static_cast<int64_t>(d) * d) return;
    int a = static_cast<int>(e / d), b = static_cast<int>(e % d);
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
    const int bi = a / CV_TILE, bj = b / CV_TILE;
    const int u = bi * nb - bi * (bi - 1) / 2 + (bj - bi);
    const int64_t off = static_cast<int64_t>(u) * CV_TILE * CV_TILE + (a % CV_TILE) * CV_TILE + (b % CV_TILE);
    double s = 0.0;
    for (int c = 0; c < chunks; c++) s += part[static_cast<int64_t>(c) * ntile * CV_TILE * CV_TILE + off];
    cov[e] = s / static_cast<double>(n - 1);
}

// ---------------------------------------------------------------------------
// Spectral decomposition: cyclic Jacobi with the round-robin ordering, so
// every step applies dp/2 disjoint rotations at once.  The matrix stays in
// LDS, the accumulated rotations V in global memory.  An odd d is padded by
// one zero row and column, which no rotation touches (its coupling is 0).
// ---------------------------------------------------------------------------

constexpr int EIG_BLOCK = 1024;
constexpr int EIG_SWEEPS = 40;

__global__ __launch_bounds__(EIG_BLOCK) void k_jacobi(const double *__restrict__ cov, int d, int dp,
                                                      double *__restrict__ evals,
                                                      double *__restrict__ evecs,
                                                      double *__restrict__ V) {
    extern __shared__ double A[];  // [dp][dp]
    __shared__ double cs[EIG_MAX];
    __shared__ int pq[EIG_MAX];
    __shared__ double red[EIG_BLOCK / WAVE];
    __shared__ int rank[EIG_MAX];
    const int tid = threadIdx.x;
    const int np = dp / 2;
    for (int i = tid; i < dp * dp; i += EIG_BLOCK) {
        const int r = i / dp, c = i % dp;
        A[i] = (r < d && c < d) ? cov[r * d + c] : 0.0;
        V[i] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    double f = 0.0;
    for (int i = tid; i < dp * dp; i += EIG_BLOCK) f += A[i] * A[i];
    const double fro = block_sum<EIG_BLOCK>(f, red);
    // Stop once the off-diagonal mass is below (1e-13 |A|_F)^2.
    const double tol = 1e-26 * fro;
    for (int sweep = 0; sweep < EIG_SWEEPS; sweep++) {
        double o = 0.0;
        for (int i = tid; i < dp * dp; i += EIG_BLOCK)
            if (i / dp != i % dp) o += A[i] * A[i];
        const double off = block_sum<EIG_BLOCK>(o, red);
        if (!(off > tol)) break;
        for (int step = 0; step < dp - 1; step++) {
            if (tid < np) {
                // Circle method: slot 0 fixed, slots 1..dp-1 rotate by step;
                // slot i meets slot dp-1-i.
                const int a = tid == 0 ? 0 : 1 + (tid - 1 + step) % (dp - 1);
                const int b = 1 + (dp - 2 - tid + step) % (dp - 1);
                const int p = min(a, b), q = max(a, b);
                const double apq = A[p * dp + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    const double tau = (A[q * dp + q] - A[p * dp + p]) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                pq[2 * tid] = p;
                pq[2 * tid + 1] = q;
                cs[2 * tid] = c;
                cs[2 * tid + 1] = s;
            }
            __syncthreads();
            // rows p, q of J^T A
            for (int i = tid; i < np * dp; i += EIG_BLOCK) {
                const int r = i / dp, k = i % dp;
                const int p = pq[2 * r], q = pq[2 * r + 1];
                const double c = cs[2 * r], s = cs[2 * r + 1];
                const double ap = A[p * dp + k], aq = A[q * dp + k];
                A[p * dp + k] = c * ap - s * aq;
                A[q * dp + k] = s * ap + c * aq;
            }
            __syncthreads();
            // columns p, q of (J^T A) J and of V J
            for (int i = tid; i < np * dp; i += EIG_BLOCK) {
                const int r = i % np, k = i / np;
                const int p = pq[2 * r], q = pq[2 * r + 1];
                const double c = cs[2 * r], s = cs[2 * r + 1];
                const double ap = A[k * dp + p], aq = A[k * dp + q];
                A[k * dp + p] = c * ap - s * aq;
                A[k * dp + q] = s * ap + c * aq;
                const double vp = V[k * dp + p], vq = V[k * dp + q];
                V[k * dp + p] = c * vp - s * vq;
                V[k * dp + q] = s * vp + c * vq;
            }
            __syncthreads();
            if (tid < np && cs[2 * tid + 1] != 0.0) {
                const int p = pq[2 * tid], q = pq[2 * tid + 1];
                A[p * dp + q] = 0.0;
                A[q * dp + p] = 0.0;
            }
            __syncthreads();
        }
    }
    // Descending order (ties to the lower index) and sign convention.
    if (tid < d) {
        const double li = A[tid * dp + tid];
        int r = 0;
        for (int j = 0; j < d; j++) {
            const double lj = A[j * dp + j];
            r += (lj > li) || (lj == li && j < tid);
        }
        rank[tid] = r;
        evals[r] = li;
        int piv = 0;
        double best = -1.0;
        for (int k = 0; k < d; k++) {
            const double m = fabs(V[k * dp + tid]);
            if (m > best) {
                best = m;
                piv = k;
            }
        }
        cs[tid] = V[piv * dp + tid] < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
    for (int i = tid; i < d * d; i += EIG_BLOCK) {
        const int k = i / d, c = i % d;
        evecs[k * d + rank[c]] = cs[c] * V[k * dp + c];
    }
}

// ---------------------------------------------------------------------------
// Spectral decomposition for larger d: one-sided (Hestenes) Jacobi.  U = A V
// is kept column by column; each step orthogonalizes dp/2 disjoint column
// pairs (round-robin ordering, one workgroup per pair) and applies the same
// rotation to V.  At convergence the columns of U are lambda_i v_i, so for
// the positive semi-definite covariance lambda_i = sign(u_i . v_i) |u_i|.
// Columns are contiguous (column-major), so no step needs a grid-wide
// barrier; the host launches steps and checks a rotation counter per sweep.
// ---------------------------------------------------------------------------

constexpr int OSJ_BLOCK = 256;
constexpr int OSJ_SWEEPS = 40;
constexpr double OSJ_EPS = 2.220446049250313e-16;  // rotate while |u_p.u_q| > dp eps |u_p| |u_q|

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

// U (column-major) = A, padded by a zero column and row for odd d; V = I.
__global__ __launch_bounds__(256) void k_osj_init(const double *__restrict__ cov, int d, int dp,
                                                  double *__restrict__ U, double *__restrict__ V) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i >= static_cast<int64_t>(dp) * dp) return;
    const int c = static_cast<int>(i / dp), r = static_cast<int>(i % dp);
    U[i] = (r < d && c < d) ? cov[static_cast<int64_t>(r) * d + c] : 0.0;
    V[i] = r == c ? 1.0 : 0.0;
}

__global__ __launch_bounds__(OSJ_BLOCK) void k_osj_step(double *__restrict__ U, double *__restrict__ V,
                                                        int dp, int step, uint32_t *__restrict__ rotated) {
    __shared__ double red[3][OSJ_BLOCK / WAVE];
    const int pr = blockIdx.x;
    const int a = pr == 0 ? 0 : 1 + (pr - 1 + step) % (dp - 1);
    const int b = 1 + (dp - 2 - pr + step) % (dp - 1);
    const int p = min(a, b), q = max(a, b);
    double *up = U + static_cast<int64_t>(p) * dp, *uq = U + static_cast<int64_t>(q) * dp;
    double *vp = V + static_cast<int64_t>(p) * dp, *vq = V + static_cast<int64_t>(q) * dp;
    double al = 0.0, be = 0.0, ga = 0.0;
    for (int r = threadIdx.x; r < dp; r += OSJ_BLOCK) {
        const double x = up[r], y = uq[r];
        al += x * x;
        be += y * y;
        ga += x * y;
    }
    al = wave_sum(al);
    be = wave_sum(be);
    ga = wave_sum(ga);
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x % WAVE) == 0) {
        red[0][w] = al;
        red[1][w] = be;
        red[2][w] = ga;
    }
    __syncthreads();
    al = be = ga = 0.0;
    for (int i = 0; i < OSJ_BLOCK / WAVE; i++) {
        al += red[0][i];
        be += red[1][i];
        ga += red[2][i];
    }
    if (!(fabs(ga) > dp * OSJ_EPS * sqrt(al * be)) || ga == 0.0) return;  // uniform
    const double zeta = (be - al) / (2.0 * ga);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
    for (int r = threadIdx.x; r < dp; r += OSJ_BLOCK) {
        const double x = up[r], y = uq[r];
        up[r] = c * x - sn * y;
        uq[r] = sn * x + c * y;
        const double xv = vp[r], yv = vq[r];
        vp[r] = c * xv - sn * yv;
        vq[r] = sn * xv + c * yv;
    }
    if (threadIdx.x == 0) atomicAdd(rotated, 1u);
}

// lam[i] = sign(u_i . v_i) |u_i|, one workgroup per column i < d.
__global__ __launch_bounds__(OSJ_BLOCK) void k_osj_values(const double *__restrict__ U,
                                                          const double *__restrict__ V, int dp,
                                                          double *__restrict__ lam) {
    __shared__ double red[2][OSJ_BLOCK / WAVE];
    const int i = blockIdx.x;
    const double *u = U + static_cast<int64_t>(i) * dp, *v = V + static_cast<int64_t>(i) * dp;
    double nn = 0.0, uv = 0.0;
    for (int r = threadIdx.x; r < dp; r += OSJ_BLOCK) {
        nn += u[r] * u[r];
        uv += u[r] * v[r];
    }
    nn = wave_sum(nn);
    uv = wave_sum(uv);
    if ((threadIdx.x % WAVE) == 0) {
        red[0][threadIdx.x / WAVE] = nn;
        red[1][threadIdx.x / WAVE] = uv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        nn = uv = 0.0;
        for (int k = 0; k < OSJ_BLOCK / WAVE; k++) {
            nn += red[0][k];
            uv += red[1][k];
        }
        lam[i] = uv < 0.0 ? -sqrt(nn) : sqrt(nn);
    }
}

// Descending order (ties to the lower index) and the sign convention; one
// thread per eigenpair.  rank and sign: [d] scratch.
__global__ __launch_bounds__(256) void k_osj_order(const double *__restrict__ lam, const double *__restrict__ V,
                                                   int d, int dp, double *__restrict__ evals,
                                                   int *__restrict__ rank, double *__restrict__ sgn) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= d) return;
    const double li = lam[i];
    int r = 0;
    for (int j = 0; j < d; j++) r += (lam[j] > li) || (lam[j] == li && j < i);
    rank[i] = r;
    evals[r] = li;
    const double *v = V + static_cast<int64_t>(i) * dp;
    int piv = 0;
    double best = -1.0;
    for (int k = 0; k < d; k++) {
        const double m = fabs(v[k]);
        if (m > best) {
            best = m;
            piv = k;
        }
    }
    sgn[i] = v[piv] < 0.0 ? -1.0 : 1.0;
}

__global__ __launch_bounds__(256) void k_osj_vectors(const double *__restrict__ V, int d, int dp,
                                                     const int *__restrict__ rank, const double *__restrict__ sgn,
                                                     double *__restrict__ evecs) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= static_cast<int64_t>(d) * d) return;
    const int c = static_cast<int>(e / d), k = static_cast<int>(e % d);
    evecs[static_cast<int64_t>(k) * d + rank[c]] = sgn[c] * V[static_cast<int64_t>(c) * dp + k];
}

// ---------------------------------------------------------------------------
// k-means, all 2*Ns halves in one grid dimension.
// ---------------------------------------------------------------------------

struct Half {
    int off, h;
};

__device__ __forceinline__ Half half_of(int g, int s) {
    const int h1 = s / 2;
    Half r;
    r.off = (g / 2) * s + ((g & 1) ? h1 : 0);
    r.h = (g & 1) ? s - h1 : h1;
    return r;
}

__device__ __forceinline__ int64_t row_of(const int64_t *train, int64_t p) { return train ? train[p] : p; }

// cent[g][c][:h] = the seed point's half, in FP64.
__global__ __launch_bounds__(256) void k_km_seed(KmArgs a, int HM, int nblk, double *__restrict__ cent,
                                                 uint32_t *__restrict__ pcnt) {
    const int g = blockIdx.x;
    const Half H = half_of(g, a.s);
    for (int i = threadIdx.x; i < nblk * a.l; i += 256) pcnt[static_cast<int64_t>(g) * nblk * a.l + i] = 0u;
    for (int i = threadIdx.x; i < a.l * H.h; i += 256) {
        const int c = i / H.h, t = i % H.h;
        const int64_t r = row_of(a.train, a.init[static_cast<int64_t>(g) * a.l + c]);
        cent[(static_cast<int64_t>(g) * a.l + c) * HM + t] = static_cast<double>(a.T[r * a.ld + H.off + t]);
    }
}

constexpr int KM_APW = 256;  // sample positions per assignment workgroup (one per thread)
static_assert(KM_BLOCK % KM_APW == 0, "a label-counting workgroup must lie in one block");

// Label and FP64 distance of each sample point to its nearest centroid.
// grid (ceil(nt/256), 2*Ns).  Also counts the labels of each partial-sum
// block (a workgroup's positions lie in one block); integer adds in any
// order give the same counts.
template <int HX>
__global__ __launch_bounds__(256) void k_km_assign(KmArgs a, int HM, int nblk, const double *__restrict__ cent,
                                                   int32_t *__restrict__ lab, double *__restrict__ far,
                                                   uint32_t *__restrict__ pcnt) {
    __shared__ double C[64 * HX];  // row c: the centroid, zero-padded to HX
    __shared__ uint32_t hc[64];
    const int g = blockIdx.y;
    const Half H = half_of(g, a.s);
    for (int i = threadIdx.x; i < a.l * HX; i += 256) {
        const int c = i / HX, t = i % HX;
        C[i] = t < H.h ? cent[(static_cast<int64_t>(g) * a.l + c) * HM + t] : 0.0;
    }
    if (threadIdx.x < 64) hc[threadIdx.x] = 0;
    __syncthreads();
    const int64_t pb = static_cast<int64_t>(blockIdx.x) * KM_APW;
    const int64_t b = pb / KM_BLOCK;
    const int64_t p = pb + threadIdx.x;
    if (p < a.nt) {
        const float *x = a.T + row_of(a.train, p) * a.ld + H.off;
        double xv[HX];
#pragma unroll
        for (int t = 0; t < HX; t++) xv[t] = t < H.h ? static_cast<double>(x[t]) : 0.0;
        // Terms past h are (+0 - +0)^2 = +0, which leave the sum unchanged.
        int best = 0;
        double bd = 0.0;
        for (int c = 0; c < a.l; c++) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < HX; t++) {
                const double u = xv[t] - C[c * HX + t];
                s += u * u;
            }
            if (c == 0 || s < bd) {
                bd = s;
                best = c;
            }
        }
        lab[static_cast<int64_t>(g) * a.nt + p] = best;
        far[static_cast<int64_t>(g) * a.nt + p] = bd;
        atomicAdd(&hc[best], 1u);
    }
    __syncthreads();
    if (threadIdx.x < a.l && hc[threadIdx.x])
        atomicAdd(&pcnt[(static_cast<int64_t>(g) * nblk + b) * a.l + threadIdx.x], hc[threadIdx.x]);
}

constexpr int KM_PBLOCK = 1024;                  // threads of the partial-sum kernel
constexpr int KM_PW = KM_PBLOCK / WAVE;           // its waves
constexpr int KM_XVALS = 8192;                    // staged values per chunk
constexpr int KM_XPT = KM_XVALS / KM_PBLOCK;      // staged values per thread
constexpr int KM_PPT = 64 * KM_HMAX / KM_PBLOCK;  // (cluster, dim) pairs per thread

// psum[g][b][c][t]: sums of x_t over the points of block b labelled c, in
// ascending position order.  grid (nblk, 2*Ns).  The block streams through
// LDS in chunks of ch = min(1024, 8192/h) points, thread j holding point j of
// the chunk; the next chunk is loaded into registers while the current one
// is summed.  Per chunk, the points are listed cluster by cluster in position
// order (a stable counting sort: per-wave membership masks, prefix sums over
// waves and clusters), then each (cluster, dim) pair adds its own cluster's
// points in list order, i.e. in position order.
__global__ __launch_bounds__(KM_PBLOCK) void k_km_partial(KmArgs a, int HM, int nblk,
                                                          const int32_t *__restrict__ lab,
                                                          double *__restrict__ psum) {
    __shared__ float X[2][KM_XVALS];
    __shared__ unsigned long long wm[2][KM_PW][64];  // wm[.][w][c]: lanes of wave w labelled c
    __shared__ uint32_t wbase[KM_PW][64];            // points of cluster c in earlier waves
    __shared__ uint32_t cst[64], ctot[64];           // list start and size of cluster c
    __shared__ uint16_t list[KM_PBLOCK];
    const int g = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
    const int lane = tid % WAVE, w = tid / WAVE;
    const Half H = half_of(g, a.s);
    const int hh = H.h;
    const int ch = min(KM_PBLOCK, KM_XVALS / hh);
    const int64_t lo = static_cast<int64_t>(b) * KM_BLOCK;
    const int64_t hi = min(lo + KM_BLOCK, a.nt);
    const int nch = static_cast<int>((hi - lo + ch - 1) / ch);
    const int pairs = a.l * hh;
    const int32_t *lg = lab + static_cast<int64_t>(g) * a.nt;
    double acc[KM_PPT];
    int pc[KM_PPT], pt[KM_PPT];
#pragma unroll
    for (int u = 0; u < KM_PPT; u++) {
        const int idx = u * KM_PBLOCK + tid;
        pc[u] = idx < pairs ? idx / hh : -1;
        pt[u] = idx < pairs ? idx % hh : 0;
        acc[u] = 0.0;
    }
    int rl;
    float rv[KM_XPT];
    auto fetch = [&](int k) {
        const int64_t p0 = lo + static_cast<int64_t>(k) * ch;
        const int m = static_cast<int>(min<int64_t>(ch, hi - p0));
        rl = tid < m ? lg[p0 + tid] : -1;
#pragma unroll
        for (int u = 0; u < KM_XPT; u++) {
            const int i = u * KM_PBLOCK + tid;
            const int pi = i / hh, tt = i - pi * hh;
            rv[u] = pi < m ? a.T[row_of(a.train, p0 + pi) * a.ld + H.off + tt] : 0.0f;
        }
    };
    reinterpret_cast<unsigned long long *>(wm)[tid] = 0ull;
    reinterpret_cast<unsigned long long *>(wm)[KM_PBLOCK + tid] = 0ull;
    fetch(0);
    __syncthreads();
    for (int k = 0; k < nch; k++) {
        const int buf = k & 1;
        const int lb = rl;
#pragma unroll
        for (int u = 0; u < KM_XPT; u++) X[buf][u * KM_PBLOCK + tid] = rv[u];
        if (lb >= 0) atomicOr(&wm[buf][w][lb], 1ull << lane);
        __syncthreads();
        if (k + 1 < nch) fetch(k + 1);
        reinterpret_cast<unsigned long long *>(wm[buf ^ 1])[tid] = 0ull;  // for chunk k + 1
        if (w == 0) {
            uint32_t run = 0;
            if (lane < a.l) {
                for (int v = 0; v < KM_PW; v++) {
                    wbase[v][lane] = run;
                    run += static_cast<uint32_t>(__popcll(wm[buf][v][lane]));
                }
                ctot[lane] = run;
            }
            uint32_t incl = run;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o, WAVE);
                if (lane >= o) incl += y;
            }
            if (lane < a.l) cst[lane] = incl - run;
        }
        __syncthreads();
        if (lb >= 0) {
            const unsigned long long below = (1ull << lane) - 1ull;
            const uint32_t rank = static_cast<uint32_t>(__popcll(wm[buf][w][lb] & below));
            list[cst[lb] + wbase[w][lb] + rank] = static_cast<uint16_t>(tid);
        }
        __syncthreads();
        const float *xb = X[buf];
#pragma unroll
        for (int u = 0; u < KM_PPT; u++) {
            if (pc[u] < 0) continue;
            const int e0 = cst[pc[u]], e1 = e0 + ctot[pc[u]];
            const float *xt = xb + pt[u];
            double s = acc[u];
            for (int e = e0; e < e1; e++) s += static_cast<double>(xt[list[e] * hh]);
            acc[u] = s;
        }
    }
#pragma unroll
    for (int u = 0; u < KM_PPT; u++)
        if (pc[u] >= 0) psum[((static_cast<int64_t>(g) * nblk + b) * a.l + pc[u]) * HM + pt[u]] = acc[u];
}

constexpr int KM_UBLOCK = 1024;

// New centroids of half g: block sums added in block order, divided by the
// count; an empty cluster takes the sample point farthest from its own
// centroid (ties to the lower position) among those not yet taken this step.
// grid (2*Ns).
__global__ __launch_bounds__(KM_UBLOCK) void k_km_update(KmArgs a, int HM, int nblk,
                                                         const double *__restrict__ psum,
                                                         uint32_t *__restrict__ pcnt,
                                                         const double *__restrict__ far,
                                                         double *__restrict__ cent) {
    __shared__ int64_t cnt[64];
    __shared__ int64_t used[64];
    __shared__ double bf[KM_UBLOCK / WAVE];
    __shared__ int64_t bp[KM_UBLOCK / WAVE];
    const int g = blockIdx.x;
    const Half H = half_of(g, a.s);
    const int tid = threadIdx.x;
    for (int c = tid; c < a.l; c += KM_UBLOCK) {
        int64_t s = 0;
        for (int b = 0; b < nblk; b++) {
            uint32_t *pc = pcnt + (static_cast<int64_t>(g) * nblk + b) * a.l + c;
            s += *pc;
            *pc = 0u;  // the next assignment step counts afresh
        }
        cnt[c] = s;
    }
    __syncthreads();
    for (int i = tid; i < a.l * H.h; i += KM_UBLOCK) {
        const int c = i / H.h, t = i % H.h;
        if (cnt[c] == 0) continue;
        double s = 0.0;
        for (int b = 0; b < nblk; b++) s += psum[((static_cast<int64_t>(g) * nblk + b) * a.l + c) * HM + t];
        cent[(static_cast<int64_t>(g) * a.l + c) * HM + t] = s / static_cast<double>(cnt[c]);
    }
    int nused = 0;
    const double *fg = far + static_cast<int64_t>(g) * a.nt;
    for (int c = 0; c < a.l; c++) {
        if (cnt[c] != 0) continue;
        double best = -1.0;
        int64_t arg = -1;
        for (int64_t p = tid; p < a.nt; p += KM_UBLOCK) {
            const double v = fg[p];
            if (arg >= 0 && !(v > best)) continue;
            bool taken = false;
            for (int u = 0; u < nused; u++) taken |= used[u] == p;
            if (!taken) {
                best = v;
                arg = p;
            }
        }
        // workgroup arg-max, ties to the lower position
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, WAVE);
            const int64_t oa = __shfl_xor(arg, o, WAVE);
            if (oa >= 0 && (arg < 0 || ob > best || (ob == best && oa < arg))) {
                best = ob;
                arg = oa;
            }
        }
        __syncthreads();
        if ((tid % WAVE) == 0) {
            bf[tid / WAVE] = best;
            bp[tid / WAVE] = arg;
        }
        __syncthreads();
        best = -1.0;
        arg = -1;
        for (int w = 0; w < KM_UBLOCK / WAVE; w++) {
            const double ob = bf[w];
            const int64_t oa = bp[w];
            if (oa >= 0 && (arg < 0 || ob > best || (ob == best && oa < arg))) {
                best = ob;
                arg = oa;
            }
        }
        if (tid < H.h && arg >= 0)
            cent[(static_cast<int64_t>(g) * a.l + c) * HM + tid] =
                static_cast<double>(a.T[row_of(a.train, arg) * a.ld + H.off + tid]);
        if (tid == 0) used[nused] = arg;
        nused++;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_km_round(const double *__restrict__ cent, int64_t count,
                                                  float *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < count) out[i] = static_cast<float>(cent[i]);
}

// Final label of every row with the FP32 query-side chain.  grid
// (ceil(n/256), 2*Ns).
template <int HX>
__global__ __launch_bounds__(256) void k_km_label(KmArgs a, int HM, const float *__restrict__ cent,
                                                  int32_t *__restrict__ assign) {
    __shared__ float C[64 * HX];  // row c: the centroid, zero-padded to HX
    const int g = blockIdx.y;
    const Half H = half_of(g, a.s);
    for (int i = threadIdx.x; i < a.l * HX; i += 256) {
        const int c = i / HX, t = i % HX;
        C[i] = t < H.h ? cent[(static_cast<int64_t>(g) * a.l + c) * HM + t] : 0.0f;
    }
    __syncthreads();
    const int64_t r = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (r >= a.n) return;
    const float *x = a.T + r * a.ld + H.off;
    float xv[HX];
#pragma unroll
    for (int t = 0; t < HX; t++) xv[t] = t < H.h ? x[t] : 0.0f;
    int best = 0;
    float bd = 0.0f;
    // Terms past h are fmaf(+0, +0, acc) = acc.
    for (int c = 0; c < a.l; c++) {
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < HX; t++) {
            const float u = xv[t] - C[c * HX + t];
            acc = fmaf(u, u, acc);
        }
        if (c == 0 || acc < bd) {
            bd = acc;
            best = c;
        }
    }
    assign[static_cast<int64_t>(g) * a.n + r] = best;
}

// ---------------------------------------------------------------------------
// IMI: stable counting sort of the points by cell, per subspace.
// ---------------------------------------------------------------------------

constexpr int IMI_BLOCK = 256;

// Cell of point i in subspace j, or -1 for a label outside [0, l) (such a
// point is left out, so the offsets then end below n).
__device__ __forceinline__ int cell_of(const int32_t *assign, int64_t n, int j, int l, int64_t i) {
    const int a = assign[(2 * static_cast<int64_t>(j)) * n + i];
    const int b = assign[(2 * static_cast<int64_t>(j) + 1) * n + i];
    return (static_cast<unsigned>(a) < static_cast<unsigned>(l) && static_cast<unsigned>(b) < static_cast<unsigned>(l))
               ? a * l + b
               : -1;
}

// tcnt[j][tile][cell] = points of the tile in the cell.  grid (ntile, Ns).
__global__ __launch_bounds__(IMI_BLOCK) void k_imi_count(const int32_t *__restrict__ assign, int64_t n,
                                                         int l, int ntile, uint32_t *__restrict__ tcnt) {
    __shared__ uint32_t cnt[IMI_KMAX];
    const int j = blockIdx.y, K = l * l;
    for (int c = threadIdx.x; c < K; c += IMI_BLOCK) cnt[c] = 0;
    __syncthreads();
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * IMI_TILE;
    const int64_t hi = min(lo + IMI_TILE, n);
    for (int64_t i = lo + threadIdx.x; i < hi; i += IMI_BLOCK) {
        const int c = cell_of(assign, n, j, l, i);
        if (c >= 0) atomicAdd(&cnt[c], 1u);
    }
    __syncthreads();
    uint32_t *o = tcnt + (static_cast<int64_t>(j) * ntile + blockIdx.x) * K;
    for (int c = threadIdx.x; c < K; c += IMI_BLOCK) o[c] = cnt[c];
}

// Tile counts -> exclusive prefix over tiles (in place); tot[j][cell].
// grid (ceil(K/256), Ns).
__global__ __launch_bounds__(IMI_BLOCK) void k_imi_tiles(uint32_t *__restrict__ tcnt, int ntile, int K,
                                                         uint32_t *__restrict__ tot) {
    const int j = blockIdx.y;
    const int c = blockIdx.x * IMI_BLOCK + threadIdx.x;
    if (c >= K) return;
    uint32_t run = 0;
    for (int t = 0; t < ntile; t++) {
        uint32_t *p = tcnt + (static_cast<int64_t>(j) * ntile + t) * K + c;
        const uint32_t v = *p;
        *p = run;
        run += v;
    }
    tot[static_cast<int64_t>(j) * K + c] = run;
}

// offsets[j][c] = exclusive prefix of tot[j][:]; offsets[j][K] = n.  grid Ns,
// one thread per 4 cells.
__global__ __launch_bounds__(1024) void k_imi_offsets(const uint32_t *__restrict__ tot, int K,
                                                      uint32_t *__restrict__ offsets) {
    __shared__ uint32_t part[1024];
    const int j = blockIdx.x, tid = threadIdx.x;
    const uint32_t *tj = tot + static_cast<int64_t>(j) * K;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int c = tid * 4 + u;
        v[u] = c < K ? tj[c] : 0u;
        s += v[u];
    }
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t add = tid >= o ? part[tid - o] : 0u;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    uint32_t run = part[tid] - s;
    uint32_t *oj = offsets + static_cast<int64_t>(j) * (K + 1);
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int c = tid * 4 + u;
        if (c < K) oj[c] = run;
        run += v[u];
    }
    if (tid == 1023) oj[K] = part[1023];
}

// Points of each tile in index order; a point's slot is its cell's offset,
// plus the tile's base in the cell, plus the earlier points of the tile in
// the same cell.  grid (ntile, Ns).
__global__ __launch_bounds__(IMI_BLOCK) void k_imi_scatter(const int32_t *__restrict__ assign, int64_t n,
                                                           int l, int ntile,
                                                           const uint32_t *__restrict__ tcnt,
                                                           const uint32_t *__restrict__ offsets,
                                                           uint32_t *__restrict__ ids) {
    __shared__ uint32_t seen[IMI_KMAX];
    __shared__ int key[IMI_BLOCK];
    const int j = blockIdx.y, K = l * l, tid = threadIdx.x;
    for (int c = tid; c < K; c += IMI_BLOCK) seen[c] = 0;
    const uint32_t *tb = tcnt + (static_cast<int64_t>(j) * ntile + blockIdx.x) * K;
    const uint32_t *oj = offsets + static_cast<int64_t>(j) * (K + 1);
    uint32_t *idj = ids + static_cast<int64_t>(j) * n;
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * IMI_TILE;
    const int64_t hi = min(lo + IMI_TILE, n);
    for (int64_t r0 = lo; r0 < hi; r0 += IMI_BLOCK) {
        const int64_t i = r0 + tid;
        const int k = i < hi ? cell_of(assign, n, j, l, i) : -1;
        __syncthreads();
        key[tid] = k;
        __syncthreads();
        if (k >= 0) {
            uint32_t rank = 0;
            for (int u = 0; u < tid; u++) rank += key[u] == k;
            idj[oj[k] + tb[k] + seen[k] + rank] = static_cast<uint32_t>(i);
        }
        __syncthreads();
        if (k >= 0) atomicAdd(&seen[k], 1u);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------

namespace {
// Row chunks of the covariance: about 4096 workgroups in all, at most 256.
int cov_chunks(int64_t n, int ntile) {
    const int64_t want = std::max<int64_t>(1, std::min<int64_t>(CV_CHUNKS, 4096 / ntile));
    const int64_t rows = std::max<int64_t>(chunk_rows(n, static_cast<int>(want)), 1);
    return static_cast<int>((n + rows - 1) / rows);
}
}  // namespace

size_t stats_scratch(int64_t n, int d) {
    const int nb = (d + CV_TILE - 1) / CV_TILE;
    const int ntile = nb * (nb + 1) / 2;
    return std::max(size_t(ST_CHUNKS) * d, size_t(cov_chunks(n, ntile)) * ntile * CV_TILE * CV_TILE);
}

hipError_t launch_stats(const float *X, int64_t n, int d, double *mean, double *cov, double *scratch,
                        hipStream_t st) {
    const int64_t rows = chunk_rows(n, ST_CHUNKS);
    const int chunks = static_cast<int>((n + rows - 1) / rows);
    k_colsum<<<chunks, 256, 0, st>>>(X, n, d, rows, scratch);
    k_mean<<<(d + 255) / 256, 256, 0, st>>>(scratch, chunks, n, d, mean);
    const int nb = (d + CV_TILE - 1) / CV_TILE;
    const int ntile = nb * (nb + 1) / 2;
    const int cchunks = cov_chunks(n, ntile);
    const int64_t crow = std::max<int64_t>(chunk_rows(n, cchunks), 1);
    k_cov_part<<<dim3(ntile, cchunks), 256, 0, st>>>(X, n, d, mean, crow, nb, scratch);
    const int64_t dd = int64_t(d) * d;
    k_cov_final<<<static_cast<unsigned>((dd + 255) / 256), 256, 0, st>>>(scratch, cchunks, ntile, nb, n, d, cov);
    return hipGetLastError();
}

size_t eigen_scratch(int d) {
    const int dp = d + (d & 1);
    if (dp <= EIG_ONE_WG) return size_t(dp) * dp;
    // U, V, lambda, signs, ranks and the rotation counter
    return 2 * size_t(dp) * dp + 3 * size_t(d) + 2;
}

namespace {
hipError_t eigen_one_sided(const double *cov, int d, double *evals, double *evecs, double *scratch,
                           hipStream_t st) {
    const int dp = d + (d & 1);
    double *U = scratch, *V = U + size_t(dp) * dp;
    double *lam = V + size_t(dp) * dp, *sgn = lam + d;
    int *rank = reinterpret_cast<int *>(sgn + d);
    uint32_t *rot = reinterpret_cast<uint32_t *>(lam + 3 * size_t(d) + 1);
    const int64_t e2 = int64_t(dp) * dp;
    k_osj_init<<<static_cast<unsigned>((e2 + 255) / 256), 256, 0, st>>>(cov, d, dp, U, V);
    for (int sweep = 0; sweep < OSJ_SWEEPS; sweep++) {
        k_zero_u32<<<1, 1, 0, st>>>(rot);
        hipError_t e;
        for (int step = 0; step < dp - 1; step++) k_osj_step<<<dp / 2, OSJ_BLOCK, 0, st>>>(U, V, dp, step, rot);
        uint32_t h = 0;
        if ((e = hipMemcpyAsync(&h, rot, sizeof h, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        if (h == 0) break;
    }
    k_osj_values<<<d, OSJ_BLOCK, 0, st>>>(U, V, dp, lam);
    k_osj_order<<<(d + 255) / 256, 256, 0, st>>>(lam, V, d, dp, evals, rank, sgn);
    const int64_t dd = int64_t(d) * d;
    k_osj_vectors<<<static_cast<unsigned>((dd + 255) / 256), 256, 0, st>>>(V, d, dp, rank, sgn, evecs);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_eigen(const double *cov, int d, double *evals, double *evecs, double *scratch,
                        hipStream_t st) {
    const int dp = d + (d & 1);
    if (d < 1 || d > EIG_MAX_ONE_SIDED) return hipErrorInvalidValue;
    if (dp > EIG_ONE_WG) return eigen_one_sided(cov, d, evals, evecs, scratch, st);
    static_assert(EIG_ONE_WG <= EIG_MAX, "the one-workgroup form holds at most EIG_MAX");
    const size_t lds = sizeof(double) * size_t(dp) * dp;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_jacobi),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    k_jacobi<<<1, EIG_BLOCK, lds, st>>>(cov, d, dp, evals, evecs, scratch);
    return hipGetLastError();
}

namespace {
int km_hm(const KmArgs &a) { return a.s - a.s / 2; }
int64_t km_nblk(const KmArgs &a) { return (a.nt + KM_BLOCK - 1) / KM_BLOCK; }
}  // namespace

size_t km_scratch_bytes(const KmArgs &a) {
    const int64_t G = 2 * int64_t(a.Ns), HM = km_hm(a), nb = km_nblk(a);
    size_t b = 0;
    b += sizeof(double) * size_t(G * a.l * HM);   // FP64 centroids
    b += sizeof(int32_t) * size_t(G * a.nt);      // labels
    b += sizeof(double) * size_t(G * a.nt);       // distances
    b += sizeof(double) * size_t(G * nb * a.l * HM);
    b += sizeof(uint32_t) * size_t(G * nb * a.l);
    return b + 5 * 256;
}

hipError_t launch_kmeans(const KmArgs &a, float *cent, int32_t *assign, void *scratch, hipStream_t st) {
    const int G = 2 * a.Ns, HM = km_hm(a);
    const int64_t nb = km_nblk(a);
    if (HM > KM_HMAX || a.l < 1 || a.l > 64 || a.nt < a.l) return hipErrorInvalidValue;
    auto carve = [](unsigned char *&p, size_t bytes) {
        unsigned char *r = p;
        p += (bytes + 255) / 256 * 256;
        return r;
    };
    unsigned char *p = static_cast<unsigned char *>(scratch);
    double *c64 = reinterpret_cast<double *>(carve(p, sizeof(double) * size_t(G) * a.l * HM));
    int32_t *lab = reinterpret_cast<int32_t *>(carve(p, sizeof(int32_t) * size_t(G * a.nt)));
    double *far = reinterpret_cast<double *>(carve(p, sizeof(double) * size_t(G * a.nt)));
    double *psum = reinterpret_cast<double *>(carve(p, sizeof(double) * size_t(G * nb * a.l * HM)));
    uint32_t *pcnt = reinterpret_cast<uint32_t *>(carve(p, sizeof(uint32_t) * size_t(G * nb * a.l)));
    const int nbi = static_cast<int>(nb);
    k_km_seed<<<G, 256, 0, st>>>(a, HM, nbi, c64, pcnt);
    const dim3 ga(static_cast<unsigned>((a.nt + KM_APW - 1) / KM_APW), G);
    for (int it = 0; it < a.iters; it++) {
        if (HM <= 8)
            k_km_assign<8><<<ga, 256, 0, st>>>(a, HM, nbi, c64, lab, far, pcnt);
        else if (HM <= 16)
            k_km_assign<16><<<ga, 256, 0, st>>>(a, HM, nbi, c64, lab, far, pcnt);
        else
            k_km_assign<32><<<ga, 256, 0, st>>>(a, HM, nbi, c64, lab, far, pcnt);
        k_km_partial<<<dim3(static_cast<unsigned>(nb), G), KM_PBLOCK, 0, st>>>(a, HM, nbi, lab, psum);
        k_km_update<<<G, KM_UBLOCK, 0, st>>>(a, HM, static_cast<int>(nb), psum, pcnt, far, c64);
    }
    const int64_t cc = int64_t(G) * a.l * HM;
    k_km_round<<<static_cast<unsigned>((cc + 255) / 256), 256, 0, st>>>(c64, cc, cent);
    const dim3 gl(static_cast<unsigned>((a.n + 255) / 256), G);
    if (HM <= 8)
        k_km_label<8><<<gl, 256, 0, st>>>(a, HM, cent, assign);
    else if (HM <= 16)
        k_km_label<16><<<gl, 256, 0, st>>>(a, HM, cent, assign);
    else
        k_km_label<32><<<gl, 256, 0, st>>>(a, HM, cent, assign);
    return hipGetLastError();
}

size_t imi_scratch_words(int64_t n, int Ns, int l) {
    const int64_t ntile = (n + IMI_TILE - 1) / IMI_TILE, K = int64_t(l) * l;
    return size_t(Ns) * size_t(ntile * K + K);
}

hipError_t launch_imi(const int32_t *assign, int64_t n, int Ns, int l, uint32_t *offsets, uint32_t *ids,
                      uint32_t *scratch, hipStream_t st) {
    const int K = l * l;
    if (K > IMI_KMAX || n <= 0) return hipErrorInvalidValue;
    const int ntile = static_cast<int>((n + IMI_TILE - 1) / IMI_TILE);
    uint32_t *tcnt = scratch;
    uint32_t *tot = scratch + size_t(Ns) * ntile * K;
    k_imi_count<<<dim3(ntile, Ns), IMI_BLOCK, 0, st>>>(assign, n, l, ntile, tcnt);
    k_imi_tiles<<<dim3((K + IMI_BLOCK - 1) / IMI_BLOCK, Ns), IMI_BLOCK, 0, st>>>(tcnt, ntile, K, tot);
    k_imi_offsets<<<Ns, 1024, 0, st>>>(tot, K, offsets);
    k_imi_scatter<<<dim3(ntile, Ns), IMI_BLOCK, 0, st>>>(assign, n, l, ntile, tcnt, offsets, ids);
    return hipGetLastError();
}

}  // namespace bld
}  // namespace taco

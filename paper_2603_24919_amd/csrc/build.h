// Index construction on the GPU (Alg 1 and Alg 3 of the paper; Alg 2 is
// host code in runtime.cpp).  Launchers enqueue on the given stream and
// return the first HIP error; buffers are owned by the caller.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace taco {
namespace bld {

// ---- Alg 1: mean and covariance in FP64 ----------------------------------
// Doubles of scratch launch_stats needs for an n x d input.
size_t stats_scratch(int64_t n, int d);
// mean[d] = column means; cov[d][d] = 1/(n-1) sum (x - mean)(x - mean)^T.
// Fixed reduction order (chunk partials summed in chunk order): the result
// does not depend on the launch.  n >= 2.
hipError_t launch_stats(const float *X, int64_t n, int d, double *mean, double *cov,
                        double *scratch, hipStream_t st);

// ---- Alg 1: spectral decomposition (cyclic Jacobi, one workgroup) --------
constexpr int EIG_MAX = 128;             // largest d the one-workgroup form can hold (matrix in LDS)
constexpr int EIG_ONE_WG = 32;           // d up to which that form is used (faster only for small d)
constexpr int EIG_MAX_ONE_SIDED = 4096;  // largest d of the one-sided form
// Doubles of scratch launch_eigen needs (the accumulated rotations).
size_t eigen_scratch(int d);
// evals[d] descending; evecs[r][c] = component r of eigenvector c, each
// vector's largest-magnitude component (the first on ties) positive.  For
// d > EIG_ONE_WG the one-sided form synchronizes the stream once per sweep
// (the host reads its rotation counter), so it cannot be captured in a graph.
hipError_t launch_eigen(const double *cov, int d, double *evals, double *evecs,
                        double *scratch, hipStream_t st);

// ---- Alg 3: k-means on every half-subspace at once -----------------------
// Half g = 2*j + hf (subspace j, half hf) covers columns
// [j*s + hf*(s/2), ... + h) of T (n x ld, row-major), h = s/2 or s - s/2.
struct KmArgs {
    const float *T = nullptr;
    int64_t n = 0;  // rows of T (the final assignment covers them all)
    int ld = 0;
    int Ns = 0, s = 0, l = 0, iters = 0;
    const int64_t *init = nullptr;   // [2*Ns][l] Forgy seeds, positions into the sample
    const int64_t *train = nullptr;  // [nt] training rows, ascending, or null (all rows)
    int64_t nt = 0;                  // training sample size
};
constexpr int KM_HMAX = 32;       // largest half width
constexpr int KM_BLOCK = 65536;   // points per partial-sum block
size_t km_scratch_bytes(const KmArgs &a);
// cent[2*Ns][l][s - s/2] FP32 centroids (rows of width s - s/2; the first
// h entries used), assign[2*Ns][n] final labels.
hipError_t launch_kmeans(const KmArgs &a, float *cent, int32_t *assign, void *scratch,
                         hipStream_t st);

// ---- Alg 3: IMI as CSR, by a stable counting sort on the cell -----------
constexpr int IMI_TILE = 4096;
constexpr int IMI_KMAX = 4096;
size_t imi_scratch_words(int64_t n, int Ns, int l);
// offsets[Ns][l*l + 1], ids[Ns][n]; cell = assign[2j][i]*l + assign[2j+1][i],
// ids ascending inside each cell.
hipError_t launch_imi(const int32_t *assign, int64_t n, int Ns, int l, uint32_t *offsets,
                      uint32_t *ids, uint32_t *scratch, hipStream_t st);

}  // namespace bld
}  // namespace taco

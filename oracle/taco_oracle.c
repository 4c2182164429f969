/*
 * taco_oracle.c -- plain CPU oracle for the query stage of TaCo
 * (data-adaptive, query-aware subspace-collision ANN search).
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines the expected results that the
 * GPU path is checked against; it is used by the tests, the smoke check and
 * the CPU-baseline leg of the benchmark, never by the product.  It shares no
 * code, header, table or helper with the GPU library: the two meet only in the
 * serialized index file, which each side reads and writes with its own code.
 *
 * Everything here is written for clarity, not speed: scalar loops, full
 * sorts (Scalable Dynamic Activation is written as the cell order it
 * produces, all cells sorted by key).  OpenMP is used
 * only across independent points or queries, and every reduction is done in a
 * fixed order, so results do not depend on the thread count.
 *
 * Precision.  The paper fixes none.  Values that decide an integer result
 * (which cells are probed, hence every collision count and candidate) are
 * computed in FP32 with one canonical evaluation order, the same order the GPU
 * kernels use, so both sides take the same integer decisions:
 *   query transform   q'_m = acc <- fmaf(B[t][m], fl32(q_t - mean_t), acc), t ascending
 *   half distance     D[c] = acc <- fmaf(u, u, acc), u = fl32(q'_x - C[c][x]), x ascending
 *   cell key          fl32(D1[idx1[r]] + D2[idx2[c]])
 * Re-rank distances are given both in that FP32 chain (dist32, which orders
 * the oracle's top-k) and in FP64 (dist64, for error reports and recall).
 * Index-build statistics (mean, covariance, k-means training) are FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EIO -2
#define ORC_EFORMAT -3
#define ORC_ENOMEM -4

/* Candidates-selection readings (Alg 5, see orc_select), and the
 * fixed-budget rule of SuCo that the paper compares Alg 5 against. */
#define ORC_RULE_PRINTED 0
#define ORC_RULE_PROSE 1
#define ORC_RULE_FIXED 2

/* Fixed reduction block: partial sums are formed per block of this many
 * points and then added in block order, independent of the thread count. */
#define ORC_BLOCK 65536

/* ------------------------------------------------------------------------- */
/* Alg 1, step "transform": r = B^T (o - mean), concatenated over subspaces.   */
/* ------------------------------------------------------------------------- */

/* T[i][m] = sum_t B[t][m] * fl32(X[i][t] - mean[t]) in the canonical FP32
 * chain (t ascending, one fused multiply-add per term).  B is d x M row-major
 * (column m is the m-th allocated eigenvector), T is n x M. */
void orc_transform(const float *X, int64_t n, int d, const float *mean,
                   const float *B, int M, float *T)
{
#pragma omp parallel
    {
        float *e = (float *)malloc(sizeof(float) * (size_t)d);
        float *acc = (float *)malloc(sizeof(float) * (size_t)M);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            const float *x = X + i * d;
            for (int t = 0; t < d; t++) e[t] = x[t] - mean[t];
            for (int m = 0; m < M; m++) acc[m] = 0.0f;
            for (int t = 0; t < d; t++) {
                const float *brow = B + (size_t)t * M;
                const float et = e[t];
                for (int m = 0; m < M; m++) acc[m] = fmaf(brow[m], et, acc[m]);
            }
            memcpy(T + i * M, acc, sizeof(float) * (size_t)M);
        }
        free(e);
        free(acc);
    }
}

/* Squared L2 distance of an h-dim half-vector to each of l centroids, in the
 * canonical FP32 chain.  C is l x h row-major. */
void orc_half_dists(const float *x, const float *C, int l, int h, float *D)
{
    for (int c = 0; c < l; c++) {
        float acc = 0.0f;
        for (int t = 0; t < h; t++) {
            float u = x[t] - C[c * h + t];
            acc = fmaf(u, u, acc);
        }
        D[c] = acc;
    }
}

/* ------------------------------------------------------------------------- */
/* Alg 3 inner step: k-means on one half-subspace (Lloyd iterations).          */
/* ------------------------------------------------------------------------- */

/* Distance of point row p (h floats) to a FP64 centroid, in FP64. */
static double d64_to(const float *p, const double *c, int h)
{
    double s = 0.0;
    for (int t = 0; t < h; t++) {
        double u = (double)p[t] - c[t];
        s += u * u;
    }
    return s;
}

/*
 * k-means with l centroids on columns [off, off+h) of the n x ld matrix T.
 * Training points are the rows listed in train[0..n_train) (all rows when
 * train == NULL).  Centroids start at the training points init[0..l) (Forgy)
 * and take `iters` Lloyd steps in FP64: assign each training point to its
 * nearest centroid (ties -> lower centroid id), then move each centroid to
 * the mean of its points.  A centroid left without points is moved onto the
 * training point farthest from its own centroid (ties -> lower position),
 * each such point used once per step.  The centroids are then rounded to FP32
 * and every row of T (not only the training rows) gets one final assignment
 * with the canonical FP32 distance (ties -> lower id).
 */
int orc_kmeans(const float *T, int64_t n, int ld, int off, int h, int l, int iters,
               const int64_t *init, const int64_t *train, int64_t n_train,
               float *cent_out, int32_t *assign_out)
{
    if (n <= 0 || h <= 0 || l <= 0 || n_train < l) return ORC_EINVAL;
    int64_t nt = train ? n_train : n;
    double *cent = (double *)malloc(sizeof(double) * (size_t)l * h);
    int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)nt);
    double *far = (double *)malloc(sizeof(double) * (size_t)nt);
    int64_t nblk = (nt + ORC_BLOCK - 1) / ORC_BLOCK;
    double *psum = (double *)malloc(sizeof(double) * (size_t)nblk * l * h);
    int64_t *pcnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)nblk * l);
    double *sum = (double *)malloc(sizeof(double) * (size_t)l * h);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)l);
    char *used = (char *)malloc((size_t)nt);
    if (!cent || !lab || !far || !psum || !pcnt || !sum || !cnt || !used) {
        free(cent); free(lab); free(far); free(psum); free(pcnt); free(sum); free(cnt); free(used);
        return ORC_ENOMEM;
    }
#define ROW(p) (T + (train ? train[(p)] : (p)) * (int64_t)ld + off)
    for (int c = 0; c < l; c++)
        for (int t = 0; t < h; t++) cent[c * h + t] = (double)ROW(init[c])[t];

    for (int it = 0; it < iters; it++) {
        /* assignment */
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < nt; p++) {
            const float *x = ROW(p);
            int best = 0;
            double bd = d64_to(x, cent, h);
            for (int c = 1; c < l; c++) {
                double dd = d64_to(x, cent + c * h, h);
                if (dd < bd) { bd = dd; best = c; }
            }
            lab[p] = best;
            far[p] = bd;
        }
        /* update: per-block partial sums, then added in block order */
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < nblk; b++) {
            double *ps = psum + b * l * h;
            int64_t *pc = pcnt + b * l;
            memset(ps, 0, sizeof(double) * (size_t)l * h);
            memset(pc, 0, sizeof(int64_t) * (size_t)l);
            int64_t lo = b * ORC_BLOCK, hi = lo + ORC_BLOCK < nt ? lo + ORC_BLOCK : nt;
            for (int64_t p = lo; p < hi; p++) {
                const float *x = ROW(p);
                int c = lab[p];
                pc[c]++;
                for (int t = 0; t < h; t++) ps[c * h + t] += (double)x[t];
            }
        }
        memset(sum, 0, sizeof(double) * (size_t)l * h);
        memset(cnt, 0, sizeof(int64_t) * (size_t)l);
        for (int64_t b = 0; b < nblk; b++)
            for (int c = 0; c < l; c++) {
                cnt[c] += pcnt[b * l + c];
                for (int t = 0; t < h; t++) sum[c * h + t] += psum[(b * l + c) * h + t];
            }
        memset(used, 0, (size_t)nt);
        for (int c = 0; c < l; c++) {
            if (cnt[c] > 0) {
                for (int t = 0; t < h; t++) cent[c * h + t] = sum[c * h + t] / (double)cnt[c];
            } else {
                int64_t arg = -1;
                for (int64_t p = 0; p < nt; p++)
                    if (!used[p] && (arg < 0 || far[p] > far[arg])) arg = p;
                used[arg] = 1;
                for (int t = 0; t < h; t++) cent[c * h + t] = (double)ROW(arg)[t];
            }
        }
    }
#undef ROW
    for (int c = 0; c < l * h; c++) cent_out[c] = (float)cent[c];
    /* final assignment of every row with the canonical FP32 distance */
#pragma omp parallel
    {
        float *D = (float *)malloc(sizeof(float) * (size_t)l);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            orc_half_dists(T + i * (int64_t)ld + off, cent_out, l, h, D);
            int best = 0;
            for (int c = 1; c < l; c++)
                if (D[c] < D[best]) best = c;
            assign_out[i] = best;
        }
        free(D);
    }
    free(cent); free(lab); free(far); free(psum); free(pcnt); free(sum); free(cnt); free(used);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Index file: written by the oracle's build, read by the oracle's query and   */
/* (with its own reader) by the GPU library.  Little-endian layout:            */
/*   header, 128 bytes: magic "TACOIDX1", u32 version=1, u32 header_bytes=128, */
/*     i64 n, i32 d, Ns, s, h1, h2, l, u64 seed, u64 flags, zero padding       */
/*   f32 mean[d]; f32 B[d][Ns*s]; f32 C1[Ns][l][h1]; f32 C2[Ns][l][h2];        */
/*   u64 offsets[Ns][l*l+1]  (cell a*l+b: a = half-1 centroid, b = half-2);    */
/*   u32 ids[Ns][n]          (ascending inside each cell);                     */
/*   f32 base[n][d];                                                           */
/*   u64 checksum = FNV-1a 64 over every preceding byte.                       */
/* ------------------------------------------------------------------------- */

#define ORC_MAGIC "TACOIDX1"
#define ORC_VERSION 1u
#define ORC_HDR 128

typedef struct {
    int64_t n;
    int32_t d, Ns, s, h1, h2, l, M, K;
    uint64_t seed, flags;
    float *mean, *B, *C1, *C2, *base;
    uint64_t *offsets;
    uint32_t *ids;
} orc_index;

/* FNV-1a, 64-bit: offset basis 14695981039346656037, prime 1099511628211. */
static uint64_t fnv1a(uint64_t hsh, const void *p, size_t nb)
{
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < nb; i++) {
        hsh ^= c[i];
        hsh *= 1099511628211ULL;
    }
    return hsh;
}

static int put(FILE *f, uint64_t *hsh, const void *p, size_t nb)
{
    *hsh = fnv1a(*hsh, p, nb);
    return fwrite(p, 1, nb, f) == nb ? 0 : -1;
}

int orc_write_index(const char *path, int64_t n, int d, int Ns, int s, int l, uint64_t seed,
                    const float *mean, const float *B, const float *C1, const float *C2,
                    const uint64_t *offsets, const uint32_t *ids, const float *base)
{
    if (n <= 0 || d <= 0 || Ns <= 0 || s < 2 || l <= 0 || (int64_t)Ns * s > d) return ORC_EINVAL;
    FILE *f = fopen(path, "wb");
    if (!f) return ORC_EIO;
    int32_t h1 = s / 2, h2 = s - s / 2, M = Ns * s;
    int64_t K = (int64_t)l * l;
    unsigned char hdr[ORC_HDR];
    memset(hdr, 0, sizeof hdr);
    uint32_t ver = ORC_VERSION, hb = ORC_HDR;
    uint64_t flags = 0;
    int32_t dims[6] = {d, Ns, s, h1, h2, l};
    memcpy(hdr, ORC_MAGIC, 8);
    memcpy(hdr + 8, &ver, 4);
    memcpy(hdr + 12, &hb, 4);
    memcpy(hdr + 16, &n, 8);
    memcpy(hdr + 24, dims, 24);
    memcpy(hdr + 48, &seed, 8);
    memcpy(hdr + 56, &flags, 8);
    uint64_t hsh = 14695981039346656037ULL;
    int bad = 0;
    bad |= put(f, &hsh, hdr, ORC_HDR);
    bad |= put(f, &hsh, mean, sizeof(float) * (size_t)d);
    bad |= put(f, &hsh, B, sizeof(float) * (size_t)d * M);
    bad |= put(f, &hsh, C1, sizeof(float) * (size_t)Ns * l * h1);
    bad |= put(f, &hsh, C2, sizeof(float) * (size_t)Ns * l * h2);
    bad |= put(f, &hsh, offsets, sizeof(uint64_t) * (size_t)Ns * (K + 1));
    bad |= put(f, &hsh, ids, sizeof(uint32_t) * (size_t)Ns * n);
    bad |= put(f, &hsh, base, sizeof(float) * (size_t)n * d);
    bad |= fwrite(&hsh, 1, 8, f) == 8 ? 0 : -1;
    bad |= fclose(f);
    return bad ? ORC_EIO : ORC_OK;
}

static int get(FILE *f, uint64_t *hsh, void **dst, size_t nb)
{
    *dst = malloc(nb ? nb : 1);
    if (!*dst) return ORC_ENOMEM;
    if (fread(*dst, 1, nb, f) != nb) return ORC_EFORMAT;
    *hsh = fnv1a(*hsh, *dst, nb);
    return ORC_OK;
}

void orc_free_index(orc_index *x)
{
    if (!x) return;
    free(x->mean); free(x->B); free(x->C1); free(x->C2);
    free(x->offsets); free(x->ids); free(x->base);
    free(x);
}

int orc_load_index(const char *path, orc_index **out)
{
    *out = NULL;
    FILE *f = fopen(path, "rb");
    if (!f) return ORC_EIO;
    orc_index *x = (orc_index *)calloc(1, sizeof(orc_index));
    unsigned char hdr[ORC_HDR];
    uint64_t hsh = 14695981039346656037ULL, want = 0;
    int rc = ORC_EFORMAT;
    if (fread(hdr, 1, ORC_HDR, f) != ORC_HDR) goto fail;
    hsh = fnv1a(hsh, hdr, ORC_HDR);
    uint32_t ver, hb;
    int32_t dims[6];
    memcpy(&ver, hdr + 8, 4);
    memcpy(&hb, hdr + 12, 4);
    if (memcmp(hdr, ORC_MAGIC, 8) != 0 || ver != ORC_VERSION || hb != ORC_HDR) goto fail;
    memcpy(&x->n, hdr + 16, 8);
    memcpy(dims, hdr + 24, 24);
    memcpy(&x->seed, hdr + 48, 8);
    memcpy(&x->flags, hdr + 56, 8);
    x->d = dims[0]; x->Ns = dims[1]; x->s = dims[2]; x->h1 = dims[3]; x->h2 = dims[4]; x->l = dims[5];
    x->M = x->Ns * x->s;
    x->K = x->l * x->l;
    if (x->n <= 0 || x->d <= 0 || x->Ns <= 0 || x->s < 2 || x->l <= 0 || x->M > x->d ||
        x->h1 != x->s / 2 || x->h2 != x->s - x->s / 2)
        goto fail;
    if ((rc = get(f, &hsh, (void **)&x->mean, sizeof(float) * (size_t)x->d))) goto fail;
    if ((rc = get(f, &hsh, (void **)&x->B, sizeof(float) * (size_t)x->d * x->M))) goto fail;
    if ((rc = get(f, &hsh, (void **)&x->C1, sizeof(float) * (size_t)x->Ns * x->l * x->h1))) goto fail;
    if ((rc = get(f, &hsh, (void **)&x->C2, sizeof(float) * (size_t)x->Ns * x->l * x->h2))) goto fail;
    if ((rc = get(f, &hsh, (void **)&x->offsets, sizeof(uint64_t) * (size_t)x->Ns * (x->K + 1)))) goto fail;
    if ((rc = get(f, &hsh, (void **)&x->ids, sizeof(uint32_t) * (size_t)x->Ns * x->n))) goto fail;
    if ((rc = get(f, &hsh, (void **)&x->base, sizeof(float) * (size_t)x->n * x->d))) goto fail;
    rc = ORC_EFORMAT;
    if (fread(&want, 1, 8, f) != 8 || want != hsh) goto fail;
    fclose(f);
    *out = x;
    return ORC_OK;
fail:
    fclose(f);
    orc_free_index(x);
    return rc;
}

void orc_index_info(const orc_index *x, int64_t *n, int32_t *dims /* d,Ns,s,h1,h2,l */)
{
    *n = x->n;
    dims[0] = x->d; dims[1] = x->Ns; dims[2] = x->s; dims[3] = x->h1; dims[4] = x->h2; dims[5] = x->l;
}

/* Read-only views of the loaded arrays (for the tests' index invariants). */
const uint64_t *orc_index_offsets(const orc_index *x) { return x->offsets; }
const uint32_t *orc_index_ids(const orc_index *x) { return x->ids; }
const float *orc_index_centroids(const orc_index *x, int half) { return half ? x->C2 : x->C1; }
const float *orc_index_B(const orc_index *x) { return x->B; }
const float *orc_index_mean(const orc_index *x) { return x->mean; }
const float *orc_index_base(const orc_index *x) { return x->base; }

/* ------------------------------------------------------------------------- */
/* Alg 6 step "sorted indices": stable ascending argsort (ties -> lower id).   */
/* ------------------------------------------------------------------------- */
void orc_argsort(const float *D, int l, int32_t *idx)
{
    /* insertion sort: moves an element only past strictly larger keys */
    for (int c = 0; c < l; c++) {
        int p = c;
        while (p > 0 && D[idx[p - 1]] > D[c]) {
            idx[p] = idx[p - 1];
            p--;
        }
        idx[p] = c;
    }
}

/* ------------------------------------------------------------------------- */
/* Alg 4: Scalable Dynamic Activation, by the order it visits cells.           */
/* ------------------------------------------------------------------------- */

/*
 * What Alg 4 computes (Section 4.2).  Half 1's centroids in ascending
 * distance make the rows of an l x l grid, half 2's the columns; a cell's key
 * is the sum of its two half distances, fl32(D1[idx1[r]] + D2[idx2[c]]).
 * Each row is non-decreasing along its columns, row r only becomes active
 * after row r-1 has given up its first cell, and the active rows offer their
 * next cell through a min-priority queue of (key, row).  The cells therefore
 * come out in ascending key order, equal keys in ascending row and then
 * column rank (a row holds one queue entry at a time and hands out its
 * columns in order).  Retrieval stops at the first cell that brings the
 * retrieved total to at least A.  This function states exactly that: every
 * cell tagged with (key, row rank, column rank), the whole grid sorted, and
 * the sorted list cut after the first prefix whose sizes reach A (at least
 * one cell is always taken).  Writes the probed cell ids c = a*l + b in
 * retrieval order and returns the number of points retrieved.  A must not
 * exceed the total of size[].
 */
typedef struct {
    float key;
    int32_t r, c;
} kcell;

static int kcmp(const void *pa, const void *pb)
{
    const kcell *a = (const kcell *)pa, *b = (const kcell *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->r != b->r) return a->r < b->r ? -1 : 1;
    return (a->c > b->c) - (a->c < b->c);
}

int64_t orc_probe(const float *D1, const int32_t *idx1, const float *D2, const int32_t *idx2,
                  int l, const int64_t *size, int64_t A, int32_t *cells, int32_t *ncells)
{
    int K = l * l;
    kcell *all = (kcell *)malloc(sizeof(kcell) * (size_t)K);
    for (int r = 0; r < l; r++)
        for (int c = 0; c < l; c++) {
            all[r * l + c].key = D1[idx1[r]] + D2[idx2[c]];
            all[r * l + c].r = r;
            all[r * l + c].c = c;
        }
    qsort(all, (size_t)K, sizeof(kcell), kcmp);
    int64_t got = 0;
    int nc = 0;
    for (int i = 0; i < K; i++) {
        int32_t cell = idx1[all[i].r] * l + idx2[all[i].c];
        cells[nc++] = cell;
        got += size[cell];
        if (got >= A) break;
    }
    free(all);
    *ncells = nc;
    return got;
}

/* ------------------------------------------------------------------------- */
/* Alg 5: Query-aware Candidates Selection.                                    */
/* ------------------------------------------------------------------------- */

/*
 * Alg 5's threshold (Section 4.3) from the level histogram hist[0..Ns] and
 * the re-rank budget R = floor(beta*n).  Write S(v) for the number of points
 * whose SC-score is at least v.  Alg 5 walks the levels from Ns downwards
 * and stops at the first level where the budget is exceeded; the threshold
 * is that level, and -1 when no level exceeds it.  "Exceeded" at level v is
 *   ORC_RULE_PRINTED: hist[v] + S(v) > R  (the test as the algorithm prints
 *                     it: the level's count against beta*n minus a running
 *                     total that already includes it), or
 *   ORC_RULE_PROSE:   S(v) > R            (the text's reading: stop once the
 *                     accumulated candidates exceed beta*n).
 * So the threshold is the highest level that exceeds the budget.
 */
int orc_threshold(const int64_t *hist, int Ns, int64_t R, int rule)
{
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)(Ns + 2));
    S[Ns + 1] = 0;
    for (int v = Ns; v >= 0; v--) S[v] = S[v + 1] + hist[v];
    int top = -1;
    for (int v = 0; v <= Ns; v++) {
        int64_t load = rule == ORC_RULE_PROSE ? S[v] : hist[v] + S[v];
        if (load > R) top = v;
    }
    free(S);
    return top;
}

static int u64cmp(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* The fixed-budget rule (the candidate selection SuCo uses, which Section
 * 4.3 contrasts with Alg 5): the R points of highest SC-score, ties by lower
 * id -- the first min(R, n) of all points sorted by (SC descending, id
 * ascending).  Written as that sort.  cand: the chosen ids ascending;
 * last_out: L + 1, where L, the boundary level, is the SC-score of the last
 * point chosen (Ns + 1 when R = 0).  The chosen points are every point with
 * SC > L and the first R - #{SC > L} points of level L in id order, so
 * level L itself may be taken whole or in part.  Returns the number chosen. */
static int64_t select_fixed(const uint8_t *SC, int64_t n, int Ns, int64_t R, int32_t *last_out,
                            int32_t *cand)
{
    int64_t take = R < n ? R : n;
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    if (!key) return -1;
    for (int64_t i = 0; i < n; i++) key[i] = ((uint64_t)(255 - SC[i]) << 32) | (uint64_t)i;
    qsort(key, (size_t)n, sizeof(uint64_t), u64cmp);
    *last_out = take > 0 ? (int32_t)SC[key[take - 1] & 0xffffffffu] + 1 : Ns + 1;
    for (int64_t j = 0; j < take; j++) key[j] &= 0xffffffffu;
    qsort(key, (size_t)take, sizeof(uint64_t), u64cmp);
    for (int64_t j = 0; j < take; j++) cand[j] = (int32_t)key[j];
    free(key);
    return take;
}

/* Level histogram of SC[0..n), threshold, and the candidates
 * C = { i : SC[i] >= last } in ascending i (for ORC_RULE_FIXED see
 * select_fixed).  Returns |C|, or -1 if memory runs out. */
int64_t orc_select(const uint8_t *SC, int64_t n, int Ns, int64_t R, int rule,
                   int64_t *hist, int32_t *last_out, int32_t *cand)
{
    for (int v = 0; v <= Ns; v++) hist[v] = 0;
    for (int64_t i = 0; i < n; i++) hist[SC[i]]++;
    if (rule == ORC_RULE_FIXED) return select_fixed(SC, n, Ns, R, last_out, cand);
    int last = orc_threshold(hist, Ns, R, rule);
    int64_t nc = 0;
    for (int64_t i = 0; i < n; i++)
        if ((int)SC[i] >= last) cand[nc++] = (int32_t)i;
    *last_out = last;
    return nc;
}

/* ------------------------------------------------------------------------- */
/* Alg 6: k-ANNS query.                                                        */
/* ------------------------------------------------------------------------- */

/* Squared L2 distance of the query to base row i: FP32 canonical chain and
 * FP64. */
static void row_dist(const float *q, const float *x, int d, float *d32, double *d64)
{
    float a = 0.0f;
    double b = 0.0;
    for (int t = 0; t < d; t++) {
        float u = q[t] - x[t];
        a = fmaf(u, u, a);
        double v = (double)q[t] - (double)x[t];
        b += v * v;
    }
    *d32 = a;
    *d64 = b;
}

typedef struct {
    float key;
    int32_t id;
    double d64;
} rres;

static int rcmp(const void *pa, const void *pb)
{
    const rres *a = (const rres *)pa, *b = (const rres *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* Per-stage outputs of one query; any pointer may be NULL. */
typedef struct {
    float *qt;            /* [M]          transformed query                    */
    float *cdist;         /* [Ns][2][l]   half-centroid distances              */
    int32_t *corder;      /* [Ns][2][l]   ascending order of each half         */
    int32_t *cells;       /* [Ns][K]      probed cells, retrieval order        */
    int32_t *ncells;      /* [Ns]         number of probed cells               */
    int64_t *retrieved;   /* [Ns]         points retrieved per subspace        */
    uint8_t *sc;          /* [n]          SC-scores                            */
    int64_t *hist;        /* [Ns+1]       level histogram                      */
    int32_t *last;        /* [1]          last_collision                       */
    int32_t *cand;        /* [n]          candidates, ascending id             */
    int64_t *ncand;       /* [1]          |C|                                  */
    float *cand_d32;      /* [n]          candidate distances, FP32 chain      */
    double *cand_d64;     /* [n]          candidate distances, FP64            */
} orc_dump;

typedef struct {
    float *qt, *D, *q;
    int32_t *order, *cells;
    int64_t *size;
    uint8_t *sc;
    int32_t *cand;
    rres *res;
} orc_work;

static int work_init(const orc_index *x, orc_work *w)
{
    memset(w, 0, sizeof *w);
    w->qt = (float *)malloc(sizeof(float) * (size_t)x->M);
    w->D = (float *)malloc(sizeof(float) * 2 * (size_t)x->l);
    w->order = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)x->l);
    w->cells = (int32_t *)malloc(sizeof(int32_t) * (size_t)x->K);
    w->size = (int64_t *)malloc(sizeof(int64_t) * (size_t)x->K);
    w->sc = (uint8_t *)malloc((size_t)x->n);
    w->cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)x->n);
    w->res = (rres *)malloc(sizeof(rres) * (size_t)x->n);
    return (w->qt && w->D && w->order && w->cells && w->size && w->sc && w->cand && w->res)
               ? ORC_OK : ORC_ENOMEM;
}

static void work_free(orc_work *w)
{
    free(w->qt); free(w->D); free(w->order); free(w->cells); free(w->size);
    free(w->sc); free(w->cand); free(w->res);
}

/* Budgets in IEEE double, as the library computes them:
 * A = ceil(alpha*n) clamped to [1, n], R = floor(beta*n) clamped to [0, n]. */
static int64_t budget_A(double alpha, int64_t n)
{
    double a = ceil(alpha * (double)n);
    if (a < 1.0) a = 1.0;
    if (a > (double)n) a = (double)n;
    return (int64_t)a;
}

static int64_t budget_R(double beta, int64_t n)
{
    double r = floor(beta * (double)n);
    if (r < 0.0) r = 0.0;
    if (r > (double)n) r = (double)n;
    return (int64_t)r;
}

static int query_one(const orc_index *x, orc_work *w, const float *q, double alpha, double beta,
                     int k, int rule, int64_t *ids, float *d32, double *d64, orc_dump *dp)
{
    const int d = x->d, M = x->M, Ns = x->Ns, s = x->s, l = x->l, K = x->K;
    const int64_t n = x->n;
    const int64_t A = budget_A(alpha, n), R = budget_R(beta, n);

    /* line 1-2: transform q and split it into Ns subspaces */
    for (int m = 0; m < M; m++) w->qt[m] = 0.0f;
    for (int t = 0; t < d; t++) {
        float e = q[t] - x->mean[t];
        for (int m = 0; m < M; m++) w->qt[m] = fmaf(x->B[(size_t)t * M + m], e, w->qt[m]);
    }
    if (dp && dp->qt) memcpy(dp->qt, w->qt, sizeof(float) * (size_t)M);

    memset(w->sc, 0, (size_t)n);
    for (int j = 0; j < Ns; j++) {
        /* line 4-5: halves, distances to each half's centroids, sorted order */
        float *D1 = w->D, *D2 = w->D + l;
        int32_t *o1 = w->order, *o2 = w->order + l;
        orc_half_dists(w->qt + j * s, x->C1 + (size_t)j * l * x->h1, l, x->h1, D1);
        orc_half_dists(w->qt + j * s + x->h1, x->C2 + (size_t)j * l * x->h2, l, x->h2, D2);
        orc_argsort(D1, l, o1);
        orc_argsort(D2, l, o2);
        if (dp && dp->cdist) memcpy(dp->cdist + (size_t)j * 2 * l, w->D, sizeof(float) * 2 * (size_t)l);
        if (dp && dp->corder) memcpy(dp->corder + (size_t)j * 2 * l, w->order, sizeof(int32_t) * 2 * (size_t)l);

        /* line 6: Scalable Dynamic Activation */
        const uint64_t *off = x->offsets + (size_t)j * (K + 1);
        for (int c = 0; c < K; c++) w->size[c] = (int64_t)(off[c + 1] - off[c]);
        int32_t nc = 0;
        int64_t got = orc_probe(D1, o1, D2, o2, l, w->size, A, w->cells, &nc);
        if (dp && dp->cells) memcpy(dp->cells + (size_t)j * K, w->cells, sizeof(int32_t) * (size_t)nc);
        if (dp && dp->ncells) dp->ncells[j] = nc;
        if (dp && dp->retrieved) dp->retrieved[j] = got;

        /* line 7: one collision for every point of every retrieved cell */
        const uint32_t *ids_j = x->ids + (size_t)j * n;
        for (int i = 0; i < nc; i++)
            for (uint64_t p = off[w->cells[i]]; p < off[w->cells[i] + 1]; p++) w->sc[ids_j[p]]++;
    }
    if (dp && dp->sc) memcpy(dp->sc, w->sc, (size_t)n);

    /* line 8: Query-aware Candidates Selection */
    int64_t hist[256];
    int32_t last = 0;
    int64_t nc = orc_select(w->sc, n, Ns, R, rule, hist, &last, w->cand);
    if (nc < 0) return ORC_ENOMEM;
    if (dp && dp->hist) memcpy(dp->hist, hist, sizeof(int64_t) * (size_t)(Ns + 1));
    if (dp && dp->last) dp->last[0] = last;
    if (dp && dp->ncand) dp->ncand[0] = nc;
    if (dp && dp->cand) memcpy(dp->cand, w->cand, sizeof(int32_t) * (size_t)nc);

    /* line 9: exact distances of the candidates, top-k by (distance, id) */
    for (int64_t i = 0; i < nc; i++) {
        int32_t id = w->cand[i];
        row_dist(q, x->base + (size_t)id * d, d, &w->res[i].key, &w->res[i].d64);
        w->res[i].id = id;
        if (dp && dp->cand_d32) dp->cand_d32[i] = w->res[i].key;
        if (dp && dp->cand_d64) dp->cand_d64[i] = w->res[i].d64;
    }
    qsort(w->res, (size_t)nc, sizeof(rres), rcmp);
    for (int i = 0; i < k; i++) {
        if (i < nc) {
            ids[i] = w->res[i].id;
            if (d32) d32[i] = w->res[i].key;
            if (d64) d64[i] = w->res[i].d64;
        } else {
            ids[i] = -1;
            if (d32) d32[i] = INFINITY;
            if (d64) d64[i] = INFINITY;
        }
    }
    return ORC_OK;
}

static int check_args(const orc_index *x, double alpha, double beta, int k, int rule)
{
    if (!x || !(alpha > 0.0 && alpha <= 1.0) || !(beta >= 0.0 && beta <= 1.0) || k < 1 ||
        (int64_t)k > x->n || (rule != ORC_RULE_PRINTED && rule != ORC_RULE_PROSE && rule != ORC_RULE_FIXED) || x->Ns > 255)
        return ORC_EINVAL;
    return ORC_OK;
}

/* One query with optional per-stage dumps. */
int orc_query(const orc_index *x, const float *q, double alpha, double beta, int k, int rule,
              int64_t *ids, float *d32, double *d64, orc_dump *dump)
{
    int rc = check_args(x, alpha, beta, k, rule);
    if (rc) return rc;
    orc_work w;
    rc = work_init(x, &w);
    if (!rc) rc = query_one(x, &w, q, alpha, beta, k, rule, ids, d32, d64, dump);
    work_free(&w);
    return rc;
}

/* A batch of queries, in parallel over queries on `nthreads` threads
 * (<= 0: the OpenMP default).  alpha may be per query (alpha_per_q != NULL)
 * or shared.  Outputs are nq x k. */
int orc_query_batch(const orc_index *x, const float *Q, int64_t nq, double alpha,
                    const double *alpha_per_q, double beta, int k, int rule, int nthreads,
                    int64_t *ids, float *d32, double *d64)
{
    int rc = check_args(x, alpha_per_q ? 0.5 : alpha, beta, k, rule);
    if (rc) return rc;
    int err = ORC_OK;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
#pragma omp parallel num_threads(nthreads)
    {
        orc_work w;
        int lrc = work_init(x, &w);
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < nq; i++) {
            if (lrc) continue;
            double a = alpha_per_q ? alpha_per_q[i] : alpha;
            if (!(a > 0.0 && a <= 1.0)) { lrc = ORC_EINVAL; continue; }
            query_one(x, &w, Q + (size_t)i * x->d, a, beta, k, rule, ids + (size_t)i * k,
                      d32 ? d32 + (size_t)i * k : NULL, d64 ? d64 + (size_t)i * k : NULL, NULL);
        }
        if (lrc) {
#pragma omp critical
            err = lrc;
        }
        work_free(&w);
    }
    return err;
}

/* Threads the OpenMP runtime would use by default. */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* SC-Linear (Section 2.3; Definitions 5 and 6): the index-free baseline.      */
/* ------------------------------------------------------------------------- */

typedef struct {
    float dist;
    int32_t id;
} sdist;

static int sdcmp(const void *pa, const void *pb)
{
    const sdist *a = (const sdist *)pa, *b = (const sdist *)pb;
    if (a->dist != b->dist) return a->dist < b->dist ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

/*
 * SC-Linear for one query.  Subspace j is the j-th block of s columns of the
 * transformed space (the index's own subspaces): the query and every base
 * point are transformed with the canonical chain (T holds the base, n x M),
 * and their squared distance in subspace j is the canonical half-distance
 * chain over the block's s coordinates.  A point collides with the query in
 * subspace j when it is among the A = ceil(alpha*n) nearest there (Definition
 * 5), nearest meaning ascending (distance, id); its SC-score counts those
 * subspaces (Definition 6).  The candidates are the R = floor(beta*n) points
 * of highest SC-score, ties by the lower id (the selection SC-Linear makes,
 * Section 2.3); they are re-ranked by the FP32 distance in the original
 * space and the k smallest (distance, id) returned, padded with -1 / +inf.
 * Written as the definitions: a full sort per subspace, a full sort of the
 * scores.  sc_out (n, may be NULL) receives the SC-scores; cand_out (n, may
 * be NULL) the candidates in ascending id and ncand_out their number.
 */
int orc_sclinear(const orc_index *x, const float *T, const float *q, double alpha, double beta, int k,
                 int64_t *ids, float *d32, uint8_t *sc_out, int32_t *cand_out, int64_t *ncand_out)
{
    if (check_args(x, alpha, beta, k, ORC_RULE_FIXED)) return ORC_EINVAL;
    const int d = x->d, M = x->M, Ns = x->Ns, s = x->s;
    const int64_t n = x->n;
    const int64_t A = budget_A(alpha, n), R = budget_R(beta, n);
    float *qt = (float *)malloc(sizeof(float) * (size_t)M);
    sdist *all = (sdist *)malloc(sizeof(sdist) * (size_t)n);
    uint8_t *sc = (uint8_t *)calloc((size_t)n, 1);
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    rres *res = (rres *)malloc(sizeof(rres) * (size_t)n);
    int rc = ORC_ENOMEM;
    if (!qt || !all || !sc || !cand || !res) goto out;
    for (int m = 0; m < M; m++) qt[m] = 0.0f;
    for (int t = 0; t < d; t++) {
        float e = q[t] - x->mean[t];
        for (int m = 0; m < M; m++) qt[m] = fmaf(x->B[(size_t)t * M + m], e, qt[m]);
    }
    /* collisions: the A nearest points of every subspace */
    for (int j = 0; j < Ns; j++) {
        for (int64_t i = 0; i < n; i++) {
            const float *r = T + (size_t)i * M + (size_t)j * s;
            float acc = 0.0f;
            for (int c = 0; c < s; c++) {
                float u = qt[j * s + c] - r[c];
                acc = fmaf(u, u, acc);
            }
            all[i].dist = acc;
            all[i].id = (int32_t)i;
        }
        qsort(all, (size_t)n, sizeof(sdist), sdcmp);
        for (int64_t z = 0; z < A; z++) sc[all[z].id]++;
    }
    /* candidates: the R highest SC-scores, ties by the lower id */
    int32_t last = 0;
    int64_t nc = select_fixed(sc, n, Ns, R, &last, cand);
    if (nc < 0) goto out;
    /* refinement in the original space */
    for (int64_t i = 0; i < nc; i++) {
        double unused;
        row_dist(q, x->base + (size_t)cand[i] * d, d, &res[i].key, &unused);
        res[i].id = cand[i];
        res[i].d64 = unused;
    }
    qsort(res, (size_t)nc, sizeof(rres), rcmp);
    for (int i = 0; i < k; i++) {
        ids[i] = i < nc ? res[i].id : -1;
        if (d32) d32[i] = i < nc ? res[i].key : INFINITY;
    }
    if (sc_out) memcpy(sc_out, sc, (size_t)n);
    if (cand_out) memcpy(cand_out, cand, sizeof(int32_t) * (size_t)nc);
    if (ncand_out) *ncand_out = nc;
    rc = ORC_OK;
out:
    free(qt); free(all); free(sc); free(cand); free(res);
    return rc;
}

/* SC-Linear for a batch of queries, in parallel over queries on `nthreads`
 * threads (<= 0: the OpenMP default).  Outputs nq x k. */
int orc_sclinear_batch(const orc_index *x, const float *T, const float *Q, int64_t nq, double alpha,
                       double beta, int k, int nthreads, int64_t *ids, float *d32)
{
    if (check_args(x, alpha, beta, k, ORC_RULE_FIXED)) return ORC_EINVAL;
    int err = ORC_OK;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < nq; i++) {
        int rc = orc_sclinear(x, T, Q + (size_t)i * x->d, alpha, beta, k, ids + (size_t)i * k,
                              d32 ? d32 + (size_t)i * k : NULL, NULL, NULL, NULL);
        if (rc) {
#pragma omp critical
            err = rc;
        }
    }
    return err;
}

/* ------------------------------------------------------------------------- */
/* Ground truth: exact k-NN by brute force in FP64 (Definition 2).             */
/* ------------------------------------------------------------------------- */

/* For each query, the k base rows with the smallest FP64 squared distance,
 * ascending by (distance, id). */
void orc_bruteforce(const float *X, int64_t n, int d, const float *Q, int64_t nq, int k,
                    int64_t *ids, double *dist)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < nq; qi++) {
        const float *q = Q + (size_t)qi * d;
        int64_t *bi = ids + (size_t)qi * k;
        double *bd = dist + (size_t)qi * k;
        int have = 0;
        for (int64_t i = 0; i < n; i++) {
            const float *x = X + (size_t)i * d;
            double s = 0.0;
            for (int t = 0; t < d; t++) {
                double u = (double)q[t] - (double)x[t];
                s += u * u;
            }
            /* keep the k best so far in ascending (distance, id) order; ids
             * arrive ascending, so an equal distance never displaces */
            if (have == k && !(s < bd[k - 1])) continue;
            int p = have < k ? have++ : k - 1;
            while (p > 0 && bd[p - 1] > s) {
                bd[p] = bd[p - 1];
                bi[p] = bi[p - 1];
                p--;
            }
            bd[p] = s;
            bi[p] = i;
        }
        for (int p = have; p < k; p++) {
            bd[p] = INFINITY;
            bi[p] = -1;
        }
    }
}

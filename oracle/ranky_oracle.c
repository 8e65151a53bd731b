/*
 * ranky_oracle.c -- plain CPU FP64 reference for the rank-safe column-block SVD
 * of a short-and-fat sparse matrix (Tugay & Gunduz Oguducu, "Ranky", arXiv
 * 2009.09767, Sec. III, Eq. (1)-(3), Alg. 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library neither
 * links nor calls it, and the two share no code, header or constant.
 *
 * Everything is written for a reader checking it against the paper and the
 * textbook definitions, not for speed: dense FP64 arrays, loops that follow
 * the definitions, OpenMP only over independent items (disjoint rotation
 * pairs, independent columns).  No BLAS, no LAPACK.
 *
 * What it computes (one function per step):
 *   ro_check_csc      input contract: colptr monotone, rows sorted/unique/in range, finite values
 *   ro_occupancy      Alg. 1 scan: per-(block,row) nonzero counts -> lonely rows (count 0)
 *                     and rows with exactly one entry (the NO of Eq. 4)
 *   ro_rank_prob      Eq. 4: Pr ~= 1 - NO/NC
 *   ro_gram           G = A A^T = sum over blocks of A^i A^i^T (Eq. 2), by definition
 *   ro_bf16_split     x (FP32) = hi + lo + rest, hi = bf16(x), lo = bf16(x - hi), round to nearest even
 *   ro_gram_bf16x3    sum over columns of hi_p hi_q + hi_p lo_q + lo_p hi_q for a chosen set of rows:
 *                     the split-bf16 product of the mixed path's dense tiles, by definition
 *   ro_hestenes       one-sided (Hestenes) Jacobi SVD of a dense row block: the "truth" route
 *   ro_qr_r           Householder QR of a tall matrix (R factor only), a preconditioner for Hestenes
 *   ro_eig_jacobi     two-sided cyclic Jacobi eigensolver of a dense symmetric matrix
 *   ro_svd            the whole pipeline: O-A (whole-matrix Hestenes), O-B (the paper's block
 *                     merge through the proxy matrix P, Sec. III / Alg. 1), O-G (Gram + eig),
 *                     then the rank-safe threshold, sign convention and back-projection of V
 *   ro_backproject    V = A^T U Sigma^{-1} on the retained triplets only (zero columns beyond rank)
 *
 * Readings of the paper that this file commits to (the paper leaves them open):
 *   - block b holds columns [floor(b N / D), floor((b+1) N / D)) (every column is covered);
 *   - loop bounds of Alg. 1 are half-open (0..D-1, 0..M-1);
 *   - a block keeps every triplet with sigma > 0: a row that is empty inside a block only
 *     removes a zero singular value, which contributes nothing to the proxy matrix, so the
 *     merge of Eq. (2)-(3) is exact for any block rank and no entry of A is altered;
 *   - rank threshold: sigma_i counts as zero iff sigma_i <= tau with
 *     tau = max(tol, sqrt(M' * u_G)) * sigma_1, M' = number of non-empty rows and u_G the
 *     unit roundoff in which the Gram entries of the path under test are accumulated;
 *   - globally empty rows are removed before the solve and come back as sigma = 0 with
 *     U column e_row, in ascending row order, after the eigenvectors of the other rows;
 *   - sign: the entry of largest magnitude of each returned left vector is positive (lowest
 *     row index on an exact tie).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RO_OK 0
#define RO_E_INVALID 1
#define RO_E_CSC 2
#define RO_E_NONFINITE 3
#define RO_E_NOMEM 4
#define RO_E_NOT_CONVERGED 8

/* value types of the CSC values array */
#define RO_F32 0
#define RO_F64 1

/* methods of ro_svd */
#define RO_METHOD_WHOLE 0    /* O-A: Hestenes on the dense non-empty rows of A */
#define RO_METHOD_WHOLE_QR 1 /* O-A with Householder QR preconditioning of A^T */
#define RO_METHOD_MERGE 2    /* O-B: per-block SVD, proxy matrix, SVD of the proxy */
#define RO_METHOD_GRAM 3     /* O-G: Gram matrix + two-sided Jacobi eigensolver */

static double value_at(const void *vals, int dtype, int64_t k) {
    if (dtype == RO_F64) return ((const double *)vals)[k];
    return (double)((const float *)vals)[k];
}

/* ------------------------------------------------------------------------- */
/* Input contract                                                            */
/* ------------------------------------------------------------------------- */

/* Returns RO_OK, RO_E_INVALID (bad sizes), RO_E_CSC (structure) or
 * RO_E_NONFINITE.  A structural error takes precedence over a non-finite value. */
int ro_check_csc(int32_t M, int64_t N, int64_t nnz, const int32_t *colptr,
                 const int32_t *rowidx, const void *vals, int dtype) {
    if (M < 1 || N < 1 || nnz < 0 || (dtype != RO_F32 && dtype != RO_F64)) return RO_E_INVALID;
    if (colptr[0] != 0 || (int64_t)colptr[N] != nnz) return RO_E_CSC;
    for (int64_t j = 0; j < N; ++j)
        if (colptr[j + 1] < colptr[j]) return RO_E_CSC;
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t k = colptr[j]; k < colptr[j + 1]; ++k) {
            int32_t r = rowidx[k];
            if (r < 0 || r >= M) return RO_E_CSC;
            if (k > colptr[j] && rowidx[k - 1] >= r) return RO_E_CSC; /* unsorted or duplicate */
        }
    }
    for (int64_t k = 0; k < nnz; ++k)
        if (!isfinite(value_at(vals, dtype, k))) return RO_E_NONFINITE;
    return RO_OK;
}

/* Balanced block boundaries: start[b] = floor(b N / D), start[D] = N. */
int ro_block_bounds(int64_t N, int32_t D, int64_t *start) {
    if (D < 1 || N < 1 || D > N) return RO_E_INVALID;
    for (int32_t b = 0; b <= D; ++b) start[b] = ((int64_t)b * N) / D;
    return RO_OK;
}

/* ------------------------------------------------------------------------- */
/* Alg. 1 scan: which rows are lonely inside which block                     */
/* ------------------------------------------------------------------------- */

/* cnt[b*M + m] = number of nonzeros of row m inside block b;
 * rownnz[m]    = number of nonzeros of row m in the whole matrix;
 * lonely[b]    = number of rows with no entry inside block b (Alg. 1 "Checker" stays true);
 * single[b]    = number of rows with exactly one entry inside block b (NO of Eq. 4). */
int ro_occupancy(int32_t M, int64_t N, const int32_t *colptr, const int32_t *rowidx,
                 int32_t D, const int64_t *start, int32_t *cnt, int32_t *rownnz,
                 int32_t *lonely, int32_t *single) {
    memset(cnt, 0, sizeof(int32_t) * (size_t)D * (size_t)M);
    memset(rownnz, 0, sizeof(int32_t) * (size_t)M);
    for (int32_t b = 0; b < D; ++b) {
        for (int64_t j = start[b]; j < start[b + 1]; ++j) {
            for (int64_t k = colptr[j]; k < colptr[j + 1]; ++k) {
                cnt[(size_t)b * M + rowidx[k]] += 1;
                rownnz[rowidx[k]] += 1;
            }
        }
        lonely[b] = 0;
        single[b] = 0;
        for (int32_t m = 0; m < M; ++m) {
            if (cnt[(size_t)b * M + m] == 0) lonely[b] += 1;
            if (cnt[(size_t)b * M + m] == 1) single[b] += 1;
        }
    }
    (void)N;
    return RO_OK;
}

/* Eq. 4: probability that a block keeps the rank of A after a random fill,
 * with NC columns in the block and NO rows holding exactly one entry. */
double ro_rank_prob(int64_t NC, int64_t NO) { return 1.0 - (1.0 / (double)NC) * (double)NO; }

/* ------------------------------------------------------------------------- */
/* Gram matrix, Eq. (2): A A^T = sum_i A^i A^i^T = sum over columns a_j a_j^T */
/* ------------------------------------------------------------------------- */

/* G is M x M row-major, full (both triangles).  Columns are visited in order,
 * which visits the blocks in order, so G accumulates G_1 + G_2 + ... + G_D. */
/* bf16 of an FP32 value, round to nearest even (finite values), returned as the FP32
 * value it stands for: the top 16 bits of the FP32 pattern after adding half an ulp of
 * bf16 (plus one when the kept part is odd, which breaks ties to even). */
static float bf16_rne(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    float y;
    memcpy(&y, &r, 4);
    return y;
}

int ro_bf16_split(int64_t n, const float *x, float *hi, float *lo) {
    for (int64_t i = 0; i < n; ++i) {
        hi[i] = bf16_rne(x[i]);
        lo[i] = bf16_rne(x[i] - hi[i]);   /* exact difference in FP32 (Sterbenz) */
    }
    return RO_OK;
}

/* G[a][b], a, b < nr (rows rows[0..nr)), of the split-bf16 product: the values are taken
 * in FP32 (FP64 values are rounded to FP32 first), split, and the three kept products
 * summed in FP64. */
int ro_gram_bf16x3(int32_t M, int64_t N, const int32_t *colptr, const int32_t *rowidx, const void *vals,
                   int dtype, int32_t nr, const int32_t *rows, double *G) {
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M > 0 ? M : 1));
    if (!slot) return RO_E_NOMEM;
    for (int32_t m = 0; m < M; ++m) slot[m] = -1;
    for (int32_t a = 0; a < nr; ++a) slot[rows[a]] = a;
    memset(G, 0, sizeof(double) * (size_t)nr * (size_t)nr);
    for (int64_t j = 0; j < N; ++j)
        for (int64_t k1 = colptr[j]; k1 < colptr[j + 1]; ++k1) {
            const int32_t a = slot[rowidx[k1]];
            if (a < 0) continue;
            const float x = (float)value_at(vals, dtype, k1);
            const double h1 = bf16_rne(x), l1 = bf16_rne(x - bf16_rne(x));
            for (int64_t k2 = colptr[j]; k2 < colptr[j + 1]; ++k2) {
                const int32_t b = slot[rowidx[k2]];
                if (b < 0) continue;
                const float y = (float)value_at(vals, dtype, k2);
                const double h2 = bf16_rne(y), l2 = bf16_rne(y - bf16_rne(y));
                G[(size_t)a * nr + b] += h1 * h2 + h1 * l2 + l1 * h2;
            }
        }
    free(slot);
    return RO_OK;
}

int ro_gram(int32_t M, int64_t N, const int32_t *colptr, const int32_t *rowidx,
            const void *vals, int dtype, double *G) {
    memset(G, 0, sizeof(double) * (size_t)M * (size_t)M);
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t k1 = colptr[j]; k1 < colptr[j + 1]; ++k1) {
            double a1 = value_at(vals, dtype, k1);
            int32_t p = rowidx[k1];
            for (int64_t k2 = k1; k2 < colptr[j + 1]; ++k2) {
                int32_t q = rowidx[k2];
                G[(size_t)p * M + q] += a1 * value_at(vals, dtype, k2);
            }
        }
    }
    for (int32_t p = 0; p < M; ++p)
        for (int32_t q = 0; q < p; ++q) G[(size_t)p * M + q] = G[(size_t)q * M + p];
    return RO_OK;
}

/* ------------------------------------------------------------------------- */
/* Parallel (round-robin) ordering of index pairs                            */
/* ------------------------------------------------------------------------- */

/* Round r (0 <= r < n-1) of the round-robin tournament on n (even) players:
 * player n-1 meets r, and (r+i) mod (n-1) meets (r-i) mod (n-1) for i >= 1.
 * Over the n-1 rounds every unordered pair meets exactly once, and the n/2
 * pairs of one round are disjoint, so their rotations commute. */
static void round_robin_pair(int32_t n, int32_t r, int32_t i, int32_t *p, int32_t *q) {
    int32_t a, b;
    if (i == 0) {
        a = n - 1;
        b = r;
    } else {
        a = (r + i) % (n - 1);
        b = (r - i + (n - 1)) % (n - 1);
    }
    *p = a < b ? a : b;
    *q = a < b ? b : a;
}

/* Jacobi rotation that annihilates the (p,q) coupling, for diagonal entries
 * alpha, beta and coupling gamma != 0 (Rutishauser's stable form):
 * zeta = (beta - alpha) / (2 gamma), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
 * c = 1 / sqrt(1 + t^2), s = c t. */
static void jacobi_rotation(double alpha, double beta, double gamma, double *c, double *s,
                            double *t) {
    double zeta = (beta - alpha) / (2.0 * gamma);
    double tt;
    if (fabs(zeta) > 1e150)
        tt = 0.5 / zeta;
    else
        tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    *c = 1.0 / sqrt(1.0 + tt * tt);
    *s = (*c) * tt;
    *t = tt;
}

/* ------------------------------------------------------------------------- */
/* One-sided (Hestenes) Jacobi SVD of a dense m x n row block                 */
/* ------------------------------------------------------------------------- */

/* B (m x n, row-major) is overwritten by J^T B whose rows are mutually
 * orthogonal; U (m x m, row-major) receives J, so the input equals U * B_out,
 * and sigma[i] = ||row i of B_out||.  The singular values are not sorted.
 * Rows p, q are rotated when |<b_p,b_q>| > tol sqrt(|b_p|^2 |b_q|^2), with
 * tol = max(1e-15, sqrt(n) eps) (the dot product's own rounding is ~sqrt(n) eps).
 * A row whose squared norm is below (m n eps)^2 times the largest initial one
 * is numerical noise (its singular value is far below any rank threshold) and
 * takes part in no rotation; without this, rounding noise in a rank-deficient
 * block never becomes orthogonal to the noise of another row.
 * Returns RO_E_NOT_CONVERGED if a sweep with no rotation is not reached. */
int ro_hestenes(int32_t m, int64_t n, double *B, double *U, double *sigma, int32_t max_sweeps,
                int32_t *sweeps_out) {
    const double tol = fmax(1e-15, sqrt((double)n) * DBL_EPSILON);
    const int32_t me = m + (m & 1); /* even number of players; index m is a bye */
    for (int32_t i = 0; i < m; ++i)
        for (int32_t j = 0; j < m; ++j) U[(size_t)i * m + j] = (i == j) ? 1.0 : 0.0;
    double amax = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        double a = 0.0;
        for (int64_t c = 0; c < n; ++c) a += B[(size_t)i * n + c] * B[(size_t)i * n + c];
        if (a > amax) amax = a;
    }
    const double noise = (double)m * (double)n * DBL_EPSILON;
    const double noise2 = noise * noise * amax;
    int32_t sweep = 0, converged = (m < 2);
    while (!converged && sweep < max_sweeps) {
        int64_t rotations = 0;
        for (int32_t r = 0; r < me - 1; ++r) {
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : rotations)
            for (int32_t i = 0; i < me / 2; ++i) {
                int32_t p, q;
                round_robin_pair(me, r, i, &p, &q);
                if (q >= m) continue;
                double *bp = B + (size_t)p * n, *bq = B + (size_t)q * n;
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t c = 0; c < n; ++c) {
                    alpha += bp[c] * bp[c];
                    beta += bq[c] * bq[c];
                    gamma += bp[c] * bq[c];
                }
                if (alpha <= noise2 || beta <= noise2) continue;
                if (gamma == 0.0 || !(fabs(gamma) > tol * sqrt(alpha * beta))) continue;
                double cs, sn, t;
                jacobi_rotation(alpha, beta, gamma, &cs, &sn, &t);
                for (int64_t c = 0; c < n; ++c) {
                    double x = bp[c], y = bq[c];
                    bp[c] = cs * x - sn * y;
                    bq[c] = sn * x + cs * y;
                }
                for (int32_t row = 0; row < m; ++row) {
                    double x = U[(size_t)row * m + p], y = U[(size_t)row * m + q];
                    U[(size_t)row * m + p] = cs * x - sn * y;
                    U[(size_t)row * m + q] = sn * x + cs * y;
                }
                rotations += 1;
            }
        }
        sweep += 1;
        if (rotations == 0) converged = 1;
    }
    for (int32_t i = 0; i < m; ++i) {
        double s2 = 0.0;
        for (int64_t c = 0; c < n; ++c) s2 += B[(size_t)i * n + c] * B[(size_t)i * n + c];
        sigma[i] = sqrt(s2);
    }
    if (sweeps_out) *sweeps_out = sweep;
    return converged ? RO_OK : RO_E_NOT_CONVERGED;
}

/* ------------------------------------------------------------------------- */
/* Householder QR of a tall matrix, R factor only                             */
/* ------------------------------------------------------------------------- */

/* X is rows x cols (rows >= cols) in column-major order with leading dimension
 * rows; it is destroyed.  R (cols x cols, row-major, upper triangular) receives
 * the triangular factor of X = Q R.  Column c of X is reflected by
 * H = I - beta v v^T with v = x - alpha e_1, alpha = -sign(x_1) ||x||. */
int ro_qr_r(int64_t rows, int32_t cols, double *X, double *R) {
    if (rows < cols) return RO_E_INVALID;
    double *v = (double *)malloc(sizeof(double) * (size_t)rows);
    if (!v) return RO_E_NOMEM;
    memset(R, 0, sizeof(double) * (size_t)cols * (size_t)cols);
    for (int32_t j = 0; j < cols; ++j) {
        double *xj = X + (size_t)j * rows;
        double norm2 = 0.0;
        for (int64_t i = j; i < rows; ++i) norm2 += xj[i] * xj[i];
        double norm = sqrt(norm2);
        if (norm == 0.0) {
            R[(size_t)j * cols + j] = 0.0;
            for (int32_t c = j + 1; c < cols; ++c) R[(size_t)j * cols + c] = X[(size_t)c * rows + j];
            continue;
        }
        double alpha = (xj[j] >= 0.0) ? -norm : norm;
        int64_t len = rows - j;
        for (int64_t i = 0; i < len; ++i) v[i] = xj[j + i];
        v[0] -= alpha;
        double vnorm2 = 0.0;
        for (int64_t i = 0; i < len; ++i) vnorm2 += v[i] * v[i];
        double beta = (vnorm2 > 0.0) ? 2.0 / vnorm2 : 0.0;
#pragma omp parallel for schedule(static)
        for (int32_t c = j + 1; c < cols; ++c) {
            double *xc = X + (size_t)c * rows + j;
            double w = 0.0;
            for (int64_t i = 0; i < len; ++i) w += v[i] * xc[i];
            w *= beta;
            for (int64_t i = 0; i < len; ++i) xc[i] -= w * v[i];
        }
        R[(size_t)j * cols + j] = alpha;
        for (int32_t c = j + 1; c < cols; ++c) R[(size_t)j * cols + c] = X[(size_t)c * rows + j];
    }
    free(v);
    return RO_OK;
}

/* ------------------------------------------------------------------------- */
/* Two-sided Jacobi eigensolver of a dense symmetric matrix                   */
/* ------------------------------------------------------------------------- */

/* G (n x n, row-major, symmetric) is overwritten; on return its diagonal holds
 * the eigenvalues (unsorted) and V (n x n, row-major) the eigenvectors as
 * columns, G_in = V diag(G_out) V^T.  The pair (p,q) is rotated when
 * |g_pq| > tol sqrt(|g_pp g_qq|), tol = max(1e-15, sqrt(n) eps), and
 * |g_pq| > (n eps)^2 max_i |g_ii| (couplings below that are rounding noise of a
 * numerically null block, far below any rank threshold).  The n/2
 * rotations of one round-robin round act on disjoint index pairs; they are
 * applied to all rows first and then to all columns, which is J^T G J. */
int ro_eig_jacobi(int32_t n, double *G, double *V, int32_t max_sweeps, int32_t *sweeps_out) {
    const double tol = fmax(1e-15, sqrt((double)n) * DBL_EPSILON);
    const int32_t ne = n + (n & 1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j) V[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    int32_t npairs = ne / 2;
    int32_t *P = (int32_t *)malloc(sizeof(int32_t) * (size_t)npairs * 2);
    double *C = (double *)malloc(sizeof(double) * (size_t)npairs * 5);
    if (!P || !C) {
        free(P);
        free(C);
        return RO_E_NOMEM;
    }
    double gmax = 0.0;
    for (int32_t i = 0; i < n; ++i) gmax = fmax(gmax, fabs(G[(size_t)i * n + i]));
    const double floor_abs = ((double)n * DBL_EPSILON) * ((double)n * DBL_EPSILON) * gmax;
    int32_t sweep = 0, converged = (n < 2);
    while (!converged && sweep < max_sweeps) {
        int64_t rotations = 0;
        for (int32_t r = 0; r < ne - 1; ++r) {
            /* 1. rotation parameters of every pair from the current G */
            for (int32_t i = 0; i < npairs; ++i) {
                int32_t p, q;
                round_robin_pair(ne, r, i, &p, &q);
                P[2 * i] = p;
                P[2 * i + 1] = q;
                C[5 * i] = 1.0; /* c */
                C[5 * i + 1] = 0.0; /* s */
                C[5 * i + 2] = 0.0; /* active flag */
                if (q >= n) continue;
                double a = G[(size_t)p * n + p], b = G[(size_t)q * n + q], g = G[(size_t)p * n + q];
                if (!(fabs(g) > floor_abs) || !(fabs(g) > tol * sqrt(fabs(a * b)))) continue;
                double cs, sn, t;
                jacobi_rotation(a, b, g, &cs, &sn, &t);
                C[5 * i] = cs;
                C[5 * i + 1] = sn;
                C[5 * i + 2] = 1.0;
                C[5 * i + 3] = a - t * g; /* new g_pp */
                C[5 * i + 4] = b + t * g; /* new g_qq */
                rotations += 1;
            }
            /* 2. rows p, q <- rotation (all columns) */
#pragma omp parallel for schedule(static)
            for (int32_t i = 0; i < npairs; ++i) {
                if (C[5 * i + 2] == 0.0) continue;
                int32_t p = P[2 * i], q = P[2 * i + 1];
                double cs = C[5 * i], sn = C[5 * i + 1];
                double *gp = G + (size_t)p * n, *gq = G + (size_t)q * n;
                for (int32_t c = 0; c < n; ++c) {
                    double x = gp[c], y = gq[c];
                    gp[c] = cs * x - sn * y;
                    gq[c] = sn * x + cs * y;
                }
            }
            /* 3. columns p, q <- rotation (all rows), same for V */
#pragma omp parallel for schedule(static)
            for (int32_t row = 0; row < n; ++row) {
                double *gr = G + (size_t)row * n, *vr = V + (size_t)row * n;
                for (int32_t i = 0; i < npairs; ++i) {
                    if (C[5 * i + 2] == 0.0) continue;
                    int32_t p = P[2 * i], q = P[2 * i + 1];
                    double cs = C[5 * i], sn = C[5 * i + 1];
                    double x = gr[p], y = gr[q];
                    gr[p] = cs * x - sn * y;
                    gr[q] = sn * x + cs * y;
                    x = vr[p];
                    y = vr[q];
                    vr[p] = cs * x - sn * y;
                    vr[q] = sn * x + cs * y;
                }
            }
            /* 4. the annihilated 2x2 block takes its exact post-rotation values */
            for (int32_t i = 0; i < npairs; ++i) {
                if (C[5 * i + 2] == 0.0) continue;
                int32_t p = P[2 * i], q = P[2 * i + 1];
                G[(size_t)p * n + q] = 0.0;
                G[(size_t)q * n + p] = 0.0;
                G[(size_t)p * n + p] = C[5 * i + 3];
                G[(size_t)q * n + q] = C[5 * i + 4];
            }
        }
        sweep += 1;
        if (rotations == 0) converged = 1;
    }
    free(P);
    free(C);
    if (sweeps_out) *sweeps_out = sweep;
    return converged ? RO_OK : RO_E_NOT_CONVERGED;
}

/* ------------------------------------------------------------------------- */
/* Dense helpers                                                              */
/* ------------------------------------------------------------------------- */

/* Dense copy of the rows listed in rows[0..n) and the columns [c0, c1):
 * out is n x (c1 - c0), row-major.  rowmap[m] = position of row m in rows, or -1. */
static void densify(int32_t n, const int32_t *rowmap, int64_t c0, int64_t c1,
                    const int32_t *colptr, const int32_t *rowidx, const void *vals, int dtype,
                    double *out) {
    int64_t w = c1 - c0;
    memset(out, 0, sizeof(double) * (size_t)n * (size_t)w);
    for (int64_t j = c0; j < c1; ++j)
        for (int64_t k = colptr[j]; k < colptr[j + 1]; ++k) {
            int32_t r = rowmap[rowidx[k]];
            if (r >= 0) out[(size_t)r * w + (j - c0)] = value_at(vals, dtype, k);
        }
}

/* SVD of a dense n x w row block (left vectors and singular values only).
 * Uses Householder QR preconditioning when asked and w >= n:
 * X^T = Q R  =>  X = R^T Q^T, and the Hestenes SVD of R^T = U S W^T gives X = U S (Q W)^T. */
static int dense_left_svd(int32_t n, int64_t w, double *X, int use_qr, double *U, double *sigma,
                          int32_t max_sweeps, int32_t *sweeps) {
    if (use_qr && w >= n && n > 0) {
        /* X row-major n x w is X^T column-major w x n with leading dimension w */
        double *R = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
        double *Rt = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
        if (!R || !Rt) {
            free(R);
            free(Rt);
            return RO_E_NOMEM;
        }
        int st = ro_qr_r(w, n, X, R);
        if (st == RO_OK) {
            for (int32_t i = 0; i < n; ++i)
                for (int32_t j = 0; j < n; ++j) Rt[(size_t)i * n + j] = R[(size_t)j * n + i];
            st = ro_hestenes(n, n, Rt, U, sigma, max_sweeps, sweeps);
        }
        free(R);
        free(Rt);
        return st;
    }
    return ro_hestenes(n, w, X, U, sigma, max_sweeps, sweeps);
}

/* ------------------------------------------------------------------------- */
/* Back-projection of the right singular vectors                              */
/* ------------------------------------------------------------------------- */

/* V (N x k, row-major): V[j][i] = (sum_m a_mj U[m][i]) / sigma[i] for i < rank,
 * and 0 for i >= rank, so no vanishing sigma is ever divided by. */
int ro_backproject(int32_t M, int64_t N, const int32_t *colptr, const int32_t *rowidx,
                   const void *vals, int dtype, int32_t k, const double *U, const double *sigma,
                   int32_t rank, double *V) {
    (void)M;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        for (int32_t i = 0; i < k; ++i) {
            double acc = 0.0;
            if (i < rank) {
                for (int64_t kk = colptr[j]; kk < colptr[j + 1]; ++kk)
                    acc += value_at(vals, dtype, kk) * U[(size_t)rowidx[kk] * k + i];
                acc = acc / sigma[i];
            }
            V[(size_t)j * k + i] = acc;
        }
    }
    return RO_OK;
}

/* ------------------------------------------------------------------------- */
/* The whole pipeline                                                         */
/* ------------------------------------------------------------------------- */

/* Outputs: sigma[k], U (M x k row-major), V (N x k row-major, may be NULL),
 * rank, tau (the effective threshold), sweeps (largest sweep count of any
 * Jacobi run).  u_gram is the unit roundoff of the Gram accumulation of the
 * path under comparison (2^-53 for FP64); it only enters the threshold. */
int ro_svd(int32_t method, int32_t M, int64_t N, int64_t nnz, const int32_t *colptr,
           const int32_t *rowidx, const void *vals, int dtype, int32_t D, int32_t k, double tol,
           double u_gram, int32_t max_sweeps, double *sigma, double *U, double *V,
           int32_t *rank_out, double *tau_out, int32_t *sweeps_out) {
    if (k < 1 || k > M || tol < 0.0 || !(u_gram >= 0.0)) return RO_E_INVALID;
    int st = ro_check_csc(M, N, nnz, colptr, rowidx, vals, dtype);
    if (st != RO_OK) return st;
    if (method == RO_METHOD_MERGE && (D < 1 || D > N)) return RO_E_INVALID;

    /* 1. structural rank: non-empty rows R (kept in ascending order), empty rows E */
    int32_t *rownnz = (int32_t *)calloc((size_t)M, sizeof(int32_t));
    int32_t *rowmap = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    int32_t *empty = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    if (!rownnz || !rowmap || !rows || !empty) {
        free(rownnz);
        free(rowmap);
        free(rows);
        free(empty);
        return RO_E_NOMEM;
    }
    for (int64_t kk = 0; kk < nnz; ++kk) rownnz[rowidx[kk]] += 1;
    int32_t n = 0, ne = 0;
    for (int32_t m = 0; m < M; ++m) {
        if (rownnz[m] > 0) {
            rowmap[m] = n;
            rows[n++] = m;
        } else {
            rowmap[m] = -1;
            empty[ne++] = m;
        }
    }

    /* 2. singular values s[0..n) and left vectors W (n x n, columns) of A[R,:] */
    double *s = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *W = (double *)calloc((size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1), sizeof(double));
    int32_t sweeps = 0;
    if (!s || !W) st = RO_E_NOMEM;
    if (st == RO_OK && n > 0) {
        if (method == RO_METHOD_WHOLE || method == RO_METHOD_WHOLE_QR) {
            double *X = (double *)malloc(sizeof(double) * (size_t)n * (size_t)N);
            if (!X) st = RO_E_NOMEM;
            else {
                densify(n, rowmap, 0, N, colptr, rowidx, vals, dtype, X);
                st = dense_left_svd(n, N, X, method == RO_METHOD_WHOLE_QR, W, s, max_sweeps, &sweeps);
                free(X);
            }
        } else if (method == RO_METHOD_MERGE) {
            /* Eq. (1): reduced SVD of every block; P = [U^1 S^1 | ... | U^D S^D] (Sec. III) */
            int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(D + 1));
            int64_t pcap = 0;
            if (!start) st = RO_E_NOMEM;
            else {
                ro_block_bounds(N, D, start);
                pcap = (int64_t)D * n; /* at most n retained triplets per block */
            }
            double *Pm = NULL; /* proxy, n x pcap row-major */
            if (st == RO_OK) {
                Pm = (double *)calloc((size_t)n * (size_t)(pcap > 0 ? pcap : 1), sizeof(double));
                if (!Pm) st = RO_E_NOMEM;
            }
            int64_t pcols = 0;
            for (int32_t b = 0; st == RO_OK && b < D; ++b) {
                int64_t w = start[b + 1] - start[b];
                double *Xb = (double *)malloc(sizeof(double) * (size_t)n * (size_t)w);
                double *Ub = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
                double *sb = (double *)malloc(sizeof(double) * (size_t)n);
                if (!Xb || !Ub || !sb) st = RO_E_NOMEM;
                else {
                    int32_t sw = 0;
                    densify(n, rowmap, start[b], start[b + 1], colptr, rowidx, vals, dtype, Xb);
                    st = dense_left_svd(n, w, Xb, method == RO_METHOD_MERGE && w >= n, Ub, sb,
                                        max_sweeps, &sw);
                    if (sw > sweeps) sweeps = sw;
                    /* keep every triplet with sigma above the block's rounding-noise level
                       (n w eps sigma_max of the block, the level below which the Hestenes
                       routine treats a row as numerically zero): a block whose rank is below n
                       simply contributes fewer columns (rank-safe; A itself is never altered) */
                    double smax = 0.0;
                    for (int32_t i = 0; i < n; ++i) smax = fmax(smax, sb[i]);
                    const double keep = (double)n * (double)w * DBL_EPSILON * smax;
                    for (int32_t i = 0; st == RO_OK && i < n; ++i) {
                        if (!(sb[i] > keep)) continue;
                        if (pcols >= pcap) { st = RO_E_INVALID; break; }
                        for (int32_t r = 0; r < n; ++r)
                            Pm[(size_t)r * pcap + pcols] = Ub[(size_t)r * n + i] * sb[i];
                        pcols += 1;
                    }
                }
                free(Xb);
                free(Ub);
                free(sb);
            }
            if (st == RO_OK) {
                /* SVD of the proxy (Alg. 1, last step); compact its columns first */
                double *Pc = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(pcols > 0 ? pcols : 1));
                if (!Pc) st = RO_E_NOMEM;
                else {
                    for (int32_t r = 0; r < n; ++r)
                        for (int64_t c = 0; c < pcols; ++c) Pc[(size_t)r * pcols + c] = Pm[(size_t)r * pcap + c];
                    int32_t sw = 0;
                    st = dense_left_svd(n, pcols, Pc, pcols >= n, W, s, max_sweeps, &sw);
                    if (sw > sweeps) sweeps = sw;
                    free(Pc);
                }
            }
            free(Pm);
            free(start);
        } else if (method == RO_METHOD_GRAM) {
            double *Gf = (double *)malloc(sizeof(double) * (size_t)M * (size_t)M);
            double *Gc = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
            if (!Gf || !Gc) st = RO_E_NOMEM;
            else {
                ro_gram(M, N, colptr, rowidx, vals, dtype, Gf);
                for (int32_t a = 0; a < n; ++a)
                    for (int32_t b = 0; b < n; ++b)
                        Gc[(size_t)a * n + b] = Gf[(size_t)rows[a] * M + rows[b]];
                st = ro_eig_jacobi(n, Gc, W, max_sweeps, &sweeps);
                for (int32_t a = 0; a < n; ++a) {
                    double lam = Gc[(size_t)a * n + a];
                    s[a] = sqrt(lam > 0.0 ? lam : 0.0);
                }
            }
            free(Gf);
            free(Gc);
        } else {
            st = RO_E_INVALID;
        }
    }

    /* 3. order by descending sigma (ties keep the lower index first) */
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!order) st = (st == RO_OK) ? RO_E_NOMEM : st;
    if (st == RO_OK) {
        for (int32_t i = 0; i < n; ++i) order[i] = i;
        for (int32_t i = 1; i < n; ++i) { /* insertion sort: plain and stable */
            int32_t x = order[i], j = i - 1;
            while (j >= 0 && s[order[j]] < s[x]) {
                order[j + 1] = order[j];
                --j;
            }
            order[j + 1] = x;
        }
        /* 4. rank-safe threshold */
        double s1 = (n > 0) ? s[order[0]] : 0.0;
        double tau = fmax(tol, sqrt((double)n * u_gram)) * s1;
        int32_t rank = 0;
        for (int32_t i = 0; i < n; ++i)
            if (s[order[i]] > tau) rank += 1;
        /* 5. assemble sigma and U (M x k): eigen/singular vectors of the non-empty rows first,
              then e_row for each empty row in ascending order */
        memset(U, 0, sizeof(double) * (size_t)M * (size_t)k);
        for (int32_t i = 0; i < k; ++i) {
            if (i < n) {
                int32_t c = order[i];
                sigma[i] = (i < rank) ? s[c] : 0.0;
                int32_t best = 0;
                double bestabs = -1.0;
                for (int32_t r = 0; r < n; ++r) {
                    double a = fabs(W[(size_t)r * n + c]);
                    if (a > bestabs) {
                        bestabs = a;
                        best = r;
                    }
                }
                double sgn = (W[(size_t)best * n + c] < 0.0) ? -1.0 : 1.0;
                for (int32_t r = 0; r < n; ++r) U[(size_t)rows[r] * k + i] = sgn * W[(size_t)r * n + c];
            } else {
                sigma[i] = 0.0;
                U[(size_t)empty[i - n] * k + i] = 1.0;
            }
        }
        if (rank > k) rank = k;
        if (rank_out) *rank_out = rank;
        if (tau_out) *tau_out = tau;
        /* 6. V = A^T U Sigma^{-1} on the retained triplets */
        if (V) ro_backproject(M, N, colptr, rowidx, vals, dtype, k, U, sigma, rank, V);
    }
    if (sweeps_out) *sweeps_out = sweeps;
    free(order);
    free(s);
    free(W);
    free(rownnz);
    free(rowmap);
    free(rows);
    free(empty);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Alg. 2-4: the paper's checkers (lonely-node repair), on a copy of A        */
/* ------------------------------------------------------------------------- */

/* SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number generators", OOPSLA
 * 2014) used as a counter-based generator: output i of the stream with seed s is the
 * generator's mixing function applied to s + (i + 1) * 0x9E3779B97F4A7C15. */
static uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

#define RO_CHECK_RANDOM 0
#define RO_CHECK_NEIGHBOR 1
#define RO_CHECK_NEIGHBOR_RANDOM 2

static int cmp_i64(const void *a, const void *b) {
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* For every block b and every row m with no entry of A inside block b (Alg. 1), the checker
 * chosen by `kind` sets one entry of value 1 in row m inside block b of the copy A':
 *   RandomChecker (Alg. 2): column start[b] + (r0 mod width_b);
 *   NeighborChecker (Alg. 3): the neighbours of m are the rows that share a column with m outside
 *     block b; the candidate columns are the columns of block b holding an entry of a neighbour;
 *     the chosen one is the (r1 mod count)-th candidate in ascending column order (no candidate:
 *     the RandomChecker column);
 *   NeighborRandomChecker (Alg. 4): both entries (one if they coincide);
 * with r0 = output 2 (b M + m) and r1 = output 2 (b M + m) + 1 of the counter-based generator
 * above for `seed`.  Every decision reads the unmodified A (the repairs do not feed each other).
 * Output A' (CSC, FP64 values; rows strictly increasing in every column): colptr_out [N + 1],
 * rowidx_out and vals_out with room for nnz + 2 D M entries; *nnz_out; *inserted = entries added. */
int ro_checker(int32_t M, int64_t N, int64_t nnz, const int32_t *colptr, const int32_t *rowidx, const void *vals,
               int dtype, int32_t D, int32_t kind, uint64_t seed, int32_t *colptr_out, int32_t *rowidx_out,
               double *vals_out, int64_t *nnz_out, int64_t *inserted) {
    if (kind < RO_CHECK_RANDOM || kind > RO_CHECK_NEIGHBOR_RANDOM) return RO_E_INVALID;
    int st = ro_check_csc(M, N, nnz, colptr, rowidx, vals, dtype);
    if (st != RO_OK) return st;
    if (D < 1 || D > N) return RO_E_INVALID;
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(D + 1));
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)D * (size_t)M);
    int32_t *rownnz = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    int32_t *lon = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    int32_t *sgl = (int32_t *)malloc(sizeof(int32_t) * (size_t)D);
    int64_t *rowptr = (int64_t *)calloc((size_t)M + 1, sizeof(int64_t));
    int64_t *rcol = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)M);
    char *cand = (char *)malloc((size_t)M);
    int64_t *ins = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)D * (size_t)M);   /* col * M + row */
    char *mark = NULL;
    int64_t nins = 0;
    if (!start || !cnt || !rownnz || !lon || !sgl || !rowptr || !rcol || !fill || !cand || !ins) {
        st = RO_E_NOMEM;
        goto done;
    }
    ro_block_bounds(N, D, start);
    ro_occupancy(M, N, colptr, rowidx, D, start, cnt, rownnz, lon, sgl);
    /* the rows of A: columns of each row in ascending order */
    for (int64_t k = 0; k < nnz; ++k) rowptr[rowidx[k] + 1] += 1;
    for (int32_t m = 0; m < M; ++m) rowptr[m + 1] += rowptr[m];
    for (int32_t m = 0; m < M; ++m) fill[m] = rowptr[m];
    for (int64_t j = 0; j < N; ++j)
        for (int64_t k = colptr[j]; k < colptr[j + 1]; ++k) rcol[fill[rowidx[k]]++] = j;
    int64_t wmax = 0;
    for (int32_t b = 0; b < D; ++b)
        if (start[b + 1] - start[b] > wmax) wmax = start[b + 1] - start[b];
    mark = (char *)malloc((size_t)(wmax > 0 ? wmax : 1));
    if (!mark) {
        st = RO_E_NOMEM;
        goto done;
    }
    for (int32_t b = 0; b < D; ++b) {
        const int64_t c0 = start[b], c1 = start[b + 1], w = c1 - c0;
        for (int32_t m = 0; m < M; ++m) {
            if (cnt[(size_t)b * M + m] != 0) continue;   /* Alg. 1: the row has an entry in block b */
            const uint64_t i0 = 2 * ((uint64_t)b * (uint64_t)M + (uint64_t)m);
            const int64_t rand_col = c0 + (int64_t)(splitmix64_at(seed, i0) % (uint64_t)w);
            int64_t neigh_col = -1;
            if (kind != RO_CHECK_RANDOM) {
                /* neighbours of m: rows sharing a column with m outside block b */
                memset(cand, 0, (size_t)M);
                for (int64_t e = rowptr[m]; e < rowptr[m + 1]; ++e) {
                    const int64_t n1 = rcol[e];
                    if (n1 >= c0 && n1 < c1) continue;
                    for (int64_t k = colptr[n1]; k < colptr[n1 + 1]; ++k) cand[rowidx[k]] = 1;
                }
                /* candidate columns: block-b columns of the neighbours */
                memset(mark, 0, (size_t)w);
                int64_t count = 0;
                for (int32_t m1 = 0; m1 < M; ++m1) {
                    if (!cand[m1]) continue;
                    for (int64_t e = rowptr[m1]; e < rowptr[m1 + 1]; ++e) {
                        const int64_t n2 = rcol[e];
                        if (n2 >= c0 && n2 < c1 && !mark[n2 - c0]) {
                            mark[n2 - c0] = 1;
                            count += 1;
                        }
                    }
                }
                if (count > 0) {
                    int64_t want = (int64_t)(splitmix64_at(seed, i0 + 1) % (uint64_t)count);
                    for (int64_t c = 0; c < w; ++c) {
                        if (!mark[c]) continue;
                        if (want == 0) {
                            neigh_col = c0 + c;
                            break;
                        }
                        want -= 1;
                    }
                }
            }
            if (kind == RO_CHECK_RANDOM) {
                ins[nins++] = rand_col * M + m;
            } else if (kind == RO_CHECK_NEIGHBOR) {
                ins[nins++] = (neigh_col >= 0 ? neigh_col : rand_col) * M + m;
            } else {
                if (neigh_col >= 0) ins[nins++] = neigh_col * M + m;
                if (neigh_col != rand_col) ins[nins++] = rand_col * M + m;
            }
        }
    }
    /* A' = A plus the inserted ones, column by column, rows ascending */
    qsort(ins, (size_t)nins, sizeof(int64_t), cmp_i64);
    {
        int64_t pos = 0, q = 0;
        colptr_out[0] = 0;
        for (int64_t j = 0; j < N; ++j) {
            int64_t k = colptr[j];
            while (k < colptr[j + 1] || (q < nins && ins[q] / M == j)) {
                const int take_ins = q < nins && ins[q] / M == j &&
                                     (k >= colptr[j + 1] || (int64_t)(ins[q] % M) < (int64_t)rowidx[k]);
                if (take_ins) {
                    rowidx_out[pos] = (int32_t)(ins[q] % M);
                    vals_out[pos] = 1.0;
                    q += 1;
                } else {
                    rowidx_out[pos] = rowidx[k];
                    vals_out[pos] = value_at(vals, dtype, k);
                    k += 1;
                }
                pos += 1;
            }
            colptr_out[j + 1] = (int32_t)pos;
        }
        *nnz_out = pos;
        *inserted = nins;
    }
done:
    free(start);
    free(cnt);
    free(rownnz);
    free(lon);
    free(sgl);
    free(rowptr);
    free(rcol);
    free(fill);
    free(cand);
    free(ins);
    free(mark);
    return st;
}

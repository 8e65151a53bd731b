// k_topk.hip -- the leading eigenpairs of the Gram matrix by Chebyshev-filtered subspace
// iteration in FP64, for k much smaller than M', and the dense FP64 products it runs on.
//
// The proxy SVD of Sec. III needs the k leading singular triplets only, i.e. the k leading
// eigenpairs of G = P P^T.  A block of p > k vectors is
//   - filtered by a Chebyshev polynomial of G that stays small on [0, theta_p] (the unwanted
//     part of the spectrum, theta_p the smallest Ritz value of the block) and grows fast above;
//   - orthonormalised: blocks up to 192 wide by three Cholesky-QR passes in one workgroup
//     each (S = Y^T Y, D = diag(S)^1/2, D^-1 S D^-1 (+ a small shift on the first pass)
//     = L L^T, Y <- Y D^-1 L^-T), wider ones twice by SVQB (D^-1 S D^-1 = V L V^T,
//     Y <- Y D^-1 V L^-1/2);
//   - projected (Rayleigh-Ritz): H = Y^T G Y = Q Theta Q^T, X = Y Q, with the residuals
//     ||G x_i - theta_i x_i|| of the Ritz pairs read back to decide convergence.
// The p x p eigenproblems run on the blocked Jacobi of k_jacobi.hip; the products here are
// 64 x 64 tiles on the FP64 matrix cores (v_mfma_f64_16x16x4f64), split over k where the
// output has few tiles, with the split partials added in split order by a separate pass: no
// floating-point atomics, bitwise reproducible.
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

typedef double tk_d4 __attribute__((ext_vector_type(4)));

constexpr int kTkTile = 64;   // output tile edge
constexpr int kTkK = 16;      // k step (one LDS stage)
constexpr int kTkLd = kTkTile + 2;

// part[z] (rows x cols, row-major) = op(A) B over k in [z klen, min((z + 1) klen, K)).
// op(A) = A (rows x K, ld lda) or, with kTransA, A^T for A stored K x rows (ld lda).  B is
// K x cols (ld ldb).  rows and cols are multiples of 64, klen a multiple of 16.  Rows of a
// plain A at or past a_valid, and k at or past k_valid, read as zero (the Gram has fewer rows
// and columns than the padded blocks).  Each wave owns a 32 x 32 quadrant (2 x 2 blocks of
// 16 x 16); the next k step's tiles are loaded into registers while the current one runs
// on the matrix cores (one barrier per step).
template <bool kTransA>
__global__ __launch_bounds__(256) void k_tk_gemm(const double *__restrict__ A_, int64_t lda,
                                                 const double *__restrict__ B_, int64_t ldb,
                                                 double *__restrict__ part_, int32_t rows, int32_t cols, int32_t K,
                                                 int32_t klen, int32_t a_valid, int32_t k_valid) {
    __shared__ double As[2][kTkK][kTkLd];   // [k][m]
    __shared__ double Bs[2][kTkK][kTkLd];   // [k][n]
    const auto A = gmem(A_);
    const auto B = gmem(B_);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int64_t m0 = (int64_t)blockIdx.x * kTkTile, n0 = (int64_t)blockIdx.y * kTkTile;
    const int32_t kb = blockIdx.z * klen;
    int32_t ke = kb + klen < K ? kb + klen : K;
    const int32_t kv = ke < k_valid ? ke : k_valid;   // k past it reads as zero
    double ra[4], rb[4];
    auto load = [&](int32_t k0) {
        if (!kTransA) {
            const int64_t m = m0 + (tid >> 2);
            const int32_t k = k0 + 4 * (tid & 3);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool ok = m < a_valid && k + q < kv;
                const double v = A[(ok ? m : 0) * lda + (ok ? k + q : 0)];
                ra[q] = ok ? v : 0.0;
            }
        } else {
            const int32_t k = k0 + (tid >> 4);
            const int64_t m = m0 + 4 * (tid & 15);
            const bool ok = k < kv;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double v = A[(int64_t)(ok ? k : 0) * lda + m + q];
                ra[q] = ok ? v : 0.0;
            }
        }
        const int32_t k = k0 + (tid >> 4);
        const int64_t n = n0 + 4 * (tid & 15);
        const bool ok = k < kv;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double v = B[(int64_t)(ok ? k : 0) * ldb + n + q];
            rb[q] = ok ? v : 0.0;
        }
    };
    auto store = [&](int buf) {
        if (!kTransA) {
            const int m = tid >> 2, k = 4 * (tid & 3);
#pragma unroll
            for (int q = 0; q < 4; ++q) As[buf][k + q][m] = ra[q];
        } else {
            const int k = tid >> 4, m = 4 * (tid & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) As[buf][k][m + q] = ra[q];
        }
        const int k = tid >> 4, n = 4 * (tid & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) Bs[buf][k][n + q] = rb[q];
    };
    tk_d4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = tk_d4{0.0, 0.0, 0.0, 0.0};
    const int32_t nsteps = ke > kb ? (ke - kb + kTkK - 1) / kTkK : 0;
    if (nsteps > 0) {
        load(kb);
        store(0);
    }
    __syncthreads();
    for (int32_t s = 0; s < nsteps; ++s) {
        const int buf = s & 1;
        if (s + 1 < nsteps) load(kb + (s + 1) * kTkK);
#pragma unroll
        for (int kk = 0; kk < kTkK / 4; ++kk) {
            const int k = 4 * kk + (l >> 4);
            double a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) a[x] = As[buf][k][32 * wr + 16 * x + (l & 15)];
#pragma unroll
            for (int y = 0; y < 2; ++y) b[y] = Bs[buf][k][32 * wc + 16 * y + (l & 15)];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
        if (s + 1 < nsteps) store(buf ^ 1);
        __syncthreads();
    }
    // result layout: element i of lane l at row l / 16 + 4 i, column l % 16 of a 16 x 16 block
    const auto part = gmem(part_) + (int64_t)blockIdx.z * rows * cols;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t r = m0 + 32 * wr + 16 * x + (l >> 4) + 4 * i;
                const int64_t c = n0 + 32 * wc + 16 * y + (l & 15);
                part[r * cols + c] = acc[x][y][i];
            }
}

// The block products G Y (A = G, plain, rows x K; B = Y, K x P with P = 64 CB the whole block
// width): a workgroup owns 64 rows and all P columns, so each split reads its rows of G once
// (the 64-column tiles above read G once per column tile).  Wave w owns the CB 16-column blocks
// 16 CB w .. of every one of the four 16-row blocks; per k step of 16 it makes 16 CB products
// from 4 + CB operands read from LDS.  Same zero padding (a_valid, k_valid) and split partials
// as k_tk_gemm.
template <int CB>
__global__ __launch_bounds__(256) void k_tk_gemm_wide(const double *__restrict__ A_, int64_t lda,
                                                      const double *__restrict__ B_, int64_t ldb,
                                                      double *__restrict__ part_, int32_t rows, int32_t K,
                                                      int32_t klen, int32_t a_valid, int32_t k_valid) {
    constexpr int P = 64 * CB, BLd = P + 2;
    __shared__ double As[2][kTkK][kTkLd];   // [k][m]
    __shared__ double Bs[2][kTkK][BLd];     // [k][n]
    const auto A = gmem(A_);
    const auto B = gmem(B_);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6, lr = l & 15, lg = l >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * kTkTile;
    const int32_t kb = blockIdx.y * klen;
    const int32_t ke = kb + klen < K ? kb + klen : K;
    const int32_t kv = ke < k_valid ? ke : k_valid;   // k past it reads as zero
    double ra[4], rb[CB][4];
    auto load = [&](int32_t k0) {
        {
            const int64_t m = m0 + (tid >> 2);
            const int32_t k = k0 + 4 * (tid & 3);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool ok = m < a_valid && k + q < kv;
                const double v = A[(ok ? m : 0) * lda + (ok ? k + q : 0)];
                ra[q] = ok ? v : 0.0;
            }
        }
#pragma unroll
        for (int g = 0; g < CB; ++g) {
            const int idx = tid + 256 * g;
            const int32_t k = k0 + idx / (P / 4);
            const int n = 4 * (idx % (P / 4));
            const bool ok = k < kv;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double v = B[(int64_t)(ok ? k : 0) * ldb + n + q];
                rb[g][q] = ok ? v : 0.0;
            }
        }
    };
    auto store = [&](int buf) {
        {
            const int m = tid >> 2, k = 4 * (tid & 3);
#pragma unroll
            for (int q = 0; q < 4; ++q) As[buf][k + q][m] = ra[q];
        }
#pragma unroll
        for (int g = 0; g < CB; ++g) {
            const int idx = tid + 256 * g;
            const int k = idx / (P / 4), n = 4 * (idx % (P / 4));
#pragma unroll
            for (int q = 0; q < 4; ++q) Bs[buf][k][n + q] = rb[g][q];
        }
    };
    tk_d4 acc[4][CB];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < CB; ++y) acc[x][y] = tk_d4{0.0, 0.0, 0.0, 0.0};
    const int32_t nsteps = ke > kb ? (ke - kb + kTkK - 1) / kTkK : 0;
    if (nsteps > 0) {
        load(kb);
        store(0);
    }
    __syncthreads();
    const int c0 = 16 * CB * w;
    for (int32_t st = 0; st < nsteps; ++st) {
        const int buf = st & 1;
        if (st + 1 < nsteps) load(kb + (st + 1) * kTkK);
#pragma unroll
        for (int kk = 0; kk < kTkK / 4; ++kk) {
            const int k = 4 * kk + lg;
            double a[4], b[CB];
#pragma unroll
            for (int x = 0; x < 4; ++x) a[x] = As[buf][k][16 * x + lr];
#pragma unroll
            for (int y = 0; y < CB; ++y) b[y] = Bs[buf][k][c0 + 16 * y + lr];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < CB; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
        if (st + 1 < nsteps) store(buf ^ 1);
        __syncthreads();
    }
    // result layout: element i of lane l at row l / 16 + 4 i, column l % 16 of a 16 x 16 block
    const auto part = gmem(part_) + (int64_t)blockIdx.y * rows * P;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < CB; ++y)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t r = m0 + 16 * x + lg + 4 * i;
                part[r * P + c0 + 16 * y + lr] = acc[x][y][i];
            }
}

// out = alpha (sum over the splits, in split order, of part) + beta E + gamma F, elementwise
// over count entries (E, F may be NULL).  out may not alias part.
__global__ __launch_bounds__(256) void k_tk_combine(const double *__restrict__ part_, int32_t splits, int64_t count,
                                                    double alpha, double beta, const double *__restrict__ E_,
                                                    double gamma, const double *__restrict__ F_,
                                                    double *__restrict__ out_) {
    const auto part = gmem(part_);
    const auto out = gmem(out_);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int32_t s = 0; s < splits; ++s) v += part[(int64_t)s * count + e];
        double o = alpha * v;
        if (E_) o += beta * gmem(E_)[e];
        if (F_) o += gamma * gmem(F_)[e];
        out[e] = o;
    }
}

// 64-bit mixing (the SplitMix64 finaliser) of a counter: the start block's perturbation.
__device__ __forceinline__ double tk_noise(uint64_t c) {
    uint64_t z = c + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-52 - 1.0;   // uniform in [-1, 1)
}

// Start block X (rows x p, ld p): column j is the unit vector of the row with the j-th largest
// diagonal entry of G (ties: lower row first) plus a small fixed perturbation of every
// non-padding entry, so that no direction of the leading eigenspace is missing.  One thread
// per row i: its rank among the n diagonal entries decides which column gets the one.
__global__ __launch_bounds__(256) void k_tk_start(const double *__restrict__ G_, int64_t ldg, int32_t n, int32_t p,
                                                  int32_t rows, double *__restrict__ X_) {
    extern __shared__ double diag[];   // the n diagonal entries, staged once per workgroup
    const auto G = gmem(G_);
    const auto X = gmem(X_);
    for (int32_t j = threadIdx.x; j < n; j += blockDim.x) diag[j] = G[(int64_t)j * ldg + j];
    __syncthreads();
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    int32_t rank = n;
    if (i < n) {
        const double gi = diag[i];
        rank = 0;
        for (int32_t j = 0; j < n; ++j) {
            const double gj = diag[j];
            rank += (gj > gi) || (gj == gi && j < i);
        }
    }
    for (int32_t c = 0; c < p; ++c) {
        double v = 0.0;
        if (i < n) v = (c == rank ? 1.0 : 0.0) + 1e-3 * tk_noise((uint64_t)i * (uint64_t)p + (uint64_t)c);
        X[(int64_t)i * p + c] = v;
    }
}

// Jacobi input from a p x p product src (ld p): dst (ld p) = the symmetric part of src, and
// with dvec != NULL scaled to unit diagonal, dst_ij = s_ij / (d_i d_j), d_i = sqrt(s_ii)
// (written to dvec; a vanishing column gets d_i = 1).
__global__ __launch_bounds__(256) void k_tk_symcopy(const double *__restrict__ src_, int32_t p,
                                                    double *__restrict__ dst_, double *__restrict__ dvec_) {
    const auto src = gmem(src_);
    const auto dst = gmem(dst_);
    const int64_t count = (int64_t)p * p;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(e / p), j = (int32_t)(e % p);
        double v = 0.5 * (src[(int64_t)i * p + j] + src[(int64_t)j * p + i]);
        if (dvec_) {
            const double si = src[(int64_t)i * p + i], sj = src[(int64_t)j * p + j];
            const double di = si > 0.0 ? sqrt(si) : 1.0, dj = sj > 0.0 ? sqrt(sj) : 1.0;
            v = v / (di * dj);
            if (j == 0) gmem(dvec_)[i] = di;
        }
        dst[e] = v;
    }
}

// SVQB transform Wm = D^-1 V L^-1/2 (p x p, ld p) from the eigenpairs (V ld p, L) of the
// scaled S: eigenvalues below eps^2 max(L) are raised to that floor (the direction is kept,
// so the block never loses a column).  One workgroup.
__global__ __launch_bounds__(1024) void k_tk_svqb_w(const double *__restrict__ V_, const double *__restrict__ lam_,
                                                    const double *__restrict__ dvec_, int32_t p,
                                                    double *__restrict__ Wm_) {
    __shared__ double red[1024];
    const auto V = gmem(V_);
    const auto lam = gmem(lam_);
    const auto dvec = gmem(dvec_);
    const auto Wm = gmem(Wm_);
    double m = 0.0;
    for (int32_t j = threadIdx.x; j < p; j += blockDim.x) m = fmax(m, lam[j]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    const double floor = red[0] * 4.930380657631324e-32;   // eps^2 max
    for (int32_t e = threadIdx.x; e < p * p; e += blockDim.x) {
        const int32_t i = e / p, j = e % p;
        const double lj = fmax(lam[j], floor);
        Wm[e] = V[e] / (dvec[i] * sqrt(lj));
    }
}

// Cholesky-QR transform of one workgroup: for S = Y^T Y (p x p, ld p, p = 32 PB) with
// d_i = S_ii^-1/2, S' = diag(d) S diag(d) + shift I = L L^T, write Wm = diag(d) L^-T (upper
// triangular), so that Y Wm has the span of Y and, without shift, orthonormal columns.
//
// L and L^-T come out of one elimination: right-looking Cholesky of the stacked matrix
// [S'; I] (2p x p) turns the lower block into I L^-T.  Column l of the stack has p + 1 live
// entries, the rows 0..l of the lower block (L^-T is upper triangular) and the rows l..p-1
// of the upper block, so it is kept as one virtual column of p + 1 rows: v <= l is row v
// of the lower block, v > l row v - 1 of the upper.  Both blocks of column j then sit at the
// same virtual rows as in any later column, and step j updates column l > j at v <= j and
// v > l.  The (p + 1) x p virtual matrix lives in registers, 32 x 32 threads owning the
// rows v = r (mod 32) and columns l = c (mod 32); step j's column is finished by the 32
// lanes owning it and passed to all through LDS (two buffers, one barrier per step).
// A non-positive or non-finite pivot (or diagonal of S) sets *fail and writes Wm = I.
template <int PB>
__global__ __launch_bounds__(1024) void k_tk_chol(const double *__restrict__ S_, double shift,
                                                  double *__restrict__ Wm_, int32_t *fail) {
    constexpr int p = 32 * PB, VB = PB + 1;
    __shared__ double sc[p];
    __shared__ double col[2][p + 1];
    __shared__ int bad;
    const auto S = gmem(S_);
    const int t = threadIdx.x, c = t >> 5, r = t & 31;
    if (t == 0) bad = 0;
    if (t < p) {
        const double d = S[(int64_t)t * p + t];
        const bool ok = d > 0.0 && d < __builtin_huge_val();
        sc[t] = ok ? 1.0 / sqrt(d) : 0.0;
        if (!ok) bad = 1;
    }
    __syncthreads();
    double a[VB][PB];
#pragma unroll
    for (int vb = 0; vb < VB; ++vb) {
#pragma unroll
        for (int lb = 0; lb < PB; ++lb) {
            const int v = r + 32 * vb, l = c + 32 * lb;
            double x = 0.0;
            if (v <= l) {
                x = v == l ? 1.0 : 0.0;
            } else if (v <= p) {
                const int i = v - 1;
                x = 0.5 * (S[(int64_t)i * p + l] + S[(int64_t)l * p + i]) * sc[i] * sc[l];
                if (i == l) x += shift;
            }
            a[vb][lb] = x;
        }
    }
    const int half = (c & 1) * 32;   // this thread's half of its wave
#pragma unroll
    for (int lb = 0; lb < PB; ++lb) {
        for (int jj = 0; jj < 32; ++jj) {
            const int j = 32 * lb + jj, slot = j & 1;
            if (c == jj) {
                // the pivot sits at virtual row j + 1 of column j
                double pv = jj == 31 ? a[lb + 1][lb] : a[lb][lb];
                pv = __shfl(pv, half + ((jj + 1) & 31), 64);
                if (!(pv > 0.0 && pv < __builtin_huge_val())) {
                    bad = 1;
                    pv = 1.0;
                }
                const double piv = sqrt(pv), inv = 1.0 / piv;
#pragma unroll
                for (int vb = 0; vb < VB; ++vb) {
                    const int v = r + 32 * vb;
                    const double x = v == j + 1 ? piv : a[vb][lb] * inv;
                    a[vb][lb] = x;
                    if (v <= p) col[slot][v] = x;
                }
            }
            __syncthreads();
            // this thread's rows of column j and its columns' entries L(l, j), read once
            double cv[VB], cl[PB];
#pragma unroll
            for (int vb = 0; vb < VB; ++vb) {
                const int v = r + 32 * vb;
                cv[vb] = v <= p ? col[slot][v] : 0.0;
            }
#pragma unroll
            for (int lc = 0; lc < PB; ++lc) cl[lc] = col[slot][c + 32 * lc + 1];
#pragma unroll
            for (int lc = 0; lc < PB; ++lc) {
                const int l = c + 32 * lc;
                if (l > j) {
#pragma unroll
                    for (int vb = 0; vb < VB; ++vb) {
                        const int v = r + 32 * vb;
                        if (v <= j || v > l) a[vb][lc] = fma(-cv[vb], cl[lc], a[vb][lc]);
                    }
                }
            }
        }
    }
    __syncthreads();
    const bool failed = bad != 0;
    const auto Wm = gmem(Wm_);
#pragma unroll
    for (int vb = 0; vb < VB; ++vb) {
#pragma unroll
        for (int lb = 0; lb < PB; ++lb) {
            const int v = r + 32 * vb, l = c + 32 * lb;
            if (v < p) {
                double x = v <= l ? a[vb][lb] * sc[v] : 0.0;
                if (failed) x = v == l ? 1.0 : 0.0;
                Wm[(int64_t)v * p + l] = x;
            }
        }
    }
    if (t == 0 && failed) *fail = 1;
}

// Ritz rotation in descending order: Qs[:, j] = V[:, perm[j]], theta[j] = lam[perm[j]].
__global__ __launch_bounds__(256) void k_tk_permute(const double *__restrict__ V_, const double *__restrict__ lam_,
                                                    const int32_t *__restrict__ perm_, int32_t p,
                                                    double *__restrict__ Qs_, double *__restrict__ theta_) {
    const auto V = gmem(V_);
    const auto perm = gmem(perm_);
    const auto Qs = gmem(Qs_);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)p * p; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(e / p), j = (int32_t)(e % p);
        Qs[e] = V[(int64_t)i * p + perm[j]];
        if (i == 0) gmem(theta_)[j] = gmem(lam_)[perm[j]];
    }
}

// Residual of every Ritz pair: out[p + j] = ||GX[:, j] - theta_j X[:, j]|| over the n rows,
// out[j] = theta_j (out: host-visible memory).  One workgroup per column, rows summed in a
// fixed order.
__global__ __launch_bounds__(256) void k_tk_resid(const double *__restrict__ GX_, const double *__restrict__ X_,
                                                  const double *__restrict__ theta_, int32_t n, int32_t p,
                                                  double *__restrict__ out) {
    __shared__ double red[256];
    const auto GX = gmem(GX_);
    const auto X = gmem(X_);
    const int32_t j = blockIdx.x;
    const double th = gmem(theta_)[j];
    double s = 0.0;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double r = GX[(int64_t)i * p + j] - th * X[(int64_t)i * p + j];
        s = fma(r, r, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[j] = th;
        out[p + j] = sqrt(red[0]);
    }
}

// dst (ld ldd) columns [0, p) = src (rows x p, ld p) for the first `rows` rows.
__global__ __launch_bounds__(256) void k_tk_place(const double *__restrict__ src_, int32_t rows, int32_t p,
                                                  double *__restrict__ dst_, int64_t ldd) {
    const auto src = gmem(src_);
    const auto dst = gmem(dst_);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)rows * p; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / p, j = e % p;
        dst[i * ldd + j] = src[e];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static unsigned tk_grid(int64_t count) {
    int64_t b = (count + 255) / 256;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void launch_tk_gemm(bool trans_a, const double *A, int64_t lda, const double *B, int64_t ldb, double *part,
                    int32_t rows, int32_t cols, int32_t K, int32_t splits, int32_t klen, int32_t a_valid,
                    int32_t k_valid, hipStream_t s) {
    const dim3 grid((unsigned)(rows / kTkTile), (unsigned)(cols / kTkTile), (unsigned)splits);
    if (trans_a)
        hipLaunchKernelGGL(k_tk_gemm<true>, grid, dim3(256), 0, s, A, lda, B, ldb, part, rows, cols, K, klen, a_valid,
                           k_valid);
    else
        hipLaunchKernelGGL(k_tk_gemm<false>, grid, dim3(256), 0, s, A, lda, B, ldb, part, rows, cols, K, klen, a_valid,
                           k_valid);
}

bool launch_tk_gemm_wide(const double *A, int64_t lda, const double *B, int64_t ldb, double *part, int32_t rows,
                         int32_t cols, int32_t K, int32_t splits, int32_t klen, int32_t a_valid, int32_t k_valid,
                         hipStream_t s) {
    const dim3 grid((unsigned)(rows / kTkTile), (unsigned)splits);
    switch (cols) {
    case 64: hipLaunchKernelGGL(k_tk_gemm_wide<1>, grid, dim3(256), 0, s, A, lda, B, ldb, part, rows, K, klen, a_valid, k_valid); return true;
    case 128: hipLaunchKernelGGL(k_tk_gemm_wide<2>, grid, dim3(256), 0, s, A, lda, B, ldb, part, rows, K, klen, a_valid, k_valid); return true;
    case 192: hipLaunchKernelGGL(k_tk_gemm_wide<3>, grid, dim3(256), 0, s, A, lda, B, ldb, part, rows, K, klen, a_valid, k_valid); return true;
    default: return false;
    }
}

void launch_tk_combine(const double *part, int32_t splits, int64_t count, double alpha, double beta, const double *E,
                       double gamma, const double *F, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_tk_combine, dim3(tk_grid(count)), dim3(256), 0, s, part, splits, count, alpha, beta, E, gamma,
                       F, out);
}

void launch_tk_start(const double *G, int64_t ldg, int32_t n, int32_t p, int32_t rows, double *X, hipStream_t s) {
    hipLaunchKernelGGL(k_tk_start, dim3((unsigned)((rows + 255) / 256)), dim3(256), sizeof(double) * (size_t)(n > 0 ? n : 1),
                       s, G, ldg, n, p, rows, X);
}

void launch_tk_symcopy(const double *src, int32_t p, double *dst, double *dvec, hipStream_t s) {
    hipLaunchKernelGGL(k_tk_symcopy, dim3(tk_grid((int64_t)p * p)), dim3(256), 0, s, src, p, dst, dvec);
}

void launch_tk_svqb_w(const double *V, const double *lam, const double *dvec, int32_t p, double *Wm, hipStream_t s) {
    hipLaunchKernelGGL(k_tk_svqb_w, dim3(1), dim3(1024), 0, s, V, lam, dvec, p, Wm);
}

void launch_tk_chol(const double *S, int32_t p, double shift, double *Wm, int32_t *fail, hipStream_t s) {
    switch (p) {
    case 64: hipLaunchKernelGGL(k_tk_chol<2>, dim3(1), dim3(1024), 0, s, S, shift, Wm, fail); break;
    case 128: hipLaunchKernelGGL(k_tk_chol<4>, dim3(1), dim3(1024), 0, s, S, shift, Wm, fail); break;
    case 192: hipLaunchKernelGGL(k_tk_chol<6>, dim3(1), dim3(1024), 0, s, S, shift, Wm, fail); break;
    default: break;
    }
}

void launch_tk_permute(const double *V, const double *lam, const int32_t *perm, int32_t p, double *Qs, double *theta,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_tk_permute, dim3(tk_grid((int64_t)p * p)), dim3(256), 0, s, V, lam, perm, p, Qs, theta);
}

void launch_tk_resid(const double *GX, const double *X, const double *theta, int32_t n, int32_t p, double *out,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_tk_resid, dim3((unsigned)p), dim3(256), 0, s, GX, X, theta, n, p, out);
}

void launch_tk_place(const double *src, int32_t rows, int32_t p, double *dst, int64_t ldd, hipStream_t s) {
    hipLaunchKernelGGL(k_tk_place, dim3(tk_grid((int64_t)rows * p)), dim3(256), 0, s, src, rows, p, dst, ldd);
}

}  // namespace ranky

// k_refine.hip -- one FP64 Rayleigh-Ritz step with the exact operator A A^T.
//
// The mixed-precision path accumulates the Gram matrix in FP32, so its eigenvectors
// U0 carry FP32-size errors.  Projecting the exact operator onto span(U0),
//   H = U0^T (A A^T) U0 = Z^T Z,  Z = A^T U0  (N x k),
// and diagonalising H = Q Theta Q^T gives Ritz pairs U = U0 Q, sigma = sqrt(theta)
// whose values are accurate to second order in U0's error.  Everything here is FP64.
//
// Z is never stored: H = sum over columns j of z_j z_j^T with z_j = sum over column j's
// nonzeros of a_mj U0[m, :].  One workgroup owns one 64 x 64 tile of H and one fixed
// range of columns; per chunk of 16 columns it builds the two 64-wide slices of z_j it
// needs in LDS (U0 is small and stays in L2) and adds their outer products on the FP64
// matrix cores (each wave a 32 x 32 quarter of the tile).  The partial tiles of the
// column ranges are then added in range order: no floating-point atomics, bitwise
// reproducible.
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kRrTile = 64;     // H tile
constexpr int kRrChunk = 16;    // columns per LDS chunk
constexpr int kRrWgs = 2048;    // target workgroups per launch (tiles x column ranges)

// workgroup b -> tile t = b / R (ta <= tb, row-major over the upper triangle), range b % R
template <typename TV>
__global__ __launch_bounds__(256) void k_rr_syrk(const int32_t *__restrict__ colptr, const int32_t *__restrict__ rowidx,
                                                 const TV *__restrict__ vals, int64_t N, int32_t k, int32_t R,
                                                 const double *__restrict__ U0, double *__restrict__ part) {
    __shared__ double ZA[kRrChunk][kRrTile + 1], ZB[kRrChunk][kRrTile + 1];
    const int tid = threadIdx.x, l = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int32_t T = (k + kRrTile - 1) / kRrTile;
    const int32_t t = blockIdx.x / R, r = blockIdx.x % R;
    int32_t ta = 0, rem = t;
    while (rem >= T - ta) {
        rem -= T - ta;
        ++ta;
    }
    const int32_t tb = ta + rem;
    const int64_t c_begin = (N * r) / R, c_end = (N * (r + 1)) / R;
    // LDS build: thread -> column c of the chunk and four entries of each slice
    const int bc = tid >> 4, bq = (tid & 15) * 4;
    const int32_t ia = ta * kRrTile + bq, ib = tb * kRrTile + bq;
    // this wave's quarter of the tile
    const int wa = wave >> 1, wb = wave & 1;
    d4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t c0 = c_begin; c0 < c_end; c0 += kRrChunk) {
        double za[4] = {0.0, 0.0, 0.0, 0.0}, zb[4] = {0.0, 0.0, 0.0, 0.0};
        const int64_t j = c0 + bc;
        if (j < c_end) {
            // four nonzeros per step with independent loads, so their U0 rows are in
            // flight together (the walk is otherwise bound by one gather's latency)
            const int32_t e_end = colptr[j + 1];
            int32_t e = colptr[j];
            for (; e + 4 <= e_end; e += 4) {
                double av[4];
                const double *u[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    av[t] = static_cast<double>(vals[e + t]);
                    u[t] = U0 + (int64_t)rowidx[e + t] * k;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (ia + q < k)
                        za[q] = fma(av[3], u[3][ia + q], fma(av[2], u[2][ia + q],
                                    fma(av[1], u[1][ia + q], fma(av[0], u[0][ia + q], za[q]))));
                    if (ta != tb && ib + q < k)
                        zb[q] = fma(av[3], u[3][ib + q], fma(av[2], u[2][ib + q],
                                    fma(av[1], u[1][ib + q], fma(av[0], u[0][ib + q], zb[q]))));
                }
            }
            for (; e < e_end; ++e) {
                const double av = static_cast<double>(vals[e]);
                const double *u = U0 + (int64_t)rowidx[e] * k;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (ia + q < k) za[q] = fma(av, u[ia + q], za[q]);
                    if (ta != tb && ib + q < k) zb[q] = fma(av, u[ib + q], zb[q]);
                }
            }
            if (ta == tb) {
#pragma unroll
                for (int q = 0; q < 4; ++q) zb[q] = za[q];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ZA[bc][bq + q] = za[q];
            ZB[bc][bq + q] = zb[q];
        }
        __syncthreads();
        // acc += ZA^T ZB over the chunk: A[row][c] = ZA[c][row], B[c][col] = ZB[c][col]
#pragma unroll
        for (int kc = 0; kc < kRrChunk / 4; ++kc) {
            const int c = kc * 4 + (l >> 4);
            const double a0 = ZA[c][32 * wa + (l & 15)], a1 = ZA[c][32 * wa + 16 + (l & 15)];
            const double b0 = ZB[c][32 * wb + (l & 15)], b1 = ZB[c][32 * wb + 16 + (l & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    // result layout: element i of lane l at row l / 16 + 4 i, column l % 16 of a 16 x 16 block
    double *out = part + (int64_t)blockIdx.x * kRrTile * kRrTile;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 32 * wa + 16 * x + (l >> 4) + 4 * i, col = 32 * wb + 16 * y + (l & 15);
                out[row * kRrTile + col] = acc[x][y][i];
            }
}

// H[a][b] = H[b][a] = sum over the column ranges (in order) of the partial tiles; the
// entry (a, b), a <= b, of a diagonal tile is used for both halves.  Zero outside k x k.
__global__ __launch_bounds__(256) void k_rr_syrk_reduce(const double *__restrict__ part, int32_t k, int32_t R,
                                                        int32_t npad, double *__restrict__ H) {
    const int32_t T = (k + kRrTile - 1) / kRrTile;
    const int64_t total = (int64_t)npad * npad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = (int32_t)(e / npad), b = (int32_t)(e % npad);
        if (a > b) continue;
        double v = 0.0;
        if (b < k) {
            const int32_t ta = a / kRrTile, tb = b / kRrTile;
            const int32_t t = ta * T - ta * (ta - 1) / 2 + (tb - ta);
            const double *p = part + ((int64_t)t * R) * kRrTile * kRrTile + (a % kRrTile) * kRrTile + (b % kRrTile);
            for (int32_t r = 0; r < R; ++r) v += p[(int64_t)r * kRrTile * kRrTile];
        }
        H[(int64_t)a * npad + b] = v;
        H[(int64_t)b * npad + a] = v;
    }
}

// U[:, i] = U0 Q[:, perm[i]] with the sign rule (largest-magnitude entry positive,
// lowest row on a tie).  One workgroup per output column; Q's column is staged in LDS.
__global__ __launch_bounds__(256) void k_rr_apply(const double *__restrict__ U0, const double *__restrict__ Q,
                                                  int64_t ldq, const int32_t *__restrict__ perm, int32_t M,
                                                  int32_t k, double *__restrict__ U) {
    extern __shared__ double qcol[];
    __shared__ double best_abs[256];
    __shared__ int32_t best_row[256];
    const int32_t i = blockIdx.x;
    const int32_t c = perm[i];
    for (int32_t t = threadIdx.x; t < k; t += blockDim.x) qcol[t] = Q[(int64_t)t * ldq + c];
    __syncthreads();
    double ba = -1.0;
    int32_t br = 0x7fffffff;
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) {
        double v = 0.0;
        const double *u = U0 + (int64_t)m * k;
        for (int32_t t = 0; t < k; ++t) v = fma(u[t], qcol[t], v);
        U[(int64_t)m * k + i] = v;
        if (fabs(v) > ba) {  // rows visited in increasing order per thread
            ba = fabs(v);
            br = m;
        }
    }
    best_abs[threadIdx.x] = ba;
    best_row[threadIdx.x] = br;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            const double oa = best_abs[threadIdx.x + off];
            const int32_t orow = best_row[threadIdx.x + off];
            if (oa > best_abs[threadIdx.x] || (oa == best_abs[threadIdx.x] && orow < best_row[threadIdx.x])) {
                best_abs[threadIdx.x] = oa;
                best_row[threadIdx.x] = orow;
            }
        }
        __syncthreads();
    }
    const int32_t top = best_row[0];
    __syncthreads();
    if (U[(int64_t)top * k + i] < 0.0)
        for (int32_t m = threadIdx.x; m < M; m += blockDim.x) U[(int64_t)m * k + i] = -U[(int64_t)m * k + i];
}

// ---------------------------------------------------------------------------

int32_t rr_ranges(int64_t N, int32_t k) {
    const int32_t T = (k + kRrTile - 1) / kRrTile;
    const int32_t tiles = T * (T + 1) / 2;
    int64_t R = kRrWgs / tiles;
    const int64_t chunks = (N + kRrChunk - 1) / kRrChunk;
    if (R > chunks) R = chunks;
    if (R < 1) R = 1;
    return (int32_t)R;
}

size_t rr_part_doubles(int64_t N, int32_t k) {
    const int32_t T = (k + kRrTile - 1) / kRrTile;
    return (size_t)(T * (T + 1) / 2) * rr_ranges(N, k) * kRrTile * kRrTile;
}

void launch_rr_h(const CscView &A, int64_t N, int32_t k, const double *U0, double *part, int32_t npad, double *H,
                 hipStream_t s) {
    const int32_t T = (k + kRrTile - 1) / kRrTile;
    const int32_t R = rr_ranges(N, k);
    const unsigned blocks = (unsigned)(T * (T + 1) / 2 * R);
    if (A.dtype == 1)
        hipLaunchKernelGGL(k_rr_syrk<double>, dim3(blocks), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const double *>(A.values), N, k, R, U0, part);
    else
        hipLaunchKernelGGL(k_rr_syrk<float>, dim3(blocks), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const float *>(A.values), N, k, R, U0, part);
    int64_t rb = ((int64_t)npad * npad + 255) / 256;
    if (rb > 4096) rb = 4096;
    hipLaunchKernelGGL(k_rr_syrk_reduce, dim3((unsigned)rb), dim3(256), 0, s, part, k, R, npad, H);
}

void launch_rr_apply(const double *U0, const double *Q, int64_t ldq, const int32_t *perm, int32_t M, int32_t k,
                     double *U, hipStream_t s) {
    hipLaunchKernelGGL(k_rr_apply, dim3((unsigned)k), dim3(256), sizeof(double) * (size_t)k, s, U0, Q, ldq, perm, M,
                       k, U);
}

}  // namespace ranky

// k_select.hip -- rank-safe threshold, ordering and sign convention of the merged
// singular triplets, and the back-projection of the right singular vectors.
//
// After the eigensolve, lambda_i = G_ii.  sigma_i = sqrt(max(lambda_i, 0)); the rank
// is r = #{sigma_i > tau}, tau = max(tol, sqrt(M' u_G)) sigma_1 (squaring in the Gram
// halves the exponent, so below sqrt(M' u_G) sigma_1 a singular value cannot be told
// from zero).  Returned sigma_i for i >= r are exactly 0, and the back-projection
// V = A^T U Sigma^{-1} (Sec. V) fills those columns with zeros instead of dividing.
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

// One workgroup of 1024 threads: bitonic sort of (lambda desc, index asc) over the
// n eigenvalues, then sigma, tau and the rank.  LDS holds npow2 keys and indices.
__global__ __launch_bounds__(1024) void k_select_sort(const MatDesc *__restrict__ descs) {
    extern __shared__ double lds_key[];
    const MatDesc &d = descs[blockIdx.x];
    const double *__restrict__ lam = d.lam;
    const int32_t n = d.n, k = d.k, n_tau = d.n_tau;
    const double tol = d.tol, u_gram = d.u_gram;
    int32_t *__restrict__ perm = d.perm;
    double *__restrict__ sigma = d.sigma;
    int32_t *__restrict__ scal = d.scal;
    double *__restrict__ sdbl = d.sdbl;
    int32_t npow2 = 1;
    while (npow2 < n) npow2 <<= 1;
    int32_t *idx = reinterpret_cast<int32_t *>(lds_key + npow2);
    for (int32_t i = threadIdx.x; i < npow2; i += blockDim.x) {
        lds_key[i] = i < n ? lam[i] : -__builtin_inf();
        idx[i] = i;
    }
    __syncthreads();
    // "a before b" = larger lambda, or equal lambda and smaller index
    for (int32_t size = 2; size <= npow2; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t i = threadIdx.x; i < npow2; i += blockDim.x) {
                const int32_t j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const double ki = lds_key[i], kj = lds_key[j];
                    const int32_t ii = idx[i], ij = idx[j];
                    const bool j_first = (kj > ki) || (kj == ki && ij < ii);
                    if (j_first == up) {
                        lds_key[i] = kj;
                        lds_key[j] = ki;
                        idx[i] = ij;
                        idx[j] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }
    const double s1 = n > 0 ? sqrt(fmax(lds_key[0], 0.0)) : 0.0;
    const double tau = fmax(tol, sqrt((double)n_tau * u_gram)) * s1;
    __shared__ int32_t cnt[1024];
    int32_t c = 0;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) c += sqrt(fmax(lds_key[i], 0.0)) > tau;
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) cnt[threadIdx.x] += cnt[threadIdx.x + off];
        __syncthreads();
    }
    int32_t rank = cnt[0];
    if (rank > k) rank = k;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) perm[i] = idx[i];
    for (int32_t i = threadIdx.x; i < k; i += blockDim.x)
        sigma[i] = (i < rank) ? sqrt(fmax(lds_key[i], 0.0)) : 0.0;
    if (threadIdx.x == 0) {
        scal[kScRank] = rank;
        sdbl[kSdTau] = tau;
        sdbl[kSdSigmaMax] = s1;
    }
}

// One workgroup per output column i: the eigenvector W[:, perm[i]] scattered to the
// non-empty rows with its largest-magnitude entry made positive (lowest row on a
// tie); columns i >= M' are e_row of the empty rows in ascending order.
__global__ __launch_bounds__(256) void k_gather_u(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                  int count) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const double *__restrict__ W = d.W;
    const int64_t ld = d.npad;
    const int32_t n = d.n, M = d.M, k = d.k;
    const int32_t *__restrict__ perm = d.perm;
    const int32_t *__restrict__ m2r = d.m2r;
    const int32_t *__restrict__ empty = d.empty;
    double *__restrict__ U = d.U;
    const int32_t i = blockIdx.x - wp[mat];
    if (i >= n) {
        const int32_t e = empty[i - n];
        for (int32_t m = threadIdx.x; m < M; m += blockDim.x) U[(int64_t)m * k + i] = (m == e) ? 1.0 : 0.0;
        return;
    }
    const int32_t col = perm[i];
    __shared__ double best_abs[256];
    __shared__ int32_t best_row[256];
    double ba = -1.0;
    int32_t br = 0x7fffffff;
    for (int32_t p = threadIdx.x; p < n; p += blockDim.x) {
        const double a = fabs(W[(int64_t)p * ld + col]);
        if (a > ba) {  // rows visited in increasing order per thread: strict > keeps the lowest
            ba = a;
            br = p;
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
    const double sgn = W[(int64_t)best_row[0] * ld + col] < 0.0 ? -1.0 : 1.0;
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) {
        const int32_t p = m2r[m];
        U[(int64_t)m * k + i] = p >= 0 ? sgn * W[(int64_t)p * ld + col] : 0.0;
    }
}

// V[j][i] = (sum over the nonzeros a_mj of column j of a_mj U[m][i]) / sigma[i] for
// i < rank, else 0.  A wave handles one column at a time, over a contiguous run of
// columns; a lane owns two consecutive outputs i, so a wave covers 128 outputs per pass
// with 16-byte U loads.  The column's nonzeros are read once per pass; U rows come
// from L2, and V goes out with non-temporal stores so it does not evict them.
template <typename TV, typename TO>
__device__ void backproject_cols(const int32_t *__restrict__ colptr, const int32_t *__restrict__ rowidx,
                                 const TV *__restrict__ vals, int64_t N, int32_t k, const double *__restrict__ U,
                                 const double *__restrict__ sigma, int32_t rank, TO *__restrict__ V, int64_t wave,
                                 int64_t nwaves) {
    const int lane = threadIdx.x & 63;
    for (int32_t i0 = 0; i0 < k; i0 += 128) {
        const int32_t i = i0 + 2 * lane;
        const bool ok0 = i < k, ok1 = i + 1 < k;
        const double s0 = (ok0 && i < rank) ? sigma[i] : 0.0;
        const double s1 = (ok1 && i + 1 < rank) ? sigma[i + 1] : 0.0;
        const bool live0 = ok0 && i < rank, live1 = ok1 && i + 1 < rank;
        // a contiguous run of columns per wave: each line of colptr / rowidx / values is
        // then read by one wave, hence one XCD's L2 (a stride would pull it into all of them)
        const int64_t per = (N + nwaves - 1) / nwaves;
        const int64_t jb = wave * per, je = jb + per < N ? jb + per : N;
        for (int64_t j = jb; j < je; ++j) {
            const int32_t e0 = colptr[j], e1 = colptr[j + 1];
            double a0 = 0.0, a1 = 0.0;
            int32_t e = e0;
            // four nonzeros per step with independent loads (their U rows in flight together)
            for (; e + 4 <= e1; e += 4) {
                double av[4];
                const double *Um[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    av[t] = static_cast<double>(vals[e + t]);
                    Um[t] = U + (int64_t)rowidx[e + t] * k + i;
                }
                if (ok1) {
                    a0 = fma(av[3], Um[3][0], fma(av[2], Um[2][0], fma(av[1], Um[1][0], fma(av[0], Um[0][0], a0))));
                    a1 = fma(av[3], Um[3][1], fma(av[2], Um[2][1], fma(av[1], Um[1][1], fma(av[0], Um[0][1], a1))));
                } else if (ok0) {
                    a0 = fma(av[3], Um[3][0], fma(av[2], Um[2][0], fma(av[1], Um[1][0], fma(av[0], Um[0][0], a0))));
                }
            }
            for (; e < e1; ++e) {
                const int32_t m = rowidx[e];
                const double a = static_cast<double>(vals[e]);
                const double *Um = U + (int64_t)m * k + i;
                if (ok1) {
                    a0 = fma(a, Um[0], a0);
                    a1 = fma(a, Um[1], a1);
                } else if (ok0) {
                    a0 = fma(a, Um[0], a0);
                }
            }
            const double v0 = live0 ? a0 / s0 : 0.0;
            const double v1 = live1 ? a1 / s1 : 0.0;
            TO *out = V + j * (int64_t)k + i;
            if (ok1 && (k & 1) == 0) {
                // one 2-wide store per lane (i is even and k is even, so it is aligned)
                typedef TO TO2 __attribute__((ext_vector_type(2)));
                const TO2 w = {static_cast<TO>(v0), static_cast<TO>(v1)};
                __builtin_nontemporal_store(w, reinterpret_cast<TO2 *>(out));
            } else if (ok1) {
                __builtin_nontemporal_store(static_cast<TO>(v0), out);
                __builtin_nontemporal_store(static_cast<TO>(v1), out + 1);
            } else if (ok0) {
                __builtin_nontemporal_store(static_cast<TO>(v0), out);
            }
        }
    }
}

// Batched back-projection: matrix `mat` owns workgroups [wp[mat], wp[mat+1]) and its
// waves stride over its columns.
__global__ __launch_bounds__(256) void k_backproject(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                     int count) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int64_t wave = (((int64_t)blockIdx.x - wp[mat]) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)(wp[mat + 1] - wp[mat]) * blockDim.x) >> 6;
    const int32_t rank = d.scal[kScRank];
    if (d.dtype == 1) {
        const double *v = static_cast<const double *>(d.values);
        if (d.v_dtype == 1)
            backproject_cols<double, double>(d.colptr, d.rowidx, v, d.N, d.k, d.U, d.sigma, rank,
                                             static_cast<double *>(d.V), wave, nwaves);
        else
            backproject_cols<double, float>(d.colptr, d.rowidx, v, d.N, d.k, d.U, d.sigma, rank,
                                            static_cast<float *>(d.V), wave, nwaves);
    } else {
        const float *v = static_cast<const float *>(d.values);
        if (d.v_dtype == 1)
            backproject_cols<float, double>(d.colptr, d.rowidx, v, d.N, d.k, d.U, d.sigma, rank,
                                            static_cast<double *>(d.V), wave, nwaves);
        else
            backproject_cols<float, float>(d.colptr, d.rowidx, v, d.N, d.k, d.U, d.sigma, rank,
                                           static_cast<float *>(d.V), wave, nwaves);
    }
}

// Stand-alone back-projection with an explicit device rank (step call).
template <typename TV, typename TO>
__global__ __launch_bounds__(256) void k_backproject_one(const int32_t *__restrict__ colptr,
                                                         const int32_t *__restrict__ rowidx,
                                                         const TV *__restrict__ vals, int64_t N, int32_t k,
                                                         const double *__restrict__ U,
                                                         const double *__restrict__ sigma,
                                                         const int32_t *__restrict__ rank_ptr, TO *__restrict__ V) {
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    backproject_cols<TV, TO>(colptr, rowidx, vals, N, k, U, sigma, *rank_ptr, V, wave, nwaves);
}

// ---------------------------------------------------------------------------

void launch_select(const MatDesc *descs, int count, int32_t max_n, hipStream_t s) {
    int32_t npow2 = 1;
    while (npow2 < max_n) npow2 <<= 1;
    const size_t lds = (sizeof(double) + sizeof(int32_t)) * (size_t)npow2;
    hipLaunchKernelGGL(k_select_sort, dim3((unsigned)count), dim3(1024), lds, s, descs);
}

void launch_gather_u(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_gather_u, dim3((unsigned)nblocks), dim3(256), 0, s, descs, wp, count);
}

int64_t backproject_blocks(int64_t N, int32_t cu_count, int32_t per_cu) {
    int64_t blocks = (N + 3) / 4;
    const int64_t cap = (int64_t)cu_count * (per_cu > 0 ? per_cu : 32);
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    return blocks;
}

void launch_backproject_batch(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_backproject, dim3((unsigned)nblocks), dim3(256), 0, s, descs, wp, count);
}

void launch_backproject(const CscView &A, int64_t N, int32_t k, const double *U, const double *sigma,
                        const int32_t *rank, void *V, int32_t v_dtype, int32_t cu_count, hipStream_t s) {
    const dim3 grid((unsigned)backproject_blocks(N, cu_count)), block(256);
    if (A.dtype == 1) {
        const double *v = static_cast<const double *>(A.values);
        if (v_dtype == 1)
            hipLaunchKernelGGL((k_backproject_one<double, double>), grid, block, 0, s, A.colptr, A.rowidx, v, N, k, U,
                               sigma, rank, static_cast<double *>(V));
        else
            hipLaunchKernelGGL((k_backproject_one<double, float>), grid, block, 0, s, A.colptr, A.rowidx, v, N, k, U,
                               sigma, rank, static_cast<float *>(V));
    } else {
        const float *v = static_cast<const float *>(A.values);
        if (v_dtype == 1)
            hipLaunchKernelGGL((k_backproject_one<float, double>), grid, block, 0, s, A.colptr, A.rowidx, v, N, k, U,
                               sigma, rank, static_cast<double *>(V));
        else
            hipLaunchKernelGGL((k_backproject_one<float, float>), grid, block, 0, s, A.colptr, A.rowidx, v, N, k, U,
                               sigma, rank, static_cast<float *>(V));
    }
}

hipError_t select_set_attributes() {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_select_sort),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)((sizeof(double) + sizeof(int32_t)) * 8192));
}

}  // namespace ranky

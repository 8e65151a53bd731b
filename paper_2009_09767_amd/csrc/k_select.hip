// k_select.hip -- rank-safe threshold, ordering and sign convention of the merged
// singular triplets, and the back-projection of the right singular vectors.
//
// After the eigensolve, lambda_i = G_ii.  sigma_i = sqrt(max(lambda_i, 0)); the rank
// is r = #{sigma_i > tau}, tau = max(tol, sqrt(M' u_G)) sigma_1 (squaring in the Gram
// halves the exponent, so below sqrt(M' u_G) sigma_1 a singular value cannot be told
// from zero).  Returned sigma_i for i >= r are exactly 0, and the back-projection
// V = A^T U Sigma^{-1} (Sec. V) fills those columns with zeros instead of dividing.
#include <type_traits>

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
    // neig eigenpairs were computed (M' for the full Jacobi, the block width for the
    // subspace iteration); the threshold still counts the M' rows
    const int32_t n = d.neig, k = d.k, n_tau = d.n_tau;
    const double tol = d.tol;
    // the split-bf16 tiles run only when the scan found two dense rows or more; otherwise
    // the whole Gram came from the FP32 sparse pass and its roundoff is FP32's
    const double u_gram = (d.dwg > 0 && gmem(d.dense)[1] < 0) ? fmin(d.u_gram, 0x1p-24) : d.u_gram;
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
        for (int32_t m = threadIdx.x; m < M; m += blockDim.x) {
            U[(int64_t)m * k + i] = (m == e) ? 1.0 : 0.0;
            if (d.Uf) d.Uf[(int64_t)m * k + i] = (m == e) ? 1.f : 0.f;
        }
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
        const double u = p >= 0 ? sgn * W[(int64_t)p * ld + col] : 0.0;
        U[(int64_t)m * k + i] = u;
        if (d.Uf) d.Uf[(int64_t)m * k + i] = (float)u;
    }
}

// Lane q's copy of v, a wave-uniform lane index q (an FP64 value as its two halves).
template <typename T>
__device__ inline double readlane_val(T v, int32_t q) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)b, q);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(b >> 32), q);
        return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    } else {
        return static_cast<double>(__builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v), q)));
    }
}

// V[j][i] = (sum over the nonzeros a_mj of column j of a_mj U[m][i]) / sigma[i] for
// i < rank, else 0.  A wave handles one column at a time, over a contiguous run of
// columns whose bounds it loads 64 at a time; a lane owns P pairs of outputs,
// i = i0 + 128 p + 2 lane (P = 1 for k <= 128, 2 for k <= 256, 4 above: one pass over the
// columns covers k <= 512), so every load of a U row and every store of a V row is one
// contiguous 1 KB per wave.  The run's nonzeros are contiguous in the CSC arrays: their row
// indices and values stream through a window of 128 entries in registers (lane t holding
// entries w + t and w + 64 + t), refilled 64 at a time one refill ahead, so a column's only
// wait is on its U rows.  The column's nonzeros are taken four (P = 1) or two at a time with
// independent loads, a step stopping early at the column's end or at the window's 64-entry
// boundary; each output adds them in order, so the sums do not depend on where the steps
// stop.  A nonzero costs three lane reads (row, value), one scalar multiply and one vector
// add before its load, with no branch: the kernel is bound by its instruction issue about as
// much as by its loads.  U rows come from L2, and V goes out with non-temporal stores so it
// does not evict them.
template <typename TV, typename TO, typename TU, int P>
__device__ void backproject_cols(const int32_t *__restrict__ colptr_, const int32_t *__restrict__ rowidx_,
                                 const TV *__restrict__ vals_, int64_t N, int32_t k, const TU *__restrict__ U_,
                                 const double *__restrict__ sigma_, int32_t rank, TO *__restrict__ V_, int64_t wave,
                                 int64_t nwaves) {
    const auto colptr = gmem(colptr_);
    const auto rowidx = gmem(rowidx_);
    const auto vals = gmem(vals_);
    const auto sigma = gmem(sigma_);
    const auto V = gmem(V_);
    constexpr int kNz = P == 1 ? 4 : 2;
    const int lane = threadIdx.x & 63;
    // a contiguous run of columns per wave: each line of colptr / rowidx / values is
    // then read by one wave, hence one XCD's L2 (a stride would pull it into all of them)
    const int64_t per = (N + nwaves - 1) / nwaves;
    const int64_t jb = wave * per, je = jb + per < N ? jb + per : N;
    if (jb >= je) return;
    const int32_t eend = colptr[je];
    for (int32_t i0 = 0; i0 < k; i0 += 128 * P) {
        int32_t i[P];
        bool ok0[P], ok1[P], live0[P], live1[P];
        double s0[P], s1[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            i[p] = i0 + 128 * p + 2 * lane;
            ok0[p] = i[p] < k;
            ok1[p] = i[p] + 1 < k;
            live0[p] = ok0[p] && i[p] < rank;
            live1[p] = ok1[p] && i[p] + 1 < rank;
            s0[p] = live0[p] ? sigma[i[p]] : 0.0;
            s1[p] = live1[p] ? sigma[i[p] + 1] : 0.0;
        }
        // the entry window [w, w + 128)
        int32_t w = colptr[jb];
        int32_t r_lo, r_hi;
        TV v_lo, v_hi;
        auto fill = [&](int32_t at, int32_t &r, TV &v) {
            const int32_t q = at + lane;
            r = q < eend ? rowidx[q] : 0;
            v = q < eend ? vals[q] : TV(0);
        };
        fill(w, r_lo, v_lo);
        fill(w + 64, r_hi, v_hi);
        // entry e (w <= e < w + 64): its value and its U row as a byte offset (M k sizeof(TU) <
        // 2^32 for M <= 8192), so that a load is the 64-bit base in scalars plus a 32-bit offset
        // in a vector register: one scalar multiply per nonzero
        const auto Ub = reinterpret_cast<__attribute__((address_space(1))) const char *>(gmem(U_));
        const uint32_t kb = (uint32_t)k * (uint32_t)sizeof(TU);
        uint32_t ib[P];
#pragma unroll
        for (int p = 0; p < P; ++p) ib[p] = (uint32_t)i[p] * (uint32_t)sizeof(TU);
        auto take = [&](int32_t e, uint32_t &off, double &a) {
            const int32_t q = e - w;
            off = (uint32_t)__builtin_amdgcn_readlane(r_lo, q) * kb;
            a = readlane_val(v_lo, q);
        };
        auto urow = [&](uint32_t off, int p) {
            return reinterpret_cast<__attribute__((address_space(1))) const TU *>(Ub + (off + ib[p]));
        };
        // the step's n <= kNz nonzeros: every U load issued before the first addition
        auto add = [&](double *a0, double *a1, const double *av, const uint32_t *off, int n) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                double ux[kNz], uy[kNz];
                if (ok1[p]) {
#pragma unroll
                    for (int t = 0; t < kNz; ++t) {
                        ux[t] = uy[t] = 0.0;
                        if (t < n) {
                            const auto u = urow(off[t], p);
                            ux[t] = static_cast<double>(u[0]);
                            uy[t] = static_cast<double>(u[1]);
                        }
                    }
                    double x = a0[p], y = a1[p];
#pragma unroll
                    for (int t = 0; t < kNz; ++t) {
                        if (t < n) {
                            x = fma(av[t], ux[t], x);
                            y = fma(av[t], uy[t], y);
                        }
                    }
                    a0[p] = x;
                    a1[p] = y;
                } else if (ok0[p]) {
#pragma unroll
                    for (int t = 0; t < kNz; ++t) {
                        ux[t] = 0.0;
                        if (t < n) ux[t] = static_cast<double>(urow(off[t], p)[0]);
                    }
                    double x = a0[p];
#pragma unroll
                    for (int t = 0; t < kNz; ++t)
                        if (t < n) x = fma(av[t], ux[t], x);
                    a0[p] = x;
                }
            }
        };
        for (int64_t jc = jb; jc < je; jc += 64) {
            // the bounds of the next 64 columns in one load, lane t holding column jc + t's
            // (clamped to the run's last column, so jl + 1 <= N); each column reads its pair
            // from the lanes instead of waiting on its own load
            const int32_t nc = (int32_t)(je - jc < 64 ? je - jc : 64);
            const int64_t jl = jc + (lane < nc ? lane : nc - 1);
            const int32_t cp0 = colptr[jl], cp1 = colptr[jl + 1];
            for (int32_t c = 0; c < nc; ++c) {
                const int64_t j = jc + c;
                const int32_t e0 = __builtin_amdgcn_readlane(cp0, c);
                const int32_t e1 = __builtin_amdgcn_readlane(cp1, c);
                double a0[P], a1[P];
#pragma unroll
                for (int p = 0; p < P; ++p) a0[p] = a1[p] = 0.0;
                for (int32_t e = e0; e < e1;) {
                    // every step ends at w + 64 at the latest, so e <= w + 64 here and one
                    // slide brings e into the low half; a step then takes its entries from the
                    // low half alone (lane q = e - w), which keeps the takes free of branches
                    if (e >= w + 64) {
                        w += 64;
                        r_lo = r_hi;
                        v_lo = v_hi;
                        fill(w + 64, r_hi, v_hi);
                    }
                    const int32_t lim = e1 < w + 64 ? e1 : w + 64;
                    // a step of n nonzeros, n a compile-time constant, so a short step is as
                    // free of branches as a full one
                    auto step = [&](auto nn) {
                        constexpr int n = decltype(nn)::value;
                        double av[kNz];
                        uint32_t off[kNz];
#pragma unroll
                        for (int t = 0; t < kNz; ++t) {
                            off[t] = 0;
                            av[t] = 0.0;
                            if (t < n) take(e + t, off[t], av[t]);
                        }
                        add(a0, a1, av, off, n);
                    };
                    if (e + kNz <= lim) {
                        step(std::integral_constant<int, kNz>{});
                        e += kNz;
                    } else {
                        const int n = lim - e;   // 1 <= n < kNz
                        if (n == 1) step(std::integral_constant<int, 1>{});
                        else if (kNz > 2 && n == 2) step(std::integral_constant<int, (kNz > 2 ? 2 : 1)>{});
                        else if (kNz > 3) step(std::integral_constant<int, (kNz > 3 ? 3 : 1)>{});
                        e = lim;
                    }
                }
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const double v0 = live0[p] ? a0[p] / s0[p] : 0.0;
                    const double v1 = live1[p] ? a1[p] / s1[p] : 0.0;
                    const auto out = V + j * (int64_t)k + i[p];
                    if (ok1[p] && (k & 1) == 0) {
                        // one 2-wide store (i and k are even, so it is aligned)
                        typedef TO TO2 __attribute__((ext_vector_type(2)));
                        const TO2 w2 = {static_cast<TO>(v0), static_cast<TO>(v1)};
                        __builtin_nontemporal_store(
                            w2, reinterpret_cast<__attribute__((address_space(1))) TO2 *>(out));
                    } else if (ok1[p]) {
                        __builtin_nontemporal_store(static_cast<TO>(v0), out);
                        __builtin_nontemporal_store(static_cast<TO>(v1), out + 1);
                    } else if (ok0[p]) {
                        __builtin_nontemporal_store(static_cast<TO>(v0), out);
                    }
                }
            }
        }
    }
}

// Batched back-projection: matrix `mat` owns workgroups [wp[mat], wp[mat+1]) and its
// waves take contiguous runs of its columns.  One launch per number P of output pairs
// per lane; the matrices of other widths own no workgroups in it.
template <int P>
__global__ __launch_bounds__(256) void k_backproject(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                     int count) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    // the wave index is wave-uniform: readfirstlane lets the compiler keep the run in scalars
    const int64_t wave = (((int64_t)blockIdx.x - wp[mat]) * blockDim.x +
                          __builtin_amdgcn_readfirstlane((int32_t)threadIdx.x)) >> 6;
    const int64_t nwaves = ((int64_t)(wp[mat + 1] - wp[mat]) * blockDim.x) >> 6;
    const int32_t rank = d.scal[kScRank];
    // an FP32 V reads the FP32 copy of U (half the bytes per gathered row)
    if (d.dtype == 1) {
        const double *v = static_cast<const double *>(d.values);
        if (d.v_dtype == 1)
            backproject_cols<double, double, double, P>(d.colptr, d.rowidx, v, d.N, d.k, d.U, d.sigma, rank,
                                                        static_cast<double *>(d.V), wave, nwaves);
        else if (d.Uf)
            backproject_cols<double, float, float, P>(d.colptr, d.rowidx, v, d.N, d.k, d.Uf, d.sigma, rank,
                                                      static_cast<float *>(d.V), wave, nwaves);
        else
            backproject_cols<double, float, double, P>(d.colptr, d.rowidx, v, d.N, d.k, d.U, d.sigma, rank,
                                                       static_cast<float *>(d.V), wave, nwaves);
    } else {
        const float *v = static_cast<const float *>(d.values);
        if (d.v_dtype == 1)
            backproject_cols<float, double, double, P>(d.colptr, d.rowidx, v, d.N, d.k, d.U, d.sigma, rank,
                                                       static_cast<double *>(d.V), wave, nwaves);
        else if (d.Uf)
            backproject_cols<float, float, float, P>(d.colptr, d.rowidx, v, d.N, d.k, d.Uf, d.sigma, rank,
                                                     static_cast<float *>(d.V), wave, nwaves);
        else
            backproject_cols<float, float, double, P>(d.colptr, d.rowidx, v, d.N, d.k, d.U, d.sigma, rank,
                                                      static_cast<float *>(d.V), wave, nwaves);
    }
}

// Stand-alone back-projection with an explicit device rank (step call, and the refined
// path's final V).
template <typename TV, typename TO, typename TU, int P>
__global__ __launch_bounds__(256) void k_backproject_one(const int32_t *__restrict__ colptr,
                                                         const int32_t *__restrict__ rowidx,
                                                         const TV *__restrict__ vals, int64_t N, int32_t k,
                                                         const TU *__restrict__ U,
                                                         const double *__restrict__ sigma,
                                                         const int32_t *__restrict__ rank_ptr, TO *__restrict__ V) {
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + __builtin_amdgcn_readfirstlane((int32_t)threadIdx.x)) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    backproject_cols<TV, TO, TU, P>(colptr, rowidx, vals, N, k, U, sigma, *rank_ptr, V, wave, nwaves);
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

void launch_backproject_batch(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, int32_t pairs,
                              hipStream_t s) {
    if (nblocks <= 0) return;
    const dim3 grid((unsigned)nblocks), block(256);
    if (pairs == 4) hipLaunchKernelGGL(k_backproject<4>, grid, block, 0, s, descs, wp, count);
    else if (pairs == 2) hipLaunchKernelGGL(k_backproject<2>, grid, block, 0, s, descs, wp, count);
    else hipLaunchKernelGGL(k_backproject<1>, grid, block, 0, s, descs, wp, count);
}

template <typename TV, int P>
static void launch_one_tv(const CscView &A, const TV *v, int64_t N, int32_t k, const double *U, const float *Uf,
                          const double *sigma, const int32_t *rank, void *V, int32_t v_dtype, dim3 grid,
                          hipStream_t s) {
    const dim3 block(256);
    if (v_dtype == 1)
        hipLaunchKernelGGL((k_backproject_one<TV, double, double, P>), grid, block, 0, s, A.colptr, A.rowidx, v, N, k,
                           U, sigma, rank, static_cast<double *>(V));
    else if (Uf)   // an FP32 V from the FP32 copy of U
        hipLaunchKernelGGL((k_backproject_one<TV, float, float, P>), grid, block, 0, s, A.colptr, A.rowidx, v, N, k,
                           Uf, sigma, rank, static_cast<float *>(V));
    else
        hipLaunchKernelGGL((k_backproject_one<TV, float, double, P>), grid, block, 0, s, A.colptr, A.rowidx, v, N, k,
                           U, sigma, rank, static_cast<float *>(V));
}

template <int P>
static void launch_one(const CscView &A, int64_t N, int32_t k, const double *U, const float *Uf, const double *sigma,
                       const int32_t *rank, void *V, int32_t v_dtype, dim3 grid, hipStream_t s) {
    if (A.dtype == 1)
        launch_one_tv<double, P>(A, static_cast<const double *>(A.values), N, k, U, Uf, sigma, rank, V, v_dtype, grid, s);
    else
        launch_one_tv<float, P>(A, static_cast<const float *>(A.values), N, k, U, Uf, sigma, rank, V, v_dtype, grid, s);
}

void launch_backproject(const CscView &A, int64_t N, int32_t k, const double *U, const float *Uf, const double *sigma,
                        const int32_t *rank, void *V, int32_t v_dtype, int32_t cu_count, hipStream_t s) {
    const dim3 grid((unsigned)backproject_blocks(N, cu_count));
    const int32_t pairs = backproject_pairs(k);
    if (pairs == 4) launch_one<4>(A, N, k, U, Uf, sigma, rank, V, v_dtype, grid, s);
    else if (pairs == 2) launch_one<2>(A, N, k, U, Uf, sigma, rank, V, v_dtype, grid, s);
    else launch_one<1>(A, N, k, U, Uf, sigma, rank, V, v_dtype, grid, s);
}

hipError_t select_set_attributes() {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_select_sort),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)((sizeof(double) + sizeof(int32_t)) * 8192));
}

}  // namespace ranky

// k_refine.hip -- one FP64 Rayleigh-Ritz step with the exact operator A A^T.
//
// The mixed-precision path accumulates the Gram matrix in FP32, so its eigenvectors
// U0 carry FP32-size errors.  Projecting the exact operator onto span(U0),
//   H = U0^T (A A^T) U0 = (A^T U0)^T (A^T U0),
// and diagonalising H = Q Theta Q^T gives Ritz pairs U = U0 Q, sigma = sqrt(theta)
// whose values are accurate to second order in U0's error.  Everything here is FP64:
//   Z = A^T U0            one pass over the CSC (N x k)
//   Y = A Z = (A A^T) U0  row owners over the row-major copy, rows cut into segments
//                         whose partial rows are summed in segment order
//   H = U0^T Y            one thread per entry, fixed-order sum over the rows
// No floating-point atomics; the result is bitwise reproducible.
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

constexpr int kSeg = 2048;  // nonzeros per row segment

// Z[j][i] = sum over column j's nonzeros of a_mj U0[m][i] (wave per column).
template <typename TV>
__global__ __launch_bounds__(256) void k_rr_z(const int32_t *__restrict__ colptr, const int32_t *__restrict__ rowidx,
                                              const TV *__restrict__ vals, int64_t N, int32_t k,
                                              const double *__restrict__ U0, double *__restrict__ Z) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int32_t i0 = 0; i0 < k; i0 += 128) {
        const int32_t i = i0 + 2 * lane;
        const bool ok0 = i < k, ok1 = i + 1 < k;
        for (int64_t j = wave; j < N; j += nwaves) {
            const int32_t e0 = colptr[j], e1 = colptr[j + 1];
            double a0 = 0.0, a1 = 0.0;
            for (int32_t e = e0; e < e1; ++e) {
                const double a = static_cast<double>(vals[e]);
                const double *u = U0 + (int64_t)rowidx[e] * k + i;
                if (ok0) a0 = fma(a, u[0], a0);
                if (ok1) a1 = fma(a, u[1], a1);
            }
            double *z = Z + j * (int64_t)k + i;
            if (ok0) z[0] = a0;
            if (ok1) z[1] = a1;
        }
    }
}

// segment table: seg_ptr[m] = first segment of row m (ceil(rownnz / kSeg) segments per row)
__global__ __launch_bounds__(1024) void k_rr_segments(const int32_t *__restrict__ rownnz, int32_t M,
                                                      int32_t *__restrict__ seg_ptr) {
    __shared__ int32_t part[1024];
    const int32_t per = (M + 1023) / 1024;
    const int32_t m0 = threadIdx.x * per;
    int32_t loc = 0;
    for (int32_t m = m0; m < m0 + per && m < M; ++m) loc += (rownnz[m] + kSeg - 1) / kSeg;
    part[threadIdx.x] = loc;
    __syncthreads();
    for (int32_t off = 1; off < 1024; off <<= 1) {
        int32_t v = (int32_t)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - loc;
    for (int32_t m = m0; m < m0 + per && m < M; ++m) {
        seg_ptr[m] = run;
        run += (rownnz[m] + kSeg - 1) / kSeg;
    }
    if (threadIdx.x == 1023) seg_ptr[M] = part[1023];
}

// One wave per (row, segment): partial[seg][i] = sum over the segment's nonzeros a_mj Z[j][i].
template <typename TV>
__global__ __launch_bounds__(256) void k_rr_rows(const TV *__restrict__ vals, const int32_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ seg_ptr, int32_t M, int32_t k,
                                                 const int32_t *__restrict__ csr_k,
                                                 const int32_t *__restrict__ csr_col, const double *__restrict__ Z,
                                                 double *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int32_t seg = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int32_t nseg = seg_ptr[M];
    if (seg >= nseg) return;
    // row owning this segment: last m with seg_ptr[m] <= seg
    int32_t lo = 0, hi = M - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (seg_ptr[mid] <= seg) lo = mid;
        else hi = mid - 1;
    }
    const int32_t m = lo;
    const int32_t e_begin = rowptr[m] + (seg - seg_ptr[m]) * kSeg;
    const int32_t e_end = min(rowptr[m + 1], e_begin + kSeg);
    for (int32_t i0 = 0; i0 < k; i0 += 128) {
        const int32_t i = i0 + 2 * lane;
        const bool ok0 = i < k, ok1 = i + 1 < k;
        double a0 = 0.0, a1 = 0.0;
        for (int32_t e = e_begin; e < e_end; ++e) {
            const double a = static_cast<double>(vals[csr_k[e]]);
            const double *z = Z + (int64_t)csr_col[e] * k + i;
            if (ok0) a0 = fma(a, z[0], a0);
            if (ok1) a1 = fma(a, z[1], a1);
        }
        double *o = part + (int64_t)seg * k + i;
        if (ok0) o[0] = a0;
        if (ok1) o[1] = a1;
    }
}

// Y[m][i] = sum of row m's segment partials in segment order (zero for empty rows).
__global__ __launch_bounds__(256) void k_rr_reduce(const double *__restrict__ part, const int32_t *__restrict__ seg_ptr,
                                                   int32_t M, int32_t k, double *__restrict__ Y) {
    const int64_t total = (int64_t)M * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t m = (int32_t)(e / k), i = (int32_t)(e % k);
        double v = 0.0;
        for (int32_t s = seg_ptr[m]; s < seg_ptr[m + 1]; ++s) v += part[(int64_t)s * k + i];
        Y[e] = v;
    }
}

// H[a][b] = sum_m U0[m][a] Y[m][b] into an npad x npad buffer (zero outside k x k).
__global__ __launch_bounds__(256) void k_rr_h(const double *__restrict__ U0, const double *__restrict__ Y, int32_t M,
                                              int32_t k, int32_t npad, double *__restrict__ H) {
    const int64_t total = (int64_t)npad * npad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = (int32_t)(e / npad), b = (int32_t)(e % npad);
        double v = 0.0;
        if (a < k && b < k)
            for (int32_t m = 0; m < M; ++m) v = fma(U0[(int64_t)m * k + a], Y[(int64_t)m * k + b], v);
        H[e] = v;
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

void launch_rr_z(const CscView &A, int64_t N, int32_t k, const double *U0, double *Z, int32_t cu_count, hipStream_t s) {
    int64_t blocks = (N + 3) / 4;
    const int64_t cap = (int64_t)cu_count * 32;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    if (A.dtype == 1)
        hipLaunchKernelGGL(k_rr_z<double>, dim3((unsigned)blocks), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const double *>(A.values), N, k, U0, Z);
    else
        hipLaunchKernelGGL(k_rr_z<float>, dim3((unsigned)blocks), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const float *>(A.values), N, k, U0, Z);
}

int64_t rr_max_segments(int32_t M, int64_t nnz) { return nnz / kSeg + M + 1; }

void launch_rr_rows(const CscView &A, const int32_t *rownnz, const int32_t *rowptr, int32_t M, int64_t nnz, int32_t k,
                    const int32_t *csr_k, const int32_t *csr_col, const double *Z, int32_t *seg_ptr, double *part,
                    double *Y, hipStream_t s) {
    hipLaunchKernelGGL(k_rr_segments, dim3(1), dim3(1024), 0, s, rownnz, M, seg_ptr);
    const int64_t maxseg = rr_max_segments(M, nnz);
    const int64_t blocks = (maxseg + 3) / 4;
    if (A.dtype == 1)
        hipLaunchKernelGGL(k_rr_rows<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const double *>(A.values), rowptr, seg_ptr, M, k, csr_k, csr_col, Z, part);
    else
        hipLaunchKernelGGL(k_rr_rows<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const float *>(A.values), rowptr, seg_ptr, M, k, csr_k, csr_col, Z, part);
    int64_t rb = ((int64_t)M * k + 255) / 256;
    if (rb > 4096) rb = 4096;
    hipLaunchKernelGGL(k_rr_reduce, dim3((unsigned)rb), dim3(256), 0, s, part, seg_ptr, M, k, Y);
}

void launch_rr_h(const double *U0, const double *Y, int32_t M, int32_t k, int32_t npad, double *H, hipStream_t s) {
    int64_t b = ((int64_t)npad * npad + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_rr_h, dim3((unsigned)b), dim3(256), 0, s, U0, Y, M, k, npad, H);
}

void launch_rr_apply(const double *U0, const double *Q, int64_t ldq, const int32_t *perm, int32_t M, int32_t k,
                     double *U, hipStream_t s) {
    hipLaunchKernelGGL(k_rr_apply, dim3((unsigned)k), dim3(256), sizeof(double) * (size_t)k, s, U0, Q, ldq, perm, M,
                       k, U);
}

}  // namespace ranky

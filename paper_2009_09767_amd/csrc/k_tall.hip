// k_tall.hip -- the transposed layout for a tall-and-skinny A (M >> N): the CSC of A^T, which is
// the CSR of A.  The short-and-fat path then runs on A^T (N x M), whose column blocks are the row
// blocks of A; its left vectors are A's right vectors and its right vectors A's left vectors.
//
// Any row count M: the row counts are integer atomics (order-free), the row pointers an exclusive
// scan, the entries are placed with per-row atomic cursors (arbitrary order inside a row) and each
// row is then sorted by column -- columns are distinct inside a row, so the result does not
// depend on the order of the atomics.
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

constexpr int kTtScanBlock = 1024;   // entries per workgroup of the scan (256 threads x 4)
constexpr int kTtShort = 64;         // rows up to this length are sorted by one wave in registers
constexpr int kTtLongMax = 8192;     // longest row (the skinny side N is at most the largest M the path takes)

__global__ __launch_bounds__(256) void k_tt_count(const int32_t *__restrict__ rowidx_, int64_t nnz, int64_t M,
                                                  int32_t *__restrict__ counts) {
    const auto rowidx = gmem(rowidx_);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rowidx[e];
        if (r >= 0 && r < M) atomicAdd(&counts[r], 1);   // out-of-range rows (an unvalidated input) are dropped
    }
}

// Exclusive scan of n counts into ptr[0..n] (ptr[n] = total): per-block totals, their scan in one
// workgroup, then the blocks' own scans with their offsets.
__global__ __launch_bounds__(256) void k_tt_scan_blocks(const int32_t *__restrict__ counts, int64_t n,
                                                        int32_t *__restrict__ btot) {
    __shared__ int32_t red[256];
    const int64_t b0 = (int64_t)blockIdx.x * kTtScanBlock;
    int32_t s = 0;
    for (int q = 0; q < 4; ++q) {
        const int64_t i = b0 + 4 * threadIdx.x + q;
        s += i < n ? counts[i] : 0;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) btot[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_tt_scan_totals(int32_t *__restrict__ btot, int64_t nb) {
    __shared__ int32_t carry;
    __shared__ int32_t tmp[1024];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = i < nb ? btot[i] : 0;
        tmp[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
            const int32_t add = (int)threadIdx.x >= off ? tmp[threadIdx.x - off] : 0;
            __syncthreads();
            tmp[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) btot[i] = carry + tmp[threadIdx.x] - v;   // exclusive
        __syncthreads();
        if (threadIdx.x == 1023) carry += tmp[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_tt_scan_apply(const int32_t *__restrict__ counts, int64_t n,
                                                       const int32_t *__restrict__ boff, int32_t *__restrict__ ptr) {
    __shared__ int32_t tmp[256];
    const int64_t b0 = (int64_t)blockIdx.x * kTtScanBlock;
    int32_t v[4], s = 0;
    for (int q = 0; q < 4; ++q) {
        const int64_t i = b0 + 4 * threadIdx.x + q;
        v[q] = i < n ? counts[i] : 0;
        s += v[q];
    }
    tmp[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t add = (int)threadIdx.x >= off ? tmp[threadIdx.x - off] : 0;
        __syncthreads();
        tmp[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = boff[blockIdx.x] + tmp[threadIdx.x] - s;
    for (int q = 0; q < 4; ++q) {
        const int64_t i = b0 + 4 * threadIdx.x + q;
        if (i < n) ptr[i] = run;
        run += v[q];
        if (i == n - 1) ptr[n] = run;
    }
}

// Entry e of column j goes to row rowidx[e]'s next free slot; its column index j becomes the row
// index of A^T.  The column of e is found by binary search over colptr.
template <typename TV>
__global__ __launch_bounds__(256) void k_tt_scatter(const int32_t *__restrict__ colptr_, const int32_t *__restrict__ rowidx_,
                                                    const TV *__restrict__ vals_, int64_t M, int64_t N, int64_t nnz,
                                                    const int32_t *__restrict__ ptr_, int32_t *__restrict__ cursor,
                                                    int32_t *__restrict__ trow_, TV *__restrict__ tval_) {
    const auto colptr = gmem(colptr_);
    const auto rowidx = gmem(rowidx_);
    const auto vals = gmem(vals_);
    const auto ptr = gmem(ptr_);
    const auto trow = gmem(trow_);
    const auto tval = gmem(tval_);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = N - 1;   // last j with colptr[j] <= e
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (colptr[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int32_t r = rowidx[e];
        if (r < 0 || r >= M) continue;   // dropped by the count as well
        const int32_t pos = ptr[r] + atomicAdd(&cursor[r], 1);
        trow[pos] = (int32_t)lo;
        tval[pos] = vals[e];
    }
}

// Rows up to kTtShort entries: one wave per row, a bitonic sort of (column, value) across the lanes;
// longer rows are appended to a list for k_tt_sort_long.
template <typename TV>
__global__ __launch_bounds__(256) void k_tt_sort_short(const int32_t *__restrict__ ptr_, int64_t M,
                                                       int32_t *__restrict__ trow_, TV *__restrict__ tval_,
                                                       int32_t *__restrict__ long_rows, int32_t *__restrict__ nlong) {
    const auto ptr = gmem(ptr_);
    const auto trow = gmem(trow_);
    const auto tval = gmem(tval_);
    const int lane = threadIdx.x & 63;
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (r >= M) return;
    const int32_t b = ptr[r], len = ptr[r + 1] - b;
    if (len <= 1) return;
    if (len > kTtShort) {
        if (lane == 0) long_rows[atomicAdd(nlong, 1)] = (int32_t)r;
        return;
    }
    int32_t key = lane < len ? trow[b + lane] : 0x7fffffff;
    TV val = lane < len ? tval[b + lane] : TV(0);
    for (int size = 2; size <= 64; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int32_t ok = __shfl_xor(key, stride, 64);
            const TV ov = __shfl_xor(val, stride, 64);
            const bool up = (lane & size) == 0;
            const bool lower = (lane & stride) == 0;
            // keep the smaller key in the lower lane of an ascending pair (the larger in a descending one)
            const bool take = lower == up ? ok < key : ok > key;
            if (take) {
                key = ok;
                val = ov;
            }
        }
    }
    if (lane < len) {
        trow[b + lane] = key;
        tval[b + lane] = val;
    }
}

// The long rows of the list, one workgroup each (a loop over the list): bitonic sort in LDS.
template <typename TV>
__global__ __launch_bounds__(1024) void k_tt_sort_long(const int32_t *__restrict__ ptr_, int32_t *__restrict__ trow_,
                                                       TV *__restrict__ tval_, const int32_t *__restrict__ long_rows,
                                                       const int32_t *__restrict__ nlong) {
    __shared__ int32_t key[kTtLongMax];
    __shared__ TV val[kTtLongMax];
    const auto ptr = gmem(ptr_);
    const auto trow = gmem(trow_);
    const auto tval = gmem(tval_);
    const int32_t count = *nlong;
    for (int32_t li = blockIdx.x; li < count; li += gridDim.x) {
        const int32_t r = long_rows[li];
        const int32_t b = ptr[r], len = ptr[r + 1] - b;
        int32_t np2 = 1;
        while (np2 < len) np2 <<= 1;
        for (int32_t i = threadIdx.x; i < np2; i += blockDim.x) {
            key[i] = i < len ? trow[b + i] : 0x7fffffff;
            val[i] = i < len ? tval[b + i] : TV(0);
        }
        __syncthreads();
        for (int32_t size = 2; size <= np2; size <<= 1) {
            for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (int32_t i = threadIdx.x; i < np2; i += blockDim.x) {
                    const int32_t j = i ^ stride;
                    if (j > i) {
                        const bool up = (i & size) == 0;
                        if ((key[i] > key[j]) == up) {
                            const int32_t tk = key[i];
                            key[i] = key[j];
                            key[j] = tk;
                            const TV tv = val[i];
                            val[i] = val[j];
                            val[j] = tv;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int32_t i = threadIdx.x; i < len; i += blockDim.x) {
            trow[b + i] = key[i];
            tval[b + i] = val[i];
        }
        __syncthreads();
    }
}

// The CSC contract of a matrix with any row count, checked before the transpose: colptr starts at
// 0, never decreases and ends at nnz; each column's rows are in [0, M) and strictly increasing;
// values finite.  Status bits as the scan's (kStCsc, kStNonfinite).  One workgroup per column (a
// loop over the columns), its entries split over the threads.
template <typename TV>
__global__ __launch_bounds__(256) void k_tt_validate(const int32_t *__restrict__ colptr_, const int32_t *__restrict__ rowidx_,
                                                     const TV *__restrict__ vals_, int64_t M, int64_t N, int64_t nnz,
                                                     int32_t *__restrict__ status) {
    const auto colptr = gmem(colptr_);
    const auto rowidx = gmem(rowidx_);
    const auto vals = gmem(vals_);
    int32_t bits = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && (colptr[0] != 0 || (int64_t)colptr[N] != nnz)) bits |= kStCsc;
    for (int64_t j = blockIdx.x; j < N; j += gridDim.x) {
        const int64_t b = colptr[j], e = colptr[j + 1];
        if (e < b || b < 0 || e > nnz) {
            bits |= kStCsc;
            continue;
        }
        for (int64_t x = b + threadIdx.x; x < e; x += blockDim.x) {
            const int32_t r = rowidx[x];
            if (r < 0 || r >= M || (x + 1 < e && rowidx[x + 1] <= r)) bits |= kStCsc;
            if (!finite_value(vals[x])) bits |= kStNonfinite;
        }
    }
    if (bits) atomicOr(status, bits);
}

// ---------------------------------------------------------------------------

int64_t tall_scan_blocks(int64_t n) { return (n + kTtScanBlock - 1) / kTtScanBlock; }

void launch_exclusive_scan(const int32_t *counts, int64_t n, int32_t *btot, int32_t *ptr, hipStream_t s) {
    const int64_t nb = tall_scan_blocks(n);
    hipLaunchKernelGGL(k_tt_scan_blocks, dim3((unsigned)nb), dim3(256), 0, s, counts, n, btot);
    hipLaunchKernelGGL(k_tt_scan_totals, dim3(1), dim3(1024), 0, s, btot, nb);
    hipLaunchKernelGGL(k_tt_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, counts, n, btot, ptr);
}

template <typename TV>
static void sort_segments(const int32_t *ptr, int64_t nseg, int32_t *keys, TV *vals, int32_t *long_rows,
                          int32_t *nlong, hipStream_t s) {
    launch_fill_i32(nlong, 1, 0, s);
    const unsigned grid = (unsigned)((nseg * 64 + 255) / 256);
    hipLaunchKernelGGL(k_tt_sort_short<TV>, dim3(grid), dim3(256), 0, s, ptr, nseg, keys, vals, long_rows, nlong);
    hipLaunchKernelGGL(k_tt_sort_long<TV>, dim3(1024), dim3(1024), 0, s, ptr, keys, vals, long_rows, nlong);
}

void launch_sort_segments(const int32_t *ptr, int64_t nseg, int32_t *keys, double *vals, int32_t *long_rows,
                          int32_t *nlong, hipStream_t s) {
    if (nseg > 0) sort_segments<double>(ptr, nseg, keys, vals, long_rows, nlong, s);
}

void launch_transpose_csc(const CscView &A, int64_t M, int64_t N, int32_t *counts, int32_t *btot, int32_t *ptr,
                          int32_t *cursor, int32_t *long_rows, int32_t *nlong, int32_t *trow, void *tval,
                          hipStream_t s) {
    const int64_t nnz = A.nnz;
    launch_fill_i32(counts, M, 0, s);
    launch_fill_i32(cursor, M, 0, s);
    auto grid = [](int64_t n) {
        int64_t b = (n + 255) / 256;
        if (b > 16384) b = 16384;
        if (b < 1) b = 1;
        return (unsigned)b;
    };
    if (nnz > 0) hipLaunchKernelGGL(k_tt_count, dim3(grid(nnz)), dim3(256), 0, s, A.rowidx, nnz, M, counts);
    launch_exclusive_scan(counts, M, btot, ptr, s);
    if (nnz == 0) return;
    if (A.dtype == 1) {
        hipLaunchKernelGGL(k_tt_scatter<double>, dim3(grid(nnz)), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const double *>(A.values), M, N, nnz, ptr, cursor, trow, static_cast<double *>(tval));
        sort_segments<double>(ptr, M, trow, static_cast<double *>(tval), long_rows, nlong, s);
    } else {
        hipLaunchKernelGGL(k_tt_scatter<float>, dim3(grid(nnz)), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const float *>(A.values), M, N, nnz, ptr, cursor, trow, static_cast<float *>(tval));
        sort_segments<float>(ptr, M, trow, static_cast<float *>(tval), long_rows, nlong, s);
    }
}

void launch_validate_csc(const CscView &A, int64_t M, int64_t N, int32_t *status, hipStream_t s) {
    launch_fill_i32(status, 1, 0, s);
    const unsigned g = (unsigned)(N < 4096 ? N : 4096);
    if (A.nnz == 0) {
        hipLaunchKernelGGL(k_tt_validate<double>, dim3(g), dim3(256), 0, s, A.colptr, A.rowidx, (const double *)nullptr,
                           M, N, (int64_t)0, status);
    } else if (A.dtype == 1) {
        hipLaunchKernelGGL(k_tt_validate<double>, dim3(g), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const double *>(A.values), M, N, A.nnz, status);
    } else {
        hipLaunchKernelGGL(k_tt_validate<float>, dim3(g), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const float *>(A.values), M, N, A.nnz, status);
    }
}

}  // namespace ranky

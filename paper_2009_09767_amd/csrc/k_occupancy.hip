// k_occupancy.hip -- the Alg. 1 scan of every column block, the CSC contract
// check, the structural rank (empty rows) and the stable row-major copy of A.
//
// Alg. 1 asks, for every block d and row m, whether row m has any nonzero inside
// block d (a "lonely node" if not).  Here that scan is a histogram: one pass over
// the CSC counts, per column chunk, the nonzeros of every row; summing the chunks
// of a block gives the per-(block,row) occupancy, from which the lonely rows (count
// 0) and the rows with one entry (NO of Eq. 4) of each block are counted.  Nothing
// is repaired: a lonely row only means a zero singular value of that block.
//
// The same counts give the offsets of a stable counting sort of the nonzeros by
// row (column order kept inside a row), used by the Gram pass.
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f64(double *__restrict__ p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// One workgroup per column chunk: validate every column of the chunk and count
// its nonzeros per row in LDS; write the chunk's row histogram.  Reads are
// bounded by the colptr checks, so a malformed CSC only sets status bits.
template <typename TV>
__global__ __launch_bounds__(256) void k_occ_chunks(const int32_t *__restrict__ colptr,
                                                    const int32_t *__restrict__ rowidx,
                                                    const TV *__restrict__ vals, int32_t M, int64_t N, int64_t nnz,
                                                    int32_t D, int32_t cpb, int32_t validate,
                                                    int32_t *__restrict__ hist, int32_t *__restrict__ scal) {
    extern __shared__ int32_t lds_hist[];
    const int64_t c = blockIdx.x;
    int64_t c0, c1;
    chunk_columns(c, cpb, N, D, c0, c1);
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) lds_hist[m] = 0;
    __syncthreads();
    int32_t err = 0;
    for (int64_t j = c0 + threadIdx.x; j < c1; j += blockDim.x) {
        const int64_t e0 = colptr[j], e1 = colptr[j + 1];
        if (e0 < 0 || e1 < e0 || e1 > nnz) {
            err |= kStCsc;
            continue;
        }
        int32_t prev = -1;
        for (int64_t e = e0; e < e1; ++e) {
            const int32_t r = rowidx[e];
            if (r < 0 || r >= M) {
                err |= kStCsc;
                continue;
            }
            if (r <= prev) err |= kStCsc;
            prev = r;
            atomicAdd(&lds_hist[r], 1);
            if (validate && !finite_value(vals[e])) err |= kStNonfinite;
        }
    }
    if (threadIdx.x == 0) {
        if (c0 == 0 && c1 > 0 && colptr[0] != 0) err |= kStCsc;
        if (c1 == N && c0 < c1 && (int64_t)colptr[N] != nnz) err |= kStCsc;
    }
    if (err) atomicOr(&scal[kScStatus], err);
    __syncthreads();
    int32_t *out = hist + c * (int64_t)M;
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) out[m] = lds_hist[m];
}

// One thread per row: per-block occupancy (sum of the block's chunk histograms),
// lonely / single-entry row counts per block, and the row's total.
__global__ __launch_bounds__(256) void k_occ_rows(const int32_t *__restrict__ hist, int32_t M, int32_t D, int32_t cpb,
                                                  int32_t *__restrict__ rownnz, int32_t *__restrict__ cnt,
                                                  int32_t *__restrict__ lonely, int32_t *__restrict__ single) {
    const int32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = m < M;
    const int lane = threadIdx.x & 63;
    int32_t total = 0;
    for (int32_t b = 0; b < D; ++b) {
        int32_t cb = 0;
        if (valid)
            for (int32_t t = 0; t < cpb; ++t) cb += hist[((int64_t)b * cpb + t) * M + m];
        if (valid && cnt) cnt[(int64_t)b * M + m] = cb;
        total += cb;
        const uint64_t z = __ballot(valid && cb == 0);
        const uint64_t s = __ballot(valid && cb == 1);
        if (lane == 0) {
            if (z) atomicAdd(&lonely[b], __popcll(z));
            if (s) atomicAdd(&single[b], __popcll(s));
        }
    }
    if (valid) rownnz[m] = total;
}

// One workgroup of 1024 threads: exclusive scan of the row counts (row pointers of
// the row-major copy) and the compaction maps of the non-empty rows.
//   m2r[m] = position of row m among the non-empty rows, or -1
//   r2m[i] = the i-th non-empty row;  empty[e] = the e-th empty row (ascending)
__global__ __launch_bounds__(1024) void k_occ_scan(const int32_t *__restrict__ rownnz, int32_t M,
                                                   int32_t *__restrict__ rowptr, int32_t *__restrict__ m2r,
                                                   int32_t *__restrict__ r2m, int32_t *__restrict__ empty,
                                                   int32_t *__restrict__ scal) {
    __shared__ int64_t s_nnz[1024];
    __shared__ int32_t s_ne[1024];
    const int32_t per = (M + 1023) / 1024;
    const int32_t m0 = threadIdx.x * per;
    int64_t loc_nnz = 0;
    int32_t loc_ne = 0;
    for (int32_t m = m0; m < m0 + per && m < M; ++m) {
        loc_nnz += rownnz[m];
        loc_ne += rownnz[m] > 0;
    }
    s_nnz[threadIdx.x] = loc_nnz;
    s_ne[threadIdx.x] = loc_ne;
    __syncthreads();
    // Hillis-Steele inclusive scan (fixed order; integers)
    for (int32_t off = 1; off < 1024; off <<= 1) {
        int64_t a = 0;
        int32_t b = 0;
        if ((int32_t)threadIdx.x >= off) {
            a = s_nnz[threadIdx.x - off];
            b = s_ne[threadIdx.x - off];
        }
        __syncthreads();
        s_nnz[threadIdx.x] += a;
        s_ne[threadIdx.x] += b;
        __syncthreads();
    }
    int64_t run = s_nnz[threadIdx.x] - loc_nnz;
    int32_t nr = s_ne[threadIdx.x] - loc_ne;
    for (int32_t m = m0; m < m0 + per && m < M; ++m) {
        rowptr[m] = (int32_t)run;
        run += rownnz[m];
        if (rownnz[m] > 0) {
            m2r[m] = nr;
            r2m[nr] = m;
            ++nr;
        } else {
            m2r[m] = -1;
            empty[m - nr] = m;
        }
    }
    if (threadIdx.x == 1023) {
        rowptr[M] = (int32_t)s_nnz[1023];
        scal[kScNonempty] = s_ne[1023];
    }
}

// One thread per row: turn the chunk histograms into the start offset of every
// (chunk, row) run in the row-major copy (row pointer + earlier chunks), in place.
__global__ __launch_bounds__(256) void k_occ_offsets(int32_t *__restrict__ hist, const int32_t *__restrict__ rowptr,
                                                     int32_t M, int64_t nchunks) {
    const int32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    int32_t run = rowptr[m];
    for (int64_t c = 0; c < nchunks; ++c) {
        const int32_t h = hist[c * M + m];
        hist[c * M + m] = run;
        run += h;
    }
}

// Stable transpose: one wave per chunk, 64 columns at a time (lane = column).
// A row occurs at most once per column, so the rank of an entry among the entries
// of its row inside these 64 columns is the number of lower lanes holding that row:
// lanes publish themselves in a per-row 64-bit mask (bitwise OR commutes, so the
// mask does not depend on timing), read it back and count.  The entry's slot is
// the row's running offset plus that rank; the lowest lane then advances the offset.
// csr_k[slot] = CSC position of the entry, csr_end[slot] = end of its column,
// csr_col[slot] = its column.
__global__ __launch_bounds__(64) void k_transpose(const int32_t *__restrict__ colptr,
                                                  const int32_t *__restrict__ rowidx, int32_t M, int64_t N,
                                                  int32_t D, int32_t cpb, const int32_t *__restrict__ offs,
                                                  int32_t *__restrict__ csr_k, int32_t *__restrict__ csr_end,
                                                  int32_t *__restrict__ csr_col) {
    extern __shared__ uint64_t lds_mask[];
    int32_t *ctr = reinterpret_cast<int32_t *>(lds_mask + M);
    const int64_t c = blockIdx.x;
    int64_t c0, c1;
    chunk_columns(c, cpb, N, D, c0, c1);
    const int32_t *off = offs + c * (int64_t)M;
    for (int32_t m = threadIdx.x; m < M; m += 64) {
        lds_mask[m] = 0;
        ctr[m] = off[m];
    }
    __syncthreads();
    const int lane = threadIdx.x;
    const uint64_t bit = 1ull << lane;
    const uint64_t lower = bit - 1;
    for (int64_t g = c0; g < c1; g += 64) {
        const int64_t j = g + lane;
        int32_t e0 = 0, e1 = 0;
        if (j < c1) {
            e0 = colptr[j];
            e1 = colptr[j + 1];
        }
        for (int32_t e = e0; e < e1; ++e) atomicOr(reinterpret_cast<unsigned long long *>(&lds_mask[rowidx[e]]), bit);
        __syncthreads();
        for (int32_t e = e0; e < e1; ++e) {
            const int32_t r = rowidx[e];
            const int32_t slot = ctr[r] + __popcll(lds_mask[r] & lower);
            csr_k[slot] = e;
            csr_end[slot] = e1;
            csr_col[slot] = (int32_t)j;
        }
        __syncthreads();
        for (int32_t e = e0; e < e1; ++e) {
            const int32_t r = rowidx[e];
            const uint64_t mk = lds_mask[r];
            if ((mk & lower) == 0) ctr[r] += __popcll(mk);
        }
        __syncthreads();
        for (int32_t e = e0; e < e1; ++e) lds_mask[rowidx[e]] = 0;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

void launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

void launch_occupancy(const CscView &A, int32_t M, int64_t N, int32_t D, int32_t cpb, int64_t nchunks,
                      int32_t validate, int32_t *hist, int32_t *rownnz, int32_t *cnt, int32_t *lonely,
                      int32_t *single, int32_t *rowptr, int32_t *m2r, int32_t *r2m, int32_t *empty,
                      int32_t *scal, hipStream_t s) {
    const size_t lds = sizeof(int32_t) * (size_t)M;
    if (A.dtype == 1)
        hipLaunchKernelGGL(k_occ_chunks<double>, dim3((unsigned)nchunks), dim3(256), lds, s, A.colptr, A.rowidx,
                           static_cast<const double *>(A.values), M, N, A.nnz, D, cpb, validate, hist, scal);
    else
        hipLaunchKernelGGL(k_occ_chunks<float>, dim3((unsigned)nchunks), dim3(256), lds, s, A.colptr, A.rowidx,
                           static_cast<const float *>(A.values), M, N, A.nnz, D, cpb, validate, hist, scal);
    hipLaunchKernelGGL(k_occ_rows, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, hist, M, D, cpb, rownnz, cnt,
                       lonely, single);
    hipLaunchKernelGGL(k_occ_scan, dim3(1), dim3(1024), 0, s, rownnz, M, rowptr, m2r, r2m, empty, scal);
}

void launch_row_offsets(int32_t *hist, const int32_t *rowptr, int32_t M, int64_t nchunks, hipStream_t s) {
    hipLaunchKernelGGL(k_occ_offsets, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, hist, rowptr, M, nchunks);
}

void launch_transpose(const CscView &A, int32_t M, int64_t N, int32_t D, int32_t cpb, int64_t nchunks,
                      const int32_t *offs, int32_t *csr_k, int32_t *csr_end, int32_t *csr_col, hipStream_t s) {
    const size_t lds = (sizeof(uint64_t) + sizeof(int32_t)) * (size_t)M;
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)nchunks), dim3(64), lds, s, A.colptr, A.rowidx, M, N, D, cpb, offs,
                       csr_k, csr_end, csr_col);
}

size_t transpose_lds_bytes(int32_t M) { return (sizeof(uint64_t) + sizeof(int32_t)) * (size_t)M; }

hipError_t occupancy_set_attributes(int32_t maxM) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_transpose),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)transpose_lds_bytes(maxM));
    return e;
}

}  // namespace ranky

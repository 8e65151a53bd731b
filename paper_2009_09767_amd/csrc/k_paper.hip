// k_paper.hip -- the paper's own procedure, for comparison with the Gram-form path:
//   - the checkers of Alg. 2-4 (RandomChecker, NeighborChecker, NeighborRandomChecker), which give
//     every row at least one entry inside every block of a copy A' of A;
//   - the proxy matrix P = [U^1 S^1 | ... | U^D S^D] of Eq. 1 from the blocks' own factors, and
//     its Gram P P^T (Eq. 3), whose eigenpairs are the SVD of P (Sec. III, last step of Alg. 1);
//   - the paper's error sums e_sigma and e_u (Sec. IV).
// Every decision of a checker reads the unmodified A; its random draws come from a counter-based
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): draw i of seed s is the generator's mixing
// function applied to s + (i + 1) * 0x9E3779B97F4A7C15.
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

__device__ __forceinline__ uint64_t pp_draw(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One workgroup per (block b, row m): nothing unless row m has no entry inside block b.  Writes
// the (at most two) new entries as col * M + m into ins[2 (b M + m) + {0, 1}], -1 for none.
//   kind 0 (Alg. 2): column c0 + (draw 2i mod width)
//   kind 1 (Alg. 3): the neighbours of m are the rows sharing a column with m outside block b
//     (an LDS bit set over the M rows); the candidate columns are the block-b columns of the
//     neighbours (an LDS bit set over the block's columns); the choice is the
//     (draw 2i+1 mod count)-th candidate in ascending order, the kind-0 column when there is none
//   kind 2 (Alg. 4): both (the second dropped when they coincide)
// rowptr / csr_col: the rows of A (columns ascending inside a row), from the transpose.
__global__ __launch_bounds__(256) void k_checker(const int32_t *__restrict__ colptr_, const int32_t *__restrict__ rowidx_,
                                                 int32_t M, int64_t N, int32_t D, const int32_t *__restrict__ cnt_,
                                                 const int32_t *__restrict__ rowptr_, const int32_t *__restrict__ csr_col_,
                                                 int32_t kind, uint64_t seed, int64_t *__restrict__ ins) {
    extern __shared__ uint32_t pp_bits[];
    __shared__ uint32_t wsum[256];
    __shared__ int64_t chosen;
    const auto colptr = gmem(colptr_);
    const auto rowidx = gmem(rowidx_);
    const auto rowptr = gmem(rowptr_);
    const auto csr_col = gmem(csr_col_);
    const int64_t pair = blockIdx.x;
    const int32_t b = (int32_t)(pair / M), m = (int32_t)(pair % M);
    const int tid = threadIdx.x;
    int64_t *out = ins + 2 * pair;
    if (gmem(cnt_)[pair] != 0) {   // cnt is [D x M]: pair = b M + m
        if (tid == 0) out[0] = out[1] = -1;
        return;
    }
    const int64_t c0 = ((int64_t)b * N) / D, c1 = ((int64_t)(b + 1) * N) / D, w = c1 - c0;
    const uint64_t i0 = 2 * (uint64_t)pair;
    const int64_t rand_col = c0 + (int64_t)(pp_draw(seed, i0) % (uint64_t)w);
    if (kind == 0) {
        if (tid == 0) {
            out[0] = rand_col * M + m;
            out[1] = -1;
        }
        return;
    }
    const int32_t mw = (M + 31) / 32;
    const int64_t ww = (w + 31) / 32;
    uint32_t *cand = pp_bits;          // M bits
    uint32_t *cmask = pp_bits + mw;    // w bits
    for (int32_t x = tid; x < mw; x += blockDim.x) cand[x] = 0u;
    for (int64_t x = tid; x < ww; x += blockDim.x) cmask[x] = 0u;
    if (tid == 0) chosen = -1;
    __syncthreads();
    // neighbours: rows of the columns of row m outside block b
    for (int32_t e = rowptr[m] + tid; e < rowptr[m + 1]; e += blockDim.x) {
        const int32_t n1 = csr_col[e];
        if (n1 >= c0 && n1 < c1) continue;
        for (int32_t x = colptr[n1]; x < colptr[n1 + 1]; ++x) {
            const int32_t r = rowidx[x];
            atomicOr(&cand[r >> 5], 1u << (r & 31));
        }
    }
    __syncthreads();
    // candidate columns: the block-b entries of every neighbour (its row's entries from the
    // first column >= c0, found by binary search)
    for (int32_t r = tid; r < M; r += blockDim.x) {
        if (!(cand[r >> 5] & (1u << (r & 31)))) continue;
        int32_t lo = rowptr[r], hi = rowptr[r + 1];
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (csr_col[mid] < c0) lo = mid + 1;
            else hi = mid;
        }
        for (int32_t e = lo; e < rowptr[r + 1]; ++e) {
            const int64_t c = csr_col[e];
            if (c >= c1) break;
            const int64_t o = c - c0;
            atomicOr(&cmask[o >> 5], 1u << (o & 31));
        }
    }
    __syncthreads();
    // count the candidates: each thread owns a contiguous run of words; scan the runs' counts
    const int64_t per = (ww + blockDim.x - 1) / blockDim.x;
    const int64_t x0 = tid * per, x1 = x0 + per < ww ? x0 + per : ww;
    uint32_t mine = 0;
    for (int64_t x = x0; x < x1; ++x) mine += __popc(cmask[x]);
    wsum[tid] = mine;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {   // inclusive scan of the run counts
        const uint32_t add = tid >= off ? wsum[tid - off] : 0u;
        __syncthreads();
        wsum[tid] += add;
        __syncthreads();
    }
    const uint32_t total = wsum[255];
    if (total > 0) {
        const uint64_t want = pp_draw(seed, i0 + 1) % total;
        const uint32_t before = wsum[tid] - mine;
        if (want >= before && want < before + mine) {   // exactly one thread holds it
            uint64_t left = want - before;
            for (int64_t x = x0; x < x1; ++x) {
                uint32_t v = cmask[x];
                const uint32_t pc = __popc(v);
                if (left >= pc) {
                    left -= pc;
                    continue;
                }
                for (;;) {   // the (left)-th set bit of v
                    const int bit = __ffs(v) - 1;
                    if (left == 0) {
                        chosen = c0 + x * 32 + bit;
                        break;
                    }
                    v &= v - 1;
                    --left;
                }
                break;
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int64_t nc = chosen;
        if (kind == 1) {
            out[0] = (nc >= 0 ? nc : rand_col) * M + m;
            out[1] = -1;
        } else {
            out[0] = nc >= 0 ? nc * M + m : -1;
            out[1] = nc != rand_col ? rand_col * M + m : -1;
        }
    }
}

// counts[col] += 1 for every new entry
__global__ __launch_bounds__(256) void k_pp_count(const int64_t *__restrict__ ins, int64_t n, int32_t M,
                                                  int32_t *__restrict__ counts) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = ins[e];
        if (v >= 0) atomicAdd(&counts[v / M], 1);
    }
}

// Each new entry's row into its column's slots (arbitrary order inside a column; sorted after).
__global__ __launch_bounds__(256) void k_pp_place(const int64_t *__restrict__ ins, int64_t n, int32_t M,
                                                  const int32_t *__restrict__ iptr, int32_t *__restrict__ cursor,
                                                  int32_t *__restrict__ irow) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = ins[e];
        if (v < 0) continue;
        const int64_t col = v / M;
        irow[iptr[col] + atomicAdd(&cursor[col], 1)] = (int32_t)(v % M);
    }
}

// A' column j = A's column j merged with its new rows (sorted), FP64 values, new ones = 1.
template <typename TV>
__global__ __launch_bounds__(256) void k_pp_merge(const int32_t *__restrict__ colptr_, const int32_t *__restrict__ rowidx_,
                                                  const TV *__restrict__ vals_, int64_t N,
                                                  const int32_t *__restrict__ iptr_, const int32_t *__restrict__ irow_,
                                                  int32_t *__restrict__ colptr_out, int32_t *__restrict__ rowidx_out,
                                                  double *__restrict__ vals_out) {
    const auto colptr = gmem(colptr_);
    const auto rowidx = gmem(rowidx_);
    const auto vals = gmem(vals_);
    const auto iptr = gmem(iptr_);
    const auto irow = gmem(irow_);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= N; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t base = (int64_t)colptr[j] + iptr[j];
        colptr_out[j] = (int32_t)base;
        if (j == N) continue;
        int32_t a = colptr[j], ae = colptr[j + 1], q = iptr[j], qe = iptr[j + 1];
        int64_t o = base;
        while (a < ae || q < qe) {
            if (q < qe && (a >= ae || irow[q] < rowidx[a])) {
                rowidx_out[o] = irow[q];
                vals_out[o] = 1.0;
                ++q;
            } else {
                rowidx_out[o] = rowidx[a];
                vals_out[o] = static_cast<double>(vals[a]);
                ++a;
            }
            ++o;
        }
    }
}

// Block b's columns as a CSC of their own: colptr_b[j] = colptr[c0 + j] - colptr[c0], the
// D slices packed one after the other (block b's at offset c0 + b).
__global__ __launch_bounds__(256) void k_pp_slices(const int32_t *__restrict__ colptr_, int64_t N, int32_t D,
                                                   int32_t *__restrict__ out) {
    const auto colptr = gmem(colptr_);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N + D; t += (int64_t)gridDim.x * blockDim.x) {
        // t = c0(b) + b + j for the block b with c0(b) + b <= t < c0(b + 1) + b + 1
        int32_t lo = 0, hi = D - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (((int64_t)mid * N) / D + mid <= t) lo = mid;
            else hi = mid - 1;
        }
        const int64_t c0 = ((int64_t)lo * N) / D;
        const int64_t j = t - c0 - lo;
        out[t] = colptr[c0 + j] - colptr[c0];
    }
}

// Rows of P^T for block b's retained triplets: Pt[off + r][m2r[m]] = sigma_b[r] U_b[m][r], r < rank_b,
// over the n non-empty rows of A' (m2r maps a row to its compacted index; -1 = empty).
__global__ __launch_bounds__(256) void k_pp_proxy(const double *__restrict__ Ub_, const double *__restrict__ sb_,
                                                  int32_t M, int32_t rank, const int32_t *__restrict__ m2r_,
                                                  double *__restrict__ Pt_, int64_t ldp) {
    const auto Ub = gmem(Ub_);
    const auto sb = gmem(sb_);
    const auto m2r = gmem(m2r_);
    const auto Pt = gmem(Pt_);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)rank * M;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = (int32_t)(e / M), m = (int32_t)(e % M);
        const int32_t c = m2r[m];
        if (c >= 0) Pt[(int64_t)r * ldp + c] = sb[r] * Ub[(int64_t)m * M + r];
    }
}

// e_sigma = sum_{i<k} |sigma_hat_i - sigma_i|, e_u = sum_{i<k} sum_m |s_i u_hat_mi - u_mi| with
// s_i = sign <u_hat_i, u_i> (Sec. IV, as read here).  One workgroup per column for e_u (rows in a
// fixed order), then one workgroup adds the columns in order.
__global__ __launch_bounds__(256) void k_pp_err_cols(const double *__restrict__ Uh, const double *__restrict__ U,
                                                     int32_t M, int32_t k, double *__restrict__ col_err) {
    __shared__ double red[256];
    const int32_t i = blockIdx.x;
    double dot = 0.0;
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) dot = fma(Uh[(int64_t)m * k + i], U[(int64_t)m * k + i], dot);
    red[threadIdx.x] = dot;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    const double sgn = red[0] < 0.0 ? -1.0 : 1.0;
    __syncthreads();
    double s = 0.0;
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) s += fabs(sgn * Uh[(int64_t)m * k + i] - U[(int64_t)m * k + i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) col_err[i] = red[0];
}

__global__ void k_pp_err_sum(const double *__restrict__ sh, const double *__restrict__ s, const double *__restrict__ col_err,
                             int32_t k, double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double es = 0.0, eu = 0.0;
    for (int32_t i = 0; i < k; ++i) {
        es += fabs(sh[i] - s[i]);
        eu += col_err[i];
    }
    out[0] = es;
    out[1] = eu;
}

// ---------------------------------------------------------------------------

size_t checker_lds_bytes(int32_t M, int64_t width) {
    return sizeof(uint32_t) * ((size_t)(M + 31) / 32 + (size_t)((width + 31) / 32));
}

hipError_t paper_set_attributes(size_t lds_limit) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_checker), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds_limit);
}

static unsigned pp_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void launch_checker(const CscView &A, int32_t M, int64_t N, int32_t D, const int32_t *cnt, const int32_t *rowptr,
                    const int32_t *csr_col, int32_t kind, uint64_t seed, int64_t *ins, hipStream_t s) {
    const int64_t wmax = (N + D - 1) / D;
    hipLaunchKernelGGL(k_checker, dim3((unsigned)((int64_t)D * M)), dim3(256), checker_lds_bytes(M, wmax), s,
                       A.colptr, A.rowidx, M, N, D, cnt, rowptr, csr_col, kind, seed, ins);
}

void launch_checker_apply(const CscView &A, int32_t M, int64_t N, const int64_t *ins, int64_t nins, int32_t *counts,
                          int32_t *btot, int32_t *iptr, int32_t *cursor, int32_t *irow, double *ival,
                          int32_t *long_rows, int32_t *nlong, int32_t *colptr_out, int32_t *rowidx_out,
                          double *vals_out, hipStream_t s) {
    launch_fill_i32(counts, N, 0, s);
    launch_fill_i32(cursor, N, 0, s);
    hipLaunchKernelGGL(k_pp_count, dim3(pp_grid(nins)), dim3(256), 0, s, ins, nins, M, counts);
    launch_exclusive_scan(counts, N, btot, iptr, s);
    hipLaunchKernelGGL(k_pp_place, dim3(pp_grid(nins)), dim3(256), 0, s, ins, nins, M, iptr, cursor, irow);
    launch_sort_segments(iptr, N, irow, ival, long_rows, nlong, s);
    if (A.dtype == 1)
        hipLaunchKernelGGL(k_pp_merge<double>, dim3(pp_grid(N + 1)), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const double *>(A.values), N, iptr, irow, colptr_out, rowidx_out, vals_out);
    else
        hipLaunchKernelGGL(k_pp_merge<float>, dim3(pp_grid(N + 1)), dim3(256), 0, s, A.colptr, A.rowidx,
                           static_cast<const float *>(A.values), N, iptr, irow, colptr_out, rowidx_out, vals_out);
}

void launch_block_slices(const int32_t *colptr, int64_t N, int32_t D, int32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_pp_slices, dim3(pp_grid(N + D)), dim3(256), 0, s, colptr, N, D, out);
}

void launch_proxy_rows(const double *Ub, const double *sb, int32_t M, int32_t rank, const int32_t *m2r, double *Pt,
                       int64_t ldp, hipStream_t s) {
    if (rank <= 0) return;
    hipLaunchKernelGGL(k_pp_proxy, dim3(pp_grid((int64_t)rank * M)), dim3(256), 0, s, Ub, sb, M, rank, m2r, Pt, ldp);
}

void launch_paper_errors(const double *sh, const double *Uh, const double *s_ref, const double *U_ref, int32_t M,
                         int32_t k, double *col_err, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_pp_err_cols, dim3((unsigned)k), dim3(256), 0, s, Uh, U_ref, M, k, col_err);
    hipLaunchKernelGGL(k_pp_err_sum, dim3(1), dim3(64), 0, s, sh, s_ref, col_err, k, out);
}

}  // namespace ranky

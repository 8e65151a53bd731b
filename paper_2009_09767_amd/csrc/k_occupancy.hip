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
#include <algorithm>

#include "batch.hpp"
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
__device__ void occ_chunk(const MatDesc &d, const TV *__restrict__ vals, int64_t c, int32_t *lds_hist) {
    const int32_t M = d.M;
    const int64_t N = d.N, nnz = d.nnz;
    int64_t c0, c1;
    chunk_columns(c, d.cpb, d.ccols, N, d.D, d.bstart, c0, c1);
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) lds_hist[m] = 0;
    __syncthreads();
    int32_t err = 0;
    const auto colptr = gmem(d.colptr);
    const auto rowidx = gmem(d.rowidx);
    const auto gv = gmem(vals);
    for (int64_t j = c0 + threadIdx.x; j < c1; j += blockDim.x) {
        const int64_t e0 = colptr[j], e1 = colptr[j + 1];
        if (e0 < 0 || e1 < e0 || e1 > nnz) {
            err |= kStCsc;
            continue;
        }
        int32_t prev = -1;
        // kOccGroup entries per step, loaded unconditionally (clamped to the column's last
        // entry) so that they are all in flight before the first is used
        for (int64_t e = e0; e < e1; e += kOccGroup) {
            int32_t rr[kOccGroup];
            bool fin[kOccGroup];
#pragma unroll
            for (int t = 0; t < kOccGroup; ++t) {
                const int64_t x = e + t < e1 ? e + t : e1 - 1;
                rr[t] = rowidx[x];
                fin[t] = !d.validate || finite_value(gv[x]);
            }
#pragma unroll
            for (int t = 0; t < kOccGroup; ++t) {
                if (e + t >= e1) break;
                const int32_t r = rr[t];
                if (r < 0 || r >= M) {
                    err |= kStCsc;
                    continue;
                }
                if (r <= prev) err |= kStCsc;
                prev = r;
                atomicAdd(&lds_hist[r], 1);
                if (!fin[t]) err |= kStNonfinite;
            }
        }
    }
    if (threadIdx.x == 0) {
        if (c0 == 0 && c1 > 0 && d.colptr[0] != 0) err |= kStCsc;
        if (c1 == N && c0 < c1 && (int64_t)d.colptr[N] != nnz) err |= kStCsc;
    }
    if (err) atomicOr(&d.scal[kScStatus], err);
    __syncthreads();
    int32_t *out = d.hist + c * (int64_t)M;
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) out[m] = lds_hist[m];
}

__global__ __launch_bounds__(256) void k_occ_chunks(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                    int count) {
    extern __shared__ int32_t lds_hist[];
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int64_t c = blockIdx.x - wp[mat];
    if (d.dtype == 1)
        occ_chunk<double>(d, static_cast<const double *>(d.values), c, lds_hist);
    else
        occ_chunk<float>(d, static_cast<const float *>(d.values), c, lds_hist);
}

// One thread per (block, row): the block's occupancy of the row (sum of its chunk
// histograms), the lonely / single-entry row counts of the block, and the row's total
// (integer atomics: exact, so independent of their order).  Blocks b = blockIdx.y,
// + gridDim.y, ...
__global__ __launch_bounds__(256) void k_occ_rows(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                  int count) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int32_t M = d.M, cpb = d.cpb;
    const int32_t m = (blockIdx.x - wp[mat]) * blockDim.x + threadIdx.x;
    const bool valid = m < M;
    const int lane = threadIdx.x & 63;
    int32_t total = 0;
    for (int32_t b = blockIdx.y; b < d.D; b += gridDim.y) {
        const auto hist = gmem(d.hist) + (int64_t)b * cpb * M + (valid ? m : 0);
        int32_t cb = 0;
        int32_t t = 0;
        for (; t + 4 <= cpb; t += 4) {
            const int32_t h0 = hist[(int64_t)t * M], h1 = hist[(int64_t)(t + 1) * M];
            const int32_t h2 = hist[(int64_t)(t + 2) * M], h3 = hist[(int64_t)(t + 3) * M];
            cb += h0 + h1 + h2 + h3;
        }
        for (; t < cpb; ++t) cb += hist[(int64_t)t * M];
        if (valid && d.cnt) d.cnt[(int64_t)b * M + m] = cb;
        const uint64_t z = __ballot(valid && cb == 0);
        const uint64_t sg = __ballot(valid && cb == 1);
        if (lane == 0) {
            if (z) atomicAdd(&d.lonely[b], __popcll(z));
            if (sg) atomicAdd(&d.single[b], __popcll(sg));
        }
        total += cb;
    }
    if (valid && total) atomicAdd(&d.rownnz[m], total);
}

// One workgroup of 1024 threads: exclusive scan of the row counts (row pointers of
// the row-major copy) and the compaction maps of the non-empty rows.
//   m2r[m] = position of row m among the non-empty rows, or -1
//   r2m[i] = the i-th non-empty row;  empty[e] = the e-th empty row (ascending)
__global__ __launch_bounds__(1024) void k_occ_scan(const MatDesc *__restrict__ descs) {
    const MatDesc &d = descs[blockIdx.x];
    const int32_t M = d.M;
    const int32_t *__restrict__ rownnz = d.rownnz;
    int32_t *__restrict__ rowptr = d.rowptr;
    int32_t *__restrict__ m2r = d.m2r;
    int32_t *__restrict__ r2m = d.r2m;
    int32_t *__restrict__ empty = d.empty;
    int32_t *__restrict__ scal = d.scal;
    int32_t *__restrict__ gsegp = d.gsegp;
    int32_t *__restrict__ gslot = d.gslot;
    __shared__ int64_t s_nnz[1024];
    __shared__ int32_t s_ne[1024], s_seg[1024], s_slot[1024];
    const int32_t per = (M + 1023) / 1024;
    const int32_t m0 = threadIdx.x * per;
    // a nonempty row of deg nonzeros takes ceil(deg / gseg) Gram segments, and as many
    // partial rows when that is more than one
    const int64_t gs = d.gseg;
    auto segs = [gs](int32_t deg) { return (int32_t)(((int64_t)deg + gs - 1) / gs); };
    int64_t loc_nnz = 0;
    int32_t loc_ne = 0, loc_seg = 0, loc_slot = 0;
    for (int32_t m = m0; m < m0 + per && m < M; ++m) {
        loc_nnz += rownnz[m];
        loc_ne += rownnz[m] > 0;
        const int32_t sg = segs(rownnz[m]);
        loc_seg += sg;
        loc_slot += sg > 1 ? sg : 0;
    }
    s_nnz[threadIdx.x] = loc_nnz;
    s_ne[threadIdx.x] = loc_ne;
    s_seg[threadIdx.x] = loc_seg;
    s_slot[threadIdx.x] = loc_slot;
    __syncthreads();
    // Hillis-Steele inclusive scan (fixed order; integers)
    for (int32_t off = 1; off < 1024; off <<= 1) {
        int64_t a = 0;
        int32_t b = 0, c = 0, e = 0;
        if ((int32_t)threadIdx.x >= off) {
            a = s_nnz[threadIdx.x - off];
            b = s_ne[threadIdx.x - off];
            c = s_seg[threadIdx.x - off];
            e = s_slot[threadIdx.x - off];
        }
        __syncthreads();
        s_nnz[threadIdx.x] += a;
        s_ne[threadIdx.x] += b;
        s_seg[threadIdx.x] += c;
        s_slot[threadIdx.x] += e;
        __syncthreads();
    }
    int64_t run = s_nnz[threadIdx.x] - loc_nnz;
    int32_t nr = s_ne[threadIdx.x] - loc_ne;
    int32_t sr = s_seg[threadIdx.x] - loc_seg, pr = s_slot[threadIdx.x] - loc_slot;
    for (int32_t m = m0; m < m0 + per && m < M; ++m) {
        rowptr[m] = (int32_t)run;
        run += rownnz[m];
        if (rownnz[m] > 0) {
            m2r[m] = nr;
            r2m[nr] = m;
            if (gsegp) {
                gsegp[nr] = sr;
                gslot[nr] = pr;
            }
            const int32_t sg = segs(rownnz[m]);
            sr += sg;
            pr += sg > 1 ? sg : 0;
            ++nr;
        } else {
            m2r[m] = -1;
            empty[m - nr] = m;
        }
    }
    if (threadIdx.x == 1023) {
        rowptr[M] = (int32_t)s_nnz[1023];
        scal[kScNonempty] = s_ne[1023];
        scal[kScGramSegs] = s_seg[1023];
        scal[kScGramSlots] = s_slot[1023];
        if (gsegp) {
            gsegp[s_ne[1023]] = s_seg[1023];
            gslot[s_ne[1023]] = s_slot[1023];
        }
    }
    // the densest rows, in order of degree (then row index): one block-wide arg-max per pick
    int32_t *__restrict__ dense = d.dense;
    if (!dense) return;
    __syncthreads();
    int64_t *s_key = s_nnz;   // reused
    const int64_t tmin = d.N / 64 > 4096 ? d.N / 64 : 4096;
    int64_t last = INT64_MAX;
    for (int t = 0; t < kDenseRows; ++t) {
        int64_t best = -1;
        for (int32_t m = m0; m < m0 + per && m < M; ++m) {
            if (rownnz[m] < tmin) continue;
            const int64_t key = ((int64_t)rownnz[m] << 32) | (int64_t)(uint32_t)(M - 1 - m);
            if (key < last && key > best) best = key;
        }
        s_key[threadIdx.x] = best;
        __syncthreads();
        for (int off = 512; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off && s_key[threadIdx.x + off] > s_key[threadIdx.x])
                s_key[threadIdx.x] = s_key[threadIdx.x + off];
            __syncthreads();
        }
        best = s_key[0];
        __syncthreads();
        if (threadIdx.x == 0) dense[t] = best < 0 ? -1 : M - 1 - (int32_t)(best & 0xffffffff);
        last = best;
        if (best < 0) {
            for (int u = t + 1 + (int)threadIdx.x; u < kDenseRows; u += blockDim.x) dense[u] = -1;
            break;
        }
    }
}

// Turn the chunk histograms into the start offset of every (chunk, row) run in the
// row-major copy (row pointer + earlier chunks), in place.  A workgroup of 1024 threads
// takes 64 rows (lanes) and cuts the chunks into 16 contiguous segments (waves): each
// wave sums its segment, the segment totals are scanned in LDS, and each wave rewrites
// its segment from its starting offset.  Integer sums: exact.  blockIdx.y = which 64
// rows of the 256-row tile.
__global__ __launch_bounds__(1024) void k_occ_offsets(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                      int count) {
    __shared__ int32_t seg_sum[16][64];
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int32_t M = d.M;
    const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int32_t m = (blockIdx.x - wp[mat]) * 256 + blockIdx.y * 64 + lane;
    if ((blockIdx.x - wp[mat]) * 256 + blockIdx.y * 64 >= M) return;   // uniform per workgroup
    const bool valid = m < M;
    const int64_t nch = d.nchunks, per = (nch + 15) / 16;
    const int64_t c0 = seg * per < nch ? seg * per : nch, c1 = c0 + per < nch ? c0 + per : nch;
    const auto hist = gmem(d.hist) + (valid ? m : 0);
    int32_t sum = 0;
    int64_t c = c0;
    for (; c + 8 <= c1; c += 8) {
        int32_t h[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) h[t] = hist[(c + t) * M];
#pragma unroll
        for (int t = 0; t < 8; ++t) sum += h[t];
    }
    for (; c < c1; ++c) sum += hist[c * M];
    seg_sum[seg][lane] = sum;
    __syncthreads();
    if (!valid) return;
    int32_t run = gmem(d.rowptr)[m];
    for (int s = 0; s < seg; ++s) run += seg_sum[s][lane];
    c = c0;
    for (; c + 8 <= c1; c += 8) {
        int32_t h[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) h[t] = hist[(c + t) * M];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            hist[(c + t) * M] = run;
            run += h[t];
        }
    }
    for (; c < c1; ++c) {
        const int32_t h = hist[c * M];
        hist[c * M] = run;
        run += h;
    }
}

// Stable transpose: one wave per chunk, 64 columns at a time (lane = column).
// A row occurs at most once per column, so the rank of an entry among the entries
// of its row inside these 64 columns is the number of lower lanes holding that row:
// lanes publish themselves in a per-row 64-bit mask (bitwise OR commutes, so the
// mask does not depend on timing), read it back and count.  The entry's slot is
// the row's running offset plus that rank; the lowest lane then advances the offset.
// csr_ke[slot] = (CSC position of the entry, end of its column) as one 8-byte store,
// csr_col[slot] = its column.  With light = 1 (the heavy-row split, whose light CSC is built
// first) the light CSC is transposed instead of the CSC: the light rows' slots then hold their
// positions and column ends in it, so the Gram walk steps over light entries only, and the
// dense rows' slots are never written (nor read: their workgroups do not walk).  The per-chunk
// row offsets hold for both, a light row having all its entries in the light CSC.
// The first kTrRegs row indices of each lane's column are held in registers for the
// four passes, loaded (with the next group's column bounds) while the previous group's
// passes run; entries past kTrRegs are read from memory in each pass.
constexpr int kTrRegs = 24;

__device__ __forceinline__ void tr_load_rows(__attribute__((address_space(1))) const int32_t *rowidx, int32_t e0,
                                             int32_t e1, int32_t (&rows)[kTrRegs]) {
    const int32_t n = e1 - e0;
#pragma unroll
    for (int t = 0; t < kTrRegs; ++t) {
        // a valid address for every lane: entry 0 exists (the kernel returns when nnz = 0)
        const int32_t x = n > 0 ? e0 + (t < n ? t : n - 1) : 0;
        rows[t] = rowidx[x];
    }
}

__global__ __launch_bounds__(64) void k_transpose(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                  int count, int light_) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    if (d.nnz == 0) return;
    const int32_t M = d.M;
    const bool light = light_ != 0 && d.hwg > 0;
    const auto colptr = gmem(light ? d.lptr : d.colptr);
    const auto rowidx = gmem(light ? d.lrowidx : d.rowidx);
    typedef int32_t i2 __attribute__((ext_vector_type(2)));
    const auto csr_ke = gmem(reinterpret_cast<i2 *>(d.csrk));
    const auto csr_col = gmem(d.csrcol);
    extern __shared__ uint64_t lds_mask[];
    int32_t *ctr = reinterpret_cast<int32_t *>(lds_mask + M);
    const int64_t c = blockIdx.x - wp[mat];
    int64_t c0, c1;
    chunk_columns(c, d.cpb, d.ccols, d.N, d.D, d.bstart, c0, c1);
    const auto off = gmem(d.hist) + c * (int64_t)M;
    for (int32_t m = threadIdx.x; m < M; m += 64) {
        lds_mask[m] = 0;
        ctr[m] = off[m];
    }
    const int lane = threadIdx.x;
    const uint64_t bit = 1ull << lane;
    const uint64_t lower = bit - 1;
    int32_t e0 = 0, e1 = 0;
    if (c0 + lane < c1) {
        e0 = colptr[c0 + lane];
        e1 = colptr[c0 + lane + 1];
    }
    int32_t rows[kTrRegs];
    tr_load_rows(rowidx, e0, e1, rows);
    __syncthreads();
    for (int64_t g = c0; g < c1; g += 64) {
        const int64_t j = g + lane;
        const int32_t n = e1 - e0;
        // next group: bounds now, its rows after pass 1 (they are in flight during passes 2-4)
        int32_t f0 = 0, f1 = 0;
        if (j + 64 < c1) {
            f0 = colptr[j + 64];
            f1 = colptr[j + 65];
        }
#pragma unroll
        for (int t = 0; t < kTrRegs; ++t)
            if (t < n) atomicOr(reinterpret_cast<unsigned long long *>(&lds_mask[rows[t]]), bit);
        for (int32_t t = kTrRegs; t < n; ++t)
            atomicOr(reinterpret_cast<unsigned long long *>(&lds_mask[rowidx[e0 + t]]), bit);
        int32_t next[kTrRegs];
        tr_load_rows(rowidx, f0, f1, next);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kTrRegs; ++t)
            if (t < n) {
                const int32_t r = rows[t];
                const int32_t slot = ctr[r] + __popcll(lds_mask[r] & lower);
                csr_ke[slot] = i2{e0 + t, e1};
                csr_col[slot] = (int32_t)j;
            }
        for (int32_t t = kTrRegs; t < n; ++t) {
            const int32_t r = rowidx[e0 + t];
            const int32_t slot = ctr[r] + __popcll(lds_mask[r] & lower);
            csr_ke[slot] = i2{e0 + t, e1};
            csr_col[slot] = (int32_t)j;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kTrRegs; ++t)
            if (t < n) {
                const int32_t r = rows[t];
                const uint64_t mk = lds_mask[r];
                if ((mk & lower) == 0) ctr[r] += __popcll(mk);
            }
        for (int32_t t = kTrRegs; t < n; ++t) {
            const int32_t r = rowidx[e0 + t];
            const uint64_t mk = lds_mask[r];
            if ((mk & lower) == 0) ctr[r] += __popcll(mk);
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kTrRegs; ++t)
            if (t < n) lds_mask[rows[t]] = 0;
        for (int32_t t = kTrRegs; t < n; ++t) lds_mask[rowidx[e0 + t]] = 0;
        __syncthreads();
        e0 = f0;
        e1 = f1;
#pragma unroll
        for (int t = 0; t < kTrRegs; ++t) rows[t] = next[t];
    }
}

// Per matrix: clear the scalar block and the per-block counters (one workgroup each).
__global__ __launch_bounds__(256) void k_batch_prep(const MatDesc *__restrict__ descs) {
    const MatDesc &d = descs[blockIdx.x];
    for (int32_t i = threadIdx.x; i < kScCount; i += blockDim.x) d.scal[i] = 0;
    for (int32_t b = threadIdx.x; b < d.D; b += blockDim.x) {
        d.lonely[b] = 0;
        d.single[b] = 0;
    }
    for (int32_t m = threadIdx.x; m < d.M; m += blockDim.x) d.rownnz[m] = 0;
}

// Gather every matrix's scalars into one compact array for a single read-back:
// out_i32[10i..10i+9] = status, M', rank, sweeps, not-converged, lonely max, blocks with
// lonely rows, active, Gram segments, Gram partial rows;  out_f64[2i..2i+1] = tau, sigma_1.
// With out_blk != NULL also the Alg. 1 counts per block: out_blk[2 blk_off + b] = lonely rows of
// block b, out_blk[2 blk_off + D + b] = rows with one entry in block b.
__global__ __launch_bounds__(256) void k_batch_collect(const MatDesc *__restrict__ descs, int count,
                                                       int32_t *__restrict__ out_i32, double *__restrict__ out_f64,
                                                       int32_t *__restrict__ out_blk) {
    const int i = blockIdx.x;
    if (i >= count) return;
    const MatDesc &d = descs[i];
    if (out_blk) {
        int32_t *ob = out_blk + 2 * (int64_t)d.blk_off;
        for (int32_t b = threadIdx.x; b < d.D; b += blockDim.x) {
            ob[b] = d.lonely[b];
            ob[d.D + b] = d.single[b];
        }
    }
    __shared__ int32_t mx[256], nz[256];
    int32_t m = 0, z = 0;
    for (int32_t b = threadIdx.x; b < d.D; b += blockDim.x) {
        m = max(m, d.lonely[b]);
        z += d.lonely[b] > 0;
    }
    mx[threadIdx.x] = m;
    nz[threadIdx.x] = z;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            mx[threadIdx.x] = max(mx[threadIdx.x], mx[threadIdx.x + off]);
            nz[threadIdx.x] += nz[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int32_t *o = out_i32 + (size_t)kColI * i;
        o[0] = d.scal[kScStatus];
        o[1] = d.scal[kScNonempty];
        o[2] = d.scal[kScRank];
        o[3] = d.jstate ? d.jstate[kJsSweeps] : 0;
        o[4] = d.jstate ? d.jstate[kJsNotConv] : 0;
        o[5] = mx[0];
        o[6] = nz[0];
        o[7] = d.jstate ? d.jstate[kJsActive] : 0;
        o[8] = d.scal[kScGramSegs];
        o[9] = d.scal[kScGramSlots];
        int32_t heavy = 0;   // dense rows split out of the sparse Gram walk
        if (d.hwg > 0 && d.dense)
            for (int t = 0; t < kDenseRows; ++t) heavy += d.dense[t] >= 0;
        o[10] = heavy;
        out_f64[2 * i + 0] = d.sdbl[kSdTau];
        out_f64[2 * i + 1] = d.sdbl[kSdSigmaMax];
    }
}

void launch_batch_prep(const MatDesc *descs, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)count), dim3(256), 0, s, descs);
}

void launch_batch_collect(const MatDesc *descs, int count, int32_t *out_i32, double *out_f64, int32_t *out_blk,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_batch_collect, dim3((unsigned)count), dim3(256), 0, s, descs, count, out_i32, out_f64,
                       out_blk);
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

void launch_occupancy(const MatDesc *descs, const int32_t *wp_chunks, int64_t n_chunk_blocks,
                      const int32_t *wp_rows, int64_t n_row_blocks, int count, int32_t maxM, int32_t maxD,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_occ_chunks, dim3((unsigned)n_chunk_blocks), dim3(256), sizeof(int32_t) * (size_t)maxM, s,
                       descs, wp_chunks, count);
    hipLaunchKernelGGL(k_occ_rows, dim3((unsigned)n_row_blocks, (unsigned)std::min(maxD, 1024)), dim3(256), 0, s,
                       descs, wp_rows, count);
    hipLaunchKernelGGL(k_occ_scan, dim3((unsigned)count), dim3(1024), 0, s, descs);
}

void launch_row_offsets(const MatDesc *descs, const int32_t *wp_rows, int64_t n_row_blocks, int count, hipStream_t s) {
    if (n_row_blocks <= 0) return;
    hipLaunchKernelGGL(k_occ_offsets, dim3((unsigned)n_row_blocks, 4), dim3(1024), 0, s, descs, wp_rows, count);
}

void launch_transpose(const MatDesc *descs, const int32_t *wp_chunks, int64_t n_chunk_blocks, int count, int32_t maxM,
                      bool light, hipStream_t s) {
    if (n_chunk_blocks <= 0) return;
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)n_chunk_blocks), dim3(64), transpose_lds_bytes(maxM), s, descs,
                       wp_chunks, count, light ? 1 : 0);
}

size_t transpose_lds_bytes(int32_t M) { return (sizeof(uint64_t) + sizeof(int32_t)) * (size_t)M; }

hipError_t occupancy_set_attributes(int32_t maxM) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_transpose),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)transpose_lds_bytes(maxM));
    return e;
}

}  // namespace ranky

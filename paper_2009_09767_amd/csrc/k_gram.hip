// k_gram.hip -- the block Grams A^i A^i^T reduced into G (Eq. 2-3).
//
// G = sum_i A^i A^i^T = sum_j a_j a_j^T over all columns j.  Owner computes: the
// workgroup of compacted row i (original row p) produces row i of G, entries
// G[p][q] for q > p, by walking row p's nonzeros (j, a_pj) in column order (hence
// block by block) and, for each, the later entries (q, a_qj) of column j.  Its waves
// split row p's nonzeros into contiguous runs (so runs of blocks), each wave summing
// into a private LDS row; the runs are then added in wave order: a fixed-order
// segmented reduction over the blocks, with no floating-point atomics.
//
// Inside a wave the 64 lanes hold 64 different columns, and two of them may reach
// the same q at the same step.  Each such collision is resolved by electing the
// lowest lane through an integer min in LDS; the winner adds its product, the others
// retry, so the sum per address runs in lane order.  The tag row of the election is
// shared by the workgroup's waves (ids are workgroup-wide lane numbers): a winner
// clears the tag only while it still holds its own id (compare-and-swap), so no wave
// can erase another wave's id, and within a wave a higher lane never reads its own id
// while a lower lane of the same wave is pending on the same q.  Each wave adds into
// its own row, so the additions per address still run in lane order, and the result
// is independent of timing.
//
// The diagonal a_pj^2 terms are summed per lane and reduced by a fixed shuffle tree.
// G is written in compacted coordinates (empty rows removed), symmetric, padded
// with zeros up to npad; every entry is written exactly once.
//
// The densest rows (up to kDenseRows, chosen by the scan) meet in most columns, so most
// lanes of a wave would elect on the same few addresses; their products go instead to
// lane-private LDS slots, reduced over the lanes by a fixed shuffle tree at the end.
//
// A row with more than gseg nonzeros (a per-matrix power of two, at most 2^16) is cut
// into segments of gseg consecutive nonzeros (in column order), one workgroup each, so
// a dense row does not serialise the whole launch.  Each segment writes its partial row (FP64) to a slot, and
// k_gram_reduce adds the slots in segment order: the sum order is a function of the
// row alone (not of the block count D or of timing).  Rows of one segment write G
// directly, as before.
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

template <typename Acc>
__device__ __forceinline__ Acc wave_sum(Acc v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One light-CSC record, loaded (returns the row, the value in x) or stored as one vector access.
// The vector's elements are copied to scalars before any bit cast (a bit cast applied to a
// vector element expression has been compiled as a cast of element 0).
template <typename TV>
__device__ __forceinline__ int32_t light_rec_load(__attribute__((address_space(1))) const LightRec<TV> *p, TV &x) {
    if constexpr (sizeof(TV) == 4) {
        typedef int32_t i2 __attribute__((ext_vector_type(2)));
        const i2 w = *reinterpret_cast<__attribute__((address_space(1))) const i2 *>(p);
        const int32_t row = w[0], bits = w[1];
        x = __builtin_bit_cast(TV, bits);
        return row;
    } else {
        typedef int32_t i4 __attribute__((ext_vector_type(4)));
        const i4 w = *reinterpret_cast<__attribute__((address_space(1))) const i4 *>(p);
        const int32_t row = w[0], lo = w[2], hi = w[3];
        x = __builtin_bit_cast(TV, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
        return row;
    }
}

template <typename TV>
__device__ __forceinline__ void light_rec_store(__attribute__((address_space(1))) LightRec<TV> *p, int32_t row, TV x) {
    if constexpr (sizeof(TV) == 4) {
        typedef int32_t i2 __attribute__((ext_vector_type(2)));
        const i2 w = {row, __builtin_bit_cast(int32_t, x)};
        *reinterpret_cast<__attribute__((address_space(1))) i2 *>(p) = w;
    } else {
        typedef int32_t i4 __attribute__((ext_vector_type(4)));
        const uint64_t b = __builtin_bit_cast(uint64_t, x);
        const i4 w = {row, 0, (int32_t)(uint32_t)b, (int32_t)(uint32_t)(b >> 32)};
        *reinterpret_cast<__attribute__((address_space(1))) i4 *>(p) = w;
    }
}

// kRec: the heavy split's walk over the light CSC, read as (row, value) records
template <typename TV, typename Acc, bool kRec>
__device__ __forceinline__ void gram_row(const MatDesc &dsc, const TV *__restrict__ vals_, int32_t i, int32_t seg, int32_t nseg,
                         double *lds_raw) {
    const int32_t M = dsc.M, n = dsc.n, npad = dsc.npad;
    const int64_t ld = npad;
    // global (not FLAT) accesses: FLAT ones would also hold up the LDS waits below
    const auto vals = gmem(vals_);
    const auto rowidx = gmem(dsc.rowidx);
    const auto rec = gmem(static_cast<const LightRec<TV> *>(dsc.lvals));
    auto value_at = [&](int32_t at) -> TV {
        if constexpr (kRec) {
            TV x;
            light_rec_load(rec + at, x);
            return x;
        } else {
            return vals[at];
        }
    };
    const auto rowptr = gmem(dsc.rowptr);
    const auto r2m = gmem(dsc.r2m);
    typedef int32_t i2 __attribute__((ext_vector_type(2)));
    const auto csr_ke = gmem(reinterpret_cast<const i2 *>(dsc.csrk));   // (position, column end) per slot
    const auto dense = gmem(dsc.dense);
    const auto G = gmem(dsc.G);
    // the matrix's own wave count (a function of its M alone, so a batch sums in the order a
    // single call does); waves of a wider launch at or past it take no part in the walk
    const int nw = dsc.gwaves;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const bool walker = wave < nw;
    if (i >= n) {  // padding row and column of the Jacobi layout (all of them: with the heavy
                   // split no dense row's workgroup writes its part of them)
        for (int32_t j = threadIdx.x; j < npad; j += blockDim.x) {
            G[(int64_t)i * ld + j] = 0.0;
            G[(int64_t)j * ld + i] = 0.0;
        }
        return;
    }
    Acc *acc = reinterpret_cast<Acc *>(lds_raw);                  // nw x M
    // nw x kDenseRows x 64 lane-private slots, 16-byte aligned (M may be odd); none with the
    // heavy-row split, whose dense rows' pairs come from the gathers
    const int nslot = dsc.hwg > 0 ? 0 : kDenseRows * 64;
    Acc *dslot = reinterpret_cast<Acc *>(reinterpret_cast<char *>(lds_raw) +
                                         ((((size_t)nw * M * sizeof(Acc)) + 15) & ~(size_t)15));
    int32_t *tag = reinterpret_cast<int32_t *>(dslot + (size_t)nw * nslot);  // M, shared
    int8_t *dmap = reinterpret_cast<int8_t *>(tag + M);  // M: dense index or -1
    __shared__ Acc dsum[16];
    __syncthreads();
    for (int32_t t = threadIdx.x; t < nw * M; t += blockDim.x) acc[t] = Acc(0);
    for (int32_t t = threadIdx.x; t < M; t += blockDim.x) tag[t] = kTagFree;
    for (int32_t t = threadIdx.x; t < nw * nslot; t += blockDim.x) dslot[t] = Acc(0);
    for (int32_t t = threadIdx.x; t < M; t += blockDim.x) dmap[t] = -1;
    __syncthreads();
    if (threadIdx.x < kDenseRows && dense[threadIdx.x] >= 0) dmap[dense[threadIdx.x]] = (int8_t)threadIdx.x;
    __syncthreads();

    const int32_t p = r2m[i];
    // heavy split: a dense row's entries of G come from the heavy tiles and from the other
    // rows' gathers, so its workgroups have nothing to do
    constexpr bool heavy = kRec;   // launched for a matrix with the split (dsc.hwg > 0)
    if (heavy && dmap[p] >= 0) return;
    // with dense tiles on, a dense row's pairs with other dense rows are theirs; with the
    // heavy split every pair with a dense row comes from the gathers below
    const bool skip_dense = heavy || (dsc.dwg > 0 && dmap[p] >= 0);
    const int32_t r_begin = rowptr[p], r_end = rowptr[p + 1];
    const int32_t gs = dsc.gseg;
    const int32_t e_begin = r_begin + seg * gs;
    const int32_t e_end = (nseg == 1 || r_end - e_begin <= gs) ? r_end : e_begin + gs;
    const int32_t deg = e_end - e_begin;
    const int32_t run = (deg + nw - 1) / nw;   // contiguous run of this segment per wave
    const int32_t wb = e_begin + wave * run;
    const int32_t we = (wb + run < e_end) ? wb + run : e_end;
    Acc *my = acc + (size_t)wave * M;
    const int32_t gid = threadIdx.x;   // workgroup-wide id in the election
    Acc *myslot = dslot + (size_t)wave * nslot + lane;   // not used with the heavy split
    Acc dg = Acc(0);

    // Each lane walks the later entries of its column kGramStep steps at a time: the
    // loads of a group are all issued before the first product is added.  Batches of 64
    // nonzeros are pipelined: while a batch's additions run, the next batch's value and
    // first group of column entries and the positions of the batch after it are in
    // flight.  The additions still run step by step in lane order, so the sums are those of
    // a one-step walk.  Lanes past the end of the run load the run's last entry (a valid
    // address) and discard it: with no conditional loads, all of a group's loads stay in
    // flight.
    auto clampe = [&](int32_t x) { return x < we ? x : we - 1; };
    auto load_group = [&](int32_t k0, int32_t k1, int32_t s, int32_t(&qs)[kGramStep], Acc(&vs)[kGramStep]) {
#pragma unroll
        for (int u = 0; u < kGramStep; ++u) {
            const int32_t at = k0 + s + u < k1 ? k0 + s + u : k0;
            if constexpr (kRec) {
                TV x;
                qs[u] = light_rec_load(rec + at, x);
                vs[u] = static_cast<Acc>(x);
            } else {
                qs[u] = rowidx[at];
                vs[u] = static_cast<Acc>(vals[at]);
            }
        }
    };
    int32_t kk = 0, kend = 0, kk1 = 0, kend1 = 0;
    TV ta = TV(0);   // the value of this lane's nonzero (a in the walk's precision)
    Acc a = Acc(0);
    int32_t q0[kGramStep];
    Acc v0[kGramStep];
#pragma unroll
    for (int u = 0; u < kGramStep; ++u) {
        q0[u] = 0;
        v0[u] = Acc(0);
    }
    // heavy split: the pairs with the dense rows, sum_j a_pj aht[j][h] over this wave's run, are
    // gathered batch by batch inside the walk (the batch's values are at hand).  A row of aht
    // (kDenseRows values) is read by kLpn lanes with 16-byte loads (kVec values each), so a step
    // covers kNps nonzeros, one per lane group g, and a batch of 64 nonzeros takes kHlSteps
    // steps, all of its row loads issued before the walk's additions and summed after them.
    // Group g sums the nonzeros u = g (mod kNps) in order; the groups are added in order at the
    // end.
    constexpr int kVec = 16 / (int)sizeof(TV), kLpn = kDenseRows / kVec, kNps = 64 / kLpn;
    constexpr int kHlSteps = 64 / kNps;
    typedef TV tv_vec __attribute__((ext_vector_type(kVec)));
    const auto aht = gmem(static_cast<const TV *>(dsc.aht));
    const auto csr_col = gmem(dsc.csrcol);
    const int g = lane / kLpn, hq = lane % kLpn;
    double hs[kVec];
#pragma unroll
    for (int c = 0; c < kVec; ++c) hs[c] = 0.0;
    int32_t jl0 = 0, jl1 = 0;   // the columns of this batch's and the next batch's nonzeros
    if (walker && wb < we) {
        const int32_t e0 = clampe(wb + lane), e1 = clampe(wb + 64 + lane);
        const i2 w0 = csr_ke[e0], w1 = csr_ke[e1];
        kk = w0[0];
        kend = w0[1];
        kk1 = w1[0];
        kend1 = w1[1];
        if (heavy) {
            jl0 = csr_col[e0];
            jl1 = csr_col[e1];
        }
        ta = value_at(kk);
        a = static_cast<Acc>(ta);
        load_group(kk, kend, 1, q0, v0);
    }
    for (int32_t base = wb; walker && base < we; base += 64) {
        const bool has = base + lane < we;
        // ahead: the positions of the batch after next, the next batch's value and first group
        const int32_t e2 = clampe(base + 128 + lane);
        const i2 w2 = csr_ke[e2];
        const int32_t kk2 = w2[0], kend2 = w2[1];
        const TV ta1 = value_at(kk1);
        const Acc a1 = static_cast<Acc>(ta1);
        int32_t q1[kGramStep];
        Acc v1[kGramStep];
        load_group(kk1, kend1, 1, q1, v1);
        // this batch's rows of aht
        tv_vec xs[kHlSteps];
        double as[kHlSteps];
        int32_t jl2 = 0;
        if (heavy) {
            const double am = has ? static_cast<double>(ta) : 0.0;
#pragma unroll
            for (int v = 0; v < kHlSteps; ++v) {
                const int sl = v * kNps + g;   // nonzero v kNps + g of the batch
                const int32_t j = __shfl(jl0, sl, 64);
                as[v] = __shfl(am, sl, 64);
                xs[v] = *reinterpret_cast<__attribute__((address_space(1))) const tv_vec *>(
                    aht + (int64_t)j * kDenseRows + kVec * hq);
            }
            jl2 = csr_col[e2];
        }
        __builtin_amdgcn_sched_barrier(0);
        auto add_group = [&](const int32_t(&qs)[kGramStep], const Acc(&vs)[kGramStep], int32_t s) {
#pragma unroll
            for (int u = 0; u < kGramStep; ++u) {
                const bool act = has && (kk + s + u < kend);
                const int32_t q = qs[u];
                const Acc v = a * vs[u];
                int di = -1;
                if (act) {
                    di = dmap[q];
                    if (di >= 0 && !skip_dense) myslot[di * 64] += v;
                }
                bool pend = act && di < 0;
                while (__ballot(pend) != 0) {
                    if (pend) atomicMin(&tag[q], gid);
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    const bool win = pend && (__hip_atomic_load(&tag[q], __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_WORKGROUP) == gid);
                    if (win) {
                        my[q] += v;
                        atomicCAS(&tag[q], gid, kTagFree);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    pend = pend && !win;
                }
            }
        };
        if (__ballot(has && kk + 1 < kend) != 0) {
            add_group(q0, v0, 1);   // loaded a batch ago
            for (int32_t s = 1 + kGramStep;; s += kGramStep) {
                if (__ballot(has && kk + s < kend) == 0) break;
                int32_t qs[kGramStep];
                Acc vs[kGramStep];
                load_group(kk, kend, s, qs, vs);
                __builtin_amdgcn_sched_barrier(0);   // keep every load of the group ahead of its uses
                add_group(qs, vs, s);
            }
        }
        if (has) dg += a * a;
        if (heavy) {
#pragma unroll
            for (int v = 0; v < kHlSteps; ++v)
#pragma unroll
                for (int c = 0; c < kVec; ++c) hs[c] = fma(as[v], static_cast<double>(xs[v][c]), hs[c]);
            jl0 = jl1;
            jl1 = jl2;
        }
        kk = kk1;
        kend = kend1;
        kk1 = kk2;
        kend1 = kend2;
        ta = ta1;
        a = a1;
#pragma unroll
        for (int u = 0; u < kGramStep; ++u) {
            q0[u] = q1[u];
            v0[u] = v1[u];
        }
    }
    if (heavy && walker) {
        // lane hq of group 0 adds the groups' sums in group order and writes dense rows kVec hq + c
#pragma unroll
        for (int c = 0; c < kVec; ++c) {
            double tot = 0.0;
#pragma unroll
            for (int gg = 0; gg < kNps; ++gg) tot += __shfl(hs[c], gg * kLpn + hq, 64);
            if (lane < kLpn) {
                const int32_t q = dense[kVec * hq + c];
                if (q >= 0) my[q] = static_cast<Acc>(tot);
            }
        }
    }
    dg = wave_sum(dg);
    if (lane == 0) dsum[wave] = dg;
    // the dense rows: lane-private sums reduced over the lanes into the wave's row
    for (int t = 0; walker && !heavy && t < kDenseRows; ++t) {
        const int32_t q = dense[t];
        if (q < 0) break;
        const Acc v = wave_sum(myslot[t * 64]);
        if (lane == 0) my[q] = v;
    }
    __syncthreads();

    if (nseg == 1) {
        // row part G[i][j] and column part G[j][i] for j > i, summing the waves in order
        for (int32_t j = i + 1 + threadIdx.x; j < npad; j += blockDim.x) {
            double v = 0.0;
            if (j < n) {
                const int32_t q = r2m[j];
                for (int w = 0; w < nw; ++w) v += static_cast<double>(acc[(size_t)w * M + q]);
            }
            G[(int64_t)i * ld + j] = v;
            G[(int64_t)j * ld + i] = v;
        }
        if (threadIdx.x == 0) {
            double d = 0.0;
            for (int w = 0; w < nw; ++w) d += static_cast<double>(dsum[w]);
            G[(int64_t)i * ld + i] = d;
        }
        // heavy split: the dense rows before row i (the loop above wrote those after it)
        if (heavy && threadIdx.x < kDenseRows) {
            const int32_t q = dense[threadIdx.x];
            const int32_t jc = q >= 0 ? gmem(dsc.m2r)[q] : -1;
            if (jc >= 0 && jc < i) {
                double v = 0.0;
                for (int w = 0; w < nw; ++w) v += static_cast<double>(acc[(size_t)w * M + q]);
                G[(int64_t)i * ld + jc] = v;
                G[(int64_t)jc * ld + i] = v;
            }
        }
        return;
    }
    // partial row of this segment: entry j >= i (the diagonal at j = i)
    const auto part = gmem(dsc.gpart) + (int64_t)(gmem(dsc.gslot)[i] + seg) * ld;
    for (int32_t j = i + 1 + threadIdx.x; j < n; j += blockDim.x) {
        const int32_t q = r2m[j];
        double v = 0.0;
        for (int w = 0; w < nw; ++w) v += static_cast<double>(acc[(size_t)w * M + q]);
        part[j] = v;
    }
    if (threadIdx.x == 0) {
        double d = 0.0;
        for (int w = 0; w < nw; ++w) d += static_cast<double>(dsum[w]);
        part[i] = d;
    }
    if (heavy && threadIdx.x < kDenseRows) {
        const int32_t q = dense[threadIdx.x];
        const int32_t jc = q >= 0 ? gmem(dsc.m2r)[q] : -1;
        if (jc >= 0 && jc < i) {
            double v = 0.0;
            for (int w = 0; w < nw; ++w) v += static_cast<double>(acc[(size_t)w * M + q]);
            part[jc] = v;
        }
    }
}


// Workgroup b of a matrix: segment b of the nonempty rows' segments (gsegp maps it to
// compacted row i and segment seg), then one workgroup per padding row n..npad-1.
template <bool kHeavy>
__global__ __launch_bounds__(512) void k_gram_rows(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                   int count) {
    extern __shared__ double lds_raw[];
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int32_t b = blockIdx.x - wp[mat];
    const auto gsegp = gmem(d.gsegp);
    const int32_t total = gsegp[d.n];
    int32_t i, seg = 0, nseg = 1;
    if (b >= total) {
        i = d.n + (b - total);
    } else {
        int32_t lo = 0, hi = d.n - 1;   // last i with gsegp[i] <= b
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (gsegp[mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        i = lo;
        seg = b - gsegp[i];
        nseg = gsegp[i + 1] - gsegp[i];
    }
    // the walk's columns: the light CSC's records with the heavy split (FP64 or FP32 Gram only),
    // else the CSC
    if (d.dtype == 1) {
        const double *v = static_cast<const double *>(d.values);
        if (d.prec == 0) gram_row<double, double, kHeavy>(d, v, i, seg, nseg, lds_raw);
        else gram_row<double, float, kHeavy>(d, v, i, seg, nseg, lds_raw);
    } else {
        const float *v = static_cast<const float *>(d.values);
        if (d.prec == 0) gram_row<float, double, kHeavy>(d, v, i, seg, nseg, lds_raw);
        else gram_row<float, float, kHeavy>(d, v, i, seg, nseg, lds_raw);
    }
}

// One workgroup per compacted row; rows cut into segments add their partial rows in
// segment order and write G[i][j], G[j][i] (j > i) and G[i][i].
__global__ __launch_bounds__(256) void k_gram_reduce(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                     int count) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int32_t i = blockIdx.x - wp[mat];
    if (i >= d.n) return;
    const int32_t nseg = gmem(d.gsegp)[i + 1] - gmem(d.gsegp)[i];
    if (nseg <= 1) return;
    const bool heavy = d.hwg > 0;
    if (heavy) {   // a dense row's entries come from the heavy tiles and the other rows
        const int32_t p = gmem(d.r2m)[i];
        for (int t = 0; t < kDenseRows; ++t)
            if (gmem(d.dense)[t] == p) return;
    }
    const int64_t ld = d.npad;
    const auto part = gmem(d.gpart) + (int64_t)gmem(d.gslot)[i] * ld;
    const auto G = gmem(d.G);
    if (heavy && threadIdx.x < kDenseRows) {   // the dense rows before row i
        const int32_t q = gmem(d.dense)[threadIdx.x];
        const int32_t jc = q >= 0 ? gmem(d.m2r)[q] : -1;
        if (jc >= 0 && jc < i) {
            double v = 0.0;
            for (int32_t s = 0; s < nseg; ++s) v += part[(int64_t)s * ld + jc];
            G[(int64_t)i * ld + jc] = v;
            G[(int64_t)jc * ld + i] = v;
        }
    }
    for (int32_t j = i + threadIdx.x; j < d.n; j += blockDim.x) {
        double v = 0.0;
        for (int32_t s = 0; s < nseg; ++s) v += part[(int64_t)s * ld + j];
        G[(int64_t)i * ld + j] = v;
        if (j != i) G[(int64_t)j * ld + i] = v;
    }
    for (int32_t j = d.n + threadIdx.x; j < ld; j += blockDim.x) {
        G[(int64_t)i * ld + j] = 0.0;
        G[(int64_t)j * ld + i] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Split-bf16 Gram tiles of the densest rows on the matrix cores (gram_prec BF16X3).
//
// The densest rows H (the scan's dense list, |H| <= 32) meet in most columns, so their
// block of the Gram, G_HH = A_H A_H^T, is a dense contraction: each workgroup owns a fixed
// range of columns (a function of N alone), densifies A[H, 64 columns] in LDS (FP32) step
// by step, splits every value as x = hi + lo (two bf16, round to nearest even) and adds
// hi hi^T + hi lo^T + lo hi^T with v_mfma_f32_16x16x16_bf16 (lo lo^T, about 2^-16 of the
// product, is dropped), FP32 within a step and FP64 across steps.  The sparse pass leaves
// the pairs of two dense rows out.  The 32 x 32 output is four 16 x 16 blocks; waves 0, 1,
// 2 own blocks (0,0), (0,1), (1,1), the upper triangle.  Partial tiles go to dpart[wg], and
// k_gram_dense_reduce adds them in workgroup order into G: bitwise reproducible and
// independent of D.  (FP64 and FP32 keep these pairs in the sparse pass: measured, tiles
// over every column cost more than the few dense-slot additions they replace.)
constexpr int kDc = 64;          // columns per densified step
constexpr int kDcLd = kDc + 4;   // LDS row stride

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

// round to nearest even (finite inputs), as the top 16 bits of an FP32
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__global__ __launch_bounds__(256) void k_gram_dense(const MatDesc *__restrict__ descs) {
    __shared__ float X[kDenseRows][kDcLd];
    __shared__ int8_t dmap[kMaxM];
    const MatDesc &d = descs[0];
    const int32_t M = d.M;
    const int64_t N = d.N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const auto dense = gmem(d.dense);
    if (dense[1] < 0) return;   // fewer than two dense rows: no pair to compute
    const auto colptr = gmem(d.colptr);
    const auto rowidx = gmem(d.rowidx);
    for (int32_t m = tid; m < M; m += 256) dmap[m] = -1;
    __syncthreads();
    if (tid < kDenseRows && dense[tid] >= 0) dmap[dense[tid]] = (int8_t)tid;
    // this wave's 16 x 16 block (qa, qb) of the 32 x 32 tile
    const int qa = wave == 2 ? 1 : 0, qb = wave == 0 ? 0 : 1;
    const bool mm = wave < 3;
    double acc64[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t c_begin = (N * blockIdx.x) / gridDim.x, c_end = (N * (blockIdx.x + 1)) / gridDim.x;
    const int col = tid & (kDc - 1), sub = tid >> 6;   // 4 threads per column
    for (int64_t c0 = c_begin; c0 < c_end; c0 += kDc) {
        for (int e = tid; e < kDenseRows * kDc; e += 256) X[e / kDc][e % kDc] = 0.f;
        __syncthreads();
        const int64_t j = c0 + col;
        if (j < c_end) {
            const int32_t e1 = colptr[j + 1];
            for (int32_t e = colptr[j] + sub; e < e1; e += 4) {
                const int h = dmap[rowidx[e]];
                if (h >= 0) {
                    if (d.dtype == 1) X[h][col] = (float)gmem(static_cast<const double *>(d.values))[e];
                    else X[h][col] = gmem(static_cast<const float *>(d.values))[e];
                }
            }
        }
        __syncthreads();
        if (mm) {
            const int ra = 16 * qa + (lane & 15), rb = 16 * qb + (lane & 15);
            f4v a32 = {0.f, 0.f, 0.f, 0.f};
            // operands: lane l holds A[l % 16][4 (l / 16) + v] and B[4 (l / 16) + v][l % 16], B = X^T
#pragma unroll
            for (int kb = 0; kb < kDc; kb += 16) {
                s4v ahi, alo, bhi, blo;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int kk = kb + 4 * (lane >> 4) + v;
                    const float xa = X[ra][kk], xb = X[rb][kk];
                    const uint32_t ha = bf16_bits(xa), hb = bf16_bits(xb);
                    ahi[v] = (short)ha;
                    bhi[v] = (short)hb;
                    alo[v] = (short)bf16_bits(xa - __uint_as_float(ha << 16));
                    blo[v] = (short)bf16_bits(xb - __uint_as_float(hb << 16));
                }
                a32 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, a32, 0, 0, 0);
                a32 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, a32, 0, 0, 0);
                a32 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, a32, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) acc64[i] += (double)a32[i];
        }
        __syncthreads();
    }
    if (!mm) return;
    // result layout: element i of lane l at row 4 (l / 16) + i, column l % 16
    const auto out = gmem(d.dpart) + (int64_t)blockIdx.x * kDenseRows * kDenseRows;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        out[(16 * qa + 4 * (lane >> 4) + i) * kDenseRows + 16 * qb + (lane & 15)] = acc64[i];
}

// G[a][b] = G[b][a] for the dense rows a < b (compacted indices): the partial tiles added
// in workgroup order.  Runs after the sparse pass, which left these entries zero.
__global__ __launch_bounds__(1024) void k_gram_dense_reduce(const MatDesc *__restrict__ descs) {
    const MatDesc &d = descs[0];
    const int t = threadIdx.x, h1 = t / kDenseRows, h2 = t % kDenseRows;
    const auto dense = gmem(d.dense);
    if (h1 >= h2 || dense[h1] < 0 || dense[h2] < 0) return;
    const auto part = gmem(d.dpart) + h1 * kDenseRows + h2;
    double v = 0.0;
    for (int32_t b = 0; b < d.dwg; ++b) v += part[(int64_t)b * kDenseRows * kDenseRows];
    const int64_t i1 = gmem(d.m2r)[dense[h1]], i2 = gmem(d.m2r)[dense[h2]];
    const auto G = gmem(d.G);
    G[i1 * d.npad + i2] = v;
    G[i2 * d.npad + i1] = v;
}

// ---------------------------------------------------------------------------
// Heavy-row split of the Gram (FP64 and FP32 accumulation, large single matrices).
//
// The densest rows H (the scan's dense list) hold most nonzeros of a power-law matrix and
// meet in most columns: in the sparse walk they make most of the pairs and most of the
// election collisions.  With the split they leave the walk:
//   - k_gram_heavy_build writes aht[j][h] = a_{H[h], j} (zeros elsewhere), one row of
//     kDenseRows values per column, in the matrix's value type (exact);
//   - G_HH = sum_j aht[j] aht[j]^T on the FP64 matrix cores (k_gram_heavy_tiles): each
//     workgroup owns a fixed column range (a function of N alone), its four waves a fixed
//     quarter of it, summed in wave order into one partial tile per workgroup, which
//     k_gram_heavy_reduce adds in a fixed tree over the workgroups;
//   - the other ("light") rows' entries of every column are copied in row order to a light
//     CSC (k_gram_light_scatter, after a scan of the per-column counts), before the transpose,
//     which then transposes the light CSC, so the light rows' row-major slots hold positions in
//     it: the walk steps over light entries only;
//   - every light row p adds sum_j a_pj aht[j] (one coalesced row per nonzero) in the walk
//     kernel.
// Every sum keeps an order fixed by the matrix alone, so the result is bitwise
// reproducible and independent of D.

// Both kernels below take ranges of kHpCols consecutive columns, one workgroup (256 threads)
// per range in turn: the range's entries are contiguous in the CSC, so they are read in
// coalesced passes of 256 (thread t: entry base + t), an entry's column found by a binary search
// over the range's column starts in LDS, its row's dense slot h from a byte map in LDS.
constexpr int kHpCols = 256;

// the range's dense-row map and column starts (cs[c] = colptr[c0 + c], c = 0 .. nc)
__device__ __forceinline__ void hp_map(const MatDesc &d, int8_t *dmap) {
    const auto dense = gmem(d.dense);
    for (int32_t m = threadIdx.x; m < d.M; m += blockDim.x) dmap[m] = -1;
    __syncthreads();
    if (threadIdx.x < kDenseRows && dense[threadIdx.x] >= 0) dmap[dense[threadIdx.x]] = (int8_t)threadIdx.x;
    __syncthreads();
}

// the column (range-relative) of entry e: the largest c with cs[c] <= e (empty columns share
// their start with the next column, so the column that holds e wins)
__device__ __forceinline__ int32_t hp_col(const int32_t *cs, int32_t nc, int32_t e) {
    int32_t lo = 0, hi = nc - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (cs[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// aht rows of the range cleared, then every dense entry a_{H[h], j} written to aht[j][h]; the
// light entries counted per column (LDS counters, written to lcnt).  The clearing stores are
// complete before the value stores start (the barrier between them).
template <typename TV>
__global__ __launch_bounds__(256) void k_gram_heavy_build(const MatDesc *__restrict__ descs) {
    __shared__ int8_t dmap[kMaxM];
    __shared__ int32_t cs[kHpCols + 1], cnt[kHpCols];
    const MatDesc &d = descs[0];
    hp_map(d, dmap);
    const auto colptr = gmem(d.colptr);
    const auto rowidx = gmem(d.rowidx);
    const auto vals = gmem(static_cast<const TV *>(d.values));
    const auto aht = gmem(static_cast<TV *>(d.aht));
    const auto lcnt = gmem(d.lcnt);
    const int64_t N = d.N, ranges = (N + kHpCols - 1) / kHpCols;
    for (int64_t r = blockIdx.x; r < ranges; r += gridDim.x) {
        const int64_t c0 = r * kHpCols;
        const int32_t nc = (int32_t)(N - c0 < kHpCols ? N - c0 : kHpCols);
        for (int32_t c = threadIdx.x; c <= nc; c += blockDim.x) cs[c] = colptr[c0 + c];
        for (int32_t c = threadIdx.x; c < nc; c += blockDim.x) cnt[c] = 0;
        // clear the range's rows of aht (contiguous: nc * kDenseRows values)
        const int64_t nv = (int64_t)nc * kDenseRows;
        for (int64_t t = threadIdx.x; t < nv; t += blockDim.x) aht[c0 * kDenseRows + t] = TV(0);
        __syncthreads();
        const int64_t e0 = cs[0], e1 = cs[nc];
        for (int64_t base = e0; base < e1; base += blockDim.x) {
            const int64_t e = base + threadIdx.x;
            if (e < e1) {
                const int32_t m = rowidx[e];
                const TV v = vals[e];
                const int32_t c = hp_col(cs, nc, (int32_t)e);
                const int h = dmap[m];
                if (h >= 0) aht[(c0 + c) * kDenseRows + h] = v;
                else atomicAdd(&cnt[c], 1);
            }
        }
        __syncthreads();
        for (int32_t c = threadIdx.x; c < nc; c += blockDim.x) lcnt[c0 + c] = cnt[c];
        __syncthreads();
    }
}

// The light entries in CSC order to the light CSC: a range's light entries start at lptr[c0]
// and keep their order, so entry e's position is that start plus the number of light entries
// before it in the range (a prefix count over the 256-entry passes: ballots within a wave,
// the waves' totals through LDS).
template <typename TV>
__global__ __launch_bounds__(256) void k_gram_light_scatter(const MatDesc *__restrict__ descs) {
    __shared__ int8_t dmap[kMaxM];
    __shared__ int32_t wtot[4];
    const MatDesc &d = descs[0];
    hp_map(d, dmap);
    const auto colptr = gmem(d.colptr);
    const auto rowidx = gmem(d.rowidx);
    const auto vals = gmem(static_cast<const TV *>(d.values));
    const auto lptr = gmem(d.lptr);
    const auto lrow = gmem(d.lrowidx);
    const auto lrec = gmem(static_cast<LightRec<TV> *>(d.lvals));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t N = d.N, ranges = (N + kHpCols - 1) / kHpCols;
    for (int64_t r = blockIdx.x; r < ranges; r += gridDim.x) {
        const int64_t c0 = r * kHpCols;
        const int64_t c1 = c0 + kHpCols < N ? c0 + kHpCols : N;
        const int64_t e0 = colptr[c0], e1 = colptr[c1];
        int32_t out = lptr[c0];
        for (int64_t base = e0; base < e1; base += blockDim.x) {
            const int64_t e = base + threadIdx.x;
            int32_t m = 0;
            TV v = TV(0);
            bool light = false;
            if (e < e1) {
                m = rowidx[e];
                v = vals[e];
                light = dmap[m] < 0;
            }
            const uint64_t bal = __builtin_amdgcn_ballot_w64(light);
            if (lane == 0) wtot[wave] = __popcll(bal);
            __syncthreads();
            int32_t before = out;
            for (int w = 0; w < wave; ++w) before += wtot[w];
            const int32_t pos = before + __popcll(bal & ((1ull << lane) - 1));
            if (e < e1 && light) {
                lrow[pos] = m;
                light_rec_store(lrec + pos, m, v);
            }
            out += wtot[0] + wtot[1] + wtot[2] + wtot[3];
            __syncthreads();
        }
    }
}

// G_HH partial tile of workgroup b over columns [N b / hwg, N (b + 1) / hwg).  The 32 x 32
// tile is the 16 x 16 blocks (0,0), (0,1), (1,1) (the upper triangle); every wave runs all
// three with v_mfma_f64_16x16x4f64 over its quarter of the range, four columns per product
// (lane l holds aht[j0 + l / 16][16 x + l % 16] as both operands' entry), kHhUnroll products
// with their loads issued ahead.
constexpr int kHhUnroll = 4;

template <typename TV>
__global__ __launch_bounds__(256) void k_gram_heavy_tiles(const MatDesc *__restrict__ descs) {
    __shared__ double red[4][3][256];
    const MatDesc &d = descs[0];
    if (gmem(d.dense)[0] < 0) return;
    const auto aht = gmem(static_cast<const TV *>(d.aht));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t N = d.N, hwg = d.hwg;
    const int64_t c0 = (N * blockIdx.x) / hwg, c1 = (N * (blockIdx.x + 1)) / hwg;
    const int64_t q0 = c0 + ((c1 - c0) * wave) / 4, q1 = c0 + ((c1 - c0) * (wave + 1)) / 4;
    typedef double d4 __attribute__((ext_vector_type(4)));
    d4 a00 = {0.0, 0.0, 0.0, 0.0}, a01 = a00, a11 = a00;
    const int kr = lane >> 4, hc = lane & 15;
    for (int64_t j0 = q0; j0 < q1; j0 += 4 * kHhUnroll) {
        double x0[kHhUnroll], x1[kHhUnroll];
#pragma unroll
        for (int u = 0; u < kHhUnroll; ++u) {
            const int64_t j = j0 + 4 * u + kr;
            const bool ok = j < q1;
            const int64_t jj = ok ? j : q0;
            const double v0 = static_cast<double>(aht[jj * kDenseRows + hc]);
            const double v1 = static_cast<double>(aht[jj * kDenseRows + 16 + hc]);
            x0[u] = ok ? v0 : 0.0;
            x1[u] = ok ? v1 : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kHhUnroll; ++u) {
            a00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u], x0[u], a00, 0, 0, 0);
            a01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u], x1[u], a01, 0, 0, 0);
            a11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[u], x1[u], a11, 0, 0, 0);
        }
    }
    // result layout: element i of lane l at row l / 16 + 4 i, column l % 16
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = (kr + 4 * i) * 16 + hc;
        red[wave][0][e] = a00[i];
        red[wave][1][e] = a01[i];
        red[wave][2][e] = a11[i];
    }
    __syncthreads();
    const auto out = gmem(d.hpart) + (int64_t)blockIdx.x * kDenseRows * kDenseRows;
    for (int t = tid; t < 3 * 256; t += 256) {
        const int blk = t >> 8, e = t & 255, r = e >> 4, c = e & 15;
        const double v = ((red[0][blk][e] + red[1][blk][e]) + red[2][blk][e]) + red[3][blk][e];
        const int ra = blk == 2 ? 16 : 0, cb = blk == 0 ? 0 : 16;
        out[(ra + r) * kDenseRows + cb + c] = v;
    }
}

// G entries of the dense rows among themselves (the diagonal included): one workgroup per
// upper-triangle entry (h1 <= h2 by position in the dense list) adds the hwg partial tiles,
// thread t the tiles t, t + 256, ... in order, then a fixed tree over the threads; both G
// entries are written.
__global__ __launch_bounds__(256) void k_gram_heavy_reduce(const MatDesc *__restrict__ descs) {
    __shared__ double red[256];
    const MatDesc &d = descs[0];
    int h1 = 0, rem = blockIdx.x;
    while (rem >= kDenseRows - h1) {
        rem -= kDenseRows - h1;
        ++h1;
    }
    const int h2 = h1 + rem;
    const auto dense = gmem(d.dense);
    if (dense[h1] < 0 || dense[h2] < 0) return;
    const auto part = gmem(d.hpart) + h1 * kDenseRows + h2;
    double v = 0.0;
    for (int32_t b = threadIdx.x; b < d.hwg; b += blockDim.x) v += part[(int64_t)b * kDenseRows * kDenseRows];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t i1 = gmem(d.m2r)[dense[h1]], i2 = gmem(d.m2r)[dense[h2]];
        const auto G = gmem(d.G);
        G[i1 * d.npad + i2] = red[0];
        G[i2 * d.npad + i1] = red[0];
    }
}

int32_t gram_heavy_wgs(int64_t N) {
    const int64_t w = (N + 8191) / 8192;
    return (int32_t)(w < 1 ? 1 : (w > 2048 ? 2048 : w));
}

static unsigned heavy_cols_grid(int64_t n) {
    int64_t b = (n + kHpCols - 1) / kHpCols;
    if (b > 8192) b = 8192;
    return (unsigned)(b < 1 ? 1 : b);
}

void launch_gram_heavy_prep(const MatDesc *descs, const MatDesc &host, hipStream_t s) {
    if (host.hwg <= 0) return;
    const unsigned g = heavy_cols_grid(host.N);
    if (host.dtype == 1) hipLaunchKernelGGL(k_gram_heavy_build<double>, dim3(g), dim3(256), 0, s, descs);
    else hipLaunchKernelGGL(k_gram_heavy_build<float>, dim3(g), dim3(256), 0, s, descs);
    launch_exclusive_scan(host.lcnt, host.N, host.lbtot, host.lptr, s);
    if (host.dtype == 1) hipLaunchKernelGGL(k_gram_light_scatter<double>, dim3(g), dim3(256), 0, s, descs);
    else hipLaunchKernelGGL(k_gram_light_scatter<float>, dim3(g), dim3(256), 0, s, descs);
}

void launch_gram_heavy_tiles(const MatDesc *descs, int32_t dtype, int32_t hwg, hipStream_t s) {
    if (hwg <= 0) return;
    if (dtype == 1)
        hipLaunchKernelGGL(k_gram_heavy_tiles<double>, dim3((unsigned)hwg), dim3(256), 0, s, descs);
    else
        hipLaunchKernelGGL(k_gram_heavy_tiles<float>, dim3((unsigned)hwg), dim3(256), 0, s, descs);
    hipLaunchKernelGGL(k_gram_heavy_reduce, dim3(kDenseRows * (kDenseRows + 1) / 2), dim3(256), 0, s, descs);
}

int32_t gram_dense_wgs(int64_t N) {
    const int64_t w = (N + 4095) / 4096;
    return (int32_t)(w < 1 ? 1 : (w > 1024 ? 1024 : w));
}

void launch_gram_dense(const MatDesc *descs, int32_t dwg, hipStream_t s) {
    if (dwg <= 0) return;
    hipLaunchKernelGGL(k_gram_dense, dim3((unsigned)dwg), dim3(256), 0, s, descs);
}

void launch_gram_dense_reduce(const MatDesc *descs, int32_t dwg, hipStream_t s) {
    if (dwg <= 0) return;
    hipLaunchKernelGGL(k_gram_dense_reduce, dim3(1), dim3(kDenseRows * kDenseRows), 0, s, descs);
}

// LDS per wave: one accumulator row and the lane-private dense slots (none with the heavy-row
// split, whose dense rows' pairs come from the gathers); per workgroup: the shared tag row, one
// dense-index byte per row and the alignment pad.
static size_t gram_wave_bytes(int32_t M, int32_t acc_bytes, bool slots) {
    return (size_t)M * acc_bytes + (slots ? (size_t)kDenseRows * 64 * acc_bytes : 0);
}

static size_t gram_fixed_bytes(int32_t M) {
    return (size_t)M * sizeof(int32_t) + (((size_t)M + 15) & ~(size_t)15) + 16;
}

int gram_waves(int32_t M, int32_t acc_bytes, size_t lds_limit, bool slots) {
    const size_t fixed = gram_fixed_bytes(M);
    int w = lds_limit > fixed ? (int)((lds_limit - fixed) / gram_wave_bytes(M, acc_bytes, slots)) : 1;
    if (w > 8) w = 8;
    if (w < 1) w = 1;
    return w;
}

size_t gram_lds_bytes(int32_t M, int32_t acc_bytes, int32_t nw, bool slots) {
    return (size_t)nw * gram_wave_bytes(M, acc_bytes, slots) + gram_fixed_bytes(M);
}

void launch_gram(const MatDesc *descs, const int32_t *wp, int64_t nblocks, const int32_t *wp_red, int64_t nblocks_red,
                 int count, int32_t max_waves, size_t lds_bytes, bool heavy, hipStream_t s) {
    if (nblocks <= 0) return;
    if (heavy)
        hipLaunchKernelGGL(k_gram_rows<true>, dim3((unsigned)nblocks), dim3((unsigned)(64 * max_waves)), lds_bytes, s,
                           descs, wp, count);
    else
        hipLaunchKernelGGL(k_gram_rows<false>, dim3((unsigned)nblocks), dim3((unsigned)(64 * max_waves)), lds_bytes,
                           s, descs, wp, count);
    if (nblocks_red > 0)
        hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)nblocks_red), dim3(256), 0, s, descs, wp_red, count);
}

int64_t gram_part_slots(int64_t nnz) {
    // rows longer than the segment length s number at most nnz / s, and each takes at
    // most deg / s + 1 slots
    const int64_t s = gram_seg_len(nnz);
    return nnz > s ? 2 * (nnz / s) + 1 : 0;
}

hipError_t gram_set_attributes(size_t lds_limit) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_gram_rows<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_gram_rows<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit);
    return e;
}

}  // namespace ranky

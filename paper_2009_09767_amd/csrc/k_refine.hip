// k_refine.hip -- one FP64 Rayleigh-Ritz step with the exact operator A A^T.
//
// The mixed-precision path accumulates the Gram matrix in FP32, so its eigenvectors
// U0 carry FP32-size errors.  Projecting the exact operator onto span(U0),
//   H = U0^T (A A^T) U0 = Z^T Z,  Z = A^T U0  (N x k),
// and diagonalising H = Q Theta Q^T gives Ritz pairs U = U0 Q, sigma = sqrt(theta)
// whose values are accurate to second order in U0's error.  Everything here is FP64.
//
// Z is never stored: H = sum over columns j of z_j z_j^T with z_j = sum over column j's
// nonzeros of a_mj U0[m, :].  One workgroup owns one 128 x 128 tile of H and one fixed
// range of columns; per chunk of 16 columns it builds the 128-wide slices of z_j it
// needs in LDS (U0 is small and stays in L2; 16 lanes read one row slice as sixteen
// 16-byte loads, eight nonzeros in flight) and adds their outer products on the FP64
// matrix cores (each wave one 64 x 64 quadrant; a diagonal tile skips its lower one).
// With k <= 128 there is one tile, so every U0 row is gathered once per nonzero.  The
// partial tiles of the column ranges are then added in range order: no floating-point
// atomics, bitwise reproducible.
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kRrTile = 128;    // H tile
constexpr int kRrChunk = 16;    // columns per LDS chunk
constexpr int kRrWgs = 512;     // target workgroups per launch (tiles x column ranges)
constexpr int kRrLd = kRrTile + 2;   // LDS row stride (doubles): 16-byte rows, staggered banks

// Nonzeros of a chunk staged in LDS (row index and value), one chunk ahead; a chunk with
// more reads the rest from memory.
constexpr int kRrStage = 1024;
// Nonzeros of a column whose U0 rows are gathered together; the first kRrNz0 of a chunk's
// column are gathered ahead, during the previous chunk's matrix-core step.
constexpr int kRrNz = 8;
constexpr int kRrNz0 = 4;

// One pair of U0 entries (row, c), (row, c + 1) with c even; an entry at or past k reads
// as zero.  Branch-free (clamped addresses, masked values), so a group's loads all stay in
// flight.  With k even the pair is one aligned 16-byte load.
template <bool kEven>
__device__ __forceinline__ double2 u0_pair(__attribute__((address_space(1))) const double *U0, int64_t row, int32_t k,
                                           int32_t c) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    double2 r;
    if (kEven) {
        const int32_t cc = c < k ? c : 0;
        const d2v v = *reinterpret_cast<__attribute__((address_space(1))) const d2v *>(U0 + row * k + cc);
        r.x = c < k ? v.x : 0.0;
        r.y = c < k ? v.y : 0.0;
    } else {
        const int32_t c0 = c < k ? c : 0, c1 = c + 1 < k ? c + 1 : 0;
        const double x0 = U0[row * k + c0], x1 = U0[row * k + c1];
        r.x = c < k ? x0 : 0.0;
        r.y = c + 1 < k ? x1 : 0.0;
    }
    return r;
}

// z slice of one column: lane t (0..15) of the column's 16 holds entries 2t + 32q, +1
// (q = 0..3) of the 128-wide slice starting at row offset i0 of U0 (k columns).  The
// column's nonzeros [e, e_end) come from the staged copy (index e - base) when the whole
// chunk is staged (a uniform choice), else from memory.
template <typename TV, bool kEven>
__device__ __forceinline__ void rr_build_slices(const int32_t *srow, const double *sval, int32_t base, bool staged,
                                                __attribute__((address_space(1))) const int32_t *rowidx,
                                                __attribute__((address_space(1))) const TV *vals,
                                                __attribute__((address_space(1))) const double *U0, int32_t k,
                                                int32_t e, int32_t e_end, int32_t ia, int32_t ib, bool two,
                                                double2 (&za)[4], double2 (&zb)[4]) {
    for (; e < e_end; e += kRrNz) {
        double av[kRrNz];
        int64_t rw[kRrNz];
        if (staged) {
#pragma unroll
            for (int t = 0; t < kRrNz; ++t) {
                const int32_t li = (e + t < e_end ? e + t : e) - base;
                rw[t] = srow[li];
                av[t] = e + t < e_end ? sval[li] : 0.0;
            }
        } else {
#pragma unroll
            for (int t = 0; t < kRrNz; ++t) {
                const int32_t x = e + t < e_end ? e + t : e;
                rw[t] = rowidx[x];
                const double v = static_cast<double>(vals[x]);
                av[t] = e + t < e_end ? v : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double2 ua[kRrNz];
#pragma unroll
            for (int t = 0; t < kRrNz; ++t) ua[t] = u0_pair<kEven>(U0, rw[t], k, ia + 32 * q);
#pragma unroll
            for (int t = 0; t < kRrNz; ++t) {
                za[q].x = fma(av[t], ua[t].x, za[q].x);
                za[q].y = fma(av[t], ua[t].y, za[q].y);
            }
            if (two) {
                double2 ub[kRrNz];
#pragma unroll
                for (int t = 0; t < kRrNz; ++t) ub[t] = u0_pair<kEven>(U0, rw[t], k, ib + 32 * q);
#pragma unroll
                for (int t = 0; t < kRrNz; ++t) {
                    zb[q].x = fma(av[t], ub[t].x, zb[q].x);
                    zb[q].y = fma(av[t], ub[t].y, zb[q].y);
                }
            }
        }
    }
}

// workgroup b -> tile t = b / R (ta <= tb, row-major over the upper triangle), range b % R.
// Z is double-buffered in LDS: iteration q issues the U0 gathers of chunk q + 1's first
// nonzeros, runs the matrix-core step of chunk q while they are in flight, then finishes
// chunk q + 1's slices; the nonzeros of chunk q + 2 are staged meanwhile.  One barrier per
// chunk.
template <typename TV, bool kEven>
__global__ __launch_bounds__(256) void k_rr_syrk(const int32_t *__restrict__ colptr_, const int32_t *__restrict__ rowidx_,
                                                 const TV *__restrict__ vals_, int64_t N, int32_t k, int32_t R,
                                                 const double *__restrict__ U0_, double *__restrict__ part) {
    constexpr int kZ = 2 * kRrChunk * kRrLd;     // one chunk's slices A and B
    __shared__ double Z[2 * kZ];                 // chunk q in Z[(q & 1) kZ ..]
    __shared__ int32_t Srow[2][kRrStage];
    __shared__ double Sval[2][kRrStage];
    const auto colptr = gmem(colptr_);
    const auto rowidx = gmem(rowidx_);
    const auto vals = gmem(vals_);
    const auto U0 = gmem(U0_);
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
    const bool two = ta != tb;
    const int64_t c_begin = (N * r) / R, c_end = (N * (r + 1)) / R;
    const int64_t nchunks = (c_end - c_begin + kRrChunk - 1) / kRrChunk;
    // build: thread -> column bc of the chunk, lane bt of its 16
    const int bc = tid >> 4, bt = tid & 15;
    const int32_t ia = ta * kRrTile + 2 * bt, ib = tb * kRrTile + 2 * bt;
    // this wave's 64 x 64 quadrant (qa, qb); a diagonal tile needs (0,0), (0,1), (1,1)
    const int qa = two ? (wave >> 1) : (wave == 2 ? 1 : 0);
    const int qb = two ? (wave & 1) : (wave == 0 ? 0 : 1);
    const bool mm = two || wave < 3;
    const int zb_off = two ? kRrChunk * kRrLd : 0;
    // chunk q: columns [c_begin + 16 q, min(+16, c_end)); its nonzeros [lo(q), hi(q))
    auto col_lo = [&](int64_t q) { return c_begin + q * kRrChunk; };
    auto col_hi = [&](int64_t q) { return c_begin + q * kRrChunk + kRrChunk < c_end ? c_begin + q * kRrChunk + kRrChunk : c_end; };
    auto range = [&](int64_t q, int32_t &lo, int32_t &hi) {
        lo = hi = 0;
        if (q < nchunks) {
            lo = colptr[col_lo(q)];
            hi = colptr[col_hi(q)];
        }
    };
    auto bounds = [&](int64_t q, int32_t &eb, int32_t &ee) {
        eb = ee = 0;
        if (q < nchunks && col_lo(q) + bc < col_hi(q)) {
            eb = colptr[col_lo(q) + bc];
            ee = colptr[col_lo(q) + bc + 1];
        }
    };
    auto write_z = [&](double *zbuf, const double2 (&za)[4], const double2 (&zb)[4]) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            *reinterpret_cast<double2 *>(&zbuf[bc * kRrLd + 2 * bt + 32 * x]) = za[x];
            if (two) *reinterpret_cast<double2 *>(&zbuf[kRrChunk * kRrLd + bc * kRrLd + 2 * bt + 32 * x]) = zb[x];
        }
    };
    d4 acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    // acc += A^T B over one chunk: A[row][c] = slice A[c][row], B[c][col] = slice B (or A)[c][col]
    auto mfma_chunk = [&](const double *zbuf) {
#pragma unroll
        for (int kc = 0; kc < kRrChunk / 4; ++kc) {
            const int c = kc * 4 + (l >> 4);
            double a[4], b[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                a[x] = zbuf[c * kRrLd + 64 * qa + 16 * x + (l & 15)];
                b[x] = zbuf[zb_off + c * kRrLd + 64 * qb + 16 * x + (l & 15)];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    };
    if (nchunks <= 0) goto write_out;
    {
        // prologue: chunk 0 staged and built into Z[0]; chunk 1 staged
        int32_t lo0, hi0, lo1, hi1, lo2, hi2, eb0, ee0, eb1, ee1;
        range(0, lo0, hi0);
        for (int32_t x = tid; x < hi0 - lo0 && x < kRrStage; x += 256) {
            Srow[0][x] = rowidx[lo0 + x];
            Sval[0][x] = static_cast<double>(vals[lo0 + x]);
        }
        bounds(0, eb0, ee0);
        range(1, lo1, hi1);
        __syncthreads();
        {
            double2 za[4], zb[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) za[x] = zb[x] = make_double2(0.0, 0.0);
            rr_build_slices<TV, kEven>(Srow[0], Sval[0], lo0, hi0 - lo0 <= kRrStage, rowidx, vals, U0, k, eb0, ee0, ia,
                                       ib, two, za, zb);
            write_z(Z, za, zb);
        }
        for (int32_t x = tid; x < hi1 - lo1 && x < kRrStage; x += 256) {
            Srow[1][x] = rowidx[lo1 + x];
            Sval[1][x] = static_cast<double>(vals[lo1 + x]);
        }
        bounds(1, eb1, ee1);
        range(2, lo2, hi2);
        __syncthreads();
        for (int64_t q = 0; q < nchunks; ++q) {
            const int zq = (int)(q & 1), zn = zq ^ 1;
            // chunk q + 1's first kRrNz0 nonzeros of this thread's column (empty: row 0, weight 0)
            const bool st1 = hi1 - lo1 <= kRrStage;
            int32_t rw[kRrNz0];
            double av[kRrNz0];
#pragma unroll
            for (int u = 0; u < kRrNz0; ++u) {
                const bool in = eb1 + u < ee1;
                const int32_t x = in ? eb1 + u : 0;
                int32_t rr;
                double vv;
                if (st1) {
                    const int32_t li = in ? x - lo1 : 0;
                    rr = Srow[zn][li];
                    vv = Sval[zn][li];
                } else {
                    rr = rowidx[x];
                    vv = static_cast<double>(vals[x]);
                }
                rw[u] = in ? rr : 0;
                av[u] = in ? vv : 0.0;
            }
            double2 ua[4][kRrNz0], ub[4][kRrNz0];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int u = 0; u < kRrNz0; ++u) ua[x][u] = u0_pair<kEven>(U0, rw[u], k, ia + 32 * x);
            if (two) {
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int u = 0; u < kRrNz0; ++u) ub[x][u] = u0_pair<kEven>(U0, rw[u], k, ib + 32 * x);
            }
            // chunk q + 2's nonzeros (staged after the step) and the next bounds
            const int32_t st2 = hi2 - lo2 < kRrStage ? hi2 - lo2 : kRrStage;
            int32_t pr[kRrStage / 256];
            double pv[kRrStage / 256];
#pragma unroll
            for (int i = 0; i < kRrStage / 256; ++i) {
                const int32_t x = tid + 256 * i;
                const int32_t at = x < st2 ? lo2 + x : 0;   // entry 0 exists (the matrix has a nonzero)
                pr[i] = rowidx[at];
                pv[i] = static_cast<double>(vals[at]);
            }
            int32_t eb2, ee2, lo3, hi3;
            bounds(q + 2, eb2, ee2);
            range(q + 3, lo3, hi3);
            // the matrix-core step of chunk q while the gathers are in flight
            if (mm) mfma_chunk(Z + zq * kZ);
            // chunk q + 1's slices: the first nonzeros from the registers, the rest from memory
            double2 za[4], zb[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                za[x] = zb[x] = make_double2(0.0, 0.0);
#pragma unroll
                for (int u = 0; u < kRrNz0; ++u) {
                    za[x].x = fma(av[u], ua[x][u].x, za[x].x);
                    za[x].y = fma(av[u], ua[x][u].y, za[x].y);
                    if (two) {
                        zb[x].x = fma(av[u], ub[x][u].x, zb[x].x);
                        zb[x].y = fma(av[u], ub[x][u].y, zb[x].y);
                    }
                }
            }
            rr_build_slices<TV, kEven>(Srow[zn], Sval[zn], lo1, st1, rowidx, vals, U0, k, eb1 + kRrNz0, ee1, ia, ib,
                                       two, za, zb);
            write_z(Z + zn * kZ, za, zb);
#pragma unroll
            for (int i = 0; i < kRrStage / 256; ++i) {
                const int32_t x = tid + 256 * i;
                if (x < st2) {
                    Srow[zq][x] = pr[i];
                    Sval[zq][x] = pv[i];
                }
            }
            __syncthreads();
            lo1 = lo2;
            hi1 = hi2;
            lo2 = lo3;
            hi2 = hi3;
            eb1 = eb2;
            ee1 = ee2;
        }
    }
write_out:
    // result layout: element i of lane l at row l / 16 + 4 i, column l % 16 of a 16 x 16 block
    if (!mm) return;
    const auto out = gmem(part) + (int64_t)blockIdx.x * kRrTile * kRrTile;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 64 * qa + 16 * x + (l >> 4) + 4 * i, col = 64 * qb + 16 * y + (l & 15);
                out[row * kRrTile + col] = acc[x][y][i];
            }
}

// H[a][b] = H[b][a] = sum over the column ranges (in order) of the partial tiles; the
// entry (a, b), a <= b, of a diagonal tile is used for both halves.  Zero outside k x k.
// A workgroup takes 64 consecutive entries (lanes) and cuts the R ranges into 16
// contiguous segments (waves); the segment sums are added in segment order.
__global__ __launch_bounds__(1024) void k_rr_syrk_reduce(const double *__restrict__ part_, int32_t k, int32_t R,
                                                         int32_t npad, double *__restrict__ H_) {
    __shared__ double seg_sum[16][64];
    const auto part = gmem(part_);
    const auto H = gmem(H_);
    const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int32_t T = (k + kRrTile - 1) / kRrTile;
    const int64_t total = (int64_t)npad * npad;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    const int32_t a = e < total ? (int32_t)(e / npad) : 0, b = e < total ? (int32_t)(e % npad) : 0;
    const bool live = e < total && a <= b && b < k;
    double v = 0.0;
    if (live) {
        const int32_t ta = a / kRrTile, tb = b / kRrTile;
        const int32_t t = ta * T - ta * (ta - 1) / 2 + (tb - ta);
        const auto p = part + ((int64_t)t * R) * kRrTile * kRrTile + (a % kRrTile) * kRrTile + (b % kRrTile);
        const int32_t per = (R + 15) / 16, r0 = seg * per < R ? seg * per : R, r1 = r0 + per < R ? r0 + per : R;
        int32_t r = r0;
        for (; r + 4 <= r1; r += 4) {
            const double x0 = p[(int64_t)r * kRrTile * kRrTile], x1 = p[(int64_t)(r + 1) * kRrTile * kRrTile];
            const double x2 = p[(int64_t)(r + 2) * kRrTile * kRrTile], x3 = p[(int64_t)(r + 3) * kRrTile * kRrTile];
            v += x0;
            v += x1;
            v += x2;
            v += x3;
        }
        for (; r < r1; ++r) v += p[(int64_t)r * kRrTile * kRrTile];
    }
    seg_sum[seg][lane] = v;
    __syncthreads();
    if (seg != 0 || e >= total || a > b) return;
    double sum = 0.0;
    for (int g = 0; g < 16; ++g) sum += seg_sum[g][lane];
    H[(int64_t)a * npad + b] = sum;
    H[(int64_t)b * npad + a] = sum;
}

// U[:, i] = U0 Q[:, perm[i]] with the sign rule (largest-magnitude entry positive,
// lowest row on a tie).  One workgroup per output column; Q's column is staged in LDS.
__global__ __launch_bounds__(256) void k_rr_apply(const double *__restrict__ U0, const double *__restrict__ Q,
                                                  int64_t ldq, const int32_t *__restrict__ perm, int32_t M,
                                                  int32_t k, double *__restrict__ U, float *__restrict__ Uf) {
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
    // every wave reads the pivot before any wave flips it (the pivot row is one of the rows
    // flipped below)
    const bool flip = U[(int64_t)top * k + i] < 0.0;
    __syncthreads();
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) {
        const double u = flip ? -U[(int64_t)m * k + i] : U[(int64_t)m * k + i];
        if (flip) U[(int64_t)m * k + i] = u;
        if (Uf) Uf[(int64_t)m * k + i] = (float)u;
    }
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
    const bool even = (k & 1) == 0;
    if (A.dtype == 1) {
        const double *v = static_cast<const double *>(A.values);
        if (even) hipLaunchKernelGGL((k_rr_syrk<double, true>), dim3(blocks), dim3(256), 0, s, A.colptr, A.rowidx, v, N, k, R, U0, part);
        else hipLaunchKernelGGL((k_rr_syrk<double, false>), dim3(blocks), dim3(256), 0, s, A.colptr, A.rowidx, v, N, k, R, U0, part);
    } else {
        const float *v = static_cast<const float *>(A.values);
        if (even) hipLaunchKernelGGL((k_rr_syrk<float, true>), dim3(blocks), dim3(256), 0, s, A.colptr, A.rowidx, v, N, k, R, U0, part);
        else hipLaunchKernelGGL((k_rr_syrk<float, false>), dim3(blocks), dim3(256), 0, s, A.colptr, A.rowidx, v, N, k, R, U0, part);
    }
    const int64_t rb = ((int64_t)npad * npad + 63) / 64;
    hipLaunchKernelGGL(k_rr_syrk_reduce, dim3((unsigned)rb), dim3(1024), 0, s, part, k, R, npad, H);
}

void launch_rr_apply(const double *U0, const double *Q, int64_t ldq, const int32_t *perm, int32_t M, int32_t k,
                     double *U, float *Uf, hipStream_t s) {
    hipLaunchKernelGGL(k_rr_apply, dim3((unsigned)k), dim3(256), sizeof(double) * (size_t)k, s, U0, Q, ldq, perm, M,
                       k, U, Uf);
}

}  // namespace ranky

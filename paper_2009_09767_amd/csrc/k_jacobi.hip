// k_jacobi.hip -- FP64 two-sided blocked Jacobi eigensolver of the Gram matrix.
//
// The SVD of the proxy matrix P (Sec. III, last step of Alg. 1) is, in Gram form,
// the eigendecomposition G = W Lambda W^T of G = P P^T.  Jacobi keeps relative
// accuracy in the small eigenvalues, which the rank decision relies on.
//
// Layout: G (two ping-pong copies) and W are npad x npad row-major, npad a multiple
// of 32; indices >= n are zero padding that no rotation touches (their couplings
// stay exactly zero).  G is scaled by a power of two at the start (max |g_ii| in
// [1/2, 1)), so the rotation formulas below can neither overflow nor underflow; the
// eigenvalues are scaled back when they are read out.  The index range is cut into
// nb = npad / 16 blocks; one sweep is nb - 1 rounds of a round-robin tournament on
// the blocks, and in a round the nb / 2 block pairs are disjoint.  Every round is
// ONE launch of k_jround:
//   * workgroups [0, npairs) solve the round's 32 x 32 subproblems S = M_r[s, s]
//     (s = the pair's two blocks) with one cyclic Jacobi sweep in LDS and write the
//     rotation J (32 x 32) and the rotated S.  The sweep is full (all 496 pairs, 31
//     steps) in about every quarter of the rounds, round 0 included, and covers only
//     the 256 pairs joining the two blocks (16 steps) in the others: every pair of
//     indices is still rotated at least once per sweep of the whole matrix, while the
//     pairs inside a block are not swept again in every round.  The diagonal blocks of S are the
//     previous round's rotated subproblems, the off-diagonal block is
//     J_a^T M_{r-1}[s_a, s_b] J_b, so no workgroup waits for the update.
//   * the other workgroups apply the previous round, one 32 x 32 tile per wave on the
//     FP64 matrix cores: M_r = Jp^T M_{r-1} Jp tile by tile into the other G buffer
//     (the diagonal tiles are the rotated subproblems themselves), W <- W Jp in place.
// A flush launch (update only) ends every sweep; k_jcheck then tests every
// off-diagonal entry: g_pq is rotated iff |g_pq| > floor and g_pq^2 > tol^2 |g_pp g_qq|,
// tol = max(1e-15, sqrt(n) eps), floor = (n eps)^2 max|g_ii| (the solve uses the same
// test, so the two can never disagree).
//
// Rotation of the pair (p, q), d = g_qq - g_pp, a = 2 g_pq, h = sqrt(d^2 + a^2),
// w = |d| + h: the smaller-angle rotation has c = sqrt(w / (2h)), s = sign(d) a / sqrt(2hw)
// and tangent t = s / c = sign(d) a / w (sign(0) = +1); then g_pp -= t g_pq,
// g_qq += t g_pq, g_pq = 0.  Rows: r_p <- c r_p - s r_q, r_q <- s r_p + c r_q; columns
// likewise; J <- J R.
//
// Inside a subproblem the 16 pairs of a step sit at fixed positions (i, 31 - i); after
// every step the positions turn one place (the round-robin of the 32 indices), which
// the step folds into where it writes, so every thread's LDS addresses are fixed for
// the whole sweep and after 31 steps the positions are the indices again.  S lives in
// LDS as one triangle, ping-pong between two buffers (one barrier per step).  Waves 0
// and 1 rotate the 120 off-diagonal 2 x 2 blocks, wave 2 the 16 diagonal blocks (and
// records every rotation of the sweep), wave 3 holds one row of J per lane in
// registers and applies step k's rotations while step k + 1 runs.
#include <algorithm>
#include <cstring>

#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

constexpr int kB = 16;           // block of indices
constexpr int kP = 32;           // subproblem = two blocks
constexpr int kPS = 33;          // LDS row stride of 32-wide tiles
constexpr int kSteps = kP - 1;   // steps of a full sweep over a subproblem (all 496 pairs)
constexpr int kCrossSteps = kB;  // steps of a cross sweep (the 256 pairs joining the two blocks)
constexpr int kTileWaves = 4;    // update tiles per workgroup (one per wave)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Round r of the round-robin tournament on `players` (even) seats: seat 0 stays, the
// others turn one place per round; pair i joins seat i and seat players-1-i.
__device__ __forceinline__ int seat_block(int players, int r, int seat) {
    return seat == 0 ? 0 : 1 + (seat - 1 + r) % (players - 1);
}
__device__ __forceinline__ void tournament_pair(int players, int r, int i, int &a, int &b) {
    a = seat_block(players, r, i);
    b = seat_block(players, r, players - 1 - i);
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
}
// Where block X sat in round r: its pair and whether it was the larger block of it.
__device__ __forceinline__ void block_seat(int players, int r, int X, int &pair, int &half) {
    const int ring = players - 1;
    const int seat = X == 0 ? 0 : 1 + (((X - 1 - r) % ring) + ring) % ring;
    pair = seat < players - seat ? seat : players - 1 - seat;
    const int other = seat_block(players, r, players - 1 - seat);
    half = X > other ? 1 : 0;
}

// global index of position l (0..31) of the super-block made of blocks (P, Q)
__device__ __forceinline__ int gidx(int l, int P, int Q) { return l < kB ? P * kB + l : Q * kB + (l - kB); }

// Per-matrix arguments of one round launch (a table of these covers a batch).
struct RoundArgs {
    const double *Gin;     // M_{r-1}; set in-kernel for the update part
    double *Gout;          // receives M_r = Jp^T M_{r-1} Jp (update part); set in-kernel
    double *G0, *G1;       // the two G buffers
    double *W;             // eigenvectors, updated in place by Jp
    int64_t ld;
    int32_t nb;            // blocks
    int32_t round_cur;     // pairing of the subproblems solved now (if do_solve)
    int32_t round_prev;    // pairing of the previous round (if has_prev)
    int32_t has_prev, do_solve;
    const double *Jprev;   // [npairs][32][32]
    const int32_t *fprev;  // [npairs] 1 if Jprev[i] is not the identity
    const double *Sprev;   // [npairs][32][32] rotated subproblems of the previous round
    double *Jcur;
    int32_t *fcur;
    double *Scur;
    const double *sdbl;
    const int32_t *jstate; // sweeps done / active (device state of this matrix)
    double tol;
    int32_t inner_sweeps;
    int32_t cross;         // 1: the solve sweeps only the pairs that join the two blocks
    int32_t ntiles_g;      // npairs (npairs + 1) / 2
    int32_t nrowtiles;     // npad / 32
    int32_t sched;         // bit 0: update tiles grouped per XCD (see k_jround); bit 1 is host-side
};

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- subproblem solve -------------------------------------------------------

// One FP64 MFMA 16 x 16 x 4 step: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// element i of lane l's result is C[l / 16 + 4 i][l % 16].
__device__ __forceinline__ d4 mfma4(double x, double y, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

// position after one step of the in-subproblem round-robin
__device__ __forceinline__ int turn(int p) { return p == 0 ? 0 : (p == 1 ? kP - 1 : p - 1); }
// cross sweep: the first block's positions stay, the second block's shift by one
__device__ __forceinline__ int turn_cross(int p) { return p < kB ? p : kB + ((p - kB + kB - 1) & (kB - 1)); }
// one-triangle storage of a symmetric 32 x 32 tile
__device__ __forceinline__ int sym(int a, int b) { return a < b ? a * kPS + b : b * kPS + a; }
// index that sits at position `seat` after r steps
__device__ __forceinline__ constexpr int pos_index(int seat, int r) { return seat == 0 ? 0 : 1 + (seat - 1 + r) % 31; }

// 1/sqrt(x) for a normal x > 0 (every input below): the hardware estimate and one
// third-order correction, e = 1 - x y^2, y (1 + e/2 + 3e^2/8); within 1 ulp like the
// library rsqrt (measured over 4M values in [1e-70, 1e2]) with three fewer dependent
// steps, as it skips the special-value handling.
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// The rotation of one pair; c = 1, s = t = 0 when the pair passes the test.
__device__ __forceinline__ bool pair_rotation(double app, double aqq, double apq, double tol2, double floor_abs,
                                              double &c, double &s, double &t) {
#pragma clang fp contract(off)
    const bool act = fabs(apq) > floor_abs && apq * apq > tol2 * fabs(app * aqq);
    const double d = aqq - app, a = 2.0 * apq;
    const double x2 = act ? fma(d, d, a * a) : 1.0;
    const double h = x2 * rsqrt_pos(x2);
    const double w = fabs(d) + h;
    const double q = rsqrt_pos((2.0 * h) * w);
    const double sa = d >= 0.0 ? a : -a;
    c = act ? w * q : 1.0;
    s = act ? sa * q : 0.0;
    t = act ? s * ((2.0 * h) * q) : 0.0;
    return act;
}

// J row (in registers) <- row * R_K for the 16 rotations of step K.
template <int K>
__device__ __forceinline__ void jrow_step(double (&jr)[kP], const double2 *__restrict__ cs) {
#pragma unroll
    for (int i = 0; i < kP / 2; ++i) {
        const int x = pos_index(i, K), y = pos_index(kP - 1 - i, K);
        const double2 r = cs[i];
        const double u = jr[x], v = jr[y];
        jr[x] = r.x * u - r.y * v;
        jr[y] = r.y * u + r.x * v;
    }
}
// Step K's rotations are applied after the barrier that ends step K; one barrier
// between consecutive steps (kSteps - 1 in all).
template <int K>
__device__ __forceinline__ void jrow_sweep(double (&jr)[kP], const double2 (*tab)[kP / 2]) {
    if constexpr (K < kSteps) {
        jrow_step<K>(jr, tab[K]);
        if constexpr (K + 1 < kSteps) {
            __syncthreads();
            jrow_sweep<K + 1>(jr, tab);
        }
    }
}

// Cross sweep: step K pairs index i (first block) with index 16 + (i + K) mod 16.
template <int K>
__device__ __forceinline__ void jrow_step_cross(double (&jr)[kP], const double2 *__restrict__ cs) {
#pragma unroll
    for (int i = 0; i < kB; ++i) {
        const int x = i, y = kB + ((i + K) & (kB - 1));
        const double2 r = cs[i];
        const double u = jr[x], v = jr[y];
        jr[x] = r.x * u - r.y * v;
        jr[y] = r.y * u + r.x * v;
    }
}
template <int K>
__device__ __forceinline__ void jrow_sweep_cross(double (&jr)[kP], const double2 (*tab)[kP / 2]) {
    if constexpr (K < kCrossSteps) {
        jrow_step_cross<K>(jr, tab[K]);
        if constexpr (K + 1 < kCrossSteps) {
            __syncthreads();
            jrow_sweep_cross<K + 1>(jr, tab);
        }
    }
}

// LDS of a solve workgroup (doubles): S0 | S1 | rotation table [31][16] | per-wave (c, s).
// The build of S uses the table area for the partial product P_1 (16 x 16).
constexpr int kSoS1 = kP * kPS, kSoTab = 2 * kP * kPS, kSoWcs = kSoTab + 2 * kSteps * (kP / 2),
              kSoEnd = kSoWcs + 2 * 2 * (kP / 2);
constexpr int kSmemDoubles = kTileWaves * kP * kPS;
static_assert(kSoEnd + 2 <= kSmemDoubles, "solve LDS (and the four votes) fits the update LDS");
static_assert(kB * kB <= 2 * kSteps * (kP / 2), "P_1 fits the table area");

__device__ __forceinline__ void solve_pair(const RoundArgs &a, int pair, int32_t launch_r, double *smem) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double *S0 = smem, *S1 = smem + kSoS1;
    double2(*tab)[kP / 2] = reinterpret_cast<double2(*)[kP / 2]>(smem + kSoTab);
    double2(*wcs)[kP / 2] = reinterpret_cast<double2(*)[kP / 2]>(smem + kSoWcs);
    int P, Q;
    tournament_pair(a.nb, a.round_cur, pair, P, Q);

    // ---- build S (upper triangle) ----
    // Every global load of the build is issued before the first wait: the sweep state
    // (it says which G buffer holds M_{r-1}), the tile from both G buffers, the two
    // diagonal blocks and the J slices (the previous round stored J for every pair,
    // the identity included), so the build costs one memory round trip.  With a
    // previous round, the off-diagonal block J_pp[:, hp]^T M_{r-1}[s_pp, s_pq] J_pq[:, hq]
    // is two products on the FP64 matrix cores: wave w (0, 1) takes tile rows
    // 16w .. 16w + 15, U_w = T_w JB (k = 32) and P_w = JA_w^T U_w (k = 16, U_w stays in
    // registers: the product's result layout is the next product's B layout), and
    // S_PQ = P_0 + P_1.  Waves 2 and 3 bring the diagonal blocks.
    const int32_t active = gmem(a.jstate)[kJsActive], sweeps = gmem(a.jstate)[kJsSweeps];
    const double floor_abs = gmem(a.sdbl)[kSdFloor];   // loaded with the build, used by the test
    const int l16 = lane & 15, l4 = lane >> 4;
    // the sweep's fixed indices and J = I, set up while the build's loads are in flight
    const bool cross = a.cross != 0;
    // A full sweep rotates the 16 pairs at positions (i, 31 - i) in each of 31 steps (all
    // 496 pairs); a cross sweep rotates (i, 16 + i) in each of 16 steps (the 256 pairs
    // that join the two blocks).  After every step the positions turn (full: round-robin
    // of positions 1..31; cross: the second block's positions shift by one), which the
    // step folds into where it writes.  Every lane works: lanes without a block of their
    // own repeat another lane's block and write the same values to the same places.
    const int nsteps = cross ? kCrossSteps : kSteps;
    // rotation lanes: lane & 15 reads pair (rP, rQ) of the step (rP < rQ)
    const int rP = lane & 15, rQ = cross ? rP + kB : kP - 1 - rP;
    const int aPP = rP * kPS + rP, aQQ = rQ * kPS + rQ, aPQ = rP * kPS + rQ;
    // off-diagonal block (bi < bj) of waves 0-1, numbered row by row (row i holds 15 - i
    // blocks and starts at 15 i - i (i - 1) / 2); diagonal block rP of wave 2
    int bi = 0, bj = 1;
    if (wave < 2) {
        const int b = tid < 120 ? tid : 0;
        int i = 0;
#pragma unroll
        for (int r = 1; r < kB; ++r) i += b >= 15 * r - r * (r - 1) / 2 ? 1 : 0;
        bi = i;
        bj = i + 1 + (b - (15 * i - i * (i - 1) / 2));
    }
    const int Pi = wave == 2 ? rP : bi, Pj = bj;
    const int Qi = cross ? Pi + kB : kP - 1 - Pi, Qj = cross ? Pj + kB : kP - 1 - Pj;
    const int tPi = cross ? turn_cross(Pi) : turn(Pi), tQi = cross ? turn_cross(Qi) : turn(Qi);
    const int tPj = cross ? turn_cross(Pj) : turn(Pj), tQj = cross ? turn_cross(Qj) : turn(Qj);
    const int b00 = sym(Pi, Pj), b01 = sym(Pi, Qj), b10 = sym(Qi, Pj), b11 = sym(Qi, Qj);
    const int w00 = sym(tPi, tPj), w01 = sym(tPi, tQj), w10 = sym(tQi, tPj), w11 = sym(tQi, tQj);
    const int dPP = tPi * kPS + tPi, dQQ = tQi * kPS + tQi, dPQ = sym(tPi, tQi);
    double jr[kP];
#pragma unroll
    for (int c = 0; c < kP; ++c) jr[c] = c == (lane & 31) ? 1.0 : 0.0;
    double *Sfin = (nsteps & 1) ? S1 : S0;   // where the sweep leaves S
    double g0[8], g1[8], jb[8], ja[4], dg[4];
    int pp = 0, hp = 0, pq = 0, hq = 0;
    if (!a.has_prev) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + 256 * j, x = e >> 5, y = e & 31;
            g0[j] = g1[j] = 0.0;
            if (x <= y) {
                const int64_t off = (int64_t)gidx(x, P, Q) * a.ld + gidx(y, P, Q);
                g0[j] = gmem(a.G0)[off];
                g1[j] = gmem(a.G1)[off];
            }
        }
    } else {
        block_seat(a.nb, a.round_prev, P, pp, hp);
        block_seat(a.nb, a.round_prev, Q, pq, hq);
        if (wave < 2) {
            int Pa, Qa, Pb, Qb;
            tournament_pair(a.nb, a.round_prev, pp, Pa, Qa);
            tournament_pair(a.nb, a.round_prev, pq, Pb, Qb);
            // U_w: step q's contraction index for lane group l4 is k = 8 l4 + q, so each
            // lane reads 8 consecutive entries of its T row (one block: 8 divides 16)
            const int64_t off = (int64_t)gidx(16 * wave + l16, Pa, Qa) * a.ld + gidx(8 * l4, Pb, Qb);
            const auto t0 = reinterpret_cast<__attribute__((address_space(1))) const d2 *>(gmem(a.G0) + off);
            const auto t1 = reinterpret_cast<__attribute__((address_space(1))) const d2 *>(gmem(a.G1) + off);
            const auto jpa = gmem(a.Jprev) + (int64_t)pp * kP * kP + hp * kB + l16;
            const auto jpb = gmem(a.Jprev) + (int64_t)pq * kP * kP + hq * kB + l16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const d2 x0 = t0[v], x1 = t1[v];   // T[16w + l16][8 l4 + 2v, + 1]
                g0[2 * v] = x0.x;
                g0[2 * v + 1] = x0.y;
                g1[2 * v] = x1.x;
                g1[2 * v + 1] = x1.y;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) jb[q] = jpb[(8 * l4 + q) * kP];   // JB[8 l4 + q][l16]
#pragma unroll
            for (int q = 0; q < 4; ++q) ja[q] = jpa[(16 * wave + 4 * q + l4) * kP];   // JA[16w + 4q + l4][l16]
        } else {
            // diagonal blocks: the previous round's rotated subproblems (upper triangles)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int e = tid - 128 + 128 * j, x = e >> 4, y = e & 15;
                dg[j] = dg[2 + j] = 0.0;
                if (x <= y) {
                    dg[j] = gmem(a.Sprev)[(int64_t)pp * kP * kP + (hp * kB + x) * kP + hp * kB + y];
                    dg[2 + j] = gmem(a.Sprev)[(int64_t)pq * kP * kP + (hq * kB + x) * kP + hq * kB + y];
                }
            }
        }
    }
    if (active == 0) return;
    // G buffer holding M_{r-1}: one flip per launch with a previous round, nb - 1 per sweep
    const bool odd = ((sweeps * (a.nb - 1) + (launch_r > 0 ? launch_r - 1 : 0)) & 1) != 0;
    if (!a.has_prev) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + 256 * j, x = e >> 5, y = e & 31;
            if (x <= y) S0[x * kPS + y] = odd ? g1[j] : g0[j];
        }
    } else {
        double *part = smem + kSoTab;   // P_1, 16 x 16
        d4 pw = {0.0, 0.0, 0.0, 0.0};
        if (wave < 2) {
            d4 u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 8; ++q) u = mfma4(odd ? g1[q] : g0[q], jb[q], u);
#pragma unroll
            for (int q = 0; q < 4; ++q) pw = mfma4(ja[q], u[q], pw);
            if (wave == 1) {
#pragma unroll
                for (int i = 0; i < 4; ++i) part[(l4 + 4 * i) * kB + l16] = pw[i];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int e = tid - 128 + 128 * j, x = e >> 4, y = e & 15;
                if (x <= y) {
                    S0[x * kPS + y] = dg[j];
                    S0[(kB + x) * kPS + kB + y] = dg[2 + j];
                }
            }
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) S0[(l4 + 4 * i) * kPS + kB + l16] = pw[i] + part[(l4 + 4 * i) * kB + l16];
        }
    }
    __syncthreads();

    const double tol2 = a.tol * a.tol;
    // a subproblem whose entries to be swept all pass the rotation test is left as is
    // (a cross sweep's 256 entries one per thread, a full sweep's four candidates per
    // thread, loads issued at once; one vote per wave, one barrier)
    {
        bool bad = false;
        if (cross) {
            const int x = tid >> 4, y = kB + (tid & 15);
            const double g = S0[x * kPS + y], gx = S0[x * kPS + x], gy = S0[y * kPS + y];
            // `&`, not `&&`: all three loads leave before the first compare
            bad = (fabs(g) > floor_abs) & (g * g > tol2 * fabs(gx * gy));
        } else {
            double g[4], gx[4], gy[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = tid + 256 * j, x = e >> 5, y = e & 31;
                g[j] = S0[sym(x, y)];
                gx[j] = S0[x * kPS + x];
                gy[j] = S0[y * kPS + y];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int e = tid + 256 * j, x = e >> 5, y = e & 31;
                bad |= (x < y) & (fabs(g[j]) > floor_abs) & (g[j] * g[j] > tol2 * fabs(gx[j] * gy[j]));
            }
        }
        int32_t *vote = reinterpret_cast<int32_t *>(smem + kSoEnd);
        const bool wave_bad = __ballot(bad) != 0;
        if (lane == 0) vote[wave] = wave_bad;
        __syncthreads();
        const bool any_bad = (vote[0] | vote[1] | vote[2] | vote[3]) != 0;
        if (!any_bad) {
            for (int e = tid; e < kP * kP; e += 256) {
                const int x = e >> 5, y = e & 31;
                __builtin_nontemporal_store(S0[sym(x, y)], &gmem(a.Scur)[(int64_t)pair * kP * kP + e]);
                __builtin_nontemporal_store(x == y ? 1.0 : 0.0, &gmem(a.Jcur)[(int64_t)pair * kP * kP + e]);
            }
            if (tid == 0) gmem(a.fcur)[pair] = 0;
            return;
        }
    }

    // ---- sweep ----
    int rotated = 0;
    for (int sw = 0; sw < a.inner_sweeps; ++sw) {
        int rot = 0;
        if (wave == 3) {
            __syncthreads();   // end of step 0; the sweep holds the other nsteps - 1 barriers
            if (cross) jrow_sweep_cross<0>(jr, tab);
            else jrow_sweep<0>(jr, tab);
        } else {
            // each role issues its own loads and computes the rotation in its own branch
            // (one straight path per wave and step)
            for (int k = 0; k < nsteps; ++k) {
                const double *__restrict__ Sc = (k & 1) ? S1 : S0;
                double *__restrict__ Sn = (k & 1) ? S0 : S1;
                if (wave == 2) {
                    const double app = Sc[aPP], aqq = Sc[aQQ], apq = Sc[aPQ];
                    double c, s, t;
                    const bool act = pair_rotation(app, aqq, apq, tol2, floor_abs, c, s, t);
                    rot |= act;
                    tab[k][rP] = make_double2(c, s);
                    Sn[dPP] = fma(-t, apq, app);
                    Sn[dQQ] = fma(t, apq, aqq);
                    Sn[dPQ] = act ? 0.0 : apq;
                } else {
                    const double x00 = Sc[b00], x01 = Sc[b01], x10 = Sc[b10], x11 = Sc[b11];
                    const double app = Sc[aPP], aqq = Sc[aQQ], apq = Sc[aPQ];
                    double c, s, t;
                    pair_rotation(app, aqq, apq, tol2, floor_abs, c, s, t);
                    wcs[wave][rP] = make_double2(c, s);
                    wave_fence();
                    const double2 ri = wcs[wave][bi], rj = wcs[wave][bj];
                    const double y00 = ri.x * x00 - ri.y * x10, y01 = ri.x * x01 - ri.y * x11;
                    const double y10 = ri.y * x00 + ri.x * x10, y11 = ri.y * x01 + ri.x * x11;
                    Sn[w00] = rj.x * y00 - rj.y * y01;
                    Sn[w01] = rj.y * y00 + rj.x * y01;
                    Sn[w10] = rj.x * y10 - rj.y * y11;
                    Sn[w11] = rj.y * y10 + rj.x * y11;
                }
                __syncthreads();
            }
        }
        if (a.inner_sweeps == 1) {
            // only wave 2 records rotations; the other waves need no further barrier (the
            // last step's barrier published S, and wave 3 finishes J on its own)
            if (wave == 2) rotated = __ballot(rot != 0) != 0;
            break;
        }
        rot = __syncthreads_or(rot);
        rotated |= rot;
        if (!rot || sw + 1 == a.inner_sweeps) break;
        // another sweep (single-pair matrices): start again from S0
        if (Sfin != S0) {
            for (int e = tid; e < kP * kPS; e += 256) S0[e] = Sfin[e];
            __syncthreads();
        }
    }
    // positions are the indices again
    for (int e = tid; e < kP * kP; e += 256) {
        const int x = e >> 5, y = e & 31;
        __builtin_nontemporal_store(Sfin[sym(x, y)], &gmem(a.Scur)[(int64_t)pair * kP * kP + e]);
    }
    if (wave == 3 && lane < kP) {
        const auto dst = gmem(a.Jcur) + (int64_t)pair * kP * kP + lane * kP;
#pragma unroll
        for (int c = 0; c < kP; ++c) __builtin_nontemporal_store(jr[c], &dst[c]);
    }
    if (tid == 128) gmem(a.fcur)[pair] = rotated;   // lane 0 of wave 2 holds the flag
}

// ---- update of the previous round (FP64 matrix cores) ----------------------
//
// v_mfma_f64_16x16x4: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; the
// 16 x 16 result leaves element i of lane l at row l / 16 + 4 i, column l % 16.  That
// result layout is exactly the B-operand layout of the next product over the same
// rows (k-chunk 4 * rowblock + i), so J_a^T (G J_b) keeps G J_b in registers.


// acc = A B, A a 32 x 32 tile in LDS (stride kPS), B row-major 32 x 32 in memory.
__device__ __forceinline__ void mm_lds_mem(const double *__restrict__ A, __attribute__((address_space(1))) const double *__restrict__ B, d4 (&acc)[2][2],
                                           int l) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
        const int k = kc * 4 + (l >> 4);
        const double a0 = A[(l & 15) * kPS + k], a1 = A[(16 + (l & 15)) * kPS + k];
        const double b0 = B[k * kP + (l & 15)], b1 = B[k * kP + 16 + (l & 15)];
        acc[0][0] = mfma4(a0, b0, acc[0][0]);
        acc[0][1] = mfma4(a0, b1, acc[0][1]);
        acc[1][0] = mfma4(a1, b0, acc[1][0]);
        acc[1][1] = mfma4(a1, b1, acc[1][1]);
    }
}
// out = Ja^T T, T in result layout (registers), Ja row-major 32 x 32 in memory.
__device__ __forceinline__ void mm_t_reg(__attribute__((address_space(1))) const double *__restrict__ Ja, const d4 (&T)[2][2], d4 (&out)[2][2], int l) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) out[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
        const int k = kc * 4 + (l >> 4);
        const double a0 = Ja[k * kP + (l & 15)], a1 = Ja[k * kP + 16 + (l & 15)];
        const double b0 = T[kc >> 2][0][kc & 3], b1 = T[kc >> 2][1][kc & 3];
        out[0][0] = mfma4(a0, b0, out[0][0]);
        out[0][1] = mfma4(a0, b1, out[0][1]);
        out[1][0] = mfma4(a1, b0, out[1][0]);
        out[1][1] = mfma4(a1, b1, out[1][1]);
    }
}
// result layout <- 32 x 32 tile in LDS
__device__ __forceinline__ void lds_to_acc(const double *__restrict__ A, d4 (&acc)[2][2], int l) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[rb][cb][i] = A[(16 * rb + (l >> 4) + 4 * i) * kPS + 16 * cb + (l & 15)];
}

// A 32 x 32 tile whose row x starts at rows[x] and whose columns are gidx(., Pb, Qb),
// staged in LDS (stride kPS) by one wave: all eight 16-byte loads of a lane are issued
// before the first LDS store, so the tile costs one memory round trip.
__device__ __forceinline__ void tile_to_lds(__attribute__((address_space(1))) const double *__restrict__ base, const int64_t (&rows)[8], int Pb, int Qb,
                                            double *buf, int l) {
    const int y = 2 * (l & 15), col = gidx(y, Pb, Qb);
    d2 v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = *reinterpret_cast<__attribute__((address_space(1))) const d2 *>(base + rows[j] + col);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int x = (l >> 4) + 4 * j;
        buf[x * kPS + y] = v[j].x;
        buf[x * kPS + y + 1] = v[j].y;
    }
}

__device__ __forceinline__ void update_tile(const RoundArgs &a, int u, double *buf) {
    const int l = threadIdx.x & 63;
    const int npairs = a.nb / 2;
    if (u < a.ntiles_g) {
        int ia = 0, rem = u;
        while (rem >= npairs - ia) {
            rem -= npairs - ia;
            ++ia;
        }
        const int ib = ia + rem;
        int Pa, Qa, Pb, Qb;
        tournament_pair(a.nb, a.round_prev, ia, Pa, Qa);
        tournament_pair(a.nb, a.round_prev, ib, Pb, Qb);
        if (ia == ib) {
            // diagonal tile: the rotated subproblem itself (loads first, then the stores)
            const auto s = reinterpret_cast<__attribute__((address_space(1))) const d2 *>(gmem(a.Sprev) + (int64_t)ia * kP * kP);
            d2 v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = s[l + 64 * j];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int e = 2 * (l + 64 * j), x = e >> 5, y = e & 31;
                const auto d = &gmem(a.Gout)[(int64_t)gidx(x, Pa, Qa) * a.ld + gidx(y, Pa, Qa)];
                __builtin_nontemporal_store(v[j].x, d);
                __builtin_nontemporal_store(v[j].y, d + 1);
            }
            return;
        }
        const bool fa = gmem(a.fprev)[ia] != 0, fb = gmem(a.fprev)[ib] != 0;
        {
            int64_t rows[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) rows[j] = (int64_t)gidx((l >> 4) + 4 * j, Pa, Qa) * a.ld;
            tile_to_lds(gmem(a.Gin), rows, Pb, Qb, buf, l);
        }
        wave_fence();
        d4 t[2][2], o[2][2];
        if (fb) mm_lds_mem(buf, gmem(a.Jprev) + (int64_t)ib * kP * kP, t, l);
        else lds_to_acc(buf, t, l);
        if (fa) {
            mm_t_reg(gmem(a.Jprev) + (int64_t)ia * kP * kP, t, o, l);
        } else {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) o[rb][cb] = t[rb][cb];
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const d4 v = o[rb][cb];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int x = 16 * rb + (l >> 4) + 4 * i, y = 16 * cb + (l & 15);
                    __builtin_nontemporal_store(v[i], &gmem(a.Gout)[(int64_t)gidx(x, Pa, Qa) * a.ld + gidx(y, Pb, Qb)]);
                }
            }
        // the mirror tile through LDS, so its stores are row runs as well
        wave_fence();
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const d4 v = o[rb][cb];
#pragma unroll
                for (int i = 0; i < 4; ++i) buf[(16 * rb + (l >> 4) + 4 * i) * kPS + 16 * cb + (l & 15)] = v[i];
            }
        wave_fence();
        for (int e = l; e < kP * kP; e += 64) {
            const int x = e >> 5, y = e & 31;   // element (y, x) of the tile = (x, y) of its mirror
            __builtin_nontemporal_store(buf[y * kPS + x], &gmem(a.Gout)[(int64_t)gidx(x, Pb, Qb) * a.ld + gidx(y, Pa, Qa)]);
        }
        return;
    }
    u -= a.ntiles_g;
    if (u >= a.nrowtiles * npairs) return;   // spare wave of the last workgroup
    // W tiles: row-tile-major (linear schedule) or pair-major (grouped schedule: the tiles
    // that share J_ib are consecutive, so one XCD's L2 serves them)
    const int rt = a.sched ? u % a.nrowtiles : u / npairs, ib = a.sched ? u / a.nrowtiles : u % npairs;
    if (rt >= a.nrowtiles || !gmem(a.fprev)[ib]) return;
    int Pb, Qb;
    tournament_pair(a.nb, a.round_prev, ib, Pb, Qb);
    {
        int64_t rows[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) rows[j] = (int64_t)(rt * kP + (l >> 4) + 4 * j) * a.ld;
        tile_to_lds(gmem(a.W), rows, Pb, Qb, buf, l);
    }
    wave_fence();
    d4 t[2][2];
    mm_lds_mem(buf, gmem(a.Jprev) + (int64_t)ib * kP * kP, t, l);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = 16 * rb + (l >> 4) + 4 * i, y = 16 * cb + (l & 15);
                __builtin_nontemporal_store(t[rb][cb][i], &gmem(a.W)[(int64_t)(rt * kP + x) * a.ld + gidx(y, Pb, Qb)]);
            }
}

// kOne: the launch covers a single matrix whose arguments arrive by value in `one`
// (no dependent load before the round's own loads); otherwise a batch reads them from
// `table` (`one` unused).
template <bool kOne>
__global__ __launch_bounds__(256, 2) void k_jround(const RoundArgs one, const RoundArgs *__restrict__ table,
                                                   const int32_t *__restrict__ wp, int count, int32_t launch_r) {
    __shared__ __align__(16) double smem[kSmemDoubles];
    RoundArgs a;
    int b = (int)blockIdx.x;
    if constexpr (kOne) {
        a = one;
    } else {
        const int mat = find_mat(wp, count, blockIdx.x);
        a = table[mat];
        b -= wp[mat];
    }
    const int npairs = a.nb / 2;
    if (a.do_solve) {
        if (b < npairs) {
            solve_pair(a, b, launch_r, smem);
            return;
        }
        b -= npairs;
    }
    if (gmem(a.jstate)[kJsActive] == 0) return;
    // G buffer holding M_{r-1}: one flip per launch with a previous round, nb - 1 per sweep
    const int32_t flips = gmem(a.jstate)[kJsSweeps] * (a.nb - 1) + (launch_r > 0 ? launch_r - 1 : 0);
    a.Gin = (flips & 1) ? a.G1 : a.G0;
    a.Gout = (flips & 1) ? a.G0 : a.G1;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (a.sched & 1) {
        // consecutive workgroups go to consecutive XCDs; give the workgroups of one XCD a
        // contiguous range of tiles (a bijection on the first 8 floor(U / 8) of them)
        const int tiles = a.ntiles_g + a.nrowtiles * npairs;
        const int U = (tiles + kTileWaves - 1) / kTileWaves, Q = U / 8;
        if (b < 8 * Q) b = (b % 8) * Q + b / 8;
    }
    update_tile(a, b * kTileWaves + wave, smem + wave * kP * kPS);
}

// The G buffer holding the matrix after `sweeps` complete sweeps (plus the sweep just run
// when `pending`: the test at the end of a sweep runs before its count is updated).
__device__ __forceinline__ const double *current_g(const MatDesc &d, bool pending = false) {
    const int32_t nb = d.npad / kB;
    const int32_t sw = d.jstate[kJsSweeps] + (pending ? d.jstate[kJsActive] : 0);
    return ((sw * (nb - 1)) & 1) ? d.G2 : d.G;
}

// Sets jstate[kJsCheck] = 1 if an off-diagonal entry of the leading n x n part
// still fails the rotation test (run at the end of a sweep, before the state update).  One workgroup per 64 x 64 tile (ti <= tj) of the
// upper triangle; the tile's row and column diagonal entries are staged in LDS.
__global__ __launch_bounds__(256) void k_jcheck(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                int count) {
    constexpr int kT = kJacobiCheckTile;
    __shared__ double drow[kT], dcol[kT];
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int32_t n = d.n;
    const int64_t ld = d.npad;
    const double *__restrict__ G = current_g(d, true);
    const double floor_abs = d.sdbl[kSdFloor];
    const double tol = d.jtol > 0.0 ? d.jtol : fmax(1e-15, sqrt((double)n) * 2.220446049250313e-16);
    const double tol2 = tol * tol;
    const int T = (n + kT - 1) / kT;
    int ti = 0, rem = blockIdx.x - wp[mat];
    while (rem >= T - ti) {
        rem -= T - ti;
        ++ti;
    }
    const int tj = ti + rem;
    const int64_t r0 = (int64_t)ti * kT, c0 = (int64_t)tj * kT;
    // every load of the tile issued first, then the diagonal's, before any test (a load under
    // the test's branch would wait on its own); indices clamped into the n x n part, so each
    // load is in bounds
    constexpr int kPer = kT * kT / 256;
    const auto Gm = gmem(G);
    double g[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int e = threadIdx.x + 256 * t;
        const int64_t p = min(r0 + e / kT, (int64_t)n - 1), q = min(c0 + e % kT, (int64_t)n - 1);
        g[t] = Gm[p * ld + q];
    }
    if (threadIdx.x < kT) {
        const int64_t p = r0 + threadIdx.x;
        drow[threadIdx.x] = p < n ? G[p * ld + p] : 0.0;
    } else if (threadIdx.x < 2 * kT) {
        const int64_t q = c0 + threadIdx.x - kT;
        dcol[threadIdx.x - kT] = q < n ? G[q * ld + q] : 0.0;
    }
    __syncthreads();
    int bad = 0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int e = threadIdx.x + 256 * t;
        const int r = e / kT, c = e % kT;
        const int64_t p = r0 + r, q = c0 + c;
        if (q > p && q < n && fabs(g[t]) > floor_abs && g[t] * g[t] > tol2 * fabs(drow[r] * dcol[c])) bad = 1;
    }
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(&d.jstate[kJsCheck], 1);
}

// End of a sweep, per matrix (after the rounds and the convergence test): count the sweep
// if it ran, take the test's verdict, decide the next sweep (not converged and under the
// cap), clear the test flag, and publish active / sweeps / not-converged to `out` (host
// memory; NULL: no copy), then the launch's epoch.  One workgroup for all matrices.
__global__ __launch_bounds__(256) void k_jstate(const MatDesc *__restrict__ descs, int count, int32_t max_sweeps,
                                                int32_t *__restrict__ out, int32_t *__restrict__ epoch) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        int32_t *js = descs[i].jstate;
        int32_t active = 0, sweeps = js[kJsSweeps], nc = 0;
        if (descs[i].n > 0) {
            sweeps += js[kJsActive];
            nc = js[kJsCheck];
            active = (nc != 0 && sweeps < max_sweeps) ? 1 : 0;
        }
        js[kJsSweeps] = sweeps;
        js[kJsNotConv] = nc;
        js[kJsCheck] = 0;
        js[kJsActive] = active;
        if (out) {
            out[3 * i + 0] = active;
            out[3 * i + 1] = sweeps;
            out[3 * i + 2] = nc;
        }
    }
    if (!out) return;
    // every entry out before the epoch: the device counter, incremented once per launch and
    // copied to out[3 count], tells the host which launch's entries it is reading
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t e = *epoch + 1;
        *epoch = e;
        out[3 * count] = e;
        __threadfence_system();
    }
}

// Per matrix: W = I; workgroup 0 also finds m = max|g_ii|, the power of two 2^-e that
// brings m into [1/2, 1) and the floor (n eps)^2 m 2^-e, and clears the state.
__global__ __launch_bounds__(256) void k_jinit(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                               int count) {
    __shared__ double red[256];
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int64_t npad = d.npad;
    const int64_t nblk = wp[mat + 1] - wp[mat];
    const int64_t b = blockIdx.x - wp[mat];
    for (int64_t e = b * blockDim.x + threadIdx.x; e < npad * npad; e += nblk * blockDim.x)
        d.W[e] = (e / npad == e % npad) ? 1.0 : 0.0;
    if (b != 0) return;
    double m = 0.0;
    for (int32_t i = threadIdx.x; i < d.n; i += 256) m = fmax(m, fabs(d.G[(int64_t)i * npad + i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mx = red[0];
        int e = 0;
        if (mx > 0.0) (void)frexp(mx, &e);
        const double scale = ldexp(1.0, -e);
        const double ne = (double)d.n * 2.220446049250313e-16;
        d.sdbl[kSdScale] = scale;
        d.sdbl[kSdFloor] = ne * ne * (mx * scale);
        d.jstate[kJsSweeps] = 0;
        d.jstate[kJsActive] = 0;
        d.jstate[kJsNotConv] = 0;
        d.jstate[kJsCheck] = 0;
    }
}

// G *= 2^-e (exact), after k_jinit.
__global__ __launch_bounds__(256) void k_jscale(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                int count) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int64_t npad = d.npad;
    const int64_t nblk = wp[mat + 1] - wp[mat];
    const int64_t b = blockIdx.x - wp[mat];
    const double scale = d.sdbl[kSdScale];
    if (scale == 1.0) return;
    for (int64_t e = b * blockDim.x + threadIdx.x; e < npad * npad; e += nblk * blockDim.x) d.G[e] *= scale;
}

// lambda_i = g_ii 2^e
__global__ __launch_bounds__(256) void k_jdiag(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                               int count) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int32_t i = (blockIdx.x - wp[mat]) * blockDim.x + threadIdx.x;
    if (i < d.n) d.lam[i] = current_g(d)[(int64_t)i * d.npad + i] / d.sdbl[kSdScale];
}

// ---------------------------------------------------------------------------

int32_t jacobi_npad(int32_t n) { return ((n + kP - 1) / kP) * kP; }

void launch_jacobi_init(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_jinit, dim3((unsigned)nblocks), dim3(256), 0, s, descs, wp, count);
    hipLaunchKernelGGL(k_jscale, dim3((unsigned)nblocks), dim3(256), 0, s, descs, wp, count);
}

void launch_jacobi_state(const MatDesc *descs, int count, int32_t max_sweeps, int32_t *out, int32_t *epoch,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_jstate, dim3(1), dim3(256), 0, s, descs, count, max_sweeps, out, epoch);
}

void launch_jacobi_round(const void *host_table, const void *table, const int32_t *wp, int64_t nblocks, int count,
                         int32_t launch_r, size_t lds_pad, hipStream_t s) {
    if (nblocks <= 0) return;
    RoundArgs one = {};
    if (count == 1) {
        one = *static_cast<const RoundArgs *>(host_table);
        hipLaunchKernelGGL(k_jround<true>, dim3((unsigned)nblocks), dim3(256), lds_pad, s, one,
                           static_cast<const RoundArgs *>(table), wp, count, launch_r);
    } else {
        hipLaunchKernelGGL(k_jround<false>, dim3((unsigned)nblocks), dim3(256), lds_pad, s, one,
                           static_cast<const RoundArgs *>(table), wp, count, launch_r);
    }
}

size_t jround_solo_pad(size_t lds_per_cu) {
    const size_t own = sizeof(double) * kSmemDoubles, half = lds_per_cu / 2 + 1024;
    return half > own ? half - own : 0;
}

void launch_jacobi_check(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_jcheck, dim3((unsigned)nblocks), dim3(256), 0, s, descs, wp, count);
}

void launch_jacobi_diag(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_jdiag, dim3((unsigned)nblocks), dim3(256), 0, s, descs, wp, count);
}

size_t round_args_bytes() { return sizeof(RoundArgs); }

void fill_round_args(void *dst, const MatDesc &d, int32_t r, int32_t inner_sweeps) {
    RoundArgs a;
    std::memset(&a, 0, sizeof(a));   // padding too: the bytes are hashed to key captured graphs
    const int32_t nb = d.npad / kB;
    const int32_t npairs = nb / 2;
    const size_t jsz = (size_t)npairs * kP * kP;
    a.Gin = nullptr;
    a.Gout = nullptr;
    a.G0 = d.G;
    a.G1 = d.G2;
    a.W = d.W;
    a.ld = d.npad;
    a.nb = nb;
    a.round_cur = r;
    a.round_prev = r - 1;
    a.has_prev = r > 0 && r <= nb - 1;
    a.do_solve = r < nb - 1;
    a.Jprev = d.J + ((r + 1) & 1) * jsz;
    a.Sprev = d.S + ((r + 1) & 1) * jsz;
    a.fprev = d.jflag + ((r + 1) & 1) * npairs;
    a.Jcur = d.J + (r & 1) * jsz;
    a.Scur = d.S + (r & 1) * jsz;
    a.fcur = d.jflag + (r & 1) * npairs;
    a.sdbl = d.sdbl;
    a.jstate = d.jstate;
    a.tol = d.jtol > 0.0 ? d.jtol : fmax(1e-15, sqrt((double)d.n) * 2.220446049250313e-16);
    a.inner_sweeps = npairs == 1 ? 40 : inner_sweeps;
    // a full subproblem sweep in about every quarter of the rounds (round 0 included, so
    // every pair inside a block is rotated once per sweep), cross sweeps in the others
    a.cross = npairs > 1 && r % std::max(1, (nb - 1) / 4) != 0;
    a.ntiles_g = npairs * (npairs + 1) / 2;
    a.nrowtiles = d.npad / kP;
    a.sched = d.jsched;
    std::memcpy(dst, &a, sizeof(a));
}

// workgroups matrix d needs in launch r of a sweep (0 when it has no work there)
int64_t round_blocks(const MatDesc &d, int32_t r) {
    if (d.n <= 0) return 0;
    const int32_t nb = d.npad / kB;
    const int32_t npairs = nb / 2;
    int64_t b = 0;
    if (r < nb - 1) b += npairs;
    if (r > 0 && r <= nb - 1) {
        const int64_t tiles = (int64_t)npairs * (npairs + 1) / 2 + (int64_t)(d.npad / kP) * npairs;
        b += (tiles + kTileWaves - 1) / kTileWaves;
    }
    return b;
}

}  // namespace ranky

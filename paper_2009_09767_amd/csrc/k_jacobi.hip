// k_jacobi.hip -- FP64 two-sided blocked Jacobi eigensolver of the Gram matrix.
//
// The SVD of the proxy matrix P (Sec. III, last step of Alg. 1) is, in Gram form,
// the eigendecomposition G = W Lambda W^T of G = P P^T.  Jacobi keeps relative
// accuracy in the small eigenvalues, which the rank decision relies on.
//
// Layout: G (two ping-pong copies) and W are npad x npad row-major, npad a multiple
// of 32; indices >= n are zero padding that no rotation touches (their couplings
// stay exactly zero).  The index range is cut into nb = npad / 16 blocks; one sweep
// is nb - 1 rounds of a round-robin tournament on the blocks, and in a round the
// nb / 2 block pairs are disjoint.  Every round is ONE launch of k_jround:
//   * workgroups [0, npairs) solve the round's 32 x 32 subproblems S = M_r[s, s]
//     (s = the pair's two blocks) by cyclic Jacobi in LDS and write the rotation J
//     (32 x 32) and the rotated S.  M_r is the matrix after the previous rounds; its
//     diagonal subproblem blocks are built directly from M_{r-1} and the previous
//     round's J (J_a^T M_{r-1}[s_a, s_b] J_b), so no workgroup waits for the update.
//   * the other workgroups apply the previous round: M_r = Jp^T M_{r-1} Jp tile by
//     tile (32 x 32 tiles of the previous pairing; the diagonal tiles are the rotated
//     subproblems themselves) into the other G buffer, and W <- W Jp in place.
// A flush launch (update only) ends every sweep; k_jcheck then tests every
// off-diagonal entry against |g_pq| > max(tol sqrt|g_pp g_qq|, floor) with
// tol = max(1e-15, sqrt(n) eps), floor = (n eps)^2 max|g_ii|.
// Rotation (Rutishauser): zeta = (g_qq - g_pp) / (2 g_pq), t = sign(zeta) / (|zeta| +
// sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = c t; then g_pp -= t g_pq, g_qq += t g_pq.
// Rows: r_p <- c r_p - s r_q, r_q <- s r_p + c r_q; columns likewise.
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

constexpr int kB = 16;       // block of indices
constexpr int kP = 32;       // subproblem = two blocks
constexpr int kPS = 33;      // LDS row stride of 32-wide tiles

// Round r of the round-robin tournament on `players` (even) seats: seat 0 stays, the
// others turn one place per round; pair i joins seat i and seat players-1-i.
__device__ __forceinline__ void tournament_pair(int players, int r, int i, int &a, int &b) {
    const int ring = players - 1;
    const int sa = i, sb = players - 1 - i;
    a = sa == 0 ? 0 : 1 + (sa - 1 + r) % ring;
    b = sb == 0 ? 0 : 1 + (sb - 1 + r) % ring;
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
}

// global index of position l (0..31) of the super-block made of blocks (P, Q)
__device__ __forceinline__ int gidx(int l, int P, int Q) { return l < kB ? P * kB + l : Q * kB + (l - kB); }

__device__ __forceinline__ void rotation(double app, double aqq, double apq, double &c, double &s, double &t) {
    const double zeta = (aqq - app) / (2.0 * apq);
    double tt;
    if (fabs(zeta) > 1e150)
        tt = 0.5 / zeta;
    else
        tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    c = 1.0 / sqrt(1.0 + tt * tt);
    s = c * tt;
    t = tt;
}

// Per-matrix arguments of one round launch (a table of these covers a batch).
struct RoundArgs {
    const double *Gin;     // M_{r-1} (or M_r itself when there is no previous round); set in-kernel
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
    int32_t ntiles_g;      // npairs (npairs + 1) / 2
    int32_t nrowtiles;     // npad / 32
};

// ---- subproblem solve -------------------------------------------------------

__device__ void solve_pair(const RoundArgs &a, int pair, double *S, double *J, double *T, double *JA, double *JB,
                           int *pos) {
    const int tid = threadIdx.x;
    const int npairs = a.nb / 2;
    int P, Q;
    tournament_pair(a.nb, a.round_cur, pair, P, Q);
    if (!a.has_prev) {
        for (int e = tid; e < kP * kP; e += 256) {
            const int x = e >> 5, y = e & 31;
            S[x * kPS + y] = a.Gin[(int64_t)gidx(x, P, Q) * a.ld + gidx(y, P, Q)];
        }
    } else {
        // where blocks P and Q sat in the previous round: pos[block] = pair * 2 + half
        for (int j = tid; j < npairs; j += 256) {
            int x, y;
            tournament_pair(a.nb, a.round_prev, j, x, y);
            pos[x] = 2 * j;
            pos[y] = 2 * j + 1;
        }
        __syncthreads();
        const int pp = pos[P] >> 1, hp = pos[P] & 1, pq = pos[Q] >> 1, hq = pos[Q] & 1;
        // diagonal blocks: the previous round's rotated subproblems
        for (int e = tid; e < kB * kB; e += 256) {
            const int x = e >> 4, y = e & 15;
            S[x * kPS + y] = a.Sprev[(int64_t)pp * kP * kP + (hp * kB + x) * kP + hp * kB + y];
            S[(kB + x) * kPS + kB + y] = a.Sprev[(int64_t)pq * kP * kP + (hq * kB + x) * kP + hq * kB + y];
        }
        // off-diagonal block: J_pp[:, hp]^T  M_{r-1}[s_pp, s_pq]  J_pq[:, hq]
        int Pa, Qa, Pb, Qb;
        tournament_pair(a.nb, a.round_prev, pp, Pa, Qa);
        tournament_pair(a.nb, a.round_prev, pq, Pb, Qb);
        const bool fa = a.fprev[pp] != 0, fb = a.fprev[pq] != 0;
        for (int e = tid; e < kP * kP; e += 256) {
            const int x = e >> 5, y = e & 31;
            T[x * kPS + y] = a.Gin[(int64_t)gidx(x, Pa, Qa) * a.ld + gidx(y, Pb, Qb)];
        }
        for (int e = tid; e < kP * kB; e += 256) {
            const int x = e >> 4, y = e & 15;
            JA[x * kB + y] = fa ? a.Jprev[(int64_t)pp * kP * kP + x * kP + hp * kB + y] : (x == hp * kB + y ? 1.0 : 0.0);
            JB[x * kB + y] = fb ? a.Jprev[(int64_t)pq * kP * kP + x * kP + hq * kB + y] : (x == hq * kB + y ? 1.0 : 0.0);
        }
        __syncthreads();
        // U1 = T JB (32 x 16): two outputs per thread, kept in registers
        double u0 = 0.0, u1 = 0.0;
        {
            const int x = tid >> 3, y = (tid & 7) * 2;
            for (int z = 0; z < kP; ++z) {
                const double t = T[x * kPS + z];
                u0 = fma(t, JB[z * kB + y], u0);
                u1 = fma(t, JB[z * kB + y + 1], u1);
            }
        }
        __syncthreads();
        {
            const int x = tid >> 3, y = (tid & 7) * 2;
            T[x * kPS + y] = u0;
            T[x * kPS + y + 1] = u1;
        }
        __syncthreads();
        // S_PQ = JA^T U1 (16 x 16): one output per thread
        {
            const int x = tid >> 4, y = tid & 15;
            double v = 0.0;
            for (int z = 0; z < kP; ++z) v = fma(JA[z * kB + x], T[z * kPS + y], v);
            S[x * kPS + kB + y] = v;
            S[(kB + y) * kPS + x] = v;
        }
    }
    for (int e = tid; e < kP * kP; e += 256) {
        const int x = e >> 5, y = e & 31;
        J[x * kPS + y] = (x == y) ? 1.0 : 0.0;
    }
    __syncthreads();

    __shared__ double rc[kP / 2], rs[kP / 2], rpp[kP / 2], rqq[kP / 2];
    __shared__ int ra[kP / 2], rb[kP / 2], ract[kP / 2];
    const double floor_abs = a.sdbl[kSdFloor];
    int rotated = 0;
    const int bi = tid >> 4, bj = tid & 15;   // this thread's 2x2 block of pair slots
    for (int sw = 0; sw < a.inner_sweeps; ++sw) {
        int sweep_rot = 0;
        for (int step = 0; step < kP - 1; ++step) {
            int act = 0;
            if (tid < kP / 2) {
                int x, y;
                tournament_pair(kP, step, tid, x, y);
                const double app = S[x * kPS + x], aqq = S[y * kPS + y], apq = S[x * kPS + y];
                double c = 1.0, s = 0.0;
                if (fabs(apq) > floor_abs && fabs(apq) > a.tol * sqrt(fabs(app * aqq))) {
                    double t;
                    rotation(app, aqq, apq, c, s, t);
                    rpp[tid] = app - t * apq;
                    rqq[tid] = aqq + t * apq;
                    act = 1;
                }
                ra[tid] = x;
                rb[tid] = y;
                rc[tid] = c;
                rs[tid] = s;
                ract[tid] = act;
            }
            if (__syncthreads_or(act) == 0) continue;
            sweep_rot += 1;
            // two-sided update of this thread's 2x2 block: R_i^T X R_j
            {
                const int ai = ra[bi], bi2 = rb[bi], aj = ra[bj], bj2 = rb[bj];
                const int acti = ract[bi], actj = ract[bj];
                if (bi == bj) {
                    if (acti) {
                        S[ai * kPS + ai] = rpp[bi];
                        S[bi2 * kPS + bi2] = rqq[bi];
                        S[ai * kPS + bi2] = 0.0;
                        S[bi2 * kPS + ai] = 0.0;
                    }
                } else if (acti || actj) {
                    double x00 = S[ai * kPS + aj], x01 = S[ai * kPS + bj2];
                    double x10 = S[bi2 * kPS + aj], x11 = S[bi2 * kPS + bj2];
                    if (acti) {
                        const double c = rc[bi], s = rs[bi];
                        const double y00 = c * x00 - s * x10, y01 = c * x01 - s * x11;
                        const double y10 = s * x00 + c * x10, y11 = s * x01 + c * x11;
                        x00 = y00;
                        x01 = y01;
                        x10 = y10;
                        x11 = y11;
                    }
                    if (actj) {
                        const double c = rc[bj], s = rs[bj];
                        const double y00 = c * x00 - s * x01, y01 = s * x00 + c * x01;
                        const double y10 = c * x10 - s * x11, y11 = s * x10 + c * x11;
                        x00 = y00;
                        x01 = y01;
                        x10 = y10;
                        x11 = y11;
                    }
                    S[ai * kPS + aj] = x00;
                    S[ai * kPS + bj2] = x01;
                    S[bi2 * kPS + aj] = x10;
                    S[bi2 * kPS + bj2] = x11;
                }
            }
            // J <- J R: columns of the pair, two rows per thread
            {
                const int p = tid & 15;
                if (ract[p]) {
                    const int x0 = ra[p], y0 = rb[p];
                    const double c = rc[p], s = rs[p];
                    for (int row = tid >> 4; row < kP; row += 16) {
                        const double u = J[row * kPS + x0], v = J[row * kPS + y0];
                        J[row * kPS + x0] = c * u - s * v;
                        J[row * kPS + y0] = s * u + c * v;
                    }
                }
            }
            __syncthreads();
        }
        rotated += sweep_rot;
        if (sweep_rot == 0) break;
    }
    for (int e = tid; e < kP * kP; e += 256) {
        const int x = e >> 5, y = e & 31;
        a.Jcur[(int64_t)pair * kP * kP + e] = J[x * kPS + y];
        a.Scur[(int64_t)pair * kP * kP + e] = S[x * kPS + y];
    }
    if (tid == 0) a.fcur[pair] = rotated > 0;
}

// ---- update of the previous round ------------------------------------------

// C (2x2 per thread... 4 outputs) = A (32x32) * B (32x32); transA reads A^T.
template <bool transA>
__device__ __forceinline__ void gemm32(const double *__restrict__ A, const double *__restrict__ B, double c[4],
                                       int row, int col0) {
    c[0] = c[1] = c[2] = c[3] = 0.0;
    for (int z = 0; z < kP; ++z) {
        const double av = transA ? A[z * kPS + row] : A[row * kPS + z];
        const double *b = B + z * kPS + col0;
        c[0] = fma(av, b[0], c[0]);
        c[1] = fma(av, b[1], c[1]);
        c[2] = fma(av, b[2], c[2]);
        c[3] = fma(av, b[3], c[3]);
    }
}

__device__ void update_tile(const RoundArgs &a, int u, double *A, double *B) {
    const int tid = threadIdx.x;
    const int npairs = a.nb / 2;
    const int row = tid >> 3, col0 = (tid & 7) * 4;
    double c[4];
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
            const double *s = a.Sprev + (int64_t)ia * kP * kP;
            for (int e = tid; e < kP * kP; e += 256)
                a.Gout[(int64_t)gidx(e >> 5, Pa, Qa) * a.ld + gidx(e & 31, Pa, Qa)] = s[e];
            return;
        }
        const bool fa = a.fprev[ia] != 0, fb = a.fprev[ib] != 0;
        for (int e = tid; e < kP * kP; e += 256) {
            const int x = e >> 5, y = e & 31;
            A[x * kPS + y] = a.Gin[(int64_t)gidx(x, Pa, Qa) * a.ld + gidx(y, Pb, Qb)];
        }
        if (fb) {
            const double *jb = a.Jprev + (int64_t)ib * kP * kP;
            for (int e = tid; e < kP * kP; e += 256) B[(e >> 5) * kPS + (e & 31)] = jb[e];
            __syncthreads();
            gemm32<false>(A, B, c, row, col0);
            __syncthreads();
            for (int v = 0; v < 4; ++v) A[row * kPS + col0 + v] = c[v];
        }
        if (fa) {
            const double *ja = a.Jprev + (int64_t)ia * kP * kP;
            __syncthreads();
            for (int e = tid; e < kP * kP; e += 256) B[(e >> 5) * kPS + (e & 31)] = ja[e];
            __syncthreads();
            gemm32<true>(B, A, c, row, col0);
            __syncthreads();
            for (int v = 0; v < 4; ++v) A[row * kPS + col0 + v] = c[v];
        }
        __syncthreads();
        for (int e = tid; e < kP * kP; e += 256) {
            const int x = e >> 5, y = e & 31;
            const double v = A[x * kPS + y];
            a.Gout[(int64_t)gidx(x, Pa, Qa) * a.ld + gidx(y, Pb, Qb)] = v;
            a.Gout[(int64_t)gidx(y, Pb, Qb) * a.ld + gidx(x, Pa, Qa)] = v;
        }
        return;
    }
    u -= a.ntiles_g;
    const int rt = u / npairs, ib = u % npairs;
    if (rt >= a.nrowtiles || !a.fprev[ib]) return;
    int Pb, Qb;
    tournament_pair(a.nb, a.round_prev, ib, Pb, Qb);
    const double *jb = a.Jprev + (int64_t)ib * kP * kP;
    for (int e = tid; e < kP * kP; e += 256) {
        const int x = e >> 5, y = e & 31;
        A[x * kPS + y] = a.W[(int64_t)(rt * kP + x) * a.ld + gidx(y, Pb, Qb)];
        B[x * kPS + y] = jb[e];
    }
    __syncthreads();
    gemm32<false>(A, B, c, row, col0);
    for (int v = 0; v < 4; ++v) a.W[(int64_t)(rt * kP + row) * a.ld + gidx(col0 + v, Pb, Qb)] = c[v];
}

__global__ __launch_bounds__(256) void k_jround(const RoundArgs *__restrict__ table, const int32_t *__restrict__ wp,
                                                int count, int32_t launch_r) {
    __shared__ double L0[kP * kPS], L1[kP * kPS], L2[kP * kPS];
    __shared__ double L3[kP * kB], L4[kP * kB];
    __shared__ int pos[512];
    const int mat = find_mat(wp, count, blockIdx.x);
    RoundArgs a = table[mat];
    if (a.jstate[kJsActive] == 0) return;
    // G buffer holding M_{r-1}: one flip per launch with a previous round, nb - 1 per sweep
    const int32_t flips = a.jstate[kJsSweeps] * (a.nb - 1) + (launch_r > 0 ? launch_r - 1 : 0);
    a.Gin = (flips & 1) ? a.G1 : a.G0;
    a.Gout = (flips & 1) ? a.G0 : a.G1;
    const int npairs = a.nb / 2;
    int b = blockIdx.x - wp[mat];
    if (a.do_solve) {
        if (b < npairs) {
            solve_pair(a, b, L0, L1, L2, L3, L4, pos);
            return;
        }
        b -= npairs;
    }
    update_tile(a, b, L0, L1);
}

// The G buffer holding the matrix after `sweeps` complete sweeps.
__device__ __forceinline__ const double *current_g(const MatDesc &d) {
    const int32_t nb = d.npad / kB;
    return ((d.jstate[kJsSweeps] * (nb - 1)) & 1) ? d.G2 : d.G;
}

// Sets jstate[kJsNotConv] = 1 if an off-diagonal entry of the leading n x n part
// still fails the rotation test (one thread per entry of the upper triangle).
__global__ __launch_bounds__(256) void k_jcheck(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                                int count) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int32_t n = d.n;
    const int64_t ld = d.npad;
    const double *__restrict__ G = current_g(d);
    const double floor_abs = d.sdbl[kSdFloor];
    const double tol = fmax(1e-15, sqrt((double)n) * 2.220446049250313e-16);
    const int64_t nblk = wp[mat + 1] - wp[mat];
    int bad = 0;
    for (int64_t p = blockIdx.x - wp[mat]; p < n; p += nblk) {
        const double gpp = G[p * ld + p];
        for (int64_t q = p + 1 + threadIdx.x; q < n; q += blockDim.x) {
            const double g = G[p * ld + q];
            if (fabs(g) > floor_abs && fabs(g) > tol * sqrt(fabs(gpp * G[q * ld + q]))) bad = 1;
        }
    }
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(&d.jstate[kJsNotConv], 1);
}

// Per matrix: start of a sweep (active = not converged and under the cap, clear the
// flag) or end of a sweep (count it).
__global__ __launch_bounds__(256) void k_jstate(const MatDesc *__restrict__ descs, int count, int32_t phase,
                                                int32_t max_sweeps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    int32_t *js = descs[i].jstate;
    if (descs[i].n <= 0) {
        js[kJsActive] = 0;
        return;
    }
    if (phase == 0) {
        js[kJsActive] = (js[kJsNotConv] != 0 && js[kJsSweeps] < max_sweeps) ? 1 : 0;
    } else if (phase == 1) {
        if (js[kJsActive]) js[kJsSweeps] += 1;
        js[kJsNotConv] = 0;
    }
}

// Per matrix: W = I, floor = (n eps)^2 max|g_ii|, state cleared.  One workgroup per
// (matrix, slice) for the identity; slice 0 also does the floor.
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
        const double ne = (double)d.n * 2.220446049250313e-16;
        d.sdbl[kSdFloor] = ne * ne * red[0];
        d.jstate[kJsSweeps] = 0;
        d.jstate[kJsActive] = 0;
        d.jstate[kJsNotConv] = 0;
    }
}

__global__ __launch_bounds__(256) void k_jdiag(const MatDesc *__restrict__ descs, const int32_t *__restrict__ wp,
                                               int count) {
    const int mat = find_mat(wp, count, blockIdx.x);
    const MatDesc &d = descs[mat];
    const int32_t i = (blockIdx.x - wp[mat]) * blockDim.x + threadIdx.x;
    if (i < d.n) d.lam[i] = current_g(d)[(int64_t)i * d.npad + i];
}

// ---------------------------------------------------------------------------

int32_t jacobi_npad(int32_t n) { return ((n + kP - 1) / kP) * kP; }

void launch_jacobi_init(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_jinit, dim3((unsigned)nblocks), dim3(256), 0, s, descs, wp, count);
}

void launch_jacobi_state(const MatDesc *descs, int count, int32_t phase, int32_t max_sweeps, hipStream_t s) {
    hipLaunchKernelGGL(k_jstate, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, descs, count, phase,
                       max_sweeps);
}

void launch_jacobi_round(const void *table, const int32_t *wp, int64_t nblocks, int count, int32_t launch_r,
                         hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_jround, dim3((unsigned)nblocks), dim3(256), 0, s, static_cast<const RoundArgs *>(table), wp,
                       count, launch_r);
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
    a.tol = fmax(1e-15, sqrt((double)d.n) * 2.220446049250313e-16);
    a.inner_sweeps = npairs == 1 ? 40 : inner_sweeps;
    a.ntiles_g = npairs * (npairs + 1) / 2;
    a.nrowtiles = d.npad / kP;
    *static_cast<RoundArgs *>(dst) = a;
}

// workgroups matrix d needs in launch r of a sweep (0 when it has no work there)
int64_t round_blocks(const MatDesc &d, int32_t r) {
    if (d.n <= 0) return 0;
    const int32_t nb = d.npad / kB;
    const int32_t npairs = nb / 2;
    int64_t b = 0;
    if (r < nb - 1) b += npairs;
    if (r > 0 && r <= nb - 1) b += (int64_t)npairs * (npairs + 1) / 2 + (int64_t)(d.npad / kP) * npairs;
    return b;
}

}  // namespace ranky

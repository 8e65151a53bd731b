// k_jacobi.hip -- FP64 two-sided blocked Jacobi eigensolver of the Gram matrix.
//
// The SVD of the proxy matrix P (Sec. III, last step of Alg. 1) is, in Gram form,
// the eigendecomposition G = W Lambda W^T of G = P P^T.  Jacobi keeps relative
// accuracy in the small eigenvalues, which the rank decision relies on.
//
// Layout: G and W are npad x npad row-major (npad a multiple of 64; indices >= n
// are zero padding that no rotation ever touches, since their couplings stay
// exactly zero).  The index range is cut into nb = npad / 32 blocks.  One sweep is
// nb - 1 rounds of a round-robin tournament on the blocks; in a round the nb / 2
// block pairs are disjoint, so their subproblems are independent:
//   k_jsolve   one workgroup per pair (P, Q): the 64 x 64 subproblem S = G[s, s],
//              s = P u Q, is diagonalised in LDS by cyclic Jacobi (a round-robin
//              over its 64 indices, 32 rotations at a time); the accumulated
//              rotation J (64 x 64) and the rotated S are written back.
//   k_jupdate  one workgroup per 64 x 64 tile: G[s_a, s_b] <- J_a^T G[s_a, s_b] J_b
//              for a < b (mirrored into (b, a)), and W[rows, s_b] <- W[rows, s_b] J_b.
//              Tiles whose J are both the identity are skipped.
//   k_jcheck   after a sweep: does any off-diagonal entry still fail the test
//              |g_pq| > max(tol sqrt|g_pp g_qq|, floor)?  (tol = max(1e-15, sqrt(n) eps),
//              floor = (n eps)^2 max|g_ii|.)  The host stops when none does.
// Rotation (Rutishauser): zeta = (g_qq - g_pp) / (2 g_pq), t = sign(zeta) / (|zeta| +
// sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = c t; g_pp -= t g_pq, g_qq += t g_pq.
#include "common.hpp"
#include "launch.hpp"

namespace ranky {

// Round r of the round-robin tournament on `players` (even) seats: seat 0 stays,
// the others turn one place per round; pair i joins seat i and seat players-1-i.
__device__ __forceinline__ void tournament_pair(int players, int r, int i, int &a, int &b) {
    const int ring = players - 1;
    auto seat = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + r) % ring; };
    a = seat(i);
    b = seat(players - 1 - i);
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
}

__device__ __forceinline__ int sub_index(int l, int P, int Q) { return l < kJB ? P * kJB + l : Q * kJB + (l - kJB); }

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

__global__ __launch_bounds__(256) void k_jeye(double *__restrict__ W, int32_t npad) {
    const int64_t total = (int64_t)npad * npad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        W[e] = (e / npad == e % npad) ? 1.0 : 0.0;
}

// max |g_ii| -> floor = (n eps)^2 max|g_ii| (one workgroup).
__global__ __launch_bounds__(256) void k_jprep(const double *__restrict__ G, int64_t ld, int32_t n,
                                               double *__restrict__ sdbl) {
    __shared__ double red[256];
    double m = 0.0;
    for (int32_t i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(G[(int64_t)i * ld + i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ne = (double)n * 2.220446049250313e-16;
        sdbl[kSdFloor] = ne * ne * red[0];
    }
}

__global__ __launch_bounds__(256) void k_jsolve(double *__restrict__ G, int64_t ld, int32_t nb, int32_t round,
                                                double tol, const double *__restrict__ sdbl,
                                                double *__restrict__ Jbuf, int32_t *__restrict__ jflag,
                                                int32_t inner_sweeps) {
    __shared__ double S[kJP * kJS];
    __shared__ double J[kJP * kJS];
    __shared__ double rc[kJP / 2], rs[kJP / 2], rpp[kJP / 2], rqq[kJP / 2];
    __shared__ int32_t ra[kJP / 2], rb[kJP / 2], ract[kJP / 2];
    __shared__ int32_t s_rot;
    const int pair = blockIdx.x;
    int P, Q;
    tournament_pair(nb, round, pair, P, Q);
    const double floor_abs = sdbl[kSdFloor];
    const int tid = threadIdx.x;

    for (int e = tid; e < kJP * kJP; e += 256) {
        const int a = e >> 6, b = e & 63;
        S[a * kJS + b] = G[(int64_t)sub_index(a, P, Q) * ld + sub_index(b, P, Q)];
        J[a * kJS + b] = (a == b) ? 1.0 : 0.0;
    }
    if (tid == 0) s_rot = 0;
    __syncthreads();

    int total_rot = 0;
    for (int sw = 0; sw < inner_sweeps; ++sw) {
        int sweep_rot = 0;
        for (int step = 0; step < kJP - 1; ++step) {
            if (tid < kJP / 2) {
                int a, b;
                tournament_pair(kJP, step, tid, a, b);
                const double app = S[a * kJS + a], aqq = S[b * kJS + b], apq = S[a * kJS + b];
                int act = 0;
                double c = 1.0, s = 0.0;
                if (fabs(apq) > floor_abs && fabs(apq) > tol * sqrt(fabs(app * aqq))) {
                    double t;
                    rotation(app, aqq, apq, c, s, t);
                    rpp[tid] = app - t * apq;
                    rqq[tid] = aqq + t * apq;
                    act = 1;
                }
                ra[tid] = a;
                rb[tid] = b;
                rc[tid] = c;
                rs[tid] = s;
                ract[tid] = act;
            }
            __syncthreads();
            int any = 0;
            for (int k = 0; k < kJP / 2; ++k) any |= ract[k];
            if (any) {
                // rows a, b of S
                for (int w = tid; w < (kJP / 2) * kJP; w += 256) {
                    const int pr = w >> 6, x = w & 63;
                    if (!ract[pr]) continue;
                    const int a = ra[pr], b = rb[pr];
                    const double c = rc[pr], s = rs[pr];
                    const double xa = S[a * kJS + x], xb = S[b * kJS + x];
                    S[a * kJS + x] = c * xa - s * xb;
                    S[b * kJS + x] = s * xa + c * xb;
                }
                __syncthreads();
                // columns a, b of S and of J
                for (int w = tid; w < (kJP / 2) * kJP; w += 256) {
                    const int pr = w >> 6, x = w & 63;
                    if (!ract[pr]) continue;
                    const int a = ra[pr], b = rb[pr];
                    const double c = rc[pr], s = rs[pr];
                    double xa = S[x * kJS + a], xb = S[x * kJS + b];
                    S[x * kJS + a] = c * xa - s * xb;
                    S[x * kJS + b] = s * xa + c * xb;
                    xa = J[x * kJS + a];
                    xb = J[x * kJS + b];
                    J[x * kJS + a] = c * xa - s * xb;
                    J[x * kJS + b] = s * xa + c * xb;
                }
                __syncthreads();
                if (tid < kJP / 2 && ract[tid]) {
                    const int a = ra[tid], b = rb[tid];
                    S[a * kJS + a] = rpp[tid];
                    S[b * kJS + b] = rqq[tid];
                    S[a * kJS + b] = 0.0;
                    S[b * kJS + a] = 0.0;
                }
                sweep_rot += 1;
            }
            __syncthreads();
        }
        total_rot += sweep_rot;
        if (sweep_rot == 0) break;
    }
    // write back S (rotated diagonal block) and J
    for (int e = tid; e < kJP * kJP; e += 256) {
        const int a = e >> 6, b = e & 63;
        G[(int64_t)sub_index(a, P, Q) * ld + sub_index(b, P, Q)] = S[a * kJS + b];
        Jbuf[(int64_t)pair * kJP * kJP + e] = J[a * kJS + b];
    }
    if (tid == 0) jflag[pair] = total_rot > 0;
}

// C (4x4 per thread) = A (64 x 64, LDS) * B (64 x 64, LDS); transA reads A^T.
template <bool transA>
__device__ __forceinline__ void tile_gemm(const double *__restrict__ A, const double *__restrict__ B, double c[4][4],
                                          int ty, int tx) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) c[u][v] = 0.0;
    for (int x = 0; x < kJP; ++x) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = transA ? A[x * kJS + 4 * ty + u] : A[(4 * ty + u) * kJS + x];
#pragma unroll
        for (int v = 0; v < 4; ++v) b[v] = B[x * kJS + 4 * tx + v];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) c[u][v] = fma(a[u], b[v], c[u][v]);
    }
}

__global__ __launch_bounds__(256) void k_jupdate(double *__restrict__ G, double *__restrict__ W, int64_t ld,
                                                 int32_t nb, int32_t round, const double *__restrict__ Jbuf,
                                                 const int32_t *__restrict__ jflag, int32_t ntiles_g,
                                                 int32_t nrowtiles) {
    __shared__ double A[kJP * kJS];
    __shared__ double B[kJP * kJS];
    const int npairs = nb / 2;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    int t = blockIdx.x;
    double c[4][4];
    if (t < ntiles_g) {
        // tile (ia, ib), ia < ib, from the row-major upper-triangular enumeration
        int ia = 0, rem = t;
        while (rem >= npairs - 1 - ia) {
            rem -= npairs - 1 - ia;
            ++ia;
        }
        const int ib = ia + 1 + rem;
        const int fa = jflag[ia], fb = jflag[ib];
        if (!fa && !fb) return;
        int Pa, Qa, Pb, Qb;
        tournament_pair(nb, round, ia, Pa, Qa);
        tournament_pair(nb, round, ib, Pb, Qb);
        for (int e = tid; e < kJP * kJP; e += 256) {
            const int r = e >> 6, q = e & 63;
            A[r * kJS + q] = G[(int64_t)sub_index(r, Pa, Qa) * ld + sub_index(q, Pb, Qb)];
        }
        if (fb) {
            const double *Jb = Jbuf + (int64_t)ib * kJP * kJP;
            for (int e = tid; e < kJP * kJP; e += 256) B[(e >> 6) * kJS + (e & 63)] = Jb[e];
            __syncthreads();
            tile_gemm<false>(A, B, c, ty, tx);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) A[(4 * ty + u) * kJS + 4 * tx + v] = c[u][v];
        }
        if (fa) {
            const double *Ja = Jbuf + (int64_t)ia * kJP * kJP;
            __syncthreads();
            for (int e = tid; e < kJP * kJP; e += 256) B[(e >> 6) * kJS + (e & 63)] = Ja[e];
            __syncthreads();
            tile_gemm<true>(B, A, c, ty, tx);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) A[(4 * ty + u) * kJS + 4 * tx + v] = c[u][v];
        }
        __syncthreads();
        for (int e = tid; e < kJP * kJP; e += 256) {
            const int r = e >> 6, q = e & 63;
            const double v = A[r * kJS + q];
            G[(int64_t)sub_index(r, Pa, Qa) * ld + sub_index(q, Pb, Qb)] = v;
            G[(int64_t)sub_index(q, Pb, Qb) * ld + sub_index(r, Pa, Qa)] = v;
        }
        return;
    }
    t -= ntiles_g;
    const int rt = t / npairs, ib = t % npairs;
    if (rt >= nrowtiles || !jflag[ib]) return;
    int Pb, Qb;
    tournament_pair(nb, round, ib, Pb, Qb);
    const double *Jb = Jbuf + (int64_t)ib * kJP * kJP;
    for (int e = tid; e < kJP * kJP; e += 256) {
        const int r = e >> 6, q = e & 63;
        A[r * kJS + q] = W[(int64_t)(rt * kJP + r) * ld + sub_index(q, Pb, Qb)];
        B[r * kJS + q] = Jb[e];
    }
    __syncthreads();
    tile_gemm<false>(A, B, c, ty, tx);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            W[(int64_t)(rt * kJP + 4 * ty + u) * ld + sub_index(4 * tx + v, Pb, Qb)] = c[u][v];
}

// Sets scal[kScNotConv] = 1 if an off-diagonal entry of the leading n x n part still
// fails the rotation test.  Grid: one thread per (row, 64-column strip), upper part only.
__global__ __launch_bounds__(256) void k_jcheck(const double *__restrict__ G, int64_t ld, int32_t n, double tol,
                                                const double *__restrict__ sdbl, int32_t *__restrict__ scal) {
    const double floor_abs = sdbl[kSdFloor];
    const int64_t strips = (n + 63) / 64;
    int bad = 0;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < (int64_t)n * strips;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = w / strips, st = w % strips;
        const double gpp = G[p * ld + p];
        for (int64_t q = st * 64; q < st * 64 + 64 && q < n; ++q) {
            if (q <= p) continue;
            const double g = G[p * ld + q];
            if (fabs(g) > floor_abs && fabs(g) > tol * sqrt(fabs(gpp * G[q * ld + q]))) bad = 1;
        }
    }
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(&scal[kScNotConv], 1);
}

// eigenvalues = diag(G)
__global__ __launch_bounds__(256) void k_jdiag(const double *__restrict__ G, int64_t ld, int32_t n,
                                               double *__restrict__ lam) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) lam[i] = G[(int64_t)i * ld + i];
}

// ---------------------------------------------------------------------------

void launch_jacobi_init(double *W, int32_t npad, const double *G, int64_t ld, int32_t n, double *sdbl,
                        hipStream_t s) {
    int64_t blocks = ((int64_t)npad * npad + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_jeye, dim3((unsigned)blocks), dim3(256), 0, s, W, npad);
    hipLaunchKernelGGL(k_jprep, dim3(1), dim3(256), 0, s, G, ld, n, sdbl);
}

void launch_jacobi_round(double *G, double *W, int64_t ld, int32_t npad, int32_t round, double tol,
                         const double *sdbl, double *Jbuf, int32_t *jflag, int32_t inner_sweeps, hipStream_t s) {
    const int32_t nb = npad / kJB;
    const int32_t npairs = nb / 2;
    hipLaunchKernelGGL(k_jsolve, dim3((unsigned)npairs), dim3(256), 0, s, G, ld, nb, round, tol, sdbl, Jbuf, jflag,
                       inner_sweeps);
    const int32_t ntiles_g = npairs * (npairs - 1) / 2;
    const int32_t nrowtiles = npad / kJP;
    const int32_t total = ntiles_g + nrowtiles * npairs;
    hipLaunchKernelGGL(k_jupdate, dim3((unsigned)total), dim3(256), 0, s, G, W, ld, nb, round, Jbuf, jflag, ntiles_g,
                       nrowtiles);
}

void launch_jacobi_check(const double *G, int64_t ld, int32_t n, double tol, const double *sdbl, int32_t *scal,
                         hipStream_t s) {
    const int64_t work = (int64_t)n * ((n + 63) / 64);
    int64_t blocks = (work + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_jcheck, dim3((unsigned)blocks), dim3(256), 0, s, G, ld, n, tol, sdbl, scal);
}

void launch_jacobi_diag(const double *G, int64_t ld, int32_t n, double *lam, hipStream_t s) {
    hipLaunchKernelGGL(k_jdiag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, ld, n, lam);
}

}  // namespace ranky

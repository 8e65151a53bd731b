// ranky_api.cpp -- host runtime behind include/ranky.h: argument checks, the
// workspace plan, stream-ordered enqueue of the kernels and status read-back.
#include "ranky.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "launch.hpp"
#include "launch_util.hpp"

struct ranky_ctx {
    int device;
    int cu_count;
    size_t lds_limit;   // dynamic LDS the Gram kernel may use per workgroup
    int32_t *pinned;    // host pinned read-back of the device scalars
    hipEvent_t ev[9];
};

namespace {

using namespace ranky;

thread_local char g_err[512] = "";
constexpr int32_t kMaxM = 8192;
constexpr int32_t kDefaultSweeps = 40;
constexpr int32_t kInnerSweeps = 1;
constexpr double kEps = 2.220446049250313e-16;

ranky_status fail(ranky_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(RANKY_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }
int32_t round_up64(int32_t x) { return jacobi_npad(x); }  // padded order of the eigensolver

// Workspace plan: offsets of every device array for the given sizes.
struct Plan {
    int32_t M = 0, k = 0, D = 0, cpb = 0, npad = 0;
    int64_t N = 0, nnz = 0, nchunks = 0;
    size_t o_scal = 0, o_sdbl = 0, o_hist = 0, o_rownnz = 0, o_rowptr = 0, o_m2r = 0, o_r2m = 0, o_empty = 0;
    size_t o_lonely = 0, o_single = 0, o_csrk = 0, o_csrend = 0, o_G = 0, o_G2 = 0, o_W = 0, o_J = 0, o_S = 0,
           o_jflag = 0;
    size_t o_lam = 0, o_perm = 0, o_csrcol = 0, o_U0 = 0, o_Z = 0, o_part = 0, o_Y = 0, o_seg = 0, total = 0;
    bool refine = false;
};

Plan make_plan(int32_t M, int64_t N, int64_t nnz, int32_t k, int32_t D, bool with_solver, bool refine = false) {
    Plan p;
    p.M = M;
    p.N = N;
    p.nnz = nnz;
    p.k = k;
    p.D = D;
    const int64_t maxw = (N + D - 1) / D;
    p.cpb = (int32_t)((maxw + kChunkCols - 1) / kChunkCols);
    if (p.cpb < 1) p.cpb = 1;
    p.nchunks = (int64_t)D * p.cpb;
    p.npad = round_up64(M);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    p.o_scal = take(sizeof(int32_t) * kScCount);
    p.o_sdbl = take(sizeof(double) * kSdCount);
    p.o_hist = take(sizeof(int32_t) * (size_t)p.nchunks * M);
    p.o_rownnz = take(sizeof(int32_t) * M);
    p.o_rowptr = take(sizeof(int32_t) * (M + 1));
    p.o_m2r = take(sizeof(int32_t) * M);
    p.o_r2m = take(sizeof(int32_t) * M);
    p.o_empty = take(sizeof(int32_t) * M);
    p.o_lonely = take(sizeof(int32_t) * D);
    p.o_single = take(sizeof(int32_t) * D);
    p.o_csrk = take(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    p.o_csrend = take(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    p.o_csrcol = take(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    p.o_G = take(sizeof(double) * (size_t)p.npad * p.npad);
    if (with_solver) {
        const size_t npairs = (size_t)(p.npad / kJacobiPair);
        p.o_G2 = take(sizeof(double) * (size_t)p.npad * p.npad);
        p.o_W = take(sizeof(double) * (size_t)p.npad * p.npad);
        p.o_J = take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair);
        p.o_S = take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair);
        p.o_jflag = take(sizeof(int32_t) * 2 * npairs);
        p.o_lam = take(sizeof(double) * p.npad);
        p.o_perm = take(sizeof(int32_t) * p.npad);
        if (refine) {
            p.refine = true;
            p.o_U0 = take(sizeof(double) * (size_t)M * k);
            p.o_Z = take(sizeof(double) * (size_t)N * k);
            p.o_part = take(sizeof(double) * (size_t)rr_max_segments(M, nnz) * k);
            p.o_Y = take(sizeof(double) * (size_t)M * k);
            p.o_seg = take(sizeof(int32_t) * (size_t)(M + 1));
        }
    }
    p.total = off;
    return p;
}

struct Ptrs {
    int32_t *scal, *hist, *rownnz, *rowptr, *m2r, *r2m, *empty, *lonely, *single, *csrk, *csrend, *csrcol, *jflag,
        *perm, *seg;
    double *sdbl, *G, *G2, *W, *J, *S, *lam, *U0, *Z, *part, *Y;
};

Ptrs carve(const Plan &p, void *ws) {
    char *b = static_cast<char *>(ws);
    Ptrs q;
    q.scal = reinterpret_cast<int32_t *>(b + p.o_scal);
    q.sdbl = reinterpret_cast<double *>(b + p.o_sdbl);
    q.hist = reinterpret_cast<int32_t *>(b + p.o_hist);
    q.rownnz = reinterpret_cast<int32_t *>(b + p.o_rownnz);
    q.rowptr = reinterpret_cast<int32_t *>(b + p.o_rowptr);
    q.m2r = reinterpret_cast<int32_t *>(b + p.o_m2r);
    q.r2m = reinterpret_cast<int32_t *>(b + p.o_r2m);
    q.empty = reinterpret_cast<int32_t *>(b + p.o_empty);
    q.lonely = reinterpret_cast<int32_t *>(b + p.o_lonely);
    q.single = reinterpret_cast<int32_t *>(b + p.o_single);
    q.csrk = reinterpret_cast<int32_t *>(b + p.o_csrk);
    q.csrend = reinterpret_cast<int32_t *>(b + p.o_csrend);
    q.csrcol = reinterpret_cast<int32_t *>(b + p.o_csrcol);
    q.U0 = p.refine ? reinterpret_cast<double *>(b + p.o_U0) : nullptr;
    q.Z = p.refine ? reinterpret_cast<double *>(b + p.o_Z) : nullptr;
    q.part = p.refine ? reinterpret_cast<double *>(b + p.o_part) : nullptr;
    q.Y = p.refine ? reinterpret_cast<double *>(b + p.o_Y) : nullptr;
    q.seg = p.refine ? reinterpret_cast<int32_t *>(b + p.o_seg) : nullptr;
    q.G = reinterpret_cast<double *>(b + p.o_G);
    q.G2 = reinterpret_cast<double *>(b + p.o_G2);
    q.W = reinterpret_cast<double *>(b + p.o_W);
    q.J = reinterpret_cast<double *>(b + p.o_J);
    q.S = reinterpret_cast<double *>(b + p.o_S);
    q.jflag = reinterpret_cast<int32_t *>(b + p.o_jflag);
    q.lam = reinterpret_cast<double *>(b + p.o_lam);
    q.perm = reinterpret_cast<int32_t *>(b + p.o_perm);
    return q;
}

int32_t default_blocks(int64_t N) {
    int64_t d = (N + 16383) / 16384;
    if (d < 1) d = 1;
    if (d > N) d = N;
    return (int32_t)d;
}

constexpr int32_t kMaxRefineK = 1024;

ranky_opts resolved(const ranky_opts *in, int64_t N) {
    ranky_opts o;
    ranky_default_opts(&o);
    if (in) o = *in;
    if (o.n_blocks == 0) o.n_blocks = default_blocks(N);
    if (o.max_sweeps <= 0) o.max_sweeps = kDefaultSweeps;
    return o;
}

bool wants_refine(const ranky_opts &o, int32_t k) { return o.refine > 0 && k <= kMaxRefineK; }

ranky_status check_csc_args(const ranky_csc *A, int32_t M, int64_t N) {
    if (!A) return fail(RANKY_E_INVALID, "A is NULL");
    if (M < 1 || N < 1) return fail(RANKY_E_INVALID, "M=%d N=%lld must be >= 1", M, (long long)N);
    if (M > kMaxM) return fail(RANKY_E_INVALID, "M=%d exceeds %d", M, kMaxM);
    if (N > (int64_t)0x7ffffffe) return fail(RANKY_E_INVALID, "N=%lld exceeds int32 column pointers", (long long)N);
    if (A->nnz < 0 || A->nnz > (int64_t)0x7fffffff) return fail(RANKY_E_INVALID, "nnz=%lld out of range", (long long)A->nnz);
    if (!A->colptr || (A->nnz > 0 && (!A->rowidx || !A->values)))
        return fail(RANKY_E_INVALID, "NULL CSC array");
    if (A->dtype != RANKY_F32 && A->dtype != RANKY_F64) return fail(RANKY_E_INVALID, "bad dtype %d", A->dtype);
    return RANKY_OK;
}

CscView view(const ranky_csc *A) {
    CscView v;
    v.nnz = A->nnz;
    v.colptr = A->colptr;
    v.rowidx = A->rowidx;
    v.values = A->values;
    v.dtype = A->dtype;
    return v;
}

// Runs the occupancy pass and reads back the status word and M'.
ranky_status run_occupancy(ranky_ctx *ctx, const Plan &p, const Ptrs &w, const CscView &A, int32_t validate,
                           int32_t *cnt, int32_t *lonely, int32_t *single, int32_t *rownnz, hipStream_t s,
                           int32_t *n_out) {
    launch_fill_i32(w.scal, kScCount, 0, s);
    launch_fill_i32(lonely, p.D, 0, s);
    launch_fill_i32(single, p.D, 0, s);
    launch_occupancy(A, p.M, p.N, p.D, p.cpb, p.nchunks, validate, w.hist, rownnz, cnt, lonely, single, w.rowptr,
                     w.m2r, w.r2m, w.empty, w.scal, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ctx->pinned, w.scal, sizeof(int32_t) * kScCount, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int32_t st = ctx->pinned[kScStatus];
    if (st & kStCsc) return fail(RANKY_E_CSC, "CSC contract violated (colptr, row range or row order)");
    if (st & kStNonfinite) return fail(RANKY_E_NONFINITE, "non-finite value in A");
    *n_out = ctx->pinned[kScNonempty];
    return RANKY_OK;
}

// Blocked Jacobi on G (leading n x n of an npad x npad array in w.G, ld = npad); on
// return *Gcur points at the buffer (w.G or w.G2) that holds the rotated matrix, W
// holds the eigenvectors and lam the eigenvalues.
ranky_status run_jacobi(ranky_ctx *ctx, const Ptrs &w, int32_t n, int32_t max_sweeps, hipStream_t s,
                        int32_t *sweeps_out) {
    const int32_t npad = round_up64(n);
    const int64_t ld = npad;
    const int32_t nb = npad / (kJacobiPair / 2);
    const int32_t npairs = nb / 2;
    const size_t jsz = (size_t)npairs * kJacobiPair * kJacobiPair;
    const double tol = std::fmax(1e-15, std::sqrt((double)n) * kEps);
    launch_jacobi_init(w.W, npad, w.G, ld, n, w.sdbl, s);
    double *buf[2] = {w.G, w.G2};
    int cur = 0;
    int32_t sweeps = 0;
    bool converged = false;
    for (;;) {
        launch_fill_i32(w.scal + kScNotConv, 1, 0, s);
        launch_jacobi_check(buf[cur], ld, n, tol, w.sdbl, w.scal, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(ctx->pinned + kScNotConv, w.scal + kScNotConv, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (ctx->pinned[kScNotConv] == 0) {
            converged = true;
            break;
        }
        if (sweeps >= max_sweeps) break;
        for (int32_t r = 0; r <= nb - 1; ++r) {  // r = nb - 1 is the flush of the last round
            JacobiRound jr;
            jr.Gin = buf[cur];
            jr.Gout = buf[cur ^ 1];
            jr.W = w.W;
            jr.ld = ld;
            jr.npad = npad;
            jr.round_cur = r;
            jr.round_prev = r - 1;
            jr.has_prev = r > 0;
            jr.do_solve = r < nb - 1;
            jr.Jprev = w.J + ((r + 1) & 1) * jsz;
            jr.Sprev = w.S + ((r + 1) & 1) * jsz;
            jr.fprev = w.jflag + ((r + 1) & 1) * npairs;
            jr.Jcur = w.J + (r & 1) * jsz;
            jr.Scur = w.S + (r & 1) * jsz;
            jr.fcur = w.jflag + (r & 1) * npairs;
            jr.sdbl = w.sdbl;
            jr.tol = tol;
            jr.inner_sweeps = npairs == 1 ? 40 : 1;
            launch_jacobi_round(jr, s);
            if (jr.has_prev) cur ^= 1;
        }
        HIP_TRY(hipGetLastError());
        sweeps += 1;
    }
    launch_jacobi_diag(buf[cur], ld, n, w.lam, s);
    HIP_TRY(hipGetLastError());
    if (sweeps_out) *sweeps_out = sweeps;
    if (!converged) return fail(RANKY_E_NOT_CONVERGED, "Jacobi did not converge in %d sweeps", max_sweeps);
    return RANKY_OK;
}

}  // namespace

extern "C" {

const char *ranky_last_error(void) { return g_err; }
const char *ranky_version(void) { return "ranky-mi355x 0.1 (gfx950)"; }

ranky_status ranky_default_opts(ranky_opts *o) {
    if (!o) return fail(RANKY_E_INVALID, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->n_blocks = 0;
    o->gram_prec = RANKY_PREC_FP64;
    o->refine = 0;
    o->max_sweeps = kDefaultSweeps;
    o->validate = 1;
    o->v_dtype = RANKY_F64;
    o->timing = 0;
    return RANKY_OK;
}

ranky_status ranky_ctx_create(int device, ranky_ctx **out) {
    if (!out) return fail(RANKY_E_INVALID, "out is NULL");
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(RANKY_E_INVALID, "device %d of %d", device, count);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    ranky_ctx *c = new ranky_ctx();
    c->device = device;
    c->cu_count = prop.multiProcessorCount;
    size_t lds = prop.sharedMemPerBlock;
    if (lds > 160 * 1024) lds = 160 * 1024;
    c->lds_limit = lds > 4096 ? lds - 4096 : lds;  // room for the kernels' static LDS
    void *pin = nullptr;
    hipError_t e = hipHostMalloc(&pin, 4096, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return fail(RANKY_E_DEVICE, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    c->pinned = static_cast<int32_t *>(pin);
    for (auto &ev : c->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) return fail(RANKY_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
    e = occupancy_set_attributes(kMaxM);
    if (e == hipSuccess) e = gram_set_attributes(c->lds_limit);
    if (e == hipSuccess) e = select_set_attributes();
    if (e != hipSuccess) return fail(RANKY_E_DEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(e));
    *out = c;
    return RANKY_OK;
}

ranky_status ranky_ctx_destroy(ranky_ctx *ctx) {
    if (!ctx) return RANKY_OK;
    for (auto &ev : ctx->ev) hipEventDestroy(ev);
    hipHostFree(ctx->pinned);
    delete ctx;
    return RANKY_OK;
}

size_t ranky_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t k, const ranky_opts *opts) {
    if (M < 1 || N < 1 || k < 1 || k > M || M > kMaxM || nnz < 0) return 0;
    const ranky_opts o = resolved(opts, N);
    if (o.n_blocks < 1 || o.n_blocks > N) return 0;
    return make_plan(M, N, nnz, k, o.n_blocks, true, wants_refine(o, k)).total;
}

size_t ranky_step_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t D) {
    if (M < 1 || N < 1 || M > kMaxM || nnz < 0 || D < 1 || D > N) return 0;
    return make_plan(M, N, nnz, 1, D, false).total;
}

ranky_status ranky_svd(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, double tol,
                       const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, double *U, void *V,
                       ranky_info *info, ranky_stream_t stream) {
    if (info) std::memset(info, 0, sizeof(*info));
    auto finish = [&](ranky_status st) {
        if (info) info->status = st;
        return st;
    };
    if (!ctx) return finish(fail(RANKY_E_INVALID, "ctx is NULL"));
    ranky_status st = check_csc_args(A, M, N);
    if (st) return finish(st);
    if (k < 1 || k > M) return finish(fail(RANKY_E_INVALID, "k=%d must be in [1, M=%d]", k, M));
    if (!(tol >= 0.0)) return finish(fail(RANKY_E_INVALID, "tol must be >= 0"));
    if (!sigma || !U || !V) return finish(fail(RANKY_E_INVALID, "NULL output"));
    const ranky_opts o = resolved(opts, N);
    if (o.n_blocks < 1 || o.n_blocks > N) return finish(fail(RANKY_E_INVALID, "n_blocks=%d outside [1, N]", o.n_blocks));
    if (o.gram_prec != RANKY_PREC_FP64 && o.gram_prec != RANKY_PREC_FP32)
        return finish(fail(RANKY_E_INVALID, "gram_prec=%d", o.gram_prec));
    if (o.v_dtype != RANKY_F32 && o.v_dtype != RANKY_F64) return finish(fail(RANKY_E_INVALID, "v_dtype=%d", o.v_dtype));
    if (o.refine < 0 || o.refine > 1) return finish(fail(RANKY_E_INVALID, "refine=%d (0 or 1)", o.refine));
    if (o.refine && k > kMaxRefineK) return finish(fail(RANKY_E_INVALID, "refine needs k <= %d", kMaxRefineK));
    const bool refine = wants_refine(o, k);
    const Plan p = make_plan(M, N, A->nnz, k, o.n_blocks, true, refine);
    if (!workspace || ws_bytes < p.total)
        return finish(fail(RANKY_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, p.total));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return finish(fail(RANKY_E_DEVICE, "hipSetDevice"));
    const Ptrs w = carve(p, workspace);
    const CscView Av = view(A);
    const bool timing = o.timing != 0;
    if (timing) hipEventRecord(ctx->ev[0], s);

    int32_t n = 0;
    st = run_occupancy(ctx, p, w, Av, o.validate, nullptr, w.lonely, w.single, w.rownnz, s, &n);
    if (st) return finish(st);
    if (timing) hipEventRecord(ctx->ev[1], s);
    int32_t sweeps = 0;
    const int32_t npad = round_up64(n > 0 ? n : 1);
    if (n > 0) {
        launch_row_offsets(w.hist, w.rowptr, M, p.nchunks, s);
        launch_transpose(Av, M, N, p.D, p.cpb, p.nchunks, w.hist, w.csrk, w.csrend, w.csrcol, s);
        if (timing) hipEventRecord(ctx->ev[2], s);
        launch_gram(Av, M, n, npad, npad, w.rowptr, w.r2m, w.csrk, w.csrend, w.G, o.gram_prec, ctx->lds_limit, s);
        if (hipGetLastError() != hipSuccess) return finish(fail(RANKY_E_DEVICE, "Gram launch failed"));
        if (timing) hipEventRecord(ctx->ev[3], s);
        st = run_jacobi(ctx, w, n, o.max_sweeps, s, &sweeps);
        if (st) return finish(st);
    } else if (timing) {
        hipEventRecord(ctx->ev[2], s);
        hipEventRecord(ctx->ev[3], s);
    }
    if (timing) hipEventRecord(ctx->ev[4], s);
    const double u64 = std::ldexp(1.0, -53);
    const double u_gram = (o.gram_prec == RANKY_PREC_FP64 || refine) ? u64 : std::ldexp(1.0, -24);
    launch_select(w.lam, n, k, n, tol, u_gram, w.perm, sigma, w.scal, w.sdbl, s);
    launch_gather_u(w.W, npad, n, M, k, w.perm, w.m2r, w.empty, refine ? w.U0 : U, s);
    if (timing) hipEventRecord(ctx->ev[5], s);
    if (refine) {
        // Rayleigh-Ritz with the exact operator: H = U0^T (A A^T) U0 in FP64
        if (n > 0) {
            launch_rr_z(Av, N, k, w.U0, w.Z, ctx->cu_count, s);
            launch_rr_rows(Av, w.rownnz, w.rowptr, M, A->nnz, k, w.csrk, w.csrcol, w.Z, w.seg, w.part, w.Y, s);
        } else {
            launch_fill_f64(w.Y, (int64_t)M * k, 0.0, s);
        }
        const int32_t kpad = round_up64(k);
        launch_rr_h(w.U0, w.Y, M, k, kpad, w.G, s);
        if (hipGetLastError() != hipSuccess) return finish(fail(RANKY_E_DEVICE, "refine launch failed"));
        int32_t sw2 = 0;
        st = run_jacobi(ctx, w, k, o.max_sweeps, s, &sw2);
        if (st) return finish(st);
        sweeps += sw2;
        launch_select(w.lam, k, k, n, tol, u64, w.perm, sigma, w.scal, w.sdbl, s);
        launch_rr_apply(w.U0, w.W, kpad, w.perm, M, k, U, s);
    }
    if (timing) hipEventRecord(ctx->ev[6], s);
    launch_backproject(Av, N, k, U, sigma, w.scal + kScRank, V, o.v_dtype, ctx->cu_count, s);
    if (timing) hipEventRecord(ctx->ev[7], s);
    if (hipGetLastError() != hipSuccess) return finish(fail(RANKY_E_DEVICE, "kernel launch failed"));
    HIP_TRY(hipMemcpyAsync(ctx->pinned, w.scal, sizeof(int32_t) * kScCount, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ctx->pinned + kScCount, w.sdbl, sizeof(double) * kSdCount, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        const double *sd = reinterpret_cast<const double *>(ctx->pinned + kScCount);
        info->rank = ctx->pinned[kScRank];
        info->n_nonempty = n;
        info->empty_rows = M - n;
        info->sweeps = sweeps;
        info->n_blocks = p.D;
        info->tau = sd[kSdTau];
        info->sigma_max = sd[kSdSigmaMax];
        std::vector<int32_t> lon(p.D);
        HIP_TRY(hipMemcpy(lon.data(), w.lonely, sizeof(int32_t) * p.D, hipMemcpyDeviceToHost));
        for (int32_t b = 0; b < p.D; ++b) {
            if (lon[b] > info->lonely_max) info->lonely_max = lon[b];
            info->lonely_blocks += lon[b] > 0;
        }
        if (timing) {
            float t = 0.f;
            const int pairs[7][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}, {5, 6}, {6, 7}};
            for (int i = 0; i < 7; ++i) {
                hipEventElapsedTime(&t, ctx->ev[pairs[i][0]], ctx->ev[pairs[i][1]]);
                info->ms[i] = t;
            }
            hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[7]);
            info->ms[7] = t;
        }
    }
    return finish(RANKY_OK);
}

ranky_status ranky_occupancy(const ranky_csc *A, int32_t M, int64_t N, int32_t D, int32_t *cnt, int32_t *rownnz,
                             int32_t *lonely, int32_t *single, void *workspace, size_t ws_bytes,
                             ranky_stream_t stream) {
    ranky_status st = check_csc_args(A, M, N);
    if (st) return st;
    if (D < 1 || D > N) return fail(RANKY_E_INVALID, "D=%d outside [1, N]", D);
    if (!cnt || !rownnz || !lonely || !single) return fail(RANKY_E_INVALID, "NULL output");
    const Plan p = make_plan(M, N, A->nnz, 1, D, false);
    if (!workspace || ws_bytes < p.total) return fail(RANKY_E_NOMEM, "workspace %zu < %zu", ws_bytes, p.total);
    // the occupancy pass needs only a context-free pinned read-back; use a local one
    ranky_ctx tmp;
    int32_t pin_local[kScCount];
    void *pin = nullptr;
    HIP_TRY(hipHostMalloc(&pin, sizeof(pin_local), hipHostMallocDefault));
    tmp.pinned = static_cast<int32_t *>(pin);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Ptrs w = carve(p, workspace);
    int32_t n = 0;
    st = run_occupancy(&tmp, p, w, view(A), 1, cnt, lonely, single, rownnz, s, &n);
    hipHostFree(pin);
    return st;
}

ranky_status ranky_gram(const ranky_csc *A, int32_t M, int64_t N, int32_t prec, double *G, void *workspace,
                        size_t ws_bytes, ranky_stream_t stream) {
    ranky_status st = check_csc_args(A, M, N);
    if (st) return st;
    if (!G) return fail(RANKY_E_INVALID, "G is NULL");
    if (prec != RANKY_PREC_FP64 && prec != RANKY_PREC_FP32) return fail(RANKY_E_INVALID, "prec=%d", prec);
    const int32_t D = default_blocks(N);
    const Plan p = make_plan(M, N, A->nnz, 1, D, false);
    if (!workspace || ws_bytes < p.total) return fail(RANKY_E_NOMEM, "workspace %zu < %zu", ws_bytes, p.total);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    size_t lds = prop.sharedMemPerBlock;
    if (lds > 160 * 1024) lds = 160 * 1024;
    lds = lds > 4096 ? lds - 4096 : lds;
    HIP_TRY(occupancy_set_attributes(kMaxM));
    HIP_TRY(gram_set_attributes(lds));
    ranky_ctx tmp;
    void *pin = nullptr;
    HIP_TRY(hipHostMalloc(&pin, sizeof(int32_t) * kScCount, hipHostMallocDefault));
    tmp.pinned = static_cast<int32_t *>(pin);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Ptrs w = carve(p, workspace);
    const CscView Av = view(A);
    int32_t n = 0;
    st = run_occupancy(&tmp, p, w, Av, 1, nullptr, w.lonely, w.single, w.rownnz, s, &n);
    hipHostFree(pin);
    if (st) return st;
    const int32_t npad = round_up64(n > 0 ? n : 1);
    if (n > 0) {
        launch_row_offsets(w.hist, w.rowptr, M, p.nchunks, s);
        launch_transpose(Av, M, N, p.D, p.cpb, p.nchunks, w.hist, w.csrk, w.csrend, w.csrcol, s);
        launch_gram(Av, M, n, npad, npad, w.rowptr, w.r2m, w.csrk, w.csrend, w.G, prec, lds, s);
        launch_scatter_gram(w.G, npad, w.m2r, M, G, s);
    } else {
        launch_fill_f64(G, (int64_t)M * M, 0.0, s);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return RANKY_OK;
}

size_t ranky_eigh_workspace_bytes(int32_t n) {
    if (n < 1 || n > kMaxM) return 0;
    const int32_t npad = round_up64(n);
    size_t b = 0;
    b += align_up(sizeof(int32_t) * kScCount) + align_up(sizeof(double) * kSdCount);
    const size_t npairs = (size_t)(npad / kJacobiPair);
    b += 3 * align_up(sizeof(double) * (size_t)npad * npad);
    b += 2 * align_up(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair);
    b += align_up(sizeof(int32_t) * 2 * npairs);
    b += align_up(sizeof(double) * npad);
    return b;
}

ranky_status ranky_eigh(int32_t n, const double *G, double *lambda, double *Q, int32_t max_sweeps, int32_t *sweeps,
                        void *workspace, size_t ws_bytes, ranky_stream_t stream) {
    if (n < 1 || n > kMaxM) return fail(RANKY_E_INVALID, "n=%d outside [1, %d]", n, kMaxM);
    if (!G || !lambda || !Q) return fail(RANKY_E_INVALID, "NULL argument");
    const size_t need = ranky_eigh_workspace_bytes(n);
    if (!workspace || ws_bytes < need) return fail(RANKY_E_NOMEM, "workspace %zu < %zu", ws_bytes, need);
    const int32_t npad = round_up64(n);
    char *b = static_cast<char *>(workspace);
    Ptrs w;
    std::memset(&w, 0, sizeof(w));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *ptr = b + off;
        off += align_up(bytes);
        return ptr;
    };
    w.scal = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * kScCount));
    w.sdbl = reinterpret_cast<double *>(take(sizeof(double) * kSdCount));
    const size_t npairs = (size_t)(npad / kJacobiPair);
    w.G = reinterpret_cast<double *>(take(sizeof(double) * (size_t)npad * npad));
    w.G2 = reinterpret_cast<double *>(take(sizeof(double) * (size_t)npad * npad));
    w.W = reinterpret_cast<double *>(take(sizeof(double) * (size_t)npad * npad));
    w.J = reinterpret_cast<double *>(take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair));
    w.S = reinterpret_cast<double *>(take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair));
    w.jflag = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * 2 * npairs));
    w.lam = reinterpret_cast<double *>(take(sizeof(double) * npad));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ranky_ctx tmp;
    void *pin = nullptr;
    HIP_TRY(hipHostMalloc(&pin, sizeof(int32_t) * kScCount, hipHostMallocDefault));
    tmp.pinned = static_cast<int32_t *>(pin);
    launch_fill_i32(w.scal, kScCount, 0, s);
    launch_pad_copy(G, n, w.G, npad, npad, s);
    int32_t sw = 0;
    ranky_status st = run_jacobi(&tmp, w, n, max_sweeps > 0 ? max_sweeps : kDefaultSweeps, s, &sw);
    hipHostFree(pin);
    if (sweeps) *sweeps = sw;
    hipMemcpyAsync(lambda, w.lam, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
    launch_unpad_copy(w.W, npad, n, Q, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return st;
}

ranky_status ranky_backproject(const ranky_csc *A, int32_t M, int64_t N, int32_t k, const double *U,
                               const double *sigma, const int32_t *rank, void *V, int32_t v_dtype,
                               ranky_stream_t stream) {
    ranky_status st = check_csc_args(A, M, N);
    if (st) return st;
    if (k < 1 || k > M) return fail(RANKY_E_INVALID, "k=%d outside [1, M]", k);
    if (!U || !sigma || !rank || !V) return fail(RANKY_E_INVALID, "NULL argument");
    if (v_dtype != RANKY_F32 && v_dtype != RANKY_F64) return fail(RANKY_E_INVALID, "v_dtype=%d", v_dtype);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    launch_backproject(view(A), N, k, U, sigma, rank, V, v_dtype, cus, reinterpret_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return RANKY_OK;
}

}  // extern "C"

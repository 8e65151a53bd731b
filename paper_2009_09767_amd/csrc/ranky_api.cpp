// ranky_api.cpp -- host runtime behind include/ranky.h: argument checks, the
// workspace plan, a batch engine that drives every kernel over a table of
// per-matrix descriptors (a single matrix is a batch of one), and status read-back.
#include "ranky.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "launch_util.hpp"

// Launch-shape choices of the autotuner for one problem shape (results do not depend on them).
struct TuneCfg {
    int32_t bp_per_cu = 32;   // back-projection workgroups per CU
    int32_t jsched = 0;       // Jacobi round launch shape (MatDesc::jsched)
};
// M, N, nnz, k, value dtype, V dtype, Gram precision
using TuneKey = std::tuple<int32_t, int64_t, int64_t, int32_t, int32_t, int32_t, int32_t>;

struct ranky_ctx {
    std::map<TuneKey, TuneCfg> tuned;     // filled by ranky_autotune
    int device = 0;
    int cu_count = 0;
    size_t lds_limit = 0;      // dynamic LDS the Gram kernel may use per workgroup
    void *pinned = nullptr;    // host staging for descriptor uploads and scalar read-back
    void *pinned_dev = nullptr;   // the same memory as a device address (kernels write sweep state there)
    size_t pinned_bytes = 0;
    hipEvent_t ev[11] = {};     // [0..7] phase marks, [9] [10] span of a sweep's round launches
    hipGraphExec_t sweep_graph = nullptr;  // captured Jacobi sweep of the last graph batch
    const void *sweep_graph_key = nullptr;
    size_t sweep_graph_sig = 0;
    // ranky_svd_async: at most one call in flight per context, run on `worker`
    std::mutex amu;
    std::thread worker;
    uint64_t aticket = 0;    // ticket of the last call started
    int astate = 0;          // 0 idle (or result handed over), 1 running, 2 finished, not yet queried
    ranky_status aresult = RANKY_OK;
    ranky_info ainfo = {};
    std::string aerr;
    // per-block lonely and single-entry counts of the last call (ranky_info points here)
    std::vector<int32_t> blk_host;
};

namespace {

using namespace ranky;

thread_local char g_err[512] = "";
constexpr int32_t kDefaultSweeps = 40;
constexpr int32_t kInnerSweeps = 1;
constexpr int32_t kMaxRefineK = 1024;
constexpr double kJacobiTolFp32Gram = 1e-8;

ranky_status fail(ranky_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(RANKY_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kWorkspaceAlign = 256;   // workspace base; every carved buffer keeps it
size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Kernel attributes (dynamic LDS limits) are set once per device for the whole process,
// under a lock: contexts created on several threads (serving slots) never set them while
// another thread launches.
std::mutex g_attr_mu;
std::vector<int> g_attr_devices;

hipError_t kernel_attributes(int device, size_t lds_limit) {
    std::lock_guard<std::mutex> lk(g_attr_mu);
    if (std::find(g_attr_devices.begin(), g_attr_devices.end(), device) != g_attr_devices.end()) return hipSuccess;
    hipError_t e = occupancy_set_attributes(kMaxM);
    if (e == hipSuccess) e = gram_set_attributes(lds_limit);
    if (e == hipSuccess) e = select_set_attributes();
    if (e == hipSuccess) g_attr_devices.push_back(device);
    return e;
}

// ---------------------------------------------------------------------------
// per-matrix workspace plan
// ---------------------------------------------------------------------------

struct Plan {
    int32_t M = 0, k = 0, D = 0, cpb = 0, ccols = 0, npad = 0;
    int64_t N = 0, nnz = 0, nchunks = 0;
    size_t o_scal = 0, o_sdbl = 0, o_jstate = 0, o_hist = 0, o_rownnz = 0, o_rowptr = 0, o_m2r = 0, o_r2m = 0;
    size_t o_empty = 0, o_lonely = 0, o_single = 0, o_csrk = 0, o_csrend = 0, o_csrcol = 0;
    size_t o_gsegp = 0, o_gslot = 0, o_gpart = 0, o_dense = 0, o_dpart = 0;
    int32_t dwg = 0;
    size_t o_G = 0, o_G2 = 0, o_W = 0, o_J = 0, o_S = 0, o_jflag = 0, o_lam = 0, o_perm = 0;
    size_t o_U0 = 0, o_part = 0, o_uf = 0, total = 0;
    size_t o_bstart = 0;
    bool solver = false, refine = false, explicit_blocks = false, uf = false;
};

// bstart (host, may be NULL): the caller's D + 1 block boundaries; the widest block sets
// the chunks per block, and the boundaries get a device copy in the workspace.
// dense: room for the split-bf16 dense tiles (a single matrix; used with gram_prec BF16X3).
// uf: room for an FP32 copy of U (solver plans with an FP32 V: the back-projection gathers it).
Plan make_plan(int32_t M, int64_t N, int64_t nnz, int32_t k, int32_t D, bool solver, bool refine,
               const int64_t *bstart = nullptr, bool dense = false, bool uf = false) {
    Plan p;
    p.M = M;
    p.N = N;
    p.nnz = nnz;
    p.k = k;
    p.D = D;
    int64_t maxw = (N + D - 1) / D;
    if (bstart) {
        maxw = 0;
        for (int32_t b = 0; b < D; ++b) maxw = std::max<int64_t>(maxw, bstart[b + 1] - bstart[b]);
    }
    // chunks of kChunkCols columns, halved (down to kChunkColsMin) while the matrix has
    // fewer than kChunkTarget of them: the scan and the transpose run one workgroup per
    // chunk, and the row-major copy does not depend on the cut
    p.ccols = kChunkCols;
    auto chunks_of = [&](int64_t cc) { return (int64_t)D * std::max<int64_t>(1, (maxw + cc - 1) / cc); };
    while (p.ccols > kChunkColsMin && chunks_of(p.ccols) < kChunkTarget) p.ccols /= 2;
    p.cpb = (int32_t)std::max<int64_t>(1, (maxw + p.ccols - 1) / p.ccols);
    p.nchunks = (int64_t)D * p.cpb;
    p.npad = jacobi_npad(M);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    p.explicit_blocks = bstart != nullptr;
    if (bstart) p.o_bstart = take(sizeof(int64_t) * ((size_t)D + 1));
    const size_t nz = (size_t)(nnz > 0 ? nnz : 1);
    p.o_scal = take(sizeof(int32_t) * kScCount);
    p.o_sdbl = take(sizeof(double) * kSdCount);
    p.o_jstate = take(sizeof(int32_t) * kJsCount);
    p.o_hist = take(sizeof(int32_t) * (size_t)p.nchunks * M);
    p.o_rownnz = take(sizeof(int32_t) * M);
    p.o_rowptr = take(sizeof(int32_t) * (M + 1));
    p.o_m2r = take(sizeof(int32_t) * M);
    p.o_r2m = take(sizeof(int32_t) * M);
    p.o_empty = take(sizeof(int32_t) * M);
    p.o_lonely = take(sizeof(int32_t) * D);
    p.o_single = take(sizeof(int32_t) * D);
    p.o_csrk = take(sizeof(int32_t) * nz);
    p.o_csrend = take(sizeof(int32_t) * nz);
    p.o_csrcol = take(sizeof(int32_t) * nz);
    p.o_gsegp = take(sizeof(int32_t) * (M + 1));
    p.o_gslot = take(sizeof(int32_t) * (M + 1));
    p.o_gpart = take(sizeof(double) * (size_t)gram_part_slots(nnz) * p.npad);
    p.o_dense = take(sizeof(int32_t) * kDenseRows);
    p.dwg = dense ? gram_dense_wgs(N) : 0;
    p.o_dpart = take(sizeof(double) * kDenseRows * kDenseRows * (size_t)p.dwg);
    p.o_G = take(sizeof(double) * (size_t)p.npad * p.npad);
    if (solver) {
        p.solver = true;
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
            p.o_part = take(sizeof(double) * rr_part_doubles(N, k));
        }
        if (uf) {
            p.uf = true;
            p.o_uf = take(sizeof(float) * (size_t)M * k);
        }
    }
    p.total = off;
    return p;
}

struct Refine {
    double *U0 = nullptr, *part = nullptr;   // U0 (M x k) and the partial H tiles
};

// Descriptor of one matrix with its workspace carved at `base`.
MatDesc carve(const Plan &p, char *base, Refine *rf) {
    MatDesc d;
    std::memset(&d, 0, sizeof(d));
    auto i32 = [&](size_t o) { return reinterpret_cast<int32_t *>(base + o); };
    auto f64 = [&](size_t o) { return reinterpret_cast<double *>(base + o); };
    d.M = p.M;
    d.N = p.N;
    d.nnz = p.nnz;
    d.k = p.k;
    d.D = p.D;
    d.cpb = p.cpb;
    d.ccols = p.ccols;
    d.gseg = gram_seg_len(p.nnz);
    d.bstart = p.explicit_blocks ? reinterpret_cast<const int64_t *>(base + p.o_bstart) : nullptr;
    d.nchunks = p.nchunks;
    d.npad = kJacobiPair;
    d.scal = i32(p.o_scal);
    d.sdbl = f64(p.o_sdbl);
    d.jstate = i32(p.o_jstate);
    d.hist = i32(p.o_hist);
    d.rownnz = i32(p.o_rownnz);
    d.rowptr = i32(p.o_rowptr);
    d.m2r = i32(p.o_m2r);
    d.r2m = i32(p.o_r2m);
    d.empty = i32(p.o_empty);
    d.lonely = i32(p.o_lonely);
    d.single = i32(p.o_single);
    d.csrk = i32(p.o_csrk);
    d.csrend = i32(p.o_csrend);
    d.csrcol = i32(p.o_csrcol);
    d.gsegp = i32(p.o_gsegp);
    d.gslot = i32(p.o_gslot);
    d.gpart = f64(p.o_gpart);
    d.dense = i32(p.o_dense);
    d.dwg = p.dwg;
    d.dpart = f64(p.o_dpart);
    d.bp_per_cu = 32;
    d.jsched = 0;
    d.G = f64(p.o_G);
    if (p.solver) {
        d.G2 = f64(p.o_G2);
        d.W = f64(p.o_W);
        d.J = f64(p.o_J);
        d.S = f64(p.o_S);
        d.jflag = i32(p.o_jflag);
        d.lam = f64(p.o_lam);
        d.perm = i32(p.o_perm);
        d.Uf = p.uf ? reinterpret_cast<float *>(base + p.o_uf) : nullptr;
    }
    if (rf && p.refine) {
        rf->U0 = f64(p.o_U0);
        rf->part = f64(p.o_part);
    }
    return d;
}

// ---------------------------------------------------------------------------
// batch header: device descriptor table, workgroup maps, round tables, read-back
// ---------------------------------------------------------------------------

// kPhBack, kPhBack2, kPhBack4: back-projection of the matrices with 1, 2, 4 output pairs per lane
enum Phase { kPhChunks, kPhRows, kPhGram, kPhGramRed, kPhJinit, kPhJcheck, kPhJdiag, kPhGather, kPhBack, kPhBack2, kPhBack4, kPhCount };

struct Header {
    size_t o_desc = 0, o_wp = 0, o_rwp = 0, o_rtab = 0, o_col_i = 0, o_col_f = 0, o_col_b = 0, o_js = 0, total = 0;
    int32_t count = 0, slots = 0, nb_max = 0;
    int64_t sum_d = 0;   // blocks over all matrices (the per-block counts read back at the end)
};

Header make_header(int32_t count, int32_t slots, int32_t nb_max, int64_t sum_d = 0) {
    Header h;
    h.count = count;
    h.slots = slots;
    h.nb_max = nb_max;
    h.sum_d = sum_d;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    h.o_desc = take(sizeof(MatDesc) * slots);
    h.o_wp = take(sizeof(int32_t) * (size_t)kPhCount * (slots + 1));
    h.o_rwp = take(sizeof(int32_t) * (size_t)nb_max * (slots + 1));
    h.o_rtab = take(round_args_bytes() * (size_t)nb_max * slots);
    h.o_col_i = take(sizeof(int32_t) * kColI * slots);
    h.o_col_f = take(sizeof(double) * 2 * slots);
    h.o_col_b = take(sizeof(int32_t) * 2 * (size_t)(sum_d > 0 ? sum_d : 1));
    // the sweep state the device writes to host memory (3 per matrix, then the epoch); the
    // device copy of this range holds the epoch counter
    h.o_js = take(sizeof(int32_t) * (3 * (size_t)slots + 1));
    h.total = off;
    return h;
}

int32_t default_blocks(int64_t N) {
    int64_t d = (N + 16383) / 16384;
    if (d < 1) d = 1;
    if (d > N) d = N;
    return (int32_t)d;
}

// refining: the call runs the Rayleigh-Ritz step for a single matrix (ranky_svd and its
// relatives, serving); refine = -1 (automatic) resolves to 1 there for a non-FP64 Gram and
// k <= kMaxRefineK, and to 0 everywhere else (ranky_batch).
ranky_opts resolved(const ranky_opts *in, bool refining, int32_t k = 1) {
    ranky_opts o;
    ranky_default_opts(&o);
    if (in) o = *in;
    if (o.max_sweeps <= 0) o.max_sweeps = kDefaultSweeps;
    if (o.refine < 0) o.refine = refining && o.gram_prec != RANKY_PREC_FP64 && k <= kMaxRefineK ? 1 : 0;
    return o;
}

bool wants_refine(const ranky_opts &o, int32_t k) { return o.refine > 0 && k <= kMaxRefineK; }

ranky_status check_csc_args(const ranky_csc *A, int32_t M, int64_t N) {
    if (!A) return fail(RANKY_E_INVALID, "A is NULL");
    if (M < 1 || N < 1) return fail(RANKY_E_INVALID, "M=%d N=%lld must be >= 1", M, (long long)N);
    if (M > kMaxM) return fail(RANKY_E_INVALID, "M=%d exceeds %d", M, kMaxM);
    if (N > (int64_t)0x7ffffffe) return fail(RANKY_E_INVALID, "N=%lld exceeds int32 column pointers", (long long)N);
    if (A->nnz < 0 || A->nnz > (int64_t)0x7fffffff)
        return fail(RANKY_E_INVALID, "nnz=%lld out of range", (long long)A->nnz);
    if (!A->colptr || (A->nnz > 0 && (!A->rowidx || !A->values))) return fail(RANKY_E_INVALID, "NULL CSC array");
    if (A->dtype != RANKY_F32 && A->dtype != RANKY_F64) return fail(RANKY_E_INVALID, "bad dtype %d", A->dtype);
    return RANKY_OK;
}

ranky_status check_opts(const ranky_opts &o) {
    if (o.gram_prec != RANKY_PREC_FP64 && o.gram_prec != RANKY_PREC_FP32 && o.gram_prec != RANKY_PREC_BF16X3)
        return fail(RANKY_E_INVALID, "gram_prec=%d", o.gram_prec);
    if (o.v_dtype != RANKY_F32 && o.v_dtype != RANKY_F64) return fail(RANKY_E_INVALID, "v_dtype=%d", o.v_dtype);
    if (o.refine < 0 || o.refine > 1) return fail(RANKY_E_INVALID, "refine=%d (0, 1, or -1 = automatic)", o.refine);
    return RANKY_OK;
}

// One matrix of a job (host view).
struct Job {
    ranky_csc A;
    const int64_t *bstart;   // host: the caller's block boundaries, or NULL
    int64_t N;
    int32_t M, k, D;
    double *sigma, *U;
    void *V;
};

ranky_status ensure_pinned(ranky_ctx *ctx, size_t bytes) {
    if (ctx->pinned_bytes >= bytes) return RANKY_OK;
    // a call that failed part-way may have left kernels writing sweep state into the old
    // buffer: let them finish before it is freed
    if (ctx->pinned) {
        hipDeviceSynchronize();
        hipHostFree(ctx->pinned);
    }
    ctx->pinned = nullptr;
    ctx->pinned_dev = nullptr;
    ctx->pinned_bytes = 0;
    const size_t want = std::max<size_t>(bytes, 1 << 16);
    HIP_TRY(hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
    HIP_TRY(hipHostGetDevicePointer(&ctx->pinned_dev, ctx->pinned, 0));
    ctx->pinned_bytes = want;
    return RANKY_OK;
}

// Fills the workgroup prefix for one phase: wp[i+1] = wp[i] + blocks(i).
template <typename F>
int64_t fill_wp(int32_t *wp, int count, F blocks) {
    wp[0] = 0;
    for (int i = 0; i < count; ++i) wp[i + 1] = wp[i] + (int32_t)blocks(i);
    return wp[count];
}

// Drives the kernels for `count` matrices whose descriptors live in a device header.
// Every staging write is followed by its upload and, before the staging area is
// reused, by a read-back that synchronises the stream.
struct Engine {
    ranky_ctx *ctx = nullptr;
    hipStream_t s = nullptr;
    int count = 0;
    std::vector<MatDesc> d;          // host copies
    std::vector<int32_t> status;     // per matrix ranky_status so far
    std::vector<int32_t> sweeps, notconv;
    std::vector<int32_t> gsegs;      // Gram workgroups of the nonempty rows, per matrix (from the scan)
    Header h;
    char *hdr = nullptr;             // device header base
    int64_t nblk[kPhCount] = {};
    std::vector<int64_t> rblk;
    int32_t maxM = 1, maxn = 1, nb_max = 0;
    int32_t sweeps_cap = kDefaultSweeps;
    bool time_rounds = false;        // timing mode: events around the round launches of each active sweep
    double round_ms = 0.0;
    int32_t round_launches = 0;
    size_t jround_lds = 0;           // dynamic LDS of the round launches (one workgroup per CU when set)

    char *stage() { return static_cast<char *>(ctx->pinned); }
    MatDesc *ddesc() { return reinterpret_cast<MatDesc *>(hdr + h.o_desc); }
    int32_t *dwp(int ph) { return reinterpret_cast<int32_t *>(hdr + h.o_wp) + (size_t)ph * (h.slots + 1); }
    int32_t *drwp(int r) { return reinterpret_cast<int32_t *>(hdr + h.o_rwp) + (size_t)r * (h.slots + 1); }
    void *drtab(int r) { return hdr + h.o_rtab + round_args_bytes() * (size_t)r * h.slots; }
    int32_t *hwp(int ph) { return reinterpret_cast<int32_t *>(stage() + h.o_wp) + (size_t)ph * (h.slots + 1); }
    int32_t *hrwp(int r) { return reinterpret_cast<int32_t *>(stage() + h.o_rwp) + (size_t)r * (h.slots + 1); }
    char *hrtab(int r) { return stage() + h.o_rtab + round_args_bytes() * (size_t)r * h.slots; }

    ranky_status upload(size_t from, size_t bytes) {
        HIP_TRY(hipMemcpyAsync(hdr + from, stage() + from, bytes, hipMemcpyHostToDevice, s));
        return RANKY_OK;
    }
    ranky_status upload_desc() {
        std::memcpy(stage() + h.o_desc, d.data(), sizeof(MatDesc) * count);
        return upload(h.o_desc, sizeof(MatDesc) * count);
    }
    // compact per-matrix scalars (blocking); with blk != NULL also every matrix's per-block
    // lonely and single-entry counts (the header must have room for them: sum_d)
    ranky_status collect(std::vector<int32_t> &iv, std::vector<double> &fv, std::vector<int32_t> *blk = nullptr) {
        int32_t *ci = reinterpret_cast<int32_t *>(hdr + h.o_col_i);
        double *cf = reinterpret_cast<double *>(hdr + h.o_col_f);
        int32_t *cb = blk && h.sum_d > 0 ? reinterpret_cast<int32_t *>(hdr + h.o_col_b) : nullptr;
        launch_batch_collect(ddesc(), count, ci, cf, cb, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(stage() + h.o_col_i, ci, sizeof(int32_t) * kColI * count, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(stage() + h.o_col_f, cf, sizeof(double) * 2 * count, hipMemcpyDeviceToHost, s));
        if (cb)
            HIP_TRY(hipMemcpyAsync(stage() + h.o_col_b, cb, sizeof(int32_t) * 2 * (size_t)h.sum_d,
                                   hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const int32_t *pi = reinterpret_cast<const int32_t *>(stage() + h.o_col_i);
        const double *pf = reinterpret_cast<const double *>(stage() + h.o_col_f);
        iv.assign(pi, pi + kColI * count);
        fv.assign(pf, pf + 2 * count);
        if (cb) {
            const int32_t *pb = reinterpret_cast<const int32_t *>(stage() + h.o_col_b);
            blk->assign(pb, pb + 2 * h.sum_d);
        }
        return RANKY_OK;
    }

    // Alg. 1 scan, validation and structural rank of every matrix; sets n / npad.
    ranky_status scan() {
        int32_t maxD = 1;
        for (const MatDesc &x : d) {
            maxM = std::max(maxM, x.M);
            maxD = std::max(maxD, x.D);
        }
        nblk[kPhChunks] = fill_wp(hwp(kPhChunks), count, [&](int i) { return d[i].nchunks; });
        nblk[kPhRows] = fill_wp(hwp(kPhRows), count, [&](int i) { return (int64_t)(d[i].M + 255) / 256; });
        ranky_status st = upload_desc();
        if (!st) st = upload(h.o_wp, sizeof(int32_t) * (size_t)kPhCount * (h.slots + 1));
        if (st) return st;
        launch_batch_prep(ddesc(), count, s);
        launch_occupancy(ddesc(), dwp(kPhChunks), nblk[kPhChunks], dwp(kPhRows), nblk[kPhRows], count, maxM, maxD, s);
        HIP_TRY(hipGetLastError());
        std::vector<int32_t> iv;
        std::vector<double> fv;
        st = collect(iv, fv);
        if (st) return st;
        for (int i = 0; i < count; ++i) {
            const int32_t bits = iv[kColI * i];
            if (bits & kStCsc) status[i] = RANKY_E_CSC;
            else if (bits & kStNonfinite) status[i] = RANKY_E_NONFINITE;
            d[i].n = status[i] == RANKY_OK ? iv[kColI * i + 1] : 0;
            gsegs[i] = status[i] == RANKY_OK ? iv[kColI * i + 8] : 0;
            d[i].n_tau = d[i].n;
            d[i].npad = jacobi_npad(d[i].n > 0 ? d[i].n : 1);
            maxn = std::max(maxn, d[i].n);
        }
        return RANKY_OK;
    }

    bool live(int i) const { return status[i] == RANKY_OK && d[i].n > 0; }

    // Maps of every later phase and the round tables; one upload.  A matrix whose
    // scan reported a contract violation gets no workgroup in any later phase (the
    // transpose and the Gram index LDS and the row-major copy by its row indices).
    ranky_status plan_rest() {
        nblk[kPhChunks] = fill_wp(hwp(kPhChunks), count, [&](int i) { return status[i] == RANKY_OK ? d[i].nchunks : 0; });
        nblk[kPhRows] = fill_wp(hwp(kPhRows), count,
                                [&](int i) { return status[i] == RANKY_OK ? (int64_t)(d[i].M + 255) / 256 : 0; });
        nblk[kPhGram] = fill_wp(hwp(kPhGram), count,
                                [&](int i) { return live(i) ? (int64_t)gsegs[i] + (d[i].npad - d[i].n) : 0; });
        nblk[kPhGramRed] = fill_wp(hwp(kPhGramRed), count, [&](int i) { return live(i) ? (int64_t)d[i].n : 0; });
        nblk[kPhJinit] = fill_wp(hwp(kPhJinit), count, [&](int i) -> int64_t {
            if (!live(i)) return 0;
            const int64_t sl = ((int64_t)d[i].npad * d[i].npad + 8191) / 8192;
            return std::min<int64_t>(std::max<int64_t>(sl, 1), 64);
        });
        nblk[kPhJcheck] = fill_wp(hwp(kPhJcheck), count, [&](int i) -> int64_t {
            if (!live(i)) return 0;
            const int64_t t = (d[i].n + kJacobiCheckTile - 1) / kJacobiCheckTile;
            return t * (t + 1) / 2;
        });
        nblk[kPhJdiag] = fill_wp(hwp(kPhJdiag), count, [&](int i) { return live(i) ? (int64_t)(d[i].n + 255) / 256 : 0; });
        nblk[kPhGather] = fill_wp(hwp(kPhGather), count, [&](int i) { return status[i] == RANKY_OK ? (int64_t)d[i].k : 0; });
        // back-projection: one matrix gets the tuned grid; a batch shares one grid of that
        // size in proportion to each matrix's V bytes (at least one workgroup each), so the
        // waves walk longer column runs instead of launching millions of tiny workgroups.
        // Each output width (backproject_pairs) has its own launch and workgroup table.
        std::vector<int64_t> bpb(count, 0);
        if (count == 1) {
            if (status[0] == RANKY_OK) bpb[0] = backproject_blocks(d[0].N, ctx->cu_count, d[0].bp_per_cu);
        } else {
            // the width classes run one after the other, so each launch gets the whole grid
            double work[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            int32_t per_cu = 0;
            for (int i = 0; i < count; ++i)
                if (status[i] == RANKY_OK) {
                    work[backproject_pairs(d[i].k)] += (double)d[i].N * d[i].k;
                    per_cu = std::max(per_cu, d[i].bp_per_cu);
                }
            const double grid = (double)ctx->cu_count * (per_cu > 0 ? per_cu : 32);
            for (int i = 0; i < count; ++i)
                if (status[i] == RANKY_OK) {
                    const double w = work[backproject_pairs(d[i].k)];
                    const int64_t share = (int64_t)(grid * ((double)d[i].N * d[i].k) / (w > 0.0 ? w : 1.0));
                    bpb[i] = std::max<int64_t>(1, std::min(share, backproject_blocks(d[i].N, ctx->cu_count, d[i].bp_per_cu)));
                }
        }
        const int32_t widths[3] = {1, 2, 4};
        for (int c = 0; c < 3; ++c)
            nblk[kPhBack + c] = fill_wp(hwp(kPhBack + c), count, [&](int i) -> int64_t {
                return backproject_pairs(d[i].k) == widths[c] ? bpb[i] : 0;
            });
        nb_max = 0;
        bool solo = false, all_solo = true;
        for (int i = 0; i < count; ++i)
            if (live(i)) {
                nb_max = std::max(nb_max, d[i].npad / kJacobiBlock);
                solo = true;
                all_solo = all_solo && (d[i].jsched & 2) != 0;
            }
        // a round's solve workgroups are its critical path: with bit 1 of the schedule set
        // on every matrix, each CU holds one round workgroup, so no update workgroup
        // competes with a subproblem sweep for the CU's issue slots and LDS
        jround_lds = solo && all_solo ? jround_solo_pad(ctx->lds_limit + 4096) : 0;
        rblk.assign(nb_max, 0);
        for (int r = 0; r < nb_max; ++r) {
            rblk[r] = fill_wp(hrwp(r), count, [&](int i) { return live(i) ? round_blocks(d[i], r) : (int64_t)0; });
            for (int i = 0; i < count; ++i) fill_round_args(hrtab(r) + round_args_bytes() * i, d[i], r, kInnerSweeps);
        }
        ranky_status st = upload_desc();
        if (!st) st = upload(h.o_wp, sizeof(int32_t) * (size_t)kPhCount * (h.slots + 1));
        if (!st && nb_max > 0) st = upload(h.o_rwp, sizeof(int32_t) * (size_t)nb_max * (h.slots + 1));
        if (!st && nb_max > 0) st = upload(h.o_rtab, round_args_bytes() * (size_t)nb_max * h.slots);
        return st;
    }

    void enqueue_transpose() {
        launch_row_offsets(ddesc(), dwp(kPhRows), nblk[kPhRows], count, s);
        launch_transpose(ddesc(), dwp(kPhChunks), nblk[kPhChunks], count, maxM, s);
    }

    // sweep state per matrix (active, sweeps, not converged), written by the device
    int32_t *js_dev() { return reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned_dev) + h.o_js); }
    const int32_t *js_host() { return reinterpret_cast<const int32_t *>(stage() + h.o_js); }
    int32_t *epoch_dev() { return reinterpret_cast<int32_t *>(hdr + h.o_js); }
    volatile int32_t *epoch_host() { return reinterpret_cast<volatile int32_t *>(stage() + h.o_js) + 3 * count; }
    int32_t epochs = 0;   // state launches queued (run, not captured) since the counter was reset

    // Waits until the state of the last queued launch is in host memory: the host watches the
    // epoch word instead of sleeping in a stream synchronisation, and falls back to one when
    // the stream has ended or failed (a failure is then reported by the synchronisation).
    ranky_status wait_state() {
        volatile int32_t *ep = epoch_host();
        for (uint32_t it = 1;; ++it) {
            if (*ep == epochs) {
                std::atomic_thread_fence(std::memory_order_acquire);
                return RANKY_OK;
            }
            if ((it & 63) == 0 && hipStreamQuery(s) != hipErrorNotReady) break;
        }
        HIP_TRY(hipStreamSynchronize(s));
        return RANKY_OK;
    }
    bool any_active() {
        const int32_t *js = js_host();
        for (int i = 0; i < count; ++i)
            if (js[3 * i] != 0) return true;
        return false;
    }

    // end of a sweep: convergence test of the current matrices, then the state update
    // (sweep count, verdict, next sweep's activity) published to host memory
    void enqueue_activity() {
        launch_jacobi_check(ddesc(), dwp(kPhJcheck), nblk[kPhJcheck], count, s);
        launch_jacobi_state(ddesc(), count, sweeps_cap, js_dev(), epoch_dev(), s);
    }

    void enqueue_sweep() {
        for (int r = 0; r < nb_max; ++r) launch_jacobi_round(hrtab(r), drtab(r), drwp(r), rblk[r], count, r, jround_lds, s);
        enqueue_activity();
    }

    // Jacobi on every live matrix.  Each sweep = nb_max round launches, sweep count, then
    // the convergence test and activity of the next sweep; one read-back per sweep decides
    // whether any matrix is still active, so no sweep is launched only to find that the
    // previous one converged.  With use_graph the sweep is a replayed HIP graph.
    ranky_status eigensolve(bool use_graph) {
        // the epoch counter starts again at 0 on both sides (the previous solve on this context
        // ended with a synchronisation, so no device write to the host word is pending)
        *epoch_host() = 0;
        epochs = 0;
        launch_fill_i32(epoch_dev(), 1, 0, s);
        launch_jacobi_init(ddesc(), dwp(kPhJinit), nblk[kPhJinit], count, s);
        HIP_TRY(hipGetLastError());
        sweeps.assign(count, 0);
        notconv.assign(count, 0);
        if (nb_max == 0) return RANKY_OK;
        hipGraphExec_t exec = nullptr;
        if (use_graph && s != nullptr && !time_rounds) {
            size_t sig = (size_t)count * 1315423911u ^ (size_t)nb_max;
            for (int r = 0; r < nb_max; ++r) sig = sig * 31 + (size_t)rblk[r];
            for (int ph = 0; ph < kPhCount; ++ph) sig = sig * 31 + (size_t)nblk[ph];
            sig = sig * 31 + jround_lds;
            sig = sig * 31 + reinterpret_cast<uintptr_t>(ctx->pinned_dev);
            // a single matrix's round arguments are captured by value: any change re-captures
            for (int r = 0; r < nb_max; ++r)
                for (size_t i = 0, nb = round_args_bytes() * (size_t)count; i < nb; ++i)
                    sig = sig * 131 + (unsigned char)hrtab(r)[i];
            if (ctx->sweep_graph && ctx->sweep_graph_key == hdr && ctx->sweep_graph_sig == sig) {
                exec = ctx->sweep_graph;
            } else {
                if (ctx->sweep_graph) hipGraphExecDestroy(ctx->sweep_graph);
                ctx->sweep_graph = nullptr;
                hipGraph_t g = nullptr;
                HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                enqueue_sweep();
                HIP_TRY(hipStreamEndCapture(s, &g));
                const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
                hipGraphDestroy(g);
                if (ie != hipSuccess) return fail(RANKY_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
                ctx->sweep_graph = exec;
                ctx->sweep_graph_key = hdr;
                ctx->sweep_graph_sig = sig;
            }
        }
        // the first sweep's activity (read back only when its rounds are timed; otherwise a
        // matrix that is already diagonal just runs one sweep of rounds that exit at once)
        enqueue_activity();
        ++epochs;
        HIP_TRY(hipGetLastError());
        bool active = true;
        if (time_rounds) {
            HIP_TRY(hipStreamSynchronize(s));
            active = any_active();
        }
        for (int32_t sw = 0; sw <= sweeps_cap && active; ++sw) {
            if (exec) {
                HIP_TRY(hipGraphLaunch(exec, s));
            } else if (time_rounds) {
                HIP_TRY(hipEventRecord(ctx->ev[9], s));
                for (int r = 0; r < nb_max; ++r)
                    launch_jacobi_round(hrtab(r), drtab(r), drwp(r), rblk[r], count, r, jround_lds, s);
                HIP_TRY(hipEventRecord(ctx->ev[10], s));
                enqueue_activity();
                HIP_TRY(hipGetLastError());
            } else {
                enqueue_sweep();
                HIP_TRY(hipGetLastError());
            }
            ++epochs;
            if (!time_rounds) {
                const ranky_status ws = wait_state();
                if (ws) return ws;
            } else {
                HIP_TRY(hipStreamSynchronize(s));
                float t = 0.f;
                HIP_TRY(hipEventElapsedTime(&t, ctx->ev[9], ctx->ev[10]));
                round_ms += t;
                for (int r = 0; r < nb_max; ++r) round_launches += rblk[r] > 0 ? 1 : 0;
            }
            active = any_active();
        }
        // the last state holds the convergence test of the final matrices (synchronise in
        // case no sweep ran)
        HIP_TRY(hipStreamSynchronize(s));
        for (int i = 0; i < count; ++i) {
            sweeps[i] = js_host()[3 * i + 1];
            notconv[i] = js_host()[3 * i + 2];
        }
        launch_jacobi_diag(ddesc(), dwp(kPhJdiag), nblk[kPhJdiag], count, s);
        HIP_TRY(hipGetLastError());
        return RANKY_OK;
    }
};

ranky_status make_engine(ranky_ctx *ctx, hipStream_t s, const Header &h, char *hdr, int count, Engine &e) {
    ranky_status st = ensure_pinned(ctx, h.total);
    if (st) return st;
    e.ctx = ctx;
    e.s = s;
    e.count = count;
    e.h = h;
    e.hdr = hdr;
    e.status.assign(count, RANKY_OK);
    e.gsegs.assign(count, 0);
    return RANKY_OK;
}

size_t path_bytes(const std::vector<Job> &jobs, const ranky_opts &o) {
    const int count = (int)jobs.size();
    const bool refine = count == 1 && wants_refine(o, jobs[0].k);
    int32_t maxM = 1;
    int64_t sum_d = 0;
    size_t total = 0;
    for (const Job &j : jobs) {
        total += make_plan(j.M, j.N, j.A.nnz, j.k, j.D, true, refine, j.bstart, count == 1, o.v_dtype == RANKY_F32)
                     .total;
        maxM = std::max(maxM, j.M);
        sum_d += j.D;
    }
    return total + make_header(count, count, jacobi_npad(maxM) / kJacobiBlock, sum_d).total;
}

// The whole path for a batch (Rayleigh-Ritz refinement only for a batch of one).
ranky_status run_path(ranky_ctx *ctx, const std::vector<Job> &jobs, double tol, const ranky_opts &o, void *workspace,
                      size_t ws_bytes, ranky_info *infos, hipStream_t s, bool use_graph) {
    const int count = (int)jobs.size();
    const bool refine = count == 1 && wants_refine(o, jobs[0].k);
    std::vector<Plan> plans(count);
    std::vector<int32_t> blk_off(count);
    int32_t maxM = 1;
    int64_t sum_d = 0;
    for (int i = 0; i < count; ++i) {
        plans[i] = make_plan(jobs[i].M, jobs[i].N, jobs[i].A.nnz, jobs[i].k, jobs[i].D, true, refine, jobs[i].bstart,
                             count == 1, o.v_dtype == RANKY_F32);
        maxM = std::max(maxM, jobs[i].M);
        blk_off[i] = (int32_t)sum_d;
        sum_d += jobs[i].D;
    }
    const Header h = make_header(count, count, jacobi_npad(maxM) / kJacobiBlock, sum_d);
    size_t need = h.total;
    std::vector<size_t> base(count);
    for (int i = 0; i < count; ++i) {
        base[i] = need;
        need += plans[i].total;
    }
    if (!workspace || ws_bytes < need) return fail(RANKY_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % kWorkspaceAlign)
        return fail(RANKY_E_INVALID, "workspace is not %d-byte aligned", kWorkspaceAlign);
    char *ws = static_cast<char *>(workspace);
    Engine e;
    ranky_status st = make_engine(ctx, s, h, ws, count, e);
    if (st) return st;
    e.sweeps_cap = o.max_sweeps;
    e.d.resize(count);
    Refine rf;
    for (int i = 0; i < count; ++i) {
        const Job &j = jobs[i];
        MatDesc &x = e.d[i];
        x = carve(plans[i], ws + base[i], i == 0 ? &rf : nullptr);
        x.blk_off = blk_off[i];
        if (j.bstart)
            HIP_TRY(hipMemcpyAsync(const_cast<int64_t *>(x.bstart), j.bstart, sizeof(int64_t) * ((size_t)j.D + 1),
                                   hipMemcpyHostToDevice, s));
        x.colptr = j.A.colptr;
        x.rowidx = j.A.rowidx;
        x.values = j.A.values;
        x.dtype = j.A.dtype;
        x.v_dtype = o.v_dtype;
        x.prec = o.gram_prec;
        if (x.prec != RANKY_PREC_BF16X3) x.dwg = 0;   // FP64 / FP32: the sparse pass takes every pair
        x.validate = o.validate;
        x.tol = tol;
        const auto tc = ctx->tuned.find(TuneKey{j.M, j.N, j.A.nnz, j.k, j.A.dtype, o.v_dtype, o.gram_prec});
        if (tc != ctx->tuned.end()) {
            x.bp_per_cu = tc->second.bp_per_cu;
            x.jsched = tc->second.jsched;
        }
        // unit roundoff of the Gram entries as they are computed: FP64, FP32, or the bf16x3
        // products (2^-16) when the split-bf16 tiles run (a single matrix; the selection
        // falls back to 2^-24 when the scan found fewer than two dense rows, since then no tile
        // runs and the whole Gram is the FP32 sparse pass)
        x.u_gram = o.gram_prec == RANKY_PREC_FP64 ? std::ldexp(1.0, -53)
                   : (o.gram_prec == RANKY_PREC_BF16X3 && x.dwg > 0) ? std::ldexp(1.0, -16) : std::ldexp(1.0, -24);
        // an FP32 Gram is accurate to about 6e-8: Jacobi stops at 1e-8 (the FP64 step of the
        // Rayleigh-Ritz refinement, or the mixed-precision bar, covers the rest)
        x.jtol = (o.gram_prec == RANKY_PREC_FP64) ? 0.0 : kJacobiTolFp32Gram;
        x.sigma = j.sigma;
        x.U = refine ? rf.U0 : j.U;
        x.V = j.V;
    }
    const bool timing = o.timing != 0 && count == 1;
    e.time_rounds = timing;
    if (timing) hipEventRecord(ctx->ev[0], s);
    st = e.scan();
    if (st) return st;
    if (count == 1 && e.status[0] != RANKY_OK) {
        if (infos) {
            std::memset(infos, 0, sizeof(ranky_info));
            infos[0].status = e.status[0];
        }
        return e.status[0] == RANKY_E_CSC ? fail(RANKY_E_CSC, "CSC contract violated (colptr, row range or row order)")
                                          : fail(RANKY_E_NONFINITE, "non-finite value in A");
    }
    if (timing) hipEventRecord(ctx->ev[1], s);
    st = e.plan_rest();
    if (st) return st;
    e.enqueue_transpose();
    if (timing) hipEventRecord(ctx->ev[2], s);
    int32_t gram_acc = 4;   // accumulator bytes: FP64 if any matrix of the launch asks for it
    for (int i = 0; i < count; ++i)
        if (e.d[i].prec == RANKY_PREC_FP64) gram_acc = 8;
    if (count == 1) launch_gram_dense(e.ddesc(), e.d[0].dwg, s);
    launch_gram(e.ddesc(), e.dwp(kPhGram), e.nblk[kPhGram], e.dwp(kPhGramRed), e.nblk[kPhGramRed], count, maxM,
                gram_acc, ctx->lds_limit, s);
    if (count == 1) launch_gram_dense_reduce(e.ddesc(), e.d[0].dwg, s);
    HIP_TRY(hipGetLastError());
    if (timing) hipEventRecord(ctx->ev[3], s);
    st = e.eigensolve(use_graph);
    if (st) return st;
    if (timing) hipEventRecord(ctx->ev[4], s);
    launch_select(e.ddesc(), count, e.maxn, s);
    launch_gather_u(e.ddesc(), e.dwp(kPhGather), e.nblk[kPhGather], count, s);
    HIP_TRY(hipGetLastError());
    if (timing) hipEventRecord(ctx->ev[5], s);
    std::vector<int32_t> iv;
    std::vector<double> fv;
    int32_t refine_sweeps = 0, refine_notconv = 0;
    if (refine && e.status[0] == RANKY_OK) {
        // Rayleigh-Ritz with the exact operator: H = U0^T (A A^T) U0 in FP64, eigensolved
        // by the same engine on a descriptor for H, then U = U0 Q, sigma = sqrt(theta).
        const MatDesc x = e.d[0];
        const Job &j = jobs[0];
        const CscView Av{j.A.nnz, j.A.colptr, j.A.rowidx, j.A.values, j.A.dtype};
        const int32_t k = j.k;
        const int32_t kpad = jacobi_npad(k);
        if (x.n > 0) launch_rr_h(Av, j.N, k, rf.U0, rf.part, kpad, x.G, s);
        else launch_fill_f64(x.G, (int64_t)kpad * kpad, 0.0, s);
        HIP_TRY(hipGetLastError());
        // the main matrix's header entries are no longer read: reuse them for H
        Engine eh;
        st = make_engine(ctx, s, h, ws, 1, eh);
        if (st) return st;
        eh.sweeps_cap = o.max_sweeps;
        eh.d.assign(1, x);
        MatDesc &y = eh.d[0];
        y.n = k;
        y.npad = kpad;
        y.n_tau = x.n;
        y.k = k;
        y.u_gram = std::ldexp(1.0, -53);
        y.dwg = 0;      // no split-bf16 tiles in H: its threshold keeps the FP64 roundoff
        y.jtol = 0.0;   // H is exact to FP64 rounding: the full-accuracy stopping test
        y.U = j.U;
        eh.maxn = k;
        st = eh.plan_rest();
        if (st) return st;
        st = eh.eigensolve(false);
        if (st) return st;
        refine_sweeps = eh.sweeps[0];
        refine_notconv = eh.notconv[0];
        launch_select(eh.ddesc(), 1, k, s);
        launch_rr_apply(rf.U0, y.W, kpad, y.perm, j.M, k, j.U, x.Uf, s);
        launch_backproject(Av, j.N, k, j.U, x.Uf, j.sigma, y.scal + kScRank, j.V, o.v_dtype, ctx->cu_count, s);
        HIP_TRY(hipGetLastError());
        e.d[0].U = j.U;
        st = e.upload_desc();
        if (st) return st;
    }
    if (timing) hipEventRecord(ctx->ev[6], s);
    if (!refine) {
        const int32_t widths[3] = {1, 2, 4};
        for (int c = 0; c < 3; ++c)
            launch_backproject_batch(e.ddesc(), e.dwp(kPhBack + c), e.nblk[kPhBack + c], count, widths[c], s);
    }
    HIP_TRY(hipGetLastError());
    if (timing) hipEventRecord(ctx->ev[7], s);
    st = e.collect(iv, fv, &ctx->blk_host);
    if (st) return st;
    ranky_status overall = RANKY_OK;
    for (int i = 0; i < count; ++i) {
        ranky_status si = static_cast<ranky_status>(e.status[i]);
        if (si == RANKY_OK && (e.notconv[i] != 0 || refine_notconv != 0)) si = RANKY_E_NOT_CONVERGED;
        if (si != RANKY_OK && overall == RANKY_OK) overall = si;
        if (infos) {
            ranky_info &in = infos[i];
            std::memset(&in, 0, sizeof(in));
            in.status = si;
            in.rank = iv[kColI * i + 2];
            in.n_nonempty = e.d[i].n;
            in.empty_rows = jobs[i].M - e.d[i].n;
            in.sweeps = e.sweeps[i];
            in.rr_sweeps = refine_sweeps;
            in.n_blocks = jobs[i].D;
            in.lonely_max = iv[kColI * i + 5];
            in.lonely_blocks = iv[kColI * i + 6];
            if (e.status[i] == RANKY_OK) {
                in.lonely_per_block = ctx->blk_host.data() + 2 * (size_t)blk_off[i];
                in.single_per_block = in.lonely_per_block + jobs[i].D;
            }
            in.tau = fv[2 * i];
            in.sigma_max = fv[2 * i + 1];
            if (timing) {
                float t = 0.f;
                for (int q = 0; q < 7; ++q) {
                    hipEventElapsedTime(&t, ctx->ev[q], ctx->ev[q + 1]);
                    in.ms[q] = t;
                }
                hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[7]);
                in.ms[7] = t;
                in.round_ms = (float)e.round_ms;
                in.round_launches = e.round_launches;
            }
        }
    }
    if (overall == RANKY_E_CSC) return fail(RANKY_E_CSC, "CSC contract violated (colptr, row range or row order)");
    if (overall == RANKY_E_NONFINITE) return fail(RANKY_E_NONFINITE, "non-finite value in A");
    if (overall == RANKY_E_NOT_CONVERGED)
        return fail(RANKY_E_NOT_CONVERGED, "Jacobi did not converge in %d sweeps", o.max_sweeps);
    return overall;
}

ranky_status check_block_start(const int64_t *bstart, int32_t D, int64_t N) {
    if (!bstart) return RANKY_OK;
    if (D < 1) return fail(RANKY_E_INVALID, "block_start needs n_blocks >= 1");
    if (bstart[0] != 0 || bstart[D] != N)
        return fail(RANKY_E_INVALID, "block_start must run from 0 to N=%lld", (long long)N);
    for (int32_t b = 0; b < D; ++b)
        if (bstart[b + 1] < bstart[b]) return fail(RANKY_E_INVALID, "block_start decreases at block %d", b);
    return RANKY_OK;
}

ranky_status make_job(const ranky_csc *A, int32_t M, int64_t N, int32_t k, int32_t D, double *sigma, double *U,
                      void *V, Job *out, const int64_t *bstart = nullptr) {
    ranky_status st = check_csc_args(A, M, N);
    if (st) return st;
    if (k < 1 || k > M) return fail(RANKY_E_INVALID, "k=%d must be in [1, M=%d]", k, M);
    if (bstart && D < 1) return fail(RANKY_E_INVALID, "block_start needs n_blocks >= 1");
    if (D == 0) D = default_blocks(N);
    if (D < 1 || D > N) return fail(RANKY_E_INVALID, "n_blocks=%d outside [1, N]", D);
    st = check_block_start(bstart, D, N);
    if (st) return st;
    out->bstart = bstart;
    out->A = *A;
    out->N = N;
    out->M = M;
    out->k = k;
    out->D = D;
    out->sigma = sigma;
    out->U = U;
    out->V = V;
    return RANKY_OK;
}

// Context-free pieces for the step calls.
struct StepCtx {
    ranky_ctx c;
    ~StepCtx() {
        if (c.pinned) hipHostFree(c.pinned);
    }
};

ranky_status step_device(StepCtx &sc) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    size_t lds = prop.sharedMemPerBlock;
    if (lds > 160 * 1024) lds = 160 * 1024;
    sc.c.lds_limit = lds > 4096 ? lds - 4096 : lds;
    sc.c.cu_count = prop.multiProcessorCount;
    sc.c.device = dev;
    HIP_TRY(kernel_attributes(dev, sc.c.lds_limit));
    return RANKY_OK;
}

ranky_status step_scan(StepCtx &sc, const ranky_csc *A, int32_t M, int64_t N, int32_t D, void *workspace,
                       size_t ws_bytes, hipStream_t s, Engine &e, int32_t *cnt, int32_t *rownnz, int32_t *lonely,
                       int32_t *single) {
    const Plan p = make_plan(M, N, A->nnz, 1, D, false, false, nullptr, true);
    const Header h = make_header(1, 1, 1);
    if (!workspace || ws_bytes < h.total + p.total)
        return fail(RANKY_E_NOMEM, "workspace %zu < %zu", ws_bytes, h.total + p.total);
    if (reinterpret_cast<uintptr_t>(workspace) % kWorkspaceAlign)
        return fail(RANKY_E_INVALID, "workspace is not %d-byte aligned", kWorkspaceAlign);
    ranky_status st = step_device(sc);
    if (st) return st;
    char *ws = static_cast<char *>(workspace);
    st = make_engine(&sc.c, s, h, ws, 1, e);
    if (st) return st;
    e.d.assign(1, carve(p, ws + h.total, nullptr));
    MatDesc &x = e.d[0];
    x.colptr = A->colptr;
    x.rowidx = A->rowidx;
    x.values = A->values;
    x.dtype = A->dtype;
    x.validate = 1;
    if (cnt) x.cnt = cnt;
    if (rownnz) x.rownnz = rownnz;
    if (lonely) x.lonely = lonely;
    if (single) x.single = single;
    st = e.scan();
    if (st) return st;
    if (e.status[0] == RANKY_E_CSC) return fail(RANKY_E_CSC, "CSC contract violated (colptr, row range or row order)");
    if (e.status[0] == RANKY_E_NONFINITE) return fail(RANKY_E_NONFINITE, "non-finite value in A");
    return RANKY_OK;
}

}  // namespace

extern "C" {

const char *ranky_last_error(void) { return g_err; }
const char *ranky_version(void) { return "ranky-mi355x 0.2 (gfx950)"; }

ranky_status ranky_default_opts(ranky_opts *o) {
    if (!o) return fail(RANKY_E_INVALID, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->n_blocks = 0;
    o->gram_prec = RANKY_PREC_FP64;
    o->refine = -1;
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
    for (auto &ev : c->ev) {
        const hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            ranky_ctx_destroy(c);
            return fail(RANKY_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    const hipError_t e = kernel_attributes(device, c->lds_limit);
    if (e != hipSuccess) {
        ranky_ctx_destroy(c);
        return fail(RANKY_E_DEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(e));
    }
    *out = c;
    return RANKY_OK;
}

ranky_status ranky_ctx_destroy(ranky_ctx *ctx) {
    if (!ctx) return RANKY_OK;
    if (ctx->worker.joinable()) ctx->worker.join();   // an async call still running finishes first
    for (auto &ev : ctx->ev)
        if (ev) hipEventDestroy(ev);
    if (ctx->sweep_graph) hipGraphExecDestroy(ctx->sweep_graph);
    if (ctx->pinned) hipHostFree(ctx->pinned);
    delete ctx;
    return RANKY_OK;
}

size_t ranky_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t k, const ranky_opts *opts) {
    if (M < 1 || N < 1 || k < 1 || k > M || M > kMaxM || nnz < 0) return 0;
    const ranky_opts o = resolved(opts, true, k);
    if (o.block_start && o.n_blocks < 1) return 0;
    const int32_t D = o.n_blocks == 0 ? default_blocks(N) : o.n_blocks;
    if (D < 1 || D > N) return 0;
    Job j;
    std::memset(&j, 0, sizeof(j));
    j.bstart = o.block_start;
    j.A.nnz = nnz;
    j.M = M;
    j.N = N;
    j.k = k;
    j.D = D;
    return path_bytes({j}, o);
}

ranky_status ranky_svd(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, double tol,
                       const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, double *U, void *V,
                       ranky_info *info, ranky_stream_t stream) {
    ranky_info local;
    ranky_info *inf = info ? info : &local;
    std::memset(inf, 0, sizeof(*inf));
    auto finish = [&](ranky_status st) {
        if (inf->status == RANKY_OK) inf->status = st;
        return st;
    };
    if (!ctx) return finish(fail(RANKY_E_INVALID, "ctx is NULL"));
    if (!(tol >= 0.0)) return finish(fail(RANKY_E_INVALID, "tol must be >= 0"));
    if (!sigma || !U || !V) return finish(fail(RANKY_E_INVALID, "NULL output"));
    const ranky_opts o = resolved(opts, true, k);
    ranky_status st = check_opts(o);
    if (st) return finish(st);
    Job j;
    st = make_job(A, M, N, k, o.n_blocks, sigma, U, V, &j, o.block_start);
    if (st) return finish(st);
    if (o.refine && k > kMaxRefineK) return finish(fail(RANKY_E_INVALID, "refine needs k <= %d", kMaxRefineK));
    if (hipSetDevice(ctx->device) != hipSuccess) return finish(fail(RANKY_E_DEVICE, "hipSetDevice"));
    return finish(run_path(ctx, {j}, tol, o, workspace, ws_bytes, inf, reinterpret_cast<hipStream_t>(stream),
                           o.graph == 1));
}

ranky_status ranky_svd_async(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, double tol,
                             const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, double *U,
                             void *V, ranky_stream_t stream, uint64_t *ticket) {
    if (!ctx || !ticket) return fail(RANKY_E_INVALID, "ctx or ticket is NULL");
    // the host-checkable errors of ranky_svd, at once
    if (!(tol >= 0.0)) return fail(RANKY_E_INVALID, "tol must be >= 0");
    if (!sigma || !U || !V) return fail(RANKY_E_INVALID, "NULL output");
    const ranky_opts o = resolved(opts, true, k);
    ranky_status st = check_opts(o);
    if (st) return st;
    Job j;
    st = make_job(A, M, N, k, o.n_blocks, sigma, U, V, &j, o.block_start);
    if (st) return st;
    if (o.refine && k > kMaxRefineK) return fail(RANKY_E_INVALID, "refine needs k <= %d", kMaxRefineK);
    std::lock_guard<std::mutex> lk(ctx->amu);
    if (ctx->astate != 0) return fail(RANKY_E_BUSY, "an asynchronous call is in flight on this context");
    if (ctx->worker.joinable()) ctx->worker.join();
    const ranky_csc a = *A;
    const uint64_t t = ++ctx->aticket;
    ctx->astate = 1;
    ctx->worker = std::thread([ctx, a, M, N, k, tol, o, workspace, ws_bytes, sigma, U, V, stream]() {
        ranky_info inf;
        const ranky_status rs = ranky_svd(ctx, &a, M, N, k, tol, &o, workspace, ws_bytes, sigma, U, V, &inf, stream);
        std::lock_guard<std::mutex> g(ctx->amu);
        ctx->aresult = rs;
        ctx->ainfo = inf;
        ctx->aerr = rs ? ranky_last_error() : "";
        ctx->astate = 2;
    });
    *ticket = t;
    return RANKY_OK;
}

ranky_status ranky_query(ranky_ctx *ctx, uint64_t ticket, ranky_info *info) {
    if (!ctx) return fail(RANKY_E_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->amu);
    if (ticket == 0 || ticket != ctx->aticket || ctx->astate == 0)
        return fail(RANKY_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    if (ctx->astate == 1) return RANKY_PENDING;
    ctx->worker.join();   // finished: the worker only returns after setting astate
    ctx->astate = 0;
    if (info) *info = ctx->ainfo;
    if (ctx->aresult) return fail(ctx->aresult, "%s", ctx->aerr.c_str());
    return RANKY_OK;
}

ranky_status ranky_tune_set(ranky_ctx *ctx, int32_t M, int64_t N, int64_t nnz, int32_t k, ranky_dtype dtype,
                            const ranky_opts *opts, int32_t bp_per_cu, int32_t jacobi_schedule) {
    if (!ctx) return fail(RANKY_E_INVALID, "ctx is NULL");
    const ranky_opts o = resolved(opts, true, k);
    const ranky_status st = check_opts(o);
    if (st) return st;
    if (bp_per_cu < 1 || bp_per_cu > 1024) return fail(RANKY_E_INVALID, "bp_per_cu=%d", bp_per_cu);
    if (jacobi_schedule < 0 || jacobi_schedule > 3) return fail(RANKY_E_INVALID, "jacobi_schedule=%d", jacobi_schedule);
    TuneCfg c;
    c.bp_per_cu = bp_per_cu;
    c.jsched = jacobi_schedule;
    ctx->tuned[TuneKey{M, N, nnz, k, dtype, o.v_dtype, o.gram_prec}] = c;
    return RANKY_OK;
}

ranky_status ranky_autotune(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k,
                            const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, double *U, void *V,
                            ranky_tune_report *report, ranky_stream_t stream) {
    if (!ctx) return fail(RANKY_E_INVALID, "ctx is NULL");
    if (!sigma || !U || !V) return fail(RANKY_E_INVALID, "NULL output");
    ranky_opts o = resolved(opts, true, k);
    ranky_status st = check_opts(o);
    if (st) return st;
    Job j;
    st = make_job(A, M, N, k, o.n_blocks, sigma, U, V, &j, o.block_start);
    if (st) return st;
    if (o.refine && k > kMaxRefineK) return fail(RANKY_E_INVALID, "refine needs k <= %d", kMaxRefineK);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RANKY_E_DEVICE, "hipSetDevice");
    o.timing = 1;      // phase times from HIP events
    o.graph = 0;       // direct launches while timing
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const TuneKey key{M, N, j.A.nnz, k, j.A.dtype, o.v_dtype, o.gram_prec};
    const int32_t bp_cands[4] = {8, 16, 32, 64};
    const int32_t sched_cands[4] = {0, 1, 2, 3};
    const int reps = 2;
    TuneCfg best;
    ranky_info in;
    // phase ms of the best of `reps` runs with configuration c: [6] back-projection, [3] eigensolve
    auto measure = [&](const TuneCfg &c, int phase, float &ms) -> ranky_status {
        ctx->tuned[key] = c;
        ms = 1e30f;
        for (int r = 0; r < reps; ++r) {
            std::memset(&in, 0, sizeof(in));
            const ranky_status rs = run_path(ctx, {j}, 0.0, o, workspace, ws_bytes, &in, s, false);
            if (rs) return rs;
            ms = std::min(ms, in.ms[phase]);
        }
        return RANKY_OK;
    };
    float bp_ms[4] = {0, 0, 0, 0}, eig_ms[4] = {0, 0, 0, 0}, t = 0.f;
    st = measure(best, 3, t);   // warm-up (kernel loading, caches)
    const bool has_bp = !wants_refine(o, k);   // with refinement V comes from the Rayleigh-Ritz step
    if (!st && has_bp) {
        float bmin = 1e30f;
        for (int c = 0; c < 4 && !st; ++c) {
            TuneCfg cfg = best;
            cfg.bp_per_cu = bp_cands[c];
            st = measure(cfg, 6, bp_ms[c]);
            if (!st && bp_ms[c] < bmin) {
                bmin = bp_ms[c];
                best.bp_per_cu = bp_cands[c];
            }
        }
    }
    if (!st) {
        float emin = 1e30f;
        for (int c = 0; c < 4 && !st; ++c) {
            TuneCfg cfg = best;
            cfg.jsched = sched_cands[c];
            st = measure(cfg, 3, eig_ms[c]);
            if (!st && eig_ms[c] < emin) {
                emin = eig_ms[c];
                best.jsched = sched_cands[c];
            }
        }
    }
    if (st) {
        ctx->tuned.erase(key);
        return st;
    }
    ctx->tuned[key] = best;
    if (report) {
        std::memset(report, 0, sizeof(*report));
        report->bp_per_cu = has_bp ? best.bp_per_cu : 0;
        report->jacobi_schedule = best.jsched;
        for (int c = 0; c < 4; ++c) {
            report->bp_candidates[c] = bp_cands[c];
            report->bp_ms[c] = has_bp ? bp_ms[c] : 0.f;
        }
        for (int c = 0; c < 4; ++c) {
            report->schedule_candidates[c] = sched_cands[c];
            report->eig_ms[c] = eig_ms[c];
        }
    }
    return RANKY_OK;
}

size_t ranky_batch_workspace_bytes(int32_t count, const ranky_batch_item *items, const ranky_opts *opts) {
    if (count < 1 || !items) return 0;
    ranky_opts o = resolved(opts, false);
    if (o.refine != 0) return 0;
    if (o.block_start) return 0;
    std::vector<Job> jobs(count);
    for (int i = 0; i < count; ++i) {
        const ranky_batch_item &it = items[i];
        if (it.M < 1 || it.N < 1 || it.k < 1 || it.k > it.M || it.M > kMaxM || it.A.nnz < 0) return 0;
        const int32_t D = it.n_blocks == 0 ? default_blocks(it.N) : it.n_blocks;
        if (D < 1 || D > it.N) return 0;
        std::memset(&jobs[i], 0, sizeof(Job));
        jobs[i].A.nnz = it.A.nnz;
        jobs[i].M = it.M;
        jobs[i].N = it.N;
        jobs[i].k = it.k;
        jobs[i].D = D;
    }
    return path_bytes(jobs, o);
}

ranky_status ranky_batch(ranky_ctx *ctx, int32_t count, const ranky_batch_item *items, double tol,
                         const ranky_opts *opts, void *workspace, size_t ws_bytes, ranky_info *infos,
                         ranky_stream_t stream) {
    if (!ctx) return fail(RANKY_E_INVALID, "ctx is NULL");
    if (count < 1 || !items) return fail(RANKY_E_INVALID, "empty batch");
    if (!(tol >= 0.0)) return fail(RANKY_E_INVALID, "tol must be >= 0");
    const ranky_opts o = resolved(opts, false);
    ranky_status st = check_opts(o);
    if (st) return st;
    if (o.refine) return fail(RANKY_E_INVALID, "ranky_batch runs without refinement (use ranky_svd per matrix)");
    if (o.block_start) return fail(RANKY_E_INVALID, "block_start is for one matrix (ranky_svd)");
    std::vector<Job> jobs(count);
    for (int i = 0; i < count; ++i) {
        const ranky_batch_item &it = items[i];
        if (!it.sigma || !it.U || !it.V) return fail(RANKY_E_INVALID, "item %d: NULL output", i);
        st = make_job(&it.A, it.M, it.N, it.k, it.n_blocks, it.sigma, it.U, it.V, &jobs[i]);
        if (st) return st;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RANKY_E_DEVICE, "hipSetDevice");
    return run_path(ctx, jobs, tol, o, workspace, ws_bytes, infos, reinterpret_cast<hipStream_t>(stream),
                    o.graph == 1);
}

// ---------------------------------------------------------------------------
// step calls
// ---------------------------------------------------------------------------

size_t ranky_step_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t D) {
    if (M < 1 || N < 1 || M > kMaxM || nnz < 0 || D < 1 || D > N) return 0;
    return make_header(1, 1, 1).total + make_plan(M, N, nnz, 1, D, false, false, nullptr, true).total;
}

ranky_status ranky_occupancy(const ranky_csc *A, int32_t M, int64_t N, int32_t D, int32_t *cnt, int32_t *rownnz,
                             int32_t *lonely, int32_t *single, void *workspace, size_t ws_bytes,
                             ranky_stream_t stream) {
    ranky_status st = check_csc_args(A, M, N);
    if (st) return st;
    if (D < 1 || D > N) return fail(RANKY_E_INVALID, "D=%d outside [1, N]", D);
    if (!cnt || !rownnz || !lonely || !single) return fail(RANKY_E_INVALID, "NULL output");
    StepCtx sc;
    Engine e;
    return step_scan(sc, A, M, N, D, workspace, ws_bytes, reinterpret_cast<hipStream_t>(stream), e, cnt, rownnz,
                     lonely, single);
}

ranky_status ranky_gram(const ranky_csc *A, int32_t M, int64_t N, int32_t prec, double *G, void *workspace,
                        size_t ws_bytes, ranky_stream_t stream) {
    ranky_status st = check_csc_args(A, M, N);
    if (st) return st;
    if (!G) return fail(RANKY_E_INVALID, "G is NULL");
    if (prec != RANKY_PREC_FP64 && prec != RANKY_PREC_FP32 && prec != RANKY_PREC_BF16X3)
        return fail(RANKY_E_INVALID, "prec=%d", prec);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    StepCtx sc;
    Engine e;
    st = step_scan(sc, A, M, N, default_blocks(N), workspace, ws_bytes, s, e, nullptr, nullptr, nullptr, nullptr);
    if (st) return st;
    MatDesc &x = e.d[0];
    x.prec = prec;
    if (x.prec != RANKY_PREC_BF16X3) x.dwg = 0;
    if (x.n > 0) {
        e.nblk[kPhGram] = fill_wp(e.hwp(kPhGram), 1, [&](int) { return (int64_t)e.gsegs[0] + (x.npad - x.n); });
        e.nblk[kPhGramRed] = fill_wp(e.hwp(kPhGramRed), 1, [&](int) { return (int64_t)x.n; });
        st = e.upload_desc();
        if (!st) st = e.upload(e.h.o_wp, sizeof(int32_t) * (size_t)kPhCount * (e.h.slots + 1));
        if (st) return st;
        e.enqueue_transpose();
        launch_gram_dense(e.ddesc(), x.dwg, s);
        launch_gram(e.ddesc(), e.dwp(kPhGram), e.nblk[kPhGram], e.dwp(kPhGramRed), e.nblk[kPhGramRed], 1, M,
                    prec == RANKY_PREC_FP64 ? 8 : 4, sc.c.lds_limit, s);
        launch_gram_dense_reduce(e.ddesc(), x.dwg, s);
        launch_scatter_gram(x.G, x.npad, x.m2r, M, G, s);
    } else {
        launch_fill_f64(G, (int64_t)M * M, 0.0, s);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return RANKY_OK;
}

size_t ranky_eigh_workspace_bytes(int32_t n) {
    if (n < 1 || n > kMaxM) return 0;
    const int32_t npad = jacobi_npad(n);
    const size_t npairs = (size_t)(npad / kJacobiPair);
    size_t b = make_header(1, 1, npad / kJacobiBlock).total;
    b += align_up(sizeof(int32_t) * kScCount) + align_up(sizeof(double) * kSdCount) +
         align_up(sizeof(int32_t) * kJsCount);
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
    if (reinterpret_cast<uintptr_t>(workspace) % kWorkspaceAlign)
        return fail(RANKY_E_INVALID, "workspace is not %d-byte aligned", kWorkspaceAlign);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int32_t npad = jacobi_npad(n);
    const size_t npairs = (size_t)(npad / kJacobiPair);
    const Header h = make_header(1, 1, npad / kJacobiBlock);
    char *b = static_cast<char *>(workspace);
    size_t off = h.total;
    auto take = [&](size_t bytes) {
        char *ptr = b + off;
        off += align_up(bytes);
        return ptr;
    };
    MatDesc x;
    std::memset(&x, 0, sizeof(x));
    x.scal = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * kScCount));
    x.sdbl = reinterpret_cast<double *>(take(sizeof(double) * kSdCount));
    x.jstate = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * kJsCount));
    x.G = reinterpret_cast<double *>(take(sizeof(double) * (size_t)npad * npad));
    x.G2 = reinterpret_cast<double *>(take(sizeof(double) * (size_t)npad * npad));
    x.W = reinterpret_cast<double *>(take(sizeof(double) * (size_t)npad * npad));
    x.J = reinterpret_cast<double *>(take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair));
    x.S = reinterpret_cast<double *>(take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair));
    x.jflag = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * 2 * npairs));
    x.lam = reinterpret_cast<double *>(take(sizeof(double) * npad));
    x.M = n;
    x.k = n;
    x.D = 0;  // no column blocks: no per-block counters to read back
    x.n = n;
    x.n_tau = n;
    x.npad = npad;
    StepCtx sc;
    ranky_status st = step_device(sc);
    if (st) return st;
    Engine e;
    st = make_engine(&sc.c, s, h, b, 1, e);
    if (st) return st;
    e.d.assign(1, x);
    e.sweeps_cap = max_sweeps > 0 ? max_sweeps : kDefaultSweeps;
    launch_fill_i32(x.scal, kScCount, 0, s);
    launch_pad_copy(G, n, x.G, npad, npad, s);
    st = e.plan_rest();
    if (st) return st;
    st = e.eigensolve(false);
    if (st) return st;
    if (sweeps) *sweeps = e.sweeps[0];
    HIP_TRY(hipMemcpyAsync(lambda, x.lam, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    launch_unpad_copy(x.W, npad, n, Q, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    if (e.notconv[0] != 0) return fail(RANKY_E_NOT_CONVERGED, "Jacobi did not converge in %d sweeps", e.sweeps_cap);
    return RANKY_OK;
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
    const CscView Av{A->nnz, A->colptr, A->rowidx, A->values, A->dtype};
    launch_backproject(Av, N, k, U, nullptr, sigma, rank, V, v_dtype, cus, reinterpret_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return RANKY_OK;
}

}  // extern "C"

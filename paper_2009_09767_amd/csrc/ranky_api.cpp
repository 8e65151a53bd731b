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
#include "internal.hpp"
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
    bool no_alloc = false;   // set during ranky_svd_noalloc: the staging must not grow
};

namespace {

using namespace ranky;

thread_local char g_err[512] = "";
constexpr int32_t kDefaultSweeps = 40;
constexpr size_t kStagingBytes = 1 << 20;   // host staging allocated with a context
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
    if (e == hipSuccess) e = paper_set_attributes(lds_limit);
    if (e == hipSuccess) g_attr_devices.push_back(device);
    return e;
}

// ---------------------------------------------------------------------------
// subspace iteration for the k leading eigenpairs (k << M')
// ---------------------------------------------------------------------------

constexpr int32_t kTopkMaxBlock = 256;    // widest block (the p x p problems run on the Jacobi)
constexpr int32_t kTopkWgTarget = 768;    // workgroups a split product aims for (three per CU)
constexpr int32_t kTopkWideTarget = 512;  // the same for the whole-width G Y products (two per CU: LDS)
constexpr int32_t kTopkWideMaxP = 192;    // block widths the whole-width product takes
constexpr int32_t kTopkWideMinK = 1024;   // and inner sizes (shorter ones stay on the 64 x 64 tiles)
constexpr int32_t kTopkDefaultIters = 60;
constexpr int64_t kHeavyMinNnz = (int64_t)1 << 22;   // automatic heavy-row split of the Gram from here

// Block width for k wanted pairs: k plus half again (at least 32) of oversampling, in 64s.
int32_t topk_block(int32_t k) {
    const int32_t want = k + std::max(k / 2, 32);
    return ((want + kTopkTile - 1) / kTopkTile) * kTopkTile;
}

// k split of a product with `tiles` output tiles over K: (splits, klen), klen a multiple of 16.
void topk_split(int64_t tiles, int32_t K, int32_t &splits, int32_t &klen, int64_t target = kTopkWgTarget) {
    int64_t sp = (target + tiles - 1) / tiles;
    if (sp > K / 64) sp = K / 64;
    if (sp < 1) sp = 1;
    klen = (int32_t)((((K + sp - 1) / sp) + 15) / 16 * 16);
    splits = (K + klen - 1) / klen;
}

struct TopkLayout {
    int32_t p = 0, rows = 0;   // block width; block rows (the eigensolver order rounded up to 64)
    size_t o_blk[5] = {}, o_part = 0, o_Sp = 0, o_Wm = 0, o_Qs = 0, o_theta = 0, o_dvec = 0, o_sig = 0;
    size_t o_hdr = 0, o_jscal = 0, o_jsdbl = 0, o_jstate = 0, o_jG = 0, o_jG2 = 0, o_jW = 0, o_jJ = 0, o_jS = 0;
    size_t o_jflag = 0, o_jlam = 0, o_jperm = 0, part_doubles = 0, hdr_bytes = 0, total = 0;
};

size_t topk_small_header_bytes(int32_t p);

// Region of the subspace iteration for an M-row matrix and block width p, at offset 0.
TopkLayout topk_layout(int32_t M, int32_t p) {
    TopkLayout t;
    t.p = p;
    const int32_t npad = jacobi_npad(M);
    t.rows = ((npad + kTopkTile - 1) / kTopkTile) * kTopkTile;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t blk = sizeof(double) * (size_t)t.rows * p, sq = sizeof(double) * (size_t)p * p;
    for (size_t &o : t.o_blk) o = take(blk);
    int32_t sp1, kl1, sp2, kl2;
    topk_split((int64_t)(t.rows / kTopkTile) * (p / kTopkTile), npad, sp1, kl1);     // G Y
    topk_split((int64_t)(p / kTopkTile) * (p / kTopkTile), t.rows, sp2, kl2);        // Y^T Y, Y^T T
    int32_t sp3, kl3;
    topk_split((int64_t)(t.rows / kTopkTile) * (p / kTopkTile), p, sp3, kl3);        // Y W
    int32_t sp4, kl4;
    topk_split(t.rows / kTopkTile, npad, sp4, kl4, kTopkWideTarget);                // G Y, whole width
    t.part_doubles = std::max({(size_t)sp1 * t.rows * p, (size_t)sp2 * p * p, (size_t)sp3 * t.rows * p,
                               (size_t)sp4 * t.rows * p});
    t.o_part = take(sizeof(double) * t.part_doubles);
    t.o_Sp = take(sq);
    t.o_Wm = take(sq);
    t.o_Qs = take(sq);
    t.o_theta = take(sizeof(double) * p);
    t.o_dvec = take(sizeof(double) * p);
    t.o_sig = take(sizeof(double) * p);
    t.hdr_bytes = topk_small_header_bytes(p);
    t.o_hdr = take(t.hdr_bytes);
    const size_t npairs = (size_t)(p / kJacobiPair);
    t.o_jscal = take(sizeof(int32_t) * kScCount);
    t.o_jsdbl = take(sizeof(double) * kSdCount);
    t.o_jstate = take(sizeof(int32_t) * kJsCount);
    t.o_jG = take(sq);
    t.o_jG2 = take(sq);
    t.o_jW = take(sq);
    t.o_jJ = take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair);
    t.o_jS = take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair);
    t.o_jflag = take(sizeof(int32_t) * 2 * npairs);
    t.o_jlam = take(sizeof(double) * p);
    t.o_jperm = take(sizeof(int32_t) * p);
    t.total = off;
    return t;
}

// ---------------------------------------------------------------------------
// per-matrix workspace plan
// ---------------------------------------------------------------------------

struct Plan {
    int32_t M = 0, k = 0, D = 0, cpb = 0, ccols = 0, npad = 0;
    int64_t N = 0, nnz = 0, nchunks = 0;
    size_t o_scal = 0, o_sdbl = 0, o_jstate = 0, o_hist = 0, o_rownnz = 0, o_rowptr = 0, o_m2r = 0, o_r2m = 0;
    size_t o_empty = 0, o_lonely = 0, o_single = 0, o_csrk = 0, o_csrcol = 0;
    size_t o_gsegp = 0, o_gslot = 0, o_gpart = 0, o_dense = 0, o_dpart = 0;
    int32_t dwg = 0;
    size_t o_G = 0, o_G2 = 0, o_W = 0, o_J = 0, o_S = 0, o_jflag = 0, o_lam = 0, o_perm = 0;
    size_t o_U0 = 0, o_part = 0, o_uf = 0, total = 0;
    size_t o_bstart = 0;
    bool solver = false, refine = false, explicit_blocks = false, uf = false;
    size_t o_topk = 0;     // the subspace iteration's region (topk.p > 0)
    TopkLayout topk;
    int32_t hwg = 0;       // heavy-row split of the Gram: tile workgroups (0: off)
    size_t o_aht = 0, o_hpart = 0, o_lcnt = 0, o_lptr = 0, o_lbtot = 0, o_lrow = 0, o_lval = 0;
};

// bstart (host, may be NULL): the caller's D + 1 block boundaries; the widest block sets
// the chunks per block, and the boundaries get a device copy in the workspace.
// dense: room for the split-bf16 dense tiles (a single matrix; used with gram_prec BF16X3).
// uf: room for an FP32 copy of U (solver plans with an FP32 V: the back-projection gathers it).
// topk_p: block width of the subspace iteration (0: the full Jacobi only).
// heavy: room for the heavy-row split of the Gram (needs dense): the dense rows' values per
// column (N x kDenseRows, 8-byte slots) and one partial tile per tile workgroup.
Plan make_plan(int32_t M, int64_t N, int64_t nnz, int32_t k, int32_t D, bool solver, bool refine,
               const int64_t *bstart = nullptr, bool dense = false, bool uf = false, int32_t topk_p = 0,
               bool heavy = false) {
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
    p.o_csrk = take(2 * sizeof(int32_t) * nz);
    p.o_csrcol = take(sizeof(int32_t) * nz);
    p.o_gsegp = take(sizeof(int32_t) * (M + 1));
    p.o_gslot = take(sizeof(int32_t) * (M + 1));
    p.o_gpart = take(sizeof(double) * (size_t)gram_part_slots(nnz) * p.npad);
    p.o_dense = take(sizeof(int32_t) * kDenseRows);
    p.dwg = dense ? gram_dense_wgs(N) : 0;
    p.o_dpart = take(sizeof(double) * kDenseRows * kDenseRows * (size_t)p.dwg);
    if (dense && heavy) {
        p.hwg = gram_heavy_wgs(N);
        p.o_aht = take(sizeof(double) * kDenseRows * (size_t)N);
        p.o_hpart = take(sizeof(double) * kDenseRows * kDenseRows * (size_t)p.hwg);
        p.o_lcnt = take(sizeof(int32_t) * (size_t)N);
        p.o_lptr = take(sizeof(int32_t) * ((size_t)N + 1));
        p.o_lbtot = take(sizeof(int32_t) * (size_t)tall_scan_blocks(N));
        p.o_lrow = take(sizeof(int32_t) * nz);
        p.o_lval = take(sizeof(LightRec<double>) * nz);
    }
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
        if (topk_p > 0) {
            p.topk = topk_layout(M, topk_p);
            p.o_topk = take(p.topk.total);
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
    d.csrcol = i32(p.o_csrcol);
    d.gsegp = i32(p.o_gsegp);
    d.gslot = i32(p.o_gslot);
    d.gpart = f64(p.o_gpart);
    d.dense = i32(p.o_dense);
    d.dwg = p.dwg;
    d.dpart = f64(p.o_dpart);
    d.hwg = p.hwg;
    d.aht = p.hwg > 0 ? static_cast<void *>(base + p.o_aht) : nullptr;
    d.hpart = p.hwg > 0 ? f64(p.o_hpart) : nullptr;
    d.lcnt = p.hwg > 0 ? i32(p.o_lcnt) : nullptr;
    d.lptr = p.hwg > 0 ? i32(p.o_lptr) : nullptr;
    d.lbtot = p.hwg > 0 ? i32(p.o_lbtot) : nullptr;
    d.lrowidx = p.hwg > 0 ? i32(p.o_lrow) : nullptr;
    d.lvals = p.hwg > 0 ? static_cast<void *>(base + p.o_lval) : nullptr;
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
    if (o.eigensolver < 0 || o.eigensolver > 2) return fail(RANKY_E_INVALID, "eigensolver=%d (0, 1 or 2)", o.eigensolver);
    if (o.max_iters < 0) return fail(RANKY_E_INVALID, "max_iters=%d", o.max_iters);
    if (o.gram_split < 0 || o.gram_split > 2) return fail(RANKY_E_INVALID, "gram_split=%d", o.gram_split);
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
    if (ctx->no_alloc)
        return fail(RANKY_E_NOMEM, "the context's staging holds %zu bytes, %zu needed (no allocation in this call)",
                    ctx->pinned_bytes, bytes);
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

// Launch shape of the Gram walk over a batch: as many waves as the matrix with the most, and
// the LDS of the hungriest matrix (each matrix's workgroups use its own count and layout).
void gram_shape(const std::vector<MatDesc> &d, size_t lds_limit, int32_t &max_waves, size_t &lds_bytes) {
    max_waves = 1;
    lds_bytes = 0;
    for (const MatDesc &x : d) {
        const int32_t acc = x.prec == RANKY_PREC_FP64 ? 8 : 4;
        max_waves = std::max(max_waves, x.gwaves);
        lds_bytes = std::max(lds_bytes, gram_lds_bytes(x.M, acc, x.gwaves, x.hwg == 0));   // <= lds_limit by gram_waves
    }
    (void)lds_limit;
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

    // this engine's part of the context's pinned staging: an engine made while another one's
    // uploads may still be pending (the subspace iteration's p x p Jacobi) stages past it
    size_t stage_off = 0;
    char *stage() { return static_cast<char *>(ctx->pinned) + stage_off; }
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
            d[i].neig = d[i].n;
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
        for (int i = 0; i < count; ++i)
            if (d[i].V == nullptr) bpb[i] = 0;   // a member whose right vectors are not wanted
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

    // light: the heavy-row split's light CSC is built (the Gram walk then steps over it)
    void enqueue_transpose(bool light = false) {
        launch_row_offsets(ddesc(), dwp(kPhRows), nblk[kPhRows], count, s);
        launch_transpose(ddesc(), dwp(kPhChunks), nblk[kPhChunks], count, maxM, light, s);
    }

    // sweep state per matrix (active, sweeps, not converged), written by the device
    int32_t *js_dev() { return reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned_dev) + stage_off + h.o_js); }
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

ranky_status make_engine(ranky_ctx *ctx, hipStream_t s, const Header &h, char *hdr, int count, Engine &e,
                         size_t stage_off = 0) {
    ranky_status st = ensure_pinned(ctx, stage_off + h.total);
    if (st) return st;
    e.stage_off = stage_off;
    e.ctx = ctx;
    e.s = s;
    e.count = count;
    e.h = h;
    e.hdr = hdr;
    e.status.assign(count, RANKY_OK);
    e.gsegs.assign(count, 0);
    return RANKY_OK;
}

size_t topk_small_header_bytes(int32_t p) { return make_header(1, 1, p / kJacobiBlock).total; }

// Block width of the subspace iteration for a call on `count` matrices of which the first has
// M rows and k wanted pairs (0: the full Jacobi runs).  eigensolver 2 asks for it whenever the
// block is at most half the rows; 0 (automatic) takes it when the block is at most an eighth.
int32_t topk_plan_p(const ranky_opts &o, int count, int32_t M, int32_t k) {
    if (count != 1 || o.eigensolver == 1) return 0;
    const int32_t p = topk_block(k);
    if (p > kTopkMaxBlock) return 0;
    return (o.eigensolver == 2 ? 2 * p : 8 * p) <= M ? p : 0;
}

// The subspace iteration on the main matrix of engine e (a batch of one): Chebyshev filter,
// orthonormalisation (Cholesky-QR, or SVQB for wide blocks), Rayleigh-Ritz, until the k leading Ritz pairs have residuals at most
// tol_r theta_1 (or stop improving at the rounding level).  On success the Ritz values are in
// lam[0, p) (descending), the Ritz vectors in W's first p columns, neig = p, and *iters
// holds the iterations; *iters = 0 when it did not converge (the caller runs the Jacobi).
struct Topk {
    ranky_ctx *ctx;
    hipStream_t s;
    TopkLayout L;
    char *base;               // the region in the workspace
    MatDesc *x;               // the main matrix (host copy)
    Engine es;                // the p x p Jacobi
    double *blk[5];
    double *part, *Sp, *Wm, *Qs, *theta, *dvec;
    int32_t *cflag = nullptr;   // set by a failed Cholesky-QR (host-visible)
    int32_t n = 0;           // rows of G (the products' useful rows)
    double flops = 0.0;      // algorithmic flops of the products: 2 (useful rows) x cols x (useful k)

    double *at(size_t o) { return reinterpret_cast<double *>(base + o); }

    // out = alpha op(A) B + beta E + gamma F  (rows x cols, ld cols)
    void gemm(bool ta, const double *A, int64_t lda, const double *B, int64_t ldb, double *out, int32_t rows,
              int32_t cols, int32_t K, int32_t a_valid, int32_t k_valid, double alpha, double beta = 0.0,
              const double *E = nullptr, double gamma = 0.0, const double *F = nullptr) {
        int32_t splits, klen;
        flops += 2.0 * (ta ? rows : std::min(rows, n)) * cols * std::min(K, std::min(k_valid, n));
        bool done = false;
        if (!ta && cols <= kTopkWideMaxP && K >= kTopkWideMinK) {
            topk_split(rows / kTopkTile, K, splits, klen, kTopkWideTarget);
            done = launch_tk_gemm_wide(A, lda, B, ldb, part, rows, cols, K, splits, klen, a_valid, k_valid, s);
        }
        if (!done) {
            topk_split((int64_t)(rows / kTopkTile) * (cols / kTopkTile), K, splits, klen);
            launch_tk_gemm(ta, A, lda, B, ldb, part, rows, cols, K, splits, klen, a_valid, k_valid, s);
        }
        launch_tk_combine(part, splits, (int64_t)rows * cols, alpha, beta, E, gamma, F, out, s);
    }
    // the p x p Jacobi on the matrix already in es's G; eigenvectors in its W, values in lam
    ranky_status eig() {
        launch_fill_i32(es.d[0].scal, kScCount, 0, s);
        const ranky_status st = es.eigensolve(false);
        if (st) return st;
        if (es.notconv[0]) return fail(RANKY_E_NOT_CONVERGED, "Jacobi on a %d x %d block did not converge", L.p, L.p);
        return RANKY_OK;
    }
    // one Cholesky-QR pass: S = Y^T Y, out = Y diag(S)^-1/2 L^-T (a failed factorisation sets
    // *cflag and leaves out = Y)
    void cholqr(const double *Y, double *out, double shift) {
        const int32_t p = L.p;
        gemm(true, Y, p, Y, p, Sp, p, p, L.rows, L.rows, L.rows, 1.0);
        launch_tk_chol(Sp, p, shift, Wm, cflag, s);
        gemm(false, Y, p, Wm, p, out, L.rows, p, p, L.rows, p, 1.0);
    }
    // out = an orthonormal basis of span(Y) (tmp: scratch of the same shape).  Blocks up to
    // kTopkCholMax wide: three Cholesky-QR passes, the first shifted so that it cannot break
    // down on an ill-conditioned block (its triangular factor keeps every column's direction
    // close to its own, so the Rayleigh-Ritz matrix that follows stays near diagonal); wider
    // blocks: two SVQB passes.
    ranky_status orth(const double *Y, double *out, double *tmp) {
        const int32_t p = L.p;
        if (p <= kTopkCholMax) {
            const double shift = 11.0 * ((double)n * p + (double)p * (p + 1)) * std::ldexp(1.0, -53) * p;
            cholqr(Y, out, shift);
            cholqr(out, tmp, 0.0);
            cholqr(tmp, out, 0.0);
            return RANKY_OK;
        }
        const ranky_status st = svqb(Y, tmp);
        if (st) return st;
        return svqb(tmp, out);
    }
    // Y (orthonormal afterwards) <- Y D^-1 V L^-1/2, written to out
    ranky_status svqb(const double *Y, double *out) {
        const int32_t p = L.p;
        gemm(true, Y, p, Y, p, Sp, p, p, L.rows, L.rows, L.rows, 1.0);
        launch_tk_symcopy(Sp, p, es.d[0].G, dvec, s);
        ranky_status st = eig();
        if (st) return st;
        launch_tk_svqb_w(es.d[0].W, es.d[0].lam, dvec, p, Wm, s);
        gemm(false, Y, p, Wm, p, out, L.rows, p, p, L.rows, p, 1.0);
        return RANKY_OK;
    }
};

// start (or NULL): a start block (rows x p, ld p) in place of the one built from G's diagonal.
ranky_status topk_eigensolve(ranky_ctx *ctx, Engine &e, const Plan &plan, char *mat_base, double tol_r,
                             int32_t max_iters, hipStream_t s, int32_t *iters, double *flops,
                             const double *start = nullptr) {
    *iters = 0;
    MatDesc &x = e.d[0];
    Topk t;
    t.n = x.n;
    t.ctx = ctx;
    t.s = s;
    t.L = plan.topk;
    t.base = mat_base + plan.o_topk;
    t.x = &x;
    for (int i = 0; i < 5; ++i) t.blk[i] = t.at(t.L.o_blk[i]);
    t.part = t.at(t.L.o_part);
    t.Sp = t.at(t.L.o_Sp);
    t.Wm = t.at(t.L.o_Wm);
    t.Qs = t.at(t.L.o_Qs);
    t.theta = t.at(t.L.o_theta);
    t.dvec = t.at(t.L.o_dvec);
    const int32_t p = t.L.p, rows = t.L.rows, n = x.n, npad = x.npad, k = x.k;
    // the p x p Jacobi: its own descriptor and header in the region; the read-back of the Ritz
    // values and residuals (2p doubles) goes through the pinned staging past both headers.  The
    // staging is sized first, so that no later growth drops what the small engine stages there.
    const Header hs = make_header(1, 1, p / kJacobiBlock);
    const size_t small_off = align_up(e.stage_off + e.h.total);   // the main engine's uploads may be pending
    const size_t rb_off = align_up(small_off + hs.total);
    ranky_status st = ensure_pinned(ctx, rb_off + sizeof(double) * 2 * (size_t)p + sizeof(int32_t));
    if (st) return st;
    st = make_engine(ctx, s, hs, t.base + t.L.o_hdr, 1, t.es, small_off);
    if (st) return st;
    MatDesc jd;
    std::memset(&jd, 0, sizeof(jd));
    jd.scal = reinterpret_cast<int32_t *>(t.base + t.L.o_jscal);
    jd.sdbl = t.at(t.L.o_jsdbl);
    jd.jstate = reinterpret_cast<int32_t *>(t.base + t.L.o_jstate);
    jd.G = t.at(t.L.o_jG);
    jd.G2 = t.at(t.L.o_jG2);
    jd.W = t.at(t.L.o_jW);
    jd.J = t.at(t.L.o_jJ);
    jd.S = t.at(t.L.o_jS);
    jd.jflag = reinterpret_cast<int32_t *>(t.base + t.L.o_jflag);
    jd.lam = t.at(t.L.o_jlam);
    jd.perm = reinterpret_cast<int32_t *>(t.base + t.L.o_jperm);
    jd.sigma = t.at(t.L.o_sig);
    jd.M = jd.k = jd.n = jd.n_tau = jd.neig = jd.npad = p;
    jd.u_gram = std::ldexp(1.0, -53);
    t.es.d.assign(1, jd);
    t.es.sweeps_cap = kDefaultSweeps;
    t.es.maxn = p;
    st = t.es.plan_rest();
    if (st) return st;

    double *rb_dev = reinterpret_cast<double *>(static_cast<char *>(ctx->pinned_dev) + rb_off);
    const double *rb_host = reinterpret_cast<const double *>(static_cast<const char *>(ctx->pinned) + rb_off);
    const size_t flag_off = rb_off + sizeof(double) * 2 * (size_t)p;
    t.cflag = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned_dev) + flag_off);
    volatile int32_t *cflag_host = reinterpret_cast<volatile int32_t *>(static_cast<char *>(ctx->pinned) + flag_off);
    *cflag_host = 0;

    // three rotating block buffers (the basis Y, the Ritz vectors X, the filter's third term)
    // plus T = G Y and G X
    double *R3[3] = {t.blk[0], t.blk[1], t.blk[2]};
    double *T = t.blk[3], *GX = t.blk[4];
    const double *G = x.G;
    if (start)
        HIP_TRY(hipMemcpyAsync(R3[1], start, sizeof(double) * (size_t)rows * p, hipMemcpyDeviceToDevice, s));
    else
        launch_tk_start(G, npad, n, p, rows, R3[1], s);
    double *Y = R3[0];
    st = t.orth(R3[1], Y, R3[2]);
    if (st) return st;
    double prev_res = 1e300;
    bool done = false;
    double *X = R3[1];   // Ritz vectors of the current iteration
    int32_t it = 0;
    for (; it < max_iters; ++it) {
        // Rayleigh-Ritz on the orthonormal Y
        t.gemm(false, G, npad, Y, p, T, rows, p, npad, npad, npad, 1.0);
        t.gemm(true, Y, p, T, p, t.Sp, p, p, rows, rows, rows, 1.0);
        launch_tk_symcopy(t.Sp, p, t.es.d[0].G, nullptr, s);
        st = t.eig();
        if (st) return st;
        launch_select(t.es.ddesc(), 1, p, s);
        launch_tk_permute(t.es.d[0].W, t.es.d[0].lam, t.es.d[0].perm, p, t.Qs, t.theta, s);
        X = (Y == R3[0]) ? R3[1] : R3[0];
        t.gemm(false, Y, p, t.Qs, p, X, rows, p, p, rows, p, 1.0);
        t.gemm(false, T, p, t.Qs, p, GX, rows, p, p, rows, p, 1.0);
        launch_tk_resid(GX, X, t.theta, n, p, rb_dev, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        if (*cflag_host) return RANKY_OK;   // a Cholesky-QR broke down: the full Jacobi takes over
        const double th0 = rb_host[0];
        double worst = 0.0;
        for (int32_t i = 0; i < k; ++i) worst = std::max(worst, rb_host[p + i]);
        if (!(th0 > 0.0) || worst <= tol_r * th0) {
            done = true;
            break;
        }
        // at the rounding level the residuals stop shrinking: accept once they are close to it
        if (it >= 3 && worst > 0.5 * prev_res && worst <= 8.0 * tol_r * th0) {
            done = true;
            break;
        }
        prev_res = worst;
        // Chebyshev filter of X damping [0, b], b = the smallest Ritz value, scaled at theta_1;
        // the degree keeps the growth of the leading direction within what the
        // orthonormalisation takes: the shifted Cholesky-QR pass any condition number below
        // about 1/u (growth 1e10, degree up to 16), SVQB about 1/sqrt(u) (1e7, degree 8)
        const bool chol = p <= kTopkCholMax;
        const double growth = chol ? 1e10 : 1e7;
        const int32_t max_deg = chol ? 16 : 8;
        const double b = std::max(rb_host[p - 1], th0 * 1e-12);
        const double c = 0.5 * b, ew = 0.5 * b;
        const double x0 = (th0 - c) / ew;
        int32_t m = 1;
        if (x0 > 1.0) {
            const double ac = std::acosh(x0);
            while (m < max_deg && std::cosh((m + 1) * ac) <= growth) ++m;
        }
        const double sigma1 = ew / (th0 - c);
        const double tau = 2.0 / sigma1;
        double sig = sigma1;
        // the recurrence's three terms rotate over the three buffers, starting from X (Y is free now)
        double *prev = X, *cur = nullptr, *spare = nullptr;
        for (double *b : R3)
            if (b != X) (cur ? spare : cur) = b;
        t.gemm(false, G, npad, prev, p, cur, rows, p, npad, npad, npad, sigma1 / ew, -c * sigma1 / ew, prev);
        for (int32_t d = 2; d <= m; ++d) {
            const double sig2 = 1.0 / (tau - sig);
            t.gemm(false, G, npad, cur, p, spare, rows, p, npad, npad, npad, 2.0 * sig2 / ew, -c * 2.0 * sig2 / ew, cur,
                   -sig * sig2, prev);
            double *np_ = prev;
            prev = cur;
            cur = spare;
            spare = np_;
            sig = sig2;
        }
        // orthonormalise the filtered block into a free buffer as the next Y
        st = t.orth(cur, prev, spare);
        if (st) return st;
        Y = prev;
    }
    if (!done) return RANKY_OK;   // *iters stays 0: the caller falls back to the full Jacobi
    *iters = it + 1;
    *flops = t.flops;
    // the Ritz pairs become the eigensolve's output: lam[0, p) and W[:, 0, p)
    HIP_TRY(hipMemcpyAsync(x.lam, t.theta, sizeof(double) * p, hipMemcpyDeviceToDevice, s));
    launch_tk_place(X, npad, p, x.W, npad, s);
    HIP_TRY(hipGetLastError());
    x.neig = p;
    return e.upload_desc();
}

// The heavy-row split of the Gram: a single matrix with an FP64 or FP32 Gram, automatic from
// kHeavyMinNnz nonzeros (below it the walk over every pair is cheap and the split's per-column
// pass is not), or as opts.gram_split asks.
bool heavy_split(const ranky_opts &o, int count, int64_t nnz) {
    if (count != 1 || o.gram_prec == RANKY_PREC_BF16X3 || o.gram_split == 1) return false;
    return o.gram_split == 2 || nnz >= kHeavyMinNnz;
}

size_t path_bytes(const std::vector<Job> &jobs, const ranky_opts &o) {
    const int count = (int)jobs.size();
    const bool refine = count == 1 && wants_refine(o, jobs[0].k);
    int32_t maxM = 1;
    int64_t sum_d = 0;
    size_t total = 0;
    const int32_t topk_p = topk_plan_p(o, count, jobs[0].M, jobs[0].k);
    for (const Job &j : jobs) {
        total += make_plan(j.M, j.N, j.A.nnz, j.k, j.D, true, refine, j.bstart, count == 1, o.v_dtype == RANKY_F32,
                           topk_p, heavy_split(o, count, j.A.nnz))
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
    const int32_t topk_p = topk_plan_p(o, count, jobs[0].M, jobs[0].k);
    for (int i = 0; i < count; ++i) {
        plans[i] = make_plan(jobs[i].M, jobs[i].N, jobs[i].A.nnz, jobs[i].k, jobs[i].D, true, refine, jobs[i].bstart,
                             count == 1, o.v_dtype == RANKY_F32, topk_p, heavy_split(o, count, jobs[i].A.nnz));
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
        x.gwaves = gram_waves(x.M, x.prec == RANKY_PREC_FP64 ? 8 : 4, ctx->lds_limit, x.hwg == 0);
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
    const bool heavy = count == 1 && e.d[0].hwg > 0;
    if (heavy) launch_gram_heavy_prep(e.ddesc(), e.d[0], s);
    e.enqueue_transpose(heavy);
    if (timing) hipEventRecord(ctx->ev[2], s);
    int32_t gram_nw = 1;
    size_t gram_lds = 0;
    gram_shape(e.d, ctx->lds_limit, gram_nw, gram_lds);
    if (count == 1) launch_gram_dense(e.ddesc(), e.d[0].dwg, s);
    launch_gram(e.ddesc(), e.dwp(kPhGram), e.nblk[kPhGram], e.dwp(kPhGramRed), e.nblk[kPhGramRed], count, gram_nw,
                gram_lds, heavy, s);
    if (count == 1) launch_gram_dense_reduce(e.ddesc(), e.d[0].dwg, s);
    if (count == 1) launch_gram_heavy_tiles(e.ddesc(), e.d[0].dtype, e.d[0].hwg, s);
    HIP_TRY(hipGetLastError());
    if (timing) hipEventRecord(ctx->ev[3], s);
    // the k leading pairs by subspace iteration when the block is narrow next to M' (and the
    // full Jacobi if that does not converge); otherwise the full Jacobi
    int32_t eig_iters = 0;
    double eig_flops = 0.0;
    const int32_t tkp = plans[0].topk.p;
    if (tkp > 0 && e.status[0] == RANKY_OK && (o.eigensolver == 2 ? 2 * tkp : 8 * tkp) <= e.d[0].n &&
        jobs[0].k <= tkp) {
        const double tol_r = e.d[0].prec == RANKY_PREC_FP64 ? std::sqrt((double)e.d[0].n) * std::ldexp(1.0, -52)
                                                             : kJacobiTolFp32Gram;
        st = topk_eigensolve(ctx, e, plans[0], ws + base[0], tol_r, o.max_iters > 0 ? o.max_iters : kTopkDefaultIters,
                             s, &eig_iters, &eig_flops);
        if (st) return st;
        if (eig_iters == 0) st = e.plan_rest();   // the staging was reused: rebuild the round tables
        if (st) return st;
    }
    if (eig_iters > 0) {
        e.sweeps.assign(count, 0);
        e.notconv.assign(count, 0);
    } else {
        st = e.eigensolve(use_graph);
        if (st) return st;
    }
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
        // the main matrix's header entries are no longer read: reuse them for H (staged past
        // the main engine's staging, whose last upload may still be pending)
        Engine eh;
        st = make_engine(ctx, s, h, ws, 1, eh, align_up(e.stage_off + e.h.total));
        if (st) return st;
        eh.sweeps_cap = o.max_sweeps;
        eh.d.assign(1, x);
        MatDesc &y = eh.d[0];
        y.n = k;
        y.neig = k;
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
            in.eig_iters = i == 0 ? eig_iters : 0;
            in.eig_flops = i == 0 ? eig_flops : 0.0;
            in.topk_block = (i == 0 && eig_iters > 0) ? plans[0].topk.p : 0;
            in.heavy_rows = iv[kColI * i + 10];
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
                       int32_t *single, bool heavy = false) {
    const Plan p = make_plan(M, N, A->nnz, 1, D, false, false, nullptr, true, false, 0, heavy);
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

// ---------------------------------------------------------------------------
// the paper's own procedure: checkers, per-block factors, proxy matrix
// ---------------------------------------------------------------------------

// Checker region: the scan's workspace (with the [D x M] occupancy), the new entries and the
// scratch of A' = A plus them.
struct CheckerPlan {
    Plan scan;
    Header h;
    size_t o_scan = 0, o_cnt = 0, o_ins = 0, o_counts = 0, o_cursor = 0, o_long = 0, o_btot = 0, o_iptr = 0;
    size_t o_nlong = 0, o_irow = 0, o_ival = 0, total = 0;
};

CheckerPlan checker_plan(int32_t M, int64_t N, int64_t nnz, int32_t D) {
    CheckerPlan c;
    c.h = make_header(1, 1, 1);
    c.scan = make_plan(M, N, nnz, 1, D, false, false, nullptr, true);   // the step scan's own plan
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    c.o_scan = take(c.h.total + c.scan.total);
    const size_t nin = 2 * (size_t)D * (size_t)M;
    c.o_cnt = take(sizeof(int32_t) * (size_t)D * M);
    c.o_ins = take(sizeof(int64_t) * nin);
    c.o_counts = take(sizeof(int32_t) * (size_t)N);
    c.o_cursor = take(sizeof(int32_t) * (size_t)N);
    c.o_long = take(sizeof(int32_t) * (size_t)N);
    c.o_btot = take(sizeof(int32_t) * (size_t)tall_scan_blocks(N));
    c.o_iptr = take(sizeof(int32_t) * ((size_t)N + 1));
    c.o_nlong = take(sizeof(int32_t));
    c.o_irow = take(sizeof(int32_t) * nin);
    c.o_ival = take(sizeof(double) * nin);
    c.total = off;
    return c;
}

ranky_status check_checker_args(const ranky_csc *A, int32_t M, int64_t N, int32_t D, int32_t kind) {
    ranky_status st = check_csc_args(A, M, N);
    if (st) return st;
    if (D < 1 || D > N) return fail(RANKY_E_INVALID, "D=%d outside [1, N]", D);
    if (kind < 0 || kind > 2) return fail(RANKY_E_INVALID, "checker kind %d (0, 1 or 2)", kind);
    const int64_t wmax = (N + D - 1) / D;
    if (checker_lds_bytes(M, wmax) > 150 * 1024)
        return fail(RANKY_E_INVALID, "blocks of %lld columns are too wide for the neighbour sets", (long long)wmax);
    return RANKY_OK;
}

// A' into (colptr_out, rowidx_out, vals_out); *added (host) = entries added.  Blocking.
ranky_status run_checker(StepCtx &sc, const ranky_csc *A, int32_t M, int64_t N, int32_t D, int32_t kind, uint64_t seed,
                         int32_t *colptr_out, int32_t *rowidx_out, double *vals_out, char *ws, hipStream_t s,
                         int64_t *added) {
    const CheckerPlan c = checker_plan(M, N, A->nnz, D);
    auto i32 = [&](size_t o) { return reinterpret_cast<int32_t *>(ws + o); };
    Engine e;
    ranky_status st = step_scan(sc, A, M, N, D, ws + c.o_scan, c.h.total + c.scan.total, s, e, i32(c.o_cnt), nullptr,
                                nullptr, nullptr);
    if (st) return st;
    const MatDesc &x = e.d[0];
    e.enqueue_transpose();   // the rows of A: rowptr and the column of every entry
    const CscView Av{A->nnz, A->colptr, A->rowidx, A->values, A->dtype};
    int64_t *ins = reinterpret_cast<int64_t *>(ws + c.o_ins);
    launch_checker(Av, M, N, D, i32(c.o_cnt), x.rowptr, x.csrcol, kind, seed, ins, s);
    launch_fill_f64(reinterpret_cast<double *>(ws + c.o_ival), 2 * (int64_t)D * M, 1.0, s);
    launch_checker_apply(Av, M, N, ins, 2 * (int64_t)D * M, i32(c.o_counts), i32(c.o_btot), i32(c.o_iptr),
                         i32(c.o_cursor), i32(c.o_irow), reinterpret_cast<double *>(ws + c.o_ival), i32(c.o_long),
                         i32(c.o_nlong), colptr_out, rowidx_out, vals_out, s);
    HIP_TRY(hipGetLastError());
    int32_t tot = 0;
    HIP_TRY(hipMemcpyAsync(&tot, i32(c.o_iptr) + N, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *added = tot;
    return RANKY_OK;
}

// Layout of the paper's route for an M x N matrix with nnz entries, D blocks, k outputs: the
// checker's region and A' (when a checker runs), the scan of A', the D block matrices' batch
// (each block's Gram, full Jacobi, its U and sigma), P^T and the products' partials, and the
// Jacobi of P P^T with its selection.  Block entries are bounded by nnz + 2 D M (the checker adds
// at most two entries per (block, row)) and by the block's size.
struct PaperPlan {
    CheckerPlan chk;
    Plan scan;
    Header hscan;
    int32_t np = 0;           // P P^T order: M rounded up to 64
    int64_t nnz1 = 0;         // entries of A' at most
    size_t o_chk = 0, o_cp = 0, o_ri = 0, o_va = 0, o_scan = 0, o_slices = 0, o_bsig = 0, o_bU = 0, o_rank = 0;
    size_t o_Pt = 0, o_part = 0, o_Gp = 0, o_jhdr = 0, o_jscal = 0, o_jsdbl = 0, o_jstate = 0, o_jG2 = 0, o_jW = 0;
    size_t o_jJ = 0, o_jS = 0, o_jflag = 0, o_jlam = 0, o_jperm = 0, o_err = 0, o_batch = 0, batch = 0, total = 0;
    int32_t part_splits = 1;
};

std::vector<Job> paper_block_jobs(int32_t M, int64_t N, int32_t D, const std::vector<int64_t> &bnnz) {
    std::vector<Job> jobs(D);
    for (int32_t b = 0; b < D; ++b) {
        std::memset(&jobs[b], 0, sizeof(Job));
        jobs[b].A.nnz = bnnz[b];
        jobs[b].A.dtype = RANKY_F64;
        jobs[b].M = M;
        jobs[b].N = ((int64_t)(b + 1) * N) / D - ((int64_t)b * N) / D;
        jobs[b].k = M;
        jobs[b].D = 1;
    }
    return jobs;
}

ranky_opts paper_block_opts() {
    ranky_opts o;
    ranky_default_opts(&o);
    o.refine = 0;
    o.eigensolver = 1;
    o.max_sweeps = kDefaultSweeps;
    return o;
}

PaperPlan paper_plan(int32_t M, int64_t N, int64_t nnz, int32_t k, int32_t D, bool checker) {
    PaperPlan pp;
    pp.np = ((M + kTopkTile - 1) / kTopkTile) * kTopkTile;
    pp.nnz1 = checker ? nnz + 2 * (int64_t)D * M : nnz;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t nz1 = (size_t)(pp.nnz1 > 0 ? pp.nnz1 : 1);
    if (checker) {
        pp.chk = checker_plan(M, N, nnz, D);
        pp.o_chk = take(pp.chk.total);
        pp.o_cp = take(sizeof(int32_t) * ((size_t)N + 1));
        pp.o_ri = take(sizeof(int32_t) * nz1);
        pp.o_va = take(sizeof(double) * nz1);
    }
    pp.hscan = make_header(1, 1, 1);
    pp.scan = make_plan(M, N, pp.nnz1, 1, D, false, false, nullptr, true);
    pp.o_scan = take(pp.hscan.total + pp.scan.total);
    pp.o_slices = take(sizeof(int32_t) * ((size_t)N + D));
    pp.o_bsig = take(sizeof(double) * (size_t)D * M);
    pp.o_bU = take(sizeof(double) * (size_t)D * M * M);
    pp.o_rank = take(sizeof(int32_t) * (size_t)D);
    const size_t np = pp.np;
    // at most M retained triplets per block; the product reads the rows padded to a multiple of 16
    const size_t pt_rows = std::max<size_t>(16, (((size_t)D * M + 15) / 16) * 16);
    pp.o_Pt = take(sizeof(double) * pt_rows * np);
    int32_t klen = 0;
    topk_split((int64_t)(np / kTopkTile) * (np / kTopkTile), (int32_t)std::min<int64_t>((int64_t)D * M, 0x7fffffff),
               pp.part_splits, klen);
    pp.o_part = take(sizeof(double) * (size_t)pp.part_splits * np * np);
    pp.o_Gp = take(sizeof(double) * np * np);
    const Header hj = make_header(1, 1, (int32_t)(np / kJacobiBlock));
    pp.o_jhdr = take(hj.total);
    const size_t npairs = np / kJacobiPair;
    pp.o_jscal = take(sizeof(int32_t) * kScCount);
    pp.o_jsdbl = take(sizeof(double) * kSdCount);
    pp.o_jstate = take(sizeof(int32_t) * kJsCount);
    pp.o_jG2 = take(sizeof(double) * np * np);
    pp.o_jW = take(sizeof(double) * np * np);
    pp.o_jJ = take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair);
    pp.o_jS = take(sizeof(double) * 2 * npairs * kJacobiPair * kJacobiPair);
    pp.o_jflag = take(sizeof(int32_t) * 2 * npairs);
    pp.o_jlam = take(sizeof(double) * np);
    pp.o_jperm = take(sizeof(int32_t) * np);
    pp.o_err = take(sizeof(double) * ((size_t)k + 2));
    // the blocks' batch, each block sized for the most entries it can hold
    std::vector<int64_t> bnnz(D);
    for (int32_t b = 0; b < D; ++b) {
        const int64_t w = ((int64_t)(b + 1) * N) / D - ((int64_t)b * N) / D;
        bnnz[b] = std::min<int64_t>(pp.nnz1, w * (int64_t)M);
    }
    pp.batch = path_bytes(paper_block_jobs(M, N, D, bnnz), paper_block_opts());
    pp.o_batch = take(pp.batch);
    pp.total = off;
    return pp;
}

// ---------------------------------------------------------------------------
// incremental merge: a resident Gram that column blocks are added to
// ---------------------------------------------------------------------------

struct IncLayout {
    Plan step, solve;
    Header hstep, hsolve;
    int32_t p = 0;
    size_t o_G = 0, o_step = 0, o_solve = 0, o_keep = 0, o_start = 0, total = 0;
};

IncLayout inc_layout(int32_t M, int64_t max_cols, int64_t max_nnz, int32_t k, const ranky_opts &o) {
    IncLayout L;
    L.p = topk_plan_p(o, 1, M, k);
    const int32_t D = default_blocks(max_cols);
    L.hstep = make_header(1, 1, 1);
    // the largest step plan over the blocks the state takes: the partial Gram rows per entry are
    // largest just below each doubling of the segment length, so those sizes are tried too
    L.step = make_plan(M, max_cols, max_nnz, 1, D, false, false, nullptr, true);
    for (int64_t seg = kGramSegMin; seg <= kGramSeg; seg *= 2) {
        const int64_t nz = std::min<int64_t>(max_nnz, seg * kGramSegTarget * 2 - 1);
        const Plan q = make_plan(M, max_cols, nz, 1, D, false, false, nullptr, true);
        if (q.total > L.step.total) L.step = q;
    }
    L.hsolve = make_header(1, 1, jacobi_npad(M) / kJacobiBlock);
    L.solve = make_plan(M, 1, 0, k, 1, true, false, nullptr, false, false, L.p);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t of = off;
        off = align_up(off + bytes);
        return of;
    };
    L.o_G = take(sizeof(double) * (size_t)M * M);
    L.o_step = take(L.hstep.total + L.step.total);
    L.o_solve = take(L.hsolve.total + L.solve.total);
    if (L.p > 0) {
        L.o_keep = take(sizeof(double) * (size_t)M * L.p);
        L.o_start = take(sizeof(double) * (size_t)L.solve.topk.rows * L.p);
    }
    L.total = off;
    return L;
}

// Tall-and-skinny layout: the transposed CSC and the scratch of the transpose, ahead of the
// short-and-fat path's workspace for A^T (values sized for FP64).
struct TallPlan {
    size_t o_status = 0, o_counts = 0, o_cursor = 0, o_long = 0, o_btot = 0, o_ptr = 0, o_nlong = 0, o_trow = 0;
    size_t o_tval = 0, o_path = 0;
};

TallPlan tall_plan(int64_t M, int64_t nnz) {
    TallPlan t;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t nz = (size_t)(nnz > 0 ? nnz : 1);
    t.o_status = take(sizeof(int32_t));
    t.o_counts = take(sizeof(int32_t) * (size_t)M);
    t.o_cursor = take(sizeof(int32_t) * (size_t)M);
    t.o_long = take(sizeof(int32_t) * (size_t)M);
    t.o_btot = take(sizeof(int32_t) * (size_t)tall_scan_blocks(M));
    t.o_ptr = take(sizeof(int32_t) * ((size_t)M + 1));
    t.o_nlong = take(sizeof(int32_t));
    t.o_trow = take(sizeof(int32_t) * nz);
    t.o_tval = take(sizeof(double) * nz);
    t.o_path = off;
    return t;
}

ranky_status check_tall_args(const ranky_csc *A, int64_t M, int32_t N, int32_t k) {
    if (!A) return fail(RANKY_E_INVALID, "A is NULL");
    if (M < 1 || N < 1) return fail(RANKY_E_INVALID, "M=%lld N=%d must be >= 1", (long long)M, N);
    if (N > kMaxM) return fail(RANKY_E_INVALID, "N=%d exceeds %d (the narrow side of a tall matrix)", N, kMaxM);
    if (M > (int64_t)0x7ffffffe) return fail(RANKY_E_INVALID, "M=%lld exceeds int32 row pointers", (long long)M);
    if (A->nnz < 0 || A->nnz > (int64_t)0x7fffffff) return fail(RANKY_E_INVALID, "nnz=%lld out of range", (long long)A->nnz);
    if (!A->colptr || (A->nnz > 0 && (!A->rowidx || !A->values))) return fail(RANKY_E_INVALID, "NULL CSC array");
    if (A->dtype != RANKY_F32 && A->dtype != RANKY_F64) return fail(RANKY_E_INVALID, "bad dtype %d", A->dtype);
    if (k < 1 || k > N) return fail(RANKY_E_INVALID, "k=%d must be in [1, N=%d]", k, N);
    return RANKY_OK;
}

}  // namespace

struct ranky_inc {
    ranky_ctx *ctx = nullptr;
    int32_t M = 0, k = 0;
    int64_t max_cols = 0, max_nnz = 0;
    ranky_opts o;
    IncLayout L;
    char *ws = nullptr;
    int64_t blocks = 0, cols = 0, nnz = 0;
    bool has_prev = false;   // Ritz vectors of an earlier solve are kept for a warm start
};

namespace ranky {

ranky_status set_error(ranky_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

int ctx_device(const ranky_ctx *ctx) { return ctx ? ctx->device : -1; }

ranky_status svd_fixed_workspace(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, double tol,
                                 const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, double *U,
                                 void *V, ranky_info *info, ranky_stream_t stream) {
    ranky_opts o;
    ranky_default_opts(&o);
    if (opts) o = *opts;
    o.graph = 0;   // a captured graph is instantiated with allocations of its own
    ctx->no_alloc = true;
    const ranky_status st = ranky_svd(ctx, A, M, N, k, tol, &o, workspace, ws_bytes, sigma, U, V, info, stream);
    ctx->no_alloc = false;
    return st;
}

}  // namespace ranky

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
    hipError_t e = kernel_attributes(device, c->lds_limit);
    if (e == hipSuccess) e = noalloc_setup(device);
    if (e != hipSuccess) {
        ranky_ctx_destroy(c);
        return fail(RANKY_E_DEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(e));
    }
    // staging sized for a single matrix of any size up front, so that the call that may not
    // allocate (ranky_svd_noalloc) finds it ready
    const ranky_status ps = ensure_pinned(c, kStagingBytes);
    if (ps != RANKY_OK) {
        ranky_ctx_destroy(c);
        return ps;
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
    const int32_t bp_cands[4] = {16, 32, 64, 128};
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
    return make_header(1, 1, 1).total +
           make_plan(M, N, nnz, 1, D, false, false, nullptr, true, false, 0, nnz >= kHeavyMinNnz).total;
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
    // the heavy-row split as the path takes it (FP64 / FP32 Grams of at least kHeavyMinNnz nonzeros)
    const bool heavy = prec != RANKY_PREC_BF16X3 && A->nnz >= kHeavyMinNnz;
    st = step_scan(sc, A, M, N, default_blocks(N), workspace, ws_bytes, s, e, nullptr, nullptr, nullptr, nullptr,
                   heavy);
    if (st) return st;
    MatDesc &x = e.d[0];
    x.prec = prec;
    if (x.prec != RANKY_PREC_BF16X3) x.dwg = 0;
    x.gwaves = gram_waves(M, prec == RANKY_PREC_FP64 ? 8 : 4, sc.c.lds_limit, x.hwg == 0);
    if (x.n > 0) {
        e.nblk[kPhGram] = fill_wp(e.hwp(kPhGram), 1, [&](int) { return (int64_t)e.gsegs[0] + (x.npad - x.n); });
        e.nblk[kPhGramRed] = fill_wp(e.hwp(kPhGramRed), 1, [&](int) { return (int64_t)x.n; });
        st = e.upload_desc();
        if (!st) st = e.upload(e.h.o_wp, sizeof(int32_t) * (size_t)kPhCount * (e.h.slots + 1));
        if (st) return st;
        if (x.hwg > 0) launch_gram_heavy_prep(e.ddesc(), x, s);
        e.enqueue_transpose(x.hwg > 0);
        launch_gram_dense(e.ddesc(), x.dwg, s);
        int32_t gram_nw = 1;
        size_t gram_lds = 0;
        gram_shape(e.d, sc.c.lds_limit, gram_nw, gram_lds);
        launch_gram(e.ddesc(), e.dwp(kPhGram), e.nblk[kPhGram], e.dwp(kPhGramRed), e.nblk[kPhGramRed], 1, gram_nw,
                    gram_lds, x.hwg > 0, s);
        launch_gram_dense_reduce(e.ddesc(), x.dwg, s);
        launch_gram_heavy_tiles(e.ddesc(), x.dtype, x.hwg, s);
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
    x.neig = n;
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

// ---------------------------------------------------------------------------
// tall and skinny
// ---------------------------------------------------------------------------

size_t ranky_tall_workspace_bytes(int64_t M, int32_t N, int64_t nnz, int32_t k, const ranky_opts *opts) {
    if (M < 1 || N < 1 || N > kMaxM || k < 1 || k > N || nnz < 0 || M > (int64_t)0x7ffffffe) return 0;
    const size_t path = ranky_workspace_bytes(N, M, nnz, k, opts);
    if (path == 0) return 0;
    return tall_plan(M, nnz).o_path + path;
}

ranky_status ranky_transpose(const ranky_csc *A, int64_t M, int64_t N, int32_t *colptr_t, int32_t *rowidx_t,
                             void *values_t, void *workspace, size_t ws_bytes, ranky_stream_t stream) {
    if (!A || M < 1 || N < 1 || M > (int64_t)0x7ffffffe || N > (int64_t)0x7ffffffe)
        return fail(RANKY_E_INVALID, "bad sizes");
    if (A->nnz < 0 || A->nnz > (int64_t)0x7fffffff) return fail(RANKY_E_INVALID, "nnz out of range");
    if (!A->colptr || (A->nnz > 0 && (!A->rowidx || !A->values || !rowidx_t || !values_t)) || !colptr_t)
        return fail(RANKY_E_INVALID, "NULL array");
    if (A->dtype != RANKY_F32 && A->dtype != RANKY_F64) return fail(RANKY_E_INVALID, "bad dtype %d", A->dtype);
    const TallPlan t = tall_plan(M, A->nnz);
    if (!workspace || ws_bytes < t.o_trow) return fail(RANKY_E_NOMEM, "workspace %zu < %zu", ws_bytes, t.o_trow);
    if (reinterpret_cast<uintptr_t>(workspace) % kWorkspaceAlign)
        return fail(RANKY_E_INVALID, "workspace is not %d-byte aligned", kWorkspaceAlign);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(workspace);
    auto i32 = [&](size_t o) { return reinterpret_cast<int32_t *>(w + o); };
    const CscView Av{A->nnz, A->colptr, A->rowidx, A->values, A->dtype};
    launch_validate_csc(Av, M, N, i32(t.o_status), s);
    int32_t bits = 0;
    HIP_TRY(hipMemcpyAsync(&bits, i32(t.o_status), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bits & kStCsc) return fail(RANKY_E_CSC, "CSC contract violated (colptr, row range or row order)");
    if (bits & kStNonfinite) return fail(RANKY_E_NONFINITE, "non-finite value in A");
    launch_transpose_csc(Av, M, N, i32(t.o_counts), i32(t.o_btot), colptr_t, i32(t.o_cursor), i32(t.o_long),
                         i32(t.o_nlong), rowidx_t, values_t, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return RANKY_OK;
}

size_t ranky_inc_workspace_bytes(int32_t M, int64_t max_cols, int64_t max_nnz, int32_t k, const ranky_opts *opts) {
    if (M < 1 || M > kMaxM || max_cols < 1 || max_nnz < 0 || k < 1 || k > M || max_cols > (int64_t)0x7ffffffe) return 0;
    const ranky_opts o = resolved(opts, false, k);
    return inc_layout(M, max_cols, max_nnz, k, o).total;
}

ranky_status ranky_inc_create(ranky_ctx *ctx, int32_t M, int32_t k, int64_t max_cols, int64_t max_nnz,
                              const ranky_opts *opts, void *workspace, size_t ws_bytes, ranky_inc **out,
                              ranky_stream_t stream) {
    if (!ctx || !out) return fail(RANKY_E_INVALID, "ctx or out is NULL");
    const ranky_opts o = resolved(opts, false, k);
    ranky_status st = check_opts(o);
    if (st) return st;
    const size_t need = ranky_inc_workspace_bytes(M, max_cols, max_nnz, k, &o);
    if (need == 0) return fail(RANKY_E_INVALID, "invalid sizes");
    if (!workspace || ws_bytes < need) return fail(RANKY_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % kWorkspaceAlign)
        return fail(RANKY_E_INVALID, "workspace is not %d-byte aligned", kWorkspaceAlign);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RANKY_E_DEVICE, "hipSetDevice");
    ranky_inc *inc = new ranky_inc();
    inc->ctx = ctx;
    inc->M = M;
    inc->k = k;
    inc->max_cols = max_cols;
    inc->max_nnz = max_nnz;
    inc->o = o;
    inc->L = inc_layout(M, max_cols, max_nnz, k, o);
    inc->ws = static_cast<char *>(workspace);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    launch_fill_f64(reinterpret_cast<double *>(inc->ws + inc->L.o_G), (int64_t)M * M, 0.0, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        delete inc;
        return fail(RANKY_E_DEVICE, "%s", hipGetErrorString(e));
    }
    *out = inc;
    return RANKY_OK;
}

ranky_status ranky_inc_append(ranky_inc *inc, const ranky_csc *block, int64_t cols, ranky_stream_t stream) {
    if (!inc) return fail(RANKY_E_INVALID, "inc is NULL");
    ranky_status st = check_csc_args(block, inc->M, cols);
    if (st) return st;
    if (cols > inc->max_cols || block->nnz > inc->max_nnz)
        return fail(RANKY_E_INVALID, "block of %lld columns / %lld entries beyond the state's %lld / %lld",
                    (long long)cols, (long long)block->nnz, (long long)inc->max_cols, (long long)inc->max_nnz);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const IncLayout &L = inc->L;
    StepCtx sc;
    Engine e;
    const int32_t D = default_blocks(cols);
    // the block's own Gram (Eq. 2 summand) on the step region, then added to the resident G in
    // the order the blocks arrive
    const Plan p = make_plan(inc->M, cols, block->nnz, 1, D, false, false, nullptr, true);
    if (L.hstep.total + p.total > L.hstep.total + L.step.total) return fail(RANKY_E_NOMEM, "step region too small");
    st = step_scan(sc, block, inc->M, cols, D, inc->ws + L.o_step, L.hstep.total + L.step.total, s, e, nullptr,
                   nullptr, nullptr, nullptr);
    if (st) return st;
    MatDesc &x = e.d[0];
    if (x.n > 0) {
        x.prec = RANKY_PREC_FP64;
        x.dwg = 0;
        x.gwaves = gram_waves(inc->M, 8, sc.c.lds_limit);
        e.nblk[kPhGram] = fill_wp(e.hwp(kPhGram), 1, [&](int) { return (int64_t)e.gsegs[0] + (x.npad - x.n); });
        e.nblk[kPhGramRed] = fill_wp(e.hwp(kPhGramRed), 1, [&](int) { return (int64_t)x.n; });
        st = e.upload_desc();
        if (!st) st = e.upload(e.h.o_wp, sizeof(int32_t) * (size_t)kPhCount * (e.h.slots + 1));
        if (st) return st;
        e.enqueue_transpose();
        int32_t gram_nw = 1;
        size_t gram_lds = 0;
        gram_shape(e.d, sc.c.lds_limit, gram_nw, gram_lds);
        launch_gram(e.ddesc(), e.dwp(kPhGram), e.nblk[kPhGram], e.dwp(kPhGramRed), e.nblk[kPhGramRed], 1, gram_nw,
                    gram_lds, x.hwg > 0, s);
        launch_scatter_add_gram(x.G, x.npad, x.m2r, inc->M, reinterpret_cast<double *>(inc->ws + L.o_G), s);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    inc->blocks += 1;
    inc->cols += cols;
    inc->nnz += block->nnz;
    return RANKY_OK;
}

ranky_status ranky_inc_solve(ranky_inc *inc, double tol, double *sigma, double *U, ranky_info *info,
                             ranky_stream_t stream) {
    if (!inc) return fail(RANKY_E_INVALID, "inc is NULL");
    if (!(tol >= 0.0)) return fail(RANKY_E_INVALID, "tol must be >= 0");
    if (!sigma || !U) return fail(RANKY_E_INVALID, "NULL output");
    ranky_ctx *ctx = inc->ctx;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RANKY_E_DEVICE, "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const IncLayout &L = inc->L;
    const int32_t M = inc->M, k = inc->k;
    char *base = inc->ws + L.o_solve + L.hsolve.total;
    MatDesc x = carve(L.solve, base, nullptr);
    const double *Gfull = reinterpret_cast<const double *>(inc->ws + L.o_G);
    // the rows with an entry so far, and G restricted to them
    launch_fill_i32(x.scal, kScCount, 0, s);
    launch_inc_rows(Gfull, M, x.m2r, x.r2m, x.empty, x.scal + kScNonempty, s);
    ranky_status st = ensure_pinned(ctx, 64);
    if (st) return st;
    HIP_TRY(hipMemcpyAsync(ctx->pinned, x.scal + kScNonempty, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int32_t n = *static_cast<int32_t *>(ctx->pinned);
    x.n = x.n_tau = x.neig = n;
    x.npad = jacobi_npad(n > 0 ? n : 1);
    launch_inc_gather(Gfull, M, x.r2m, x.scal + kScNonempty, x.npad, x.G, s);
    x.M = M;
    x.k = k;
    x.D = 0;
    x.prec = RANKY_PREC_FP64;
    x.tol = tol;
    x.u_gram = std::ldexp(1.0, -53);
    x.jtol = 0.0;
    x.sigma = sigma;
    x.U = U;
    x.V = nullptr;
    Engine e;
    st = make_engine(ctx, s, L.hsolve, inc->ws + L.o_solve, 1, e);
    if (st) return st;
    e.d.assign(1, x);
    e.sweeps_cap = inc->o.max_sweeps;
    e.maxn = n > 0 ? n : 1;
    st = e.plan_rest();
    if (st) return st;
    // the leading pairs: the subspace iteration from the previous solve's Ritz vectors when it
    // applies (the appended blocks move the leading subspace a little), else the full Jacobi
    int32_t iters = 0;
    double flops = 0.0;
    const int32_t p = L.p;
    if (p > 0 && n > 0 && (inc->o.eigensolver == 2 ? 2 * p : 8 * p) <= n) {
        double *start = nullptr;
        if (inc->has_prev) {
            start = reinterpret_cast<double *>(inc->ws + L.o_start);
            launch_inc_start(reinterpret_cast<const double *>(inc->ws + L.o_keep), x.r2m, n, L.solve.topk.rows, p,
                             start, s);
        }
        st = topk_eigensolve(ctx, e, L.solve, base, std::sqrt((double)n) * std::ldexp(1.0, -52),
                             inc->o.max_iters > 0 ? inc->o.max_iters : kTopkDefaultIters, s, &iters, &flops, start);
        if (st) return st;
        if (iters > 0) {
            launch_inc_keep(e.d[0].W, e.d[0].npad, e.d[0].m2r, M, p, reinterpret_cast<double *>(inc->ws + L.o_keep), s);
            inc->has_prev = true;
        } else {
            st = e.plan_rest();
            if (st) return st;
        }
    }
    if (iters == 0) {
        st = e.eigensolve(false);
        if (st) return st;
    }
    launch_select(e.ddesc(), 1, e.maxn, s);
    launch_gather_u(e.ddesc(), e.dwp(kPhGather), e.nblk[kPhGather], 1, s);
    HIP_TRY(hipGetLastError());
    std::vector<int32_t> iv;
    std::vector<double> fv;
    st = e.collect(iv, fv);
    if (st) return st;
    const bool notconv = iters == 0 && n > 0 && e.notconv[0] != 0;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->status = notconv ? RANKY_E_NOT_CONVERGED : RANKY_OK;
        info->rank = iv[2];
        info->n_nonempty = n;
        info->empty_rows = M - n;
        info->sweeps = iters == 0 && n > 0 ? e.sweeps[0] : 0;
        info->n_blocks = (int32_t)std::min<int64_t>(inc->blocks, 0x7fffffff);
        info->tau = fv[0];
        info->sigma_max = fv[1];
        info->eig_iters = iters;
        info->eig_flops = flops;
    }
    if (notconv) return fail(RANKY_E_NOT_CONVERGED, "Jacobi did not converge in %d sweeps", inc->o.max_sweeps);
    return RANKY_OK;
}

ranky_status ranky_inc_destroy(ranky_inc *inc) {
    delete inc;
    return RANKY_OK;
}

size_t ranky_paper_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t k, int32_t D, int32_t checker) {
    if (M < 1 || N < 1 || M > kMaxM || nnz < 0 || D < 1 || D > N || k < 1 || k > M || checker < -1 || checker > 2)
        return 0;
    return paper_plan(M, N, nnz, k, D, checker >= 0).total;
}

ranky_status ranky_svd_paper(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, int32_t D,
                             int32_t checker, uint64_t seed, double tol, void *workspace, size_t ws_bytes,
                             double *sigma, double *U, ranky_paper_info *pinfo, ranky_stream_t stream) {
    if (!ctx) return fail(RANKY_E_INVALID, "ctx is NULL");
    if (!(tol >= 0.0)) return fail(RANKY_E_INVALID, "tol must be >= 0");
    if (!sigma || !U) return fail(RANKY_E_INVALID, "NULL output");
    if (k < 1 || k > M) return fail(RANKY_E_INVALID, "k=%d must be in [1, M=%d]", k, M);
    ranky_status st = checker >= 0 ? check_checker_args(A, M, N, D, checker) : check_csc_args(A, M, N);
    if (st) return st;
    if (D < 1 || D > N) return fail(RANKY_E_INVALID, "D=%d outside [1, N]", D);
    const PaperPlan pp = paper_plan(M, N, A->nnz, k, D, checker >= 0);
    if (!workspace || ws_bytes < pp.total) return fail(RANKY_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, pp.total);
    if (reinterpret_cast<uintptr_t>(workspace) % kWorkspaceAlign)
        return fail(RANKY_E_INVALID, "workspace is not %d-byte aligned", kWorkspaceAlign);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(RANKY_E_DEVICE, "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(workspace);
    auto i32 = [&](size_t o) { return reinterpret_cast<int32_t *>(w + o); };
    auto f64 = [&](size_t o) { return reinterpret_cast<double *>(w + o); };
    if (pinfo) std::memset(pinfo, 0, sizeof(*pinfo));
    hipEvent_t *ev = ctx->ev;
    HIP_TRY(hipEventRecord(ev[0], s));
    // 1. A' (Alg. 2-4) or A itself
    ranky_csc A1 = *A;
    int64_t added = 0;
    if (checker >= 0) {
        StepCtx sc;
        st = run_checker(sc, A, M, N, D, checker, seed, i32(pp.o_cp), i32(pp.o_ri), f64(pp.o_va), w + pp.o_chk, s, &added);
        if (st) return st;
        A1.nnz = A->nnz + added;
        A1.colptr = i32(pp.o_cp);
        A1.rowidx = i32(pp.o_ri);
        A1.values = f64(pp.o_va);
        A1.dtype = RANKY_F64;
    } else if (A->dtype != RANKY_F64) {
        return fail(RANKY_E_INVALID, "without a checker the paper's route takes FP64 values");
    }
    HIP_TRY(hipEventRecord(ev[1], s));
    // 2. the scan of A' (validation, non-empty rows: the compaction of P P^T)
    StepCtx sc2;
    Engine es;
    st = step_scan(sc2, &A1, M, N, D, w + pp.o_scan, pp.hscan.total + pp.scan.total, s, es, nullptr, nullptr, nullptr,
                   nullptr);
    if (st) return st;
    const MatDesc xs = es.d[0];
    const int32_t n = xs.n;
    // 3. every block's reduced factors (Eq. 1): the D blocks as a batch, V not formed
    launch_block_slices(A1.colptr, N, D, i32(pp.o_slices), s);
    std::vector<int32_t> bcol(D + 1);
    {
        st = ensure_pinned(ctx, sizeof(int32_t) * ((size_t)D + 1));
        if (st) return st;
        int32_t *hp = static_cast<int32_t *>(ctx->pinned);
        for (int32_t b = 0; b <= D; ++b)
            HIP_TRY(hipMemcpyAsync(hp + b, A1.colptr + ((int64_t)b * N) / D, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int32_t b = 0; b <= D; ++b) bcol[b] = hp[b];
    }
    std::vector<int64_t> bnnz(D);
    for (int32_t b = 0; b < D; ++b) bnnz[b] = bcol[b + 1] - bcol[b];
    std::vector<Job> jobs = paper_block_jobs(M, N, D, bnnz);
    for (int32_t b = 0; b < D; ++b) {
        const int64_t c0 = ((int64_t)b * N) / D;
        jobs[b].A.colptr = i32(pp.o_slices) + c0 + b;
        jobs[b].A.rowidx = A1.rowidx + bcol[b];
        jobs[b].A.values = static_cast<const double *>(A1.values) + bcol[b];
        jobs[b].sigma = f64(pp.o_bsig) + (size_t)b * M;
        jobs[b].U = f64(pp.o_bU) + (size_t)b * M * M;
        jobs[b].V = nullptr;
    }
    std::vector<ranky_info> binfo(D);
    st = run_path(ctx, jobs, 0.0, paper_block_opts(), w + pp.o_batch, pp.batch, binfo.data(), s, false);
    if (st) return st;
    HIP_TRY(hipEventRecord(ev[2], s));
    // 4. the proxy P = [U^1 S^1 | ... | U^D S^D] over the retained triplets, as rows of P^T
    const int32_t np = pp.np;
    int64_t R = 0;
    for (int32_t b = 0; b < D; ++b) R += binfo[b].rank;
    const int64_t Rpad = std::max<int64_t>(16, ((R + 15) / 16) * 16);   // R <= D M: within the Pt rows
    launch_fill_f64(f64(pp.o_Pt), Rpad * np, 0.0, s);
    for (int32_t b = 0, off = 0; b < D; off += binfo[b].rank, ++b)
        launch_proxy_rows(f64(pp.o_bU) + (size_t)b * M * M, f64(pp.o_bsig) + (size_t)b * M, M, binfo[b].rank, xs.m2r,
                          f64(pp.o_Pt) + (size_t)off * np, np, s);
    // 5. P P^T (Eq. 3) on the FP64 matrix cores, the k splits added in order
    {
        int32_t splits, klen;
        topk_split((int64_t)(np / kTopkTile) * (np / kTopkTile), (int32_t)Rpad, splits, klen);
        splits = std::min(splits, pp.part_splits);
        klen = (int32_t)((((Rpad + splits - 1) / splits) + 15) / 16 * 16);
        splits = (int32_t)((Rpad + klen - 1) / klen);
        launch_tk_gemm(true, f64(pp.o_Pt), np, f64(pp.o_Pt), np, f64(pp.o_part), np, np, (int32_t)Rpad, splits, klen,
                       np, (int32_t)Rpad, s);
        launch_tk_combine(f64(pp.o_part), splits, (int64_t)np * np, 1.0, 0.0, nullptr, 0.0, nullptr, f64(pp.o_Gp), s);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipEventRecord(ev[3], s));
    // 6. the SVD of P by the eigenpairs of P P^T (the last step of Alg. 1), threshold, signs
    int32_t rank = 0;
    double tau = 0.0;
    if (n > 0) {
        const Header hj = make_header(1, 1, np / kJacobiBlock);
        Engine ej;
        st = make_engine(ctx, s, hj, w + pp.o_jhdr, 1, ej);
        if (st) return st;
        MatDesc jd = xs;
        jd.scal = i32(pp.o_jscal);
        jd.sdbl = f64(pp.o_jsdbl);
        jd.jstate = i32(pp.o_jstate);
        jd.G = f64(pp.o_Gp);
        jd.G2 = f64(pp.o_jG2);
        jd.W = f64(pp.o_jW);
        jd.J = f64(pp.o_jJ);
        jd.S = f64(pp.o_jS);
        jd.jflag = i32(pp.o_jflag);
        jd.lam = f64(pp.o_jlam);
        jd.perm = i32(pp.o_jperm);
        jd.npad = np;
        jd.n = n;
        jd.neig = n;
        jd.n_tau = n;
        jd.k = k;
        jd.tol = tol;
        jd.u_gram = std::ldexp(1.0, -53);
        jd.jtol = 0.0;
        jd.dwg = 0;
        jd.jsched = 0;
        jd.sigma = sigma;
        jd.U = U;
        jd.Uf = nullptr;
        jd.V = nullptr;
        ej.d.assign(1, jd);
        ej.sweeps_cap = kDefaultSweeps;
        ej.maxn = n;
        ej.status.assign(1, RANKY_OK);
        st = ej.plan_rest();
        if (st) return st;
        launch_fill_i32(jd.scal, kScCount, 0, s);
        st = ej.eigensolve(false);
        if (st) return st;
        if (ej.notconv[0]) return fail(RANKY_E_NOT_CONVERGED, "Jacobi on P P^T did not converge");
        launch_select(ej.ddesc(), 1, n, s);
        launch_gather_u(ej.ddesc(), ej.dwp(kPhGather), ej.nblk[kPhGather], 1, s);
        HIP_TRY(hipGetLastError());
        std::vector<int32_t> iv;
        std::vector<double> fv;
        st = ej.collect(iv, fv);
        if (st) return st;
        rank = iv[2];
        tau = fv[0];
    } else {
        launch_fill_f64(sigma, k, 0.0, s);
        launch_fill_f64(U, (int64_t)M * k, 0.0, s);
    }
    HIP_TRY(hipEventRecord(ev[4], s));
    HIP_TRY(hipStreamSynchronize(s));
    if (pinfo) {
        pinfo->added = added;
        pinfo->nnz_repaired = A1.nnz;
        pinfo->proxy_cols = R;
        pinfo->rank = rank;
        pinfo->n_nonempty = n;
        pinfo->tau = tau;
        for (int q = 0; q < 4; ++q) hipEventElapsedTime(&pinfo->ms[q], ev[q], ev[q + 1]);
    }
    return RANKY_OK;
}

ranky_status ranky_paper_errors(int32_t M, int32_t k, const double *sigma_hat, const double *U_hat, const double *sigma,
                                const double *U, double *e_sigma, double *e_u, void *workspace, size_t ws_bytes,
                                ranky_stream_t stream) {
    if (M < 1 || k < 1 || k > M || !sigma_hat || !U_hat || !sigma || !U || !e_sigma || !e_u)
        return fail(RANKY_E_INVALID, "bad arguments");
    const size_t need = sizeof(double) * ((size_t)k + 2);
    if (!workspace || ws_bytes < need) return fail(RANKY_E_NOMEM, "workspace %zu < %zu", ws_bytes, need);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double *col = static_cast<double *>(workspace);
    launch_paper_errors(sigma_hat, U_hat, sigma, U, M, k, col, col + k, s);
    HIP_TRY(hipGetLastError());
    double out[2] = {0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(out, col + k, sizeof(out), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *e_sigma = out[0];
    *e_u = out[1];
    return RANKY_OK;
}

size_t ranky_checker_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t D) {
    if (M < 1 || N < 1 || M > kMaxM || nnz < 0 || D < 1 || D > N) return 0;
    return checker_plan(M, N, nnz, D).total;
}

ranky_status ranky_checker(const ranky_csc *A, int32_t M, int64_t N, int32_t D, int32_t kind, uint64_t seed,
                           int32_t *colptr_out, int32_t *rowidx_out, double *values_out, int64_t capacity,
                           int64_t *nnz_out, int64_t *added, void *workspace, size_t ws_bytes, ranky_stream_t stream) {
    ranky_status st = check_checker_args(A, M, N, D, kind);
    if (st) return st;
    if (!colptr_out || !rowidx_out || !values_out || !nnz_out || !added) return fail(RANKY_E_INVALID, "NULL output");
    if (capacity < A->nnz + 2 * (int64_t)D * M)
        return fail(RANKY_E_INVALID, "capacity %lld < nnz + 2 D M = %lld", (long long)capacity,
                    (long long)(A->nnz + 2 * (int64_t)D * M));
    const size_t need = ranky_checker_workspace_bytes(M, N, A->nnz, D);
    if (!workspace || ws_bytes < need) return fail(RANKY_E_NOMEM, "workspace %zu < %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) % kWorkspaceAlign)
        return fail(RANKY_E_INVALID, "workspace is not %d-byte aligned", kWorkspaceAlign);
    StepCtx sc;
    int64_t add = 0;
    st = run_checker(sc, A, M, N, D, kind, seed, colptr_out, rowidx_out, values_out, static_cast<char *>(workspace),
                     reinterpret_cast<hipStream_t>(stream), &add);
    if (st) return st;
    *added = add;
    *nnz_out = A->nnz + add;
    return RANKY_OK;
}

ranky_status ranky_svd_tall(ranky_ctx *ctx, const ranky_csc *A, int64_t M, int32_t N, int32_t k, double tol,
                            const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, void *U, double *V,
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
    ranky_status st = check_tall_args(A, M, N, k);
    if (st) return finish(st);
    const ranky_opts o = resolved(opts, true, k);
    st = check_opts(o);
    if (st) return finish(st);
    if (o.block_start) return finish(fail(RANKY_E_INVALID, "block_start is for ranky_svd"));
    if (o.refine && k > kMaxRefineK) return finish(fail(RANKY_E_INVALID, "refine needs k <= %d", kMaxRefineK));
    const TallPlan t = tall_plan(M, A->nnz);
    const size_t need = ranky_tall_workspace_bytes(M, N, A->nnz, k, &o);
    if (need == 0) return finish(fail(RANKY_E_INVALID, "invalid sizes"));
    if (!workspace || ws_bytes < need) return finish(fail(RANKY_E_NOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need));
    if (reinterpret_cast<uintptr_t>(workspace) % kWorkspaceAlign)
        return finish(fail(RANKY_E_INVALID, "workspace is not %d-byte aligned", kWorkspaceAlign));
    if (hipSetDevice(ctx->device) != hipSuccess) return finish(fail(RANKY_E_DEVICE, "hipSetDevice"));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(workspace);
    auto i32 = [&](size_t off) { return reinterpret_cast<int32_t *>(w + off); };
    const CscView Av{A->nnz, A->colptr, A->rowidx, A->values, A->dtype};
    // the contract of A (any row count), then A^T = the CSR of A
    if (o.validate) {
        st = ensure_pinned(ctx, 64);
        if (st) return finish(st);
        launch_validate_csc(Av, M, N, i32(t.o_status), s);
        int32_t *bits = static_cast<int32_t *>(ctx->pinned);
        HIP_TRY(hipMemcpyAsync(bits, i32(t.o_status), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (*bits & kStCsc) return finish(fail(RANKY_E_CSC, "CSC contract violated (colptr, row range or row order)"));
        if (*bits & kStNonfinite) return finish(fail(RANKY_E_NONFINITE, "non-finite value in A"));
    }
    launch_transpose_csc(Av, M, N, i32(t.o_counts), i32(t.o_btot), i32(t.o_ptr), i32(t.o_cursor), i32(t.o_long),
                         i32(t.o_nlong), i32(t.o_trow), w + t.o_tval, s);
    HIP_TRY(hipGetLastError());
    // the short-and-fat path on A^T (N x M): its column blocks are A's row blocks; its left
    // vectors (N x k, FP64) are A's right vectors V, its right vectors (M x k) A's left vectors U
    ranky_csc At;
    At.nnz = A->nnz;
    At.colptr = i32(t.o_ptr);
    At.rowidx = i32(t.o_trow);
    At.values = w + t.o_tval;
    At.dtype = A->dtype;
    Job j;
    ranky_opts ot = o;
    ot.validate = 0;   // A^T is well formed by construction (A was checked, or the caller vouches for it)
    st = make_job(&At, N, M, k, ot.n_blocks, sigma, V, U, &j);
    if (st) return finish(st);
    return finish(run_path(ctx, {j}, tol, ot, w + t.o_path, ws_bytes - t.o_path, inf, s, ot.graph == 1));
}

}  // extern "C"

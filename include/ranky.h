/*
 * ranky.h -- C-ABI of the MI355X-native rank-safe column-block SVD of a
 * short-and-fat sparse matrix (Tugay & Gunduz Oguducu, "Ranky: An Approach to
 * Solve Distributed SVD on Large Sparse Matrices", arXiv 2009.09767).
 *
 * The method (Sec. III): split A (M x N, N >> M) column-wise into D blocks
 * A = [A^1 | ... | A^D]; each block has a reduced SVD A^i = U^i S^i V^i^T (Eq. 1);
 * the proxy matrix P = [U^1 S^1 | ... | U^D S^D] has the same singular values and
 * left singular vectors as A because A A^T = sum_i U^i S^i S^i^T U^i^T = P P^T
 * (Eq. 2, Eq. 3).  This library evaluates that merge in Gram form:
 * G = sum_i A^i A^i^T (which is P P^T), an FP64 eigensolve of G gives Sigma^2 and U,
 * and the right vectors come from the back-projection V = A^T U Sigma^{-1}, which
 * the paper leaves as future work (Sec. V).  Blocks whose rank falls below M need
 * no repair: an empty row inside a block only drops a zero singular value from
 * that block's factor, which adds nothing to P P^T.  No entry of A is altered and
 * no vanishing sigma is ever divided by (see the rank rule under ranky_svd).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - Matrices are dense row-major unless stated; "M x k row-major" means element
 *     (m, i) at index m * k + i.
 *   - The caller owns every buffer (inputs, outputs, workspace); the library never
 *     frees caller memory and never allocates device memory inside these calls.
 *   - A workspace must start on a 256-byte boundary (hipMalloc and torch
 *     allocations do); RANKY_E_INVALID otherwise.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the legacy default
 *     stream).  Calls documented as "blocking" synchronise that stream before
 *     returning; the others are stream-ordered and return after enqueueing.
 *   - Errors are status codes; nothing throws across the ABI.  On an error the
 *     outputs are undefined.  ranky_last_error() returns a thread-local message.
 *   - Results are bitwise deterministic: every floating-point reduction runs in
 *     a fixed order, so the same inputs give the same bits on every run.  There is
 *     no non-deterministic mode to opt into (no floating-point atomics anywhere), so
 *     there is no option for it.
 */
#ifndef RANKY_H
#define RANKY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same type as hipStream_t (declared here so that callers need no HIP header). */
typedef struct ihipStream_t *ranky_stream_t;

typedef enum {
    RANKY_OK = 0,
    RANKY_E_INVALID = 1,       /* a size, pointer or option is out of range (host-checked) */
    RANKY_E_CSC = 2,           /* colptr not monotone / not spanning [0, nnz], row index out of
                                  range, or rows not strictly increasing inside a column (device-checked) */
    RANKY_E_NONFINITE = 3,     /* a value is NaN or +-Inf (device-checked; E_CSC takes precedence) */
    RANKY_E_NOMEM = 4,         /* the workspace is smaller than ranky_workspace_bytes() */
    RANKY_E_DEVICE = 5,        /* a HIP runtime call failed */
    RANKY_E_BUSY = 6,          /* serving: no slot or memory free (back-pressure) */
    RANKY_E_CANCELLED = 7,     /* serving: the request was cancelled */
    RANKY_E_NOT_CONVERGED = 8, /* the Jacobi eigensolver hit max_sweeps */
    RANKY_PENDING = 9          /* serving: the request has not finished */
} ranky_status;

typedef enum { RANKY_F32 = 0, RANKY_F64 = 1 } ranky_dtype;

/* Precision of the Gram accumulation (step 2 of the path).  The eigensolve, the
 * rank decision and the Rayleigh-Ritz refinement are FP64 in every mode.
 * For a single matrix the Gram block of its densest rows (up to 32 rows with at least
 * max(4096, N/64) nonzeros each) is computed as dense tiles on the matrix cores in the
 * mode's precision; every other pair of rows goes through the sparse pass. */
typedef enum {
    RANKY_PREC_FP64 = 0,  /* products and sums in FP64 (FP32 inputs are promoted exactly) */
    RANKY_PREC_FP32 = 1,  /* products and sums in FP32, merged into the FP64 Gram per row */
    RANKY_PREC_BF16X3 = 2 /* as FP32, with the dense tiles as split-bf16 products
                             hi*hi + hi*lo + lo*hi (x = hi + lo, FP32 accumulation, FP64
                             across 64-column steps): relative product error ~2^-16, so
                             the refinement step is what brings sigma back */
} ranky_prec;

/* Compressed sparse columns.  colptr[0] = 0, colptr non-decreasing,
 * colptr[N] = nnz; rowidx strictly increasing inside a column, in [0, M);
 * values finite.  int32 indices (nnz <= 2^31 - 1). */
typedef struct {
    int64_t nnz;
    const int32_t *colptr; /* device, N + 1 */
    const int32_t *rowidx; /* device, nnz */
    const void *values;    /* device, nnz elements of `dtype` */
    int32_t dtype;         /* ranky_dtype */
} ranky_csc;

typedef struct {
    int32_t n_blocks;   /* D; block b = columns [floor(b N / D), floor((b+1) N / D)).
                           0 selects ceil(N / 16384).  1 <= D <= N. */
    int32_t gram_prec;  /* ranky_prec (default FP64) */
    int32_t refine;     /* Rayleigh-Ritz steps after the eigensolve: 0, 1, or -1 = automatic
                           (the default): 1 when gram_prec != FP64 and the call refines (ranky_svd,
                           ranky_svd_async, ranky_autotune, serving; k <= 1024), else 0 */
    int32_t max_sweeps; /* Jacobi sweep cap (0 = 40) */
    int32_t validate;   /* 1 = check the CSC contract and finiteness on the device (default 1) */
    int32_t v_dtype;    /* ranky_dtype of the output V (default F64) */
    int32_t timing;     /* 1 = fill ranky_info.ms with per-phase times (adds event records) */
    int32_t graph;      /* 1 = replay the Jacobi sweep as a captured HIP graph (ranky_svd and
                           ranky_batch; needs a non-NULL stream, ignored on the NULL stream) */
    int32_t eigensolver; /* how the k leading eigenpairs of G are found (the proxy SVD needs only
                           those): 0 = automatic (the default), 1 = the full two-sided Jacobi,
                           2 = Chebyshev-filtered subspace iteration whenever its block of
                           p = k + max(k/2, 32) rounded up to 64 vectors is at most M'/2 (and 256).
                           Automatic takes the subspace iteration for a single matrix when p is at
                           most M'/8, the full Jacobi otherwise (always in ranky_batch).  A subspace
                           iteration that has not converged after max_iters falls back to the full
                           Jacobi; ranky_info.eig_iters tells which ran. */
    int32_t max_iters;  /* cap on the subspace iterations (0 = 60) */
    int32_t gram_split; /* heavy-row split of the Gram (Eq. 2 summed in three parts: the densest
                           rows' block on the FP64 matrix cores, their pairs with the other rows
                           from one gathered row per nonzero, the other pairs in the sparse walk):
                           0 = automatic (the default: a single matrix of at least 2^22 nonzeros
                           with an FP64 or FP32 Gram), 1 = off, 2 = on for a single matrix with an
                           FP64 or FP32 Gram.  Changes the order of the sums (not the result beyond
                           rounding); costs N x 32 x 8 bytes of workspace. */
    const int64_t *block_start; /* host, optional: D + 1 column boundaries, block b = columns
                           [block_start[b], block_start[b+1]); block_start[0] = 0, non-decreasing,
                           block_start[D] = N, with n_blocks = D >= 1 given (E_INVALID otherwise).
                           NULL = floor(bN/D).  Read during the call (ranky_svd_async: until the
                           query answers); ranky_svd, ranky_svd_async and ranky_autotune only
                           (E_INVALID in ranky_batch and serving, whose matrices differ in N) */
} ranky_opts;

typedef struct {
    int32_t status;        /* ranky_status of the call */
    int32_t rank;          /* r = #{sigma_i > tau}, at most k */
    int32_t n_nonempty;    /* M' = rows with at least one nonzero */
    int32_t empty_rows;    /* |E| = M - M' */
    int32_t sweeps;        /* Jacobi sweeps of the eigensolve of G */
    int32_t n_blocks;      /* D actually used */
    int32_t lonely_max;    /* largest number of rows empty inside one block (Alg. 1 scan) */
    int32_t lonely_blocks; /* number of blocks with at least one empty row */
    double tau;            /* effective threshold tau */
    double sigma_max;      /* sigma_1 */
    float ms[8];           /* with opts.timing: [0] occupancy+plan, [1] transpose, [2] Gram,
                              [3] eigensolve, [4] select, [5] refine, [6] back-projection, [7] total */
    float round_ms;        /* with opts.timing (ranky_svd): summed span of the Jacobi round launches of
                              the sweeps that did work (HIP events on the call's stream; the sweep is
                              launched directly, not replayed, in timing mode) */
    int32_t round_launches; /* number of round launches inside round_ms */
    int32_t rr_sweeps;     /* Jacobi sweeps of the Rayleigh-Ritz eigensolve of H (0 without refinement) */
    int32_t eig_iters;     /* subspace iterations of the eigensolve of G (0: the full Jacobi ran, and
                              sweeps counts its sweeps) */
    double eig_flops;      /* algorithmic FP64 flops of the subspace iteration's matrix products
                              (2 x rows x columns x inner length over the unpadded sizes; 0 for the Jacobi) */
    /* Alg. 1 scan of every block, host copies of D entries each (NULL when the call failed before
     * the scan): rows with no entry inside block b (lonely rows), and rows with exactly one entry
     * (NO of Eq. 4).  The memory belongs to the library: it stays valid until the next call on the
     * same context (ranky_svd, ranky_batch, ranky_autotune), and for a served request until
     * ranky_serve_destroy. */
    const int32_t *lonely_per_block;
    const int32_t *single_per_block;
    int32_t topk_block;    /* block width p of the subspace iteration (0 when the full Jacobi ran) */
    int32_t heavy_rows;    /* dense rows the Gram took out of the sparse walk (opts.gram_split;
                              0 when the split was off or found no dense row) */
} ranky_info;

typedef struct ranky_ctx ranky_ctx;

/* ------------------------------------------------------------------------- */
/* Context                                                                    */
/* ------------------------------------------------------------------------- */

/* Binds the calling thread's work to `device` and caches its properties.
 * *out receives a handle owned by the caller (ranky_ctx_destroy).  Returns
 * E_INVALID for a bad device, E_DEVICE if HIP fails. */
ranky_status ranky_ctx_create(int device, ranky_ctx **out);
ranky_status ranky_ctx_destroy(ranky_ctx *ctx);

/* Fills *opts (host) with the defaults listed in ranky_opts. */
ranky_status ranky_default_opts(ranky_opts *opts);

/* Thread-local text of the last error (never NULL). */
const char *ranky_last_error(void);
const char *ranky_version(void);

/* ------------------------------------------------------------------------- */
/* The whole path                                                             */
/* ------------------------------------------------------------------------- */

/* Bytes of device workspace ranky_svd needs for these sizes and options
 * (0 if they are invalid).  Depends on M, N, nnz, k and opts only. */
size_t ranky_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t k, const ranky_opts *opts);

/* Top-k singular triplets of A (M x N) by the block merge of Sec. III in Gram
 * form (Eq. 2-3), with the right vectors back-projected.  Blocking.
 *
 * Steps (all on the device): the Alg. 1 scan of every block (per-block row
 * occupancy: lonely rows are counted, not repaired); the block Grams
 * A^i A^i^T reduced in block order into G restricted to the M' non-empty rows;
 * a two-sided Jacobi FP64 eigensolve of G (the SVD of the proxy P, Sec. III);
 * the rank-safe threshold; with gram_prec != FP64 and refine = 1 one FP64
 * Rayleigh-Ritz step with the exact operator; V = A^T U Sigma^{-1}.
 *
 * Rank rule: sigma_i = sqrt(max(lambda_i, 0)); sigma_i counts as zero iff
 * sigma_i <= tau = max(tol, sqrt(M' u_G)) sigma_1, u_G = the unit roundoff of what was
 * accumulated: 2^-53 for the FP64 Gram and after the FP64 Rayleigh-Ritz step, 2^-24 for
 * the FP32 Gram, 2^-16 for a BF16X3 Gram whose split-bf16 tiles ran (at least two dense
 * rows; otherwise it is an FP32 Gram).  rank = #{sigma_i > tau}.
 *
 * Outputs (device, caller-allocated):
 *   sigma [k]            descending; sigma_i = 0 exactly for i >= rank
 *   U     [M x k]        row-major; column i < min(k, M') is the eigenvector of
 *                        G scattered to the non-empty rows (zero on empty rows),
 *                        sign fixed so its entry of largest magnitude is positive
 *                        (lowest row on an exact tie); columns i >= M' are e_row for
 *                        the empty rows in ascending row order
 *   V     [N x k]        row-major, v_dtype; V[:, i] = A^T u_i / sigma_i for i < rank,
 *                        exactly 0 for i >= rank (no division by a vanishing sigma).
 *                        An F32 V is formed from U rounded to FP32 (a copy kept in
 *                        the workspace), with FP64 products and sums and one
 *                        rounding at the store; an F64 V from the FP64 U
 *   info  (host, may be NULL)
 * Errors: E_INVALID (M < 1, N < 1, k < 1 or k > M, tol < 0 or NaN, nnz outside
 * [0, 2^31), D outside [1, N], M > 8192, a NULL pointer), E_NOMEM (ws_bytes too
 * small), E_CSC / E_NONFINITE (device validation), E_NOT_CONVERGED, E_DEVICE. */
ranky_status ranky_svd(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, double tol,
                       const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, double *U,
                       void *V, ranky_info *info, ranky_stream_t stream);

/* Non-blocking ranky_svd: validates the arguments like ranky_svd (its host-checkable
 * errors are returned here, at once), starts the same computation on a worker thread
 * of the context and returns RANKY_OK with *ticket (host) set.  A, opts (copied), the
 * workspace and the outputs must stay valid, and the context unused by other calls,
 * until ranky_query has returned a status other than RANKY_PENDING for the ticket.
 * At most one call is in flight per context: E_BUSY otherwise.  The result is the
 * result of ranky_svd on the same arguments, bit for bit. */
ranky_status ranky_svd_async(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, double tol,
                             const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, double *U,
                             void *V, ranky_stream_t stream, uint64_t *ticket);

/* State of an asynchronous call: RANKY_PENDING while it runs; then, once, the status
 * ranky_svd returned, with *info (host, may be NULL) filled and ranky_last_error() set
 * on an error.  The ticket is released by that answer: E_INVALID for a ticket that is
 * unknown, superseded or already answered.  Non-blocking. */
ranky_status ranky_query(ranky_ctx *ctx, uint64_t ticket, ranky_info *info);

/* ------------------------------------------------------------------------- */
/* Autotuner                                                                  */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t bp_per_cu;              /* chosen back-projection workgroups per CU (0: not timed,
                                       the refinement path computes V itself) */
    int32_t jacobi_schedule;        /* chosen Jacobi round launch shape, bit 0: update tiles grouped
                                       per XCD (else linear), bit 1: one round workgroup per CU */
    int32_t bp_candidates[4];       /* workgroups per CU tried ... */
    float bp_ms[4];                 /* ... and the best back-projection time of each (ms) */
    int32_t schedule_candidates[4]; /* schedules tried ... */
    float eig_ms[4];                /* ... and the best eigensolve time of each (ms) */
} ranky_tune_report;

/* Picks the launch shapes of this problem shape by measurement and stores them in the
 * context: later ranky_svd / ranky_batch calls on the same context with the same
 * (M, N, nnz, k, value dtype, opts->v_dtype, opts->gram_prec) use them.  Candidates:
 * back-projection workgroups per CU {16, 32, 64, 128} and the Jacobi round launch shape
 * {0..3}: bit 0 groups the update tiles per XCD (the tiles that share a rotation J run on
 * one XCD's L2), bit 1 gives every round workgroup a CU of its own (extra LDS), so no update
 * workgroup shares a CU with a subproblem sweep, the round's critical path.
 * Neither changes any result (each V column and each tile is computed the same way
 * whatever the launch shape), only the time.  Runs the whole path on A about a dozen
 * times with phase timing (HIP events on `stream`), so it belongs before a timed region,
 * not inside one.  Arguments and errors as ranky_svd (the outputs hold the last run's
 * result); report (host) may be NULL.  Blocking; the context must not be in use by
 * another thread. */
ranky_status ranky_autotune(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k,
                            const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, double *U, void *V,
                            ranky_tune_report *report, ranky_stream_t stream);

/* Stores launch shapes for a problem shape without measuring (a configuration kept
 * from an earlier ranky_autotune, or a fixed choice).  Same key as ranky_autotune.
 * E_INVALID for bp_per_cu outside [1, 1024] or a schedule outside [0, 3].  In a batch, bit 1
 * applies only when every matrix of the call has it. */
ranky_status ranky_tune_set(ranky_ctx *ctx, int32_t M, int64_t N, int64_t nnz, int32_t k, ranky_dtype dtype,
                            const ranky_opts *opts, int32_t bp_per_cu, int32_t jacobi_schedule);

/* ------------------------------------------------------------------------- */
/* Batches of independent matrices                                            */
/* ------------------------------------------------------------------------- */

/* One matrix of a batch: its CSC, sizes and caller-allocated outputs (device),
 * laid out exactly as for ranky_svd. */
typedef struct {
    ranky_csc A;
    int64_t N;
    int32_t M;
    int32_t k;        /* 1 <= k <= M */
    int32_t n_blocks; /* D for this matrix; 0 selects ceil(N / 16384) */
    int32_t pad;      /* alignment padding, ignored */
    double *sigma;    /* [k] */
    double *U;        /* [M x k] row-major */
    void *V;          /* [N x k] row-major, opts->v_dtype */
} ranky_batch_item;

/* Bytes of workspace ranky_batch needs (0 if an item is invalid).  items: host. */
size_t ranky_batch_workspace_bytes(int32_t count, const ranky_batch_item *items, const ranky_opts *opts);

/* The whole path of ranky_svd for `count` independent matrices of different sizes,
 * run together: every phase is one launch whose workgroups are spread over all
 * matrices (a per-matrix descriptor table maps workgroups to matrices), and the
 * Jacobi sweeps of all matrices advance in lock-step, each matrix dropping out when
 * its own convergence test passes.  With opts->graph = 1 the sweep is captured
 * once as a HIP graph and replayed.  Blocking.
 *   items [count] host; infos [count] host (may be NULL): per-matrix ranky_info.
 * The return value is RANKY_OK only if every matrix succeeded; a matrix whose CSC
 * breaks the contract gets its own status in infos[i].status and does not stop the
 * others.  opts->refine must be 0 or -1 (Rayleigh-Ritz is per matrix: use ranky_svd); the
 * split-bf16 tiles are a single-matrix step, so BF16X3 runs as FP32 here and the threshold
 * uses the FP32 Gram's u_G = 2^-24. */
ranky_status ranky_batch(ranky_ctx *ctx, int32_t count, const ranky_batch_item *items, double tol,
                         const ranky_opts *opts, void *workspace, size_t ws_bytes, ranky_info *infos,
                         ranky_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Serving: continuous admission of requests into a device arena              */
/* ------------------------------------------------------------------------- */

typedef struct ranky_server ranky_server;

typedef struct {
    void *arena;          /* device memory the server carves for admitted requests (caller-owned,
                             256-byte aligned) */
    size_t arena_bytes;
    int32_t max_slots;    /* requests on the device at once (each has its own stream), >= 1 */
    int32_t max_queue;    /* waiting requests before submit answers RANKY_E_BUSY, >= 1 */
    int device;
    int32_t pad;          /* alignment padding, ignored */
    ranky_opts opts;      /* path options used for every request */
} ranky_serve_cfg;

/* One request.  A and the outputs are device pointers; A must stay valid until the
 * request completes (the server copies it into the arena when it is admitted and
 * computes from that copy); the outputs are written once, at completion. */
typedef struct {
    ranky_csc A;
    int64_t N;
    int32_t M;
    int32_t k;
    double tol;
    double *sigma;   /* [k] */
    double *U;       /* [M x k] row-major */
    void *V;         /* [N x k] row-major, opts.v_dtype */
} ranky_request;

typedef struct {
    double p50_us, p99_us, mean_us, max_us; /* latency = completion - submit, completed requests */
    double span_s;                           /* first submit to last completion */
    double req_per_s, nnz_per_s;             /* completed requests (nnz) / span */
    int64_t submitted, admitted, completed, failed, cancelled, rejected;
    int64_t queued_now, running_now, peak_running;
    size_t arena_peak_bytes;
} ranky_serve_summary;

/* Creates max_slots contexts and HIP streams on the calling thread, one after the other,
 * then starts one worker thread per slot.  The arena is used as a first-fit heap: a
 * request is admitted (FIFO) when a slot is free and its footprint (CSC copy +
 * ranky_workspace_bytes) fits; requests that arrive while others run join as soon as
 * memory and a slot free up, and their kernels overlap on the device.  Results are
 * bitwise those of ranky_svd alone (no shared state).  E_INVALID for a bad cfg (NULL or
 * unaligned arena, max_slots or max_queue < 1, block_start set), E_DEVICE / E_INVALID
 * from creating a slot's context or stream. */
ranky_status ranky_serve_create(const ranky_serve_cfg *cfg, ranky_server **out);
/* E_BUSY when the queue is full (back-pressure); E_NOMEM when the request could never
 * fit in the arena; E_INVALID for bad sizes.  *ticket receives the request's id. */
ranky_status ranky_serve_submit(ranky_server *srv, const ranky_request *req, uint64_t *ticket);
/* RANKY_PENDING while queued or running; else the request's final status (info filled). */
ranky_status ranky_serve_poll(ranky_server *srv, uint64_t ticket, ranky_info *info);
/* Waits up to timeout_us (< 0: forever); returns as ranky_serve_poll. */
ranky_status ranky_serve_wait(ranky_server *srv, uint64_t ticket, int64_t timeout_us, ranky_info *info);
/* A queued request is dropped (status E_CANCELLED); a running one completes but
 * reports E_CANCELLED. */
ranky_status ranky_serve_cancel(ranky_server *srv, uint64_t ticket);
ranky_status ranky_serve_stats(ranky_server *srv, ranky_serve_summary *stats);
/* Stops admission, drains queued and running requests, joins the workers. */
ranky_status ranky_serve_destroy(ranky_server *srv);

/* ------------------------------------------------------------------------- */
/* Individual steps (the same kernels ranky_svd runs), for composition and    */
/* per-step checking.  Stream-ordered unless marked blocking.                 */
/* ------------------------------------------------------------------------- */

/* Bytes of workspace the step calls below need for these sizes. */
size_t ranky_step_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t D);

/* Alg. 1 scan (the lonely-node test of every block and row) plus the CSC
 * contract check.  Blocking.
 *   cnt    [D x M] int32   nonzeros of row m inside block b (row-major by block)
 *   rownnz [M]     int32   nonzeros of row m
 *   lonely [D]     int32   rows with no entry inside block b
 *   single [D]     int32   rows with exactly one entry inside block b (NO of Eq. 4)
 * Returns E_CSC / E_NONFINITE for an input that breaks the contract. */
ranky_status ranky_occupancy(const ranky_csc *A, int32_t M, int64_t N, int32_t D, int32_t *cnt, int32_t *rownnz,
                             int32_t *lonely, int32_t *single, void *workspace, size_t ws_bytes,
                             ranky_stream_t stream);

/* The Gram matrix G = sum_i A^i A^i^T (Eq. 2), full M x M row-major FP64 in the
 * original row order (rows and columns of empty rows are zero), accumulated
 * in `prec` (a ranky_prec; with RANKY_PREC_BF16X3 the densest rows' block comes from
 * the split-bf16 tiles).  Blocking (it reads back the validation status).
 * E_INVALID for another `prec`. */
ranky_status ranky_gram(const ranky_csc *A, int32_t M, int64_t N, int32_t prec, double *G, void *workspace,
                        size_t ws_bytes, ranky_stream_t stream);

/* Bytes of workspace ranky_eigh needs for an n x n problem. */
size_t ranky_eigh_workspace_bytes(int32_t n);

/* Two-sided blocked Jacobi eigensolve of a dense symmetric n x n FP64 matrix
 * (the proxy SVD of Sec. III / Alg. 1 in Gram form).  Blocking.
 *   G      [n x n]  input, row-major; read only (copied into the workspace)
 *   lambda [n]      eigenvalues, unsorted (pairing with the columns of Q)
 *   Q      [n x n]  row-major, column j is the unit eigenvector of lambda[j]
 *   sweeps (host, may be NULL) receives the number of sweeps.
 * Convergence: every |g_pq| <= max(1e-15, sqrt(n) eps) sqrt(|g_pp g_qq|) or below
 * (n eps)^2 max|g_ii|.  Returns E_NOT_CONVERGED after max_sweeps (0 = 40). */
ranky_status ranky_eigh(int32_t n, const double *G, double *lambda, double *Q, int32_t max_sweeps, int32_t *sweeps,
                        void *workspace, size_t ws_bytes, ranky_stream_t stream);

/* Back-projection V = A^T U Sigma^{-1} on the retained triplets (Sec. V asks for
 * V; the rank rule forbids dividing by a vanishing sigma):
 *   V[j][i] = (sum_m a_mj U[m][i]) / sigma[i]   for i < *rank
 *   V[j][i] = 0                                 for i >= *rank
 *   U [M x k] FP64 row-major, sigma [k] FP64, rank: device int32 scalar,
 *   V [N x k] row-major of v_dtype (FP64 products and sums from the FP64 U, one
 *   rounding at the store; ranky_svd's F32 V reads U rounded to FP32 instead, so
 *   the two F32 results may differ in the last bits).  Stream-ordered; no workspace. */
ranky_status ranky_backproject(const ranky_csc *A, int32_t M, int64_t N, int32_t k, const double *U,
                               const double *sigma, const int32_t *rank, void *V, int32_t v_dtype,
                               ranky_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Incremental merge: column blocks added over time to a resident Gram         */
/* ------------------------------------------------------------------------- */

/* The Gram form of the merge is additive over blocks (Eq. 2-3: A A^T = sum_i A^i A^i^T), so the
 * blocks of a matrix may arrive in any number of steps: each append adds one block's Gram (FP64) to
 * a resident M x M Gram in the original row order, in the order the blocks arrive, and a solve
 * returns the leading singular values and left vectors of all columns appended so far.  A solve
 * starts the subspace iteration (when it applies: opts.eigensolver as for ranky_svd) from the Ritz
 * vectors of the previous solve, so a solve after a small append takes few iterations.  Rows whose
 * entries arrive late simply join the non-empty rows.  V is not kept (the blocks are not stored):
 * V of any block is ranky_backproject(block, U, sigma, rank).  The state lives in the caller's
 * workspace; one call at a time per state.  max_cols / max_nnz bound one appended block. */
typedef struct ranky_inc ranky_inc;
size_t ranky_inc_workspace_bytes(int32_t M, int64_t max_cols, int64_t max_nnz, int32_t k, const ranky_opts *opts);
ranky_status ranky_inc_create(ranky_ctx *ctx, int32_t M, int32_t k, int64_t max_cols, int64_t max_nnz,
                              const ranky_opts *opts, void *workspace, size_t ws_bytes, ranky_inc **out,
                              ranky_stream_t stream);
/* Adds block^T's Gram: block is an M x cols CSC (the contract of ranky_svd, checked).  Blocking. */
ranky_status ranky_inc_append(ranky_inc *inc, const ranky_csc *block, int64_t cols, ranky_stream_t stream);
/* sigma [k], U [M x k] as ranky_svd (rank rule with u_G = 2^-53, sign and empty-row rules) for the
 * matrix of every block appended so far.  info (host, may be NULL): rank, non-empty rows, sweeps or
 * eig_iters, n_blocks = blocks appended.  Blocking. */
ranky_status ranky_inc_solve(ranky_inc *inc, double tol, double *sigma, double *U, ranky_info *info,
                             ranky_stream_t stream);
ranky_status ranky_inc_destroy(ranky_inc *inc);

/* ------------------------------------------------------------------------- */
/* The paper's own procedure (for comparison with the Gram-form path)         */
/* ------------------------------------------------------------------------- */

/* The checkers of Alg. 2-4, on the device, for the blocks b = columns [floor(bN/D), floor((b+1)N/D)):
 * for every block b and row m with no entry of A inside block b (the Alg. 1 scan), one entry of
 * value 1 is set in row m inside block b of a copy A' (A is never altered):
 *   kind 0 RandomChecker (Alg. 2): column c0 + (r0 mod width);
 *   kind 1 NeighborChecker (Alg. 3): the neighbours of m are the rows that share a column with m
 *          outside block b; the candidates are the columns of block b holding an entry of a
 *          neighbour; the chosen one is the (r1 mod count)-th candidate in ascending order, and
 *          the RandomChecker column when there is no candidate;
 *   kind 2 NeighborRandomChecker (Alg. 4): both entries (one when they coincide).
 * Every decision reads the unmodified A (a repair does not feed later ones).  r0 and r1 are draws
 * 2(bM + m) and 2(bM + m) + 1 of a counter-based SplitMix64 (Steele, Lea and Flood 2014): draw i
 * of `seed` is the generator's mixing function applied to seed + (i + 1) * 0x9E3779B97F4A7C15.
 *   colptr_out [N + 1], rowidx_out / values_out (FP64) with room for `capacity` >= nnz + 2 D M
 *   entries (device); nnz_out, added (host): entries of A' and entries added.
 * The width of a block is limited by the LDS bit set of its columns (about 1.2 M columns; E_INVALID
 * beyond).  Blocking.  The result is a function of (A, D, kind, seed) alone. */
size_t ranky_checker_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t D);
ranky_status ranky_checker(const ranky_csc *A, int32_t M, int64_t N, int32_t D, int32_t kind, uint64_t seed,
                           int32_t *colptr_out, int32_t *rowidx_out, double *values_out, int64_t capacity,
                           int64_t *nnz_out, int64_t *added, void *workspace, size_t ws_bytes, ranky_stream_t stream);

typedef struct {
    int64_t added;        /* entries the checker added */
    int64_t nnz_repaired; /* entries of A' */
    int64_t proxy_cols;   /* columns of P: the blocks' retained triplets */
    int32_t rank;         /* rank of P (the rank rule of ranky_svd on P P^T) */
    int32_t n_nonempty;   /* non-empty rows of A' */
    double tau;           /* threshold on the singular values of P */
    float ms[4];          /* [0] checker, [1] scan and block factors, [2] proxy and P P^T, [3] its eigensolve */
} ranky_paper_info;

/* The paper's route (Alg. 1 with Eq. 1-3), all on the device: the optional checker (checker = -1:
 * none, A must then be FP64; 0, 1, 2: the kinds of ranky_checker), the reduced factors U^i S^i of
 * every block (its Gram and a full Jacobi eigensolve; triplets above the block's rank threshold are
 * kept), the proxy P = [U^1 S^1 | ... | U^D S^D] (Eq. 1), P P^T on the FP64 matrix cores (Eq. 3), and
 * its eigenpairs as the SVD of P: sigma [k] (descending, exactly 0 past the rank) and U [M x k]
 * (row-major, the sign and empty-row rules of ranky_svd).  No V (the paper computes none).
 * Blocking.  pinfo (host) may be NULL. */
size_t ranky_paper_workspace_bytes(int32_t M, int64_t N, int64_t nnz, int32_t k, int32_t D, int32_t checker);
ranky_status ranky_svd_paper(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, int32_t D,
                             int32_t checker, uint64_t seed, double tol, void *workspace, size_t ws_bytes,
                             double *sigma, double *U, ranky_paper_info *pinfo, ranky_stream_t stream);

/* The paper's error sums (Sec. IV, as read here): e_sigma = sum_{i<k} |sigma_hat_i - sigma_i| and
 * e_u = sum_{i<k} sum_m |s_i U_hat[m][i] - U[m][i]| with s_i = sign <u_hat_i, u_i>, on the device
 * (fixed-order sums).  U_hat, U: M x k row-major; e_sigma, e_u: host.  workspace: (k + 2) doubles.
 * Blocking. */
ranky_status ranky_paper_errors(int32_t M, int32_t k, const double *sigma_hat, const double *U_hat, const double *sigma,
                                const double *U, double *e_sigma, double *e_u, void *workspace, size_t ws_bytes,
                                ranky_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Without allocation                                                         */
/* ------------------------------------------------------------------------- */

/* Bytes of the fixed device array ranky_svd_noalloc works in (one per GPU, held by the library
 * from the first context on that GPU until the process ends). */
#define RANKY_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)

/* ranky_svd without a workspace argument and without any allocation inside the call, for callers
 * that cannot allocate device or pinned memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is the library's fixed device array of
 * RANKY_NOALLOC_WORKSPACE_BYTES on the context's device; the host staging is the one the context
 * allocated when it was created.  Everything else -- arguments, outputs, results, bit for bit, and
 * errors -- is as ranky_svd with the same options, except that opts->graph is ignored (no graph
 * is captured).  E_NOMEM when ranky_workspace_bytes(M, N, nnz, k, opts) exceeds the array, or when
 * the context's staging is too small for the problem (it is sized for any single matrix the array
 * can hold).  All calls on one GPU share its array: calls that overlap on one GPU (from several
 * threads or on several streams at once) race and must not be issued; consecutive calls are
 * independent (the path initialises everything it reads).  Blocking. */
ranky_status ranky_svd_noalloc(ranky_ctx *ctx, const ranky_csc *A, int32_t M, int64_t N, int32_t k, double tol,
                               const ranky_opts *opts, double *sigma, double *U, void *V, ranky_info *info,
                               ranky_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Tall and skinny (M >> N)                                                   */
/* ------------------------------------------------------------------------- */

/* The CSC of A^T (= the CSR of A) for any row count M: colptr_t [M + 1], rowidx_t [nnz] (the
 * column indices of A, increasing inside each row), values_t [nnz] of A's dtype.  The CSC contract
 * of A is checked first (E_CSC / E_NONFINITE).  workspace: at least
 * ranky_tall_workspace_bytes(M, 1, nnz, 1, NULL) bytes (the transpose's counters use a prefix of
 * it).  Blocking.  Integer work: the result is exact and does not depend on scheduling. */
ranky_status ranky_transpose(const ranky_csc *A, int64_t M, int64_t N, int32_t *colptr_t, int32_t *rowidx_t,
                             void *values_t, void *workspace, size_t ws_bytes, ranky_stream_t stream);

/* Bytes of workspace ranky_svd_tall needs (0 if the sizes are invalid). */
size_t ranky_tall_workspace_bytes(int64_t M, int32_t N, int64_t nnz, int32_t k, const ranky_opts *opts);

/* Top-k singular triplets of a tall-and-skinny A (M x N, M >> N; the paper's problem statement
 * takes the short-and-fat case, Sec. I, and notes the split by rows for the other, Sec. II) by the
 * same method on A^T: A is transposed on the device (ranky_transpose), A^T's column blocks are A's
 * row blocks (opts.n_blocks D splits the M rows as floor(bM/D)), and the path of ranky_svd runs on
 * A^T, whose left vectors are A's right vectors and whose right vectors are A's left vectors.
 *   sigma [k]          as ranky_svd
 *   U     [M x k]      row-major, opts.v_dtype: u_i = A v_i / sigma_i for i < rank, 0 beyond
 *   V     [N x k]      row-major FP64: eigenvectors of A^T A, sign fixed so the entry of largest
 *                      magnitude is positive; columns of A with no entry come last as e_col
 *   info  (host, may be NULL): n_nonempty counts A's non-empty columns; the per-block counts are
 *                      those of A's row blocks (columns of A empty inside a row block)
 * N <= 8192 and 1 <= k <= N (E_INVALID otherwise); M up to 2^31 - 2.  Blocking. */
ranky_status ranky_svd_tall(ranky_ctx *ctx, const ranky_csc *A, int64_t M, int32_t N, int32_t k, double tol,
                            const ranky_opts *opts, void *workspace, size_t ws_bytes, double *sigma, void *U, double *V,
                            ranky_info *info, ranky_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RANKY_H */

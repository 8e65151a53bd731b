// launch.hpp -- host-side launchers of the HIP kernels (internal to libranky.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "batch.hpp"

namespace ranky {

struct CscView {
    int64_t nnz;
    const int32_t *colptr;
    const int32_t *rowidx;
    const void *values;
    int32_t dtype;  // 0 = f32, 1 = f64
};

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);

// occupancy / validation / structural rank / stable transpose (k_occupancy.hip)
void launch_batch_prep(const MatDesc *descs, int count, hipStream_t s);
// out_blk (or NULL): the per-block lonely and single-entry counts of every matrix (MatDesc::blk_off)
void launch_batch_collect(const MatDesc *descs, int count, int32_t *out_i32, double *out_f64, int32_t *out_blk,
                          hipStream_t s);
void launch_occupancy(const MatDesc *descs, const int32_t *wp_chunks, int64_t n_chunk_blocks,
                      const int32_t *wp_rows, int64_t n_row_blocks, int count, int32_t maxM, int32_t maxD,
                      hipStream_t s);
void launch_row_offsets(const MatDesc *descs, const int32_t *wp_rows, int64_t n_row_blocks, int count, hipStream_t s);
// light: a single matrix whose light CSC (heavy-row split) is built: that is transposed instead,
// so the light rows' slots point into it
void launch_transpose(const MatDesc *descs, const int32_t *wp_chunks, int64_t n_chunk_blocks, int count, int32_t maxM,
                      bool light, hipStream_t s);
size_t transpose_lds_bytes(int32_t M);
hipError_t occupancy_set_attributes(int32_t maxM);

// Gram (k_gram.hip)
// waves per Gram workgroup of an M-row matrix (a function of the matrix alone: it fixes the
// order of the sums) and the LDS that matrix's workgroups use with nw waves
// slots: the walk keeps lane-private slots for the dense rows (not with the heavy-row split)
int gram_waves(int32_t M, int32_t acc_bytes, size_t lds_limit, bool slots = true);
size_t gram_lds_bytes(int32_t M, int32_t acc_bytes, int32_t nw, bool slots = true);
int64_t gram_part_slots(int64_t nnz);   // partial Gram rows the workspace must hold
// max_waves, lds_bytes: the largest MatDesc::gwaves and LDS over the launch's matrices
void launch_gram(const MatDesc *descs, const int32_t *wp, int64_t nblocks, const int32_t *wp_red, int64_t nblocks_red,
                 int count, int32_t max_waves, size_t lds_bytes, bool heavy, hipStream_t s);
hipError_t gram_set_attributes(size_t lds_limit);
int32_t gram_dense_wgs(int64_t N);
int32_t gram_heavy_wgs(int64_t N);   // workgroups of the heavy-row tiles (a function of N)
// The heavy split's preparation, before the transpose (which then transposes the light CSC,
// so that the light rows' slots point into it): aht and the light CSC (the walk's columns).
// host: the matrix's descriptor as the host holds it (its workspace pointers).
void launch_gram_heavy_prep(const MatDesc *descs, const MatDesc &host, hipStream_t s);
void launch_gram_heavy_tiles(const MatDesc *descs, int32_t dtype, int32_t hwg, hipStream_t s);   // workgroups of the split-bf16 dense-row tiles (a function of N)
void launch_gram_dense(const MatDesc *descs, int32_t dwg, hipStream_t s);   // BF16X3 dense tiles
void launch_gram_dense_reduce(const MatDesc *descs, int32_t dwg, hipStream_t s);

// Jacobi eigensolver (k_jacobi.hip)
int32_t jacobi_npad(int32_t n);  // multiple of the 32-wide subproblem
constexpr int32_t kJacobiPair = 32;
constexpr int32_t kJacobiBlock = 16;
constexpr int32_t kJacobiCheckTile = 64;   // k_jcheck: one workgroup per 64 x 64 tile of the upper triangle
size_t round_args_bytes();
void fill_round_args(void *dst, const MatDesc &d, int32_t r, int32_t inner_sweeps);
int64_t round_blocks(const MatDesc &d, int32_t r);
void launch_jacobi_init(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s);
// end of a sweep (one workgroup): state per matrix, and with out != NULL the entries
// (active, sweeps, not converged) per matrix in out[3 i ..] followed by the launch's epoch
// (the device counter *epoch, incremented) in out[3 count]
void launch_jacobi_state(const MatDesc *descs, int count, int32_t max_sweeps, int32_t *out, int32_t *epoch,
                         hipStream_t s);
// host_table: the host copy of the launch's argument table (read when count == 1)
void launch_jacobi_round(const void *host_table, const void *table, const int32_t *wp, int64_t nblocks, int count,
                         int32_t launch_r, size_t lds_pad, hipStream_t s);
// dynamic LDS that makes a round workgroup take more than half of a CU's `lds_per_cu`
// bytes, so no two round workgroups share a CU
size_t jround_solo_pad(size_t lds_per_cu);
void launch_jacobi_check(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s);
void launch_jacobi_diag(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s);

// select / gather / back-projection (k_select.hip)
void launch_select(const MatDesc *descs, int count, int32_t max_n, hipStream_t s);
void launch_gather_u(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, hipStream_t s);
int64_t backproject_blocks(int64_t N, int32_t cu_count, int32_t per_cu = 32);
// output pairs per lane of the back-projection for k outputs per column (one pass for k <= 512)
inline int32_t backproject_pairs(int32_t k) { return k <= 128 ? 1 : (k <= 256 ? 2 : 4); }
void launch_backproject_batch(const MatDesc *descs, const int32_t *wp, int64_t nblocks, int count, int32_t pairs,
                              hipStream_t s);
// Uf (or NULL): the FP32 copy of U, read instead of U when V is FP32
void launch_backproject(const CscView &A, int64_t N, int32_t k, const double *U, const float *Uf,
                        const double *sigma, const int32_t *rank, void *V, int32_t v_dtype, int32_t cu_count,
                        hipStream_t s);
hipError_t select_set_attributes();

// Rayleigh-Ritz refinement with the exact operator (k_refine.hip)
size_t rr_part_doubles(int64_t N, int32_t k);   // partial H tiles of the Rayleigh-Ritz SYRK
void launch_rr_h(const CscView &A, int64_t N, int32_t k, const double *U0, double *part, int32_t npad, double *H,
                 hipStream_t s);
// U = U0 Q (sign rule applied); Uf (or NULL) gets the same U in FP32
void launch_rr_apply(const double *U0, const double *Q, int64_t ldq, const int32_t *perm, int32_t M, int32_t k,
                     double *U, float *Uf, hipStream_t s);

// Leading eigenpairs by Chebyshev-filtered subspace iteration (k_topk.hip).  Block matrices are
// rows x p row-major (ld p); rows and p are multiples of 64.
constexpr int32_t kTopkTile = 64;
constexpr int32_t kTopkCholMax = 192;   // widest block the one-workgroup Cholesky-QR takes
// part[z] = op(A) B over the z-th k range of klen (k ranges past K empty); then
// launch_tk_combine adds the splits in order: out = alpha sum + beta E + gamma F
void launch_tk_gemm(bool trans_a, const double *A, int64_t lda, const double *B, int64_t ldb, double *part,
                    int32_t rows, int32_t cols, int32_t K, int32_t splits, int32_t klen, int32_t a_valid,
                    int32_t k_valid, hipStream_t s);
// G Y with the whole block width in one workgroup (cols = 64, 128 or 192; false otherwise, nothing
// launched): grid rows / 64 x splits, partials as launch_tk_gemm's
bool launch_tk_gemm_wide(const double *A, int64_t lda, const double *B, int64_t ldb, double *part, int32_t rows,
                         int32_t cols, int32_t K, int32_t splits, int32_t klen, int32_t a_valid, int32_t k_valid,
                         hipStream_t s);
void launch_tk_combine(const double *part, int32_t splits, int64_t count, double alpha, double beta, const double *E,
                       double gamma, const double *F, double *out, hipStream_t s);
void launch_tk_start(const double *G, int64_t ldg, int32_t n, int32_t p, int32_t rows, double *X, hipStream_t s);
void launch_tk_symcopy(const double *src, int32_t p, double *dst, double *dvec, hipStream_t s);
// p in {64, 128, 192}; other p launch nothing (the caller checks kTopkCholMax).
void launch_tk_chol(const double *S, int32_t p, double shift, double *Wm, int32_t *fail, hipStream_t s);
void launch_tk_svqb_w(const double *V, const double *lam, const double *dvec, int32_t p, double *Wm, hipStream_t s);
void launch_tk_permute(const double *V, const double *lam, const int32_t *perm, int32_t p, double *Qs, double *theta,
                       hipStream_t s);
void launch_tk_resid(const double *GX, const double *X, const double *theta, int32_t n, int32_t p, double *out,
                     hipStream_t s);
void launch_tk_place(const double *src, int32_t rows, int32_t p, double *dst, int64_t ldd, hipStream_t s);

// Tall-and-skinny layout (k_tall.hip): the CSC of A^T (= the CSR of A) for any row count M.
// counts, cursor, long_rows: M ints; btot: tall_scan_blocks(M) ints; ptr: M + 1 (the colptr of
// A^T); nlong: 1; trow: nnz ints (row indices of A^T); tval: nnz values of A's dtype.  Rows of
// A outside [0, M) are dropped (run launch_validate_csc first to report them).
int64_t tall_scan_blocks(int64_t M);
void launch_transpose_csc(const CscView &A, int64_t M, int64_t N, int32_t *counts, int32_t *btot, int32_t *ptr,
                          int32_t *cursor, int32_t *long_rows, int32_t *nlong, int32_t *trow, void *tval,
                          hipStream_t s);
// the CSC contract of A (any M) into *status (kStCsc / kStNonfinite bits)
void launch_validate_csc(const CscView &A, int64_t M, int64_t N, int32_t *status, hipStream_t s);
// ptr[0..n] = exclusive scan of counts[0..n) (btot: tall_scan_blocks(n) ints of scratch)
void launch_exclusive_scan(const int32_t *counts, int64_t n, int32_t *btot, int32_t *ptr, hipStream_t s);
// each segment [ptr[i], ptr[i+1]) of keys (distinct inside a segment, at most 8192 long) sorted
// ascending with its values; long_rows: nseg ints of scratch, nlong: 1
void launch_sort_segments(const int32_t *ptr, int64_t nseg, int32_t *keys, double *vals, int32_t *long_rows,
                          int32_t *nlong, hipStream_t s);

// The paper's own procedure (k_paper.hip): checkers, proxy matrix, error sums.
size_t checker_lds_bytes(int32_t M, int64_t width);
hipError_t paper_set_attributes(size_t lds_limit);
// ins [2 D M]: the new entries (col * M + row) of every (block, row) pair, -1 for none.  cnt is the
// scan's [D x M] occupancy, rowptr / csr_col the rows of A from the transpose.
void launch_checker(const CscView &A, int32_t M, int64_t N, int32_t D, const int32_t *cnt, const int32_t *rowptr,
                    const int32_t *csr_col, int32_t kind, uint64_t seed, int64_t *ins, hipStream_t s);
// A' = A plus the new entries: counts, cursor, long_rows: N ints; btot: tall_scan_blocks(N); iptr:
// N + 1; irow, ival: the new entries (nins); nlong: 1.  colptr_out [N + 1], rowidx_out / vals_out (FP64).
void launch_checker_apply(const CscView &A, int32_t M, int64_t N, const int64_t *ins, int64_t nins, int32_t *counts,
                          int32_t *btot, int32_t *iptr, int32_t *cursor, int32_t *irow, double *ival,
                          int32_t *long_rows, int32_t *nlong, int32_t *colptr_out, int32_t *rowidx_out,
                          double *vals_out, hipStream_t s);
// out [N + D]: block b's columns as their own CSC column pointers, at offset floor(bN/D) + b
void launch_block_slices(const int32_t *colptr, int64_t N, int32_t D, int32_t *out, hipStream_t s);
// rows [0, rank) of P^T from one block's U_b (M x M) and sigma_b over the compacted rows
void launch_proxy_rows(const double *Ub, const double *sb, int32_t M, int32_t rank, const int32_t *m2r, double *Pt,
                       int64_t ldp, hipStream_t s);
// out[0] = e_sigma, out[1] = e_u over k columns (col_err: k doubles of scratch)
void launch_paper_errors(const double *sh, const double *Uh, const double *s_ref, const double *U_ref, int32_t M,
                         int32_t k, double *col_err, double *out, hipStream_t s);

}  // namespace ranky

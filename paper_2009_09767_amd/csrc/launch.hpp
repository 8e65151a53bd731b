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
void launch_transpose(const MatDesc *descs, const int32_t *wp_chunks, int64_t n_chunk_blocks, int count, int32_t maxM,
                      hipStream_t s);
size_t transpose_lds_bytes(int32_t M);
hipError_t occupancy_set_attributes(int32_t maxM);

// Gram (k_gram.hip)
int gram_waves(int32_t M, int32_t acc_bytes, size_t lds_limit);
size_t gram_lds_bytes(int32_t maxM, int32_t acc_bytes, size_t lds_limit);
int64_t gram_part_slots(int64_t nnz);   // partial Gram rows the workspace must hold
void launch_gram(const MatDesc *descs, const int32_t *wp, int64_t nblocks, const int32_t *wp_red, int64_t nblocks_red,
                 int count, int32_t maxM, int32_t acc_bytes, size_t lds_limit, hipStream_t s);
hipError_t gram_set_attributes(size_t lds_limit);
int32_t gram_dense_wgs(int64_t N);   // workgroups of the split-bf16 dense-row tiles (a function of N)
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

}  // namespace ranky

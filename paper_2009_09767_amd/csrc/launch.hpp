// launch.hpp -- host-side launchers of the HIP kernels (internal to libranky.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

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

// occupancy / validation / structural rank (k_occupancy.hip)
void launch_occupancy(const CscView &A, int32_t M, int64_t N, int32_t D, int32_t cpb, int64_t nchunks,
                      int32_t validate, int32_t *hist, int32_t *rownnz, int32_t *cnt, int32_t *lonely,
                      int32_t *single, int32_t *rowptr, int32_t *m2r, int32_t *r2m, int32_t *empty,
                      int32_t *scal, hipStream_t s);
void launch_row_offsets(int32_t *hist, const int32_t *rowptr, int32_t M, int64_t nchunks, hipStream_t s);
void launch_transpose(const CscView &A, int32_t M, int64_t N, int32_t D, int32_t cpb, int64_t nchunks,
                      const int32_t *offs, int32_t *csr_k, int32_t *csr_end, int32_t *csr_col, hipStream_t s);
size_t transpose_lds_bytes(int32_t M);
hipError_t occupancy_set_attributes(int32_t maxM);

// Gram (k_gram.hip); prec 0 = FP64 accumulation, 1 = FP32
int gram_waves(int32_t M, int32_t acc_bytes, size_t lds_limit);
void launch_gram(const CscView &A, int32_t M, int32_t n, int32_t npad, int64_t ld, const int32_t *rowptr,
                 const int32_t *r2m, const int32_t *csr_k, const int32_t *csr_end, double *G, int32_t prec,
                 size_t lds_limit, hipStream_t s);
hipError_t gram_set_attributes(size_t lds_limit);

// Jacobi eigensolver (k_jacobi.hip)
struct JacobiRound {
    const double *Gin;
    double *Gout;
    double *W;
    int64_t ld;
    int32_t npad;
    int32_t round_cur, round_prev, has_prev, do_solve;
    const double *Jprev;
    const int32_t *fprev;
    const double *Sprev;
    double *Jcur;
    int32_t *fcur;
    double *Scur;
    const double *sdbl;
    double tol;
    int32_t inner_sweeps;
};
int32_t jacobi_npad(int32_t n);  // multiple of the 32-wide subproblem
constexpr int32_t kJacobiPair = 32;
void launch_jacobi_init(double *W, int32_t npad, const double *G, int64_t ld, int32_t n, double *sdbl,
                        hipStream_t s);
void launch_jacobi_round(const JacobiRound &r, hipStream_t s);
void launch_jacobi_check(const double *G, int64_t ld, int32_t n, double tol, const double *sdbl, int32_t *scal,
                         hipStream_t s);
void launch_jacobi_diag(const double *G, int64_t ld, int32_t n, double *lam, hipStream_t s);

// select / gather / back-projection (k_select.hip)
void launch_select(const double *lam, int32_t n, int32_t k, int32_t n_tau, double tol, double u_gram, int32_t *perm,
                   double *sigma, int32_t *scal, double *sdbl, hipStream_t s);
void launch_gather_u(const double *W, int64_t ld, int32_t n, int32_t M, int32_t k, const int32_t *perm,
                     const int32_t *m2r, const int32_t *empty, double *U, hipStream_t s);
void launch_backproject(const CscView &A, int64_t N, int32_t k, const double *U, const double *sigma,
                        const int32_t *rank, void *V, int32_t v_dtype, int32_t cu_count, hipStream_t s);
hipError_t select_set_attributes();

// Rayleigh-Ritz refinement with the exact operator (k_refine.hip)
void launch_rr_z(const CscView &A, int64_t N, int32_t k, const double *U0, double *Z, int32_t cu_count, hipStream_t s);
int64_t rr_max_segments(int32_t M, int64_t nnz);
void launch_rr_rows(const CscView &A, const int32_t *rownnz, const int32_t *rowptr, int32_t M, int64_t nnz, int32_t k,
                    const int32_t *csr_k, const int32_t *csr_col, const double *Z, int32_t *seg_ptr, double *part,
                    double *Y, hipStream_t s);
void launch_rr_h(const double *U0, const double *Y, int32_t M, int32_t k, int32_t npad, double *H, hipStream_t s);
void launch_rr_apply(const double *U0, const double *Q, int64_t ldq, const int32_t *perm, int32_t M, int32_t k,
                     double *U, hipStream_t s);

}  // namespace ranky

// launch_util.hpp -- layout helpers (k_util.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranky {

void launch_pad_copy(const double *src, int32_t n, double *dst, int32_t npad, int64_t ld, hipStream_t s);
void launch_unpad_copy(const double *src, int64_t ld, int32_t n, double *dst, hipStream_t s);
void launch_scatter_gram(const double *Gc, int64_t ld, const int32_t *m2r, int32_t M, double *G, hipStream_t s);
// resident Gram of an incrementally merged matrix (M x M, original row order)
void launch_scatter_add_gram(const double *Gc, int64_t ld, const int32_t *m2r, int32_t M, double *G, hipStream_t s);
void launch_inc_rows(const double *G, int32_t M, int32_t *m2r, int32_t *r2m, int32_t *empty, int32_t *n_out,
                     hipStream_t s);
void launch_inc_gather(const double *G, int32_t M, const int32_t *r2m, const int32_t *n_in, int32_t npad, double *Gc,
                       hipStream_t s);
void launch_inc_start(const double *Xprev, const int32_t *r2m, int32_t n, int32_t rows, int32_t p, double *X,
                      hipStream_t s);
void launch_inc_keep(const double *X, int64_t ldx, const int32_t *m2r, int32_t M, int32_t p, double *Xkeep,
                     hipStream_t s);

}  // namespace ranky

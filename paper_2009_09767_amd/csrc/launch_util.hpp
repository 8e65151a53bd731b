// launch_util.hpp -- layout helpers (k_util.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranky {

void launch_pad_copy(const double *src, int32_t n, double *dst, int32_t npad, int64_t ld, hipStream_t s);
void launch_unpad_copy(const double *src, int64_t ld, int32_t n, double *dst, hipStream_t s);
void launch_scatter_gram(const double *Gc, int64_t ld, const int32_t *m2r, int32_t M, double *G, hipStream_t s);

}  // namespace ranky

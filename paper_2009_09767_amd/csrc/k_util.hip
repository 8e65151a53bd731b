// k_util.hip -- layout moves between the caller's dense n x n / M x M arrays and
// the padded, compacted layout of the eigensolver.
#include "common.hpp"
#include "launch_util.hpp"

namespace ranky {

// dst (npad x npad, ld) <- src (n x n, row-major), zero outside the leading n x n.
__global__ __launch_bounds__(256) void k_pad_copy(const double *__restrict__ src, int32_t n, double *__restrict__ dst,
                                                  int32_t npad, int64_t ld) {
    const int64_t total = (int64_t)npad * npad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / npad, c = e % npad;
        dst[r * ld + c] = (r < n && c < n) ? src[r * n + c] : 0.0;
    }
}

// dst (n x n, row-major) <- leading n x n of src (ld).
__global__ __launch_bounds__(256) void k_unpad_copy(const double *__restrict__ src, int64_t ld, int32_t n,
                                                    double *__restrict__ dst) {
    const int64_t total = (int64_t)n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = src[(e / n) * ld + e % n];
}

// Full M x M Gram in original row order from the compacted one (zero rows/columns
// for the empty rows).
__global__ __launch_bounds__(256) void k_scatter_gram(const double *__restrict__ Gc, int64_t ld,
                                                      const int32_t *__restrict__ m2r, int32_t M,
                                                      double *__restrict__ G) {
    const int64_t total = (int64_t)M * M;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = m2r[e / M], b = m2r[e % M];
        G[e] = (a >= 0 && b >= 0) ? Gc[(int64_t)a * ld + b] : 0.0;
    }
}

static unsigned grid_for(int64_t work) {
    int64_t b = (work + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

void launch_pad_copy(const double *src, int32_t n, double *dst, int32_t npad, int64_t ld, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_copy, dim3(grid_for((int64_t)npad * npad)), dim3(256), 0, s, src, n, dst, npad, ld);
}

void launch_unpad_copy(const double *src, int64_t ld, int32_t n, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_unpad_copy, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, src, ld, n, dst);
}

void launch_scatter_gram(const double *Gc, int64_t ld, const int32_t *m2r, int32_t M, double *G, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_gram, dim3(grid_for((int64_t)M * M)), dim3(256), 0, s, Gc, ld, m2r, M, G);
}

}  // namespace ranky

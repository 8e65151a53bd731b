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

// G += the compacted Gc scattered back to the original row order (rows of empty rows add 0).
__global__ __launch_bounds__(256) void k_scatter_add_gram(const double *__restrict__ Gc, int64_t ld,
                                                          const int32_t *__restrict__ m2r, int32_t M,
                                                          double *__restrict__ G) {
    const int64_t total = (int64_t)M * M;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = m2r[e / M], b = m2r[e % M];
        if (a >= 0 && b >= 0) G[e] += Gc[(int64_t)a * ld + b];
    }
}

// The rows of a resident Gram that have an entry: G_mm > 0 exactly when row m of the matrix has a
// nonzero (a sum of squares of real values).  One workgroup: m2r[m] = compacted index or -1,
// r2m[i] = the i-th such row, empty[e] = the e-th row without, n_out[0] = their count.
__global__ __launch_bounds__(1024) void k_inc_rows(const double *__restrict__ G, int32_t M, int32_t *__restrict__ m2r,
                                                   int32_t *__restrict__ r2m, int32_t *__restrict__ empty,
                                                   int32_t *__restrict__ n_out) {
    __shared__ int32_t run[1024];
    __shared__ int32_t base_nz, base_e;
    if (threadIdx.x == 0) base_nz = base_e = 0;
    __syncthreads();
    for (int32_t c0 = 0; c0 < M; c0 += 1024) {
        const int32_t m = c0 + threadIdx.x;
        const int32_t nz = m < M && G[(int64_t)m * M + m] > 0.0 ? 1 : 0;
        run[threadIdx.x] = nz;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t add = (int)threadIdx.x >= off ? run[threadIdx.x - off] : 0;
            __syncthreads();
            run[threadIdx.x] += add;
            __syncthreads();
        }
        if (m < M) {
            const int32_t before = run[threadIdx.x] - nz;
            if (nz) {
                m2r[m] = base_nz + before;
                r2m[base_nz + before] = m;
            } else {
                m2r[m] = -1;
                empty[base_e + (threadIdx.x - before)] = m;
            }
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            base_nz += run[1023];
            base_e += (M - c0 < 1024 ? M - c0 : 1024) - run[1023];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) n_out[0] = base_nz;
}

// Gc (npad x npad) = G restricted to the n rows r2m (zero padding).
__global__ __launch_bounds__(256) void k_inc_gather(const double *__restrict__ G, int32_t M,
                                                    const int32_t *__restrict__ r2m, const int32_t *__restrict__ n_in,
                                                    int32_t npad, double *__restrict__ Gc) {
    const int32_t n = n_in[0];
    const int64_t total = (int64_t)npad * npad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(e / npad), j = (int32_t)(e % npad);
        Gc[e] = (i < n && j < n) ? G[(int64_t)r2m[i] * M + r2m[j]] : 0.0;
    }
}

// X (rows x p, ld p) <- the previous Ritz vectors (M x p in the original row order, ld p) mapped to
// the current compaction, plus a small fixed perturbation, as a warm start block.
__global__ __launch_bounds__(256) void k_inc_start(const double *__restrict__ Xprev, const int32_t *__restrict__ r2m,
                                                   int32_t n, int32_t rows, int32_t p, double *__restrict__ X) {
    const int64_t total = (int64_t)rows * p;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = (int32_t)(e / p), c = (int32_t)(e % p);
        double v = 0.0;
        if (i < n) {
            uint64_t z = (uint64_t)e + 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            v = Xprev[(int64_t)r2m[i] * p + c] + 1e-3 * ((double)(z >> 11) * 0x1.0p-52 - 1.0);
        }
        X[e] = v;
    }
}

// Xkeep (M x p, original rows) <- X (compacted rows x p, ld ldx): the Ritz vectors kept for the next start.
__global__ __launch_bounds__(256) void k_inc_keep(const double *__restrict__ X, int64_t ldx,
                                                  const int32_t *__restrict__ m2r, int32_t M, int32_t p,
                                                  double *__restrict__ Xkeep) {
    const int64_t total = (int64_t)M * p;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t m = (int32_t)(e / p), c = (int32_t)(e % p);
        const int32_t i = m2r[m];
        Xkeep[e] = i >= 0 ? X[(int64_t)i * ldx + c] : 0.0;
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

void launch_scatter_add_gram(const double *Gc, int64_t ld, const int32_t *m2r, int32_t M, double *G, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_add_gram, dim3(grid_for((int64_t)M * M)), dim3(256), 0, s, Gc, ld, m2r, M, G);
}

void launch_inc_rows(const double *G, int32_t M, int32_t *m2r, int32_t *r2m, int32_t *empty, int32_t *n_out,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_inc_rows, dim3(1), dim3(1024), 0, s, G, M, m2r, r2m, empty, n_out);
}

void launch_inc_gather(const double *G, int32_t M, const int32_t *r2m, const int32_t *n_in, int32_t npad, double *Gc,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_inc_gather, dim3(grid_for((int64_t)npad * npad)), dim3(256), 0, s, G, M, r2m, n_in, npad, Gc);
}

void launch_inc_start(const double *Xprev, const int32_t *r2m, int32_t n, int32_t rows, int32_t p, double *X,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_inc_start, dim3(grid_for((int64_t)rows * p)), dim3(256), 0, s, Xprev, r2m, n, rows, p, X);
}

void launch_inc_keep(const double *X, int64_t ldx, const int32_t *m2r, int32_t M, int32_t p, double *Xkeep,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_inc_keep, dim3(grid_for((int64_t)M * p)), dim3(256), 0, s, X, ldx, m2r, M, p, Xkeep);
}

}  // namespace ranky

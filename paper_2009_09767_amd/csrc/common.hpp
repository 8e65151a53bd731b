// common.hpp -- shared constants and small device helpers of the HIP path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranky {

// Columns handled by one workgroup of the occupancy and transpose passes: at most
// kChunkCols, halved down to kChunkColsMin while a matrix has fewer than kChunkTarget
// chunks (so a matrix of a million columns still fills the device).
constexpr int kChunkCols = 4096;
// Largest row count M the library takes.
constexpr int32_t kMaxM = 8192;
constexpr int kChunkColsMin = 512;
constexpr int kChunkTarget = 1024;

// Bits of the device status word.
enum : int32_t { kStCsc = 1, kStNonfinite = 2 };

// Integer slots and double slots of the device scalar block (in the workspace).
enum : int32_t {
    kScStatus = 0,     // status bits
    kScNonempty = 1,   // M' (rows with a nonzero)
    kScRank = 2,       // rank after the threshold
    kScNotConv = 3,    // 1 if some off-diagonal entry still fails the Jacobi test
    kScGramSegs = 4,   // Gram workgroups for the nonempty rows (one per row segment)
    kScGramSlots = 5,  // partial rows of the rows cut into more than one segment
    kScCount = 16
};
// Nonzeros of one row segment of the Gram: a longer row is cut into segments handled by
// separate workgroups, whose partial rows are added in segment order.
constexpr int32_t kGramSeg = 1 << 16;
// A matrix's segment length: nnz / kGramSegTarget rounded down to a power of two, within
// [kGramSegMin, kGramSeg], so that a few dense rows of a small matrix do not leave one
// workgroup with most of the work.  A function of the matrix alone (not of D).
constexpr int32_t kGramSegMin = 1 << 12;
constexpr int64_t kGramSegTarget = 1024;
inline int32_t gram_seg_len(int64_t nnz) {
    int32_t s = kGramSeg;
    while (s > kGramSegMin && (int64_t)s * kGramSegTarget > nnz) s >>= 1;
    return s;
}
// Densest rows of the Gram (at most this many, each with at least max(4096, N / 64)
// nonzeros): their products go to lane-private slots instead of the shared row, since
// most lanes of a wave would otherwise meet on the same few rows.
constexpr int kDenseRows = 32;
// Column entries each lane of the Gram walk loads ahead (one group of gathers in flight).
constexpr int kGramStep = 4;
// Column entries the occupancy scan loads per step.
constexpr int kOccGroup = 8;
// Free value of a Gram election tag (above every workgroup-wide lane id).
constexpr int32_t kTagFree = 0x7fffffff;
// Ints per matrix in the per-matrix read-back (status, M', rank, sweeps, not-converged,
// lonely max, lonely blocks, active, Gram segments, Gram partial rows).
constexpr int kColI = 11;
enum : int32_t { kSdTau = 0, kSdSigmaMax = 1, kSdFloor = 2, kSdScale = 3, kSdCount = 8 };

// Column range of chunk c: block b = c / cpb owns columns [floor(bN/D), floor((b+1)N/D)),
// or [bstart[b], bstart[b+1]) when the caller gave the boundaries, and its t-th chunk
// (t = c % cpb) is the t-th run of cc columns of it.
__device__ __forceinline__ void chunk_columns(int64_t c, int32_t cpb, int32_t cc, int64_t N, int32_t D,
                                              const int64_t *__restrict__ bstart, int64_t &c0, int64_t &c1) {
    const int64_t b = c / cpb, t = c % cpb;
    const int64_t bs = bstart ? bstart[b] : (b * N) / D, be = bstart ? bstart[b + 1] : ((b + 1) * N) / D;
    c0 = bs + t * cc;
    c1 = c0 + cc < be ? c0 + cc : be;
    if (c0 > c1) c0 = c1;
}

// Global-memory view of a device pointer the compiler cannot prove global (one read from
// a descriptor table): its accesses become global loads and stores instead of FLAT ones,
// which also count against the LDS / scalar wait counter.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

template <typename T>
__device__ __forceinline__ double as_double(T v) {
    return static_cast<double>(v);
}

__device__ __forceinline__ bool finite_value(double v) { return __builtin_isfinite(v); }
__device__ __forceinline__ bool finite_value(float v) { return __builtin_isfinite(v); }

}  // namespace ranky

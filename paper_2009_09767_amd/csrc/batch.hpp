// batch.hpp -- per-matrix descriptors and the workgroup -> matrix mapping shared by
// every kernel.  A launch covers a batch of independent matrices: workgroups
// [wp[i], wp[i+1]) belong to matrix i, so uneven matrices share one grid.  The
// single-matrix entry point is the same code with a batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ranky {

// A light-CSC entry of the heavy-row split: its row and value side by side, so that the Gram
// walk reads both with one load (8 bytes for FP32 values, 16 for FP64).
template <typename TV>
struct LightRec;
template <>
struct alignas(8) LightRec<float> {
    int32_t row;
    float val;
};
template <>
struct alignas(16) LightRec<double> {
    int32_t row, pad;
    double val;
};

struct MatDesc {
    // input (caller-owned)
    const int32_t *colptr;
    const int32_t *rowidx;
    const void *values;
    int64_t nnz;
    int64_t N;
    int64_t nchunks;
    const int64_t *bstart;    // D + 1 column boundaries of the blocks, or NULL for floor(bN/D)
    int32_t M, k, D, cpb;
    int32_t ccols;            // columns per chunk (the last chunk of a block may be shorter)
    int32_t gseg;             // Gram segment length (nonzeros of a row per workgroup)
    int32_t dtype, v_dtype;
    int32_t n, npad;          // non-empty rows and the eigensolver order (set after the scan)
    int32_t neig;             // eigenpairs the eigensolve leaves in lam / W (n, or the subspace block width)
    int32_t prec;             // Gram accumulation: 0 FP64, 1 FP32, 2 FP32 with BF16x3 dense tiles
    int32_t validate;
    int32_t n_tau;            // row count entering the threshold sqrt(n_tau u_gram)
    int32_t dwg;              // split-bf16 dense-tile workgroups (0: the dense rows stay in the sparse pass)
    int32_t blk_off;          // first entry of this matrix's per-block counts in the read-back array
    int32_t gwaves;           // Gram walk waves per workgroup (a function of M and the accumulator alone)
    double tol;               // rank threshold option
    double u_gram;            // unit roundoff of the Gram entries for the threshold
    double jtol;              // Jacobi rotation test tolerance (0: max(1e-15, sqrt(n) eps))
    // workspace (library-carved from caller memory)
    int32_t *scal, *hist, *rownnz, *rowptr, *m2r, *r2m, *empty, *lonely, *single;
    // row-major copy of the nonzeros: csrk holds a (CSC position, column end) pair per slot (one
    // 8-byte access each), csrcol the column
    int32_t *csrk, *csrcol, *jflag, *perm;
    int32_t *cnt;             // optional [D x M] occupancy output (step call only)
    int32_t *jstate;          // Jacobi state: [0] sweeps done, [1] active this sweep, [2] not converged
    int32_t *gsegp;           // [n + 1] first Gram segment of compacted row i (set by the scan)
    int32_t *gslot;           // [n + 1] first partial row of compacted row i (rows with one segment take none)
    double *gpart;            // [slots][npad] partial Gram rows of the cut rows
    double *dpart;            // [dwg][kDenseRows^2] partial dense-row Gram tiles
    int32_t *dense;           // [kDenseRows] the densest rows (original index, by degree), -1 when unused
    // heavy-row split of the Gram (hwg > 0): the dense rows leave the sparse walk; their
    // values per column go to aht (N x kDenseRows, the matrix's value type, zeros elsewhere),
    // their block of G comes from FP64 matrix-core tiles over column ranges (hpart, one
    // kDenseRows^2 tile per workgroup) and their pairs with the other rows from rows of aht
    void *aht;
    double *hpart;
    int32_t hwg;              // heavy-tile workgroups (0: off)
    int32_t hpad;
    // with the split, the walk runs on a copy of the columns without the dense rows (the light
    // CSC): per-column light counts, their exclusive scan (N + 1), its block totals, the light
    // rows, and the light entries as (row, value) records (LightRec: one load per entry)
    int32_t *lcnt, *lptr, *lbtot, *lrowidx;
    void *lvals;
    // launch-shape knobs (results do not depend on them; set from the context's tuning cache)
    int32_t bp_per_cu;        // back-projection workgroups per compute unit
    int32_t jsched;           // Jacobi round launch: bit 0 update tiles grouped per XCD, bit 1 one round workgroup per CU
    double *sdbl, *G, *G2, *W, *J, *S, *lam;
    // outputs (caller-owned)
    double *sigma, *U;
    float *Uf;                // FP32 copy of U for an FP32 V (the back-projection reads it), or NULL
    void *V;
};

// kJsCheck: the running convergence test's flag, folded into kJsNotConv by the state update
enum : int32_t { kJsSweeps = 0, kJsActive = 1, kJsNotConv = 2, kJsCheck = 3, kJsCount = 4 };

// Matrix owning workgroup b: the last i with wp[i] <= b (wp has count + 1 entries).
__device__ __forceinline__ int find_mat(const int32_t *__restrict__ wp, int count, int b) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wp[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace ranky

"""A matrix with dense rows through the C-ABI against the CPU oracle: 8 rows of 4096 to
15000 nonzeros over 20000 columns (the scan's dense rows: at least max(4096, N / 64)
nonzeros) and 88 sparse rows.  FP64 and FP32 take every pair in the sparse pass (the dense
rows in lane-private slots); BF16X3 computes the dense rows' block as split-bf16 tiles on
the matrix cores."""
import numpy as np
import pytest

from paper_2009_09767_amd import gen

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24
DENSE = {3: 15000, 10: 12000, 17: 9000, 30: 7000, 44: 6000, 58: 5000, 71: 4500, 90: 4096}


@pytest.fixture(scope="module")
def R():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_09767_amd import ranky

    ranky.lib()
    return ranky


def dense_rows_matrix(dtype=np.float64, seed=31, M=96, N=20000):
    rng = np.random.Generator(np.random.PCG64(seed))
    rows, cols = [], []
    for m in range(M):
        d = DENSE.get(m, int(rng.integers(20, 400)))
        rows.append(np.full(d, m))
        cols.append(rng.choice(N, size=d, replace=False))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    return gen.from_coo(M, N, rows, cols, rng.standard_normal(rows.size).astype(dtype))


def absgram(orc, A):
    return orc.gram(A.M, A.N, A.colptr, A.rowidx, np.abs(A.values.astype(np.float64)))


def max_row_nnz(A):
    return int(np.bincount(A.rowidx, minlength=A.M).max())


def test_dense_tiles_fp64(R, orc):
    A = dense_rows_matrix()
    dA = R.to_device(A)
    G = R.gram(dA, prec="fp64").cpu().numpy()
    ref = orc.gram(A.M, A.N, A.colptr, A.rowidx, A.values)
    assert np.all(np.abs(G - ref) <= 2.0 * max_row_nnz(A) * U64 * absgram(orc, A))
    assert np.array_equal(G, G.T)
    assert np.array_equal(G, R.gram(dA, prec="fp64").cpu().numpy()), "not bitwise deterministic"


def test_dense_tiles_fp32(R, orc):
    A = dense_rows_matrix(np.float32)
    G = R.gram(R.to_device(A), prec="fp32").cpu().numpy()
    ref = orc.gram(A.M, A.N, A.colptr, A.rowidx, A.values)
    assert np.all(np.abs(G - ref) <= 2.0 * (max_row_nnz(A) + 2) * U32 * absgram(orc, A))


def test_dense_tiles_bf16x3(R, orc):
    """The dense rows' block is the split-bf16 product (hi hi + hi lo + lo hi, by the
    oracle's definition) up to FP32 accumulation; every other entry is the FP32 Gram."""
    A = dense_rows_matrix(np.float32)
    G = R.gram(R.to_device(A), prec="bf16x3").cpu().numpy()
    ref = orc.gram(A.M, A.N, A.colptr, A.rowidx, A.values)
    absg = absgram(orc, A)
    rows = np.array(sorted(DENSE), dtype=np.int32)
    ref_split = orc.gram_bf16x3(A.M, A.N, A.colptr, A.rowidx, A.values, rows)
    blk = np.ix_(rows, rows)
    off = ~np.eye(rows.size, dtype=bool)
    bound = 2.0 * (max_row_nnz(A) + 2) * U32 * absg
    # the dense block (off the diagonal) follows the split-bf16 definition ...
    assert np.all(np.abs(G[blk] - ref_split)[off] <= bound[blk][off])
    # ... which differs from the exact product by up to ~2^-16 relative (so it did run)
    assert np.max(np.abs(G[blk] - ref[blk])[off]) > 0.0
    assert np.all(np.abs(G[blk] - ref[blk])[off] <= 2.0 ** -15 * absg[blk][off] + bound[blk][off])
    # every other entry, and the diagonal, is the FP32 sparse Gram
    rest = np.ones_like(G, dtype=bool)
    rest[blk] = ~off
    assert np.all(np.abs(G - ref)[rest] <= bound[rest])


def test_dense_tiles_block_count_invariant(R):
    """The tiles' column ranges depend on N only: the BF16X3 result does not depend on D."""
    import torch

    A = dense_rows_matrix(np.float32)
    dA = R.to_device(A)
    outs = [R.svd(dA, 24, 0.0, n_blocks=D, gram_prec="bf16x3", refine=1, v_dtype=torch.float32) for D in (8, 1, 64)]
    for o in outs[1:]:
        assert np.array_equal(o.sigma.cpu().numpy(), outs[0].sigma.cpu().numpy())
        assert np.array_equal(o.U.cpu().numpy(), outs[0].U.cpu().numpy())

"""Tall-and-skinny matrices (M >> N): the device transpose (ranky_transpose) bit for bit against
scipy's CSR of A, and ranky_svd_tall against the oracle run on A^T (transposed on the host by
scipy, independent of the library): sigma at 1e-10, A's right vectors V (the eigenvectors of
A^T A) and left vectors U by per-cluster angles, exact rank with empty columns of A."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2009_09767_amd import gen
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_09767_amd import ranky

    ranky.lib()
    return ranky


def tall_random(M, N, density, seed, dtype=np.float64, empty_cols=0, long_rows=0):
    rng = np.random.default_rng(seed)
    nnz = int(M * N * density)
    flat = np.unique(rng.integers(0, M * N, size=nnz))
    rows, cols = flat // N, flat % N
    if empty_cols:
        dead = rng.choice(N, size=empty_cols, replace=False)
        keep = ~np.isin(cols, dead)
        rows, cols = rows[keep], cols[keep]
    if long_rows:   # a few rows with many entries (the long-row sort)
        lr = rng.choice(M, size=long_rows, replace=False)
        extra_r = np.repeat(lr, N // 2)
        extra_c = np.concatenate([rng.choice(N, size=N // 2, replace=False) for _ in lr])
        flat = np.unique(np.concatenate([rows * N + cols, extra_r * N + extra_c]))
        rows, cols = flat // N, flat % N
    vals = rng.standard_normal(rows.size)
    return gen.from_coo(M, N, rows, cols, vals.astype(dtype), dict(name="tall"))


def host_transpose(A):
    m = sp.csc_matrix((A.values, A.rowidx, A.colptr), shape=(A.M, A.N)).tocsr()
    m.sort_indices()
    return m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data


@pytest.mark.parametrize("case", ["plain", "f32_long_rows", "empty_rows_and_cols"])
def test_transpose_bit_exact(R, case):
    if case == "plain":
        A = tall_random(50000, 96, 0.02, 1)
    elif case == "f32_long_rows":
        A = tall_random(20000, 9000 // 1, 0.0005, 2, np.float32, long_rows=3)   # rows of 4500+ entries
    else:
        A = tall_random(30000, 300, 0.001, 3, empty_cols=40)
    T = R.transpose(R.to_device(A))
    cp, ri, va = host_transpose(A)
    assert (T.M, T.N) == (A.N, A.M)
    assert np.array_equal(T.colptr.cpu().numpy(), cp)
    assert np.array_equal(T.rowidx.cpu().numpy(), ri)
    assert np.array_equal(T.values.cpu().numpy(), va.astype(A.values.dtype))


def test_transpose_rejects_a_broken_csc(R):
    import torch

    A = tall_random(1000, 20, 0.05, 4)
    dA = R.to_device(A)
    ri = A.rowidx.copy()
    ri[3] = A.M + 5   # out of range: reported, never written
    dA.rowidx = torch.from_numpy(ri).cuda()
    with pytest.raises(R.RankyError) as e:
        R.transpose(dA)
    assert e.value.status == R.E_CSC


CASES = {
    "random_100k_x_128": (lambda: tall_random(100000, 128, 0.01, 10), 32),
    "powerlaw_transposed_16k_x_128": (lambda: None, 32),
    "empty_cols_50k_x_200_full": (lambda: tall_random(50000, 200, 0.004, 11, empty_cols=50), 200),
    "f32_200k_x_64": (lambda: tall_random(200000, 64, 0.01, 12, np.float32), 64),
}


def powerlaw_tall():
    """powerlaw_small (128 x 16384, Zipf rows) transposed: a tall matrix with power-law columns."""
    P = gen.powerlaw_small()
    m = sp.csc_matrix((P.values, P.rowidx, P.colptr), shape=(P.M, P.N)).T.tocsc()
    m.sort_indices()
    return gen.CSC(P.N, P.M, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data, dict(name="tall_pl"))


@pytest.mark.parametrize("name", list(CASES))
def test_svd_tall_against_oracle(R, orc, name):
    import torch

    mk, k = CASES[name]
    A = powerlaw_tall() if name.startswith("powerlaw") else mk()
    cp, ri, va = host_transpose(A)
    ref = orc.svd(A.N, A.M, cp, ri, va, k=k, method="whole_qr")   # A^T is N x M (short and fat)
    vdt = torch.float32 if A.values.dtype == np.float32 else torch.float64
    got = R.svd_tall(R.to_device(A), k, 0.0, v_dtype=vdt, n_blocks=4)
    r = ref.rank
    assert got.info["rank"] == r
    empty_cols = int(np.count_nonzero(np.diff(A.colptr) == 0))
    assert got.info["n_nonempty"] == A.N - empty_cols
    sg = got.sigma.cpu().numpy()
    err = H.rel_sigma_err(sg, ref.sigma, r)
    Vg = got.V.cpu().numpy()                   # N x k: A's right vectors = the oracle's left vectors of A^T
    Ug = got.U.double().cpu().numpy()          # M x k: A's left vectors = the oracle's right vectors of A^T
    sv, _ = H.vector_errors(Vg[:, :r], ref.U[:, :r], ref.sigma, r)
    su, _ = H.vector_errors(Ug[:, :r], ref.V[:, :r], ref.sigma, r)
    print(f"{name}: rank {r}, sigma err {err:.2e}, V sine x relgap {sv:.2e}, U sine x relgap {su:.2e}", flush=True)
    assert err <= 1e-10
    assert sv <= 1e-12
    assert su <= (1e-12 if vdt == torch.float64 else 2.0 ** -22)
    assert np.all(sg[r:] == 0.0) and np.all(Ug[:, r:] == 0.0)
    assert H.canonical_sign_ok(Vg)
    # empty columns of A come back as e_col, ascending, after the others
    dead = np.flatnonzero(np.diff(A.colptr) == 0)
    n = A.N - dead.size
    for j, c in enumerate(dead):
        if n + j < k:
            e = np.zeros(A.N)
            e[c] = 1.0
            assert np.array_equal(Vg[:, n + j], e)

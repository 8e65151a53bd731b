"""Incremental merge (ranky_inc_*): column blocks appended to a resident Gram over time (Eq. 2-3 are
additive over blocks).  After every append the solve matches the oracle on the columns appended so
far; after the last it matches ranky_svd on the whole matrix; rows whose entries arrive late join
the non-empty rows; the subspace iteration restarts from the previous solve's Ritz vectors."""
import numpy as np
import pytest

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


def column_slice(A, c0, c1):
    cp = A.colptr[c0:c1 + 1].astype(np.int64)
    e0, e1 = int(cp[0]), int(cp[-1])
    return gen.CSC(A.M, c1 - c0, (cp - e0).astype(np.int32), A.rowidx[e0:e1].copy(), A.values[e0:e1].copy(),
                   dict(name="slice"))


def check(got_sigma, got_U, info, ref, bar=1e-10):
    r = ref.rank
    assert info["rank"] == r
    sg, Ug = got_sigma.cpu().numpy(), got_U.cpu().numpy()
    err = H.rel_sigma_err(sg, ref.sigma, r)
    scaled, _ = H.vector_errors(Ug[:, :r], ref.U[:, :r], ref.sigma, r)
    assert err <= bar and scaled <= bar, (err, scaled)
    assert np.all(sg[r:] == 0.0)
    assert H.canonical_sign_ok(Ug)
    return err, scaled


def test_incremental_matches_the_oracle_after_every_append(R, orc):
    A = gen.powerlaw_small()
    k = 32
    cuts = [0, 3000, 7000, 12000, A.N]
    inc = R.Incremental(A.M, k, max_cols=6000, max_nnz=A.nnz)
    for i in range(len(cuts) - 1):
        inc.append(R.to_device(column_slice(A, cuts[i], cuts[i + 1])))
        s, U, info = inc.solve()
        P = column_slice(A, 0, cuts[i + 1])
        ref = orc.svd(P.M, P.N, P.colptr, P.rowidx, P.values, k=k, method="whole")
        err, scaled = check(s, U, info, ref)
        print(f"after {i + 1} blocks ({cuts[i + 1]} columns): rank {info['rank']}, sigma {err:.2e}, U {scaled:.2e}")
    whole = R.svd(R.to_device(A), k, 0.0)
    assert H.rel_sigma_err(s.cpu().numpy(), whole.sigma.cpu().numpy(), info["rank"]) <= 1e-12


def test_rows_arriving_late(R, orc):
    """Rows 0..63 have entries only in the first half of the columns, rows 64..127 only in the second:
    after the first append half the rows are empty (sigma 0, e_row), after the second none is."""
    rng = np.random.default_rng(3)
    M, N = 128, 4000
    rows, cols = [], []
    for m in range(M):
        lo, hi = (0, N // 2) if m < 64 else (N // 2, N)
        c = rng.choice(np.arange(lo, hi), size=40, replace=False)
        rows.append(np.full(c.size, m))
        cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    A = gen.from_coo(M, N, rows, cols, rng.standard_normal(rows.size), dict(name="late"))
    inc = R.Incremental(M, M, max_cols=N // 2, max_nnz=A.nnz)
    inc.append(R.to_device(column_slice(A, 0, N // 2)))
    s, U, info = inc.solve()
    assert info["n_nonempty"] == 64 and info["rank"] == 64
    Ug = U.cpu().numpy()
    for j, m in enumerate(range(64, 128)):
        e = np.zeros(M)
        e[m] = 1.0
        assert np.array_equal(Ug[:, 64 + j], e)
    inc.append(R.to_device(column_slice(A, N // 2, N)))
    s, U, info = inc.solve()
    assert info["n_nonempty"] == 128
    ref = orc.svd(M, N, A.colptr, A.rowidx, A.values, k=M, method="whole")
    check(s, U, info, ref)


def test_warm_started_subspace_iteration(R, orc):
    """1024 rows, k = 64 (block 128): each solve after an append restarts from the previous Ritz
    vectors; the last equals ranky_svd on the whole matrix."""
    A = gen.powerlaw_1m(N=1 << 18, nnz=400_000)
    k = 64
    cuts = np.linspace(0, A.N, 5).astype(int)
    inc = R.Incremental(A.M, k, max_cols=int(np.max(np.diff(cuts))), max_nnz=A.nnz)
    iters = []
    for i in range(4):
        inc.append(R.to_device(column_slice(A, cuts[i], cuts[i + 1])))
        s, U, info = inc.solve()
        iters.append(info["eig_iters"])
    print("subspace iterations per solve:", iters)
    assert all(it > 0 for it in iters)
    assert iters[-1] <= iters[0]         # the warm start pays off once the subspace settles
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="gram", want_v=False)
    err, scaled = check(s, U, info, ref, bar=1e-12)
    whole = R.svd(R.to_device(A), k, 0.0, n_blocks=16)
    assert H.rel_sigma_err(s.cpu().numpy(), whole.sigma.cpu().numpy(), k) <= 1e-12

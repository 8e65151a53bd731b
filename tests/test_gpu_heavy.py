"""The heavy-row split of the Gram (Eq. 2 summed in three parts: the densest rows' block on the
FP64 matrix cores, their pairs with the other rows from gathered rows, the rest in the sparse
walk) against the oracle: G entry-wise past the automatic threshold (FP32 and FP64 values, rows
cut into segments, dense rows before and after the others in row order), the whole path with the
split forced on a small matrix against the oracle's SVD, equal to the path without it up to
rounding, bitwise deterministic and independent of D."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2009_09767_amd import gen
from tests import helpers as H

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def R():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_09767_amd import ranky

    ranky.lib()
    return ranky


def powerlaw(M, N, nnz, s, seed, dtype, kind):
    """Zipf(s) row degrees capped at N (the densest rows fully dense), seeded row order."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = gen.powerlaw_rows(rng, M, N, nnz, s, kind, dtype)
    return gen.from_coo(M, N, rows, cols, vals, dict(name=f"heavy_{M}x{N}"))


def max_row_nnz(A):
    return int(np.bincount(A.rowidx, minlength=A.M).max())


def absgram(orc, A):
    return orc.gram(A.M, A.N, A.colptr, A.rowidx, np.abs(A.values.astype(np.float64)))


CASES = {
    # past the automatic threshold (2^22 nonzeros): the split runs in ranky_gram
    "fp32_512x2^18": lambda: powerlaw(512, 1 << 18, 4_500_000, 1.2, 101, np.float32, "uniform"),
    "fp64_300x2^17": lambda: powerlaw(300, 1 << 17, 4_300_000, 1.1, 102, np.float64, "normal"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_heavy_gram_entrywise(R, orc, name):
    A = CASES[name]()
    assert A.nnz >= 1 << 22
    dA = R.to_device(A)
    G = R.gram(dA).cpu().numpy()
    ref = orc.gram(A.M, A.N, A.colptr, A.rowidx, A.values)
    bound = 2.0 * max_row_nnz(A) * U64 * absgram(orc, A)
    err = np.abs(G - ref)
    print(f"{name}: nnz {A.nnz}, max |G - ref| / bound {np.max(err / np.maximum(bound, 1e-300)):.3f}")
    assert np.all(err <= bound)
    assert np.array_equal(G, G.T)
    assert np.array_equal(G, R.gram(dA).cpu().numpy()), "Gram is not bitwise deterministic"


def small_heavy(dtype=np.float64):
    """96 x 2^15 with ~600k nonzeros: the densest rows full, about 30 rows above the dense
    threshold (4096 nonzeros), the others sparse; two rows emptied (compaction)."""
    A = powerlaw(96, 1 << 15, 600_000, 1.2, 103, dtype, "normal")
    keep = ~np.isin(A.rowidx, [7, 50])
    return gen.drop_entries(A, keep)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_split_forced_whole_path_against_oracle(R, orc, dtype):
    import torch

    A = small_heavy(dtype)
    dA = R.to_device(A)
    k = 40
    on = R.svd(dA, k, 0.0, gram_split="on", eigensolver="jacobi")
    off = R.svd(dA, k, 0.0, gram_split="off", eigensolver="jacobi")
    deg = np.bincount(A.rowidx, minlength=A.M)
    dense = int(np.count_nonzero(deg >= max(4096, A.N // 64)))
    assert dense > 20
    assert on.info["heavy_rows"] == min(32, dense) and off.info["heavy_rows"] == 0
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="whole_qr")
    r = ref.rank
    assert on.info["rank"] == r == off.info["rank"]
    s_on, U_on = on.sigma.cpu().numpy(), on.U.cpu().numpy()
    err = H.rel_sigma_err(s_on, ref.sigma, r)
    scaled, _ = H.vector_errors(U_on[:, :r], ref.U[:, :r], ref.sigma, r)
    print(f"{np.dtype(dtype).name}: rank {r}, sigma err {err:.2e}, U sine x relgap {scaled:.2e}")
    assert err <= 1e-10 and scaled <= 1e-10
    assert H.rel_sigma_err(s_on, off.sigma.cpu().numpy(), r) <= 1e-12
    assert H.canonical_sign_ok(U_on)
    # V = A^T U Sigma^-1 on the split's U
    Vd = on.V.cpu().numpy()
    S = sp.csc_matrix((A.values.astype(np.float64), A.rowidx, A.colptr), shape=(A.M, A.N))
    X = (S.T @ U_on[:, :r]) / s_on[:r]
    assert np.max(np.abs(Vd[:, :r] - X)) <= 1e-10 * max(1.0, np.max(np.abs(X)))
    # an FP32 V from the same split (the heavy back-projection writes either type)
    o32 = R.svd(dA, k, 0.0, gram_split="on", eigensolver="jacobi", v_dtype=torch.float32)
    V32 = o32.V.cpu().numpy().astype(np.float64)
    X32 = (S.T @ o32.U.cpu().numpy()[:, :r]) / o32.sigma.cpu().numpy()[:r]
    assert np.max(np.abs(V32[:, :r] - X32)) <= 2.0 ** -22 * max(1.0, np.max(np.abs(X32)))
    assert np.all(V32[:, r:] == 0.0)
    # bitwise: repeated and for any D (the sums' order is a function of the matrix alone)
    again = R.svd(dA, k, 0.0, gram_split="on", eigensolver="jacobi", n_blocks=7)
    assert torch.equal(again.sigma, on.sigma) and torch.equal(again.U, on.U)


def test_split_with_few_or_no_dense_rows(R, orc):
    """Forced on a matrix with one dense row and on one with none: the split degenerates
    cleanly (a single dense row has only its diagonal in the tiles)."""
    rng = np.random.default_rng(104)
    M, N = 64, 1 << 14
    rows, cols = [], []
    for m in range(M):
        d = N if m == 9 else int(rng.integers(20, 200))
        c = rng.choice(N, size=d, replace=False)
        rows.append(np.full(d, m))
        cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    one = gen.from_coo(M, N, rows, cols, rng.standard_normal(rows.size))
    none = gen.random_sparse(64, 1 << 14, 0.01, seed=105)
    for A, want in ((one, 1), (none, 0)):
        got = R.svd(R.to_device(A), 16, 0.0, gram_split="on", eigensolver="jacobi")
        ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=16, method="whole_qr")
        assert got.info["heavy_rows"] == want
        assert got.info["rank"] == ref.rank
        assert H.rel_sigma_err(got.sigma.cpu().numpy(), ref.sigma, ref.rank) <= 1e-10


@pytest.mark.parametrize("split", ["on", "off"])
def test_result_independent_of_workspace_contents(R, split):
    """Every workspace byte the path reads it wrote first: the results are bitwise equal for a
    workspace cleared to zero, filled with 0.5, or with seeded noise."""
    import torch

    A = small_heavy(np.float64)
    dA = R.to_device(A)
    k = 40
    opts = R.make_opts(gram_split=split, eigensolver="jacobi")
    nb = R.workspace_bytes(A.M, A.N, A.nnz, k, opts)
    outs = []
    for fill in range(3):
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        f = ws[: (nb // 8) * 8].view(torch.float64)
        if fill == 0:
            f.zero_()
        elif fill == 1:
            f.fill_(0.5)
        else:
            g = torch.Generator(device="cuda")
            g.manual_seed(7)
            f.normal_(generator=g)
        o = R.svd(dA, k, 0.0, workspace=ws, gram_split=split, eigensolver="jacobi")
        outs.append((o.sigma.clone(), o.U.clone(), o.V.clone()))
    for s, U, V in outs[1:]:
        assert torch.equal(s, outs[0][0]) and torch.equal(U, outs[0][1]) and torch.equal(V, outs[0][2])


def test_split_with_long_light_columns(R, orc):
    """A few columns with an entry in every row (long columns of the light CSC, walked by many
    rows at once): the split's result equals the oracle's, V included on the long columns (400
    entries each, whose back-projection steps cross its 64-entry window several times)."""
    rng = np.random.default_rng(106)
    M, N = 400, 1 << 14
    A0 = powerlaw(M, N, 300_000, 1.2, 107, np.float64, "normal")
    full = np.array([5, 777, 9000])
    rows = np.concatenate([A0.rowidx, np.tile(np.arange(M), full.size)])
    cols = np.concatenate([np.repeat(np.arange(A0.N), np.diff(A0.colptr)), np.repeat(full, M)])
    flat = np.unique(cols.astype(np.int64) * M + rows)
    cols, rows = flat // M, flat % M
    A = gen.from_coo(M, N, rows, cols, rng.standard_normal(rows.size), dict(name="long_light_cols"))
    k = 24
    got = R.svd(R.to_device(A), k, 0.0, gram_split="on", eigensolver="jacobi")
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="whole_qr")
    assert got.info["heavy_rows"] > 0
    assert got.info["rank"] == ref.rank
    err = H.rel_sigma_err(got.sigma.cpu().numpy(), ref.sigma, ref.rank)
    scaled, _ = H.vector_errors(got.U.cpu().numpy()[:, :ref.rank], ref.U[:, :ref.rank], ref.sigma, ref.rank)
    assert err <= 1e-10 and scaled <= 1e-10
    r = ref.rank
    cols = np.concatenate([full, [0, 1, N - 1]])
    Vs = got.V.cpu().numpy()[cols]
    Vr = ref.V[cols]
    sgn = np.sign(np.sum(Vs[:, :r] * Vr[:, :r], axis=0))
    sgn[sgn == 0] = 1
    vb = np.minimum(1.0, 1e-12 / H.relgaps(ref.sigma, r)) * 4 + 1e-13
    verr = np.max(np.abs(Vs[:, :r] * sgn - Vr[:, :r]), axis=0)
    assert np.all(verr <= vb * np.maximum(np.abs(ref.V[:, :r]).max(axis=0), 1e-300))

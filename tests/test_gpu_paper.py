"""The paper's own procedure on the device: the checkers of Alg. 2-4 bit for bit against the
oracle's, and the proxy route (each block's factors U^i S^i of Eq. 1, P P^T of Eq. 3, the SVD of P)
against the oracle: with no checker it is the oracle's block merge of A (and the Gram-form path's
result), with a checker the oracle's whole-matrix SVD of the repaired A'.  The paper's error sums
e_sigma and e_u (Sec. IV) are checked against their definition, and a small version of the
Tables I-III sweep over D runs for all three checkers."""
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


def cases():
    return {
        "small_deficient": (gen.small_deficient(), 8),
        "random_lonely": (gen.random_sparse(24, 600, 0.01, seed=41), 6),
        "power_law": (gen.powerlaw_small(M=48, N=2048, D=8, k=8, seed=5), 8),
        "standin_small": (gen.paper_standin(M=96, N=6000), 16),
    }


@pytest.mark.parametrize("kind", ["random", "neighbor", "neighbor_random"])
@pytest.mark.parametrize("case", ["small_deficient", "random_lonely", "power_law", "standin_small"])
def test_checker_bit_exact(R, orc, case, kind):
    A, D = cases()[case]
    got, added = R.checker(R.to_device(A), D, kind, seed=2009)
    cp, ri, va, ins = orc.checker(A.M, A.N, A.colptr, A.rowidx, A.values, D, kind, seed=2009)
    assert added == ins > 0
    assert np.array_equal(got.colptr.cpu().numpy(), cp)
    assert np.array_equal(got.rowidx.cpu().numpy(), ri)
    assert np.array_equal(got.values.cpu().numpy(), va)


def test_proxy_route_without_checker_is_the_block_merge(R, orc):
    """No checker: the route is Eq. 1-3 on A itself, equal to the oracle's per-block SVD + proxy +
    SVD of the proxy (its block merge) and to the Gram-form path -- block-rank deficiency needs no repair."""
    A = gen.small_deficient()
    dA = R.to_device(A)
    sg, Ug, info = R.svd_paper(dA, 64, 8, "none", tol=1e-12)
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=64, tol=1e-12, method="merge", D=8)
    r = ref.rank
    assert info["rank"] == r and info["added"] == 0
    assert info["proxy_cols"] >= r
    sg, Ug = sg.cpu().numpy(), Ug.cpu().numpy()
    err = H.rel_sigma_err(sg, ref.sigma, r)
    scaled, _ = H.vector_errors(Ug[:, :r], ref.U[:, :r], ref.sigma, r)
    print(f"no checker: rank {r}, proxy columns {info['proxy_cols']}, sigma err {err:.2e}, U {scaled:.2e}")
    assert err <= 1e-10 and scaled <= 1e-10
    assert np.all(sg[r:] == 0.0)
    assert H.canonical_sign_ok(Ug)
    gram = R.svd(dA, 64, 1e-12, n_blocks=8)
    assert H.rel_sigma_err(gram.sigma.cpu().numpy(), sg, r) <= 1e-10


@pytest.mark.parametrize("kind", ["random", "neighbor", "neighbor_random"])
def test_proxy_route_with_checker_against_the_oracle(R, orc, kind):
    """With a checker the route computes the SVD of A': against the oracle's whole-matrix SVD of its
    own A' (the same bits, by the checker test above), and e_sigma / e_u by their definition."""
    import torch

    A, D = gen.powerlaw_small(M=48, N=2048, D=8, k=8, seed=5), 8
    k = 16
    sg, Ug, info = R.svd_paper(R.to_device(A), k, D, kind, seed=11)
    cp, ri, va, ins = orc.checker(A.M, A.N, A.colptr, A.rowidx, A.values, D, kind, seed=11)
    ref = orc.svd(A.M, A.N, cp, ri, va, k=k, method="whole")
    r = ref.rank
    assert info["added"] == ins and info["nnz_repaired"] == len(ri)
    assert info["rank"] == r
    s_np, U_np = sg.cpu().numpy(), Ug.cpu().numpy()
    err = H.rel_sigma_err(s_np, ref.sigma, r)
    scaled, _ = H.vector_errors(U_np[:, :r], ref.U[:, :r], ref.sigma, r)
    print(f"{kind}: added {ins}, rank {r}, sigma err {err:.2e}, U sine x relgap {scaled:.2e}")
    assert err <= 1e-10 and scaled <= 1e-10
    # e_sigma and e_u (Sec. IV, as read: sign-aligned columns) on the device vs their definition
    es, eu = R.paper_errors(sg, Ug, torch.from_numpy(ref.sigma[:k]).cuda(), torch.from_numpy(ref.U[:, :k]).cuda())
    assert abs(es - H.paper_e_sigma(s_np, ref.sigma, k)) <= 1e-12 * max(1.0, es)
    assert abs(eu - H.paper_e_u(U_np, ref.U, k)) <= 1e-12 * max(1.0, eu)


def test_tables_sweep_small(R):
    """The Tables I-III protocol at a reduced size: for each checker and D, the proxy route against the
    Gram-form path on the same repaired A' (the FP64 path): e_sigma and e_u small, ranks equal."""
    import torch

    A = gen.paper_standin(M=96, N=12000)
    dA = R.to_device(A)
    k = 10
    for kind in ("random", "neighbor", "neighbor_random"):
        for D in (2, 8, 32):
            sg, Ug, info = R.svd_paper(dA, k, D, kind, seed=D)
            rep, added = R.checker(dA, D, kind, seed=D)
            ref = R.svd(rep, k, 0.0, n_blocks=D)
            es, eu = R.paper_errors(sg, Ug, ref.sigma, ref.U)
            print(f"{kind:16s} D={D:3d}: added {added:6d}  e_sigma {es:.3e}  e_u {eu:.3e}", flush=True)
            assert info["added"] == added
            assert info["rank"] == ref.info["rank"]
            assert es <= 1e-10 * float(ref.sigma.sum())


@pytest.mark.parametrize("D", [2, 3, 5])
def test_proxy_route_full_rank_blocks(R, orc, D):
    """Every block of full rank M with D M not a multiple of 16: P^T has D M rows, and the P P^T
    product reads them padded to a multiple of 16.  The route equals the oracle's block merge and
    does not depend on the workspace's prior contents."""
    import ctypes
    import torch

    A = gen.random_sparse(37, 6000, 0.05, seed=43)
    dA = R.to_device(A)
    k = 12
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="merge", D=D)
    nb = int(R.lib().ranky_paper_workspace_bytes(A.M, A.N, A.nnz, k, D, -1))
    outs = []
    for fill in (0.0, 0.5, 1e30):
        ws = torch.full(((nb + 7) // 8,), fill, dtype=torch.float64, device="cuda")
        sigma = torch.empty(k, dtype=torch.float64, device="cuda")
        U = torch.empty((A.M, k), dtype=torch.float64, device="cuda")
        info = R.PaperInfo()
        csc = dA.struct()
        R._check(R.lib().ranky_svd_paper(R.context(0).handle, ctypes.byref(csc), A.M, A.N, k, D, -1, 0, 0.0,
                                         R._ptr(ws), nb, R._ptr(sigma), R._ptr(U), ctypes.byref(info), None))
        assert info.proxy_cols == D * A.M
        outs.append((sigma.cpu().numpy(), U.cpu().numpy()))
    r = ref.rank
    for s, U in outs:
        assert H.rel_sigma_err(s, ref.sigma, r) <= 1e-10
        scaled, _ = H.vector_errors(U[:, :r], ref.U[:, :r], ref.sigma, r)
        assert scaled <= 1e-10
        assert np.array_equal(s, outs[0][0]) and np.array_equal(U, outs[0][1])

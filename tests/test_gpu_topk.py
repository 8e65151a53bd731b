"""The k leading eigenpairs of G by Chebyshev-filtered subspace iteration (opts.eigensolver),
against the oracle: the same bars as the full Jacobi path (relative sigma <= 1e-10, per-cluster
sine x relgap <= 1e-12, exact rank, V, sign rule), on power-law matrices, a graded spectrum of
known factors, ragged sizes, a block wider than the rank of G, the FP32 Gram with refinement,
and the fallback to the full Jacobi when the block is too wide for the rows."""
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


def compare(A, got, ref, k, sig_bar=1e-10, vec_bar=1e-12):
    sg, Ug = got.sigma.cpu().numpy(), got.U.cpu().numpy()
    r = ref.rank
    assert got.info["rank"] == r, (got.info["rank"], r)
    err = H.rel_sigma_err(sg, ref.sigma, r)
    scaled, worst = H.vector_errors(Ug[:, :r], ref.U[:, :r], ref.sigma, r)
    print(f"M={A.M} k={k}: eig_iters {got.info['eig_iters']} sweeps {got.info['sweeps']}; sigma err {err:.2e}, "
          f"U sine x relgap {scaled:.2e} (worst sine {worst:.2e})", flush=True)
    assert err <= sig_bar
    assert np.all(sg[r:] == 0.0)
    assert scaled <= vec_bar
    assert H.canonical_sign_ok(Ug)
    m = min(k, A.M)
    assert np.linalg.norm(Ug[:, :m].T @ Ug[:, :m] - np.eye(m)) <= 1e-12 * max(1, m)
    if ref.V is not None:
        Vg = got.V.double().cpu().numpy()
        scaled_v, _ = H.vector_errors(Vg[:, :r], ref.V[:, :r], ref.sigma, r)
        import torch

        assert scaled_v <= max(vec_bar, 2.0 ** -22 if got.V.dtype != torch.float64 else 0.0)
        assert np.all(Vg[:, r:] == 0.0)


def graded_known_factors(M=512, N=8192, kappa=1e6, seed=5):
    s = np.geomspace(1.0, 1.0 / kappa, M)
    A, _, _, _ = gen.known_factors(s, N, seed=seed)
    return A


CASES = {
    # name: (matrix, k, oracle method)
    "powerlaw_small_k32": (lambda: gen.powerlaw_small(), 32, "whole"),
    "ragged_300_k40": (lambda: gen.random_sparse(300, 6000, 0.01, seed=300), 40, "whole_qr"),
    "graded_512_k32": (lambda: graded_known_factors(), 32, "whole_qr"),
    "batch_member_487_k100": (lambda: sorted(gen.batch_mixed(count=40), key=lambda A: -A.M)[0], 100, "whole_qr"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_subspace_against_oracle(R, orc, name):
    mk, k, method = CASES[name]
    A = mk()
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method=method)
    got = R.svd(R.to_device(A), k, 0.0, eigensolver="subspace")
    assert got.info["eig_iters"] > 0 and got.info["sweeps"] == 0
    compare(A, got, ref, k)


def test_subspace_powerlaw_1m_full_size(R, orc):
    """1024 x 2^20 (k = 128, block 192): all 128 sigmas and U against the oracle's Gram route."""
    A = gen.powerlaw_1m()
    k = 128
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="gram", want_v=False)
    got = R.svd(R.to_device(A), k, 0.0, n_blocks=64, eigensolver="subspace")
    assert got.info["eig_iters"] > 0
    compare(A, got, ref, k)


def test_subspace_block_wider_than_the_rank(R, orc):
    """G of rank 40 with 512 non-empty rows, k = 32 (block 64): the block holds null directions of
    G; the 32 leading pairs still converge.  Checked against the closed form (the known factors)
    and the oracle's Gram route.  (The oracle's QR-preconditioned one-sided Jacobi is itself only
    good to 2.9e-11 in sine x relgap on this exactly rank-deficient dense matrix, so it is not
    the reference here.)"""
    from types import SimpleNamespace

    s = np.concatenate([np.geomspace(10.0, 1.0, 40), np.zeros(472)])
    A, U, _, V = gen.known_factors(s, 8192, seed=9)
    got = R.svd(R.to_device(A), 32, 0.0, eigensolver="subspace")
    assert got.info["eig_iters"] > 0
    exact = SimpleNamespace(rank=32, sigma=s, U=U, V=V)
    compare(A, got, exact, 32)
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=32, method="gram")
    compare(A, got, ref, 32)


def test_subspace_mixed_with_refinement(R, orc):
    """FP32 Gram, subspace iteration to the FP32 level, one FP64 Rayleigh-Ritz step: sigma at the FP64
    bar (the Ritz values are second-order accurate), vectors at the mixed bar."""
    import torch

    A = gen.powerlaw_small(dtype=np.float32)
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=32, method="whole")
    got = R.svd(R.to_device(A), 32, 0.0, gram_prec="fp32", refine=1, v_dtype=torch.float32, eigensolver="subspace")
    assert got.info["eig_iters"] > 0 and got.info["rr_sweeps"] > 0
    compare(A, got, ref, 32, sig_bar=1e-10, vec_bar=1e-6)


def test_subspace_falls_back_when_the_block_is_too_wide(R, orc):
    """200 of 400 rows empty (M' = 200) with k = 50 (block 128 > M'/2): the full Jacobi runs."""
    A = gen.batch_matrix(np.random.Generator(np.random.PCG64(4)), 400, 20000, 0.01, zero_half=True)
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=50, method="whole_qr")
    got = R.svd(R.to_device(A), 50, 0.0, eigensolver="subspace")
    assert got.info["eig_iters"] == 0 and got.info["sweeps"] > 0
    compare(A, got, ref, 50)


def test_subspace_is_deterministic_and_auto_selects(R):
    """Two calls give the same bits; the automatic choice takes the subspace iteration when the block
    is at most an eighth of the rows (1024 rows, k = 64: block 128) and the full Jacobi otherwise."""
    import torch

    A = gen.powerlaw_1m(N=1 << 18, nnz=400_000)
    dA = R.to_device(A)
    a = R.svd(dA, 64, 0.0, n_blocks=16)
    b = R.svd(dA, 64, 0.0, n_blocks=16)
    assert a.info["eig_iters"] > 0
    assert torch.equal(a.sigma, b.sigma) and torch.equal(a.U, b.U) and torch.equal(a.V, b.V)
    c = R.svd(dA, 200, 0.0, n_blocks=16)   # block 320 > 256: the full Jacobi
    assert c.info["eig_iters"] == 0 and c.info["sweeps"] > 0
    j = R.svd(dA, 64, 0.0, n_blocks=16, eigensolver="jacobi")
    assert j.info["eig_iters"] == 0
    r = a.info["rank"]
    assert np.max(np.abs(a.sigma.cpu().numpy()[:r] - j.sigma.cpu().numpy()[:r]) / j.sigma.cpu().numpy()[:r]) <= 1e-12

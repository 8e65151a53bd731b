"""The 200M-nonzero power-law matrix at full size (4096 x 2^24, Zipf(1.2) rows, 256 column blocks,
k = 100), pinned to the oracle: tests/golden/powerlaw_200m_top100.npz holds the oracle's top-100
sigma and U by its Gram route (FP64 sparse Gram, cyclic two-sided Jacobi, the rank rule, the sign
rule), written by oracle/make_golden_powerlaw_200m.py, which calls only the oracle and the seeded
generator, and keyed by the SHA-256 of the generated CSC bytes.

Checked on the FP64 path (the paper's arithmetic) and the mixed path (FP32 Gram, FP64 eigensolve and
Rayleigh-Ritz, FP32 V): sigma against the golden (1e-10 / 1e-6 relative), U against the golden by
per-cluster principal angles (sine x relgap <= 1e-12 / 1e-6), the eigen-residual
||A (A^T u_i) - sigma_i^2 u_i|| / sigma_1^2 with A A^T applied by torch's own sparse products (not
this library's), and V on sampled columns against the oracle's back-projection of the golden U."""
import os

import numpy as np
import pytest

from paper_2009_09767_amd import gen
from tests import helpers as H

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]   # generation takes up to a minute

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "powerlaw_200m_top100.npz")


@pytest.fixture(scope="module")
def R():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_09767_amd import ranky

    ranky.lib()
    return ranky


@pytest.fixture(scope="module")
def case(R):
    import hashlib

    import torch

    gold = np.load(GOLDEN, allow_pickle=False)
    A = gen.powerlaw_200m(progress=lambda m: print(m, flush=True))
    h = hashlib.sha256()
    for a in (A.colptr, A.rowidx, A.values):
        h.update(np.ascontiguousarray(a).tobytes())
    assert h.hexdigest() == str(gold["csc_sha256"]), "the generator no longer draws the golden's matrix"
    print(f"powerlaw_200m: M={A.M} N={A.N} nnz={A.nnz}", flush=True)
    dA = R.to_device(A)
    # A as CSR (rows) by torch's own conversion, for A Z in the eigen-residual
    A_csr = torch.sparse_csc_tensor(dA.colptr.long(), dA.rowidx.long(), dA.values.double(),
                                    size=(A.M, A.N)).to_sparse_csr()
    At = torch.sparse_csr_tensor(dA.colptr.long(), dA.rowidx.long(), dA.values.double(), size=(A.N, A.M))
    yield A, dA, gold, A_csr, At
    del dA, A_csr, At
    torch.cuda.empty_cache()


def eigen_residual(A_csr, At, U, sig):
    """max_i ||A (A^T u_i) - sigma_i^2 u_i|| / sigma_1^2 in FP64 (torch sparse products)."""
    import torch

    Z = torch.sparse.mm(At, U)
    Y = torch.sparse.mm(A_csr, Z)
    r = torch.linalg.vector_norm(Y - U * (sig * sig)[None, :], dim=0)
    return (r.max() / (sig[0] * sig[0])).item()


def check_against_golden(A, gold, got, k, sig_bar, vec_bar, res_bar, A_csr, At, orc=None):
    import torch

    info = got.info
    print("info", {n: info[n] for n in ("status", "rank", "sweeps", "eig_iters", "rr_sweeps", "tau", "sigma_max")},
          flush=True)
    assert info["status"] == 0
    assert info["n_nonempty"] == int(gold["n_nonempty"]) == A.M   # rows are emptied inside blocks only
    r = int(gold["rank"])
    assert info["rank"] == r == k
    sg = got.sigma.cpu().numpy()
    err = H.rel_sigma_err(sg, gold["sigma"], r)
    Ug = got.U.cpu().numpy()
    scaled, worst = H.vector_errors(Ug, gold["U"], gold["sigma"], r)
    res = eigen_residual(A_csr, At, got.U, got.sigma)
    orth = np.linalg.norm(Ug.T @ Ug - np.eye(k))
    print(f"sigma err {err:.3e} (bar {sig_bar:g}); U sine x relgap {scaled:.3e} (bar {vec_bar:g}), worst sine "
          f"{worst:.3e}; eigen-residual {res:.3e} (bar {res_bar:g}); ||U^T U - I|| {orth:.3e}", flush=True)
    assert err <= sig_bar
    assert scaled <= vec_bar
    assert res <= res_bar
    assert orth <= 1e-10
    assert H.canonical_sign_ok(Ug)
    # V on a seeded sample of columns: the oracle's back-projection of the golden U and sigma
    if orc is not None:
        cols = np.sort(np.random.default_rng(11).choice(A.N, 4096, replace=False))
        counts = np.diff(A.colptr)[cols]
        starts = A.colptr[cols]
        idx = np.concatenate([np.arange(s, s + c) for s, c in zip(starts, counts)])
        sub_colptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        Vs_ref = orc.backproject(A.M, cols.size, sub_colptr, A.rowidx[idx], A.values[idx].astype(np.float64),
                                 gold["U"], gold["sigma"], r)
        Vs = got.V[torch.from_numpy(cols).to(got.V.device)].double().cpu().numpy()
        sgn = np.sign(np.sum(Vs * Vs_ref, axis=0))
        sgn[sgn == 0] = 1
        verr = np.max(np.abs(Vs * sgn - Vs_ref), axis=0) / np.maximum(np.abs(Vs_ref).max(axis=0), 1e-300)
        gaps = H.relgaps(gold["sigma"], r)
        vbar = np.minimum(1.0, vec_bar / gaps) * 4 + (1e-6 if got.V.dtype == torch.float32 else 1e-13)
        print(f"V sampled columns: worst entry error / column max {verr.max():.3e}", flush=True)
        assert np.all(verr <= vbar)


@pytest.mark.parametrize("eigensolver", ["auto", "jacobi"])
def test_powerlaw_200m_fp64_against_golden(R, case, orc, eigensolver):
    """The FP64 path (FP64 Gram of the FP32 values, promoted exactly; FP64 V), with the leading
    eigenpairs by the automatic choice (the subspace iteration here) and by the full Jacobi.  The
    eigen-residual bar is 1e-11: the Gram and the eigensolve each round at about n eps = 4.5e-13."""
    import torch

    A, dA, gold, A_csr, At = case
    k, D = A.meta["k"], A.meta["D"]
    got = R.svd(dA, k, 0.0, n_blocks=D, gram_prec="fp64", v_dtype=torch.float64, eigensolver=eigensolver)
    assert (got.info["eig_iters"] > 0) == (eigensolver == "auto")
    check_against_golden(A, gold, got, k, 1e-10, 1e-12, 1e-11, A_csr, At, orc)
    assert got.info["rr_sweeps"] == 0
    del got
    torch.cuda.empty_cache()


def test_powerlaw_200m_mixed_against_golden(R, case, orc):
    """The mixed path: FP32 Gram, FP64 eigensolve and one FP64 Rayleigh-Ritz step, FP32 V."""
    import torch

    A, dA, gold, A_csr, At = case
    k, D = A.meta["k"], A.meta["D"]
    got = R.svd(dA, k, 0.0, n_blocks=D, gram_prec="fp32", refine=1, v_dtype=torch.float32)
    check_against_golden(A, gold, got, k, 1e-6, 1e-6, 1e-6, A_csr, At, orc)
    assert got.info["rr_sweeps"] > 0
    del got
    torch.cuda.empty_cache()

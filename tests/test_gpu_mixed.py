"""Mixed-precision path (FP32 Gram accumulation, FP64 eigensolve, one FP64 Rayleigh-Ritz step
with the exact operator, FP32 V) against the FP64 CPU oracle.  Bar: relative sigma error
<= 1e-6; vectors sin(angle) <= min(1, 1e-6 / relgap); exact rank; zeros beyond the rank."""
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


@pytest.fixture(scope="module")
def orc():
    import oracle

    oracle._load()
    return oracle


CASES = {
    "powerlaw_small_f32": lambda: gen.powerlaw_small(dtype=np.float32),
    "batch_mixed_full_rank": lambda: [A for A in gen.batch_mixed(count=6, deficient_frac=0.5) if not A.meta["zeroed_rows"].size][0],
    "batch_mixed_half_rows_zero": lambda: [A for A in gen.batch_mixed(count=6, deficient_frac=0.5) if A.meta["zeroed_rows"].size][0],
    "small_deficient_f64": lambda: gen.small_deficient(),
}


def check(A, got, ref, bar):
    import torch

    sg, Ug = got.sigma.cpu().numpy(), got.U.cpu().numpy()
    Vg = got.V.to(torch.float64).cpu().numpy()
    r = ref.rank
    assert got.info["rank"] == r
    err = H.rel_sigma_err(sg, ref.sigma, r)
    assert err <= bar, err
    assert np.all(sg[r:] == 0.0)
    scaled, _ = H.vector_errors(Ug[:, :r], ref.U[:, :r], ref.sigma, r)
    assert scaled <= bar
    scaled_v, _ = H.vector_errors(Vg[:, :r], ref.V[:, :r], ref.sigma, r)
    assert scaled_v <= max(bar, 2.0 ** -22)   # V is stored in FP32
    assert np.all(Vg[:, r:] == 0.0)
    assert H.canonical_sign_ok(Ug)
    return err


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_refined_against_fp64_oracle(R, orc, name):
    import torch

    A = CASES[name]()
    k = min(A.meta.get("k", A.M), A.M, 64)
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="whole_qr" if A.M > 64 else "whole")
    got = R.svd(R.to_device(A), k, 0.0, n_blocks=min(A.meta.get("D", 8), A.N), gram_prec="fp32", refine=1,
                v_dtype=torch.float32)
    err = check(A, got, ref, 1e-6)
    # the Ritz values come from the exact operator in FP64: far inside the mixed bar
    assert err <= 1e-10


@pytest.mark.parametrize("k", [77, 129, 300])
def test_refine_tiles_and_odd_k(R, orc, k):
    """The Rayleigh-Ritz H = Z^T Z over one tile (odd k: U0 rows are not 16-byte aligned),
    two tiles (one off-diagonal tile) and three tiles of H."""
    import torch

    A = gen.random_sparse(320, 30000, 0.01, seed=21, dtype=np.float32)
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="whole_qr")
    got = R.svd(R.to_device(A), k, 0.0, n_blocks=8, gram_prec="fp32", refine=1, v_dtype=torch.float32)
    err = check(A, got, ref, 1e-6)
    assert err <= 1e-10


def test_refine_dense_columns(R, orc):
    """Columns with ~100 nonzeros: a 16-column chunk holds more nonzeros than the
    Rayleigh-Ritz kernel stages in LDS, so the rest are read from memory."""
    import torch

    A = gen.random_sparse(320, 4000, 0.3, seed=22, dtype=np.float32)
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=64, method="whole_qr")
    got = R.svd(R.to_device(A), 64, 0.0, n_blocks=8, gram_prec="fp32", refine=1, v_dtype=torch.float32)
    err = check(A, got, ref, 1e-6)
    assert err <= 1e-10


def test_mixed_without_refinement_meets_the_mixed_bar(R, orc):
    import torch

    A = CASES["batch_mixed_full_rank"]()
    k = 32
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="whole_qr")
    got = R.svd(R.to_device(A), k, 0.0, n_blocks=8, gram_prec="fp32", refine=0, v_dtype=torch.float32)
    check(A, got, ref, 1e-6)


def test_mixed_is_deterministic(R):
    import torch

    A = gen.powerlaw_small(dtype=np.float32)
    dA = R.to_device(A)
    a = R.svd(dA, 32, 0.0, n_blocks=8, gram_prec="fp32", refine=1, v_dtype=torch.float32)
    b = R.svd(dA, 32, 0.0, n_blocks=8, gram_prec="fp32", refine=1, v_dtype=torch.float32)
    assert torch.equal(a.sigma, b.sigma) and torch.equal(a.U, b.U) and torch.equal(a.V, b.V)


def test_refine_rejects_large_k(R):
    A = gen.random_sparse(1100, 3000, 0.002, seed=5, dtype=np.float32)
    with pytest.raises(R.RankyError) as e:
        R.svd(R.to_device(A), 1100, 0.0, gram_prec="fp32", refine=1)
    assert e.value.status == R.E_INVALID


def test_bf16x3_refined_against_fp64_oracle(R, orc):
    """Split-bf16 dense tiles (relative product error ~2^-16) plus the FP64 Rayleigh-Ritz
    step with the exact operator: sigma within the mixed bar of the FP64 oracle."""
    import torch

    from tests.test_gpu_dense_tiles import dense_rows_matrix

    A = dense_rows_matrix(np.float32)
    k = 32
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="whole_qr")
    got = R.svd(R.to_device(A), k, 0.0, n_blocks=8, gram_prec="bf16x3", refine=1, v_dtype=torch.float32)
    check(A, got, ref, 1e-6)


def test_bf16x3_with_the_c_default_refine(R, orc):
    """gram_prec BF16X3 with every other option at the C default (refine = -1, automatic): the
    call refines (one FP64 Rayleigh-Ritz step), so rank and sigma match the FP64 oracle."""
    import torch

    A = gen.powerlaw_small()
    k = A.meta["k"]
    got = R.svd(R.to_device(A), k, 0.0, gram_prec="bf16x3", v_dtype=torch.float32)   # refine left to the library
    assert got.info["rr_sweeps"] > 0
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="whole")
    assert got.info["rank"] == ref.rank
    assert H.rel_sigma_err(got.sigma.cpu().numpy(), ref.sigma, ref.rank) <= 1e-10


def test_bf16x3_unrefined_without_dense_rows_uses_the_fp32_threshold(R, orc):
    """Unrefined BF16X3 on a matrix with no row dense enough for the split-bf16 tiles: the whole
    Gram is the FP32 sparse pass, so tau must be sqrt(M' 2^-24) sigma_1 (not 2^-16) and the rank
    equals the oracle's with that roundoff."""
    import torch

    A = gen.powerlaw_small(seed=901, M=192, N=1 << 13, k=192)
    assert np.bincount(A.rowidx, minlength=A.M).max() < 4096     # below the dense-row threshold
    got = R.svd(R.to_device(A), A.M, 0.0, gram_prec="bf16x3", refine=0, v_dtype=torch.float32)
    ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=A.M, method="gram", u_gram=2.0 ** -24)
    n = got.info["n_nonempty"]
    assert got.info["tau"] <= np.sqrt(n * 2.0 ** -24) * got.info["sigma_max"] * (1 + 1e-12)
    assert got.info["rank"] == ref.rank == A.M

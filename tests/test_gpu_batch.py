"""Batched path (ranky_batch): many independent matrices of different sizes in one launch per
phase.  Every matrix must give exactly the bits it gives alone through ranky_svd (the kernels
read only their own matrix; the batch only changes the grid), and must match the oracle."""
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


def small_batch(count=12):
    """batch_mixed's recipe at reduced sizes so the oracle checks every member."""
    return gen.batch_mixed(seed=77, count=count, M_range=(20, 150), N_range=(1500, 6000), density=0.01,
                    deficient_frac=0.25)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_alone_and_oracle(R, orc, graph):
    import torch

    mats = small_batch()
    dms = [R.to_device(A) for A in mats]
    ks = [A.M for A in mats]
    Ds = [int(A.meta["D"]) for A in mats]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = R.batch(dms, ks, 0.0, n_blocks=Ds, graph=graph)
        outs2 = R.batch(dms, ks, 0.0, n_blocks=Ds, graph=graph)   # replay (graph reused)
    stream.synchronize()
    for A, dA, k, D, o, o2 in zip(mats, dms, ks, Ds, outs, outs2):
        assert o.info["status"] == 0
        alone = R.svd(dA, k, 0.0, n_blocks=D)
        assert torch.equal(o.sigma, alone.sigma)
        assert torch.equal(o.U, alone.U)
        assert torch.equal(o.V, alone.V)
        assert torch.equal(o2.sigma, o.sigma) and torch.equal(o2.U, o.U) and torch.equal(o2.V, o.V)
        assert o.info["rank"] == alone.info["rank"] and o.info["sweeps"] == alone.info["sweeps"]
        ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=k, method="whole_qr")
        r = ref.rank
        assert o.info["rank"] == r == A.M - A.meta["zeroed_rows"].size
        assert H.rel_sigma_err(o.sigma.cpu().numpy(), ref.sigma, r) <= 1e-10


def test_batch_isolates_a_broken_member(R):
    import torch

    mats = small_batch(5)
    dms = [R.to_device(A) for A in mats]
    bad = mats[2]
    ri = bad.rowidx.copy()
    ri[0] = bad.M + 3
    dms[2].rowidx = torch.from_numpy(ri).cuda()
    outs = R.batch(dms, [A.M for A in mats], 0.0, check=False)
    assert outs[2].info["status"] == R.E_CSC
    for i in (0, 1, 3, 4):
        assert outs[i].info["status"] == 0
        alone = R.svd(dms[i], mats[i].M, 0.0)
        assert torch.equal(outs[i].sigma, alone.sigma)


def test_batch_mixed_precision(R, orc):
    import torch

    mats = small_batch(6)
    dms = [R.to_device(A) for A in mats]
    outs = R.batch(dms, [A.M for A in mats], 0.0, gram_prec="fp32", v_dtype=torch.float32)
    for A, o in zip(mats, outs):
        ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=A.M, method="whole_qr", u_gram=2.0 ** -24)
        r = ref.rank
        assert o.info["rank"] == r
        assert H.rel_sigma_err(o.sigma.cpu().numpy(), ref.sigma, r) <= 1e-6

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


def full_size_members():
    """Eight members of the 256-matrix batch at their real sizes: the two largest (M x N), two
    half-rank members with M > 256 (k > 256: four output pairs per lane in the back-projection),
    two half-rank members with M <= 256 and two more of M > 256."""
    mats = gen.batch_mixed()
    Ms = np.array([A.M for A in mats])
    area = np.array([A.M * A.N for A in mats])
    deficient = [i for i, A in enumerate(mats) if A.meta["zeroed_rows"].size]
    pick = [int(i) for i in np.argsort(-area)[:2]]
    pick += [i for i in deficient if Ms[i] > 256 and i not in pick][:2]
    pick += [i for i in deficient if Ms[i] <= 256 and i not in pick][:2]
    pick += [i for i in range(len(mats)) if Ms[i] > 256 and i not in pick and i not in deficient][:2]
    return [mats[i] for i in pick]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_full_size_members_against_oracle(R, orc, prec):
    """ranky_batch on members at the batched workload's real sizes (M up to 512, N up to 1e5,
    k = M, half-rank members) against the oracle's whole-matrix QR-preconditioned Jacobi SVD:
    sigma at 1e-10 (FP64 Gram) or 1e-6 (FP32 Gram), exact rank, U by cluster angles, V on
    sampled columns, and bitwise the result of ranky_svd alone."""
    from concurrent.futures import ThreadPoolExecutor

    import torch

    mats = full_size_members()
    assert any(A.M > 256 and A.meta["zeroed_rows"].size for A in mats)
    print("members (M, N, nnz, zeroed):", [(A.M, A.N, A.nnz, int(A.meta["zeroed_rows"].size)) for A in mats], flush=True)
    dms = [R.to_device(A) for A in mats]
    ks = [A.M for A in mats]
    Ds = [int(A.meta["D"]) for A in mats]
    vdt = torch.float64 if prec == "fp64" else torch.float32
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        outs = R.batch(dms, ks, 0.0, n_blocks=Ds, gram_prec=prec, v_dtype=vdt, graph=True)
    stream.synchronize()
    u_g = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    with ThreadPoolExecutor(max_workers=4) as ex:
        refs = list(ex.map(lambda A: orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=A.M, method="whole_qr",
                                             u_gram=u_g), mats))
    bar = 1e-10 if prec == "fp64" else 1e-6
    for A, dA, D, o, ref in zip(mats, dms, Ds, outs, refs):
        r = ref.rank
        assert o.info["status"] == 0
        assert o.info["rank"] == r == A.M - A.meta["zeroed_rows"].size
        sg, Ug = o.sigma.cpu().numpy(), o.U.cpu().numpy()
        err = H.rel_sigma_err(sg, ref.sigma, r)
        scaled, worst = H.vector_errors(Ug[:, :r], ref.U[:, :r], ref.sigma, r)
        print(f"M={A.M} N={A.N} rank={r}: sigma err {err:.2e}, U sine x relgap {scaled:.2e}", flush=True)
        assert err <= bar
        assert np.all(sg[r:] == 0.0)
        assert scaled <= (1e-12 if prec == "fp64" else 1e-6)
        cols = np.sort(np.random.default_rng(3).choice(A.N, 512, replace=False))
        Vs = o.V[torch.from_numpy(cols).to(o.V.device)].double().cpu().numpy()
        Vr = ref.V[cols]
        sgn = np.sign(np.sum(Vs[:, :r] * Vr[:, :r], axis=0))
        sgn[sgn == 0] = 1
        gaps = H.relgaps(ref.sigma, r)
        vb = np.minimum(1.0, (1e-12 if prec == "fp64" else 1e-6) / gaps) * 4 + (1e-13 if prec == "fp64" else 1e-6)
        verr = np.max(np.abs(Vs[:, :r] * sgn - Vr[:, :r]), axis=0)
        assert np.all(verr <= vb * np.maximum(np.abs(ref.V[:, :r]).max(axis=0), 1e-300))
        assert np.all(Vs[:, r:] == 0.0)
        alone = R.svd(dA, A.M, 0.0, n_blocks=D, gram_prec=prec, refine=0, v_dtype=vdt)
        assert torch.equal(o.sigma, alone.sigma) and torch.equal(o.U, alone.U) and torch.equal(o.V, alone.V)


def test_batch_bf16x3_uses_the_fp32_threshold(R, orc):
    """A batch has no split-bf16 tiles, so gram_prec BF16X3 computes an FP32 Gram and its rank rule
    must use the FP32 roundoff (tau = sqrt(M' 2^-24) sigma_1): every member's rank equals the
    oracle's, with power-law members whose small singular values sit far below sqrt(M' 2^-16) sigma_1."""
    import torch

    mats = [gen.powerlaw_small(seed=900 + i, M=128 + 64 * i, N=1 << 13, k=128 + 64 * i) for i in range(3)]
    mats += small_batch(4)
    dms = [R.to_device(A) for A in mats]
    ks = [A.M for A in mats]
    outs = R.batch(dms, ks, 0.0, gram_prec="bf16x3", v_dtype=torch.float32)
    between = 0
    for A, o in zip(mats, outs):
        ref = orc.svd(A.M, A.N, A.colptr, A.rowidx, A.values, k=A.M, method="gram", u_gram=2.0 ** -24)
        n = o.info["n_nonempty"]
        tau16 = np.sqrt(n * 2.0 ** -16) * ref.sigma[0]
        tau24 = np.sqrt(n * 2.0 ** -24) * ref.sigma[0]
        between += int(np.sum((ref.sigma > tau24) & (ref.sigma <= tau16)))
        print(f"M={A.M}: rank {o.info['rank']} oracle {ref.rank}", flush=True)
        assert o.info["rank"] == ref.rank
        assert o.info["tau"] <= np.sqrt(n * 2.0 ** -24) * o.info["sigma_max"] * (1 + 1e-12)
        # an unrefined FP32 Gram moves lambda_i by about n u_32 lambda_1, so sigma_i by about
        # n u_32 sigma_1^2 / (2 sigma_i): bound it with a factor 8 of room
        r = ref.rank
        sg = o.sigma.cpu().numpy()[:r]
        assert np.all(np.abs(sg - ref.sigma[:r]) <= 8 * n * 2.0 ** -24 * ref.sigma[0] ** 2 / ref.sigma[:r])
    # the members do tell the two thresholds apart: 126 singular values lie between them
    assert between > 100, between

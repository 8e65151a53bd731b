"""Serving (ranky_serve_*): requests of different M, N, nnz arrive while others run, are admitted
by their HBM footprint as slots and arena memory free up, overlap on the device, and each result
is bitwise the result of ranky_svd alone."""
import time

import numpy as np
import pytest

from paper_2009_09767_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_09767_amd import ranky

    ranky.lib()
    return ranky


def request_pool(count=10, seed=31):
    reqs = gen.cfg4_requests(seed=seed, duration_s=1.0)[:count]
    out = []
    for r in reqs:
        # smaller N so the test stays short; the recipe is cfg4's (Zipf rows, U(-1,1) FP32)
        r.N = min(r.N, 1 << 15)
        r.nnz = min(r.nnz, 40 * r.N)
        out.append(gen.cfg4_matrix(r))
    return out


def alloc_out(R, torch, A, k, vdt):
    return R.SVDResult(torch.empty(k, dtype=torch.float64, device="cuda"),
                       torch.empty((A.M, k), dtype=torch.float64, device="cuda"),
                       torch.empty((A.N, k), dtype=vdt, device="cuda"), {})


def test_mix_equals_alone(R):
    import torch

    mats = request_pool()
    dms = [R.to_device(A) for A in mats]
    ks = [min(A.M, 64) for A in mats]
    srv = R.Server(arena_bytes=1 << 30, max_slots=4, max_queue=64)
    outs = [alloc_out(R, torch, A, k, torch.float64) for A, k in zip(mats, ks)]
    tickets = []
    for i, (dA, k, o) in enumerate(zip(dms, ks, outs)):
        st, t = srv.submit(dA, k, o)
        assert st == R.OK
        tickets.append(t)
        time.sleep(0.002 * (i % 3))           # arrivals while earlier requests run
    for t in tickets:
        st, info = srv.wait(t, 60_000_000)
        assert st == R.OK, (st, info)
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(mats) and stats["failed"] == 0
    assert stats["peak_running"] >= 2          # requests really overlapped on the device
    assert stats["p99_us"] >= stats["p50_us"] > 0
    for dA, k, o in zip(dms, ks, outs):
        alone = R.svd(dA, k, 0.0)
        assert torch.equal(o.sigma, alone.sigma)
        assert torch.equal(o.U, alone.U)
        assert torch.equal(o.V, alone.V)


def test_admission_by_footprint(R):
    """An arena that holds about two requests at a time: never more admitted than fit, all complete."""
    import torch

    mats = request_pool(8, seed=5)
    dms = [R.to_device(A) for A in mats]
    ks = [min(A.M, 64) for A in mats]
    probe = R.Server(arena_bytes=1 << 20, max_slots=1, max_queue=4)
    foot = [probe.footprint(dA, k) + 4 * (A.N + 1) + 8 * A.nnz + 1024 for A, dA, k in zip(mats, dms, ks)]
    probe.close()
    arena = int(2.2 * max(foot))
    srv = R.Server(arena_bytes=arena, max_slots=8, max_queue=64)
    outs = [alloc_out(R, torch, A, k, torch.float64) for A, k in zip(mats, ks)]
    tickets = [srv.submit(dA, k, o)[1] for dA, k, o in zip(dms, ks, outs)]
    for t in tickets:
        assert srv.wait(t, 60_000_000)[0] == R.OK
    st = srv.stats()
    srv.close()
    assert st["arena_peak_bytes"] <= arena
    assert st["completed"] == len(mats)
    assert st["peak_running"] <= 3


def test_back_pressure_cancel_and_isolation(R):
    import torch

    mats = request_pool(6, seed=9)
    dms = [R.to_device(A) for A in mats]
    srv = R.Server(arena_bytes=1 << 30, max_slots=1, max_queue=2)
    outs = [alloc_out(R, torch, A, min(A.M, 64), torch.float64) for A in mats]
    big = gen.cfg4_matrix(gen.Request(0.0, 1024, 1 << 20, 2_000_000, 64, 3))
    dbig = R.to_device(big)
    obig = alloc_out(R, torch, big, 64, torch.float64)
    small_srv = R.Server(arena_bytes=1 << 22, max_slots=1, max_queue=2)
    assert small_srv.submit(dbig, 64, obig)[0] == R.E_NOMEM      # could never fit
    small_srv.close()
    # a request with a broken CSC fails alone
    bad = R.to_device(mats[0])
    ri = mats[0].rowidx.copy()
    ri[0] = mats[0].M + 1
    bad.rowidx = torch.from_numpy(ri).cuda()
    st0, t0 = srv.submit(bad, min(mats[0].M, 64), outs[0])
    results = {}
    st1, t1 = srv.submit(dms[1], min(mats[1].M, 64), outs[1])
    st2, t2 = srv.submit(dms[2], min(mats[2].M, 64), outs[2])
    busy = [srv.submit(dms[3], min(mats[3].M, 64), outs[3])[0] for _ in range(4)]
    assert R.E_BUSY in busy                                         # queue of 2 overflows
    srv.cancel(t2)
    results[t0] = srv.wait(t0, 60_000_000)[0]
    results[t1] = srv.wait(t1, 60_000_000)[0]
    results[t2] = srv.wait(t2, 60_000_000)[0]
    srv.close()
    assert results[t0] == R.E_CSC
    assert results[t1] == R.OK
    assert results[t2] in (R.E_CANCELLED, R.OK)
    alone = R.svd(dms[1], min(mats[1].M, 64), 0.0)
    assert torch.equal(outs[1].sigma, alone.sigma)

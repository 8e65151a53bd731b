"""Seeded input generators: determinism and the statistics each workload recipe promises."""
import hashlib

import numpy as np
import pytest

from paper_2009_09767_amd import gen


def digest(A):
    h = hashlib.sha256()
    for a in (A.colptr, A.rowidx, A.values):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_same_seed_same_bytes():
    assert digest(gen.small_deficient()) == digest(gen.small_deficient())
    assert digest(gen.small_deficient()) != digest(gen.small_deficient(seed=1))
    assert digest(gen.powerlaw_small()) == digest(gen.powerlaw_small())


def test_csc_contract():
    for A in (gen.small_deficient(), gen.powerlaw_small(), gen.batch_mixed(count=3)[0]):
        assert A.colptr.dtype == np.int32 and A.rowidx.dtype == np.int32
        assert A.colptr[0] == 0 and A.colptr[-1] == A.nnz
        assert np.all(np.diff(A.colptr) >= 0)
        for j in range(0, A.N, max(1, A.N // 500)):
            seg = A.rowidx[A.colptr[j]:A.colptr[j + 1]]
            assert np.all(np.diff(seg) > 0)
        assert A.rowidx.min() >= 0 and A.rowidx.max() < A.M


def test_small_deficient_recipe():
    A = gen.small_deficient()
    assert (A.M, A.N) == (64, 4096)
    assert abs(A.nnz / (64 * 4096) - 0.02) < 0.002
    X = A.dense()
    assert not X[24:, 1536:2048].any()
    assert np.abs(A.values).max() < 1.0 and A.values.dtype == np.float64


def test_powerlaw_1m_recipe():
    A = gen.powerlaw_1m()
    assert (A.M, A.N) == (1024, 1 << 20)
    assert 0.95e6 < A.nnz < 1.06e6
    deg = np.bincount(A.rowidx, minlength=A.M)
    assert 170_000 < deg.max() < 190_000      # Zipf(1.1) head ~ 188k before block zeroing
    assert 60 < deg.min() < 100               # tail ~ 91
    zb = A.meta["zeroed_blocks"]
    assert len(zb) == 8
    bs = gen.block_starts(A.N, 64)
    cols = np.repeat(np.arange(A.N), np.diff(A.colptr))
    for b, rows in zb.items():
        assert len(rows) == 307
        inblk = (cols >= bs[b]) & (cols < bs[b + 1])
        assert not np.isin(A.rowidx[inblk], rows).any()


def test_batch_mixed_recipe():
    batch = gen.batch_mixed(count=20, deficient_frac=0.25)
    assert len(batch) == 20
    deficient = [A for A in batch if A.meta["zeroed_rows"].size]
    assert len(deficient) == 5
    for A in batch:
        assert 32 <= A.M <= 512 and 10_000 <= A.N <= 100_000
        assert A.values.dtype == np.float32
        assert abs(A.nnz / (A.M * A.N) - 0.005 * (0.5 if A.meta["zeroed_rows"].size else 1.0)) < 0.001


def test_serving_arrivals():
    reqs = gen.serving_requests()
    assert 11_000 < len(reqs) < 13_000       # 200/s for 60 s
    gaps = np.diff([r.arrival_s for r in reqs])
    assert abs(gaps.mean() - 1 / 200) < 2e-4
    assert all(r.M in (128, 256, 512, 1024) and r.k == min(r.M, 64) for r in reqs)
    assert max(r.nnz for r in reqs) <= 2e7
    A = gen.serving_matrix(reqs[0])
    assert A.M == reqs[0].M and A.N == reqs[0].N and abs(A.nnz - reqs[0].nnz) <= 0.01 * reqs[0].nnz + 64


def test_zipf_cap():
    deg = gen.zipf_degrees(4096, 1 << 16, 30_000_000, 1.2)
    assert deg.max() == 1 << 16
    assert abs(deg.sum() - 30_000_000) < 0.001 * 30_000_000

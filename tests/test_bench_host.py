"""Host-side pieces of the benchmark: the counted-traffic table is keyed to the kernel source it
was measured on (a changed source reports no counted figure rather than a stale one), and the
algorithmic byte and flop counts behind the roofline lines match counts made by hand."""
import hashlib
import os

import numpy as np

import bench
from paper_2009_09767_amd import gen


def _source(entry):
    return os.path.join(bench.ROOT, "paper_2009_09767_amd", "csrc", entry["source"])


def test_traffic_entries_name_existing_sources():
    assert bench.TRAFFIC
    for key, e in bench.TRAFFIC.items():
        assert os.path.isfile(_source(e)), key
        assert e["bytes"] > 0, key
        assert len(e["source_sha256"]) == 64, key


def test_counted_traffic_needs_the_measured_source(monkeypatch):
    key = ("k_backproject", "powerlaw_200m/fp64")
    e = dict(bench.TRAFFIC[key])
    with open(_source(e), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    monkeypatch.setitem(bench.TRAFFIC, key, dict(e, source_sha256=sha))
    assert bench.counted_traffic(*key) == e["bytes"]
    monkeypatch.setitem(bench.TRAFFIC, key, dict(e, source_sha256="0" * 64))
    assert bench.counted_traffic(*key) is None
    assert bench.counted_traffic("no_such_kernel", "powerlaw_200m/fp64") is None


def test_back_projection_bytes_are_the_arrays_it_touches():
    # CSC read once (row indices, values, column pointers), U read once, V written once
    A = gen.random_sparse(7, 50, 0.2, seed=3)
    k = 4
    for val_bytes, out_bytes, u_bytes in ((8, 8, 8), (4, 4, 4), (4, 8, 8)):
        by_hand = (A.rowidx.size * 4 + A.values.size * val_bytes + (A.N + 1) * 4 + A.N * k * out_bytes
                   + A.M * k * u_bytes)
        assert bench.spmm_bytes(A.nnz, A.N, k, A.M, val_bytes, out_bytes, u_bytes) == by_hand


def test_jacobi_sweep_flops_counts_the_rotations():
    # a rotation updates two rows of G (6n flops; symmetry gives the columns) and two columns of
    # W (6n flops); a cyclic sweep has n(n - 1) / 2 rotations: 6 n^3 up to the n^2 term
    for n in (2, 33, 1024):
        rotations = n * (n - 1) // 2
        assert abs(bench.jacobi_sweep_flops(n) - rotations * 12 * n) <= 6 * n * n
    assert np.isclose(bench.jacobi_sweep_flops(1024), 6.0 * 1024**3)

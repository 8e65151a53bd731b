"""Seeded synthetic inputs: CSC matrices shaped like the paper's workloads.

This module only draws inputs.  It holds none of the method's arithmetic
(no Gram, no eigensolve, no singular values), so the GPU path and the CPU
oracle can both consume its bytes without sharing any computation.

The paper's own matrix (a 539 x 170897 job/candidate bipartite graph, Sec. IV)
is not available; the generators below stand in for it with power-law row
degrees, uniform columns and seeded block-local or global zero rows, at the
sizes of the five benchmark workloads:

  small_deficient   64 x 4096, Bernoulli(0.02), U(-1,1) FP64, block 3 (0-based) rows 24..63 zeroed
  powerlaw_1m       1024 x 2^20, Zipf(1.1) row degrees (~1.05M nnz), N(0,1) FP64,
                    8 seeded blocks with 30% of rows emptied inside the block
  batch_mixed       256 matrices, M ~ U{32..512}, N ~ U{1e4..1e5}, Bernoulli(0.005), N(0,1) FP32,
                    20% of matrices with a random half of rows zeroed (global zero rows)
  serving_requests  Poisson arrivals at 200/s for 60 s; M in {128,256,512,1024}, N = 2^U{14..20},
                    nnz ~ LogUniform[1e5, min(2e7, 0.02 M N)], Zipf(1.1) rows, U(-1,1) FP32, k = min(M, 64)
  powerlaw_200m     4096 x 2^24, ~200M nnz, Zipf(1.2) rows capped at N, U(-1,1) FP32,
                    1024 rows emptied in 128 seeded blocks

All draws use numpy's PCG64 with seed = 2009097670 + the workload's stream number (1 to 5,
in the order above) unless a seed is given.  Rows are assigned degrees in a seeded random order (the heavy rows are
spread over the index range), and a row's columns are drawn without replacement.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 2009097670


@dataclass
class CSC:
    M: int
    N: int
    colptr: np.ndarray          # int32 [N+1]
    rowidx: np.ndarray          # int32 [nnz], strictly increasing inside a column
    values: np.ndarray          # float32 or float64 [nnz]
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowidx.shape[0])

    def dense(self) -> np.ndarray:
        """Dense float64 copy (small matrices only)."""
        A = np.zeros((self.M, self.N), dtype=np.float64)
        cols = np.repeat(np.arange(self.N), np.diff(self.colptr))
        A[self.rowidx, cols] = self.values
        return A

    def astype(self, dtype) -> "CSC":
        return CSC(self.M, self.N, self.colptr, self.rowidx, self.values.astype(dtype), dict(self.meta))


def rng_for(stream: int, seed: int | None = None) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + stream if seed is None else seed))


def from_coo(M: int, N: int, rows, cols, vals, meta=None) -> CSC:
    """Build a CSC from coordinates (no duplicates allowed)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals)
    order = np.lexsort((rows, cols))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate coordinates")
    counts = np.bincount(cols, minlength=N) if cols.size else np.zeros(N, dtype=np.int64)
    colptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=colptr[1:])
    if colptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32 indices")
    return CSC(M, N, colptr.astype(np.int32), rows.astype(np.int32), np.ascontiguousarray(vals), meta or {})


def block_starts(N: int, D: int) -> np.ndarray:
    """Column block boundaries floor(b N / D) (every column is covered)."""
    return (np.arange(D + 1, dtype=np.int64) * N) // D


def drop_entries(A: CSC, keep: np.ndarray) -> CSC:
    """Remove the entries where keep is False (structure only, values untouched)."""
    cols = np.repeat(np.arange(A.N, dtype=np.int64), np.diff(A.colptr))[keep]
    counts = np.bincount(cols, minlength=A.N)
    colptr = np.zeros(A.N + 1, dtype=np.int64)
    np.cumsum(counts, out=colptr[1:])
    return CSC(A.M, A.N, colptr.astype(np.int32), A.rowidx[keep].copy(), A.values[keep].copy(), dict(A.meta))


def zipf_degrees(M: int, N: int, nnz: int, s: float) -> np.ndarray:
    """Row degrees proportional to 1/r^s (r = 1..M) summing to about nnz, each in [1, N].

    Degrees above N are capped at N and the excess is handed to the uncapped
    rows in proportion to their weight, until nothing exceeds N."""
    w = 1.0 / np.arange(1, M + 1, dtype=np.float64) ** s
    deg = np.zeros(M, dtype=np.float64)
    capped = np.zeros(M, dtype=bool)
    remaining = float(nnz)
    for _ in range(64):
        free = ~capped
        share = remaining * w[free] / w[free].sum()
        deg[free] = share
        over = free & (deg > N)
        if not over.any():
            break
        capped |= over
        deg[capped] = N
        remaining = float(nnz) - N * capped.sum()
    deg = np.clip(np.rint(deg), 1, N).astype(np.int64)
    return deg


def powerlaw_rows(rng: np.random.Generator, M: int, N: int, nnz: int, s: float, value_kind: str,
                  dtype) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    deg = zipf_degrees(M, N, nnz, s)
    perm = rng.permutation(M)           # row perm[r] gets the r-th largest degree
    rows_l, cols_l = [], []
    for r in range(M):
        d = int(deg[r])
        cols_l.append(rng.choice(N, size=d, replace=False))
        rows_l.append(np.full(d, perm[r], dtype=np.int64))
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l).astype(np.int64)
    vals = draw_values(rng, rows.size, value_kind, dtype)
    return rows, cols, vals


def draw_values(rng: np.random.Generator, n: int, kind: str, dtype) -> np.ndarray:
    if kind == "normal":
        v = rng.standard_normal(n)
    elif kind == "uniform":
        v = rng.uniform(-1.0, 1.0, n)
    elif kind == "ones":
        v = np.ones(n)
    else:
        raise ValueError(kind)
    return v.astype(dtype)


# ----------------------------------------------------------------------------
# Benchmark configurations
# ----------------------------------------------------------------------------

def small_deficient(seed: int | None = None, M=64, N=4096, D=8, p=0.02, zero_block=3, zero_rows=(24, 64)) -> CSC:
    """Plain method, small: Bernoulli(p) entries, U(-1,1) FP64, one block with rows emptied."""
    rng = rng_for(1, seed)
    mask = rng.random((M, N)) < p
    rows, cols = np.nonzero(mask)
    vals = draw_values(rng, rows.size, "uniform", np.float64)
    bs = block_starts(N, D)
    c0, c1 = bs[zero_block], bs[zero_block + 1]
    keep = ~((cols >= c0) & (cols < c1) & (rows >= zero_rows[0]) & (rows < zero_rows[1]))
    return from_coo(M, N, rows[keep], cols[keep], vals[keep],
                    dict(name="small_deficient", D=D, k=M, tol=1e-12, zero_block=zero_block, zero_rows=zero_rows))


def powerlaw_1m(seed: int | None = None, M=1024, N=1 << 20, D=64, nnz=1_050_000, s=1.1, zero_blocks=8,
         zero_frac=0.3, k=128, dtype=np.float64) -> CSC:
    """Power-law rows (Zipf(s) degrees), uniform columns, N(0,1) values; zero_blocks seeded
    blocks have floor(zero_frac M) seeded rows emptied inside the block only."""
    rng = rng_for(2, seed)
    rows, cols, vals = powerlaw_rows(rng, M, N, nnz, s, "normal", dtype)
    bs = block_starts(N, D)
    blocks = rng.choice(D, size=min(zero_blocks, D), replace=False)
    nz = int(math.floor(zero_frac * M))
    keep = np.ones(rows.size, dtype=bool)
    zeroed = {}
    for b in sorted(int(x) for x in blocks):
        zr = np.sort(rng.choice(M, size=nz, replace=False))
        zeroed[b] = zr
        inblk = (cols >= bs[b]) & (cols < bs[b + 1])
        keep &= ~(inblk & np.isin(rows, zr))
    return from_coo(M, N, rows[keep], cols[keep], vals[keep],
                    dict(name="powerlaw_1m", D=D, k=k, tol=0.0, zeroed_blocks=zeroed))


def powerlaw_small(seed: int | None = None, M=128, N=1 << 14, D=8, k=32, dtype=np.float64) -> CSC:
    """powerlaw_1m's recipe at a size the oracle solves in seconds (nnz ~ N, as in powerlaw_1m)."""
    A = powerlaw_1m(seed=BASE_SEED + 20 if seed is None else seed, M=M, N=N, D=D, nnz=N, zero_blocks=2, k=k,
             dtype=dtype)
    A.meta["name"] = "powerlaw_small"
    return A


def batch_matrix(rng: np.random.Generator, M: int, N: int, density=0.005, zero_half=False,
                D: int = 8) -> CSC:
    total = M * N
    nnz = int(rng.binomial(total, density))
    flat = rng.choice(total, size=nnz, replace=False)
    rows, cols = flat // N, flat % N
    vals = draw_values(rng, nnz, "normal", np.float32)
    zeroed = np.zeros(0, dtype=np.int64)
    if zero_half:
        zeroed = np.sort(rng.choice(M, size=M // 2, replace=False))
        keep = ~np.isin(rows, zeroed)
        rows, cols, vals = rows[keep], cols[keep], vals[keep]
    return from_coo(M, N, rows, cols, vals, dict(name="batch_mixed", D=D, k=M, tol=0.0, zeroed_rows=zeroed))


def batch_mixed(seed: int | None = None, count=256, M_range=(32, 512), N_range=(10_000, 100_000),
         density=0.005, deficient_frac=0.2) -> list[CSC]:
    """Batch of independent matrices; a seeded 20% get a random half of their rows zeroed."""
    rng = rng_for(3, seed)
    Ms = rng.integers(M_range[0], M_range[1] + 1, size=count)
    Ns = rng.integers(N_range[0], N_range[1] + 1, size=count)
    Ds = rng.integers(2, 17, size=count)
    deficient = set(int(x) for x in rng.choice(count, size=int(round(deficient_frac * count)), replace=False))
    seeds = rng.integers(0, 2**62, size=count)
    out = []
    for i in range(count):
        r = np.random.Generator(np.random.PCG64(int(seeds[i])))
        A = batch_matrix(r, int(Ms[i]), int(Ns[i]), density, i in deficient, int(Ds[i]))
        A.meta["index"] = i
        out.append(A)
    return out


@dataclass
class Request:
    arrival_s: float
    M: int
    N: int
    nnz: int
    k: int
    seed: int


def serving_requests(seed: int | None = None, rate=200.0, duration_s=60.0,
                  Ms=(128, 256, 512, 1024), log2N=(14, 20), nnz_lo=1e5, nnz_hi=2e7) -> list[Request]:
    """Open-loop Poisson arrivals; each request's matrix is drawn later from its own seed."""
    rng = rng_for(4, seed)
    t, reqs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        M = int(rng.choice(Ms))
        N = 1 << int(rng.integers(log2N[0], log2N[1] + 1))
        hi = min(nnz_hi, 0.02 * M * N)
        lo = min(nnz_lo, hi)
        nnz = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        reqs.append(Request(t, M, N, nnz, min(M, 64), int(rng.integers(0, 2**62))))
    return reqs


def serving_matrix(req: Request, s=1.1) -> CSC:
    rng = np.random.Generator(np.random.PCG64(req.seed))
    rows, cols, vals = powerlaw_rows(rng, req.M, req.N, req.nnz, s, "uniform", np.float32)
    return from_coo(req.M, req.N, rows, cols, vals, dict(name="serving", D=max(1, req.N >> 14), k=req.k, tol=0.0))


def powerlaw_200m(seed: int | None = None, M=4096, N=1 << 24, D=256, nnz=200_000_000, s=1.2, zero_blocks=128,
         zero_rows=1024, k=100, progress=None) -> CSC:
    """Large single matrix: Zipf(1.2) rows capped at N; zero_rows seeded rows emptied inside each of
    zero_blocks seeded blocks.  The pre-zeroing target is scaled so about nnz entries remain.
    Rows are drawn in increasing row order, so one stable sort by column gives sorted CSC rows.
    `progress(msg)` is called every 512 rows and at each later stage."""
    rng = rng_for(5, seed)
    frac_removed = (zero_blocks / D) * (zero_rows / M)
    target = int(round(nnz / (1.0 - frac_removed)))
    deg = zipf_degrees(M, N, target, s)
    perm = rng.permutation(M)                  # row perm[r] gets the r-th largest degree
    deg_of_row = np.empty(M, dtype=np.int64)
    deg_of_row[perm] = deg
    bs = block_starts(N, D)
    blocks = np.sort(rng.choice(D, size=zero_blocks, replace=False))
    zero_sets = [np.sort(rng.choice(M, size=zero_rows, replace=False)) for _ in blocks]
    row_zero_blocks = [[] for _ in range(M)]
    for b, zr in zip(blocks, zero_sets):
        for m in zr:
            row_zero_blocks[int(m)].append(int(b))
    total = int(deg_of_row.sum())
    cols = np.empty(total, dtype=np.int32)
    rows = np.empty(total, dtype=np.int32)
    pos = 0
    for m in range(M):
        c = rng.choice(N, size=int(deg_of_row[m]), replace=False)
        if row_zero_blocks[m]:
            blk = np.searchsorted(bs, c, side="right") - 1
            c = c[~np.isin(blk, row_zero_blocks[m])]
        cols[pos:pos + c.size] = c
        rows[pos:pos + c.size] = m
        pos += c.size
        if progress is not None and m % 512 == 511:
            progress(f"powerlaw_200m: {m + 1}/{M} rows drawn, {pos} entries")
    cols = cols[:pos]
    rows = rows[:pos]
    # stable LSD radix sort by column in two 16-bit passes (numpy's stable sort is a radix
    # sort for 16-bit keys); rows stay increasing within a column
    o1 = np.argsort((cols & 0xFFFF).astype(np.uint16), kind="stable")
    o2 = np.argsort((cols[o1] >> 16).astype(np.uint16), kind="stable")
    order = o1[o2]
    del o1, o2
    if progress is not None:
        progress("powerlaw_200m: sorted by column")
    rows = rows[order]
    counts = np.bincount(cols, minlength=N)
    del order, cols
    vals = draw_values(rng, rows.size, "uniform", np.float32)
    colptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=colptr[1:])
    return CSC(M, N, colptr.astype(np.int32), rows, vals,
               dict(name="powerlaw_200m", D=D, k=k, tol=0.0, zeroed_blocks=dict(zip(blocks.tolist(), zero_sets))))


def paper_standin(seed: int | None = None, M=539, N=170_897, nnz_per_col=5.0, s=1.1) -> CSC:
    """Stand-in for the paper's job-candidate matrix (539 x 170897, 0/1 entries; the data set is not
    available): power-law row degrees (Zipf(s)) summing to about nnz_per_col * N, uniform columns,
    every value 1."""
    rng = rng_for(6, seed)
    rows, cols, vals = powerlaw_rows(rng, M, N, int(round(nnz_per_col * N)), s, "ones", np.float64)
    return from_coo(M, N, rows, cols, vals, dict(name="paper_standin", k=10, tol=0.0))


# ----------------------------------------------------------------------------
# Closed-form inputs for the pins (their singular values are known exactly)
# ----------------------------------------------------------------------------

def diagonal(d, N: int, cols=None, seed: int = 7, dtype=np.float64) -> CSC:
    """One nonzero d[m] per row m, in distinct columns (seeded when cols is None).
    Singular values |d|, left vectors signed unit vectors, right vectors signed unit vectors."""
    d = np.asarray(d, dtype=np.float64)
    M = d.size
    if cols is None:
        cols = np.random.Generator(np.random.PCG64(seed)).choice(N, size=M, replace=False)
    rows = np.arange(M)
    keep = d != 0
    return from_coo(M, N, rows[keep], np.asarray(cols)[keep], d[keep].astype(dtype),
                    dict(name="diagonal", cols=np.asarray(cols)))


def random_orthogonal(M: int, rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((M, M)))
    return q * np.sign(np.diag(r))


def known_factors(s, N: int, seed: int = 11, support=None, dtype=np.float64):
    """A = U diag(s) V^T with U a seeded orthogonal matrix and V with disjoint column supports
    (column i of V lives on its own set of rows of V, normalised), so V^T V = I exactly.
    Returns (A as CSC, U, s, V)."""
    s = np.asarray(s, dtype=np.float64)
    M = s.size
    rng = np.random.Generator(np.random.PCG64(seed))
    U = random_orthogonal(M, rng)
    if support is None:
        support = max(1, N // M)
    perm = rng.permutation(N)
    V = np.zeros((N, M))
    for i in range(M):
        idx = perm[i * support:(i + 1) * support]
        w = rng.standard_normal(idx.size)
        V[idx, i] = w / np.linalg.norm(w)
    A = (U * s) @ V.T
    rows, cols = np.nonzero(A)
    csc = from_coo(M, N, rows, cols, A[rows, cols].astype(dtype), dict(name="known_factors"))
    return csc, U, s, V


def from_dense(A: np.ndarray, dtype=np.float64) -> CSC:
    rows, cols = np.nonzero(A)
    return from_coo(A.shape[0], A.shape[1], rows, cols, A[rows, cols].astype(dtype), dict(name="dense"))


def random_sparse(M: int, N: int, density: float, seed: int, dtype=np.float64, kind="normal") -> CSC:
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = rng.random((M, N)) < density
    rows, cols = np.nonzero(mask)
    return from_coo(M, N, rows, cols, draw_values(rng, rows.size, kind, dtype), dict(name="random"))

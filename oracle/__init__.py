"""Plain CPU FP64 oracle for the rank-safe column-block SVD (Ranky, arXiv 2009.09767).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never imports, links or calls it, and shares no code with it.

This module only marshals numpy arrays into ``ranky_oracle.c`` (compiled with
gcc into ``libranky_oracle.so`` next to it); every number is computed there.
Method names follow the paper: ``merge`` is the one-level block merge through
the proxy matrix P (Sec. III, Alg. 1); ``whole`` is the one-sided Jacobi SVD of
the whole matrix; ``gram`` is the Gram matrix of Eq. (2) plus a two-sided Jacobi
eigensolver.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_DEFAULT_LIB = os.path.join(_HERE, "libranky_oracle.so")
# The mutation tests point this at a deliberately broken build of the same source.
_LIB_PATH = os.environ.get("RANKY_ORACLE_LIB", _DEFAULT_LIB)
_lib = None

OK, E_INVALID, E_CSC, E_NONFINITE, E_NOMEM, E_NOT_CONVERGED = 0, 1, 2, 3, 4, 8
METHODS = {"whole": 0, "whole_qr": 1, "merge": 2, "gram": 3}
U_FP64 = 2.0 ** -53
U_FP32 = 2.0 ** -24


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_PATH == _DEFAULT_LIB and not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.ro_check_csc.argtypes = [i32, i64, i64, vp, vp, vp, ctypes.c_int]
    lib.ro_block_bounds.argtypes = [i64, i32, vp]
    lib.ro_occupancy.argtypes = [i32, i64, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.ro_rank_prob.argtypes = [i64, i64]
    lib.ro_rank_prob.restype = dbl
    lib.ro_gram.argtypes = [i32, i64, vp, vp, vp, ctypes.c_int, vp]
    lib.ro_bf16_split.argtypes = [i64, vp, vp, vp]
    lib.ro_gram_bf16x3.argtypes = [i32, i64, vp, vp, vp, ctypes.c_int, i32, vp, vp]
    lib.ro_hestenes.argtypes = [i32, i64, vp, vp, vp, i32, vp]
    lib.ro_qr_r.argtypes = [i64, i32, vp, vp]
    lib.ro_eig_jacobi.argtypes = [i32, vp, vp, i32, vp]
    lib.ro_backproject.argtypes = [i32, i64, vp, vp, vp, ctypes.c_int, i32, vp, vp, i32, vp]
    lib.ro_svd.argtypes = [i32, i32, i64, i64, vp, vp, vp, ctypes.c_int, i32, i32, dbl, dbl, i32,
                           vp, vp, vp, vp, vp, vp]
    lib.ro_checker.argtypes = [i32, i64, i64, vp, vp, vp, ctypes.c_int, i32, i32, ctypes.c_uint64, vp, vp, vp, vp, vp]
    for name in ("ro_check_csc", "ro_block_bounds", "ro_occupancy", "ro_gram", "ro_bf16_split", "ro_gram_bf16x3",
                 "ro_hestenes",
                 "ro_qr_r", "ro_eig_jacobi", "ro_backproject", "ro_svd", "ro_checker"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csc_arrays(colptr, rowidx, values):
    colptr = np.ascontiguousarray(colptr, dtype=np.int32)
    rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
    values = np.ascontiguousarray(values)
    if values.dtype == np.float64:
        dtype = 1
    elif values.dtype == np.float32:
        dtype = 0
    else:
        raise TypeError("values must be float32 or float64")
    return colptr, rowidx, values, dtype


def check_csc(M, N, colptr, rowidx, values) -> int:
    colptr, rowidx, values, dt = _csc_arrays(colptr, rowidx, values)
    return int(_load().ro_check_csc(M, N, len(rowidx), _ptr(colptr), _ptr(rowidx), _ptr(values), dt))


def block_bounds(N: int, D: int) -> np.ndarray:
    out = np.zeros(D + 1, dtype=np.int64)
    st = _load().ro_block_bounds(N, D, _ptr(out))
    if st:
        raise OracleError(st, "block_bounds")
    return out


@dataclass
class Occupancy:
    cnt: np.ndarray      # (D, M) nonzeros of each row inside each block
    rownnz: np.ndarray   # (M,)
    lonely: np.ndarray   # (D,) rows with no entry inside the block
    single: np.ndarray   # (D,) rows with exactly one entry inside the block (NO of Eq. 4)


def occupancy(M, N, colptr, rowidx, D) -> Occupancy:
    colptr = np.ascontiguousarray(colptr, dtype=np.int32)
    rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
    start = block_bounds(N, D)
    cnt = np.zeros((D, M), dtype=np.int32)
    rownnz = np.zeros(M, dtype=np.int32)
    lonely = np.zeros(D, dtype=np.int32)
    single = np.zeros(D, dtype=np.int32)
    _load().ro_occupancy(M, N, _ptr(colptr), _ptr(rowidx), D, _ptr(start), _ptr(cnt), _ptr(rownnz),
                         _ptr(lonely), _ptr(single))
    return Occupancy(cnt, rownnz, lonely, single)


def rank_prob(NC: int, NO: int) -> float:
    return float(_load().ro_rank_prob(NC, NO))


def gram(M, N, colptr, rowidx, values) -> np.ndarray:
    colptr, rowidx, values, dt = _csc_arrays(colptr, rowidx, values)
    G = np.zeros((M, M), dtype=np.float64)
    _load().ro_gram(M, N, _ptr(colptr), _ptr(rowidx), _ptr(values), dt, _ptr(G))
    return G


def bf16_split(x) -> tuple:
    """x (FP32) = hi + lo + rest with hi = bf16(x), lo = bf16(x - hi), round to nearest even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    hi = np.empty_like(x)
    lo = np.empty_like(x)
    _load().ro_bf16_split(x.size, _ptr(x), _ptr(hi), _ptr(lo))
    return hi, lo


def gram_bf16x3(M, N, colptr, rowidx, values, rows) -> np.ndarray:
    """The split-bf16 Gram block of `rows`: sum over columns of hi_p hi_q + hi_p lo_q + lo_p hi_q."""
    colptr, rowidx, values, dt = _csc_arrays(colptr, rowidx, values)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    G = np.zeros((rows.size, rows.size), dtype=np.float64)
    _load().ro_gram_bf16x3(M, N, _ptr(colptr), _ptr(rowidx), _ptr(values), dt, rows.size, _ptr(rows), _ptr(G))
    return G


def hestenes(B: np.ndarray, max_sweeps: int = 60):
    """One-sided Jacobi SVD of dense rows: returns (U, sigma, B_rotated, sweeps), input = U @ B_rotated."""
    B = np.array(B, dtype=np.float64, order="C", copy=True)
    m, n = B.shape
    U = np.zeros((m, m), dtype=np.float64)
    s = np.zeros(m, dtype=np.float64)
    sw = np.zeros(1, dtype=np.int32)
    st = _load().ro_hestenes(m, n, _ptr(B), _ptr(U), _ptr(s), max_sweeps, _ptr(sw))
    if st:
        raise OracleError(st, "hestenes")
    return U, s, B, int(sw[0])


def qr_r(X: np.ndarray) -> np.ndarray:
    """R factor of the Householder QR of a tall matrix X (rows >= cols)."""
    X = np.asfortranarray(np.array(X, dtype=np.float64, copy=True))
    rows, cols = X.shape
    R = np.zeros((cols, cols), dtype=np.float64)
    st = _load().ro_qr_r(rows, cols, X.ctypes.data_as(ctypes.c_void_p), _ptr(R))
    if st:
        raise OracleError(st, "qr_r")
    return R


def eig_jacobi(G: np.ndarray, max_sweeps: int = 60):
    """Two-sided Jacobi: returns (eigenvalues unsorted, eigenvectors as columns, sweeps)."""
    G = np.array(G, dtype=np.float64, order="C", copy=True)
    n = G.shape[0]
    V = np.zeros((n, n), dtype=np.float64)
    sw = np.zeros(1, dtype=np.int32)
    st = _load().ro_eig_jacobi(n, _ptr(G), _ptr(V), max_sweeps, _ptr(sw))
    if st:
        raise OracleError(st, "eig_jacobi")
    return np.diag(G).copy(), V, int(sw[0])


def backproject(M, N, colptr, rowidx, values, U, sigma, rank) -> np.ndarray:
    colptr, rowidx, values, dt = _csc_arrays(colptr, rowidx, values)
    U = np.ascontiguousarray(U, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    k = U.shape[1]
    V = np.zeros((N, k), dtype=np.float64)
    _load().ro_backproject(M, N, _ptr(colptr), _ptr(rowidx), _ptr(values), dt, k, _ptr(U), _ptr(sigma),
                           rank, _ptr(V))
    return V


@dataclass
class SVD:
    sigma: np.ndarray   # (k,)
    U: np.ndarray       # (M, k)
    V: np.ndarray | None  # (N, k)
    rank: int
    tau: float
    sweeps: int


def svd(M, N, colptr, rowidx, values, k, tol=0.0, method="whole", D=1, u_gram=U_FP64,
        want_v=True, max_sweeps=60) -> SVD:
    colptr, rowidx, values, dt = _csc_arrays(colptr, rowidx, values)
    sigma = np.zeros(k, dtype=np.float64)
    U = np.zeros((M, k), dtype=np.float64)
    V = np.zeros((N, k), dtype=np.float64) if want_v else None
    rank = np.zeros(1, dtype=np.int32)
    tau = np.zeros(1, dtype=np.float64)
    sw = np.zeros(1, dtype=np.int32)
    st = _load().ro_svd(METHODS[method], M, N, len(rowidx), _ptr(colptr), _ptr(rowidx), _ptr(values), dt,
                        D, k, tol, u_gram, max_sweeps, _ptr(sigma), _ptr(U),
                        _ptr(V) if V is not None else None, _ptr(rank), _ptr(tau), _ptr(sw))
    if st:
        raise OracleError(st, f"svd[{method}]")
    return SVD(sigma, U, V, int(rank[0]), float(tau[0]), int(sw[0]))


CHECKERS = {"random": 0, "neighbor": 1, "neighbor_random": 2}


def checker(M, N, colptr, rowidx, values, D, kind, seed):
    """Alg. 2-4 on a copy of A: (colptr', rowidx', values' FP64, inserted) of A' (CSC)."""
    colptr, rowidx, values, dt = _csc_arrays(colptr, rowidx, values)
    cap = len(rowidx) + 2 * D * M
    cp = np.zeros(N + 1, dtype=np.int32)
    ri = np.zeros(max(cap, 1), dtype=np.int32)
    va = np.zeros(max(cap, 1), dtype=np.float64)
    nz = np.zeros(1, dtype=np.int64)
    ins = np.zeros(1, dtype=np.int64)
    st = _load().ro_checker(M, N, len(rowidx), _ptr(colptr), _ptr(rowidx), _ptr(values), dt, D, CHECKERS[kind],
                            int(seed), _ptr(cp), _ptr(ri), _ptr(va), _ptr(nz), _ptr(ins))
    if st:
        raise OracleError(st, "checker")
    n = int(nz[0])
    return cp, ri[:n].copy(), va[:n].copy(), int(ins[0])

"""Python binding of libranky.so (the C-ABI in include/ranky.h).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the computation runs in the library's HIP kernels.
There is no fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libranky.so")

OK, E_INVALID, E_CSC, E_NONFINITE, E_NOMEM, E_DEVICE, E_BUSY, E_CANCELLED, E_NOT_CONVERGED, PENDING = range(10)
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_CSC", 3: "E_NONFINITE", 4: "E_NOMEM", 5: "E_DEVICE", 6: "E_BUSY",
                7: "E_CANCELLED", 8: "E_NOT_CONVERGED", 9: "PENDING"}
F32, F64 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}


class RankyError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Csc(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("colptr", ctypes.c_void_p), ("rowidx", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("dtype", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("n_blocks", "gram_prec", "refine", "max_sweeps", "validate", "v_dtype", "timing", "graph",
                 "eigensolver", "max_iters", "gram_split")] + \
               [("block_start", ctypes.c_void_p)]


class BatchItem(ctypes.Structure):
    _fields_ = [("A", Csc), ("N", ctypes.c_int64), ("M", ctypes.c_int32), ("k", ctypes.c_int32),
                ("n_blocks", ctypes.c_int32), ("pad", ctypes.c_int32), ("sigma", ctypes.c_void_p),
                ("U", ctypes.c_void_p), ("V", ctypes.c_void_p)]


class ServeCfg(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("max_queue", ctypes.c_int32), ("device", ctypes.c_int), ("pad", ctypes.c_int32),
                ("opts", Opts)]


class Request(ctypes.Structure):
    _fields_ = [("A", Csc), ("N", ctypes.c_int64), ("M", ctypes.c_int32), ("k", ctypes.c_int32),
                ("tol", ctypes.c_double), ("sigma", ctypes.c_void_p), ("U", ctypes.c_void_p), ("V", ctypes.c_void_p)]


class ServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("p50_us", "p99_us", "mean_us", "max_us", "span_s", "req_per_s",
                                               "nnz_per_s")]
    _fields_ += [(n, ctypes.c_int64) for n in ("submitted", "admitted", "completed", "failed", "cancelled",
                                               "rejected", "queued_now", "running_now", "peak_running")]
    _fields_ += [("arena_peak_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("status", "rank", "n_nonempty", "empty_rows", "sweeps", "n_blocks", "lonely_max", "lonely_blocks")]
    _fields_ += [("tau", ctypes.c_double), ("sigma_max", ctypes.c_double), ("ms", ctypes.c_float * 8),
                 ("round_ms", ctypes.c_float), ("round_launches", ctypes.c_int32), ("rr_sweeps", ctypes.c_int32),
                 ("eig_iters", ctypes.c_int32), ("eig_flops", ctypes.c_double),
                 ("lonely_per_block", ctypes.POINTER(ctypes.c_int32)),
                 ("single_per_block", ctypes.POINTER(ctypes.c_int32)),
                 ("topk_block", ctypes.c_int32), ("heavy_rows", ctypes.c_int32)]

    def as_dict(self):
        """Copies every field; the per-block counts (library memory) become lists."""
        d = {n: getattr(self, n) for n, _ in self._fields_
             if n not in ("ms", "lonely_per_block", "single_per_block")}
        d["ms"] = list(self.ms)
        D = self.n_blocks
        for n in ("lonely_per_block", "single_per_block"):
            p = getattr(self, n)
            d[n] = [p[b] for b in range(D)] if p and D > 0 else None
        return d


class PaperInfo(ctypes.Structure):
    _fields_ = [("added", ctypes.c_int64), ("nnz_repaired", ctypes.c_int64), ("proxy_cols", ctypes.c_int64),
                ("rank", ctypes.c_int32), ("n_nonempty", ctypes.c_int32), ("tau", ctypes.c_double),
                ("ms", ctypes.c_float * 4)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n != "ms"}
        d["ms"] = list(self.ms)
        return d


class TuneReport(ctypes.Structure):
    _fields_ = [("bp_per_cu", ctypes.c_int32), ("jacobi_schedule", ctypes.c_int32),
                ("bp_candidates", ctypes.c_int32 * 4), ("bp_ms", ctypes.c_float * 4),
                ("schedule_candidates", ctypes.c_int32 * 4), ("eig_ms", ctypes.c_float * 4)]

    def as_dict(self):
        return {"bp_per_cu": self.bp_per_cu, "jacobi_schedule": self.jacobi_schedule,
                "bp_ms": dict(zip(list(self.bp_candidates), [round(x, 4) for x in self.bp_ms])),
                "eig_ms": dict(zip(list(self.schedule_candidates), [round(x, 4) for x in self.eig_ms]))}


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RankyError(E_DEVICE, f"{LIB_PATH} is not built (python -m paper_2009_09767_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "ranky_ctx_create": ([ctypes.c_int, P(vp)], i32),
        "ranky_ctx_destroy": ([vp], i32),
        "ranky_default_opts": ([P(Opts)], i32),
        "ranky_last_error": ([], ctypes.c_char_p),
        "ranky_version": ([], ctypes.c_char_p),
        "ranky_workspace_bytes": ([i32, i64, i64, i32, P(Opts)], sz),
        "ranky_svd": ([vp, P(Csc), i32, i64, i32, dbl, P(Opts), vp, sz, vp, vp, vp, P(Info), vp], i32),
        "ranky_svd_async": ([vp, P(Csc), i32, i64, i32, dbl, P(Opts), vp, sz, vp, vp, vp, vp, P(ctypes.c_uint64)], i32),
        "ranky_query": ([vp, ctypes.c_uint64, P(Info)], i32),
        "ranky_autotune": ([vp, P(Csc), i32, i64, i32, P(Opts), vp, sz, vp, vp, vp, P(TuneReport), vp], i32),
        "ranky_tune_set": ([vp, i32, i64, i64, i32, i32, P(Opts), i32, i32], i32),
        "ranky_batch_workspace_bytes": ([i32, P(BatchItem), P(Opts)], sz),
        "ranky_batch": ([vp, i32, P(BatchItem), dbl, P(Opts), vp, sz, P(Info), vp], i32),
        "ranky_serve_create": ([P(ServeCfg), P(vp)], i32),
        "ranky_serve_submit": ([vp, P(Request), P(ctypes.c_uint64)], i32),
        "ranky_serve_poll": ([vp, ctypes.c_uint64, P(Info)], i32),
        "ranky_serve_wait": ([vp, ctypes.c_uint64, i64, P(Info)], i32),
        "ranky_serve_cancel": ([vp, ctypes.c_uint64], i32),
        "ranky_serve_stats": ([vp, P(ServeStats)], i32),
        "ranky_serve_destroy": ([vp], i32),
        "ranky_step_workspace_bytes": ([i32, i64, i64, i32], sz),
        "ranky_occupancy": ([P(Csc), i32, i64, i32, vp, vp, vp, vp, vp, sz, vp], i32),
        "ranky_gram": ([P(Csc), i32, i64, i32, vp, vp, sz, vp], i32),
        "ranky_eigh_workspace_bytes": ([i32], sz),
        "ranky_eigh": ([i32, vp, vp, vp, i32, P(i32), vp, sz, vp], i32),
        "ranky_backproject": ([P(Csc), i32, i64, i32, vp, vp, vp, vp, i32, vp], i32),
        "ranky_transpose": ([P(Csc), i64, i64, vp, vp, vp, vp, sz, vp], i32),
        "ranky_svd_noalloc": ([vp, P(Csc), i32, i64, i32, dbl, P(Opts), vp, vp, vp, P(Info), vp], i32),
        "ranky_inc_workspace_bytes": ([i32, i64, i64, i32, P(Opts)], sz),
        "ranky_inc_create": ([vp, i32, i32, i64, i64, P(Opts), vp, sz, P(vp), vp], i32),
        "ranky_inc_append": ([vp, P(Csc), i64, vp], i32),
        "ranky_inc_solve": ([vp, dbl, vp, vp, P(Info), vp], i32),
        "ranky_inc_destroy": ([vp], i32),
        "ranky_checker_workspace_bytes": ([i32, i64, i64, i32], sz),
        "ranky_checker": ([P(Csc), i32, i64, i32, i32, ctypes.c_uint64, vp, vp, vp, i64, P(i64), P(i64), vp, sz, vp],
                          i32),
        "ranky_paper_workspace_bytes": ([i32, i64, i64, i32, i32, i32], sz),
        "ranky_svd_paper": ([vp, P(Csc), i32, i64, i32, i32, i32, ctypes.c_uint64, dbl, vp, sz, vp, vp, P(PaperInfo),
                             vp], i32),
        "ranky_paper_errors": ([i32, i32, vp, vp, vp, vp, P(dbl), P(dbl), vp, sz, vp], i32),
        "ranky_tall_workspace_bytes": ([i64, i32, i64, i32, P(Opts)], sz),
        "ranky_svd_tall": ([vp, P(Csc), i64, i32, i32, dbl, P(Opts), vp, sz, vp, vp, vp, P(Info), vp], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def last_error() -> str:
    return lib().ranky_last_error().decode()


def _check(st: int):
    if st != OK:
        raise RankyError(st, last_error())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


@dataclass
class DeviceCSC:
    """Device-resident CSC (int32 colptr/rowidx, FP32 or FP64 values)."""
    M: int
    N: int
    colptr: torch.Tensor
    rowidx: torch.Tensor
    values: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.rowidx.numel())

    def struct(self) -> Csc:
        for t in (self.colptr, self.rowidx, self.values):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("CSC arrays must be contiguous device tensors")
        if self.colptr.dtype != torch.int32 or self.rowidx.dtype != torch.int32:
            raise TypeError("colptr and rowidx must be int32")
        if self.values.dtype not in (torch.float32, torch.float64):
            raise TypeError("values must be float32 or float64")
        return Csc(self.nnz, self.colptr.data_ptr(), self.rowidx.data_ptr() if self.nnz else 0,
                   self.values.data_ptr() if self.nnz else 0, F64 if self.values.dtype == torch.float64 else F32)


def to_device(A, device="cuda") -> DeviceCSC:
    """Copy a host CSC (anything with M, N, colptr, rowidx, values numpy arrays) to the device."""
    return DeviceCSC(A.M, A.N, torch.from_numpy(A.colptr).to(device), torch.from_numpy(A.rowidx).to(device),
                     torch.from_numpy(A.values).to(device))


class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().ranky_ctx_create(device, ctypes.byref(h)))
        self.handle = h
        self.device = device
        self._ws = None

    def close(self):
        if self.handle:
            lib().ranky_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws


_default_ctx: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


EIGENSOLVER = {"auto": 0, "jacobi": 1, "subspace": 2}


GRAM_SPLIT = {"auto": 0, "off": 1, "on": 2}


def make_opts(n_blocks=0, gram_prec="fp64", refine=None, max_sweeps=0, validate=True, v_dtype=torch.float64,
              timing=False, graph=False, block_start=None, eigensolver="auto", max_iters=0,
              gram_split="auto") -> Opts:
    """block_start: optional D + 1 column boundaries (host; kept alive by the Opts).
    refine=None keeps the library's automatic choice (-1).  gram_split: "auto", "off" or "on"
    (the heavy-row split of the Gram)."""
    o = Opts()
    _check(lib().ranky_default_opts(ctypes.byref(o)))
    o.n_blocks = n_blocks
    o.gram_prec = PREC[gram_prec]
    if refine is not None:
        o.refine = int(refine)
    o.max_sweeps = max_sweeps
    o.validate = int(validate)
    o.v_dtype = F64 if v_dtype == torch.float64 else F32
    o.timing = int(timing)
    o.graph = int(graph)
    o.eigensolver = EIGENSOLVER[eigensolver]
    o.max_iters = int(max_iters)
    o.gram_split = GRAM_SPLIT[gram_split]
    if block_start is not None:
        import numpy as np

        o._block_start = np.ascontiguousarray(np.asarray(block_start, dtype=np.int64))
        o.block_start = o._block_start.ctypes.data
        if n_blocks == 0:
            o.n_blocks = o._block_start.size - 1
    return o


def workspace_bytes(M, N, nnz, k, opts: Opts) -> int:
    return int(lib().ranky_workspace_bytes(M, N, nnz, k, ctypes.byref(opts)))


@dataclass
class SVDResult:
    sigma: torch.Tensor
    U: torch.Tensor
    V: torch.Tensor
    info: dict


def svd(A: DeviceCSC, k: int, tol: float = 0.0, ctx: Context | None = None, out: SVDResult | None = None,
        workspace: torch.Tensor | None = None, stream=None, **opt_kw) -> SVDResult:
    """Top-k singular triplets of A by ranky_svd (blocking)."""
    ctx = ctx or context(A.colptr.device.index or 0)
    opts = make_opts(**opt_kw)
    vdt = torch.float64 if opts.v_dtype == F64 else torch.float32
    dev = A.colptr.device
    if out is None:
        out = SVDResult(torch.empty(k, dtype=torch.float64, device=dev),
                        torch.empty((A.M, k), dtype=torch.float64, device=dev),
                        torch.empty((A.N, k), dtype=vdt, device=dev), {})
    nbytes = workspace_bytes(A.M, A.N, A.nnz, k, opts)
    if nbytes == 0:
        raise RankyError(E_INVALID, "invalid sizes for the workspace")
    ws = workspace if workspace is not None else ctx.workspace(nbytes)
    info = Info()
    csc = A.struct()
    st = lib().ranky_svd(ctx.handle, ctypes.byref(csc), A.M, A.N, k, float(tol), ctypes.byref(opts), _ptr(ws),
                         ws.numel(), _ptr(out.sigma), _ptr(out.U), _ptr(out.V), ctypes.byref(info), _stream(stream))
    _check(st)
    out.info = info.as_dict()
    return out


def transpose(A: DeviceCSC, stream=None) -> DeviceCSC:
    """ranky_transpose: the CSC of A^T (N x M) as a new DeviceCSC."""
    dev = A.colptr.device
    colptr = torch.empty(A.M + 1, dtype=torch.int32, device=dev)
    rowidx = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)[:A.nnz]
    values = torch.empty(max(A.nnz, 1), dtype=A.values.dtype, device=dev)[:A.nnz]
    nbytes = int(lib().ranky_tall_workspace_bytes(A.M, 1, A.nnz, 1, None))
    if nbytes == 0:
        raise RankyError(E_INVALID, "invalid sizes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    csc = A.struct()
    _check(lib().ranky_transpose(ctypes.byref(csc), A.M, A.N, _ptr(colptr), _ptr(rowidx), _ptr(values), _ptr(ws),
                                 nbytes, _stream(stream)))
    return DeviceCSC(A.N, A.M, colptr, rowidx, values)


def svd_tall(A: DeviceCSC, k: int, tol: float = 0.0, ctx: Context | None = None, stream=None,
             **opt_kw) -> SVDResult:
    """Top-k singular triplets of a tall-and-skinny A by ranky_svd_tall (U is M x k of v_dtype,
    V is N x k FP64)."""
    ctx = ctx or context(A.colptr.device.index or 0)
    opts = make_opts(**opt_kw)
    vdt = torch.float64 if opts.v_dtype == F64 else torch.float32
    dev = A.colptr.device
    out = SVDResult(torch.empty(k, dtype=torch.float64, device=dev), torch.empty((A.M, k), dtype=vdt, device=dev),
                    torch.empty((A.N, k), dtype=torch.float64, device=dev), {})
    nbytes = int(lib().ranky_tall_workspace_bytes(A.M, A.N, A.nnz, k, ctypes.byref(opts)))
    if nbytes == 0:
        raise RankyError(E_INVALID, "invalid sizes for the workspace")
    ws = ctx.workspace(nbytes)
    info = Info()
    csc = A.struct()
    _check(lib().ranky_svd_tall(ctx.handle, ctypes.byref(csc), A.M, A.N, k, float(tol), ctypes.byref(opts), _ptr(ws),
                                ws.numel(), _ptr(out.sigma), _ptr(out.U), _ptr(out.V), ctypes.byref(info),
                                _stream(stream)))
    out.info = info.as_dict()
    return out


class Incremental:
    """ranky_inc_*: a resident Gram that column blocks of an M-row matrix are appended to; solve()
    gives the leading sigma and U of everything appended so far."""

    def __init__(self, M: int, k: int, max_cols: int, max_nnz: int, ctx: Context | None = None, device: int = 0,
                 stream=None, **opt_kw):
        self.ctx = ctx or context(device)
        self.M, self.k = M, k
        self.opts = make_opts(**opt_kw)
        nbytes = int(lib().ranky_inc_workspace_bytes(M, max_cols, max_nnz, k, ctypes.byref(self.opts)))
        if nbytes == 0:
            raise RankyError(E_INVALID, "invalid sizes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        h = ctypes.c_void_p()
        _check(lib().ranky_inc_create(self.ctx.handle, M, k, max_cols, max_nnz, ctypes.byref(self.opts),
                                      _ptr(self.ws), nbytes, ctypes.byref(h), _stream(stream)))
        self.handle = h

    def append(self, block: DeviceCSC, stream=None):
        csc = block.struct()
        _check(lib().ranky_inc_append(self.handle, ctypes.byref(csc), block.N, _stream(stream)))

    def solve(self, tol: float = 0.0, stream=None):
        dev = self.ws.device
        sigma = torch.empty(self.k, dtype=torch.float64, device=dev)
        U = torch.empty((self.M, self.k), dtype=torch.float64, device=dev)
        info = Info()
        _check(lib().ranky_inc_solve(self.handle, float(tol), _ptr(sigma), _ptr(U), ctypes.byref(info),
                                     _stream(stream)))
        return sigma, U, info.as_dict()

    def close(self):
        if self.handle:
            lib().ranky_inc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CHECKERS = {"none": -1, "random": 0, "neighbor": 1, "neighbor_random": 2}


def checker(A: DeviceCSC, D: int, kind: str, seed: int, stream=None):
    """ranky_checker: (A' as a DeviceCSC with FP64 values, entries added)."""
    dev = A.colptr.device
    cap = A.nnz + 2 * D * A.M
    colptr = torch.empty(A.N + 1, dtype=torch.int32, device=dev)
    rowidx = torch.empty(cap, dtype=torch.int32, device=dev)
    values = torch.empty(cap, dtype=torch.float64, device=dev)
    nbytes = int(lib().ranky_checker_workspace_bytes(A.M, A.N, A.nnz, D))
    if nbytes == 0:
        raise RankyError(E_INVALID, "invalid sizes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    nz, added = ctypes.c_int64(0), ctypes.c_int64(0)
    csc = A.struct()
    _check(lib().ranky_checker(ctypes.byref(csc), A.M, A.N, D, CHECKERS[kind], int(seed), _ptr(colptr), _ptr(rowidx),
                               _ptr(values), cap, ctypes.byref(nz), ctypes.byref(added), _ptr(ws), nbytes,
                               _stream(stream)))
    n = nz.value
    return DeviceCSC(A.M, A.N, colptr, rowidx[:n], values[:n]), added.value


def svd_paper(A: DeviceCSC, k: int, D: int, kind: str = "none", seed: int = 0, tol: float = 0.0,
              ctx: Context | None = None, stream=None):
    """ranky_svd_paper: (sigma [k], U [M x k], info dict) by the paper's proxy route."""
    ctx = ctx or context(A.colptr.device.index or 0)
    dev = A.colptr.device
    sigma = torch.empty(k, dtype=torch.float64, device=dev)
    U = torch.empty((A.M, k), dtype=torch.float64, device=dev)
    nbytes = int(lib().ranky_paper_workspace_bytes(A.M, A.N, A.nnz, k, D, CHECKERS[kind]))
    if nbytes == 0:
        raise RankyError(E_INVALID, "invalid sizes")
    ws = ctx.workspace(nbytes)
    info = PaperInfo()
    csc = A.struct()
    _check(lib().ranky_svd_paper(ctx.handle, ctypes.byref(csc), A.M, A.N, k, D, CHECKERS[kind], int(seed), float(tol),
                                 _ptr(ws), ws.numel(), _ptr(sigma), _ptr(U), ctypes.byref(info), _stream(stream)))
    return sigma, U, info.as_dict()


def paper_errors(sigma_hat, U_hat, sigma, U, stream=None):
    """ranky_paper_errors: (e_sigma, e_u) of Sec. IV over the k columns of U_hat."""
    M, k = U_hat.shape
    ws = torch.empty(k + 2, dtype=torch.float64, device=U_hat.device)
    es, eu = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().ranky_paper_errors(M, k, _ptr(sigma_hat.contiguous()), _ptr(U_hat.contiguous()),
                                    _ptr(sigma.contiguous()), _ptr(U.contiguous()), ctypes.byref(es),
                                    ctypes.byref(eu), _ptr(ws), 8 * (k + 2), _stream(stream)))
    return es.value, eu.value


NOALLOC_WORKSPACE_BYTES = 64 << 20


def svd_noalloc(A: DeviceCSC, k: int, tol: float = 0.0, ctx: Context | None = None, out: SVDResult | None = None,
                stream=None, **opt_kw) -> SVDResult:
    """ranky_svd_noalloc: the whole path in the library's fixed device array (no workspace)."""
    ctx = ctx or context(A.colptr.device.index or 0)
    opts = make_opts(**opt_kw)
    vdt = torch.float64 if opts.v_dtype == F64 else torch.float32
    dev = A.colptr.device
    if out is None:
        out = SVDResult(torch.empty(k, dtype=torch.float64, device=dev),
                        torch.empty((A.M, k), dtype=torch.float64, device=dev),
                        torch.empty((A.N, k), dtype=vdt, device=dev), {})
    info = Info()
    csc = A.struct()
    st = lib().ranky_svd_noalloc(ctx.handle, ctypes.byref(csc), A.M, A.N, k, float(tol), ctypes.byref(opts),
                                 _ptr(out.sigma), _ptr(out.U), _ptr(out.V), ctypes.byref(info), _stream(stream))
    _check(st)
    out.info = info.as_dict()
    return out


@dataclass
class AsyncSVD:
    """A ranky_svd_async call in flight: its ticket, where the result goes, and the
    tensors the call reads (kept alive until it finishes)."""
    ticket: int
    out: SVDResult
    ctx: "Context"
    keep: tuple


def svd_async(A: DeviceCSC, k: int, tol: float = 0.0, ctx: Context | None = None, out: SVDResult | None = None,
              workspace: torch.Tensor | None = None, stream=None, **opt_kw) -> AsyncSVD:
    """Starts ranky_svd_async and returns at once; `query` tells when the result is in `out`."""
    ctx = ctx or context(A.colptr.device.index or 0)
    opts = make_opts(**opt_kw)
    vdt = torch.float64 if opts.v_dtype == F64 else torch.float32
    dev = A.colptr.device
    if out is None:
        out = SVDResult(torch.empty(k, dtype=torch.float64, device=dev),
                        torch.empty((A.M, k), dtype=torch.float64, device=dev),
                        torch.empty((A.N, k), dtype=vdt, device=dev), {})
    nbytes = workspace_bytes(A.M, A.N, A.nnz, k, opts)
    if nbytes == 0:
        raise RankyError(E_INVALID, "invalid sizes for the workspace")
    ws = workspace if workspace is not None else ctx.workspace(nbytes)
    csc = A.struct()
    t = ctypes.c_uint64(0)
    st = lib().ranky_svd_async(ctx.handle, ctypes.byref(csc), A.M, A.N, k, float(tol), ctypes.byref(opts), _ptr(ws),
                               ws.numel(), _ptr(out.sigma), _ptr(out.U), _ptr(out.V), _stream(stream), ctypes.byref(t))
    _check(st)
    return AsyncSVD(t.value, out, ctx, (A, ws, opts))


def query(job: AsyncSVD) -> bool:
    """False while the call runs; True once it has finished (the result is in job.out and
    its info in job.out.info); an error of the call raises RankyError."""
    info = Info()
    st = lib().ranky_query(job.ctx.handle, job.ticket, ctypes.byref(info))
    if st == PENDING:
        return False
    _check(st)
    job.out.info = info.as_dict()
    return True


def autotune(A: DeviceCSC, k: int, ctx: Context | None = None, out: SVDResult | None = None,
             workspace: torch.Tensor | None = None, stream=None, **opt_kw) -> dict:
    """ranky_autotune: measure the launch-shape candidates on A and keep the fastest in ctx
    (later svd / batch calls on ctx with this shape use them).  Returns the report."""
    ctx = ctx or context(A.colptr.device.index or 0)
    opts = make_opts(**opt_kw)
    vdt = torch.float64 if opts.v_dtype == F64 else torch.float32
    dev = A.colptr.device
    if out is None:
        out = SVDResult(torch.empty(k, dtype=torch.float64, device=dev),
                        torch.empty((A.M, k), dtype=torch.float64, device=dev),
                        torch.empty((A.N, k), dtype=vdt, device=dev), {})
    nbytes = workspace_bytes(A.M, A.N, A.nnz, k, opts)
    ws = workspace if workspace is not None else ctx.workspace(nbytes)
    rep = TuneReport()
    csc = A.struct()
    _check(lib().ranky_autotune(ctx.handle, ctypes.byref(csc), A.M, A.N, k, ctypes.byref(opts), _ptr(ws), ws.numel(),
                                _ptr(out.sigma), _ptr(out.U), _ptr(out.V), ctypes.byref(rep), _stream(stream)))
    return rep.as_dict()


def tune_set(A: DeviceCSC, k: int, bp_per_cu: int, jacobi_schedule: int, ctx: Context | None = None, **opt_kw):
    """ranky_tune_set: fix the launch shapes for A's shape in ctx without measuring."""
    ctx = ctx or context(A.colptr.device.index or 0)
    opts = make_opts(**opt_kw)
    dt = F64 if A.values.dtype == torch.float64 else F32
    _check(lib().ranky_tune_set(ctx.handle, A.M, A.N, A.nnz, k, dt, ctypes.byref(opts), bp_per_cu, jacobi_schedule))


def occupancy(A: DeviceCSC, D: int, stream=None):
    """Alg. 1 scan: (cnt [D, M], rownnz [M], lonely [D], single [D]) as int32 device tensors."""
    dev = A.colptr.device
    cnt = torch.empty((D, A.M), dtype=torch.int32, device=dev)
    rownnz = torch.empty(A.M, dtype=torch.int32, device=dev)
    lonely = torch.empty(D, dtype=torch.int32, device=dev)
    single = torch.empty(D, dtype=torch.int32, device=dev)
    nbytes = int(lib().ranky_step_workspace_bytes(A.M, A.N, A.nnz, D))
    if nbytes == 0:
        raise RankyError(E_INVALID, "invalid sizes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    csc = A.struct()
    _check(lib().ranky_occupancy(ctypes.byref(csc), A.M, A.N, D, _ptr(cnt), _ptr(rownnz), _ptr(lonely),
                                 _ptr(single), _ptr(ws), nbytes, _stream(stream)))
    return cnt, rownnz, lonely, single


def gram(A: DeviceCSC, prec: str = "fp64", stream=None) -> torch.Tensor:
    dev = A.colptr.device
    G = torch.empty((A.M, A.M), dtype=torch.float64, device=dev)
    D = max(1, min(A.N, (A.N + 16383) // 16384))
    nbytes = int(lib().ranky_step_workspace_bytes(A.M, A.N, A.nnz, D))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    csc = A.struct()
    _check(lib().ranky_gram(ctypes.byref(csc), A.M, A.N, PREC[prec], _ptr(G), _ptr(ws), nbytes, _stream(stream)))
    return G


def eigh(G: torch.Tensor, max_sweeps: int = 0, stream=None):
    """Blocked Jacobi eigensolve of a dense symmetric FP64 matrix: (lambda unsorted, Q, sweeps)."""
    if G.dtype != torch.float64 or not G.is_cuda or G.dim() != 2 or G.shape[0] != G.shape[1]:
        raise TypeError("G must be a square float64 device tensor")
    G = G.contiguous()
    n = G.shape[0]
    lam = torch.empty(n, dtype=torch.float64, device=G.device)
    Q = torch.empty((n, n), dtype=torch.float64, device=G.device)
    nbytes = int(lib().ranky_eigh_workspace_bytes(n))
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=G.device)
    sw = ctypes.c_int32(0)
    _check(lib().ranky_eigh(n, _ptr(G), _ptr(lam), _ptr(Q), max_sweeps, ctypes.byref(sw), _ptr(ws), nbytes,
                            _stream(stream)))
    return lam, Q, int(sw.value)


def backproject(A: DeviceCSC, U: torch.Tensor, sigma: torch.Tensor, rank: int, v_dtype=torch.float64, stream=None):
    """V = A^T U Sigma^{-1} on the first `rank` columns, zero beyond (stream-ordered)."""
    k = U.shape[1]
    dev = A.colptr.device
    V = torch.empty((A.N, k), dtype=v_dtype, device=dev)
    r = torch.tensor([rank], dtype=torch.int32, device=dev)
    Uc, sc = U.contiguous(), sigma.contiguous()
    csc = A.struct()
    _check(lib().ranky_backproject(ctypes.byref(csc), A.M, A.N, k, _ptr(Uc), _ptr(sc), _ptr(r), _ptr(V),
                                   F64 if v_dtype == torch.float64 else F32, _stream(stream)))
    torch.cuda.current_stream().synchronize()
    return V


def batch(mats: list[DeviceCSC], ks: list[int], tol: float = 0.0, n_blocks: list[int] | None = None,
          ctx: Context | None = None, outs: list[SVDResult] | None = None, workspace: torch.Tensor | None = None,
          stream=None, gram_prec="fp64", v_dtype=torch.float64, graph=False, max_sweeps=0,
          check=True) -> list[SVDResult]:
    """All matrices through ranky_batch (one launch per phase for the whole batch; blocking).
    Returns one SVDResult per matrix; info["status"] carries each matrix's own status."""
    if not mats:
        raise ValueError("empty batch")
    ctx = ctx or context(mats[0].colptr.device.index or 0)
    opts = make_opts(gram_prec=gram_prec, refine=0, v_dtype=v_dtype, graph=graph, max_sweeps=max_sweeps)
    n = len(mats)
    items = (BatchItem * n)()
    if outs is None:
        outs = []
        for A, k in zip(mats, ks):
            dev = A.colptr.device
            outs.append(SVDResult(torch.empty(k, dtype=torch.float64, device=dev),
                                  torch.empty((A.M, k), dtype=torch.float64, device=dev),
                                  torch.empty((A.N, k), dtype=v_dtype, device=dev), {}))
    for i, (A, k, o) in enumerate(zip(mats, ks, outs)):
        items[i].A = A.struct()
        items[i].N = A.N
        items[i].M = A.M
        items[i].k = k
        items[i].n_blocks = 0 if n_blocks is None else n_blocks[i]
        items[i].sigma = o.sigma.data_ptr()
        items[i].U = o.U.data_ptr()
        items[i].V = o.V.data_ptr()
    nbytes = int(lib().ranky_batch_workspace_bytes(n, items, ctypes.byref(opts)))
    if nbytes == 0:
        raise RankyError(E_INVALID, "invalid batch sizes")
    ws = workspace if workspace is not None else ctx.workspace(nbytes)
    infos = (Info * n)()
    st = lib().ranky_batch(ctx.handle, n, items, float(tol), ctypes.byref(opts), _ptr(ws), ws.numel(), infos,
                           _stream(stream))
    for o, inf in zip(outs, infos):
        o.info = inf.as_dict()
    if check:
        _check(st)
    return outs


def batch_workspace_bytes(mats, ks, gram_prec="fp64", v_dtype=torch.float64, n_blocks=None) -> int:
    opts = make_opts(gram_prec=gram_prec, refine=0, v_dtype=v_dtype)
    n = len(mats)
    items = (BatchItem * n)()
    for i, (A, k) in enumerate(zip(mats, ks)):
        items[i].A.nnz = A.nnz
        items[i].N = A.N
        items[i].M = A.M
        items[i].k = k
        items[i].n_blocks = 0 if n_blocks is None else n_blocks[i]
    return int(lib().ranky_batch_workspace_bytes(n, items, ctypes.byref(opts)))


class Server:
    """Continuous-admission server (ranky_serve_*).  The arena is a device tensor owned by this
    object; request inputs and outputs are the caller's device tensors and must stay alive
    until the request completes."""

    def __init__(self, arena_bytes: int, max_slots: int = 4, max_queue: int = 1024, device: int = 0, **opt_kw):
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        cfg = ServeCfg()
        cfg.arena = self.arena.data_ptr()
        cfg.arena_bytes = arena_bytes
        cfg.max_slots = max_slots
        cfg.max_queue = max_queue
        cfg.device = device
        cfg.opts = make_opts(**opt_kw)
        self.opts = cfg.opts
        h = ctypes.c_void_p()
        _check(lib().ranky_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def footprint(self, A: DeviceCSC, k: int) -> int:
        return workspace_bytes(A.M, A.N, A.nnz, k, self.opts)

    def submit(self, A: DeviceCSC, k: int, out: SVDResult, tol: float = 0.0):
        """Returns (status, ticket); status E_BUSY / E_NOMEM is back-pressure, not an exception."""
        r = Request()
        r.A = A.struct()
        r.N, r.M, r.k, r.tol = A.N, A.M, k, float(tol)
        r.sigma, r.U, r.V = out.sigma.data_ptr(), out.U.data_ptr(), out.V.data_ptr()
        t = ctypes.c_uint64(0)
        st = lib().ranky_serve_submit(self.handle, ctypes.byref(r), ctypes.byref(t))
        if st == OK:
            self._keep[t.value] = (A, out)
        return st, t.value

    def poll(self, ticket: int):
        inf = Info()
        st = lib().ranky_serve_poll(self.handle, ticket, ctypes.byref(inf))
        return st, inf.as_dict()

    def wait(self, ticket: int, timeout_us: int = -1):
        inf = Info()
        st = lib().ranky_serve_wait(self.handle, ticket, timeout_us, ctypes.byref(inf))
        if st != PENDING:
            self._keep.pop(ticket, None)
        return st, inf.as_dict()

    def cancel(self, ticket: int) -> int:
        return lib().ranky_serve_cancel(self.handle, ticket)

    def stats(self) -> dict:
        s = ServeStats()
        _check(lib().ranky_serve_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self.handle:
            st = lib().ranky_serve_destroy(self.handle)
            self.handle = None
            self._keep.clear()
            _check(st)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

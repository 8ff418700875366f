"""MI355X (gfx950) sparse matrix-vector product and CG for finite-volume mesh
matrices -- thin Python binding over the C ABI in ``include/spmv.h``.

The binding only marshals arguments: every step of a product or a solve runs
in the HIP library ``libspmv_gfx950.so`` built next to this file.  PyTorch
provides device memory (tensors' ``data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``); nothing falls back to the CPU.
If the library cannot be loaded, every call raises.

Entry points mirror the C names: ``spmv_create`` (``Matrix(...)``),
``spmv_apply`` (``Matrix.apply``), ``spmv_apply_f32`` / ``spmv_apply_f32v`` /
``spmv_apply_bf16``, ``cg_solve`` (``Matrix.cg``), ``spmv_get_info``
(``Matrix.info``), ``spmv_plan_inspect`` (``plan_inspect``, host only).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmv_gfx950.so")

SPMV_OK, SPMV_EINVAL, SPMV_ENOMEM, SPMV_EDEVICE = 0, -1, -2, -3
SPMV_ENOTCONV, SPMV_EBUDGET, SPMV_ENOTSUP, SPMV_EBREAK = -4, -5, -6, -7
SPMV_VALUES_FP32, SPMV_VALUES_BF16, SPMV_NO_XCD_REMAP, SPMV_DEVICE_PTRS = 0x1, 0x2, 0x4, 0x8
SPMV_XCD_CONTIGUOUS = 0x10
WINDOW_AUTO, WINDOW_OFF, WINDOW_RING = 0, 1, 2
FORMAT_CSR, FORMAT_SELL = 0, 1
CG_FP64, CG_MIXED_FP32, CG_PCG_BF16, CG_MIXED_FP32V, CG_PCG_JACOBI, CG_FP64_ONE_REDUCTION = 0, 1, 2, 3, 4, 5

EXPORTED = [
    "spmv_create", "spmv_destroy", "spmv_get_info", "spmv_apply", "spmv_apply_f32",
    "spmv_apply_f32v", "spmv_apply_bf16", "cg_solve", "spmv_last_error", "spmv_plan_inspect",
    "spmv_create_bsr3", "bsr3_spmm", "bsr3_spmm_f32", "spmv_sell_inspect", "spmv_spmm", "spmv_calibrate_read",
    "cg_solve_noalloc",
]


class SpmvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class spmv_params(ctypes.Structure):
    _fields_ = [("tile_nnz", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("window_mode", ctypes.c_int32), ("ring_words", ctypes.c_int32),
                ("window_block", ctypes.c_int32), ("window_gap", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("format", ctypes.c_int32), ("sell_sigma", ctypes.c_int32),
                ("xcd_chunk", ctypes.c_int32), ("long_rows", ctypes.c_int32)]


class spmv_info(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("tile_nnz", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("n_tiles", ctypes.c_int32), ("n_stream_tiles", ctypes.c_int32),
                ("n_long_rows", ctypes.c_int32), ("n_window_tiles", ctypes.c_int32),
                ("n_window_blocks", ctypes.c_int32), ("ring_words", ctypes.c_int32),
                ("window_words", ctypes.c_int64), ("n_runs", ctypes.c_int64), ("has_fp32", ctypes.c_int32),
                ("has_bf16", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
                ("block_size", ctypes.c_int32), ("format", ctypes.c_int32), ("n_slices", ctypes.c_int32),
                ("sell_entries", ctypes.c_int64), ("n_long_pieces", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("y_scratch_ok", ctypes.c_int32)]


class cg_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("graph_seconds", ctypes.c_double)]


_lib = None


def build() -> str:
    from . import _build
    return _build.build()


def lib():
    """The loaded HIP library (built first if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_double)
        L.spmv_create.restype = ctypes.c_int
        L.spmv_create.argtypes = [i32, i32, i64, vp, vp, vp, u32, ctypes.POINTER(spmv_params),
                                  ctypes.POINTER(vp)]
        L.spmv_destroy.restype = ctypes.c_int
        L.spmv_destroy.argtypes = [vp]
        L.spmv_get_info.restype = ctypes.c_int
        L.spmv_get_info.argtypes = [vp, ctypes.POINTER(spmv_info)]
        for f in ("spmv_apply", "spmv_apply_f32", "spmv_apply_f32v", "spmv_apply_bf16"):
            getattr(L, f).restype = ctypes.c_int
            getattr(L, f).argtypes = [vp, vp, vp, vp]
        L.spmv_workspace_bytes.restype = ctypes.c_int
        L.spmv_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.spmv_apply_ws.restype = ctypes.c_int
        L.spmv_apply_ws.argtypes = [vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.spmv_create_bsr3.restype = ctypes.c_int
        L.spmv_create_bsr3.argtypes = [i32, i32, i64, vp, vp, vp, u32, ctypes.POINTER(vp)]
        for f in ("bsr3_spmm", "bsr3_spmm_f32", "spmv_spmm"):
            getattr(L, f).restype = ctypes.c_int
            getattr(L, f).argtypes = [vp, i32, vp, vp, vp]
        for f in ("cg_solve", "cg_solve_noalloc"):
            getattr(L, f).restype = ctypes.c_int
            getattr(L, f).argtypes = [vp, vp, vp, dbl, i32, i32, ctypes.POINTER(cg_info), vp]
        L.spmv_calibrate_read.restype = ctypes.c_int
        L.spmv_calibrate_read.argtypes = [vp, i64, vp, i32, vp]
        L.spmv_last_error.restype = ctypes.c_char_p
        L.spmv_last_error.argtypes = []
        L.spmv_plan_inspect.restype = ctypes.c_int
        L.spmv_plan_inspect.argtypes = [i32, i32, i64, vp, vp, ctypes.POINTER(spmv_params),
                                        ctypes.POINTER(i32), vp, vp, vp, vp, vp, vp, vp, vp,
                                        ctypes.POINTER(spmv_info)]
        L.spmv_sell_inspect.restype = ctypes.c_int
        L.spmv_sell_inspect.argtypes = [i32, i32, i64, vp, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                        ctypes.POINTER(i32), vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != SPMV_OK:
        msg = lib().spmv_last_error().decode(errors="replace")
        raise SpmvError(rc, f"{what}: {msg}")


def _params(p: dict | None):
    if not p:
        return None
    sp = spmv_params()
    names = {f for f, _ in spmv_params._fields_}
    for k, v in p.items():
        if k not in names:
            raise ValueError(f"unknown spmv_params field {k!r}")
        setattr(sp, k, v)
    return ctypes.byref(sp)


def _host_csr(row_ptr, col_idx, values):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = None if values is None else np.ascontiguousarray(values, dtype=np.float64)
    return rp, ci, va


def _ptr(a):
    return None if a is None or a.size == 0 else a.ctypes.data


def _info_dict(inf: spmv_info) -> dict:
    return {k: getattr(inf, k) for k, _ in spmv_info._fields_}


def plan_inspect(n_rows: int, n_cols: int, row_ptr, col_idx, params: dict | None = None) -> dict:
    """Run the analysis plan on the host (no GPU).  Returns tile boundaries,
    kinds (0 direct, 1 long row, 2 ring window, 3 compact window), window
    offsets/counts/blocks, compact runs (first column, window position),
    window-relative indices (16-bit per entry, and packed 12-bit per tile and
    lane for 2048-entry tiles) and the summary."""
    rp, ci, _ = _host_csr(row_ptr, col_idx, None)
    L = lib()
    nt = ctypes.c_int32(0)
    inf = spmv_info()
    _check(L.spmv_plan_inspect(n_rows, n_cols, ci.shape[0], _ptr(rp), _ptr(ci), _params(params),
                               ctypes.byref(nt), None, None, None, None, None, None, None, None, ctypes.byref(inf)),
           "spmv_plan_inspect")
    n = nt.value
    out = {k: np.zeros(n + (1 if k == "seg_bound" else 0), np.int32)
           for k in ("seg_bound", "seg_kind", "win_off", "win_cnt", "win_block")}
    out["runs"] = np.zeros((inf.n_runs, 2), np.int32)
    out["lidx"] = np.zeros(ci.shape[0] if inf.n_runs else 0, np.uint16)
    _check(L.spmv_plan_inspect(n_rows, n_cols, ci.shape[0], _ptr(rp), _ptr(ci), _params(params),
                               ctypes.byref(nt), out["seg_bound"].ctypes.data,
                               out["seg_kind"].ctypes.data, out["win_off"].ctypes.data,
                               out["win_cnt"].ctypes.data, out["win_block"].ctypes.data,
                               _ptr(out["runs"]), _ptr(out["lidx"]), None, ctypes.byref(inf)),
           "spmv_plan_inspect")
    n_compact = int(np.sum(out["seg_kind"] == 3))
    packed = inf.tile_nnz == 2048 and n_compact > 0 and inf.n_runs > 0
    out["lidx12"] = np.zeros(768 * n_compact if packed else 0, np.uint32)
    if packed:
        _check(L.spmv_plan_inspect(n_rows, n_cols, ci.shape[0], _ptr(rp), _ptr(ci), _params(params),
                                   ctypes.byref(nt), None, None, None, None, None, None, None,
                                   _ptr(out["lidx12"]), ctypes.byref(inf)), "spmv_plan_inspect")
    out["info"] = _info_dict(inf)
    return out


def sell_inspect(n_rows: int, n_cols: int, row_ptr, col_idx, sigma: int = 0) -> dict:
    """The sliced-ELLPACK layout of SPMV_FORMAT_SELL on the host (no GPU):
    slot rows (-1 empty), slot lengths, slice offsets, padded columns (long
    rows appended after the slices) and the long rows."""
    rp, ci, _ = _host_csr(row_ptr, col_idx, None)
    L = lib()
    ns, ne, nl = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int32(0)
    _check(L.spmv_sell_inspect(n_rows, n_cols, ci.shape[0], _ptr(rp), _ptr(ci), sigma, ctypes.byref(ns),
                               ctypes.byref(ne), ctypes.byref(nl), None, None, None, None, None), "spmv_sell_inspect")
    lens = np.diff(rp.astype(np.int64))
    n_long_entries = int(lens[lens > 255].sum())
    out = {"perm": np.zeros(64 * ns.value, np.int32), "len": np.zeros(64 * ns.value, np.uint8),
           "slice_ptr": np.zeros(ns.value + 1, np.int32), "col": np.zeros(ne.value + n_long_entries, np.int32),
           "long_rows": np.zeros(nl.value, np.int32)}
    _check(L.spmv_sell_inspect(n_rows, n_cols, ci.shape[0], _ptr(rp), _ptr(ci), sigma, ctypes.byref(ns),
                               ctypes.byref(ne), ctypes.byref(nl), _ptr(out["perm"]), _ptr(out["len"]),
                               out["slice_ptr"].ctypes.data, _ptr(out["col"]), _ptr(out["long_rows"])),
           "spmv_sell_inspect")
    out["n_slices"], out["n_entries"] = ns.value, ne.value
    return out


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        # the current stream's raw handle without building a Stream object
        # (2.5 us per call, a third of a small product's host cost); the same
        # stream torch.cuda.current_stream() names, capture streams included
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            return ctypes.c_void_p(raw(torch.cuda.current_device()))
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_vec(t, dtype, n: int, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")


@dataclass
class CGInfo:
    iterations: int
    refinements: int
    rel_residual: float
    seconds: float
    status: int
    graph_seconds: float = 0.0


class Matrix:
    """A resident CSR matrix (``spmv_create``).  Host arrays are copied to the
    current GPU; the handle is immutable and freed by ``close()``."""

    def __init__(self, n_rows: int, n_cols: int, row_ptr, col_idx, values, *,
                 fp32: bool = False, bf16: bool = False, xcd_remap: bool = True,
                 params: dict | None = None):
        rp, ci, va = _host_csr(row_ptr, col_idx, values)
        flags = (SPMV_VALUES_FP32 if fp32 else 0) | (SPMV_VALUES_BF16 if bf16 else 0)
        flags |= 0 if xcd_remap else SPMV_NO_XCD_REMAP
        h = ctypes.c_void_p()
        L = lib()
        _check(L.spmv_create(n_rows, n_cols, ci.shape[0], _ptr(rp), _ptr(ci), _ptr(va), flags,
                             _params(params), ctypes.byref(h)), "spmv_create")
        self._h = h
        self.n_rows, self.n_cols, self.nnz = n_rows, n_cols, int(ci.shape[0])

    @classmethod
    def from_device_csr(cls, n_rows: int, n_cols: int, row_ptr, col_idx, values, *,
                        fp32: bool = False, bf16: bool = False, xcd_remap: bool = True,
                        params: dict | None = None) -> "Matrix":
        """A resident CSR matrix from device tensors (int32 row_ptr and col_idx,
        float64 values, contiguous, on the current device) via
        ``SPMV_DEVICE_PTRS``."""
        torch = _torch()
        for t, dt, name in ((row_ptr, torch.int32, "row_ptr"), (col_idx, torch.int32, "col_idx"),
                            (values, torch.float64, "values")):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {dt} device tensor")
        if row_ptr.numel() != n_rows + 1 or values.numel() != col_idx.numel():
            raise ValueError("row_ptr needs n_rows + 1 entries and values one per column index")
        nnz = int(col_idx.numel())
        flags = SPMV_DEVICE_PTRS | (SPMV_VALUES_FP32 if fp32 else 0) | (SPMV_VALUES_BF16 if bf16 else 0)
        flags |= 0 if xcd_remap else SPMV_NO_XCD_REMAP
        h = ctypes.c_void_p()
        _check(lib().spmv_create(n_rows, n_cols, nnz, ctypes.c_void_p(row_ptr.data_ptr()),
                                 ctypes.c_void_p(col_idx.data_ptr() if nnz else None),
                                 ctypes.c_void_p(values.data_ptr() if nnz else None), flags,
                                 _params(params), ctypes.byref(h)), "spmv_create")
        self = cls.__new__(cls)
        self._h = h
        self.n_rows, self.n_cols, self.nnz = n_rows, n_cols, nnz
        return self

    @classmethod
    def from_csr(cls, A, **kw) -> "Matrix":
        if getattr(A, "block", 1) == 3:
            return cls.from_bsr3(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.values, **kw)
        return cls(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, A.values, **kw)

    @classmethod
    def from_bsr3(cls, n_block_rows: int, n_block_cols: int, brow_ptr, bcol_idx, bvalues, *,
                  fp32: bool = False, xcd_remap: bool = True, xcd_contiguous: bool = False) -> "Matrix":
        """A resident 3x3 block-CSR matrix (``spmv_create_bsr3``); bvalues has
        9 row-major values per block.  xcd_contiguous deals one contiguous
        range of tiles to each XCD (SPMV_XCD_CONTIGUOUS) instead of chunks."""
        rp, ci, _ = _host_csr(brow_ptr, bcol_idx, None)
        va = np.ascontiguousarray(bvalues, dtype=np.float64).reshape(-1)
        if va.shape[0] != 9 * ci.shape[0]:
            raise ValueError("bvalues must hold 9 values per block")
        flags = (SPMV_VALUES_FP32 if fp32 else 0) | (0 if xcd_remap else SPMV_NO_XCD_REMAP)
        flags |= SPMV_XCD_CONTIGUOUS if xcd_contiguous else 0
        h = ctypes.c_void_p()
        _check(lib().spmv_create_bsr3(n_block_rows, n_block_cols, ci.shape[0], _ptr(rp), _ptr(ci),
                                      _ptr(va), flags, ctypes.byref(h)), "spmv_create_bsr3")
        self = cls.__new__(cls)
        self._h = h
        self.n_rows, self.n_cols, self.nnz = 3 * n_block_rows, 3 * n_block_cols, int(ci.shape[0])
        return self

    def spmm(self, X, Y=None, stream=None):
        """Y = A X with k right-hand sides, X of shape (n_cols, k) row-major:
        ``bsr3_spmm`` for block-CSR handles (n_cols = 3 n_block_cols),
        ``spmv_spmm`` for scalar CSR handles."""
        torch = _torch()
        fn = "bsr3_spmm" if self.info["block_size"] == 3 else "spmv_spmm"
        return self._spmm(fn, X, Y, torch.float64, stream)

    def spmm_f32(self, X, Y=None, stream=None):
        torch = _torch()
        return self._spmm("bsr3_spmm_f32", X, Y, torch.float32, stream)

    def _spmm(self, fn, X, Y, dt, stream):
        torch = _torch()
        if X.dim() == 1:
            X = X.view(-1, 1)
        k = X.shape[1]
        _check_vec(X, dt, self.n_cols * k, "X")
        if Y is None:
            Y = torch.empty((self.n_rows, k), dtype=dt, device=X.device)
        _check_vec(Y, dt, self.n_rows * k, "Y")
        _check(getattr(lib(), fn)(self.handle, k, ctypes.c_void_p(X.data_ptr()),
                                  ctypes.c_void_p(Y.data_ptr()), _stream_ptr(stream)), fn)
        return Y

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("matrix handle is closed")
        return self._h

    @property
    def info(self) -> dict:
        inf = spmv_info()
        _check(lib().spmv_get_info(self.handle, ctypes.byref(inf)), "spmv_get_info")
        return _info_dict(inf)

    def _apply(self, fn: str, x, y, xdt, ydt, stream):
        torch = _torch()
        _check_vec(x, xdt, self.n_cols, "x")
        if y is None:
            y = torch.empty(self.n_rows, dtype=ydt, device=x.device)
        _check_vec(y, ydt, self.n_rows, "y")
        _check(getattr(lib(), fn)(self.handle, ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)), fn)
        return y

    def apply(self, x, y=None, stream=None):
        """y = A x in binary64 (``spmv_apply``)."""
        torch = _torch()
        return self._apply("spmv_apply", x, y, torch.float64, torch.float64, stream)

    @property
    def workspace_bytes(self) -> int:
        """Device bytes that ``apply_ws`` needs (``spmv_workspace_bytes``)."""
        n = ctypes.c_size_t()
        _check(lib().spmv_workspace_bytes(self.handle, ctypes.byref(n)), "spmv_workspace_bytes")
        return int(n.value)

    def apply_ws(self, x, y=None, ws=None, stream=None):
        """y = A x with the long rows' pieces on a workgroup each
        (``spmv_apply_ws``); ws: a device tensor of at least
        ``workspace_bytes`` bytes, allocated here when None."""
        torch = _torch()
        _check_vec(x, torch.float64, self.n_cols, "x")
        if y is None:
            y = torch.empty(self.n_rows, dtype=torch.float64, device=x.device)
        _check_vec(y, torch.float64, self.n_rows, "y")
        need = self.workspace_bytes
        if ws is None and need:
            ws = torch.empty((need + 7) // 8, dtype=torch.float64, device=x.device)
        wp = ws.data_ptr() if ws is not None else None
        wb = ws.numel() * ws.element_size() if ws is not None else 0
        _check(lib().spmv_apply_ws(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   ctypes.c_void_p(wp), wb, _stream_ptr(stream)), "spmv_apply_ws")
        return y

    def apply_f32(self, x, y=None, stream=None):
        torch = _torch()
        return self._apply("spmv_apply_f32", x, y, torch.float32, torch.float32, stream)

    def apply_f32v(self, x, y=None, stream=None):
        torch = _torch()
        return self._apply("spmv_apply_f32v", x, y, torch.float64, torch.float64, stream)

    def apply_bf16(self, x, y=None, stream=None):
        torch = _torch()
        return self._apply("spmv_apply_bf16", x, y, torch.float32, torch.float32, stream)

    def cg(self, b, x=None, tol: float = 1e-10, max_iter: int = 20000, mode: int = CG_FP64,
           stream=None, raise_on_error: bool = True):
        """Solve A x = b (``cg_solve``); returns (x, CGInfo)."""
        torch = _torch()
        _check_vec(b, torch.float64, self.n_rows, "b")
        if x is None:
            x = torch.zeros(self.n_rows, dtype=torch.float64, device=b.device)
        _check_vec(x, torch.float64, self.n_rows, "x")
        inf = cg_info()
        rc = lib().cg_solve(self.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                            tol, max_iter, mode, ctypes.byref(inf), _stream_ptr(stream))
        if raise_on_error and rc not in (SPMV_OK,):
            _check(rc, "cg_solve")
        return x, CGInfo(inf.iterations, inf.refinements, inf.rel_residual, inf.seconds, rc, inf.graph_seconds)

    def cg_noalloc(self, b, x=None, tol: float = 1e-10, max_iter: int = 20000, stream=None,
                   raise_on_error: bool = True):
        """``cg_solve_noalloc``: the FP64 solve on the library's per-device
        scratch array (no allocation inside the call; at most 2^19 rows; calls
        on one GPU must not overlap).  Returns (x, CGInfo)."""
        torch = _torch()
        _check_vec(b, torch.float64, self.n_rows, "b")
        if x is None:
            x = torch.zeros(self.n_rows, dtype=torch.float64, device=b.device)
        _check_vec(x, torch.float64, self.n_rows, "x")
        inf = cg_info()
        rc = lib().cg_solve_noalloc(self.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                    tol, max_iter, CG_FP64, ctypes.byref(inf), _stream_ptr(stream))
        if raise_on_error and rc not in (SPMV_OK,):
            _check(rc, "cg_solve_noalloc")
        return x, CGInfo(inf.iterations, inf.refinements, inf.rel_residual, inf.seconds, rc, inf.graph_seconds)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().spmv_destroy(self._h), "spmv_destroy")
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ------------------------------------------------------------------ serving

SRV_SPMV, SRV_CG = 0, 1


class srv_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("n_slots", ctypes.c_int32),
                ("cg_mode", ctypes.c_int32), ("max_round_tiles", ctypes.c_int32), ("preload", ctypes.c_int32),
                ("n_lanes", ctypes.c_int32), ("persistent_wgs", ctypes.c_int32),
                ("persist_idle_us", ctypes.c_int32), ("cg1_max_rows", ctypes.c_int32)]


class srv_result(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("op", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("latency_s", ctypes.c_double),
                ("queue_s", ctypes.c_double), ("wait_s", ctypes.c_double), ("copy_in_s", ctypes.c_double),
                ("compute_s", ctypes.c_double), ("copy_out_s", ctypes.c_double), ("graph_s", ctypes.c_double),
                ("dev_begin_s", ctypes.c_double), ("dev_end_s", ctypes.c_double), ("kernel_s", ctypes.c_double),
                ("_message", ctypes.c_char * 160)]

    @property
    def message(self) -> str:
        return self._message.decode(errors="replace")


class srv_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("uploads", ctypes.c_int64), ("evictions", ctypes.c_int64),
                ("used_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64), ("p50_s", ctypes.c_double),
                ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double), ("max_s", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("throughput_rps", ctypes.c_double),
                ("persist_launches", ctypes.c_int64), ("solver_reuses", ctypes.c_int64),
                ("solver_cached_bytes", ctypes.c_int64)]


EXPORTED += ["srv_create", "srv_add_matrix", "srv_submit", "srv_poll", "srv_wait", "srv_drain",
             "srv_get_stats", "srv_destroy", "srv_policy_simulate"]


def _serve_lib():
    L = lib()
    if not getattr(L, "_serve_ready", False):
        vp, i32, i64, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_double)
        L.srv_create.restype = ctypes.c_int
        L.srv_create.argtypes = [ctypes.POINTER(srv_config), ctypes.POINTER(vp)]
        L.srv_add_matrix.restype = ctypes.c_int
        L.srv_add_matrix.argtypes = [vp, i32, i32, i64, vp, vp, vp, ctypes.POINTER(i32)]
        L.srv_submit.restype = ctypes.c_int
        L.srv_submit.argtypes = [vp, i32, i32, i32, vp, vp, dbl, i32, ctypes.POINTER(u64)]
        for f in ("srv_poll", "srv_wait"):
            getattr(L, f).restype = ctypes.c_int
            getattr(L, f).argtypes = [vp, u64, ctypes.POINTER(srv_result)]
        L.srv_drain.restype = ctypes.c_int
        L.srv_drain.argtypes = [vp]
        L.srv_get_stats.restype = ctypes.c_int
        L.srv_get_stats.argtypes = [vp, ctypes.POINTER(srv_stats)]
        L.srv_destroy.restype = ctypes.c_int
        L.srv_destroy.argtypes = [vp]
        L.srv_policy_simulate.restype = ctypes.c_int
        L.srv_policy_simulate.argtypes = [u64, i32, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L._serve_ready = True
    return L


def calibrate_read(buf, partials, stream=None) -> None:
    """One streaming read of the float64 device tensor ``buf`` (16-byte
    aligned, even length) into one sum per workgroup in ``partials``
    (``spmv_calibrate_read``; grid = partials.numel() workgroups)."""
    torch = _torch()
    _check_vec(buf, torch.float64, buf.numel(), "buf")
    _check_vec(partials, torch.float64, partials.numel(), "partials")
    _check(lib().spmv_calibrate_read(ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                     ctypes.c_void_p(partials.data_ptr()), partials.numel(),
                                     _stream_ptr(stream)), "spmv_calibrate_read")


def policy_simulate(budget: int, mat_bytes, ops) -> list[tuple[int, int, int, int]]:
    """Replay the server's admission policy on the host.  ops: list of
    (kind, matrix, extra_bytes) with kind 0 = admit, 1 = release.  Returns per
    op (verdict, n_evicted, uploaded, used_bytes)."""
    L = _serve_lib()
    mb = np.ascontiguousarray(mat_bytes, np.uint64)
    kind = np.ascontiguousarray([o[0] for o in ops], np.int32)
    mat = np.ascontiguousarray([o[1] for o in ops], np.int32)
    ext = np.ascontiguousarray([o[2] for o in ops], np.uint64)
    n = len(ops)
    v, ne, up = (np.zeros(n, np.int32) for _ in range(3))
    used = np.zeros(n, np.uint64)
    _check(L.srv_policy_simulate(budget, mb.shape[0], _ptr(mb), n, _ptr(kind), _ptr(mat), _ptr(ext),
                                 _ptr(v), _ptr(ne), _ptr(up), _ptr(used)), "srv_policy_simulate")
    return [(int(a), int(b), int(c), int(d)) for a, b, c, d in zip(v, ne, up, used)]


class Server:
    """Continuous-batching request server (``srv_*``).  Host numpy buffers are
    kept alive until their request is reported done."""

    def __init__(self, hbm_budget_bytes: int = 0, n_slots: int = 0, cg_mode: int = CG_FP64,
                 max_round_tiles: int = 0, preload: bool = False, n_lanes: int = 0,
                 persistent_wgs: int = 0, persist_idle_us: int = 0, cg1_max_rows: int = 0):
        L = _serve_lib()
        cfg = srv_config(hbm_budget_bytes, n_slots, cg_mode, max_round_tiles, 1 if preload else 0, n_lanes,
                         persistent_wgs, persist_idle_us, cg1_max_rows)
        h = ctypes.c_void_p()
        _check(L.srv_create(ctypes.byref(cfg), ctypes.byref(h)), "srv_create")
        self._h = h
        self._shapes = []
        self._live = {}

    def add_matrix(self, A) -> int:
        rp, ci, va = _host_csr(A.row_ptr, A.col_idx, A.values)
        mid = ctypes.c_int32()
        _check(_serve_lib().srv_add_matrix(self._h, A.n_rows, A.n_cols, ci.shape[0], _ptr(rp), _ptr(ci),
                                           _ptr(va), ctypes.byref(mid)), "srv_add_matrix")
        self._shapes.append((A.n_rows, A.n_cols))
        return mid.value

    def submit_spmv(self, mid: int, X) -> int:
        """X: (k, n_cols) float64; the result is (k, n_rows)."""
        if not 0 <= mid < len(self._shapes):
            dummy = np.zeros(1)
            return self._submit(mid, SRV_SPMV, 1, dummy, dummy, 0.0, 0)   # the library rejects the id
        n_rows, n_cols = self._shapes[mid]
        X = np.ascontiguousarray(np.atleast_2d(X), np.float64)
        if X.shape[1] != n_cols:
            raise ValueError("X must have n_cols columns")
        Y = np.empty((X.shape[0], n_rows), np.float64)
        return self._submit(mid, SRV_SPMV, X.shape[0], X, Y, 0.0, 0)

    def submit_cg(self, mid: int, b, tol: float = 1e-8, max_iter: int = 20000) -> int:
        n_rows, _ = self._shapes[mid]
        b = np.ascontiguousarray(b, np.float64)
        x = np.empty(n_rows, np.float64)
        return self._submit(mid, SRV_CG, 1, b, x, tol, max_iter)

    def _submit(self, mid, op, k, inp, out, tol, max_iter) -> int:
        t = ctypes.c_uint64()
        _check(_serve_lib().srv_submit(self._h, mid, op, k, _ptr(inp), _ptr(out), tol, max_iter,
                                       ctypes.byref(t)), "srv_submit")
        self._live[t.value] = (inp, out)
        return t.value

    def poll(self, ticket: int):
        r = srv_result()
        _check(_serve_lib().srv_poll(self._h, ticket, ctypes.byref(r)), "srv_poll")
        return r

    def wait(self, ticket: int):
        """Blocks; returns (output array, srv_result)."""
        r = srv_result()
        _check(_serve_lib().srv_wait(self._h, ticket, ctypes.byref(r)), "srv_wait")
        inp, out = self._live.pop(ticket)
        return out, r

    def drain(self):
        _check(_serve_lib().srv_drain(self._h), "srv_drain")

    def stats(self) -> dict:
        s = srv_stats()
        _check(_serve_lib().srv_get_stats(self._h, ctypes.byref(s)), "srv_get_stats")
        return {k: getattr(s, k) for k, _ in srv_stats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_serve_lib().srv_destroy(self._h), "srv_destroy")
        self._h = None
        self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

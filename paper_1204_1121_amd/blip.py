"""Python binding of libblip (ctypes): argument marshalling only.

Every step of the evaluation runs in the HIP kernels of ``libblip.so``;
this module hands torch device pointers and the current torch stream to
the C ABI (include/blip.h) and raises on a non-zero status.  There is no
CPU fallback: if the library is missing, importing the binding raises.

PyTorch is used for device memory and streams only.  It must be imported
before the library is loaded so that both share one HIP runtime.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libblip.so")

BLIP_OK = 0
STATUS = {0: "BLIP_OK", -1: "BLIP_E_ARG", -2: "BLIP_E_OOM", -3: "BLIP_E_HIP",
          -4: "BLIP_E_DTYPE", -5: "BLIP_E_ALIGN", -6: "BLIP_E_STATE",
          -7: "BLIP_E_NODEV"}
STORAGE = {"f32": 0, "bf16": 1, "f16": 2, "c64": 3, "cbf16": 4, "cf16": 5}
KERNEL = {"auto": 0, "plain": 1, "tiled": 2, "f64acc": 3, "site": 4}


class BlipError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class EvalOpts(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("tile_pos", ctypes.c_int),
                ("vec", ctypes.c_int)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tile_pos", ctypes.c_int), ("vec", ctypes.c_int), ("us", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libblip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1204_1121_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    L.blip_load.restype = ci
    L.blip_load.argtypes = [dp, ci, ci, ci, ci, vp, ci, dp, ctypes.POINTER(vp)]
    L.blip_eval.restype = ci
    L.blip_eval.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.blip_eval_ex.restype = ci
    L.blip_eval_ex.argtypes = [vp, vp, i64, vp, vp, vp, ctypes.POINTER(EvalOpts), vp]
    L.blip_eval_batched.restype = ci
    L.blip_eval_batched.argtypes = [vp, vp, vp, ci, i64, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.blip_eval_batched_static.restype = ci
    L.blip_eval_batched_static.argtypes = [vp, vp, vp, ci, i64, vp, vp, vp, vp]
    L.blip_workspace_size.restype = ci
    L.blip_workspace_size.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_size_t)]
    L.blip_plan_create.restype = ci
    L.blip_plan_create.argtypes = [vp, vp, vp, ci, i64, vp, vp, vp, vp, ctypes.c_size_t,
                                   ctypes.POINTER(vp)]
    L.blip_plan_launch.restype = ci
    L.blip_plan_launch.argtypes = [vp, vp]
    L.blip_plan_free.restype = ci
    L.blip_plan_free.argtypes = [vp]
    L.blip_submit.restype = ci
    L.blip_submit.argtypes = [vp, vp, vp, vp, i64, vp, vp, ci, vp, vp, vp, vp, vp, vp]
    L.blip_autotune.restype = ci
    L.blip_autotune.argtypes = [vp, vp, vp, ci, i64, ci, vp, vp, vp, vp, ctypes.c_size_t, vp,
                                ctypes.POINTER(TuneResult), ci, ctypes.POINTER(ci),
                                ctypes.POINTER(TuneResult)]
    L.blip_set_shape.restype = ci
    L.blip_set_shape.argtypes = [vp, ci, i64, ci, ci]
    L.blip_get_shape.restype = ci
    L.blip_get_shape.argtypes = [vp, ci, i64, ctypes.POINTER(ci), ctypes.POINTER(ci)]
    L.blip_eval_ratio.restype = ci
    L.blip_eval_ratio.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp]
    L.blip_eval_ratio_values.restype = ci
    L.blip_eval_ratio_values.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, vp, vp, vp, vp]
    L.blip_eval_ratio_batched.restype = ci
    L.blip_eval_ratio_batched.argtypes = [vp, vp, vp, ci, i64, vp, i64, vp, vp, vp, vp, vp,
                                          ctypes.c_size_t, vp]
    L.blip_eval_ratio_values_batched.restype = ci
    L.blip_eval_ratio_values_batched.argtypes = [vp, vp, vp, ci, i64, vp, i64, vp, vp, vp, vp,
                                                 vp, vp, vp, ctypes.c_size_t, vp]
    L.blip_sm_update.restype = ci
    L.blip_sm_update.argtypes = [i64, vp, i64, vp, i64, i64, vp, vp, i64, vp, vp,
                                 ctypes.c_size_t, vp]
    L.blip_sm_workspace_size.restype = ctypes.c_size_t
    L.blip_sm_workspace_size.argtypes = [i64]
    L.blip_sm_update_batched.restype = ci
    L.blip_sm_update_batched.argtypes = [ci, i64, vp, i64, i64, vp, i64, i64, vp, i64, vp, ci,
                                         vp, i64, vp, ctypes.c_size_t, vp]
    L.blip_sm_batched_workspace_size.restype = ctypes.c_size_t
    L.blip_sm_batched_workspace_size.argtypes = [ci, i64]
    L.blip_qs_propose.restype = ci
    L.blip_qs_propose.argtypes = [i64, vp, vp, vp, vp]
    L.blip_qs_accept.restype = ci
    L.blip_qs_accept.argtypes = [ci, ci, ci, ci, vp, vp, vp, vp, vp, i64, vp, vp]
    L.blip_qs_kinetic.restype = ci
    L.blip_qs_kinetic.argtypes = [ci, ci, vp, vp, vp]
    L.blip_qs_copy_rows.restype = ci
    L.blip_qs_copy_rows.argtypes = [ci, ci, ci, vp, i64, vp, vp, i64, vp, i64, vp]
    L.blip_qs_lap_ratios.restype = ci
    L.blip_qs_lap_ratios.argtypes = [i64, ci, vp, i64, vp, i64, vp, vp]
    L.blip_stream_read.restype = ci
    L.blip_stream_read.argtypes = [vp, ctypes.c_size_t, vp, ci, vp]
    L.blip_stream_read_runs.restype = ci
    L.blip_stream_read_runs.argtypes = [vp, ctypes.c_size_t, vp, ci, ci, vp, ci, vp]
    L.blip_table_info.restype = ci
    L.blip_table_info.argtypes = [vp, ctypes.POINTER(ci), ctypes.POINTER(ci),
                                  ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.blip_free.restype = ci
    L.blip_free.argtypes = [vp]
    L.blip_last_error.restype = ctypes.c_char_p
    L.blip_last_error.argtypes = []
    L.blip_version.restype = ctypes.c_char_p
    L.blip_version.argtypes = []
    _lib = L
    return L


def check(status: int) -> None:
    if status != BLIP_OK:
        raise BlipError(status, lib().blip_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_ptr(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Table:
    """A coefficient table resident on the current GPU (``blip_load``)."""

    def __init__(self, lattice, n, coef: np.ndarray, storage: str = "f32",
                 kvec=None):
        L = lib()
        n1, n2, n3 = (int(v) for v in n)
        cplx = storage in ("c64", "cbf16", "cf16")
        want = np.complex64 if cplx else np.float32
        coef = np.ascontiguousarray(coef, dtype=want)
        if coef.ndim != 4 or coef.shape[:3] != (n1, n2, n3):
            raise ValueError("coef must be [n1, n2, n3, L]")
        self.norb = int(coef.shape[3])
        self.complex = cplx
        self.storage = storage
        self.n = (n1, n2, n3)
        self.lattice = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
        k = None if kvec is None else np.ascontiguousarray(np.asarray(kvec, np.float64).reshape(3))
        h = ctypes.c_void_p()
        check(L.blip_load(_dptr(self.lattice), n1, n2, n3, self.norb,
                          coef.ctypes.data_as(ctypes.c_void_p), STORAGE[storage],
                          _dptr(k) if k is not None else None, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise BlipError(-6, "table already freed")
        return self._h

    def info(self) -> dict:
        norb, st = ctypes.c_int(), ctypes.c_int()
        rb, db = ctypes.c_int64(), ctypes.c_int64()
        check(lib().blip_table_info(self.handle, ctypes.byref(norb), ctypes.byref(st),
                                    ctypes.byref(rb), ctypes.byref(db)))
        return {"norb": norb.value, "storage": st.value, "row_bytes": rb.value,
                "device_bytes": db.value}

    def alloc_outputs(self, npos: int, grad: bool = True, device=None, f64: bool = False):
        """Output tensors [npos, L], [npos, 3, L], [npos, L]: complex64 or
        float32 (float64 for the FP64-accumulate debug kernel)."""
        dt = torch.complex64 if self.complex else (torch.float64 if f64 else torch.float32)
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        val = torch.empty((npos, self.norb), dtype=dt, device=dev)
        if not grad:
            return val, None, None
        g = torch.empty((npos, 3, self.norb), dtype=dt, device=dev)
        lap = torch.empty((npos, self.norb), dtype=dt, device=dev)
        return val, g, lap

    def eval(self, pos: torch.Tensor, grad: bool = True, out=None, kernel: str = "auto",
             tile_pos: int = 0, vec: int = 0, stream=None):
        """Evaluate at positions ``pos`` (cuda float64 [npos, 3]); returns
        (val, grad, lap) tensors (grad/lap None for values only)."""
        if pos.dtype != torch.float64 or not pos.is_cuda or not pos.is_contiguous():
            raise ValueError("pos must be a contiguous float64 CUDA tensor [npos, 3]")
        npos = pos.shape[0]
        if out is None:
            out = self.alloc_outputs(npos, grad, pos.device, f64=(kernel == "f64acc"))
        val, g, lap = out
        sp = _stream_ptr(stream)
        if kernel == "auto" and tile_pos == 0 and vec == 0:
            check(lib().blip_eval(self.handle, _ptr(pos), npos, _ptr(val), _ptr(g), _ptr(lap), sp))
        else:
            o = EvalOpts(KERNEL[kernel], int(tile_pos), int(vec))
            check(lib().blip_eval_ex(self.handle, _ptr(pos), npos, _ptr(val), _ptr(g), _ptr(lap),
                                     ctypes.byref(o), sp))
        return val, g, lap

    def bind(self, pos: torch.Tensor, out, stream=None, kernel: str = "auto",
             tile_pos: int = 0, vec: int = 0):
        """A zero-argument callable that runs ``blip_eval`` (``blip_eval_ex``
        for an explicit kernel or shape) on fixed buffers with the ctypes
        arguments built once (low host overhead per call)."""
        if pos.dtype != torch.float64 or not pos.is_cuda or not pos.is_contiguous():
            raise ValueError("pos must be a contiguous float64 CUDA tensor [npos, 3]")
        val, g, lap = out
        args = (self.handle, _ptr(pos), ctypes.c_int64(pos.shape[0]), _ptr(val), _ptr(g),
                _ptr(lap))
        if kernel == "auto" and tile_pos == 0 and vec == 0:
            fn = lib().blip_eval
            args = args + (_stream_ptr(stream),)
        else:
            fn = lib().blip_eval_ex
            opts = EvalOpts(KERNEL[kernel], int(tile_pos), int(vec))
            args = args + (ctypes.byref(opts), _stream_ptr(stream))
        err = lib().blip_last_error

        def call():
            rc = fn(*args)
            if rc != BLIP_OK:
                raise BlipError(rc, err().decode())
        return call

    # -- fused acceptance ratios ---------------------------------------------

    def ratio(self, pos: torch.Tensor, inv_rows: torch.Tensor, row_of=None,
              grad: bool = True, out=None, stream=None):
        """Acceptance ratios against the old inverse (blip_eval_ratio).
        inv_rows: cuda float64 [nrows, >= L], row r = column of D^{-1};
        row_of: cuda int64 [npos] or None (row j for position j).
        Returns (ratio [npos], grad [npos, 3] or None, lap [npos] or None)."""
        if inv_rows.dtype != torch.float64 or inv_rows.dim() != 2 or inv_rows.stride(1) != 1:
            raise ValueError("inv_rows must be a float64 CUDA matrix with unit column stride")
        npos = pos.shape[0]
        if out is None:
            dev = pos.device
            r = torch.empty(npos, dtype=torch.float64, device=dev)
            g = torch.empty((npos, 3), dtype=torch.float64, device=dev) if grad else None
            l = torch.empty(npos, dtype=torch.float64, device=dev) if grad else None
            out = (r, g, l)
        r, g, l = out
        check(lib().blip_eval_ratio(self.handle, _ptr(pos), npos, _ptr(inv_rows),
                                    inv_rows.stride(0), _ptr(row_of), _ptr(r), _ptr(g),
                                    _ptr(l), _stream_ptr(stream)))
        return r, g, l

    def ratio_values(self, pos: torch.Tensor, inv_rows: torch.Tensor, row_of=None, out=None,
                     lap: bool = False, stream=None):
        """blip_eval_ratio_values: the ratios and, in the same pass, the orbital
        values.  Returns (ratio [npos] float64, val [npos, L] float32); with
        lap=True (ratio, grad_ratio [npos, 3], lap_ratio [npos], val,
        lap_rows [npos, L] float32)."""
        if inv_rows.dtype != torch.float64 or inv_rows.dim() != 2 or inv_rows.stride(1) != 1:
            raise ValueError("inv_rows must be a float64 CUDA matrix with unit column stride")
        npos = pos.shape[0]
        dev = pos.device
        if out is None:
            out = (torch.empty(npos, dtype=torch.float64, device=dev),
                   torch.empty((npos, self.norb), dtype=torch.float32, device=dev))
            if lap:
                out = (out[0], torch.empty((npos, 3), dtype=torch.float64, device=dev),
                       torch.empty(npos, dtype=torch.float64, device=dev), out[1],
                       torch.empty((npos, self.norb), dtype=torch.float32, device=dev))
        if lap:
            r, g, lr, v, lrow = out
        else:
            (r, v), g, lr, lrow = out, None, None, None
        check(lib().blip_eval_ratio_values(self.handle, _ptr(pos), npos, _ptr(inv_rows),
                                           inv_rows.stride(0), _ptr(row_of), _ptr(r), _ptr(g),
                                           _ptr(lr), _ptr(v), _ptr(lrow), _stream_ptr(stream)))
        return (r, g, lr, v, lrow) if lap else (r, v)

    def ratio_batched(self, pos, offsets, inv_rows, row_of=None, grad: bool = True, out=None,
                      workspace=None, capacity: int | None = None, stream=None):
        """blip_eval_ratio_batched: ratios for concatenated walker blocks."""
        cap = pos.shape[0] if capacity is None else int(capacity)
        if out is None:
            dev = pos.device
            out = (torch.empty(cap, dtype=torch.float64, device=dev),
                   torch.empty((cap, 3), dtype=torch.float64, device=dev) if grad else None,
                   torch.empty(cap, dtype=torch.float64, device=dev) if grad else None)
        if workspace is None:
            workspace = self.workspace(cap, pos.device)
        r, g, l = out
        check(lib().blip_eval_ratio_batched(self.handle, _ptr(pos), _ptr(offsets),
                                            int(offsets.shape[0]) - 1, cap, _ptr(inv_rows),
                                            inv_rows.stride(0), _ptr(row_of), _ptr(r), _ptr(g),
                                            _ptr(l), _ptr(workspace), workspace.numel(),
                                            _stream_ptr(stream)))
        return r, g, l

    def ratio_values_batched(self, pos, offsets, inv_rows, row_of=None, out=None, lap=False,
                             workspace=None, capacity: int | None = None, stream=None):
        """blip_eval_ratio_values_batched: ratio_values for concatenated
        walker blocks in one sorted persistent launch.  Returns (ratio, val),
        or with lap=True (ratio, grad_ratio, lap_ratio, val, lap_rows), with
        ``capacity`` rows."""
        if inv_rows.dtype != torch.float64 or inv_rows.dim() != 2 or inv_rows.stride(1) != 1:
            raise ValueError("inv_rows must be a float64 CUDA matrix with unit column stride")
        if offsets.dtype != torch.int64 or not offsets.is_cuda:
            raise ValueError("offsets must be a CUDA int64 tensor [nw+1]")
        cap = pos.shape[0] if capacity is None else int(capacity)
        dev = pos.device
        if out is None:
            out = (torch.empty(cap, dtype=torch.float64, device=dev),
                   torch.empty((cap, self.norb), dtype=torch.float32, device=dev))
            if lap:
                out = (out[0], torch.empty((cap, 3), dtype=torch.float64, device=dev),
                       torch.empty(cap, dtype=torch.float64, device=dev), out[1],
                       torch.empty((cap, self.norb), dtype=torch.float32, device=dev))
        if lap:
            r, g, lr, v, lrow = out
        else:
            (r, v), g, lr, lrow = out, None, None, None
        if workspace is None:
            workspace = self.workspace(cap, dev)
        check(lib().blip_eval_ratio_values_batched(
            self.handle, _ptr(pos), _ptr(offsets), int(offsets.shape[0]) - 1, cap,
            _ptr(inv_rows), inv_rows.stride(0), _ptr(row_of), _ptr(r), _ptr(g), _ptr(lr),
            _ptr(v), _ptr(lrow), _ptr(workspace), workspace.numel(), _stream_ptr(stream)))
        return (r, g, lr, v, lrow) if lap else (r, v)

    # -- batched walker blocks -------------------------------------------

    def workspace_bytes(self, capacity: int) -> int:
        n = ctypes.c_size_t()
        check(lib().blip_workspace_size(self.handle, int(capacity), ctypes.byref(n)))
        return int(n.value)

    def workspace(self, capacity: int, device=None) -> torch.Tensor:
        """Device scratch for blip_eval_batched (torch allocations are 256-B aligned)."""
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        return torch.empty(max(1, self.workspace_bytes(capacity)), dtype=torch.uint8, device=dev)

    def eval_batched(self, pos: torch.Tensor, offsets: torch.Tensor, grad: bool = True,
                     out=None, workspace=None, capacity: int | None = None, stream=None):
        """Evaluate concatenated walker blocks; offsets is a cuda int64
        tensor [nw+1].  Returns (val, grad, lap) with ``capacity`` rows."""
        if offsets.dtype != torch.int64 or not offsets.is_cuda:
            raise ValueError("offsets must be a CUDA int64 tensor [nw+1]")
        cap = pos.shape[0] if capacity is None else int(capacity)
        if out is None:
            out = self.alloc_outputs(cap, grad, pos.device)
        if workspace is None:
            workspace = self.workspace(cap, pos.device)
        val, g, lap = out
        check(lib().blip_eval_batched(self.handle, _ptr(pos), _ptr(offsets),
                                      int(offsets.shape[0]) - 1, cap, _ptr(val), _ptr(g),
                                      _ptr(lap), _ptr(workspace), workspace.numel(),
                                      _stream_ptr(stream)))
        return val, g, lap

    def eval_batched_static(self, pos: torch.Tensor, offsets: torch.Tensor, out,
                            capacity: int | None = None, stream=None):
        """blip_eval_batched_static: the batched launch with the library's
        fixed scratch; out = (val, grad, lap) preallocated by the caller
        (grad = lap = None for values only).  Nothing is allocated."""
        if offsets.dtype != torch.int64 or not offsets.is_cuda:
            raise ValueError("offsets must be a CUDA int64 tensor [nw+1]")
        cap = pos.shape[0] if capacity is None else int(capacity)
        val, g, lap = out
        check(lib().blip_eval_batched_static(self.handle, _ptr(pos), _ptr(offsets),
                                             int(offsets.shape[0]) - 1, cap, _ptr(val), _ptr(g),
                                             _ptr(lap), _stream_ptr(stream)))
        return val, g, lap

    def plan(self, pos, offsets, out, workspace, capacity: int | None = None) -> "Plan":
        return Plan(self, pos, offsets, out, workspace, capacity)

    def autotune(self, pos, out, offsets=None, workspace=None, capacity: int | None = None,
                 rotate: int = 1, stream=None):
        """Time every (P, o) and keep the fastest for this size bucket.
        Blocks: pos holds ``rotate`` blocks of out's row count, used in turn.
        Returns (best, all) as dicts {tile_pos, vec, us}."""
        val, g, lap = out
        res = (TuneResult * 32)()
        n = ctypes.c_int()
        best = TuneResult()
        if offsets is None:
            npos = val.shape[0]
            if pos.shape[0] != npos * rotate:
                raise ValueError("pos must hold rotate blocks of the outputs' row count")
            check(lib().blip_autotune(self.handle, _ptr(pos), None, 0, npos, int(rotate),
                                      _ptr(val), _ptr(g), _ptr(lap), None, 0,
                                      _stream_ptr(stream), res, 32, ctypes.byref(n),
                                      ctypes.byref(best)))
        else:
            cap = pos.shape[0] if capacity is None else int(capacity)
            if workspace is None:
                workspace = self.workspace(cap, pos.device)
            check(lib().blip_autotune(self.handle, _ptr(pos), _ptr(offsets),
                                      int(offsets.shape[0]) - 1, cap, 1, _ptr(val), _ptr(g),
                                      _ptr(lap), _ptr(workspace), workspace.numel(),
                                      _stream_ptr(stream), res, 32, ctypes.byref(n),
                                      ctypes.byref(best)))
        conv = lambda r: {"tile_pos": r.tile_pos, "vec": r.vec, "us": r.us}
        return conv(best), [conv(res[i]) for i in range(n.value)]

    @staticmethod
    def _shape_mode(batched: bool, ratio: bool) -> int:
        # blip_shape_mode: block 0, batched 1, block ratio 2, batched ratio 3
        return (1 if batched else 0) + (2 if ratio else 0)

    def set_shape(self, npos: int, tile_pos: int, vec: int, batched: bool = False,
                  ratio: bool = False) -> None:
        """Launch shape for npos's size bucket: the single-block or batched
        path, plain or with the acceptance-ratio epilogue (ratio=True)."""
        check(lib().blip_set_shape(self.handle, self._shape_mode(batched, ratio), int(npos),
                                   int(tile_pos), int(vec)))

    def get_shape(self, npos: int, batched: bool = False, ratio: bool = False):
        P, o = ctypes.c_int(), ctypes.c_int()
        check(lib().blip_get_shape(self.handle, self._shape_mode(batched, ratio), int(npos),
                                   ctypes.byref(P), ctypes.byref(o)))
        return P.value, o.value

    def free(self) -> None:
        if getattr(self, "_h", None) is not None:
            check(lib().blip_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Submitter:
    """blip_submit on fixed buffers: pinned host staging of positions (and
    offsets), the device buffers they are copied to, the outputs, an optional
    plan captured on those buffers, a stream and an event, with the ctypes
    arguments built once, so one launch of a serving loop is one library
    call.  event is a torch.cuda.Event already recorded once (so that it has
    a HIP handle)."""

    def __init__(self, table: Table, host_pos: torch.Tensor, dev_pos: torch.Tensor, out,
                 stream, event, plan: "Plan | None" = None, host_off=None, dev_off=None,
                 kernel: str = "auto"):
        if not host_pos.is_pinned():
            raise ValueError("host_pos must be pinned host memory")
        if not event.cuda_event:
            raise ValueError("record the event once before building a Submitter")
        val, g, lap = out
        self._fn = lib().blip_submit
        self._opts = (None if kernel == "auto"
                      else ctypes.byref(EvalOpts(KERNEL[kernel], 0, 0)))
        self._h = table.handle
        self._plan = plan._h if plan is not None else None
        self._hpos, self._dpos = _ptr(host_pos), _ptr(dev_pos)
        self._hoff, self._doff = _ptr(host_off), _ptr(dev_off)
        self._noff = 0 if host_off is None else int(host_off.shape[0])
        self._out = (_ptr(val), _ptr(g), _ptr(lap))
        self._stream = _stream_ptr(stream)
        self._event = ctypes.c_void_p(event.cuda_event)
        self._keep = (table, host_pos, dev_pos, out, plan, host_off, dev_off, event)

    def __call__(self, npos: int, use_plan: bool = False) -> None:
        if use_plan:
            rc = self._fn(self._h, self._plan, None, self._hpos, npos, self._dpos, self._hoff,
                          self._noff, self._doff, None, None, None, self._stream, self._event)
        else:
            rc = self._fn(self._h, None, self._opts, self._hpos, npos, self._dpos, None, 0, None,
                          *self._out, self._stream, self._event)
        if rc != 0:
            raise BlipError(rc, lib().blip_last_error().decode())


class Plan:
    """blip_eval_batched captured into a HIP graph on fixed buffers."""

    def __init__(self, table: Table, pos, offsets, out, workspace, capacity=None):
        cap = pos.shape[0] if capacity is None else int(capacity)
        val, g, lap = out
        h = ctypes.c_void_p()
        check(lib().blip_plan_create(table.handle, _ptr(pos), _ptr(offsets),
                                     int(offsets.shape[0]) - 1, cap, _ptr(val), _ptr(g),
                                     _ptr(lap), _ptr(workspace), workspace.numel(),
                                     ctypes.byref(h)))
        self._h = h
        # keep the captured buffers alive as long as the plan
        self._keep = (table, pos, offsets, out, workspace)

    def launch(self, stream=None) -> None:
        check(lib().blip_plan_launch(self._h, _stream_ptr(stream)))

    def free(self) -> None:
        if getattr(self, "_h", None) is not None:
            check(lib().blip_plan_free(self._h))
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def stream_read(buf: torch.Tensor, partial: torch.Tensor, stream=None) -> None:
    """One streaming read of the device buffer buf (blip_stream_read):
    partial (cuda float32, one entry per workgroup) receives the sums of
    what each workgroup read."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous CUDA tensor")
    if partial.dtype != torch.float32 or not partial.is_cuda or not partial.is_contiguous():
        raise ValueError("partial must be a contiguous CUDA float32 tensor")
    check(lib().blip_stream_read(_ptr(buf), buf.numel() * buf.element_size(), _ptr(partial),
                                 partial.numel(), _stream_ptr(stream)))


def stream_read_runs(buf: torch.Tensor, offsets: torch.Tensor, run_bytes: int,
                     partial: torch.Tensor, stream=None) -> None:
    """Read runs of run_bytes bytes of buf at the byte offsets (cuda int64)
    (blip_stream_read_runs); partial receives per-workgroup sums."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous CUDA tensor")
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous CUDA int64 tensor")
    if partial.dtype != torch.float32 or not partial.is_cuda or not partial.is_contiguous():
        raise ValueError("partial must be a contiguous CUDA float32 tensor")
    check(lib().blip_stream_read_runs(_ptr(buf), buf.numel() * buf.element_size(), _ptr(offsets),
                                      offsets.numel(), run_bytes, _ptr(partial), partial.numel(),
                                      _stream_ptr(stream)))


def sm_workspace(n: int, device="cuda") -> torch.Tensor:
    """Workspace for sm_update on order-n matrices (blip_sm_workspace_size)."""
    nbytes = lib().blip_sm_workspace_size(int(n))
    if nbytes == 0:
        raise ValueError(f"n = {n} is out of range for blip_sm_update")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def sm_update(inv: torch.Tensor, u: torch.Tensor, cols, u_row=None, ratios=None,
              workspace=None, stream=None):
    """Sherman-Morrison update of the transposed inverse in place
    (blip_sm_update).  inv: cuda float64 [n, >= n] with unit column stride,
    row i = column i of D^{-1}; u: cuda float32 [rows, >= n], the new orbital
    rows; cols: host sequence of accepted electrons in move order; u_row: host
    sequence of the row of u each move reads (None: row cols[m]).  Returns the
    sequential ratios (cuda float64 [k])."""
    n = inv.shape[0]
    if inv.dtype != torch.float64 or inv.dim() != 2 or inv.stride(1) != 1 or inv.shape[1] < n:
        raise ValueError("inv must be a float64 CUDA matrix [n, >= n] with unit column stride")
    if u.dtype != torch.float32 or u.dim() != 2 or u.stride(1) != 1 or u.shape[1] < n:
        raise ValueError("u must be a float32 CUDA matrix [rows, >= n] with unit column stride")
    c = np.ascontiguousarray(np.asarray(cols, dtype=np.int64).reshape(-1))
    ur = None if u_row is None else np.ascontiguousarray(np.asarray(u_row, dtype=np.int64).reshape(-1))
    if ur is not None and ur.shape != c.shape:
        raise ValueError("u_row needs one entry per move")
    if ratios is None:
        ratios = torch.empty(c.size, dtype=torch.float64, device=inv.device)
    if workspace is None:
        workspace = sm_workspace(n, inv.device)
    check(lib().blip_sm_update(n, _ptr(inv), inv.stride(0), _ptr(u), u.shape[0], u.stride(0),
                               c.ctypes.data_as(ctypes.c_void_p),
                               None if ur is None else ur.ctypes.data_as(ctypes.c_void_p),
                               c.size, _ptr(ratios), _ptr(workspace), workspace.numel(),
                               _stream_ptr(stream)))
    return ratios


def sm_update_batched(inv: torch.Tensor, u: torch.Tensor, acc_cols: torch.Tensor,
                      acc_count: torch.Tensor, max_k: int, ratios=None, workspace=None,
                      stream=None):
    """Sherman-Morrison updates of many matrices in place
    (blip_sm_update_batched).  inv: cuda float64 [nmat, n, >= n] (row i of
    matrix q = column i of its D^{-1}); u: cuda float32 [nmat, n, >= n] (row c
    = new orbitals of electron c); acc_cols: cuda int32 [nmat, >= max_k]
    (accepted electrons in move order); acc_count: cuda int32 [nmat].
    Returns the sequential ratios, cuda float64 [nmat, max_k]."""
    nmat, n = inv.shape[0], inv.shape[1]
    if inv.dtype != torch.float64 or inv.dim() != 3 or inv.stride(2) != 1 or inv.shape[2] < n:
        raise ValueError("inv must be float64 [nmat, n, >= n] with unit column stride")
    if (u.dtype != torch.float32 or u.dim() != 3 or u.stride(2) != 1 or u.shape[0] != nmat
            or u.shape[1] < n or u.shape[2] < n):
        raise ValueError("u must be float32 [nmat, >= n, >= n] with unit column stride")
    if acc_cols.dtype != torch.int32 or acc_cols.dim() != 2 or acc_cols.stride(1) != 1:
        raise ValueError("acc_cols must be int32 [nmat, >= max_k]")
    if acc_count.dtype != torch.int32 or acc_count.numel() != nmat or not acc_count.is_contiguous():
        raise ValueError("acc_count must be a contiguous int32 [nmat]")
    if ratios is None:
        ratios = torch.empty((nmat, max(int(max_k), 1)), dtype=torch.float64, device=inv.device)
    if workspace is None:
        nbytes = lib().blip_sm_batched_workspace_size(nmat, n)
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=inv.device)
    check(lib().blip_sm_update_batched(nmat, n, _ptr(inv), inv.stride(0), inv.stride(1), _ptr(u),
                                       u.stride(0), u.stride(1), _ptr(acc_cols),
                                       acc_cols.stride(0), _ptr(acc_count), int(max_k),
                                       _ptr(ratios), ratios.stride(0), _ptr(workspace),
                                       workspace.numel(), _stream_ptr(stream)))
    return ratios


def version() -> str:
    return lib().blip_version().decode()

"""Python binding of libspmttkrp.so (include/spmttkrp.h): argument marshalling only.

Every computation runs inside the library (host preprocessing in C++, the
per-mode work in HIP kernels).  torch is imported first so the library binds
to the HIP runtime torch already loaded; torch supplies device memory and
streams.  If the library is not built, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmttkrp.so")

F32 = 0
BF16 = 1
FUSE_REMAP_NEXT = 1
AUTO_REMAP = 2

_STATUS = {0: "SPT_OK", 1: "SPT_ERR_INVALID_ARG", 2: "SPT_ERR_OUT_OF_RANGE", 3: "SPT_ERR_OOM",
           4: "SPT_ERR_HIP", 5: "SPT_ERR_STATE", 6: "SPT_ERR_NOT_SPD", 7: "SPT_ERR_UNSUPPORTED"}


class SptError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = _STATUS.get(status, str(status))
        self.message = message


class spt_opts(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_int32), ("copies", ctypes.c_int32),
                ("split_cap", ctypes.c_int64), ("prep", ctypes.c_int32),
                ("dr", ctypes.c_int32), ("layout", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class spt_info(ctypes.Structure):
    _fields_ = [("nmodes", ctypes.c_int32), ("cur_mode", ctypes.c_int32),
                ("kappa", ctypes.c_int32), ("record_bytes", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("dims", ctypes.c_int64 * 8),
                ("max_load", ctypes.c_int64 * 8), ("split_rows", ctypes.c_int64 * 8),
                ("norm_sq", ctypes.c_double), ("prep_seconds", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("remap_chunk", ctypes.c_int32)]


class spt_timing(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64 * 8), ("ec_ms", ctypes.c_double * 8),
                ("fixup_ms", ctypes.c_double * 8), ("als_ms", ctypes.c_double * 8),
                ("remap_ms", ctypes.c_double * 8)]


EXPORTS = ["spt_tensor_load_coo", "spt_remap_for_mode", "spt_mttkrp", "spt_cp_als_iter",
           "spt_cp_gradient", "spt_cp_loss", "spt_cp_adjoint", "spt_copy_probe", "spt_mttkrp_noalloc", "spt_tensor_info",
           "spt_tensor_get_remap", "spt_tensor_get_records", "spt_timing_control", "spt_tensor_free",
           "spt_plan_coo", "spt_status_str", "spt_last_error"]

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2405_08470_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.spt_tensor_load_coo.argtypes = [i32, vp, i64, vp, vp, vp, vp, vp]
    L.spt_remap_for_mode.argtypes = [vp, i32, vp]
    L.spt_mttkrp.argtypes = [vp, i32, vp, i32, i32, vp, ctypes.c_uint32, vp]
    L.spt_cp_als_iter.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    L.spt_cp_gradient.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    L.spt_cp_loss.argtypes = [vp, vp, i32, i32, vp, vp]
    L.spt_cp_adjoint.argtypes = [vp, vp, i32, i32, vp, vp]
    L.spt_copy_probe.argtypes = [vp, vp, i64, vp]
    L.spt_mttkrp_noalloc.argtypes = [vp, i32, vp, i32, i32, vp, ctypes.c_uint32, vp]
    L.spt_tensor_info.argtypes = [vp, vp]
    L.spt_tensor_get_remap.argtypes = [vp, i32, vp]
    L.spt_tensor_get_records.argtypes = [vp, vp, vp, vp]
    L.spt_tensor_free.argtypes = [vp]
    L.spt_timing_control.argtypes = [vp, i32, vp]
    L.spt_plan_coo.argtypes = [i32, vp, i64, vp, vp, vp, vp, vp, vp]
    L.spt_status_str.argtypes = [i32]
    L.spt_status_str.restype = ctypes.c_char_p
    L.spt_last_error.argtypes = []
    L.spt_last_error.restype = ctypes.c_char_p
    for name in EXPORTS[:-2]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != 0:
        raise SptError(rc, lib().spt_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


LAYOUTS = {"auto": 0, "word32": 1, "half16": 2, "packed": 3, "compact": 4}


def _opts(kappa: int, split_cap: Optional[int], copies: int, prep: str = "host",
          remap: str = "staged", layout: str = "auto") -> spt_opts:
    o = spt_opts()
    o.kappa = int(kappa)
    o.copies = int(copies)
    if prep not in ("host", "device"):
        raise ValueError("prep must be 'host' or 'device'")
    o.prep = 1 if prep == "device" else 0
    if remap not in ("staged", "fused"):
        raise ValueError("remap must be 'staged' or 'fused'")
    o.dr = 0 if remap == "staged" else 1
    if layout not in LAYOUTS:
        raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
    o.layout = LAYOUTS[layout]
    # split_cap: None -> default ceil(nnz/kappa); <= 0 -> never split
    o.split_cap = 0 if split_cap is None else (int(split_cap) if split_cap > 0 else -1)
    return o


def _host_coo(dims, indices, values=None):
    dims64 = np.ascontiguousarray(np.asarray(dims, dtype=np.int64))
    idx = np.ascontiguousarray(np.asarray(indices, dtype=np.int32))
    if idx.ndim != 2 or idx.shape[0] != dims64.shape[0]:
        raise ValueError("indices must be [nmodes, nnz]")
    val = None
    if values is not None:
        val = np.ascontiguousarray(np.asarray(values, dtype=np.float32))
        if val.shape != (idx.shape[1],):
            raise ValueError("values must be [nnz]")
    return dims64, idx, val


class Tensor:
    """A loaded tensor (opaque library handle)."""

    def __init__(self, handle: int, dims: Sequence[int], nnz: int):
        self._h = ctypes.c_void_p(handle)
        self.dims = tuple(int(d) for d in dims)
        self.nmodes = len(self.dims)
        self.nnz = int(nnz)
        self._loss_gen = 0  # forward passes run (cp_loss), for CPFitLoss

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h:
            raise ValueError("tensor already freed")
        return self._h

    def free(self) -> None:
        if self._h:
            _check(lib().spt_tensor_free(self._h))
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def tensor_load_coo(dims, indices, values, kappa: int = 0, split_cap: Optional[int] = None,
                    copies: int = 0, stream=None, prep: str = "host", remap: str = "staged",
                    layout: str = "auto") -> Tensor:
    """prep: "host" (planner threads) or "device" (planner kernels).
    remap: "staged" (a remap pass after the elementwise kernel) or "fused"
    (the elementwise kernel stores each record at its next position).
    layout: "auto", "word32", "half16", "packed" or "compact" (record layout)."""
    dims64, idx, val = _host_coo(dims, indices, values)
    out = ctypes.c_void_p()
    o = _opts(kappa, split_cap, copies, prep, remap, layout)
    _check(lib().spt_tensor_load_coo(len(dims64), dims64.ctypes.data, idx.shape[1], idx.ctypes.data,
                                     val.ctypes.data, ctypes.byref(o), _stream(stream),
                                     ctypes.byref(out)))
    return Tensor(out.value, dims64.tolist(), idx.shape[1])


def plan_coo(dims, indices, kappa: int = 0, split_cap: Optional[int] = None) -> Dict[str, np.ndarray]:
    dims64, idx, _ = _host_coo(dims, indices)
    N, nnz = idx.shape
    kout = ctypes.c_int32()
    o = _opts(kappa, split_cap, 0)
    # first call for kappa, then the outputs
    _check(lib().spt_plan_coo(N, dims64.ctypes.data, nnz, idx.ctypes.data, ctypes.byref(o),
                              None, None, None, ctypes.byref(kout)))
    k = kout.value
    part = np.empty((N, nnz), dtype=np.int32)
    remap = np.empty((N, nnz), dtype=np.int64)
    ptr = np.empty((N, k + 1), dtype=np.int64)
    _check(lib().spt_plan_coo(N, dims64.ctypes.data, nnz, idx.ctypes.data, ctypes.byref(o),
                              part.ctypes.data, remap.ctypes.data, ptr.ctypes.data,
                              ctypes.byref(kout)))
    return {"part": part, "remap": remap, "ptr": ptr, "kappa": k}


def _factor_ptrs(t: Tensor, factors: Sequence[Optional[torch.Tensor]], rank: int, skip: int = -1,
                 dtype=torch.float32):
    if len(factors) != t.nmodes:
        raise ValueError("one factor matrix per mode is required")
    arr = (ctypes.c_void_p * t.nmodes)()
    for w, f in enumerate(factors):
        if f is None:
            if w != skip:
                raise ValueError(f"factor {w} is None")
            arr[w] = None
            continue
        if not (f.is_cuda and f.dtype == dtype and f.is_contiguous()
                and tuple(f.shape) == (t.dims[w], rank)):
            raise ValueError(f"factor {w} must be a contiguous CUDA {dtype} tensor of shape "
                             f"({t.dims[w]}, {rank})")
        arr[w] = f.data_ptr()
    return arr


def remap_for_mode(t: Tensor, mode: int, stream=None) -> None:
    _check(lib().spt_remap_for_mode(t.handle, int(mode), _stream(stream)))


def mttkrp(t: Tensor, mode: int, factors: Sequence[Optional[torch.Tensor]], out: torch.Tensor,
           flags: int = 0, stream=None) -> torch.Tensor:
    rank = int(out.shape[1])
    present = [f for f in factors if f is not None]
    dtype = present[0].dtype if present else torch.float32
    if dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("factors must be float32 or bfloat16")
    arr = _factor_ptrs(t, factors, rank, skip=mode, dtype=dtype)
    if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
            and tuple(out.shape) == (t.dims[mode], rank)):
        raise ValueError("out must be a contiguous CUDA float32 tensor of shape (I_mode, R)")
    _check(lib().spt_mttkrp(t.handle, int(mode), arr, BF16 if dtype == torch.bfloat16 else F32,
                            rank, out.data_ptr(), int(flags), _stream(stream)))
    return out


def mttkrp_noalloc(t: Tensor, mode: int, factors: Sequence[Optional[torch.Tensor]], out: torch.Tensor,
                   flags: int = 0, stream=None) -> torch.Tensor:
    """``mttkrp`` through the allocation-free entry point (split-row partial
    sums in the library's fixed per-device buffer)."""
    rank = int(out.shape[1])
    present = [f for f in factors if f is not None]
    dtype = present[0].dtype if present else torch.float32
    if dtype not in (torch.float32, torch.bfloat16):
        raise ValueError("factors must be float32 or bfloat16")
    arr = _factor_ptrs(t, factors, rank, skip=mode, dtype=dtype)
    if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
            and tuple(out.shape) == (t.dims[mode], rank)):
        raise ValueError("out must be a contiguous CUDA float32 tensor of shape (I_mode, R)")
    _check(lib().spt_mttkrp_noalloc(t.handle, int(mode), arr, BF16 if dtype == torch.bfloat16 else F32,
                                    rank, out.data_ptr(), int(flags), _stream(stream)))
    return out


def cp_als_iter(t: Tensor, factors: Sequence[torch.Tensor], lam: torch.Tensor,
                want_fit: bool = True, stream=None, bf16_gather: bool = False) -> Optional[float]:
    rank = int(lam.shape[0])
    arr = _factor_ptrs(t, factors, rank)
    if not (lam.is_cuda and lam.dtype == torch.float64 and lam.is_contiguous()):
        raise ValueError("lambda must be a contiguous CUDA float64 tensor of shape (R,)")
    fit = ctypes.c_double(float("nan"))
    _check(lib().spt_cp_als_iter(t.handle, arr, BF16 if bf16_gather else F32, rank, lam.data_ptr(),
                                 ctypes.byref(fit) if want_fit else None, _stream(stream)))
    return fit.value if want_fit else None


def cp_gradient(t: Tensor, factors: Sequence[torch.Tensor], grads: Optional[List[torch.Tensor]] = None,
                stream=None):
    """loss = 1/2 sum_e (x_e - m_e)^2 over the stored nonzeros and its gradient
    with respect to every factor.  Returns (loss as a CUDA float64 tensor of
    shape (1,), grads)."""
    rank = int(factors[0].shape[1])
    arr = _factor_ptrs(t, factors, rank)
    if grads is None:
        grads = [torch.empty_like(f) for f in factors]
    garr = _factor_ptrs(t, grads, rank)
    loss = torch.empty(1, dtype=torch.float64, device=factors[0].device)
    _check(lib().spt_cp_gradient(t.handle, arr, F32, rank, garr, loss.data_ptr(), _stream(stream)))
    t._loss_gen += 1
    return loss, grads


def cp_loss(t: Tensor, factors: Sequence[torch.Tensor], stream=None) -> torch.Tensor:
    """loss = 1/2 sum_e (x_e - m_e)^2 over the stored nonzeros (forward kernel
    only; the handle keeps the residual stream for ``cp_adjoint``).  Returns a
    CUDA float64 tensor of shape (1,)."""
    rank = int(factors[0].shape[1])
    arr = _factor_ptrs(t, factors, rank)
    loss = torch.empty(1, dtype=torch.float64, device=factors[0].device)
    _check(lib().spt_cp_loss(t.handle, arr, F32, rank, loss.data_ptr(), _stream(stream)))
    t._loss_gen += 1
    return loss


def cp_adjoint(t: Tensor, factors: Sequence[torch.Tensor], grads: Optional[List[torch.Tensor]] = None,
               stream=None) -> List[torch.Tensor]:
    """Gradient of the last ``cp_loss`` with respect to every factor: the
    spMTTKRP of its residual stream in every mode."""
    rank = int(factors[0].shape[1])
    arr = _factor_ptrs(t, factors, rank)
    if grads is None:
        grads = [torch.empty_like(f) for f in factors]
    garr = _factor_ptrs(t, grads, rank)
    _check(lib().spt_cp_adjoint(t.handle, arr, F32, rank, garr, _stream(stream)))
    return grads


class CPFitLoss(torch.autograd.Function):
    """Least-squares CP fit over the stored nonzeros as an autograd function:
    forward runs the model-at-nonzeros kernel only; backward runs the adjoint
    (spMTTKRP of the residuals) and scales it by the incoming gradient."""

    @staticmethod
    def forward(ctx, t, *factors):
        fs = [f.detach().contiguous() for f in factors]
        loss = cp_loss(t, fs)
        ctx.t = t
        ctx.gen = t._loss_gen
        ctx.save_for_backward(*fs)
        return loss[0]

    @staticmethod
    def backward(ctx, gout):
        fs = ctx.saved_tensors
        t = ctx.t
        if t._loss_gen != ctx.gen:
            # another forward ran on this tensor since: its residuals first
            cp_loss(t, fs)
        grads = cp_adjoint(t, fs)
        return (None,) + tuple(g * gout.to(g.dtype) for g in grads)


def cp_fit_loss(t: Tensor, factors: Sequence[torch.Tensor]) -> torch.Tensor:
    return CPFitLoss.apply(t, *factors)


def copy_probe(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """dst <- src with the library's plain streaming copy kernel (the
    measured-achievable bandwidth); both contiguous CUDA tensors of the same
    byte size, a multiple of 16."""
    nb = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()
            and dst.numel() * dst.element_size() == nb):
        raise ValueError("src and dst must be contiguous CUDA tensors of equal byte size")
    _check(lib().spt_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nb,
                                _stream(stream)))


def tensor_info(t: Tensor) -> Dict[str, object]:
    i = spt_info()
    _check(lib().spt_tensor_info(t.handle, ctypes.byref(i)))
    N = i.nmodes
    return {"nmodes": N, "cur_mode": i.cur_mode, "kappa": i.kappa, "record_bytes": i.record_bytes,
            "nnz": i.nnz, "dims": list(i.dims[:N]), "max_load": list(i.max_load[:N]),
            "split_rows": list(i.split_rows[:N]), "norm_sq": i.norm_sq,
            "prep_seconds": i.prep_seconds, "device_bytes": i.device_bytes, "remap_chunk": i.remap_chunk}


def tensor_get_remap(t: Tensor, mode: int) -> np.ndarray:
    b = np.empty(t.nnz, dtype=np.int64)
    _check(lib().spt_tensor_get_remap(t.handle, int(mode), b.ctypes.data))
    return b


def tensor_get_records(t: Tensor):
    idx = np.empty((t.nmodes, t.nnz), dtype=np.int32)
    val = np.empty(t.nnz, dtype=np.float32)
    cur = ctypes.c_int32()
    _check(lib().spt_tensor_get_records(t.handle, idx.ctypes.data, val.ctypes.data,
                                        ctypes.byref(cur)))
    return idx, val, cur.value


def timing_control(t: Tensor, enable: bool, want: bool = True) -> Optional[Dict[str, list]]:
    """Returns the per-mode kernel-time totals so far (if want), then starts
    (enable) or stops recording."""
    tm = spt_timing()
    _check(lib().spt_timing_control(t.handle, 1 if enable else 0,
                                    ctypes.byref(tm) if want else None))
    if not want:
        return None
    N = t.nmodes
    return {"calls": list(tm.calls[:N]), "ec_ms": list(tm.ec_ms[:N]),
            "fixup_ms": list(tm.fixup_ms[:N]), "als_ms": list(tm.als_ms[:N]),
            "remap_ms": list(tm.remap_ms[:N])}


def tensor_free(t: Tensor) -> None:
    t.free()

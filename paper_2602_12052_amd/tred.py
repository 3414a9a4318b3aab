"""Thin Python binding of libtred.so (the gfx950 HIP library).

Every function marshals torch device tensors into the C ABI of ``include/tred.h``
and raises on a non-OK status; all arithmetic runs in the library's kernels.
There is no fallback: if the library is missing or no GPU is present, calls fail.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtred.so")

TRED_OK, TRED_EINVAL, TRED_ECAPACITY, TRED_EDEVICE, TRED_EUNSUPPORTED = range(5)
TRED_CONV_MPCP = 1
TRED_DIRECT_SPLIT = 1


class TredError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"tred status {status}: {msg}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("spacing", C.c_float * 3), ("npix", C.c_int32 * 2),
                ("sub", C.c_int32 * 2), ("nticks", C.c_int32)]


class Physics(C.Structure):
    _fields_ = [("v_drift", C.c_float), ("lifetime", C.c_float), ("diff_T", C.c_float),
                ("diff_L", C.c_float), ("sigma_min", C.c_float * 3), ("n_sigma", C.c_float),
                ("point_frac", C.c_float), ("n_gl", C.c_int32)]


class Blocking(C.Structure):
    _fields_ = [("blk_pix", C.c_int32 * 2), ("blk_ticks", C.c_int32)]


def grid_struct(g) -> Grid:
    if isinstance(g, Grid):
        return g
    return Grid((C.c_float * 3)(*g.origin), (C.c_float * 3)(*g.spacing), (C.c_int32 * 2)(*g.npix),
                (C.c_int32 * 2)(*g.sub), int(g.nticks))


def physics_struct(p) -> Physics:
    if isinstance(p, Physics):
        return p
    return Physics(p.v_drift, p.lifetime, p.diff_T, p.diff_L, (C.c_float * 3)(*p.sigma_min),
                   p.n_sigma, p.point_frac, int(p.n_gl))


def blocking_struct(b) -> Blocking:
    if isinstance(b, Blocking):
        return b
    return Blocking((C.c_int32 * 2)(*b.blk_pix), int(b.blk_ticks))


EXPORTS = [
    "tred_status_string", "tred_last_error", "tred_abi_version", "tred_build_id",
    "tred_effq_windows", "tred_effq",
    "tred_block_count", "tred_block_bin_workspace", "tred_block_bin", "tred_conv_plan_create",
    "tred_conv_plan_set_response", "tred_conv_plan_info", "tred_conv_plan_set_timing",
    "tred_block_conv",
    "tred_scatter_workspace", "tred_scatter_waveforms", "tred_conv_plan_destroy",
    "tred_direct_plan_create", "tred_direct_plan_set_response", "tred_block_conv_direct",
    "tred_direct_plan_destroy", "tred_block_bin_events_workspace", "tred_block_bin_events",
    "tred_scatter_events_workspace", "tred_scatter_waveforms_events",
    "tred_scatter_waveforms_adjoint", "tred_block_conv_adjoint", "tred_block_bin_adjoint",
    "tred_effq_adjoint", "tred_block_row_words", "tred_block_bin_rows", "tred_block_conv_rows",
    "tred_block_bin_events_rows", "tred_block_conv_adjoint_rows", "tred_block_bin_rows_noalloc",
    "tred_effq_bin", "tred_effq_bin_events",
]

_lib = None


def lib():
    """Load libtred.so; raises if it has not been built, or if it was built from
    other sources than the tree's (its tred_build_id() differs)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2602_12052_amd.build.build()")
    from . import build as _build
    L = C.CDLL(LIB_PATH)
    P, I32, I64, U32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
    L.tred_build_id.restype = C.c_char_p
    want, got = _build.source_id(), L.tred_build_id().decode()
    if got != want:
        raise ImportError(f"{LIB_PATH} was built from other sources (build id {got[:16]}, "
                          f"tree {want[:16]}): rebuild it with paper_2602_12052_amd.build.build()")
    L.tred_status_string.argtypes = [C.c_int]
    L.tred_status_string.restype = C.c_char_p
    L.tred_last_error.restype = C.c_char_p
    L.tred_abi_version.restype = C.c_int
    L.tred_effq_windows.argtypes = [P, P, I64, P, P, P, P]
    L.tred_effq.argtypes = [P, P, I64, P, P, P, P, I64, P, P]
    L.tred_block_count.argtypes = [P, P]
    L.tred_block_count.restype = I32
    L.tred_block_bin_workspace.argtypes = [P, P]
    L.tred_block_bin_workspace.restype = I64
    L.tred_block_bin.argtypes = [P, P, I64, P, P, P, I64, P, P, P, I32, P, P]
    L.tred_conv_plan_create.argtypes = [P, P, P, I32, P, U32, I32, C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_int64)]
    L.tred_conv_plan_set_response.argtypes = [P, P, P, P]
    L.tred_conv_plan_info.argtypes = [P, P, P, P, P]
    L.tred_conv_plan_set_timing.argtypes = [P, P]
    L.tred_block_conv.argtypes = [P, P, I32, P, P, P]
    L.tred_scatter_workspace.argtypes = [P]
    L.tred_scatter_workspace.restype = I64
    L.tred_scatter_waveforms.argtypes = [P, P, P, I32, P, P, P, P, I32, P, P]
    L.tred_conv_plan_destroy.argtypes = [P]
    L.tred_conv_plan_destroy.restype = None
    L.tred_direct_plan_create.argtypes = [P, P, P, I32, U32, I32, C.POINTER(C.c_void_p),
                                          C.POINTER(C.c_int64)]
    L.tred_direct_plan_set_response.argtypes = [P, P, P, P]
    L.tred_block_conv_direct.argtypes = [P, P, I32, P, P, P]
    L.tred_direct_plan_destroy.argtypes = [P]
    L.tred_direct_plan_destroy.restype = None
    L.tred_block_bin_events_workspace.argtypes = [P, P, I32]
    L.tred_block_bin_events_workspace.restype = I64
    L.tred_block_bin_events.argtypes = [P, P, I32, P, I64, P, P, P, I64, P, P, P, I32, P, P]
    L.tred_scatter_events_workspace.argtypes = [P, I32]
    L.tred_scatter_events_workspace.restype = I64
    L.tred_scatter_waveforms_events.argtypes = [P, I32, P, P, I32, P, P, P, P, I32, P, P]
    L.tred_scatter_waveforms_adjoint.argtypes = [P, P, P, I32, P, P, I32, P, P, P]
    L.tred_block_conv_adjoint.argtypes = [P, P, I32, P, P, P]
    L.tred_block_bin_adjoint.argtypes = [P, P, I64, P, P, I64, P, P, P, I32, P, P, P]
    L.tred_effq_adjoint.argtypes = [P, P, I64, P, P, P, P, I64, P, P, P]
    L.tred_block_row_words.argtypes = [P, P]
    L.tred_block_row_words.restype = I32
    L.tred_block_bin_rows.argtypes = [P, P, I64, P, P, P, I64, P, P, P, P, I32, P, P]
    L.tred_block_conv_rows.argtypes = [P, P, I32, P, P, P, P]
    L.tred_block_bin_events_rows.argtypes = [P, P, I32, P, I64, P, P, P, I64, P, P, P, P, I32,
                                             P, P]
    L.tred_effq_bin.argtypes = [P, P, P, I64, P, P, P, P, P, P, I32, P, P, P]
    L.tred_effq_bin_events.argtypes = [P, P, P, I32, P, I64, P, P, P, P, P, P, I32, P, P, P]
    L.tred_block_conv_adjoint_rows.argtypes = [P, P, I32, P, P, P, P]
    L.tred_block_bin_rows_noalloc.argtypes = [P, P, I64, P, P, P, I64, P, P, P, P, I32, P]
    for name in ("tred_effq_windows", "tred_effq", "tred_block_bin", "tred_conv_plan_create",
                 "tred_conv_plan_set_response", "tred_conv_plan_info", "tred_conv_plan_set_timing",
    "tred_block_conv",
                 "tred_scatter_waveforms", "tred_direct_plan_create",
                 "tred_direct_plan_set_response", "tred_block_conv_direct",
                 "tred_block_bin_events", "tred_scatter_waveforms_events",
                 "tred_scatter_waveforms_adjoint", "tred_block_conv_adjoint",
                 "tred_block_bin_adjoint", "tred_effq_adjoint", "tred_block_bin_rows",
                 "tred_block_conv_rows", "tred_block_bin_events_rows",
                 "tred_block_conv_adjoint_rows", "tred_block_bin_rows_noalloc"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status: int):
    if status != TRED_OK:
        raise TredError(status, lib().tred_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _dt(t, dtype, name):
    if t is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


# ---------------------------------------------------------------------------
# C-ABI wrappers (same names, torch tensors in place of pointers)
# ---------------------------------------------------------------------------


def tred_effq_windows(grid, phys, seg, fp, off, stream=None):
    import torch
    _dt(seg, torch.float32, "seg"), _dt(fp, torch.int32, "fp"), _dt(off, torch.int64, "off")
    g, p = grid_struct(grid), physics_struct(phys)
    n = seg.shape[0] if seg is not None else 0
    _check(lib().tred_effq_windows(C.byref(g), C.byref(p), n, _ptr(seg), _ptr(fp), _ptr(off),
                                   _stream(stream)))


def tred_effq(grid, phys, seg, fp, off, val, charge_sum=None, stream=None):
    import torch
    _dt(val, torch.float32, "val"), _dt(charge_sum, torch.float64, "charge_sum")
    g, p = grid_struct(grid), physics_struct(phys)
    n = seg.shape[0]
    _check(lib().tred_effq(C.byref(g), C.byref(p), n, _ptr(seg), _ptr(fp), _ptr(off), _ptr(val),
                           val.numel(), _ptr(charge_sum), _stream(stream)))


def tred_block_count(grid, blocking) -> int:
    g, b = grid_struct(grid), blocking_struct(blocking)
    return int(lib().tred_block_count(C.byref(g), C.byref(b)))


def tred_block_bin_workspace(grid, blocking) -> int:
    g, b = grid_struct(grid), blocking_struct(blocking)
    return int(lib().tred_block_bin_workspace(C.byref(g), C.byref(b)))


def tred_block_bin(grid, blocking, fp, off, val, keys, n_active, blocks, work, stream=None):
    """keys/blocks may be None to only count the active bins (cap = 0)."""
    import torch
    _dt(keys, torch.int32, "keys"), _dt(n_active, torch.int32, "n_active")
    _dt(blocks, torch.float32, "blocks")
    g, b = grid_struct(grid), blocking_struct(blocking)
    n = fp.shape[0]
    cap = 0 if keys is None else keys.shape[0]
    if blocks is not None and blocks.shape[0] < cap:
        raise ValueError("blocks has fewer rows than keys")
    _check(lib().tred_block_bin(C.byref(g), C.byref(b), n, _ptr(fp), _ptr(off), _ptr(val),
                                val.numel(), _ptr(keys), _ptr(n_active), _ptr(blocks), cap,
                                _ptr(work), _stream(stream)))


def tred_block_bin_events_workspace(grid, blocking, n_ev) -> int:
    g, b = grid_struct(grid), blocking_struct(blocking)
    return int(lib().tred_block_bin_events_workspace(C.byref(g), C.byref(b), int(n_ev)))


def tred_block_bin_events(grid, blocking, ev_off, fp, off, val, keys, n_active, blocks, work,
                          stream=None):
    """ev_off: int64 device tensor [n_ev + 1]; keys [cap][4] (event, bx, by, bt)."""
    import torch
    _dt(ev_off, torch.int64, "ev_off"), _dt(keys, torch.int32, "keys")
    _dt(n_active, torch.int32, "n_active"), _dt(blocks, torch.float32, "blocks")
    g, b = grid_struct(grid), blocking_struct(blocking)
    n = fp.shape[0]
    cap = 0 if keys is None else keys.shape[0]
    if keys is not None and keys.shape[1] != 4:
        raise ValueError("keys must be [cap][4]")
    if blocks is not None and blocks.shape[0] < cap:
        raise ValueError("blocks has fewer rows than keys")
    _check(lib().tred_block_bin_events(C.byref(g), C.byref(b), ev_off.numel() - 1, _ptr(ev_off), n,
                                       _ptr(fp), _ptr(off), _ptr(val), val.numel(), _ptr(keys),
                                       _ptr(n_active), _ptr(blocks), cap, _ptr(work),
                                       _stream(stream)))


class ConvPlan:
    """Owner of a tred_conv_plan and its device workspace."""

    def __init__(self, grid, blocking, kpix, kticks, fft=None, mpcp=True, batch=64):
        import torch
        self.grid, self.blocking = grid_struct(grid), blocking_struct(blocking)
        kp = (C.c_int32 * 2)(*kpix)
        ff = (C.c_int32 * 3)(*(fft or (0, 0, 0)))
        h = C.c_void_p()
        ws = C.c_int64()
        _check(lib().tred_conv_plan_create(C.byref(self.grid), C.byref(self.blocking), kp,
                                           int(kticks), ff, TRED_CONV_MPCP if mpcp else 0,
                                           int(batch), C.byref(h), C.byref(ws)))
        self.handle = h
        self.kpix, self.kticks, self.mpcp = tuple(kpix), int(kticks), bool(mpcp)
        self.workspace = torch.empty(int(ws.value) + 256, dtype=torch.uint8, device="cuda")
        info = self.info()
        self.fft, self.pieces, self.channels, self.out_shape = info

    def info(self):
        f = (C.c_int32 * 3)()
        o = (C.c_int32 * 3)()
        pcs = C.c_int32()
        ch = C.c_int32()
        _check(lib().tred_conv_plan_info(self.handle, f, C.byref(pcs), C.byref(ch), o))
        return tuple(f), int(pcs.value), int(ch.value), tuple(o)

    def _ws_ptr(self):
        p = self.workspace.data_ptr()
        return (p + 255) // 256 * 256

    def set_response(self, resp, stream=None):
        import torch
        _dt(resp, torch.float32, "resp")
        _check(lib().tred_conv_plan_set_response(self.handle, _ptr(resp), self._ws_ptr(),
                                                 _stream(stream)))

    def set_timing(self, events):
        """events: six hipEvent_t handles (ints) or None."""
        if events is None:
            _check(lib().tred_conv_plan_set_timing(self.handle, None))
        else:
            arr = (C.c_void_p * 6)(*events)
            _check(lib().tred_conv_plan_set_timing(self.handle, arr))

    def __del__(self):
        try:
            if getattr(self, "handle", None) and self.handle.value:
                lib().tred_conv_plan_destroy(self.handle)
                self.handle = C.c_void_p()
        except Exception:
            pass


def tred_block_conv(plan: ConvPlan, n_active, blocks, out_blocks, stream=None):
    import torch
    _dt(out_blocks, torch.float32, "out_blocks")
    cap = blocks.shape[0]
    if out_blocks.shape[0] < cap:
        raise ValueError("out_blocks has fewer rows than blocks")
    _check(lib().tred_block_conv(plan.handle, _ptr(n_active), cap, _ptr(blocks), _ptr(out_blocks),
                                 _stream(stream)))


def tred_block_row_words(grid, blocking) -> int:
    g, b = grid_struct(grid), blocking_struct(blocking)
    return int(lib().tred_block_row_words(C.byref(g), C.byref(b)))


def tred_block_bin_rows(grid, blocking, fp, off, val, keys, n_active, blocks, rows, work,
                        stream=None):
    """As tred_block_bin, writing only the rows marked in `rows` [cap][row words] (int32
    tensor viewed as 32-bit masks)."""
    import torch
    _dt(keys, torch.int32, "keys"), _dt(n_active, torch.int32, "n_active")
    _dt(blocks, torch.float32, "blocks"), _dt(rows, torch.int32, "rows")
    g, b = grid_struct(grid), blocking_struct(blocking)
    n = fp.shape[0]
    cap = keys.shape[0]
    if blocks.shape[0] < cap or rows.shape[0] < cap:
        raise ValueError("blocks/rows have fewer rows than keys")
    if rows.shape[1] != tred_block_row_words(grid, blocking):
        raise ValueError("rows must have tred_block_row_words() columns")
    _check(lib().tred_block_bin_rows(C.byref(g), C.byref(b), n, _ptr(fp), _ptr(off), _ptr(val),
                                     val.numel(), _ptr(keys), _ptr(n_active), _ptr(blocks),
                                     _ptr(rows), cap, _ptr(work), _stream(stream)))


def _bin_out_check(grid, blocking, keys, n_active, blocks, rows, kst):
    import torch
    _dt(keys, torch.int32, "keys"), _dt(n_active, torch.int32, "n_active")
    _dt(blocks, torch.float32, "blocks"), _dt(rows, torch.int32, "rows")
    cap = 0 if keys is None else keys.shape[0]
    if cap and keys.shape[1] != kst:
        raise ValueError(f"keys must be [cap][{kst}]")
    if cap and (blocks is None or blocks.shape[0] < cap):
        raise ValueError("blocks has fewer rows than keys")
    if rows is not None:
        if rows.shape[0] < cap:
            raise ValueError("rows has fewer rows than keys")
        if rows.shape[1] != tred_block_row_words(grid, blocking):
            raise ValueError("rows must have tred_block_row_words() columns")
    return cap


def tred_effq_bin(grid, phys, blocking, seg, fp, keys, n_active, blocks, rows, work,
                  charge_sum=None, stream=None):
    """Effective charge added straight into the bins: the outputs of tred_effq followed
    by tred_block_bin_rows (rows given) or tred_block_bin (rows None), without patches."""
    import torch
    cap = _bin_out_check(grid, blocking, keys, n_active, blocks, rows, 3)
    _dt(charge_sum, torch.float64, "charge_sum")
    g, p, b = grid_struct(grid), physics_struct(phys), blocking_struct(blocking)
    _check(lib().tred_effq_bin(C.byref(g), C.byref(p), C.byref(b), seg.shape[0], _ptr(seg),
                               _ptr(fp), _ptr(keys), _ptr(n_active), _ptr(blocks), _ptr(rows),
                               cap, _ptr(charge_sum), _ptr(work), _stream(stream)))


def tred_effq_bin_events(grid, phys, blocking, ev_off, seg, fp, keys, n_active, blocks, rows,
                         work, charge_sum=None, stream=None):
    """tred_effq_bin over a batch of events (keys [cap][4])."""
    import torch
    _dt(ev_off, torch.int64, "ev_off")
    cap = _bin_out_check(grid, blocking, keys, n_active, blocks, rows, 4)
    _dt(charge_sum, torch.float64, "charge_sum")
    g, p, b = grid_struct(grid), physics_struct(phys), blocking_struct(blocking)
    _check(lib().tred_effq_bin_events(C.byref(g), C.byref(p), C.byref(b), ev_off.numel() - 1,
                                      _ptr(ev_off), seg.shape[0], _ptr(seg), _ptr(fp), _ptr(keys),
                                      _ptr(n_active), _ptr(blocks), _ptr(rows), cap,
                                      _ptr(charge_sum), _ptr(work), _stream(stream)))


def tred_block_bin_rows_noalloc(grid, blocking, fp, off, val, keys, n_active, blocks, rows,
                                stream=None):
    """tred_block_bin_rows without a workspace (the library's static per-device scratch;
    calls that overlap on one device race)."""
    import torch
    _dt(keys, torch.int32, "keys"), _dt(n_active, torch.int32, "n_active")
    _dt(blocks, torch.float32, "blocks"), _dt(rows, torch.int32, "rows")
    g, b = grid_struct(grid), blocking_struct(blocking)
    n = fp.shape[0]
    cap = keys.shape[0]
    if blocks.shape[0] < cap or rows.shape[0] < cap:
        raise ValueError("blocks/rows have fewer rows than keys")
    if rows.shape[1] != tred_block_row_words(grid, blocking):
        raise ValueError("rows must have tred_block_row_words() columns")
    _check(lib().tred_block_bin_rows_noalloc(C.byref(g), C.byref(b), n, _ptr(fp), _ptr(off),
                                             _ptr(val), val.numel(), _ptr(keys), _ptr(n_active),
                                             _ptr(blocks), _ptr(rows), cap, _stream(stream)))


def tred_block_conv_rows(plan: ConvPlan, n_active, blocks, rows, out_blocks, stream=None):
    import torch
    _dt(out_blocks, torch.float32, "out_blocks"), _dt(rows, torch.int32, "rows")
    cap = blocks.shape[0]
    if out_blocks.shape[0] < cap or rows.shape[0] < cap:
        raise ValueError("out_blocks/rows have fewer rows than blocks")
    _check(lib().tred_block_conv_rows(plan.handle, _ptr(n_active), cap, _ptr(blocks), _ptr(rows),
                                      _ptr(out_blocks), _stream(stream)))


class DirectPlan:
    """Owner of a tred_direct_plan (block-direct convolution on BF16 matrix cores)
    and its device workspace."""

    def __init__(self, grid, blocking, kpix, kticks, split=True, batch=64):
        import torch
        self.grid, self.blocking = grid_struct(grid), blocking_struct(blocking)
        kp = (C.c_int32 * 2)(*kpix)
        h = C.c_void_p()
        ws = C.c_int64()
        _check(lib().tred_direct_plan_create(C.byref(self.grid), C.byref(self.blocking), kp,
                                             int(kticks), TRED_DIRECT_SPLIT if split else 0,
                                             int(batch), C.byref(h), C.byref(ws)))
        self.handle = h
        self.kpix, self.kticks, self.split = tuple(kpix), int(kticks), bool(split)
        self.workspace = torch.empty(int(ws.value) + 256, dtype=torch.uint8, device="cuda")

    def _ws_ptr(self):
        p = self.workspace.data_ptr()
        return (p + 255) // 256 * 256

    def set_response(self, resp, stream=None):
        import torch
        _dt(resp, torch.float32, "resp")
        _check(lib().tred_direct_plan_set_response(self.handle, _ptr(resp), self._ws_ptr(),
                                                   _stream(stream)))

    def __del__(self):
        try:
            if getattr(self, "handle", None) and self.handle.value:
                lib().tred_direct_plan_destroy(self.handle)
                self.handle = C.c_void_p()
        except Exception:
            pass


def tred_block_conv_direct(plan: DirectPlan, n_active, blocks, out_blocks, cap=None, stream=None):
    """cap: bins to convolve (default: all rows of blocks)."""
    import torch
    _dt(out_blocks, torch.float32, "out_blocks")
    cap = blocks.shape[0] if cap is None else int(cap)
    if out_blocks.shape[0] < cap or blocks.shape[0] < cap:
        raise ValueError("blocks/out_blocks have fewer rows than cap")
    _check(lib().tred_block_conv_direct(plan.handle, _ptr(n_active), cap, _ptr(blocks),
                                        _ptr(out_blocks), _stream(stream)))


def tred_scatter_events_workspace(plan: ConvPlan, n_ev) -> int:
    return int(lib().tred_scatter_events_workspace(plan.handle, int(n_ev)))


def tred_scatter_waveforms_events(plan: ConvPlan, n_ev, keys, n_active, out_blocks, pix, n_pix,
                                  wf, work, stream=None):
    import torch
    _dt(pix, torch.int32, "pix"), _dt(n_pix, torch.int32, "n_pix"), _dt(wf, torch.float32, "wf")
    cap = keys.shape[0]
    _check(lib().tred_scatter_waveforms_events(plan.handle, int(n_ev), _ptr(keys), _ptr(n_active),
                                               cap, _ptr(out_blocks), _ptr(pix), _ptr(n_pix),
                                               _ptr(wf), pix.shape[0], _ptr(work), _stream(stream)))


def tred_scatter_workspace(plan: ConvPlan) -> int:
    return int(lib().tred_scatter_workspace(plan.handle))


def tred_scatter_waveforms(plan: ConvPlan, keys, n_active, out_blocks, pix, n_pix, wf, work,
                           stream=None):
    import torch
    _dt(pix, torch.int32, "pix"), _dt(n_pix, torch.int32, "n_pix"), _dt(wf, torch.float32, "wf")
    cap = keys.shape[0]
    _check(lib().tred_scatter_waveforms(plan.handle, _ptr(keys), _ptr(n_active), cap,
                                        _ptr(out_blocks), _ptr(pix), _ptr(n_pix), _ptr(wf),
                                        pix.shape[0], _ptr(work), _stream(stream)))


# ---------------------------------------------------------------------------
# Gradients: transposes of the four calls (same names with _adjoint)
# ---------------------------------------------------------------------------


def tred_scatter_waveforms_adjoint(plan: ConvPlan, keys, n_active, pix, n_pix, d_wf, d_out_blocks,
                                   stream=None):
    import torch
    _dt(d_wf, torch.float32, "d_wf"), _dt(d_out_blocks, torch.float32, "d_out_blocks")
    cap = keys.shape[0]
    _check(lib().tred_scatter_waveforms_adjoint(plan.handle, _ptr(keys), _ptr(n_active), cap,
                                                _ptr(pix), _ptr(n_pix), pix.shape[0], _ptr(d_wf),
                                                _ptr(d_out_blocks), _stream(stream)))


def tred_block_conv_adjoint(plan: ConvPlan, n_active, d_out_blocks, d_blocks, stream=None):
    import torch
    _dt(d_out_blocks, torch.float32, "d_out_blocks"), _dt(d_blocks, torch.float32, "d_blocks")
    cap = d_blocks.shape[0]
    if d_out_blocks.shape[0] < cap:
        raise ValueError("d_out_blocks has fewer rows than d_blocks")
    _check(lib().tred_block_conv_adjoint(plan.handle, _ptr(n_active), cap, _ptr(d_out_blocks),
                                         _ptr(d_blocks), _stream(stream)))


def tred_block_conv_adjoint_rows(plan: ConvPlan, n_active, d_out_blocks, rows, d_blocks,
                                 stream=None):
    """tred_block_conv_adjoint writing only the rows of d_blocks marked in `rows`."""
    import torch
    _dt(d_out_blocks, torch.float32, "d_out_blocks"), _dt(d_blocks, torch.float32, "d_blocks")
    _dt(rows, torch.int32, "rows")
    cap = d_blocks.shape[0]
    if d_out_blocks.shape[0] < cap or rows.shape[0] < cap:
        raise ValueError("d_out_blocks/rows have fewer rows than d_blocks")
    _check(lib().tred_block_conv_adjoint_rows(plan.handle, _ptr(n_active), cap, _ptr(d_out_blocks),
                                              _ptr(rows), _ptr(d_blocks), _stream(stream)))


def tred_block_bin_adjoint(grid, blocking, fp, off, keys, n_active, d_blocks, d_val, work,
                           stream=None):
    import torch
    _dt(d_blocks, torch.float32, "d_blocks"), _dt(d_val, torch.float32, "d_val")
    g, b = grid_struct(grid), blocking_struct(blocking)
    cap = keys.shape[0]
    _check(lib().tred_block_bin_adjoint(C.byref(g), C.byref(b), fp.shape[0], _ptr(fp), _ptr(off),
                                        d_val.numel(), _ptr(keys), _ptr(n_active), _ptr(d_blocks),
                                        cap, _ptr(d_val), _ptr(work), _stream(stream)))


def tred_effq_adjoint(grid, phys, seg, fp, off, d_val, d_seg, d_phys=None, stream=None):
    """d_seg [n][7] out; d_phys (float64 [3], accumulated) gets dL/d(diff_T, diff_L,
    lifetime)."""
    import torch
    _dt(d_val, torch.float32, "d_val"), _dt(d_seg, torch.float32, "d_seg")
    _dt(d_phys, torch.float64, "d_phys")
    g, p = grid_struct(grid), physics_struct(phys)
    _check(lib().tred_effq_adjoint(C.byref(g), C.byref(p), seg.shape[0], _ptr(seg), _ptr(fp),
                                   _ptr(off), _ptr(d_val), d_val.numel(), _ptr(d_seg),
                                   _ptr(d_phys), _stream(stream)))


# ---------------------------------------------------------------------------
# Whole path
# ---------------------------------------------------------------------------


class Pipeline:
    """Buffers and plan for one event shape; run() enqueues the five calls with no
    host synchronisation (capacities fixed at construction)."""

    def __init__(self, grid, phys, blocking, kpix, kticks, resp, n_dep, val_cap, block_cap,
                 pix_cap, fft=None, mpcp=True, batch=64, row_masks=True, fused=False):
        """row_masks: bin with row masks (only the rows a footprint reaches are written
        and transformed); False leaves every row of `blocks` defined (dense blocks).
        fused: the effective charge goes straight into the bins (tred_effq_bin): no
        patches are kept (results() has no "val"; val_cap only sizes the gradient's
        patch buffer)."""
        import torch
        dev = "cuda"
        self.grid, self.phys, self.blocking = grid_struct(grid), physics_struct(phys), \
            blocking_struct(blocking)
        self.n_dep = int(n_dep)
        self.fused = bool(fused)
        self.val_cap = int(val_cap)
        self.plan = ConvPlan(grid, blocking, kpix, kticks, fft, mpcp, batch)
        self.plan.set_response(resp)
        self.fp = torch.empty((self.n_dep, 6), dtype=torch.int32, device=dev)
        self.off = torch.empty(self.n_dep + 1, dtype=torch.int64, device=dev)
        self.val = None if self.fused else torch.empty(self.val_cap, dtype=torch.float32,
                                                       device=dev)
        self.charge_sum = torch.zeros(1, dtype=torch.float64, device=dev)
        self.keys = torch.empty((int(block_cap), 3), dtype=torch.int32, device=dev)
        self.n_active = torch.zeros(1, dtype=torch.int32, device=dev)
        g, b = self.grid, self.blocking
        vblk = b.blk_pix[0] * g.sub[0] * b.blk_pix[1] * g.sub[1] * b.blk_ticks
        self.blocks = torch.empty((int(block_cap), vblk), dtype=torch.float32, device=dev)
        self.rows = torch.empty((int(block_cap), tred_block_row_words(g, b)), dtype=torch.int32,
                                device=dev) if row_masks else None
        o = self.plan.out_shape
        self.out_blocks = torch.empty((int(block_cap), o[0] * o[1] * o[2]), dtype=torch.float32,
                                      device=dev)
        self.bin_work = torch.empty(max(4, tred_block_bin_workspace(g, b)), dtype=torch.uint8,
                                    device=dev)
        self.pix = torch.empty(int(pix_cap), dtype=torch.int32, device=dev)
        self.n_pix = torch.zeros(1, dtype=torch.int32, device=dev)
        self.lwf = g.nticks + int(kticks) - 1
        self.wf = torch.empty((int(pix_cap), self.lwf), dtype=torch.float32, device=dev)
        self.scat_work = torch.empty(max(4, tred_scatter_workspace(self.plan)), dtype=torch.uint8,
                                     device=dev)

    def run(self, seg, stream=None, stop_after: Optional[str] = None):
        tred_effq_windows(self.grid, self.phys, seg, self.fp, self.off, stream)
        self.charge_sum.zero_()
        if self.fused:
            if stop_after == "effq":
                raise ValueError("a fused pipeline has no separate effective-charge stage")
            tred_effq_bin(self.grid, self.phys, self.blocking, seg, self.fp, self.keys,
                          self.n_active, self.blocks, self.rows, self.bin_work, self.charge_sum,
                          stream)
        else:
            tred_effq(self.grid, self.phys, seg, self.fp, self.off, self.val, self.charge_sum,
                      stream)
            if stop_after == "effq":
                return
            self.bin(stream)
        if stop_after == "bin":
            return
        self.conv(stream)
        tred_scatter_waveforms(self.plan, self.keys, self.n_active, self.out_blocks, self.pix,
                               self.n_pix, self.wf, self.scat_work, stream)

    def bin(self, stream=None):
        if self.rows is not None:
            tred_block_bin_rows(self.grid, self.blocking, self.fp, self.off, self.val, self.keys,
                                self.n_active, self.blocks, self.rows, self.bin_work, stream)
        else:
            tred_block_bin(self.grid, self.blocking, self.fp, self.off, self.val, self.keys,
                           self.n_active, self.blocks, self.bin_work, stream)

    def conv(self, stream=None):
        if self.rows is not None:
            tred_block_conv_rows(self.plan, self.n_active, self.blocks, self.rows, self.out_blocks,
                                 stream)
        else:
            tred_block_conv(self.plan, self.n_active, self.blocks, self.out_blocks, stream)

    def backward(self, seg, d_wf, stream=None):
        """Gradients of a loss L with respect to the depositions and the transport
        parameters, given dL/dwf for the waveforms of the last run(seg): returns
        (d_seg [n][7] float32, d_phys float64 [3] = dL/d(diff_T, diff_L, lifetime)).
        The chain runs the four adjoint calls on the integer structures of run()
        (footprints, keys, pixel list); the effective charge is recomputed."""
        import torch
        if self.fused:
            # the forward pass kept no patches, so only here does the patch length meet
            # the buffer it sizes (the patch gradient): refuse a truncated gradient
            nval = int(self.off[self.n_dep].item())
            if nval > self.val_cap:
                raise TredError(TRED_ECAPACITY, f"backward: patch cells {nval} > val capacity "
                                                f"{self.val_cap}")
        if not hasattr(self, "d_out_blocks"):
            self.d_out_blocks = torch.empty_like(self.out_blocks)
            self.d_blocks = torch.empty_like(self.blocks)
            self.d_val = torch.empty(self.val_cap, dtype=torch.float32, device="cuda")
            self.d_seg = torch.empty((self.n_dep, 7), dtype=torch.float32, device="cuda")
            self.d_phys = torch.zeros(3, dtype=torch.float64, device="cuda")
        tred_scatter_waveforms_adjoint(self.plan, self.keys, self.n_active, self.pix, self.n_pix,
                                       d_wf, self.d_out_blocks, stream)
        if self.rows is not None:
            tred_block_conv_adjoint_rows(self.plan, self.n_active, self.d_out_blocks, self.rows,
                                         self.d_blocks, stream)
        else:
            tred_block_conv_adjoint(self.plan, self.n_active, self.d_out_blocks, self.d_blocks,
                                    stream)
        tred_block_bin_adjoint(self.grid, self.blocking, self.fp, self.off, self.keys,
                               self.n_active, self.d_blocks, self.d_val, self.bin_work, stream)
        self.d_phys.zero_()
        tred_effq_adjoint(self.grid, self.phys, seg, self.fp, self.off, self.d_val, self.d_seg,
                          self.d_phys, stream)
        return self.d_seg, self.d_phys

    def check_capacity(self, n_dep=None):
        """Raise TredError(TRED_ECAPACITY) if the last run overflowed a capacity (the
        patch length off[n], the active-bin count or the pixel count exceeds the
        buffer it was given, so part of the event was dropped). Synchronises."""
        n = self.n_dep if n_dep is None else int(n_dep)
        # (fused: no patches are stored, so the patch length bounds nothing)
        nval = 0 if self.fused else int(self.off[n].item())
        _check_counts(nval, self.val_cap, int(self.n_active.item()), self.keys.shape[0],
                      int(self.n_pix.item()), self.pix.shape[0])

    def results(self, check=True):
        """Host copies of the outputs (synchronises); raises TredError if the run
        overflowed a capacity, unless `check` is False (then the truncated outputs
        are returned: the first capacity-many bins and pixels in key order)."""
        import torch
        torch.cuda.synchronize()
        if check:
            self.check_capacity()
        na = int(self.n_active.item())
        npx = int(self.n_pix.item())
        nval = int(self.off[-1].item())
        return dict(fp=self.fp.cpu().numpy(), off=self.off.cpu().numpy(),
                    val=None if self.fused else self.val[:min(nval, self.val_cap)].cpu().numpy(),
                    charge_sum=float(self.charge_sum.item()), n_active=na,
                    keys=self.keys[:min(na, self.keys.shape[0])].cpu().numpy(), n_pix=npx,
                    pix=self.pix[:min(npx, self.pix.shape[0])].cpu().numpy(),
                    wf=self.wf[:min(npx, self.pix.shape[0])].cpu().numpy())


def _check_counts(nval, val_cap, na, block_cap, npx, pix_cap):
    over = []
    if nval > val_cap:
        over.append(f"patch cells {nval} > val capacity {val_cap}")
    if na > block_cap:
        over.append(f"active bins {na} > bin capacity {block_cap}")
    if npx > pix_cap:
        over.append(f"pixels {npx} > pixel capacity {pix_cap}")
    if over:
        raise TredError(TRED_ECAPACITY, "run truncated: " + "; ".join(over))


def tred_block_bin_events_rows(grid, blocking, ev_off, fp, off, val, keys, n_active, blocks, rows,
                               work, stream=None):
    """tred_block_bin_events with row masks `rows` [cap][row words] (int32 tensor)."""
    import torch
    _dt(ev_off, torch.int64, "ev_off"), _dt(keys, torch.int32, "keys")
    _dt(n_active, torch.int32, "n_active"), _dt(blocks, torch.float32, "blocks")
    _dt(rows, torch.int32, "rows")
    g, b = grid_struct(grid), blocking_struct(blocking)
    n = fp.shape[0]
    cap = keys.shape[0]
    if keys.shape[1] != 4:
        raise ValueError("keys must be [cap][4]")
    if blocks.shape[0] < cap or rows.shape[0] < cap:
        raise ValueError("blocks/rows have fewer rows than keys")
    if rows.shape[1] != tred_block_row_words(grid, blocking):
        raise ValueError("rows must have tred_block_row_words() columns")
    _check(lib().tred_block_bin_events_rows(C.byref(g), C.byref(b), ev_off.numel() - 1,
                                            _ptr(ev_off), n, _ptr(fp), _ptr(off), _ptr(val),
                                            val.numel(), _ptr(keys), _ptr(n_active), _ptr(blocks),
                                            _ptr(rows), cap, _ptr(work), _stream(stream)))


class BatchPipeline:
    """Buffers and plan for batches of events sharing one grid and response. A batch
    is a concatenation of depositions with device offsets ev_off (event e owns rows
    ev_off[e] .. ev_off[e+1]); its (event, bin) pairs form one binned tensor
    convolved in passes of `batch` bins, and waveforms are per (event, pixel).
    Capacities bound any batch given to run(), so one buffer set serves a stream of
    batches; run() enqueues every call with no host synchronisation (a caller may
    capture it in a HIP graph per batch shape)."""

    def __init__(self, grid, phys, blocking, kpix, kticks, resp, n_ev_max, n_dep_max, val_cap,
                 block_cap, pix_cap, fft=None, mpcp=True, batch=64, plan=None, row_masks=True,
                 fused=False):
        """fused: effective charge straight into the bins (tred_effq_bin_events), no
        patch buffer (val_cap is then ignored)."""
        import torch
        dev = "cuda"
        self.fused = bool(fused)
        self.grid, self.phys, self.blocking = grid_struct(grid), physics_struct(phys), \
            blocking_struct(blocking)
        self.n_ev_max, self.n_dep_max = int(n_ev_max), int(n_dep_max)
        if plan is None:
            plan = ConvPlan(grid, blocking, kpix, kticks, fft, mpcp, batch)
            plan.set_response(resp)
        self.plan = plan
        g, b = self.grid, self.blocking
        self.fp = torch.empty((self.n_dep_max, 6), dtype=torch.int32, device=dev)
        self.off = torch.empty(self.n_dep_max + 1, dtype=torch.int64, device=dev)
        self.val = None if self.fused else torch.empty(int(val_cap), dtype=torch.float32,
                                                       device=dev)
        self.charge_sum = torch.zeros(1, dtype=torch.float64, device=dev)
        self.keys = torch.empty((int(block_cap), 4), dtype=torch.int32, device=dev)
        self.n_active = torch.zeros(1, dtype=torch.int32, device=dev)
        vblk = b.blk_pix[0] * g.sub[0] * b.blk_pix[1] * g.sub[1] * b.blk_ticks
        self.blocks = torch.empty((int(block_cap), vblk), dtype=torch.float32, device=dev)
        self.rows = torch.empty((int(block_cap), tred_block_row_words(g, b)), dtype=torch.int32,
                                device=dev) if row_masks else None
        o = self.plan.out_shape
        self.out_blocks = torch.empty((int(block_cap), o[0] * o[1] * o[2]), dtype=torch.float32,
                                      device=dev)
        self.bin_work = torch.empty(max(4, tred_block_bin_events_workspace(g, b, self.n_ev_max)),
                                    dtype=torch.uint8, device=dev)
        self.pix = torch.empty(int(pix_cap), dtype=torch.int32, device=dev)
        self.n_pix = torch.zeros(1, dtype=torch.int32, device=dev)
        self.lwf = g.nticks + int(kticks) - 1
        self.wf = torch.empty((int(pix_cap), self.lwf), dtype=torch.float32, device=dev)
        self.scat_work = torch.empty(
            max(4, tred_scatter_events_workspace(self.plan, self.n_ev_max)), dtype=torch.uint8,
            device=dev)

    def run(self, seg, ev_off, stream=None, pix_cap=None):
        """seg: float32 [n, 7] device (n <= n_dep_max); ev_off: int64 device [n_ev + 1].
        pix_cap: pixel capacity of this batch (at most the pipeline's; default the
        pipeline's): the waveforms of this run are rows 0 .. pix_cap - 1 of wf, the rows
        past the batch's n_pix among them zero, and rows past pix_cap are not touched
        (a batch of small events then writes no zero waveforms for the largest batch's
        pixels)."""
        n, n_ev = seg.shape[0], ev_off.numel() - 1
        if n > self.n_dep_max or n_ev > self.n_ev_max:
            raise ValueError("batch exceeds the pipeline's capacities")
        pc = self._pix_cap(pix_cap)
        fp, off = self.fp[:n], self.off[:n + 1]
        tred_effq_windows(self.grid, self.phys, seg, fp, off, stream)
        self.charge_sum.zero_()
        if self.fused:
            tred_effq_bin_events(self.grid, self.phys, self.blocking, ev_off, seg, fp, self.keys,
                                 self.n_active, self.blocks, self.rows, self.bin_work,
                                 self.charge_sum, stream)
        else:
            tred_effq(self.grid, self.phys, seg, fp, off, self.val, self.charge_sum, stream)
            if self.rows is not None:
                tred_block_bin_events_rows(self.grid, self.blocking, ev_off, fp, off, self.val,
                                           self.keys, self.n_active, self.blocks, self.rows,
                                           self.bin_work, stream)
            else:
                tred_block_bin_events(self.grid, self.blocking, ev_off, fp, off, self.val,
                                      self.keys, self.n_active, self.blocks, self.bin_work,
                                      stream)
        if self.rows is not None:
            tred_block_conv_rows(self.plan, self.n_active, self.blocks, self.rows, self.out_blocks,
                                 stream)
        else:
            tred_block_conv(self.plan, self.n_active, self.blocks, self.out_blocks, stream)
        tred_scatter_waveforms_events(self.plan, n_ev, self.keys, self.n_active, self.out_blocks,
                                      self.pix[:pc], self.n_pix, self.wf[:pc], self.scat_work, stream)

    def _pix_cap(self, pix_cap):
        pc = self.pix.shape[0] if pix_cap is None else int(pix_cap)
        if pc < 1 or pc > self.pix.shape[0]:
            raise ValueError("pix_cap must be in 1 .. the pipeline's pixel capacity")
        return pc

    def results(self, n_dep=None, pix_cap=None):
        """Host copies of the outputs of the last run (synchronises); n_dep: depositions
        of that run, pix_cap: its pixel capacity (the value given to run(), which a graph
        replay does not record). Raises TredError if the run overflowed a capacity."""
        import torch
        torch.cuda.synchronize()
        n = self.n_dep_max if n_dep is None else int(n_dep)
        na = int(self.n_active.item())
        npx = int(self.n_pix.item())
        pc = self._pix_cap(pix_cap)
        if n_dep is not None and not self.fused:
            _check_counts(int(self.off[n].item()), self.val.numel(), na, self.keys.shape[0],
                          npx, pc)
        else:
            _check_counts(0, 0, na, self.keys.shape[0], npx, pc)
        return dict(fp=self.fp[:n].cpu().numpy(), off=self.off[:n + 1].cpu().numpy(),
                    n_active=na, keys=self.keys[:min(na, self.keys.shape[0])].cpu().numpy(),
                    n_pix=npx, pix=self.pix[:min(npx, pc)].cpu().numpy(),
                    wf=self.wf[:min(npx, pc)].cpu().numpy(),
                    charge_sum=float(self.charge_sum.item()))


def size_batch(grid, phys, blocking, kpix, seg, ev_off):
    """Capacities of a batch (as size_event, with the event dimension)."""
    import torch
    n = seg.shape[0]
    fp = torch.empty((n, 6), dtype=torch.int32, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    tred_effq_windows(grid, phys, seg, fp, off)
    g, b = grid_struct(grid), blocking_struct(blocking)
    eo = torch.from_numpy(np.asarray(ev_off, np.int64)).cuda()
    na = torch.zeros(1, dtype=torch.int32, device="cuda")
    work = torch.empty(max(4, tred_block_bin_events_workspace(g, b, eo.numel() - 1)),
                       dtype=torch.uint8, device="cuda")
    dummy = torch.empty(1, dtype=torch.float32, device="cuda")
    tred_block_bin_events(g, b, eo, fp, off, dummy, None, na, None, work)
    torch.cuda.synchronize()
    val_cap = int(off[-1].item())
    block_cap = int(na.item())
    per = (b.blk_pix[0] + kpix[0] - 1) * (b.blk_pix[1] + kpix[1] - 1)
    pix_cap = min((eo.numel() - 1) * int(g.npix[0]) * int(g.npix[1]), block_cap * per)
    return max(val_cap, 1), max(block_cap, 1), max(pix_cap, 1)


def plan_workspace_bytes(grid, blocking, kpix, kticks, fft=None, mpcp=True, batch=1) -> int:
    """Device workspace of a convolution plan (host query, nothing allocated)."""
    g, b = grid_struct(grid), blocking_struct(blocking)
    kp = (C.c_int32 * 2)(*kpix)
    ff = (C.c_int32 * 3)(*(fft or (0, 0, 0)))
    h = C.c_void_p()
    ws = C.c_int64()
    _check(lib().tred_conv_plan_create(C.byref(g), C.byref(b), kp, int(kticks), ff,
                                       TRED_CONV_MPCP if mpcp else 0, int(batch), C.byref(h),
                                       C.byref(ws)))
    lib().tred_conv_plan_destroy(h)
    return int(ws.value)


def conv_batch(grid, blocking, kpix, kticks, fft, mpcp, n_bins, scratch_bytes) -> int:
    """Bins per convolution pass whose scratch fits `scratch_bytes` (at most n_bins):
    the plan's per-bin scratch is its workspace growth per bin at large batches (at
    small batches the response set-up scratch, shared with the pass scratch, dominates)."""
    w1 = plan_workspace_bytes(grid, blocking, kpix, kticks, fft, mpcp, 1 << 16)
    w2 = plan_workspace_bytes(grid, blocking, kpix, kticks, fft, mpcp, 1 << 17)
    per_bin = max(1, -(-(w2 - w1) // (1 << 16)))
    return int(max(1, min(int(n_bins), int(scratch_bytes) // per_bin)))


# Scratch budget of the convolution on one MI355X (288 GB of HBM): the module-scale
# event (about 850 active bins, ~150 MB of spectra per bin) runs in one pass.
DEFAULT_CONV_SCRATCH = 160e9


def _event_pixels(fp, g, b, kpix) -> int:
    """Pixels of an event's waveforms from its cell footprints fp (host int32 [n, 6]):
    the union over its active bins (those a footprint reaches, as the binning marks
    them) of the bins' output footprints in x and y, clipped to the region."""
    f = fp[(fp[:, 3] >= fp[:, 0]) & (fp[:, 4] >= fp[:, 1]) & (fp[:, 5] >= fp[:, 2])]
    if len(f) == 0:
        return 0
    bf0, bf1 = b.blk_pix[0] * g.sub[0], b.blk_pix[1] * g.sub[1]
    bx0, bx1 = f[:, 0] // bf0, f[:, 3] // bf0
    by0, by1 = f[:, 1] // bf1, f[:, 4] // bf1
    act = np.zeros((int(bx1.max()) + 1, int(by1.max()) + 1), dtype=bool)
    for dx in range(int((bx1 - bx0).max()) + 1):
        for dy in range(int((by1 - by0).max()) + 1):
            m = (bx0 + dx <= bx1) & (by0 + dy <= by1)
            act[bx0[m] + dx, by0[m] + dy] = True
    npx, npy = int(g.npix[0]), int(g.npix[1])
    hx, hy = (int(kpix[0]) - 1) // 2, (int(kpix[1]) - 1) // 2
    Bx, By = b.blk_pix[0], b.blk_pix[1]
    pix = np.zeros((npx, npy), dtype=bool)
    for bx, by in zip(*np.nonzero(act)):
        pix[max(0, bx * Bx - hx):min(npx, bx * Bx + Bx + hx),
            max(0, by * By - hy):min(npy, by * By + By + hy)] = True
    return int(pix.sum())


def size_event(grid, phys, blocking, kpix, seg, exact_pixels=False):
    """Capacities of one event: exact patch length and active-bin count (footprint
    step plus a counting pass of the binning, then one synchronisation), and the
    host bound min(region pixels, bins x output pixels per bin) for the pixels, or
    with exact_pixels the event's pixel count itself (its footprints copied to the
    host; a pipeline sized by it has no slack for depositions that move)."""
    import torch
    n = seg.shape[0]
    fp = torch.empty((n, 6), dtype=torch.int32, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    tred_effq_windows(grid, phys, seg, fp, off)
    g, b = grid_struct(grid), blocking_struct(blocking)
    na = torch.zeros(1, dtype=torch.int32, device="cuda")
    work = torch.empty(max(4, tred_block_bin_workspace(g, b)), dtype=torch.uint8, device="cuda")
    dummy = torch.empty(1, dtype=torch.float32, device="cuda")
    tred_block_bin(g, b, fp, off, dummy, None, na, None, work)
    torch.cuda.synchronize()
    val_cap = int(off[-1].item())
    block_cap = int(na.item())
    per = (b.blk_pix[0] + kpix[0] - 1) * (b.blk_pix[1] + kpix[1] - 1)
    pix_cap = min(int(g.npix[0]) * int(g.npix[1]), block_cap * per)
    if exact_pixels:
        pix_cap = _event_pixels(fp.cpu().numpy(), g, b, kpix)
    return max(val_cap, 1), max(block_cap, 1), max(pix_cap, 1)


def simulate(seg, resp, grid, phys, blocking, kpix, kticks, fft=None, mpcp=True, batch=64):
    """One event through the whole path; returns host numpy outputs."""
    val_cap, block_cap, pix_cap = size_event(grid, phys, blocking, kpix, seg)
    pl = Pipeline(grid, phys, blocking, kpix, kticks, resp, seg.shape[0], val_cap, block_cap,
                  pix_cap, fft, mpcp, batch)
    pl.run(seg)
    return pl.results()


class Simulate:
    """torch.autograd.Function over a Pipeline: waveforms of the depositions seg
    (float32 [n][7] on the GPU, requires_grad for d/d(end points, charge)). The pixel
    list of the forward pass fixes the waveform rows (pipeline.pix[:n_pix]); rows at
    or past n_pix are zero and carry no gradient. backward returns dL/dseg and
    writes dL/d(diff_T, diff_L, lifetime) into pipeline.d_phys. The forward pass
    synchronises once to check the capacities: a run that would drop part of the
    event (depositions moved outside the sizes the pipeline was built for) raises
    TredError instead of returning truncated waveforms."""

    @staticmethod
    def apply(pipeline, seg):
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, s):
                pipeline.run(s)
                pipeline.check_capacity()
                ctx.save_for_backward(s)
                return pipeline.wf.clone()

            @staticmethod
            def backward(ctx, g):
                (s,) = ctx.saved_tensors
                d_seg, _ = pipeline.backward(s, g.contiguous())
                return d_seg.clone()

        return _F.apply(seg)

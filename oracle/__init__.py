"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference for the signal-formation hot path of
arXiv 2602.12052 (effective charge -> block-sparse binning -> interlaced
convolution with the field response -> per-pixel waveforms). Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
GPU library never does, and this package never imports the GPU library.

The arithmetic lives in ``oracle.c`` (binary64, OpenMP over depositions or
pixels); this module builds it with gcc and wraps it with ctypes. Written here in
numpy are the plain definitions of the output pixel set (:func:`pix_set`), of the
depositions reaching one bin (:func:`bin_members`) and of one bin's convolution
output at isolated samples (:func:`block_output_points`).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (binary64; no FMA contraction; OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class OGrid(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("spacing", C.c_float * 3), ("npix", C.c_int32 * 2),
                ("sub", C.c_int32 * 2), ("nticks", C.c_int32)]


class OPhysics(C.Structure):
    _fields_ = [("v_drift", C.c_float), ("lifetime", C.c_float), ("diff_T", C.c_float),
                ("diff_L", C.c_float), ("sigma_min", C.c_float * 3), ("n_sigma", C.c_float),
                ("point_frac", C.c_float), ("n_gl", C.c_int32)]


class OBlocking(C.Structure):
    _fields_ = [("blk_pix", C.c_int32 * 2), ("blk_ticks", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        L = _lib
        P = C.c_void_p
        L.oracle_gl_rule.argtypes = [C.c_int, P, P]
        L.oracle_transport.argtypes = [P, P, P]
        L.oracle_window_f32.argtypes = [P, P, P, P, P, P]
        L.oracle_footprint.argtypes = [P, P, P, P, P]
        L.oracle_footprint.restype = C.c_int64
        L.oracle_footprints.argtypes = [P, P, C.c_int64, P, P, P, P]
        L.oracle_q_line.argtypes = [C.c_double] * 3 + [P, P, P, C.c_double]
        L.oracle_q_line.restype = C.c_double
        L.oracle_q_point.argtypes = [C.c_double] * 3 + [P, P, C.c_double]
        L.oracle_q_point.restype = C.c_double
        L.oracle_q_seg.argtypes = [P, P, C.c_double, C.c_double, C.c_double]
        L.oracle_q_seg.restype = C.c_double
        L.oracle_effq_patch.argtypes = [P, P, P, P, P, P]
        L.oracle_effq.argtypes = [P, P, C.c_int64, P, P, P, P, P]
        L.oracle_cell_sums.argtypes = [P, P, P, P, P, P]
        L.oracle_block_keys.argtypes = [P, P, C.c_int64, P, P, C.c_int32]
        L.oracle_block_keys.restype = C.c_int32
        L.oracle_block_values.argtypes = [P, P, C.c_int64, P, P, P, P, P]
        L.oracle_waveforms.argtypes = [P, P, C.c_int32, P, C.c_int64, P, P, P, C.c_int64, P, P]
        L.oracle_waveform_points.argtypes = [P, P, C.c_int32, P, C.c_int64, P, P, P, C.c_int64,
                                             P, P]
        L.oracle_num_threads.restype = C.c_int
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def ogrid(g) -> OGrid:
    return OGrid((C.c_float * 3)(*g.origin), (C.c_float * 3)(*g.spacing), (C.c_int32 * 2)(*g.npix),
                 (C.c_int32 * 2)(*g.sub), int(g.nticks))


def ophysics(p) -> OPhysics:
    return OPhysics(p.v_drift, p.lifetime, p.diff_T, p.diff_L, (C.c_float * 3)(*p.sigma_min),
                    p.n_sigma, p.point_frac, int(p.n_gl))


def oblocking(b) -> OBlocking:
    return OBlocking((C.c_int32 * 2)(*b.blk_pix), int(b.blk_ticks))


def _seg(seg) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(seg, dtype=np.float32).reshape(-1, 7))


# ---------------------------------------------------------------------------


def gl_rule(n: int):
    xi = np.zeros(n)
    w = np.zeros(n)
    if lib().oracle_gl_rule(n, _p(xi), _p(w)) != 0:
        raise ValueError(n)
    return xi, w


def transport(physics, seg1) -> np.ndarray:
    """(t0, t1, t_mid, Q', sigma_x, sigma_y, sigma_t) of one segment, binary64."""
    out = np.zeros(7)
    s = _seg(seg1)
    ph = ophysics(physics)
    lib().oracle_transport(C.byref(ph), _p(s), _p(out))
    return out


def window_f32(grid, physics, seg1):
    lo = np.zeros(3, np.int32)
    hi = np.zeros(3, np.int32)
    ip = np.zeros(1, np.int32)
    s = _seg(seg1)
    g, ph = ogrid(grid), ophysics(physics)
    lib().oracle_window_f32(C.byref(g), C.byref(ph), _p(s), _p(lo), _p(hi), _p(ip))
    return lo, hi, bool(ip[0])


def footprints(grid, physics, seg):
    """fp [n,6] int32 (cropped lo[3], hi[3]), off [n+1] int64, is_point [n] int32."""
    s = _seg(seg)
    n = s.shape[0]
    fp = np.zeros((n, 6), np.int32)
    off = np.zeros(n + 1, np.int64)
    ip = np.zeros(n, np.int32)
    g, ph = ogrid(grid), ophysics(physics)
    lib().oracle_footprints(C.byref(g), C.byref(ph), n, _p(s), _p(fp), _p(off), _p(ip))
    return fp, off, ip


def q_line(x, y, z, p0, p1, sig, Q) -> float:
    p0 = np.ascontiguousarray(p0, np.float64)
    p1 = np.ascontiguousarray(p1, np.float64)
    sig = np.ascontiguousarray(sig, np.float64)
    return lib().oracle_q_line(x, y, z, _p(p0), _p(p1), _p(sig), Q)


def q_point(x, y, z, m, sig, Q) -> float:
    m = np.ascontiguousarray(m, np.float64)
    sig = np.ascontiguousarray(sig, np.float64)
    return lib().oracle_q_point(x, y, z, _p(m), _p(sig), Q)


def q_seg(physics, seg1, x, y, t) -> float:
    s = _seg(seg1)
    ph = ophysics(physics)
    return lib().oracle_q_seg(C.byref(ph), _p(s), x, y, t)


def effq(grid, physics, seg, fp, off):
    """Patch values (binary64) of every deposition and per-deposition node sums."""
    s = _seg(seg)
    n = s.shape[0]
    fp = np.ascontiguousarray(fp, np.int32)
    off = np.ascontiguousarray(off, np.int64)
    val = np.zeros(int(off[-1]), np.float64)
    ns = np.zeros(n, np.float64)
    g, ph = ogrid(grid), ophysics(physics)
    lib().oracle_effq(C.byref(g), C.byref(ph), n, _p(s), _p(fp), _p(off), _p(val), _p(ns))
    return val, ns


def effq_patch(grid, physics, seg1, fp1):
    s = _seg(seg1)
    fp1 = np.ascontiguousarray(fp1, np.int32).reshape(6)
    shape = tuple(int(max(0, fp1[3 + a] - fp1[a] + 1)) for a in range(3))
    val = np.zeros(int(np.prod(shape)), np.float64)
    ns = np.zeros(1)
    g, ph = ogrid(grid), ophysics(physics)
    lib().oracle_effq_patch(C.byref(g), C.byref(ph), _p(s), _p(fp1), _p(val), _p(ns))
    return val.reshape(shape), float(ns[0])


def cell_sums(grid, physics, seg1, c0, c1) -> np.ndarray:
    s = _seg(seg1)
    c0 = np.ascontiguousarray(c0, np.int32)
    c1 = np.ascontiguousarray(c1, np.int32)
    shape = tuple(int(c1[a] - c0[a] + 1) for a in range(3))
    out = np.zeros(int(np.prod(shape)))
    g, ph = ogrid(grid), ophysics(physics)
    lib().oracle_cell_sums(C.byref(g), C.byref(ph), _p(s), _p(c0), _p(c1), _p(out))
    return out.reshape(shape)


def block_keys(grid, blocking, fp) -> np.ndarray:
    fp = np.ascontiguousarray(fp, np.int32).reshape(-1, 6)
    g, b = ogrid(grid), oblocking(blocking)
    nb = [(grid.npix[0] * grid.sub[0] + blocking.blk_pix[0] * grid.sub[0] - 1) //
          (blocking.blk_pix[0] * grid.sub[0]),
          (grid.npix[1] * grid.sub[1] + blocking.blk_pix[1] * grid.sub[1] - 1) //
          (blocking.blk_pix[1] * grid.sub[1]),
          (grid.nticks + blocking.blk_ticks - 1) // blocking.blk_ticks]
    cap = int(np.prod(nb))
    keys = np.zeros((cap, 3), np.int32)
    na = lib().oracle_block_keys(C.byref(g), C.byref(b), fp.shape[0], _p(fp), _p(keys), cap)
    return keys[:na].copy()


def block_values(grid, blocking, fp, off, val, key) -> np.ndarray:
    fp = np.ascontiguousarray(fp, np.int32).reshape(-1, 6)
    off = np.ascontiguousarray(off, np.int64)
    val = np.ascontiguousarray(val, np.float64)
    key = np.ascontiguousarray(key, np.int32)
    shape = (blocking.blk_pix[0] * grid.sub[0], blocking.blk_pix[1] * grid.sub[1],
             blocking.blk_ticks)
    out = np.zeros(shape)
    g, b = ogrid(grid), oblocking(blocking)
    lib().oracle_block_values(C.byref(g), C.byref(b), fp.shape[0], _p(fp), _p(off), _p(val),
                              _p(key), _p(out))
    return out


def pix_set(grid, blocking, kpix, keys) -> np.ndarray:
    """Output pixels (Sec. III-B: overlap reduction on unique electrodes): the union,
    cropped to the region, of every kept bin's convolution output footprint
    [b*B - (K-1)/2, b*B + B - 1 + (K-1)/2] per pixel axis. Ascending px*npix_y + py."""
    keys = np.asarray(keys, np.int32).reshape(-1, 3)
    mark = np.zeros((grid.npix[0], grid.npix[1]), bool)
    hx, hy = (kpix[0] - 1) // 2, (kpix[1] - 1) // 2
    Bx, By = blocking.blk_pix
    for bx, by, _ in keys:
        x0, x1 = max(0, bx * Bx - hx), min(grid.npix[0] - 1, bx * Bx + Bx - 1 + hx)
        y0, y1 = max(0, by * By - hy), min(grid.npix[1] - 1, by * By + By - 1 + hy)
        mark[x0:x1 + 1, y0:y1 + 1] = True
    px, py = np.nonzero(mark)
    return (px * grid.npix[1] + py).astype(np.int32)


def waveforms(grid, kpix, kticks, resp, fp, off, val, pix) -> np.ndarray:
    """Induced-current waveforms [n_pix, nticks + Kt - 1] (binary64) by direct summation."""
    fp = np.ascontiguousarray(fp, np.int32).reshape(-1, 6)
    off = np.ascontiguousarray(off, np.int64)
    val = np.ascontiguousarray(val, np.float64)
    resp = np.ascontiguousarray(resp, np.float32)
    pix = np.ascontiguousarray(pix, np.int32)
    L = grid.nticks + kticks - 1
    wf = np.zeros((pix.shape[0], L))
    g = ogrid(grid)
    kp = np.ascontiguousarray(kpix, np.int32)
    lib().oracle_waveforms(C.byref(g), _p(kp), int(kticks), _p(resp), fp.shape[0], _p(fp), _p(off),
                           _p(val), pix.shape[0], _p(pix), _p(wf))
    return wf


def waveform_points(grid, kpix, kticks, resp, fp, off, val, pts) -> np.ndarray:
    """Waveform values at isolated samples pts [m, 2] = (pixel id, tick)."""
    fp = np.ascontiguousarray(fp, np.int32).reshape(-1, 6)
    off = np.ascontiguousarray(off, np.int64)
    val = np.ascontiguousarray(val, np.float64)
    resp = np.ascontiguousarray(resp, np.float32)
    pts = np.ascontiguousarray(pts, np.int32).reshape(-1, 2)
    out = np.zeros(pts.shape[0])
    g = ogrid(grid)
    kp = np.ascontiguousarray(kpix, np.int32)
    lib().oracle_waveform_points(C.byref(g), _p(kp), int(kticks), _p(resp), fp.shape[0], _p(fp),
                                 _p(off), _p(val), pts.shape[0], _p(pts), _p(out))
    return out


def simulate(grid, physics, blocking, kpix, kticks, resp, seg):
    """The whole path for a small event: footprints, patches, bins, pixels, waveforms."""
    fp, off, ip = footprints(grid, physics, seg)
    val, ns = effq(grid, physics, seg, fp, off)
    keys = block_keys(grid, blocking, fp)
    pix = pix_set(grid, blocking, kpix, keys)
    wf = waveforms(grid, kpix, kticks, resp, fp, off, val, pix)
    return dict(fp=fp, off=off, is_point=ip, val=val, node_sums=ns, keys=keys, pix=pix, wf=wf)


def bin_members(grid, blocking, fp, key) -> np.ndarray:
    """Indices of the depositions whose footprint has a cell in bin `key` (Sec. III-B:
    a bin collects every patch cell inside its box)."""
    fp = np.asarray(fp).reshape(-1, 6)
    bf = (blocking.blk_pix[0] * grid.sub[0], blocking.blk_pix[1] * grid.sub[1], blocking.blk_ticks)
    keep = np.ones(fp.shape[0], bool)
    for a in range(3):
        lo, hi = key[a] * bf[a], key[a] * bf[a] + bf[a] - 1
        keep &= (fp[:, a] <= fp[:, 3 + a]) & (fp[:, a] <= hi) & (fp[:, 3 + a] >= lo)
    return np.nonzero(keep)[0]


def block_output_points(grid, blocking, kpix, kticks, resp, bvals, pts) -> np.ndarray:
    """One bin's contribution to the induced current (Sec. II-D, eq. interlaced, summed
    over the bin's cells only) at samples pts [m, 3] = (qx, qy, t') in the bin's output
    frame: pixel (bx Bx - (Kx-1)/2 + qx, by By - (Ky-1)/2 + qy), tick bt Bt + t'.
    bvals [Bx sx][By sy][Bt] is the bin's effective charge (binary64). With charge at
    fine cell (px sx + jx, py sy + jy, t): out += Q * R[qx - px][qy - py][jx][jy][t' - t]."""
    sx, sy = grid.sub
    Bx, By = blocking.blk_pix
    Bt = blocking.blk_ticks
    Kx, Ky = kpix
    R = np.asarray(resp, np.float64).reshape(Kx, Ky, sx, sy, kticks)
    Q = np.asarray(bvals, np.float64).reshape(Bx, sx, By, sy, Bt)
    out = np.zeros(len(pts))
    for m, (qx, qy, tq) in enumerate(np.asarray(pts).reshape(-1, 3)):
        t_lo, t_hi = max(0, tq - kticks + 1), min(Bt - 1, tq)
        if t_lo > t_hi:
            continue
        acc = 0.0
        for px in range(max(0, qx - Kx + 1), min(Bx - 1, qx) + 1):
            for py in range(max(0, qy - Ky + 1), min(By - 1, qy) + 1):
                q = Q[px, :, py, :, t_lo:t_hi + 1]                       # [sx, sy, nt]
                r = R[qx - px, qy - py][:, :, tq - t_hi:tq - t_lo + 1][:, :, ::-1]
                acc += float(np.sum(q * r))
        out[m] = acc
    return out


def select_near(fp, sub, kpix, kticks, pts, margin_pix: int = 0) -> np.ndarray:
    """Indices of depositions whose footprint can reach any sample in pts (pixel id is
    split with npix_y by the caller: pts [m, 3] = (px, py, tick))."""
    fp = np.asarray(fp).reshape(-1, 6)
    hx, hy = (kpix[0] - 1) // 2, (kpix[1] - 1) // 2
    keep = np.zeros(fp.shape[0], bool)
    px0, px1 = fp[:, 0] // sub[0], fp[:, 3] // sub[0]
    py0, py1 = fp[:, 1] // sub[1], fp[:, 4] // sub[1]
    nonempty = (fp[:, 3] >= fp[:, 0]) & (fp[:, 4] >= fp[:, 1]) & (fp[:, 5] >= fp[:, 2])
    for px, py, t in np.asarray(pts).reshape(-1, 3):
        keep |= nonempty & (px0 <= px + hx + margin_pix) & (px1 >= px - hx - margin_pix) & \
            (py0 <= py + hy + margin_pix) & (py1 >= py - hy - margin_pix) & \
            (fp[:, 2] <= t) & (fp[:, 5] >= t - kticks + 1)
    return np.nonzero(keep)[0]

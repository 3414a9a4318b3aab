"""Seeded synthetic inputs for the pixel-TPC signal-formation hot path.

This module is the only code shared by the FP64 oracle tests and the GPU path.
It produces *inputs* only (parameter sets, track-segment depositions, a
synthetic field response); it contains none of the method's arithmetic
(no transport, no quadrature, no binning, no convolution).

Inputs stand in for the paper's GENIE + edep-sim ND-LAr spills and for its
COMSOL/pochoir field response (Sec. IV-A), which are not available here.
Shapes follow the paper where it states them: segments spanning tens to
hundreds of ticks, a 5x5-pixel x ~2000-tick response sampled at 10x10 impact
positions per pixel, 50 ns ticks (Sec. IV-A, Fig. frillu).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

# ----------------------------------------------------------------------------
# Parameter containers (plain data; field order mirrors the C structs)
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Grid:
    """Fine sampling grid of the field response (Sec. II-B, II-C).

    origin: x, y of the lower edge of pixel (0,0) [cm]; t of tick 0 [us].
    spacing: fine cell size h_x, h_y [cm] (= pitch / sub) and tick [us].
    """
    origin: Tuple[float, float, float]
    spacing: Tuple[float, float, float]
    npix: Tuple[int, int]
    sub: Tuple[int, int]
    nticks: int

    @property
    def nfine(self):
        return (self.npix[0] * self.sub[0], self.npix[1] * self.sub[1], self.nticks)


@dataclasses.dataclass
class Physics:
    """Transport and quadrature parameters (Sec. II-A, II-C).

    v_drift [cm/us], lifetime [us], diff_T / diff_L [cm^2/us],
    sigma_min (x [cm], y [cm], t [us]) floor on the diffusion widths,
    n_sigma window half-width in sigmas, point_frac threshold of the
    point-like switch, n_gl Gauss-Legendre points per axis per cell.
    """
    v_drift: float = 0.16
    lifetime: float = 2200.0
    diff_T: float = 8.8e-6
    diff_L: float = 4.0e-6
    sigma_min: Tuple[float, float, float] = (0.022, 0.022, 0.025)
    n_sigma: float = 4.0
    point_frac: float = 0.1
    n_gl: int = 2


@dataclasses.dataclass
class Blocking:
    """Block shape of the block-sparse binned tensor (Sec. III-B)."""
    blk_pix: Tuple[int, int]
    blk_ticks: int


@dataclasses.dataclass
class Config:
    name: str
    grid: Grid
    physics: Physics
    blocking: Blocking
    kpix: Tuple[int, int]     # response extent in pixels (odd)
    kticks: int               # response length in ticks
    fft: Tuple[int, int, int]  # FFT sizes (x, y, t) used by the conv plan
    n_dep: int
    kind: str                 # 'uniform' | 'module'
    seed: int = 1


PITCH = 0.44       # cm, 4.4 mm pixel pitch
SUB = 10           # 10 x 10 impact positions per pixel
TICK = 0.05        # us
V_DRIFT = 0.16     # cm/us


def _grid(npix, nticks):
    h = PITCH / SUB
    return Grid(origin=(0.0, 0.0, 0.0), spacing=(h, h, TICK), npix=(npix, npix),
                sub=(SUB, SUB), nticks=nticks)


def _physics(grid: Grid, **kw):
    h = grid.spacing
    p = Physics(sigma_min=(0.5 * h[0], 0.5 * h[1], 0.5 * h[2]))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def cfg_plain_small(seed: int = 1) -> Config:
    """1,000 line segments in a 32x32-pixel region, 50 cm drift, 5x5x200 response,
    blocks of 4x4 pixels x 128 ticks."""
    g = _grid(32, 6250)
    return Config("plain-small-1k", g, _physics(g), Blocking((4, 4), 128), (5, 5), 200,
                  (8, 8, 256), 1000, "uniform", seed)


def cfg_module(seed: int = 1) -> Config:
    """1e5 depositions (40 muon-like tracks + 20 shower blobs) in a 256x256-pixel region,
    21x21x2048 response, blocks of 16x16 pixels x 512 ticks."""
    g = _grid(256, 6250)
    return Config("module-1e5", g, _physics(g), Blocking((16, 16), 512), (21, 21), 2048,
                  (40, 40, 1024), 100_000, "module", seed)


def cfg_diff(seed: int = 1) -> Config:
    """2e4 depositions in a 128x128-pixel region with the module-scale response."""
    g = _grid(128, 6250)
    return Config("diff-2e4", g, _physics(g), Blocking((16, 16), 512), (21, 21), 2048,
                  (40, 40, 1024), 20_000, "module", seed)


# ----------------------------------------------------------------------------
# Depositions
# ----------------------------------------------------------------------------


def _isotropic(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def gen_uniform_segments(n: int, xy_extent: Tuple[float, float], z_range=(0.0, 50.0),
                         length_range=(0.01, 0.1), q_median=2.0e4, q_sigma=0.5,
                         seed: int = 1, xy_origin=(0.0, 0.0)) -> np.ndarray:
    """Straight line segments with midpoints uniform in the box, isotropic direction,
    length U[length_range] cm and lognormal charge (electrons after recombination).

    Returns float32 [n, 7] rows (x0, y0, z0, x1, y1, z1, Q); z is drift distance [cm].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    mid = np.empty((n, 3))
    mid[:, 0] = xy_origin[0] + rng.uniform(0.0, xy_extent[0], n)
    mid[:, 1] = xy_origin[1] + rng.uniform(0.0, xy_extent[1], n)
    mid[:, 2] = rng.uniform(z_range[0], z_range[1], n)
    d = _isotropic(rng, n)
    L = rng.uniform(length_range[0], length_range[1], n)
    p0 = mid - 0.5 * L[:, None] * d
    p1 = mid + 0.5 * L[:, None] * d
    q = rng.lognormal(math.log(q_median), q_sigma, n)
    seg = np.concatenate([p0, p1, q[:, None]], axis=1)
    # keep drift distances non-negative (a segment cannot start behind the anode)
    seg[:, 2] = np.abs(seg[:, 2])
    seg[:, 5] = np.abs(seg[:, 5])
    return seg.astype(np.float32)


def gen_module_event(n_dep: int, xy_extent: Tuple[float, float], z_max: float = 50.0,
                     n_tracks: int = 40, n_blobs: int = 20, step: float = 0.05,
                     track_len=(50.0, 150.0), blob_sigma=(1.0, 3.0),
                     seed: int = 1) -> np.ndarray:
    """Module-scale event: straight muon-like tracks stepped at `step` cm with a
    Landau-like (lognormal) charge per step, plus compact shower blobs (Gaussian
    clouds of short segments) carrying the remaining depositions up to n_dep.

    Track length U[track_len] cm, clipped to the box. Returns float32 [n_dep, 7].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.array([0.0, 0.0, 0.0])
    hi = np.array([xy_extent[0], xy_extent[1], z_max])
    rows = []
    total = 0
    for _ in range(n_tracks):
        start = rng.uniform(lo, hi)
        d = _isotropic(rng, 1)[0]
        L = rng.uniform(*track_len)
        # clip the track to the box: largest s in [0, L] with start + s d inside
        smax = L
        for a in range(3):
            if d[a] > 0:
                smax = min(smax, (hi[a] - start[a]) / d[a])
            elif d[a] < 0:
                smax = min(smax, (lo[a] - start[a]) / d[a])
        nstep = int(smax / step)
        if nstep <= 0:
            continue
        s = np.arange(nstep + 1) * step
        pts = start[None, :] + s[:, None] * d[None, :]
        q = rng.lognormal(math.log(3.0e3), 0.35, nstep)
        rows.append(np.concatenate([pts[:-1], pts[1:], q[:, None]], axis=1))
        total += nstep
        if total >= n_dep:
            break
    n_blob_dep = max(0, n_dep - total)
    if n_blob_dep > 0:
        per = np.full(n_blobs, n_blob_dep // n_blobs)
        per[: n_blob_dep % n_blobs] += 1
        for b in range(n_blobs):
            m = int(per[b])
            if m == 0:
                continue
            c = np.array([rng.uniform(0, xy_extent[0]), rng.uniform(0, xy_extent[1]),
                          rng.uniform(5.0, 45.0)])
            sb = rng.uniform(*blob_sigma)
            mid = c[None, :] + sb * rng.normal(size=(m, 3))
            # reflect into the box so every deposition lies inside the volume
            for a in range(3):
                span = hi[a] - lo[a]
                x = np.mod(mid[:, a] - lo[a], 2 * span)
                mid[:, a] = lo[a] + np.where(x > span, 2 * span - x, x)
            d = _isotropic(rng, m)
            p0 = mid - 0.5 * step * d
            p1 = mid + 0.5 * step * d
            q = rng.lognormal(math.log(3.0e3), 0.5, m)
            rows.append(np.concatenate([p0, p1, q[:, None]], axis=1))
    seg = np.concatenate(rows, axis=0)[:n_dep]
    seg[:, 2] = np.abs(seg[:, 2])
    seg[:, 5] = np.abs(seg[:, 5])
    return seg.astype(np.float32)


def gen_event_batch(n_ev: int = 64, n_range=(1_000, 200_000), npix: int = 256,
                    nticks: int = 6250, seed: int = 1):
    """A batch of module-scale events of uneven size: deposition counts log-uniform in
    n_range, each generated like the module event with a per-event mix of tracks
    (5-60) and blobs (2-30). Returns a list of float32 [n_e, 7] arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ext = (npix * PITCH, npix * PITCH)
    zmax = nticks * TICK * V_DRIFT
    out = []
    for e in range(n_ev):
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        nt = int(rng.integers(5, 61))
        nb = int(rng.integers(2, 31))
        out.append(gen_module_event(n, ext, zmax, n_tracks=nt, n_blobs=nb,
                                    seed=int(rng.integers(1, 2**31))))
    return out


def gen_segments(cfg: Config, seed: Optional[int] = None) -> np.ndarray:
    seed = cfg.seed if seed is None else seed
    g = cfg.grid
    ext = (g.npix[0] * PITCH, g.npix[1] * PITCH)
    zmax = g.nticks * g.spacing[2] * cfg.physics.v_drift
    if cfg.kind == "uniform":
        return gen_uniform_segments(cfg.n_dep, ext, (0.0, zmax), seed=seed)
    if cfg.kind == "module":
        return gen_module_event(cfg.n_dep, ext, zmax, seed=seed)
    raise ValueError(cfg.kind)


# ----------------------------------------------------------------------------
# Synthetic field response
# ----------------------------------------------------------------------------


def synthetic_response(kpix: Tuple[int, int], sub: Tuple[int, int], kticks: int,
                       pitch: float = PITCH, seed: int = 7) -> np.ndarray:
    """Seeded synthetic field response R[kx][ky][jx][jy][tau], float32.

    R[kx][ky][jx][jy][:] is the current on the pixel at offset
    (kx - (Kx-1)/2, ky - (Ky-1)/2) from the pixel holding a unit charge released
    at impact position (jx, jy) (impact centres at ((j + 1/2)/sub - 1/2) * pitch
    from the pixel centre).

    * offset (0, 0), the collecting pixel: a smooth unipolar pulse near the end of
      the window with a small negative precursor and a slow induction ramp,
      normalised to unit net area;
    * other offsets: smooth bipolar pulses with zero net area whose amplitude
      decays as exp(-|rho| / (pitch/2)) with the charge-electrode distance rho;
    * a seeded +-5% jitter (width of the collecting pulse, amplitude of the
      induction pulses), drawn once per pair {(j, k), (-j, -k)};
    * exact point symmetry R[Kx-1-kx][Ky-1-ky][sx-1-jx][sy-1-jy] = R[kx][ky][jx][jy]
      (the reflected half is a copy), as the mirror-pair packing requires.

    Computed in float64, stored float32.
    """
    Kx, Ky = kpix
    sx, sy = sub
    assert Kx % 2 == 1 and Ky % 2 == 1
    hx, hy = (Kx - 1) // 2, (Ky - 1) // 2
    rng = np.random.Generator(np.random.PCG64(seed))
    ncan = Kx * Ky * sx * sy
    jit = rng.uniform(-1.0, 1.0, size=ncan)
    tau = np.arange(kticks, dtype=np.float64)
    tc = 0.9 * kticks
    wc0 = max(1.5, kticks / 100.0)
    Lr = kticks / 4.0

    def gauss(t, mu, w):
        return np.exp(-0.5 * ((t - mu) / w) ** 2)

    ramp = np.where(tau < tc, np.exp((tau - tc) / Lr), 0.0)
    R = np.zeros((Kx, Ky, sx, sy, kticks), dtype=np.float32)
    done = np.zeros((Kx, Ky, sx, sy), dtype=bool)
    for kx in range(Kx):
        for ky in range(Ky):
            for jx in range(sx):
                for jy in range(sy):
                    if done[kx, ky, jx, jy]:
                        continue
                    rk = (Kx - 1 - kx, Ky - 1 - ky, sx - 1 - jx, sy - 1 - jy)
                    lin = ((kx * Ky + ky) * sx + jx) * sy + jy
                    lin_r = ((rk[0] * Ky + rk[1]) * sx + rk[2]) * sy + rk[3]
                    u = jit[min(lin, lin_r)]
                    lam = np.array([((jx + 0.5) / sx - 0.5) * pitch, ((jy + 0.5) / sy - 0.5) * pitch])
                    rho = lam - np.array([(kx - hx) * pitch, (ky - hy) * pitch])
                    r = float(np.hypot(rho[0], rho[1]))
                    if kx == hx and ky == hy:
                        wc = wc0 * (1.0 + r / pitch) * (1.0 + 0.05 * u)
                        s = gauss(tau, tc, wc) - 0.08 * gauss(tau, tc - 3.0 * wc, wc) + 0.02 * ramp
                        s = s / s.sum()
                    else:
                        amp = 0.3 * math.exp(-r / (0.5 * pitch)) * (1.0 + 0.05 * u)
                        wn = wc0 * 1.5
                        pulse = gauss(tau, tc - wn, wn) - gauss(tau, tc + wn, wn)
                        g0 = gauss(tau, tc, wc0)
                        body = pulse + 0.5 * ramp
                        s = amp * (body - body.sum() * g0 / g0.sum())
                    v = s.astype(np.float32)
                    R[kx, ky, jx, jy] = v
                    R[rk] = v
                    done[kx, ky, jx, jy] = True
                    done[rk] = True
    return R


def delta_response(kpix, sub, kticks, kx, ky, jx, jy, tau) -> np.ndarray:
    """All-zero response except one unit entry (for index-convention tests)."""
    R = np.zeros((kpix[0], kpix[1], sub[0], sub[1], kticks), dtype=np.float32)
    R[kx, ky, jx, jy, tau] = 1.0
    return R


def random_symmetric_response(kpix, sub, kticks, seed=3) -> np.ndarray:
    """Uniform random response with the exact point symmetry used by mirror-pair packing."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = rng.uniform(-1.0, 1.0, size=(kpix[0], kpix[1], sub[0], sub[1], kticks)).astype(np.float32)
    Rr = R[::-1, ::-1, ::-1, ::-1, :]
    Kx, Ky, sx, sy = R.shape[:4]
    idx = np.arange(Kx * Ky * sx * sy).reshape(Kx, Ky, sx, sy)
    keep = idx <= idx[::-1, ::-1, ::-1, ::-1]
    out = np.where(keep[..., None], R, Rr)
    return np.ascontiguousarray(out.astype(np.float32))

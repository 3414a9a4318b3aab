"""Pins for the FP64 oracle (CPU only).

Each test ties an oracle function to something other than itself: textbook
quadrature rules, an adaptive numerical line integral, closed forms (erf
differences, tent projections), algebraic invariants of the trilinear spread,
brute force on tiny inputs and an FFT-based convolution computed by numpy.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_grid(npix=6, sub=10, nticks=160, h=0.044, tick=0.05, t0=0.0):
    return W.Grid(origin=(0.0, 0.0, t0), spacing=(h, h, tick), npix=(npix, npix), sub=(sub, sub),
                  nticks=nticks)


def grid_at(z, npix=6, nticks=400):
    """Tiny grid whose 400-tick window is centred on drift distance z [cm]."""
    return tiny_grid(npix=npix, nticks=nticks, t0=z / 0.16 - nticks * 0.05 / 2)


def phys_for(grid, **kw):
    h = grid.spacing
    p = W.Physics(sigma_min=(0.5 * h[0], 0.5 * h[1], 0.5 * h[2]))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def Phi(x):
    return 0.5 * special.erfc(-x / math.sqrt(2.0))


# ---------------------------------------------------------------------------
# Gauss-Legendre rule
# ---------------------------------------------------------------------------


def test_gl_rule_golden_closed_forms(orc):
    rows = {}
    with open(os.path.join(GOLDEN, "gauss_legendre.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, x, w = line.split()
            env = {"sqrt": math.sqrt}
            rows.setdefault(int(n), []).append((eval(x, env), eval(w, env)))
    for n, nodes in rows.items():
        xi, w = orc.gl_rule(n)
        assert np.allclose(xi, [a for a, _ in nodes], rtol=0, atol=1e-15)
        assert np.allclose(w, [b for _, b in nodes], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", list(range(1, 17)) + [24, 32])
def test_gl_rule_vs_numpy(orc, n):
    xi, w = orc.gl_rule(n)
    X, Wt = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(xi - X)) < 1e-14
    assert np.max(np.abs(w - Wt)) < 1e-14
    # exact for polynomials of degree 2n-1
    for deg in range(2 * n):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.sum(w * xi ** deg) - exact) < 1e-13


# ---------------------------------------------------------------------------
# Line-charge density
# ---------------------------------------------------------------------------


def line_integral(x, p0, p1, sig, Q):
    """Q * int_0^1 ds N3(x - p0 - s (p1 - p0); diag(sig^2)) by adaptive quadrature."""
    p0, p1, sig, x = map(np.asarray, (p0, p1, sig, x))
    d = p1 - p0
    norm = (2 * math.pi) ** -1.5 / np.prod(sig)

    def f(s):
        r = (x - p0 - s * d) / sig
        return norm * math.exp(-0.5 * float(r @ r))

    # split at the closest point to help the integrator
    a = (x - p0) / sig ** 2
    al = float(d @ (d / sig ** 2))
    sstar = min(max(float(a @ d) / al, 0.0), 1.0)
    pts = sorted({0.0, sstar, 1.0})
    tot = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        if hi > lo:
            tot += integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-13, limit=200)[0]
    return Q * tot


@pytest.mark.parametrize("offset", [0.0, 100.0])
def test_q_line_vs_numerical_line_integral(orc, offset):
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(40):
        sig = rng.uniform(0.02, 0.1, 3)
        p0 = rng.uniform(-0.1, 0.1, 3) + offset
        p1 = p0 + rng.normal(size=3) * rng.uniform(0.5, 5.0) * sig
        x = p0 + rng.uniform(-0.5, 1.5) * (p1 - p0) + rng.normal(size=3) * 1.5 * sig
        ref = line_integral(x, p0, p1, sig, 1.0)
        got = orc.q_line(*x, p0, p1, sig, 1.0)
        if ref > 1e-6 * (2 * math.pi) ** -1.5 / np.prod(sig):
            worst = max(worst, abs(got - ref) / ref)
    tol = 1e-9 if offset == 0.0 else 2e-7  # absolute-coordinate form loses digits far out
    assert worst < tol


def test_q_line_axis_aligned_closed_form(orc):
    # segment along x: q = (Q/L)[Phi((x-x0)/sx) - Phi((x-x1)/sx)] N(y) N(z)
    sig = np.array([0.05, 0.03, 0.07])
    p0 = np.array([0.1, 0.2, 0.3])
    p1 = np.array([0.4, 0.2, 0.3])
    L = 0.3
    for x in np.linspace(-0.1, 0.6, 15):
        for y in (0.2, 0.23, 0.27):
            for z in (0.3, 0.25, 0.4):
                ref = (2.0 / L) * (Phi((x - p0[0]) / sig[0]) - Phi((x - p1[0]) / sig[0])) * \
                    math.exp(-0.5 * ((y - 0.2) / sig[1]) ** 2) / (math.sqrt(2 * math.pi) * sig[1]) * \
                    math.exp(-0.5 * ((z - 0.3) / sig[2]) ** 2) / (math.sqrt(2 * math.pi) * sig[2])
                got = orc.q_line(x, y, z, p0, p1, sig, 2.0)
                assert abs(got - ref) <= 1e-11 * max(ref, 1e-300) + 1e-300


def test_q_line_point_limit(orc):
    sig = np.array([0.05, 0.06, 0.04])
    m = np.array([0.0, 0.0, 0.0])
    d = np.array([1.0, -0.5, 0.3])
    for eps in (1e-2, 1e-3):
        p0, p1 = m - 0.5 * eps * sig * d, m + 0.5 * eps * sig * d
        for x in [(0.0, 0.0, 0.0), (0.03, -0.02, 0.05), (0.1, 0.05, -0.04)]:
            ql = orc.q_line(*x, p0, p1, sig, 1.0)
            qp = orc.q_point(*x, m, sig, 1.0)
            assert abs(ql - qp) / qp < 5 * eps ** 2 * 10  # O((L/sigma)^2)


def test_point_switch_threshold(orc):
    g = tiny_grid()
    ph = phys_for(g)
    # at z=40 cm sigma_T ~ 0.066 cm, sigma_t ~ 0.28 us; a segment along x
    tr = orc.transport(ph, [0.1, 0.1, 40.0, 0.1, 0.1, 40.0, 1.0])
    sx = tr[4]
    for frac, expect in ((0.05, True), (0.2, False)):
        seg = [0.1, 0.1, 40.0, 0.1 + frac * sx, 0.1, 40.0, 1.0]
        _, _, ip = orc.window_f32(g, ph, seg)
        assert ip == expect


def _moments(fp, Q):
    """Total, mean and variance (in cell-index units) of a patch along each axis."""
    tot = Q.sum()
    out = []
    for a in range(3):
        marg = Q.sum(axis=tuple(b for b in range(3) if b != a))
        g = np.arange(fp[a], fp[3 + a] + 1, dtype=np.float64)
        m = float((marg * g).sum() / tot)
        out.append((m, float((marg * (g - m) ** 2).sum() / tot)))
    return tot, out


def _tent_variance(n):
    """Mean over the n Gauss-Legendre nodes of f (1 - f), f = |xi| / 2: the variance the
    trilinear spread adds (in cell units) to a density that is smooth on the cell scale.
    A node at offset f from its cell's grid point pushes 1 - f there and f to the
    neighbour, so its second moment grows by f (1 - f); summed over all cells of a density
    whose width is several cells, each node offset samples the density's integral."""
    X, Wt = np.polynomial.legendre.leggauss(n)
    f = np.abs(X) / 2.0
    return float(np.sum(Wt / 2.0 * f * (1.0 - f)))


def _transport_probe(orc, seg, n_gl=2, sigma_min=None, npix=12, h=0.02, nticks=1200):
    """Patch of one deposition on a fine grid (h = 0.02 cm) centred on it, with windows
    of 8 widths so that the truncated tails are below 1e-14."""
    zc = 0.5 * (float(seg[2]) + float(seg[5]))
    t0 = zc / float(np.float32(0.16)) - nticks * 0.05 / 2
    g = W.Grid(origin=(0.0, 0.0, float(np.float32(t0))), spacing=(h, h, 0.05), npix=(npix, npix),
               sub=(10, 10), nticks=nticks)
    smin = sigma_min or (0.1 * h, 0.1 * h, 0.1 * 0.05)
    ph = W.Physics(sigma_min=smin, n_sigma=8.0, n_gl=n_gl)
    s = np.asarray(seg, np.float32)
    fp, off, ip = orc.footprints(g, ph, s)
    N = g.nfine
    assert (fp[0, :3] > 0).all() and (fp[0, 3:] < np.array(N) - 1).all(), "patch must be interior"
    val, _ = orc.effq(g, ph, s, fp, off)
    shape = tuple(int(fp[0, 3 + a] - fp[0, a] + 1) for a in range(3))
    return g, ph, fp[0], val.reshape(shape), bool(ip[0])


# Transport constants as the oracle receives them (binary32 inputs, exact in binary64).
_V = float(np.float32(0.16))
_TAU = float(np.float32(2200.0))
_DT = float(np.float32(8.8e-6))
_DL = float(np.float32(4.0e-6))


@pytest.mark.parametrize("z,n_gl", [(20.0, 2), (40.0, 2), (32.0, 3)])
def test_transport_point_moments(orc, z, n_gl):
    """A point deposition after drift z (Sec. II-A): the effective charge carries the
    surviving charge Q exp(-t/tau_e) and is a Gaussian of variance 2 D_T t (x, y, in
    cm^2) and 2 D_L t / v^2 (t, in us^2) with t = z / v, plus the tent variance of the
    trilinear spread. Read off the oracle's patch only (no call of its transport)."""
    x, y = 1.2203, 1.1311
    seg = np.array([x, y, z, x, y, z, 1.0e4], np.float32)
    g, ph, fp, Q, ip = _transport_probe(orc, seg, n_gl=n_gl)
    assert ip
    t = float(np.float32(z)) / _V
    tot, mom = _moments(fp, Q)
    assert abs(tot / (1.0e4 * math.exp(-t / _TAU)) - 1.0) < 1e-10
    c = _tent_variance(n_gl)
    h = [float(np.float32(s)) for s in g.spacing]
    exp_var = [2 * _DT * t, 2 * _DT * t, 2 * _DL * t / _V ** 2]
    for a in range(3):
        var = (mom[a][1] - c) * h[a] ** 2
        assert abs(var / exp_var[a] - 1.0) < 1e-8, (a, var, exp_var[a])
    # the centre sits at the deposition (grid point i at (i + 1/2) h, tick n at t0 + n tick)
    assert abs(g.origin[0] + (mom[0][0] + 0.5) * h[0] - float(np.float32(x))) < 1e-9
    assert abs(g.origin[1] + (mom[1][0] + 0.5) * h[1] - float(np.float32(y))) < 1e-9
    assert abs(float(np.float32(g.origin[2])) + mom[2][0] * h[2] - t) < 1e-7


def test_transport_attenuation_ratio(orc):
    """Charge surviving two drift distances differs by exp(-dz / (v tau_e))."""
    tots = []
    for z in (12.0, 44.0):
        seg = np.array([1.21, 1.23, z, 1.21, 1.23, z, 3.0e3], np.float32)
        _, _, fp, Q, _ = _transport_probe(orc, seg)
        tots.append(Q.sum())
    assert abs(tots[1] / tots[0] / math.exp(-32.0 / (_V * _TAU)) - 1.0) < 1e-10


def test_transport_line_along_drift_uses_mid_time(orc):
    """A segment along the drift direction (Sec. II-C: one width per segment): the
    transverse variance is 2 D_T t_mid at its mid drift time, the variance along t is
    the segment's duration squared / 12 plus 2 D_L t_mid / v^2, and the surviving charge
    is Q exp(-t_mid / tau_e)."""
    x, y, z0, z1 = 1.1977, 1.2048, 19.0, 21.0
    seg = np.array([x, y, z0, x, y, z1, 2.0e4], np.float32)
    g, ph, fp, Q, ip = _transport_probe(orc, seg, nticks=1200)
    assert not ip
    t0, t1 = float(np.float32(z0)) / _V, float(np.float32(z1)) / _V
    tm = 0.5 * (t0 + t1)
    tot, mom = _moments(fp, Q)
    assert abs(tot / (2.0e4 * math.exp(-tm / _TAU)) - 1.0) < 1e-10
    c = _tent_variance(2)
    h = [float(np.float32(s)) for s in g.spacing]
    for a in range(2):
        assert abs((mom[a][1] - c) * h[a] ** 2 / (2 * _DT * tm) - 1.0) < 1e-8
    var_t = (mom[2][1] - c) * h[2] ** 2
    assert abs(var_t / ((t1 - t0) ** 2 / 12.0 + 2 * _DL * tm / _V ** 2) - 1.0) < 1e-8


def test_transport_width_floor(orc):
    """Widths below the minimum diffusion scale are raised to it, per axis (x, y to
    0.07 cm, t to 0.3 us here, both above the diffused widths at 20 cm)."""
    seg = np.array([1.19, 1.22, 20.0, 1.19, 1.22, 20.0, 1.0e4], np.float32)
    smin = (0.07, 0.07, 0.3)
    g, ph, fp, Q, ip = _transport_probe(orc, seg, sigma_min=smin)
    t = float(np.float32(20.0)) / _V
    assert 2 * _DT * t < 0.07 ** 2 and 2 * _DL * t / _V ** 2 < 0.3 ** 2
    tot, mom = _moments(fp, Q)
    c = _tent_variance(2)
    h = [float(np.float32(s)) for s in g.spacing]
    for a in range(3):
        var = (mom[a][1] - c) * h[a] ** 2
        assert abs(var / float(np.float32(smin[a])) ** 2 - 1.0) < 1e-8, a
    # the floor changes the shape only: the surviving charge is unchanged
    assert abs(tot / (1.0e4 * math.exp(-t / _TAU)) - 1.0) < 1e-10


def test_select_near_keeps_every_contributor(orc):
    """The depositions select_near keeps for a set of samples give the same waveform
    values there as all depositions, and each one it drops contributes exactly zero."""
    g, ph, seg, fp, off, val = _small_event(orc, n=30, nticks=96)
    K, kt = (3, 5), 24
    R = np.abs(W.random_symmetric_response(K, g.sub, kt, seed=4)) + 0.1
    rng = np.random.default_rng(3)
    pts = np.stack([rng.integers(0, 6, 8), rng.integers(0, 6, 8), rng.integers(0, 96 + kt - 1, 8)], 1)
    ids = np.stack([pts[:, 0] * g.npix[1] + pts[:, 1], pts[:, 2]], 1)
    near = orc.select_near(fp, g.sub, K, kt, pts)
    assert 0 < len(near) < fp.shape[0]
    full = orc.waveform_points(g, K, kt, R, fp, off, val, ids)
    vol = np.prod(np.maximum(fp[near, 3:] - fp[near, :3] + 1, 0), axis=1)
    soff = np.concatenate([[0], np.cumsum(vol)]).astype(np.int64)
    sval = np.concatenate([val[off[d]:off[d + 1]] for d in near])
    part = orc.waveform_points(g, K, kt, R, fp[near], soff, sval, ids)
    assert np.array_equal(part, full)
    for d in sorted(set(range(fp.shape[0])) - set(near.tolist())):
        one = orc.waveform_points(g, K, kt, R, fp[d:d + 1], np.array([0, off[d + 1] - off[d]]),
                                  val[off[d]:off[d + 1]], ids)
        assert not one.any(), d


# ---------------------------------------------------------------------------
# Windows / footprints (discrete decisions)
# ---------------------------------------------------------------------------


def test_windows_cover_n_sigma_extent(orc):
    cfg = W.cfg_plain_small()
    seg = W.gen_segments(cfg)
    g, ph = cfg.grid, cfg.physics
    for d in range(0, 1000, 7):
        lo, hi, _ = orc.window_f32(g, ph, seg[d])
        tr = orc.transport(ph, seg[d])
        P0 = [float(seg[d, 0]), float(seg[d, 1]), tr[0]]
        P1 = [float(seg[d, 3]), float(seg[d, 4]), tr[1]]
        for a in range(3):
            h = float(np.float32(g.spacing[a]))
            sh = 0.5 if a == 2 else 0.0
            u = sorted([(P0[a] - g.origin[a]) / h + sh, (P1[a] - g.origin[a]) / h + sh])
            e = ph.n_sigma * tr[4 + a] / h
            # floor of the exact bounds, up to binary32 rounding right at a cell edge
            assert lo[a] <= u[0] - e + 1e-4 and u[0] - e - 1e-4 < lo[a] + 1
            assert hi[a] <= u[1] + e + 1e-4 and u[1] + e - 1e-4 < hi[a] + 1


def test_footprint_is_window_dilated_and_cropped(orc):
    g = tiny_grid(npix=3, sub=10, nticks=80)
    ph = phys_for(g)
    seg = np.array([[0.005, 0.06, 0.01, 0.02, 0.07, 0.03, 1e4],     # near the x, t lower edges
                    [0.12, 0.12, 0.75, 0.13, 0.125, 0.76, 1e4],     # beyond the last tick
                    [0.05, 0.05, 0.30, 0.06, 0.05, 0.31, 1e4]], np.float32)
    fp, off, _ = orc.footprints(g, ph, seg)
    N = g.nfine
    for d in range(3):
        lo, hi, _ = orc.window_f32(g, ph, seg[d])
        for a in range(3):
            assert fp[d, a] == max(lo[a] - 1, 0)
            assert fp[d, 3 + a] == min(hi[a] + 1, N[a] - 1)
    assert fp[1, 5] < fp[1, 2] and off[2] - off[1] == 0  # empty: entirely after the window end


# ---------------------------------------------------------------------------
# Effective charge
# ---------------------------------------------------------------------------


def _point_dep(x=1.302, y=1.214, z=40.0, q=1.0e4):
    return np.array([x, y, z, x + 1e-4, y, z, q], np.float32)


def test_node_sum_equals_erf_box_integral(orc):
    """Point charge in a box: the node sum over the window approximates the charge inside
    the window box, a product of erf differences; GL-2 is very accurate once sigma >~ h."""
    g = grid_at(40.0)
    ph = phys_for(g)
    seg = _point_dep(z=40.0)
    fp, off, ip = orc.footprints(g, ph, seg)
    assert ip[0] == 1
    tr = orc.transport(ph, seg)
    lo, hi, _ = orc.window_f32(g, ph, seg)
    mu = [0.5 * (float(seg[0]) + float(seg[3])), 0.5 * (float(seg[1]) + float(seg[4])), tr[2]]
    exp = tr[3]
    for a in range(3):
        h = float(np.float32(g.spacing[a]))
        if a < 2:
            A, B = lo[a] * h, (hi[a] + 1) * h
        else:
            A, B = g.origin[2] + (lo[a] - 0.5) * h, g.origin[2] + (hi[a] + 0.5) * h
        exp *= Phi((B - mu[a]) / tr[4 + a]) - Phi((A - mu[a]) / tr[4 + a])
    _, ns = orc.effq(g, ph, seg, fp, off)
    # GL-2 error of the cells at the window edge (where the slope does not cancel)
    assert abs(ns[0] - exp) / exp < 2e-6
    # and the window loses only the n_sigma tails
    assert abs(exp / tr[3] - special.erf(4 / math.sqrt(2)) ** 3) < 2e-4


def test_cell_sums_equal_per_cell_erf_products(orc):
    g = grid_at(20.0)
    ph = phys_for(g, n_gl=8)
    seg = _point_dep(z=20.0)
    tr = orc.transport(ph, seg)
    lo, hi, _ = orc.window_f32(g, ph, seg)
    c0 = lo + 3
    c1 = np.minimum(c0 + 4, hi)
    cs = orc.cell_sums(g, ph, seg, c0, c1)
    mu = [0.5 * (float(seg[0]) + float(seg[3])), 0.5 * (float(seg[1]) + float(seg[4])), tr[2]]
    edges = []
    for a in range(3):
        h = float(np.float32(g.spacing[a]))
        c = np.arange(c0[a], c1[a] + 2)
        e = c * h if a < 2 else g.origin[2] + (c - 0.5) * h
        edges.append(np.diff(Phi((e - mu[a]) / tr[4 + a])))
    ref = tr[3] * edges[0][:, None, None] * edges[1][None, :, None] * edges[2][None, None, :]
    assert np.max(np.abs(cs - ref)) < 1e-9 * tr[3]


def _patch(orc, g, ph, seg):
    fp, off, ip = orc.footprints(g, ph, seg)
    val, ns = orc.effq(g, ph, seg, fp, off)
    shape = tuple(int(fp[0, 3 + a] - fp[0, a] + 1) for a in range(3))
    return fp[0], val.reshape(shape), ns[0], ip[0]


def test_effq_conserves_node_charge_and_first_moments(orc):
    """Trilinear spread is a partition of unity and reproduces linear functions: the
    total and the first moments of Q_eff equal those of the node charges."""
    g = grid_at(30.0)
    ph = phys_for(g)
    seg = np.array([1.10, 1.22, 30.0, 1.16, 1.25, 30.3, 2.0e4], np.float32)
    fp, Q, ns, ip = _patch(orc, g, ph, seg)
    assert ip == 0
    assert abs(Q.sum() - ns) < 1e-13 * ns
    # node charges recomputed from the (separately pinned) density q and textbook GL nodes
    lo, hi, _ = orc.window_f32(g, ph, seg)
    X, Wt = np.polynomial.legendre.leggauss(2)
    h = [float(np.float32(s)) for s in g.spacing]
    jac = h[0] * h[1] * h[2] / 8.0
    mom = np.zeros(3)
    tot = 0.0
    for cx in range(lo[0], hi[0] + 1):
        for cy in range(lo[1], hi[1] + 1):
            for ct in range(lo[2], hi[2] + 1):
                for l in range(2):
                    for m in range(2):
                        for k in range(2):
                            pos = np.array([cx + X[l] / 2, cy + X[m] / 2, ct + X[k] / 2])
                            x = (pos[0] + 0.5) * h[0]
                            y = (pos[1] + 0.5) * h[1]
                            t = g.origin[2] + pos[2] * h[2]
                            v = Wt[l] * Wt[m] * Wt[k] * jac * orc.q_seg(ph, seg, x, y, t)
                            tot += v
                            mom += v * pos
    assert abs(tot - ns) < 1e-12 * ns
    gx = np.arange(fp[0], fp[3] + 1)[:, None, None]
    gy = np.arange(fp[1], fp[4] + 1)[None, :, None]
    gt = np.arange(fp[2], fp[5] + 1)[None, None, :]
    for a, gg in enumerate((gx, gy, gt)):
        assert abs((Q * gg).sum() - mom[a]) < 1e-11 * abs(mom[a])


def test_effq_point_charge_is_outer_product(orc):
    g = grid_at(25.0)
    ph = phys_for(g)
    fp, Q, ns, ip = _patch(orc, g, ph, _point_dep(z=25.0))
    assert ip == 1
    for ax in range(3):
        M = np.moveaxis(Q, ax, 0).reshape(Q.shape[ax], -1)
        s = np.linalg.svd(M, compute_uv=False)
        assert s[1] < 1e-13 * s[0]


def test_effq_mirror_symmetry(orc):
    """Reflecting the deposition through a grid-point plane reflects Q_eff."""
    g = grid_at(30.0)
    ph = phys_for(g)
    h = float(np.float32(g.spacing[0]))
    c = 30  # grid point x_c = (30 + 1/2) h
    xc = (c + 0.5) * h
    a = np.array([xc - 0.021, 1.12, 30.0, xc + 0.043, 1.15, 30.2, 1.0e4])
    b = a.copy()
    b[0], b[3] = 2 * xc - a[3], 2 * xc - a[0]
    b[1], b[4], b[2], b[5] = a[4], a[1], a[5], a[2]
    b = b.astype(np.float32)
    a = a.astype(np.float32)
    fa, Qa, _, _ = _patch(orc, g, ph, a)
    fb, Qb, _, _ = _patch(orc, g, ph, b)
    # the reflection maps x-index i -> 2c - i; compare on the common support
    xa = np.arange(fa[0], fa[3] + 1)
    for i, xi in enumerate(xa):
        j = 2 * c - xi - fb[0]
        if 0 <= j < Qb.shape[0]:
            # y and t endpoints were swapped, which describes the same segment
            A, B = Qa[i], Qb[j]
            assert A.shape == B.shape
            # reflected endpoints are rounded to binary32: allow that, nothing more
            assert np.max(np.abs(A - B)) < 1e-6 * Qa.max()


def tent_projection(mu, sig, c, h):
    """int N(x; mu, sig) max(0, 1 - |x - c|/h) dx in closed form."""
    F = lambda x: Phi((x - mu) / sig)
    n = lambda x: math.exp(-0.5 * ((x - mu) / sig) ** 2) / (math.sqrt(2 * math.pi) * sig)
    left = ((mu - c + h) * (F(c) - F(c - h)) + sig ** 2 * (n(c - h) - n(c))) / h
    right = ((c + h - mu) * (F(c + h) - F(c)) - sig ** 2 * (n(c) - n(c + h))) / h
    return left + right


def test_tent_projection_closed_form_self_check():
    mu, sig, c, h = 0.013, 0.03, 0.0, 0.044
    ref = integrate.quad(lambda x: math.exp(-0.5 * ((x - mu) / sig) ** 2) / (math.sqrt(2 * math.pi) * sig)
                         * max(0.0, 1 - abs(x - c) / h), c - h, c + h, points=[c], epsrel=1e-13)[0]
    assert abs(tent_projection(mu, sig, c, h) - ref) < 1e-13


def test_effq_converges_to_tent_projection(orc):
    """Q_eff[g] is the per-cell GL estimate of int q * tent_g; as the rule grows it
    converges to the tent projection (closed form for a point charge)."""
    g = grid_at(25.0)
    errs = []
    for n in (2, 4, 8, 16):
        ph = phys_for(g, n_gl=n)
        seg = _point_dep(z=25.0)
        fp, Q, ns, ip = _patch(orc, g, ph, seg)
        tr = orc.transport(ph, seg)
        mu = [0.5 * (float(seg[0]) + float(seg[3])), 0.5 * (float(seg[1]) + float(seg[4])), tr[2]]
        vecs = []
        for a in range(3):
            h = float(np.float32(g.spacing[a]))
            gs = np.arange(fp[a], fp[3 + a] + 1)
            centers = (gs + 0.5) * h if a < 2 else g.origin[2] + gs * h
            vecs.append(np.array([tent_projection(mu[a], tr[4 + a], cc, h) for cc in centers]))
        ref = tr[3] * vecs[0][:, None, None] * vecs[1][None, :, None] * vecs[2][None, None, :]
        # compare away from the window edge where truncation matters
        errs.append(np.max(np.abs(Q - ref)[2:-2, 2:-2, 2:-2]) / ref.max())
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 2e-3 and errs[0] < 5e-2


# ---------------------------------------------------------------------------
# Binning and pixel set
# ---------------------------------------------------------------------------


def test_block_keys_brute_force(orc):
    g = tiny_grid(npix=8, sub=3, nticks=96, h=0.44 / 3)
    ph = phys_for(g)
    blk = W.Blocking((2, 3), 16)
    seg = W.gen_uniform_segments(25, (8 * 0.44, 8 * 0.44), (0.0, 96 * 0.05 * 0.16), seed=5)
    fp, off, _ = orc.footprints(g, ph, seg)
    keys = orc.block_keys(g, blk, fp)
    brute = set()
    for f in fp:
        for x in range(f[0], f[3] + 1):
            for y in range(f[1], f[4] + 1):
                for t in range(f[2], f[5] + 1):
                    brute.add((x // 6, y // 9, t // 16))
    assert sorted(brute) == [tuple(k) for k in keys]


def test_pix_set_brute_force(orc):
    g = tiny_grid(npix=9, sub=3, nticks=64, h=0.44 / 3)
    blk = W.Blocking((2, 2), 16)
    keys = np.array([[0, 0, 1], [3, 2, 0], [4, 4, 3]], np.int32)
    pix = orc.pix_set(g, blk, (3, 5), keys)
    brute = set()
    for bx, by, bt in keys:
        for px in range(9):
            for py in range(9):
                # pixel p receives from charge pixel c iff p - c in [-(K-1)/2, (K-1)/2]
                for cx in range(bx * 2, bx * 2 + 2):
                    for cy in range(by * 2, by * 2 + 2):
                        if abs(px - cx) <= 1 and abs(py - cy) <= 2:
                            brute.add(px * 9 + py)
    assert sorted(brute) == list(pix)


# ---------------------------------------------------------------------------
# Direct convolution
# ---------------------------------------------------------------------------


def _small_event(orc, sub=3, npix=6, nticks=96, n=12, seed=2, kt=24):
    g = tiny_grid(npix=npix, sub=sub, nticks=nticks, h=0.44 / sub)
    ph = phys_for(g)
    seg = W.gen_uniform_segments(n, (npix * 0.44, npix * 0.44), (0.1, nticks * 0.05 * 0.16 - 0.1),
                                 seed=seed)
    fp, off, _ = orc.footprints(g, ph, seg)
    val, _ = orc.effq(g, ph, seg, fp, off)
    return g, ph, seg, fp, off, val


def dense_qeff(g, fp, off, val):
    N = g.nfine
    Q = np.zeros(N)
    for d in range(fp.shape[0]):
        f = fp[d]
        if (f[3:] < f[:3]).any():
            continue
        shape = tuple(int(f[3 + a] - f[a] + 1) for a in range(3))
        Q[f[0]:f[3] + 1, f[1]:f[4] + 1, f[2]:f[5] + 1] += val[off[d]:off[d + 1]].reshape(shape)
    return Q


def test_conv_delta_response_shifts_charge(orc):
    g, ph, seg, fp, off, val = _small_event(orc)
    K, kt = (3, 5), 24
    Q = dense_qeff(g, fp, off, val)
    allpix = np.arange(g.npix[0] * g.npix[1], dtype=np.int32)
    for (kx, ky, jx, jy, tau) in [(1, 2, 0, 0, 0), (0, 4, 2, 1, 7), (2, 0, 1, 2, 23)]:
        R = W.delta_response(K, g.sub, kt, kx, ky, jx, jy, tau)
        wf = orc.waveforms(g, K, kt, R, fp, off, val, allpix).reshape(g.npix[0], g.npix[1], -1)
        # pixel p at tick n + tau receives the charge of sub-pixel j of pixel p - (k - h)
        exp = np.zeros_like(wf)
        dx, dy = kx - 1, ky - 2
        for px in range(g.npix[0]):
            for py in range(g.npix[1]):
                cx, cy = px - dx, py - dy
                if 0 <= cx < g.npix[0] and 0 <= cy < g.npix[1]:
                    exp[px, py, tau:tau + g.nticks] = Q[cx * 3 + jx, cy * 3 + jy, :]
        assert np.max(np.abs(wf - exp)) < 1e-12 * np.abs(Q).max()


def test_conv_matches_numpy_fft(orc):
    """Direct interlaced sum == per-channel FFT convolution (numpy) on a tiny grid."""
    g, ph, seg, fp, off, val = _small_event(orc, n=15)
    K, kt = (3, 5), 24
    R = W.random_symmetric_response(K, g.sub, kt, seed=4).astype(np.float64)
    Q = dense_qeff(g, fp, off, val)
    NP, NT = g.npix, g.nticks
    hx, hy = 1, 2
    F = (NP[0] + K[0] - 1, NP[1] + K[1] - 1, NT + kt - 1)
    Y = np.zeros(F, complex)
    for jx in range(3):
        for jy in range(3):
            Qj = Q[jx::3, jy::3, :]
            Rj = R[:, :, jx, jy, :]
            Y += np.fft.fftn(Qj, F, axes=(0, 1, 2)) * np.fft.fftn(Rj, F, axes=(0, 1, 2))
    full = np.real(np.fft.ifftn(Y))  # full linear conv: output pixel index = charge + kx
    ref = full[hx:hx + NP[0], hy:hy + NP[1], :]
    allpix = np.arange(NP[0] * NP[1], dtype=np.int32)
    wf = orc.waveforms(g, K, kt, R.astype(np.float32), fp, off, val, allpix)
    wf = wf.reshape(NP[0], NP[1], -1)
    assert np.max(np.abs(wf - ref)) < 1e-11 * np.abs(ref).max()


def test_conv_charge_conservation_unit_area_response(orc):
    """With sum_{k,tau} R[k][j][tau] = 1 for every impact j, all charge reappears as
    integrated current when no output falls outside the region."""
    g = tiny_grid(npix=12, sub=10, nticks=400)
    ph = phys_for(g)
    K, kt = (5, 5), 60
    R = W.synthetic_response(K, g.sub, kt)
    seg = W.gen_uniform_segments(6, (1.2, 1.2), (3.0, 3.1), seed=9, xy_origin=(2.0, 2.0))
    fp, off, _ = orc.footprints(g, ph, seg)
    val, _ = orc.effq(g, ph, seg, fp, off)
    allpix = np.arange(144, dtype=np.int32)
    wf = orc.waveforms(g, K, kt, R, fp, off, val, allpix)
    rsum = R.astype(np.float64).sum(axis=(0, 1, 4))
    Q = dense_qeff(g, fp, off, val)
    exp = sum(Q[jx::10, jy::10].sum() * rsum[jx, jy] for jx in range(10) for jy in range(10))
    assert abs(wf.sum() - exp) < 1e-12 * abs(exp)
    assert abs(wf.sum() - val.sum()) < 1e-6 * val.sum()


def test_waveform_points_match_full(orc):
    g, ph, seg, fp, off, val = _small_event(orc, n=10)
    K, kt = (3, 5), 24
    R = W.random_symmetric_response(K, g.sub, kt, seed=4)
    allpix = np.arange(36, dtype=np.int32)
    wf = orc.waveforms(g, K, kt, R, fp, off, val, allpix)
    rng = np.random.default_rng(0)
    pts = np.stack([rng.integers(0, 36, 50), rng.integers(0, g.nticks + kt - 1, 50)], 1)
    got = orc.waveform_points(g, K, kt, R, fp, off, val, pts)
    assert np.max(np.abs(got - wf[pts[:, 0], pts[:, 1]])) < 1e-12 * np.abs(wf).max()


def test_block_outputs_overlap_add_to_global_convolution(orc):
    """Blocking + overlap-add reaches the global direct convolution exactly (Sec.
    III-B): each bin's output at every sample of its output frame, placed at the bin's
    origin and summed over bins (cropped to the region), equals the waveforms."""
    g, ph, seg, fp, off, val = _small_event(orc, n=10, nticks=64)
    K, kt = (3, 5), 24
    R = W.random_symmetric_response(K, g.sub, kt, seed=4)
    blk = W.Blocking((2, 4), 32)
    keys = orc.block_keys(g, blk, fp)
    NP = g.npix
    L = g.nticks + kt - 1
    total = np.zeros((NP[0], NP[1], L))
    box, boy, bot = 2 + K[0] - 1, 4 + K[1] - 1, 32 + kt - 1
    pts = np.array([(qx, qy, t) for qx in range(box) for qy in range(boy) for t in range(bot)])
    for key in keys:
        bv = orc.block_values(g, blk, fp, off, val, key)
        out = orc.block_output_points(g, blk, K, kt, R, bv, pts).reshape(box, boy, bot)
        x0, y0, t0 = key[0] * 2 - 1, key[1] * 4 - 2, key[2] * 32
        for qx in range(box):
            for qy in range(boy):
                px, py = x0 + qx, y0 + qy
                if 0 <= px < NP[0] and 0 <= py < NP[1]:
                    n = min(bot, L - t0)
                    total[px, py, t0:t0 + n] += out[qx, qy, :n]
    allpix = np.arange(NP[0] * NP[1], dtype=np.int32)
    wf = orc.waveforms(g, K, kt, R, fp, off, val, allpix).reshape(NP[0], NP[1], -1)
    assert np.max(np.abs(total - wf)) < 1e-11 * np.abs(wf).max()


def test_bin_members_brute_force(orc):
    """The depositions reaching a bin are those with a footprint cell inside it."""
    g, ph, seg, fp, off, val = _small_event(orc, n=15, nticks=64)
    blk = W.Blocking((2, 4), 32)
    bf = (2 * g.sub[0], 4 * g.sub[1], 32)
    for key in orc.block_keys(g, blk, fp):
        got = set(orc.bin_members(g, blk, fp, key).tolist())
        exp = set()
        for d in range(fp.shape[0]):
            f = fp[d]
            cells = [range(f[a], f[3 + a] + 1) for a in range(3)]
            if any(c // bf[0] == key[0] for c in cells[0]) and \
                    any(c // bf[1] == key[1] for c in cells[1]) and \
                    any(c // bf[2] == key[2] for c in cells[2]):
                exp.add(d)
        assert got == exp


# ---------------------------------------------------------------------------
# Accuracy study of the paper (Sec. IV-B): GL-2 vs grid sampling, against GL-4
# ---------------------------------------------------------------------------


def test_accuracy_study_gl2_beats_grid_sampling(orc):
    g = tiny_grid(npix=8, sub=10, nticks=600)
    K, kt = (5, 5), 60
    R = W.synthetic_response(K, g.sub, kt)
    seg = W.gen_uniform_segments(20, (1.5, 1.5), (0.5, 4.5), seed=21, xy_origin=(1.0, 1.0),
                                 length_range=(0.02, 0.1))
    out = {}
    for n in (2, 4):
        ph = phys_for(g, n_gl=n)
        fp, off, _ = orc.footprints(g, ph, seg)
        val, _ = orc.effq(g, ph, seg, fp, off)
        out[n] = (fp, off, val)
    # grid-point sampling: q at the grid point times the cell volume
    ph = phys_for(g)
    fp, off, _ = out[2][:2] + (None,)
    h = [float(np.float32(s)) for s in g.spacing]
    vs = np.zeros(int(off[-1]))
    for d in range(seg.shape[0]):
        f = fp[d]
        k = off[d]
        for x in range(f[0], f[3] + 1):
            for y in range(f[1], f[4] + 1):
                for t in range(f[2], f[5] + 1):
                    vs[k] = orc.q_seg(ph, seg[d], (x + 0.5) * h[0], (y + 0.5) * h[1], t * h[2]) * \
                        h[0] * h[1] * h[2]
                    k += 1
    out["grid"] = (fp, off, vs)
    allpix = np.arange(64, dtype=np.int32)
    acc = {}
    for key, (fp_, off_, v_) in out.items():
        wf = orc.waveforms(g, K, kt, R, fp_, off_, v_, allpix)
        c = np.cumsum(wf, axis=1)[:, 1::2]  # accumulated charge per pixel, per 100 ns
        acc[key] = np.diff(c, axis=1, prepend=0)
    dev2 = np.max(np.abs(acc[2] - acc[4]))
    devg = np.max(np.abs(acc["grid"] - acc[4]))
    assert dev2 < 0.2 * devg
    assert dev2 < 500.0


# ---------------------------------------------------------------------------
# Host sanitizer build of the oracle
# ---------------------------------------------------------------------------


def test_oracle_under_address_and_ub_sanitizers(orc, tmp_path):
    """oracle.c built with the address and undefined-behaviour sanitizers (no OpenMP)
    runs every entry point on a small event with a point-like deposition, one that
    misses the region and ones cut by the region edges, without a report, and gives
    the regular build's outputs."""
    import shutil
    import struct
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call([gcc, "-std=c11", "-D_DEFAULT_SOURCE", "-O1", "-g", "-ffp-contract=off",
                           "-fno-fast-math", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", exe,
                           os.path.join(here, "oracle.c"), os.path.join(here, "sanitize_main.c"),
                           "-lm"])
    g = tiny_grid(npix=6, sub=3, nticks=96, h=0.44 / 3)
    ph = phys_for(g)
    blk = W.Blocking((2, 4), 32)
    K, kt = (3, 5), 24
    seg = W.gen_uniform_segments(12, (6 * 0.44, 6 * 0.44), (0.1, 96 * 0.05 * 0.16 - 0.1), seed=2)
    seg = np.concatenate([seg, np.array([
        [1.0, 1.1, 0.4, 1.0, 1.1, 0.4, 5e3],           # point-like
        [-3.0, 1.0, 0.3, -2.9, 1.0, 0.31, 5e3],        # outside the region
        [0.01, 2.62, 0.02, 0.05, 2.60, 0.03, 5e3],      # x, y and t edges
    ], np.float32)]).astype(np.float32)
    R = W.random_symmetric_response(K, g.sub, kt, seed=4)
    rng = np.random.default_rng(1)
    pts = np.stack([rng.integers(0, 36, 20), rng.integers(0, 96 + kt - 1, 20)], 1).astype(np.int32)
    og, oph, ob = orc.ogrid(g), orc.ophysics(ph), orc.oblocking(blk)
    with open(tmp_path / "in.bin", "wb") as f:
        f.write(bytes(og) + bytes(oph) + bytes(ob))
        f.write(struct.pack("<iii", K[0], K[1], kt))
        f.write(struct.pack("<q", seg.shape[0]) + seg.tobytes() + R.tobytes())
        f.write(struct.pack("<q", pts.shape[0]) + pts.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe, str(tmp_path / "in.bin"), str(tmp_path / "out.bin")], env=env,
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    buf = (tmp_path / "out.bin").read_bytes()
    pos = 0

    def take(dtype, count):
        nonlocal pos
        a = np.frombuffer(buf, dtype=dtype, count=count, offset=pos)
        pos += a.nbytes
        return a

    n = seg.shape[0]
    nk = int(take(np.int64, 1)[0])
    keys = take(np.int32, 3 * nk).reshape(nk, 3)
    fp = take(np.int32, 6 * n).reshape(n, 6)
    off = take(np.int64, n + 1)
    ip = take(np.int32, n)
    val = take(np.float64, int(off[-1]))
    ns = take(np.float64, n)
    vblk = 2 * 3 * 4 * 3 * 32
    bv = take(np.float64, vblk * nk).reshape(nk, vblk)
    npx = int(take(np.int64, 1)[0])
    take(np.int32, npx)
    wf = take(np.float64, npx * (96 + kt - 1)).reshape(npx, -1)
    po = take(np.float64, pts.shape[0])
    assert pos + 8 * (27 + 16 + 2) == len(buf)
    ref = orc.simulate(g, ph, blk, K, kt, R, seg)
    assert np.array_equal(fp, ref["fp"]) and np.array_equal(off, ref["off"])
    assert np.array_equal(ip, ref["is_point"]) and ip[12] == 1 and off[14] == off[13]
    assert np.array_equal(keys, ref["keys"])
    close = lambda a, b: np.max(np.abs(a - b)) <= 1e-13 * max(np.abs(b).max(), 1e-300)
    assert close(val, ref["val"]) and close(ns, ref["node_sums"])
    allpix = np.arange(36, dtype=np.int32)
    assert close(wf, orc.waveforms(g, K, kt, R, ref["fp"], ref["off"], ref["val"], allpix))
    assert close(po, orc.waveform_points(g, K, kt, R, ref["fp"], ref["off"], ref["val"], pts))
    for k in range(nk):
        assert close(bv[k], orc.block_values(g, blk, ref["fp"], ref["off"], ref["val"],
                                              keys[k]).ravel())

"""GPU tests of the gradients (the transposes of the four calls).

* Each linear stage (overlap-add, convolution, binning) against its forward call:
  <forward(x), y> = <x, transpose(y)> on random x, y (binary64 inner products of the
  binary32 outputs); the forward calls are the ones pinned to the oracle elsewhere.
* The effective-charge gradient and the whole chain against binary64 central finite
  differences of the oracle (a linear loss sum c * output with a fixed smooth weight
  c), perturbing only where the oracle's integer structures (footprints, point/line
  decisions, pixel set) stay the same.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2602_12052_amd import tred
    tred.lib()
    return tred


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def dot(a, b):
    return float(np.dot(np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()))


def grad_cfg(npix=8, sub=3, nticks=300, blk=(2, 2, 64), kpix=(3, 5), kticks=100, fft=(8, 8, 256),
             n=6, seed=21, length=(0.05, 0.3), n_gl=2):
    """Small region whose diffusion widths are above their floor (so the widths depend
    on the drift time and the diffusion constants) and whose segments take the line
    form."""
    h = W.PITCH / sub
    g = W.Grid(origin=(0.0, 0.0, 0.0), spacing=(h, h, W.TICK), npix=(npix, npix), sub=(sub, sub),
               nticks=nticks)
    ph = W.Physics(diff_T=1.2e-3, diff_L=6.0e-4, lifetime=40.0,
                   sigma_min=(0.02 * h, 0.02 * h, 0.02 * W.TICK), n_gl=n_gl)
    zmax = nticks * W.TICK * ph.v_drift
    seg = W.gen_uniform_segments(n, (npix * W.PITCH, npix * W.PITCH), (0.15 * zmax, 0.7 * zmax),
                                 length_range=length, seed=seed)
    return g, ph, W.Blocking(blk[:2], blk[2]), kpix, kticks, fft, seg


def weight(pix, lwf):
    """Smooth fixed loss weight c[pixel id][tick]."""
    pid = np.asarray(pix, np.float64)[:, None]
    t = np.arange(lwf, dtype=np.float64)[None, :]
    return (np.sin(0.37 * pid + 0.011 * t * (1.0 + (pid % 5))) * np.exp(-t / (0.7 * lwf)))


def pipeline(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp=True, batch=8):
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, kpix, sd)
    pl = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), seg.shape[0], val_cap, bcap, pix_cap, fft,
                    mpcp, batch)
    pl.run(sd)
    return pl, sd


# ---------------------------------------------------------------------------
# transposes of the linear stages


CONV_CASES = [
    ("fs8-mpcp", dict(), True),
    ("fs8-plain-sub4", dict(sub=4, nticks=256, blk=(3, 3, 64), kpix=(3, 3), kticks=64), False),
    ("fs8-three-pieces", dict(npix=8, sub=10, nticks=400, blk=(4, 4, 128), kpix=(5, 5), kticks=300,
                              fft=(8, 8, 256), n=8), True),
    ("fs16", dict(npix=8, blk=(4, 4, 64), kpix=(9, 9), kticks=120, fft=(16, 16, 256)), True),
    ("fs24-plain", dict(npix=12, blk=(12, 12, 64), kpix=(11, 11), kticks=120, fft=(24, 24, 256)),
     False),
    ("fs40", dict(npix=32, nticks=1100, blk=(16, 16, 512), kpix=(21, 21), kticks=600,
                  fft=(40, 40, 1024), n=6), True),
    ("fs48", dict(npix=16, blk=(16, 16, 128), kpix=(15, 15), kticks=200, fft=(48, 48, 512)), True),
]


@pytest.mark.parametrize("name,kw,mpcp", CONV_CASES)
def test_conv_transpose(T, name, kw, mpcp):
    """<conv(X), Y> = <X, conv^T(Y)> on the active bins of an event."""
    import torch
    say(f"test_conv_transpose[{name}]")
    g, ph, blk, kpix, kticks, fft, seg = grid_cfg_small(**kw)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    pl, sd = pipeline(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp)
    torch.cuda.synchronize()
    na = min(int(pl.n_active.item()), pl.keys.shape[0])
    assert na > 0
    gen = torch.Generator(device="cuda").manual_seed(5)
    X = torch.randn(pl.blocks.shape, device="cuda", generator=gen)
    Y = torch.randn(pl.out_blocks.shape, device="cuda", generator=gen)
    out = torch.empty_like(pl.out_blocks)
    dX = torch.empty_like(pl.blocks)
    T.tred_block_conv(pl.plan, pl.n_active, X, out)
    T.tred_block_conv_adjoint(pl.plan, pl.n_active, Y, dX)
    torch.cuda.synchronize()
    lhs = dot(out[:na].cpu().numpy(), Y[:na].cpu().numpy())
    rhs = dot(X[:na].cpu().numpy(), dX[:na].cpu().numpy())
    scale = float(torch.linalg.norm(out[:na].double()) * torch.linalg.norm(Y[:na].double()))
    say(f"  {na} bins: <conv X, Y> {lhs:.9e}  <X, conv^T Y> {rhs:.9e}  diff/scale "
        f"{abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * scale


@pytest.mark.parametrize("name,kw,mpcp", [CONV_CASES[0], CONV_CASES[1], CONV_CASES[5]])
def test_conv_adjoint_rows_match_dense(T, name, kw, mpcp):
    """The transposed convolution with row masks writes the marked rows exactly as the
    dense transpose does and leaves the other rows untouched (here NaN)."""
    import torch
    say(f"test_conv_adjoint_rows_match_dense[{name}]")
    g, ph, blk, kpix, kticks, fft, seg = grid_cfg_small(**kw)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    pl, sd = pipeline(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp)
    torch.cuda.synchronize()
    na = min(int(pl.n_active.item()), pl.keys.shape[0])
    assert na > 0 and pl.rows is not None
    gen = torch.Generator(device="cuda").manual_seed(7)
    Y = torch.randn(pl.out_blocks.shape, device="cuda", generator=gen)
    dense = torch.empty_like(pl.blocks)
    masked = torch.full_like(pl.blocks, float("nan"))
    T.tred_block_conv_adjoint(pl.plan, pl.n_active, Y, dense)
    T.tred_block_conv_adjoint_rows(pl.plan, pl.n_active, Y, pl.rows, masked)
    torch.cuda.synchronize()
    nrow = blk.blk_pix[0] * g.sub[0] * blk.blk_pix[1] * g.sub[1]
    bits = pl.rows[:na].cpu().numpy().view(np.uint32)
    marked = ((bits[:, np.arange(nrow) // 32] >> (np.arange(nrow) % 32).astype(np.uint32)) & 1) != 0
    d = dense[:na].cpu().numpy().reshape(na, nrow, blk.blk_ticks)
    m = masked[:na].cpu().numpy().reshape(na, nrow, blk.blk_ticks)
    say(f"  {na} bins, marked rows {marked.mean():.3f}")
    assert np.array_equal(m[marked], d[marked])
    assert np.all(np.isnan(m[~marked]))


def random_pfa_config(seed):
    """A valid small configuration for the transposed convolution (prime-factor spatial
    sizes 8, 16, 24, 40, 48) from a seeded generator."""
    rng = np.random.default_rng(2000 + seed)
    sub = int(rng.integers(2, 6))
    bp = int(rng.integers(2, 17))
    kp = int(rng.choice([3, 5, 7, 9, 11, 15]))
    need = bp + kp - 1
    fits = [f for f in (8, 16, 24, 40, 48) if f >= need and bp <= 2 * (16 if f in (16, 48) else 8)]
    fs = int(fits[int(rng.integers(0, min(2, len(fits))))])
    bt = int(rng.choice([64, 128]))
    ft = int(rng.choice([256, 512]))
    kticks = int(rng.integers(40, min(4 * (ft - bt), 500)))
    return dict(npix=bp * int(rng.integers(2, 4)), sub=sub, nticks=int(rng.integers(3, 6)) * bt,
                blk=(bp, bp, bt), kpix=(kp, kp), kticks=kticks, fft=(fs, fs, ft),
                n=int(rng.integers(5, 20)), seed=seed), bool(rng.integers(0, 2))


@pytest.mark.parametrize("seed", range(8))
def test_conv_transpose_random(T, seed):
    """<conv(X), Y> = <X, conv^T(Y)> on seeded random configurations, and the transpose
    with row masks equal to the dense one on the marked rows."""
    import torch
    kw, mpcp = random_pfa_config(seed)
    say(f"test_conv_transpose_random[{seed}] {kw} mpcp={mpcp}")
    g, ph, blk, kpix, kticks, fft, seg = grid_cfg_small(**kw)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=31 + seed)
    pl, sd = pipeline(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp, batch=3)
    torch.cuda.synchronize()
    na = min(int(pl.n_active.item()), pl.keys.shape[0])
    assert na > 0
    gen = torch.Generator(device="cuda").manual_seed(50 + seed)
    X = torch.randn(pl.blocks.shape, device="cuda", generator=gen)
    Y = torch.randn(pl.out_blocks.shape, device="cuda", generator=gen)
    out = torch.empty_like(pl.out_blocks)
    dX = torch.empty_like(pl.blocks)
    dXr = torch.full_like(pl.blocks, float("nan"))
    T.tred_block_conv(pl.plan, pl.n_active, X, out)
    T.tred_block_conv_adjoint(pl.plan, pl.n_active, Y, dX)
    T.tred_block_conv_adjoint_rows(pl.plan, pl.n_active, Y, pl.rows, dXr)
    torch.cuda.synchronize()
    lhs = dot(out[:na].cpu().numpy(), Y[:na].cpu().numpy())
    rhs = dot(X[:na].cpu().numpy(), dX[:na].cpu().numpy())
    scale = float(torch.linalg.norm(out[:na].double()) * torch.linalg.norm(Y[:na].double()))
    say(f"  {na} bins: diff/scale {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * scale
    nrow = blk.blk_pix[0] * g.sub[0] * blk.blk_pix[1] * g.sub[1]
    bits = pl.rows[:na].cpu().numpy().view(np.uint32)
    marked = ((bits[:, np.arange(nrow) // 32] >> (np.arange(nrow) % 32).astype(np.uint32)) & 1) != 0
    d = dX[:na].cpu().numpy().reshape(na, nrow, blk.blk_ticks)
    m = dXr[:na].cpu().numpy().reshape(na, nrow, blk.blk_ticks)
    assert np.array_equal(m[marked], d[marked])
    assert np.all(np.isnan(m[~marked]))


def grid_cfg_small(npix=6, sub=3, nticks=200, blk=(2, 2, 64), kpix=(3, 5), kticks=100,
                   fft=(8, 8, 256), n=12, seed=1):
    h = W.PITCH / sub
    g = W.Grid(origin=(0.0, 0.0, 0.0), spacing=(h, h, W.TICK), npix=(npix, npix), sub=(sub, sub),
               nticks=nticks)
    ph = W.Physics(sigma_min=(0.5 * h, 0.5 * h, 0.5 * W.TICK))
    zmax = nticks * W.TICK * ph.v_drift
    seg = W.gen_uniform_segments(n, (npix * W.PITCH, npix * W.PITCH), (0.0, zmax), seed=seed)
    return g, ph, W.Blocking(blk[:2], blk[2]), kpix, kticks, fft, seg


def test_scatter_and_bin_transposes(T):
    """<scatter(O), W> = <O, scatter^T(W)> and <bin(V), B> = <V, bin^T(B)>."""
    import torch
    say("test_scatter_and_bin_transposes")
    g, ph, blk, kpix, kticks, fft, seg = grid_cfg_small(n=20, seed=3)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    pl, sd = pipeline(T, g, ph, blk, kpix, kticks, fft, seg, resp)
    torch.cuda.synchronize()
    na = min(int(pl.n_active.item()), pl.keys.shape[0])
    npx = min(int(pl.n_pix.item()), pl.pix.shape[0])
    nval = int(pl.off[-1].item())
    gen = torch.Generator(device="cuda").manual_seed(7)
    # overlap-add
    O = torch.randn(pl.out_blocks.shape, device="cuda", generator=gen)
    Wt = torch.randn(pl.wf.shape, device="cuda", generator=gen)
    wf = torch.empty_like(pl.wf)
    T.tred_scatter_waveforms(pl.plan, pl.keys, pl.n_active, O, pl.pix, pl.n_pix, wf, pl.scat_work)
    dO = torch.empty_like(pl.out_blocks)
    T.tred_scatter_waveforms_adjoint(pl.plan, pl.keys, pl.n_active, pl.pix, pl.n_pix, Wt, dO)
    torch.cuda.synchronize()
    lhs = dot(wf[:npx].cpu().numpy(), Wt[:npx].cpu().numpy())
    rhs = dot(O[:na].cpu().numpy(), dO[:na].cpu().numpy())
    say(f"  overlap-add: {lhs:.9e} vs {rhs:.9e}")
    assert abs(lhs - rhs) <= 1e-5 * float(torch.linalg.norm(wf[:npx].double()) *
                                          torch.linalg.norm(Wt[:npx].double()))
    # binning
    V = torch.randn(pl.val.shape, device="cuda", generator=gen)
    B = torch.randn(pl.blocks.shape, device="cuda", generator=gen)
    keys = torch.empty_like(pl.keys)
    nact = torch.zeros_like(pl.n_active)
    blocks = torch.empty_like(pl.blocks)
    T.tred_block_bin(g, blk, pl.fp, pl.off, V, keys, nact, blocks, pl.bin_work)
    dV = torch.empty_like(pl.val)
    T.tred_block_bin_adjoint(g, blk, pl.fp, pl.off, keys, nact, B, dV, pl.bin_work)
    torch.cuda.synchronize()
    lhs = dot(blocks[:na].cpu().numpy(), B[:na].cpu().numpy())
    rhs = dot(V[:nval].cpu().numpy(), dV[:nval].cpu().numpy())
    say(f"  binning: {lhs:.9e} vs {rhs:.9e}")
    assert abs(lhs - rhs) <= 1e-5 * float(torch.linalg.norm(blocks[:na].double()) *
                                          torch.linalg.norm(B[:na].double()))


# ---------------------------------------------------------------------------
# finite differences of the oracle


def fd_params(orc, g, ph, seg, loss, base_fp, h_pos=2e-4, h_rel=1e-4):
    """Central differences of loss(seg, ph) (binary64, oracle) in every deposition
    parameter and in diff_T, diff_L, lifetime. Perturbations are the binary32 values
    actually represented; a parameter whose perturbation changes the footprints is
    skipped (NaN)."""
    import copy
    n = seg.shape[0]
    g_seg = np.full((n, 7), np.nan)
    for d in range(n):
        for k in range(7):
            step = h_rel * abs(float(seg[d, k])) if k == 6 else h_pos
            sp, sm = seg.copy(), seg.copy()
            sp[d, k] = np.float32(seg[d, k] + step)
            sm[d, k] = np.float32(seg[d, k] - step)
            fpp, _, ipp = orc.footprints(g, ph, sp)
            fpm, _, ipm = orc.footprints(g, ph, sm)
            if not (np.array_equal(fpp, base_fp) and np.array_equal(fpm, base_fp)):
                continue
            g_seg[d, k] = (loss(sp, ph) - loss(sm, ph)) / (float(sp[d, k]) - float(sm[d, k]))
    g_phys = np.full(3, np.nan)
    for i, name in enumerate(("diff_T", "diff_L", "lifetime")):
        v = getattr(ph, name)
        pp, pm = copy.copy(ph), copy.copy(ph)
        setattr(pp, name, float(np.float32(v * (1 + h_rel))))
        setattr(pm, name, float(np.float32(v * (1 - h_rel))))
        fpp, _, _ = orc.footprints(g, pp, seg)
        fpm, _, _ = orc.footprints(g, pm, seg)
        if not (np.array_equal(fpp, base_fp) and np.array_equal(fpm, base_fp)):
            continue
        g_phys[i] = (loss(seg, pp) - loss(seg, pm)) / (getattr(pp, name) - getattr(pm, name))
    return g_seg, g_phys


def compare_grad(name, got, ref, tol):
    ok = np.isfinite(ref)
    assert ok.sum() > 0, f"{name}: no parameter could be differenced"
    err = np.linalg.norm(got[ok] - ref[ok]) / max(np.linalg.norm(ref[ok]), 1e-300)
    say(f"  {name}: {ok.sum()} parameters, rel error vs FD {err:.2e}")
    assert err <= tol, (name, err)


@pytest.mark.parametrize("n_gl", [2, 1, 3, 4])
def test_effq_gradient_vs_finite_differences(T, orc, n_gl):
    """dL/d(depositions, diff_T, diff_L, lifetime) for L = sum c * val (patch values), for
    Gauss-Legendre rules of 1 to 4 points per axis (odd rules have a node at the cell
    centre, which spreads onto its own grid point only)."""
    import torch
    say(f"test_effq_gradient_vs_finite_differences[n_gl={n_gl}]")
    g, ph, blk, kpix, kticks, fft, seg = grad_cfg(n_gl=n_gl)
    fp, off, ip = orc.footprints(g, ph, seg)
    assert not ip.any()
    nval = int(off[-1])
    c = np.cos(0.013 * np.arange(nval)) * (1.0 + 0.5 * np.sin(0.7 * np.arange(nval)))

    def loss(s, p):
        fps, offs, _ = orc.footprints(g, p, s)
        val, _ = orc.effq(g, p, s, fps, offs)
        return float(np.dot(val, c))

    ref_seg, ref_phys = fd_params(orc, g, ph, seg, loss, fp)
    sd = dev(seg)
    fpd = torch.empty((seg.shape[0], 6), dtype=torch.int32, device="cuda")
    offd = torch.empty(seg.shape[0] + 1, dtype=torch.int64, device="cuda")
    T.tred_effq_windows(g, ph, sd, fpd, offd)
    d_seg = torch.empty((seg.shape[0], 7), dtype=torch.float32, device="cuda")
    d_phys = torch.zeros(3, dtype=torch.float64, device="cuda")
    T.tred_effq_adjoint(g, ph, sd, fpd, offd, dev(c.astype(np.float32)), d_seg, d_phys)
    torch.cuda.synchronize()
    got_seg, got_phys = d_seg.cpu().numpy().astype(np.float64), d_phys.cpu().numpy()
    compare_grad("end points", got_seg[:, :6], ref_seg[:, :6], 1e-4)
    compare_grad("charges", got_seg[:, 6], ref_seg[:, 6], 1e-4)
    compare_grad("diff_T, diff_L, lifetime", got_phys, ref_phys, 1e-4)


@pytest.mark.parametrize("name,kw", [
    ("fs8", dict()),
    ("fs24-sub4", dict(npix=12, sub=4, blk=(12, 12, 64), kpix=(11, 11), kticks=120,
                       fft=(24, 24, 256), n=4)),
])
def test_whole_chain_gradient_vs_finite_differences(T, orc, name, kw):
    """Gradient of L = sum c * waveforms through the four transposes (Pipeline.backward)
    against central differences of the oracle's whole path (small regions, where the
    oracle's direct convolution is fast; the larger spatial sizes are covered by the
    transpose identity above)."""
    import torch
    say(f"test_whole_chain_gradient_vs_finite_differences[{name}]")
    g, ph, blk, kpix, kticks, fft, seg = grad_cfg(**kw)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    o = orc.simulate(g, ph, blk, kpix, kticks, resp, seg)
    lwf = g.nticks + kticks - 1
    c = weight(o["pix"], lwf)

    def loss(s, p):
        r = orc.simulate(g, p, blk, kpix, kticks, resp, s)
        if not np.array_equal(r["pix"], o["pix"]):
            return np.nan
        return float(np.sum(r["wf"] * c))

    ref_seg, ref_phys = fd_params(orc, g, ph, seg, loss, o["fp"])
    pl, sd = pipeline(T, g, ph, blk, kpix, kticks, fft, seg, resp)
    torch.cuda.synchronize()
    npx = int(pl.n_pix.item())
    assert np.array_equal(pl.pix[:npx].cpu().numpy(), o["pix"])
    d_wf = torch.zeros_like(pl.wf)
    d_wf[:npx] = dev(c.astype(np.float32))
    d_seg, d_phys = pl.backward(sd, d_wf)
    torch.cuda.synchronize()
    got_seg, got_phys = d_seg.cpu().numpy().astype(np.float64), d_phys.cpu().numpy()
    compare_grad("end points", got_seg[:, :6], ref_seg[:, :6], 1e-4)
    compare_grad("charges", got_seg[:, 6], ref_seg[:, 6], 1e-4)
    compare_grad("diff_T, diff_L, lifetime", got_phys, ref_phys, 1e-4)


def test_autograd_function(T):
    """Simulate.apply gives the same gradient as Pipeline.backward."""
    import torch
    say("test_autograd_function")
    g, ph, blk, kpix, kticks, fft, seg = grad_cfg()
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    pl, sd = pipeline(T, g, ph, blk, kpix, kticks, fft, seg, resp)
    torch.cuda.synchronize()
    npx = int(pl.n_pix.item())
    c = torch.zeros_like(pl.wf)
    c[:npx] = dev(weight(pl.pix[:npx].cpu().numpy(), pl.wf.shape[1]).astype(np.float32))
    x = sd.clone().requires_grad_(True)
    wf = T.Simulate.apply(pl, x)
    (wf * c).sum().backward()
    ref, _ = pl.backward(sd, c)
    torch.cuda.synchronize()
    assert torch.allclose(x.grad, ref, rtol=1e-6, atol=0)


def test_simulate_whole_output_and_capacity(T):
    """Simulate's output is defined on every row: with the waveform buffer pre-filled
    with NaN, a loss over the whole output (rows past n_pix included, with nonzero
    weights) is finite, those rows are zero, and the gradient equals the one of the
    loss over the n_pix live rows. A pipeline whose patch capacity is too small for
    the depositions raises a capacity error instead of returning truncated output."""
    import torch
    say("test_simulate_whole_output_and_capacity")
    g, ph, blk, kpix, kticks, fft, seg = grad_cfg()
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, kpix, sd)
    pl = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), seg.shape[0], val_cap, bcap,
                    pix_cap + 7, fft, True, 8)
    pl.wf.fill_(float("nan"))
    gen = torch.Generator(device="cuda").manual_seed(3)
    c = torch.randn(pl.wf.shape, device="cuda", generator=gen)
    x = sd.clone().requires_grad_(True)
    wf = T.Simulate.apply(pl, x)
    npx = int(pl.n_pix.item())
    assert npx < wf.shape[0]
    assert torch.isfinite(wf).all() and (wf[npx:] == 0).all()
    loss = (wf * c).sum()
    assert torch.isfinite(loss)
    loss.backward()
    c_live = c.clone()
    c_live[npx:] = 0
    ref, _ = pl.backward(sd, c_live)
    torch.cuda.synchronize()
    assert torch.isfinite(x.grad).all()
    assert torch.allclose(x.grad, ref, rtol=1e-6, atol=0)
    small = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), seg.shape[0], val_cap // 2, bcap,
                       pix_cap, fft, True, 8)
    with pytest.raises(T.TredError) as e:
        T.Simulate.apply(small, sd.clone().requires_grad_(True))
    assert e.value.status == T.TRED_ECAPACITY
    with pytest.raises(T.TredError):
        small.results()

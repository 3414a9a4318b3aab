"""GPU tests of the effective charge added straight into the bins (tred_effq_bin,
tred_effq_bin_events): against the two-call path (tred_effq patches, then the
binning's accumulation) on the same inputs, keys, active-bin counts and row masks
must be bit-exact and the blocks equal up to the order of the FP32 additions
(rel-L2 1e-6); the whole fused path against the FP64 oracle within rel-L2 1e-5."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5
ORDER_TOL = 1e-6   # same products, other summation order of the FP32 atomics


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


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


def config(npix=6, sub=3, nticks=200, blk=(2, 2, 64), n=20, seed=1, length=(0.01, 0.1), n_gl=2,
           diff_L=None):
    h = W.PITCH / sub
    g = W.Grid(origin=(0.0, 0.0, 0.0), spacing=(h, h, W.TICK), npix=(npix, npix), sub=(sub, sub),
               nticks=nticks)
    kw = dict(sigma_min=(0.5 * h, 0.5 * h, 0.5 * W.TICK), n_gl=n_gl)
    if diff_L is not None:
        kw["diff_L"] = diff_L
    ph = W.Physics(**kw)
    zmax = nticks * W.TICK * ph.v_drift
    seg = W.gen_uniform_segments(n, (npix * W.PITCH, npix * W.PITCH), (0.0, zmax),
                                 length_range=length, seed=seed)
    return g, ph, W.Blocking(blk[:2], blk[2]), seg


def mask_rows(blocks, rows, na, bt):
    """Values of the marked rows of the first na bins (rows: int32 masks)."""
    out = []
    r = rows[:na].view(np.uint32)
    for s in range(na):
        bits = np.unpackbits(r[s].view(np.uint8), bitorder="little").astype(bool)
        nrow = blocks.shape[1] // bt
        m = bits[:nrow]
        out.append(blocks[s].reshape(nrow, bt)[m])
    return np.concatenate(out) if out else np.zeros((0, bt), np.float32)


def two_paths(T, g, ph, blk, seg, rows_on=True, cap=None, ev=None):
    """(two-call, fused) outputs on the same footprints: keys, n_active, rows (or
    None), blocks of the held bins (marked rows only with masks), charge sums."""
    import torch
    n = seg.shape[0]
    sd = dev(seg)
    fp = torch.empty((n, 6), dtype=torch.int32, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    T.tred_effq_windows(g, ph, sd, fp, off)
    torch.cuda.synchronize()
    ncell = int(off[-1].item())
    val = torch.empty(max(ncell, 1), dtype=torch.float32, device="cuda")
    kst = 3 if ev is None else 4
    eo = None if ev is None else dev(np.asarray(ev, np.int64))
    n_ev = 1 if ev is None else len(ev) - 1
    nbins = T.tred_block_count(g, blk)
    work = torch.empty(4 * nbins * n_ev, dtype=torch.uint8, device="cuda")
    na = torch.zeros(1, dtype=torch.int32, device="cuda")
    # active count for the capacities (n_dep = 0 would not count: a count-only call)
    if ev is None:
        T.tred_block_bin(g, blk, fp, off, val, None, na, None, work)
    else:
        T.tred_block_bin_events(g, blk, eo, fp, off, val, None, na, None, work)
    torch.cuda.synchronize()
    n_act = int(na.item())
    cap = n_act if cap is None else cap
    bf = blk.blk_pix[0] * g.sub[0] * blk.blk_pix[1] * g.sub[1]
    vblk = bf * blk.blk_ticks
    nrw = T.tred_block_row_words(g, blk)
    outs = []
    for fused in (False, True):
        keys = torch.full((max(cap, 1), kst), -7, dtype=torch.int32, device="cuda")
        blocks = torch.full((max(cap, 1), vblk), float("nan"), dtype=torch.float32, device="cuda")
        rows = torch.full((max(cap, 1), nrw), -1, dtype=torch.int32, device="cuda") \
            if rows_on else None
        cs = torch.zeros(1, dtype=torch.float64, device="cuda")
        na = torch.zeros(1, dtype=torch.int32, device="cuda")
        kk = keys[:cap]
        if fused:
            if ev is None:
                T.tred_effq_bin(g, ph, blk, sd, fp, kk, na, blocks, rows, work, cs)
            else:
                T.tred_effq_bin_events(g, ph, blk, eo, sd, fp, kk, na, blocks, rows, work, cs)
        else:
            T.tred_effq(g, ph, sd, fp, off, val, cs)
            if ev is None and rows_on:
                T.tred_block_bin_rows(g, blk, fp, off, val, kk, na, blocks, rows, work)
            elif ev is None:
                T.tred_block_bin(g, blk, fp, off, val, kk, na, blocks, work)
            elif rows_on:
                T.tred_block_bin_events_rows(g, blk, eo, fp, off, val, kk, na, blocks, rows, work)
            else:
                T.tred_block_bin_events(g, blk, eo, fp, off, val, kk, na, blocks, work)
        torch.cuda.synchronize()
        h = min(int(na.item()), cap)
        bl = blocks[:h].cpu().numpy()
        rw = rows[:h].cpu().numpy() if rows_on else None
        vals = mask_rows(bl, rw, h, blk.blk_ticks) if rows_on else bl
        outs.append(dict(keys=keys[:h].cpu().numpy(), n_active=int(na.item()), rows=rw,
                         vals=vals, charge_sum=float(cs.item())))
    return outs


def check_same(a, b):
    assert a["n_active"] == b["n_active"]
    assert np.array_equal(a["keys"], b["keys"])
    if a["rows"] is not None:
        assert np.array_equal(a["rows"], b["rows"])
    assert a["vals"].shape == b["vals"].shape
    assert np.isfinite(b["vals"]).all()
    e = rel_l2(b["vals"], a["vals"])
    scale = max(float(np.abs(a["vals"]).max()), 1e-30)
    m = float(np.abs(b["vals"] - a["vals"]).max()) / scale
    say(f"  {a['n_active']} bins; blocks rel-L2 {e:.2e}, max |diff| / max {m:.2e}; charge sums "
        f"{a['charge_sum']:.9e} / {b['charge_sum']:.9e}")
    assert e < ORDER_TOL and m < 10 * ORDER_TOL
    # node sums: binary32 along a column within a tile, whose size differs between the
    # two kernels (the fused one's tables are wider), binary64 over columns; both are
    # held to the oracle's 1e-6 elsewhere
    assert abs(a["charge_sum"] - b["charge_sum"]) <= 1e-6 * abs(a["charge_sum"])


@pytest.mark.parametrize("name,kw,rows_on", [
    ("sub3-gl2-rows", dict(), True),
    ("sub3-gl1-dense", dict(n_gl=1, seed=2), False),
    ("sub10-gl3-rows", dict(npix=8, sub=10, nticks=400, blk=(4, 4, 128), n=12, seed=3, n_gl=3),
     True),
    ("sub10-gl4-dense", dict(npix=8, sub=10, nticks=400, blk=(4, 4, 128), n=8, seed=4, n_gl=4),
     False),
    # bins of 16 x 16 pixels x 512 ticks over 10 x 10 impacts (the module shape)
    ("module-bins-rows", dict(npix=32, sub=10, nticks=1100, blk=(16, 16, 512), n=25, seed=5),
     True),
    # point-like depositions (segments far shorter than the widths): the point form
    ("points-rows", dict(n=30, seed=6, length=(0.0, 1e-4)), True),
    # long drift-time spreads: footprints spanning several time bins and t tiles
    ("long-t-rows", dict(npix=4, sub=2, nticks=900, blk=(2, 2, 64), n=10, seed=7, diff_L=2e-4),
     True),
])
def test_fused_blocks_match_two_call_path(T, name, kw, rows_on):
    say(f"test_fused_blocks_match_two_call_path[{name}]")
    g, ph, blk, seg = config(**kw)
    a, b = two_paths(T, g, ph, blk, seg, rows_on)
    assert a["n_active"] > 0
    check_same(a, b)


def test_fused_capacity_truncation(T):
    """With fewer bin slots than active bins both paths hold the same first bins and
    drop the cells of the others."""
    say("test_fused_capacity_truncation")
    g, ph, blk, seg = config(npix=8, sub=4, nticks=300, blk=(2, 2, 64), n=25, seed=8)
    full, _ = two_paths(T, g, ph, blk, seg, True)
    cap = full["n_active"] // 2
    a, b = two_paths(T, g, ph, blk, seg, True, cap=cap)
    assert a["keys"].shape[0] == cap and a["n_active"] == full["n_active"]
    check_same(a, b)


def test_fused_events_match_two_call_path(T):
    """Three events (one empty) in one binned tensor, with and without row masks."""
    say("test_fused_events_match_two_call_path")
    g, ph, blk, seg = config(npix=8, sub=4, nticks=300, blk=(2, 2, 64), n=30, seed=9)
    ev = [0, 12, 12, 30]
    for rows_on in (True, False):
        a, b = two_paths(T, g, ph, blk, seg, rows_on, ev=ev)
        assert set(a["keys"][:, 0]) == {0, 2}
        check_same(a, b)


@pytest.mark.parametrize("name,kw,fft,kpix,kticks", [
    ("sub3-two-pieces", dict(n=25, seed=10), (8, 8, 256), (3, 5), 300),
    ("sub10-fs40-four-pieces", dict(npix=32, sub=10, nticks=1100, blk=(16, 16, 512), n=20,
                                    seed=11), (40, 40, 1024), (21, 21), 1800),
])
def test_fused_pipeline_matches_oracle(T, orc, name, kw, fft, kpix, kticks):
    """The whole path with the effective charge added into the bins, against the FP64
    oracle: footprints, keys and pixels bit-exact, waveforms within 1e-5."""
    say(f"test_fused_pipeline_matches_oracle[{name}]")
    g, ph, blk, seg = config(**kw)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, kpix, sd)
    pl = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), seg.shape[0], val_cap, bcap, pix_cap,
                    fft, True, 3, fused=True)
    pl.run(sd)
    r = pl.results()
    assert r["val"] is None
    o = orc.simulate(g, ph, blk, kpix, kticks, resp, seg)
    assert np.array_equal(r["fp"], o["fp"])
    assert np.array_equal(r["off"], o["off"])
    assert np.array_equal(r["keys"], o["keys"])
    assert np.array_equal(r["pix"], o["pix"])
    e = rel_l2(r["wf"], o["wf"])
    say(f"  waveforms rel-L2 {e:.2e}")
    assert e < TOL
    assert abs(r["charge_sum"] - o["node_sums"].sum()) < 1e-6 * abs(o["node_sums"].sum())


def test_fused_batch_pipeline_matches_two_call_path(T):
    """BatchPipeline(fused=True) against the two-call batch on three events: keys and
    pixels bit-exact, waveforms equal up to the summation order."""
    say("test_fused_batch_pipeline_matches_two_call_path")
    g, ph, blk, seg = config(npix=8, sub=4, nticks=300, blk=(2, 2, 64), n=30, seed=12)
    kpix, kticks, fft = (3, 3), 150, (8, 8, 256)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=5)
    ev = np.array([0, 10, 22, 30], np.int64)
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_batch(g, ph, blk, kpix, sd, ev)
    res = []
    for fused in (False, True):
        bp = T.BatchPipeline(g, ph, blk, kpix, kticks, dev(resp), 3, seg.shape[0], val_cap, bcap,
                             pix_cap, fft, True, 4, fused=fused)
        bp.run(sd, dev(ev))
        res.append(bp.results(seg.shape[0]))
    a, b = res
    assert np.array_equal(a["keys"], b["keys"])
    assert np.array_equal(a["pix"], b["pix"])
    e = rel_l2(b["wf"], a["wf"])
    say(f"  {a['n_active']} (event, bin) pairs; waveforms rel-L2 {e:.2e}")
    assert e < ORDER_TOL


def test_fused_pipeline_gradient_matches_two_call_path(T):
    """The gradient of a fixed waveform weighting through a fused pipeline (no patches
    in the forward pass; the transposed calls use a patch-sized gradient buffer of
    val_cap cells) equals the two-call pipeline's: both run the same transposed calls
    on the same footprints, keys and pixels."""
    import torch
    say("test_fused_pipeline_gradient_matches_two_call_path")
    g, ph, blk, seg = config(n=15, seed=13)
    kpix, kticks, fft = (3, 5), 100, (8, 8, 256)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=3)
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, kpix, sd)
    res = []
    for fused in (False, True):
        pl = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), seg.shape[0], val_cap, bcap,
                        pix_cap, fft, True, 4, fused=fused)
        pl.run(sd)
        npx = int(pl.n_pix.item())
        c = np.cos(0.03 * np.arange(pl.wf.numel(), dtype=np.float64)).reshape(pl.wf.shape)
        c[npx:] = 0.0
        d_seg, d_phys = pl.backward(sd, dev(c.astype(np.float32)))
        torch.cuda.synchronize()
        res.append((pl.pix[:npx].cpu().numpy(), d_seg.double().cpu().numpy(),
                    d_phys.cpu().numpy().copy()))
    (pa, ga, fa), (pb, gb, fb) = res
    assert np.array_equal(pa, pb)
    e = rel_l2(gb, ga)
    ep = float(np.max(np.abs(fb - fa) / np.maximum(np.abs(fa), 1e-300)))
    say(f"  d_seg rel-L2 {e:.2e}, d_phys max rel {ep:.2e}")
    assert e < ORDER_TOL and ep < 1e-6


def test_fused_backward_refuses_small_patch_buffer(T):
    """A fused pipeline built with fewer patch cells than the event needs runs its
    forward pass (which keeps no patches) but refuses the gradient instead of
    truncating it."""
    say("test_fused_backward_refuses_small_patch_buffer")
    g, ph, blk, seg = config(n=15, seed=14)
    kpix, kticks, fft = (3, 5), 100, (8, 8, 256)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=3)
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, kpix, sd)
    pl = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), seg.shape[0], val_cap // 2, bcap,
                    pix_cap, fft, True, 4, fused=True)
    pl.run(sd)
    r = pl.results()             # the forward pass needs no patch buffer
    assert r["n_pix"] > 0
    import torch
    with pytest.raises(T.TredError, match="patch cells"):
        pl.backward(sd, torch.zeros_like(pl.wf))

"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs. Integer outputs (footprints, offsets, active-bin keys, pixel sets)
must be bit-exact; floating-point outputs (patches, blocks, waveforms) must be
within rel-L2 1e-5 of the binary64 oracle."""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def small_cfg(npix=6, sub=3, nticks=200, blk=(2, 2, 64), kpix=(3, 5), kticks=100, fft=(8, 8, 256),
              n=20, seed=1, length=(0.01, 0.1)):
    h = W.PITCH / sub
    g = W.Grid(origin=(0.0, 0.0, 0.0), spacing=(h, h, W.TICK), npix=(npix, npix), sub=(sub, sub),
               nticks=nticks)
    ph = W.Physics(sigma_min=(0.5 * h, 0.5 * h, 0.5 * W.TICK))
    zmax = nticks * W.TICK * ph.v_drift
    seg = W.gen_uniform_segments(n, (npix * W.PITCH, npix * W.PITCH), (0.0, zmax),
                                 length_range=length, seed=seed)
    return g, ph, W.Blocking(blk[:2], blk[2]), kpix, kticks, fft, seg


def gpu_path(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp=True, batch=8, block_cap=None,
             check=True, fused=False):
    say(f"  gpu path: npix={g.npix} sub={g.sub} nticks={g.nticks} blk={blk.blk_pix}x{blk.blk_ticks}"
        f" K={kpix}x{kticks} fft={fft} n={seg.shape[0]} mpcp={mpcp} fused={fused}")
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, kpix, sd)
    pl = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), seg.shape[0], val_cap,
                    block_cap or bcap, pix_cap, fft, mpcp, batch, fused=fused)
    pl.run(sd)
    if not check:
        with pytest.raises(T.TredError, match="active bins"):
            pl.results()
    return pl.results(check=check)


def oracle_path(orc, g, ph, blk, kpix, kticks, resp, seg):
    return orc.simulate(g, ph, blk, kpix, kticks, resp, seg)


def compare_all(r, o, tol=TOL):
    assert np.array_equal(r["fp"], o["fp"])
    assert np.array_equal(r["off"], o["off"])
    assert rel_l2(r["val"], o["val"]) < tol, rel_l2(r["val"], o["val"])
    assert r["n_active"] == len(o["keys"])
    assert np.array_equal(r["keys"], o["keys"])
    assert r["n_pix"] == len(o["pix"])
    assert np.array_equal(r["pix"], o["pix"])
    e = rel_l2(r["wf"], o["wf"])
    say(f"  rel-L2 effq {rel_l2(r['val'], o['val']):.2e}  waveforms {e:.2e}")
    assert e < tol
    assert abs(r["charge_sum"] - o["node_sums"].sum()) < 1e-6 * abs(o["node_sums"].sum())


# ---------------------------------------------------------------------------


def test_footprints_bitexact_adversarial(T, orc):
    """Windows and offsets bit-exact on random segments snapped to cell edges +- 1 ulp."""
    import torch
    say("test_footprints_bitexact_adversarial")
    cfg = W.cfg_plain_small()
    g, ph = cfg.grid, cfg.physics
    rng = np.random.default_rng(5)
    n = 20000
    seg = W.gen_segments(cfg).copy()
    seg = np.concatenate([seg] * 20)[:n]
    h = np.float32(g.spacing[0])
    k = rng.integers(0, 320, (n, 2)).astype(np.float32)
    snap = (k * h).astype(np.float32)
    nudge = rng.integers(-2, 3, (n, 2))
    for c in range(2):
        snap[:, c] = np.array([np.nextafter(v, np.float32(np.inf) if s > 0 else np.float32(-np.inf))
                               if s != 0 else v for v, s in zip(snap[:, c], nudge[:, c])], np.float32)
    seg[:, 0] = snap[:, 0]
    seg[:, 1] = snap[:, 1]
    zt = (rng.integers(0, 6250, n) * np.float32(0.05) * np.float32(0.16)).astype(np.float32)
    seg[:, 2] = zt
    fp = torch.empty((n, 6), dtype=torch.int32, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    T.tred_effq_windows(g, ph, dev(seg), fp, off)
    ofp, ooff, _ = orc.footprints(g, ph, seg)
    assert np.array_equal(fp.cpu().numpy(), ofp)
    assert np.array_equal(off.cpu().numpy(), ooff)


@pytest.mark.parametrize("name,kw,mpcp", [
    ("odd-sub-one-piece", dict(), True),
    ("odd-sub-plain", dict(), False),
    ("two-pieces", dict(kticks=300, n=25, seed=2), True),
    ("fs16", dict(npix=8, blk=(4, 4, 64), kpix=(9, 9), kticks=120, fft=(16, 16, 256), seed=3), True),
    ("fs32", dict(npix=16, blk=(8, 8, 64), kpix=(21, 21), kticks=150, fft=(32, 32, 256), n=15,
                  seed=4), True),
    ("fs64", dict(npix=32, nticks=1100, blk=(16, 16, 512), kpix=(21, 21), kticks=600,
                  fft=(64, 64, 1024), n=20, seed=5), True),
    ("fs40-fold", dict(npix=32, nticks=1100, blk=(16, 16, 512), kpix=(21, 21), kticks=600,
                       fft=(40, 40, 1024), n=20, seed=12), True),
    ("fs24-fold-plain", dict(npix=12, blk=(12, 12, 64), kpix=(11, 11), kticks=120,
                             fft=(24, 24, 256), n=15, seed=13), False),
    ("fs48", dict(npix=16, blk=(16, 16, 128), kpix=(15, 15), kticks=200, fft=(48, 48, 512), n=15,
                  seed=14), True),
    ("sub10-three-pieces", dict(npix=8, sub=10, nticks=400, blk=(4, 4, 128), kpix=(5, 5), kticks=300,
                                fft=(8, 8, 256), n=12, seed=6), True),
    ("sub4-even-plain", dict(npix=6, sub=4, nticks=256, blk=(3, 3, 64), kpix=(3, 3), kticks=64,
                             fft=(8, 8, 256), n=15, seed=7), False),
    # blocks wider than half the spatial size: the stage takes all fs inputs per axis
    ("fs8-full-input", dict(npix=10, blk=(5, 5, 64), kpix=(3, 3), kticks=100, fft=(8, 8, 256),
                            n=15, seed=15), True),
    ("fs16-full-input", dict(npix=20, blk=(10, 10, 64), kpix=(5, 5), kticks=120,
                             fft=(16, 16, 256), n=15, seed=16), True),
    # the remaining prime-factor instances: L inputs per axis at sizes 24 and 40, 2 L at 48
    ("fs24-eight-inputs", dict(npix=12, blk=(6, 6, 64), kpix=(11, 11), kticks=120,
                               fft=(24, 24, 256), n=15, seed=17), True),
    ("fs40-eight-inputs", dict(npix=16, blk=(8, 8, 128), kpix=(21, 21), kticks=200,
                               fft=(40, 40, 512), n=15, seed=18), True),
    ("fs48-32-inputs", dict(npix=24, blk=(24, 24, 128), kpix=(15, 15), kticks=200,
                            fft=(48, 48, 512), n=12, seed=19), True),
    # the 36-point spatial stage (9-point sub-DFTs, a pad row in the response spectra):
    # exactly blk + kpix - 1 = 36, sixteen and eight inputs per axis, four pieces, plain
    ("fs36-module-shape", dict(npix=32, nticks=1100, blk=(16, 16, 512), kpix=(21, 21),
                               kticks=1800, fft=(36, 36, 1024), n=20, seed=22), True),
    ("fs36-plain", dict(npix=32, nticks=1100, blk=(16, 16, 512), kpix=(21, 21), kticks=600,
                        fft=(36, 36, 1024), n=20, seed=23), False),
    ("fs36-eight-inputs", dict(npix=16, blk=(8, 8, 128), kpix=(25, 25), kticks=200,
                               fft=(36, 36, 512), n=15, seed=24), True),
    # 12-pixel bins with sixteen inputs per axis at fs 40: the x pass by half rows of
    # pixels meets rows that straddle two time-spectrum groups, and rows past By
    ("fs40-12px-half-rows", dict(npix=24, nticks=700, blk=(12, 12, 512), kpix=(21, 21),
                                 kticks=1800, fft=(40, 40, 1024), n=20, seed=25), True),
])
def test_small_paths_match_oracle(T, orc, name, kw, mpcp):
    say(f"test_small_paths_match_oracle[{name}]")
    g, ph, blk, kpix, kticks, fft, seg = small_cfg(**kw)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    r = gpu_path(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp=mpcp, batch=3)
    o = oracle_path(orc, g, ph, blk, kpix, kticks, resp, seg)
    compare_all(r, o)


def random_config(seed):
    """A valid small configuration drawn from a seeded generator: spatial size one of the
    two smallest kernel sizes that hold block + response - 1 (blocks at most 2 L), time
    size 256 or 512 with at most four response pieces."""
    rng = np.random.default_rng(1000 + seed)
    sub = int(rng.integers(2, 6))
    bp = int(rng.integers(2, 17))
    kp = int(rng.choice([3, 5, 7, 9, 11, 15, 21]))
    need = bp + kp - 1
    fits = [f for f in (8, 16, 24, 32, 40, 48, 64)
            if f >= need and bp <= 2 * (16 if f in (16, 32, 48, 64) else 8)]
    fs = int(fits[int(rng.integers(0, min(2, len(fits))))])
    bt = int(rng.choice([64, 128]))
    ft = int(rng.choice([256, 512]))
    kticks = int(rng.integers(40, min(4 * (ft - bt), 600)))
    npix = bp * int(rng.integers(2, 4))
    nticks = int(rng.integers(3, 6)) * bt
    return dict(npix=npix, sub=sub, nticks=nticks, blk=(bp, bp, bt), kpix=(kp, kp), kticks=kticks,
                fft=(fs, fs, ft), n=int(rng.integers(5, 25)), seed=seed,
                length=(0.01, float(rng.choice([0.1, 0.4])))), bool(rng.integers(0, 2)), \
        int(rng.integers(1, 6))


@pytest.mark.parametrize("seed", range(12))
def test_random_configs_match_oracle(T, orc, seed):
    """Seeded sweep over sub-pixel counts, block and response sizes, FFT sizes, piece
    counts, packing and conv pass sizes (row-mask path) against the oracle."""
    kw, mpcp, batch = random_config(seed)
    say(f"test_random_configs_match_oracle[{seed}] {kw} mpcp={mpcp} batch={batch}")
    g, ph, blk, kpix, kticks, fft, seg = small_cfg(**kw)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11 + seed)
    r = gpu_path(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp=mpcp, batch=batch)
    o = oracle_path(orc, g, ph, blk, kpix, kticks, resp, seg)
    compare_all(r, o)


def test_conv_delta_response_plain(T, orc):
    """A single unit entry in the response copies the charge to one offset (plain path)."""
    say("test_conv_delta_response_plain")
    g, ph, blk, kpix, kticks, fft, seg = small_cfg(n=10, seed=8)
    resp = W.delta_response(kpix, g.sub, kticks, 2, 1, 1, 2, 37)
    r = gpu_path(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp=False)
    o = oracle_path(orc, g, ph, blk, kpix, kticks, resp, seg)
    compare_all(r, o)


def test_mpcp_rejects_asymmetric_response(T):
    say("test_mpcp_rejects_asymmetric_response")
    g, ph, blk, kpix, kticks, fft, seg = small_cfg()
    resp = W.delta_response(kpix, g.sub, kticks, 2, 1, 1, 2, 37)
    plan = T.ConvPlan(g, blk, kpix, kticks, fft, mpcp=True, batch=2)
    with pytest.raises(T.TredError) as e:
        plan.set_response(dev(resp))
    assert e.value.status == T.TRED_EINVAL


def test_plain_small_event_end_to_end(T, orc):
    """1,000 segments in 32x32 pixels, 5x5x200 response, 4x4x128 bins: both packings."""
    say("test_plain_small_event_end_to_end")
    cfg = W.cfg_plain_small()
    seg = W.gen_segments(cfg)
    resp = W.synthetic_response(cfg.kpix, cfg.grid.sub, cfg.kticks)
    o = oracle_path(orc, cfg.grid, cfg.physics, cfg.blocking, cfg.kpix, cfg.kticks, resp, seg)
    for mpcp in (True, False):
        r = gpu_path(T, cfg.grid, cfg.physics, cfg.blocking, cfg.kpix, cfg.kticks, cfg.fft, seg,
                     resp, mpcp=mpcp, batch=512)
        compare_all(r, o)


def test_block_values_match_oracle(T, orc):
    import torch
    say("test_block_values_match_oracle")
    cfg = W.cfg_plain_small()
    g, ph, blk = cfg.grid, cfg.physics, cfg.blocking
    seg = W.gen_segments(cfg, seed=3)
    sd = dev(seg)
    val_cap, bcap, _ = T.size_event(g, ph, blk, cfg.kpix, sd)
    fp = torch.empty((seg.shape[0], 6), dtype=torch.int32, device="cuda")
    off = torch.empty(seg.shape[0] + 1, dtype=torch.int64, device="cuda")
    val = torch.empty(val_cap, dtype=torch.float32, device="cuda")
    T.tred_effq_windows(g, ph, sd, fp, off)
    T.tred_effq(g, ph, sd, fp, off, val)
    keys = torch.empty((bcap, 3), dtype=torch.int32, device="cuda")
    na = torch.zeros(1, dtype=torch.int32, device="cuda")
    vb = blk.blk_pix[0] * 10 * blk.blk_pix[1] * 10 * blk.blk_ticks
    blocks = torch.empty((bcap, vb), dtype=torch.float32, device="cuda")
    work = torch.empty(T.tred_block_bin_workspace(g, blk), dtype=torch.uint8, device="cuda")
    T.tred_block_bin(g, blk, fp, off, val, keys, na, blocks, work)
    torch.cuda.synchronize()
    ofp, ooff, _ = orc.footprints(g, ph, seg)
    oval, _ = orc.effq(g, ph, seg, ofp, ooff)
    okeys = orc.block_keys(g, blk, ofp)
    n = int(na.item())
    assert n == len(okeys)
    assert np.array_equal(keys[:n].cpu().numpy(), okeys)
    rng = np.random.default_rng(0)
    pick = rng.choice(n, size=min(40, n), replace=False)
    got = blocks[torch.from_numpy(pick).cuda()].cpu().numpy()
    ref = np.stack([orc.block_values(g, blk, ofp, ooff, oval, okeys[i]).ravel() for i in pick])
    e = rel_l2(got, ref)
    say(f"  rel-L2 blocks {e:.2e}")
    assert e < TOL


@pytest.mark.parametrize("name,diff_T,n_gl,n", [
    ("gl2-t-tiles", 8.8e-6, 2, 12),
    ("gl2-xy-tiles", 1.0e-4, 2, 8),
    ("gl3-xy-tiles", 1.0e-4, 3, 6),
    ("gl1", 8.8e-6, 1, 12),
    ("gl4", 8.8e-6, 4, 8),
])
def test_effq_tiles_match_oracle(T, orc, name, diff_T, n_gl, n):
    """Patches and node-charge sum of footprints that span several tiles of the
    effective-charge kernel along t (long drift, segments up to 2 mm) and, with wide
    transverse diffusion, along x and y; 1 to 4 Gauss-Legendre points per axis."""
    import torch
    say(f"test_effq_tiles_match_oracle[{name}]")
    npix = 24
    g = W._grid(npix, 6250)
    ph = W.Physics(diff_T=diff_T, n_gl=n_gl)
    seg = W.gen_uniform_segments(n, (npix * W.PITCH, npix * W.PITCH), (30.0, 50.0),
                                 length_range=(0.01, 0.2), seed=21)
    ofp, ooff, _ = orc.footprints(g, ph, seg)
    ext = ofp[:, 3:] - ofp[:, :3] + 1
    assert ext[:, 2].min() > 30
    if diff_T > 1e-5:
        assert ext[:, :2].min() > 24
    oval, ons = orc.effq(g, ph, seg, ofp, ooff)
    sd = dev(seg)
    fp = torch.empty((n, 6), dtype=torch.int32, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    T.tred_effq_windows(g, ph, sd, fp, off)
    val = torch.empty(int(ooff[-1]), dtype=torch.float32, device="cuda")
    cs = torch.zeros(1, dtype=torch.float64, device="cuda")
    T.tred_effq(g, ph, sd, fp, off, val, cs)
    torch.cuda.synchronize()
    assert np.array_equal(fp.cpu().numpy(), ofp)
    assert np.array_equal(off.cpu().numpy(), ooff)
    e = rel_l2(val.cpu().numpy(), oval)
    say(f"  footprint cells {int(ooff[-1])}, rel-L2 patches {e:.2e}")
    assert e < TOL
    assert abs(float(cs.item()) - ons.sum()) < 1e-6 * abs(ons.sum())


@pytest.mark.parametrize("name,kw,mpcp", [
    ("odd-sub", dict(), True),
    ("fs16", dict(npix=8, blk=(4, 4, 64), kpix=(9, 9), kticks=120, fft=(16, 16, 256), seed=3), True),
    ("fs40-plain", dict(npix=32, nticks=1100, blk=(16, 16, 512), kpix=(21, 21), kticks=600,
                        fft=(40, 40, 1024), n=20, seed=12), False),
])
def test_row_masks_match_dense(T, orc, name, kw, mpcp):
    """Binning with row masks marks every row that holds charge, writes those rows as the
    dense binning does, and leaves the others untouched (here NaN); the convolution of
    the masked blocks never reads an unmarked row and equals the dense convolution."""
    import torch
    say(f"test_row_masks_match_dense[{name}]")
    g, ph, blk, kpix, kticks, fft, seg = small_cfg(**kw)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, kpix, sd)
    pl = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), seg.shape[0], val_cap, bcap, pix_cap, fft,
                    mpcp, 3, row_masks=False)
    pl.run(sd, stop_after="effq")
    n = seg.shape[0]
    keys_d = torch.empty_like(pl.keys)
    na_d = torch.zeros(1, dtype=torch.int32, device="cuda")
    blocks_d = torch.empty_like(pl.blocks)
    T.tred_block_bin(g, blk, pl.fp, pl.off, pl.val, keys_d, na_d, blocks_d, pl.bin_work)
    out_d = torch.empty_like(pl.out_blocks)
    T.tred_block_conv(pl.plan, na_d, blocks_d, out_d)
    nrw = T.tred_block_row_words(g, blk)
    keys_r = torch.empty_like(pl.keys)
    na_r = torch.zeros(1, dtype=torch.int32, device="cuda")
    blocks_r = torch.full_like(pl.blocks, float("nan"))
    rows = torch.full((bcap, nrw), -1, dtype=torch.int32, device="cuda")
    T.tred_block_bin_rows(g, blk, pl.fp, pl.off, pl.val, keys_r, na_r, blocks_r, rows, pl.bin_work)
    out_r = torch.full_like(pl.out_blocks, float("nan"))
    T.tred_block_conv_rows(pl.plan, na_r, blocks_r, rows, out_r)
    torch.cuda.synchronize()
    na = int(na_d.item())
    assert na == int(na_r.item()) and na > 0
    assert torch.equal(keys_d[:na], keys_r[:na])
    nrow = blk.blk_pix[0] * g.sub[0] * blk.blk_pix[1] * g.sub[1]
    bits = rows[:na].cpu().numpy().view(np.uint32)
    marked = ((bits[:, np.arange(nrow) // 32] >> (np.arange(nrow) % 32).astype(np.uint32)) & 1) != 0
    bd = blocks_d[:na].cpu().numpy().reshape(na, nrow, blk.blk_ticks)
    br = blocks_r[:na].cpu().numpy().reshape(na, nrow, blk.blk_ticks)
    assert not np.any(bd[~marked])                       # charge only in marked rows
    assert np.all(np.isnan(br[~marked]))                 # unmarked rows not written
    assert np.all(np.isfinite(br[marked]))
    e_b = rel_l2(br[marked], bd[marked])
    od = out_d[:na].cpu().numpy()
    orr = out_r[:na].cpu().numpy()
    assert np.all(np.isfinite(orr))
    e_o = rel_l2(orr, od)
    say(f"  marked rows {marked.mean():.3f}, rel-L2 blocks {e_b:.2e}, outputs {e_o:.2e}")
    assert e_b < 1e-6 and e_o < 1e-6


def test_empty_and_outside_events(T, orc):
    say("test_empty_and_outside_events")
    g, ph, blk, kpix, kticks, fft, seg = small_cfg()
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    # all segments beyond the readout window
    far = seg.copy()
    far[:, 2] += 100.0
    far[:, 5] += 100.0
    r = gpu_path(T, g, ph, blk, kpix, kticks, fft, far, resp)
    assert r["n_active"] == 0 and r["n_pix"] == 0
    assert (r["off"] == 0).all()
    # no segments at all
    r = gpu_path(T, g, ph, blk, kpix, kticks, fft, far[:0], resp)
    assert r["n_active"] == 0 and r["n_pix"] == 0 and r["off"].tolist() == [0]


def test_block_capacity_truncation(T, orc):
    """With fewer block slots than active bins the count reports the full number, the
    binding raises on the overflow, and only the first `cap` bins (in key order) are
    produced."""
    say("test_block_capacity_truncation")
    g, ph, blk, kpix, kticks, fft, seg = small_cfg(n=30, seed=9)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    o = oracle_path(orc, g, ph, blk, kpix, kticks, resp, seg)
    cap = max(1, len(o["keys"]) // 2)
    r = gpu_path(T, g, ph, blk, kpix, kticks, fft, seg, resp, block_cap=cap, check=False)
    assert r["n_active"] == len(o["keys"])
    assert np.array_equal(r["keys"], o["keys"][:cap])
    pix = orc.pix_set(g, blk, kpix, o["keys"][:cap])
    assert np.array_equal(r["pix"], pix)


# ---------------------------------------------------------------------------
# module-scale event at full size: exact integer outputs, sampled floating point
# ---------------------------------------------------------------------------


@pytest.fixture(scope="module", params=["patches", "fused"])
def module_run(T, request):
    """The module event through the two-call path (patches, then binning) and through
    the path bench.py times (effective charge added straight into the bins)."""
    fused = request.param == "fused"
    say(f"module-scale event (1e5 depositions, 256x256 pixels, 21x21x2048 response), "
        f"{request.param}")
    cfg = W.cfg_module()
    seg = W.gen_segments(cfg)
    resp = W.synthetic_response(cfg.kpix, cfg.grid.sub, cfg.kticks)
    # the launch configuration bench.py times: bins per pass from the same scratch budget
    import torch
    _, bcap, _ = T.size_event(cfg.grid, cfg.physics, cfg.blocking, cfg.kpix,
                              torch.from_numpy(seg).cuda())
    batch = T.conv_batch(cfg.grid, cfg.blocking, cfg.kpix, cfg.kticks, cfg.fft, True, bcap,
                         T.DEFAULT_CONV_SCRATCH)
    say(f"  {bcap} active bins, {batch} bins per convolution pass")
    r = gpu_path(T, cfg.grid, cfg.physics, cfg.blocking, cfg.kpix, cfg.kticks, cfg.fft, seg, resp,
                 mpcp=True, batch=batch, fused=fused)
    return cfg, seg, resp, r


def test_module_integer_outputs_bitexact(module_run, orc):
    say("test_module_integer_outputs_bitexact")
    cfg, seg, resp, r = module_run
    ofp, ooff, _ = orc.footprints(cfg.grid, cfg.physics, seg)
    assert np.array_equal(r["fp"], ofp)
    assert np.array_equal(r["off"], ooff)
    okeys = orc.block_keys(cfg.grid, cfg.blocking, ofp)
    assert r["n_active"] == len(okeys)
    assert np.array_equal(r["keys"], okeys)
    pix = orc.pix_set(cfg.grid, cfg.blocking, cfg.kpix, okeys)
    assert np.array_equal(r["pix"], pix)
    say(f"  active bins {len(okeys)} of {16 * 16 * 13}, pixels {len(pix)}")


def test_module_sampled_patches(module_run, orc):
    say("test_module_sampled_patches")
    cfg, seg, resp, r = module_run
    if r["val"] is None:
        pytest.skip("the fused path keeps no patches (its bins are checked by test_gpu_fused)")
    rng = np.random.default_rng(1)
    pick = np.sort(rng.choice(seg.shape[0], 300, replace=False))
    fp, off = r["fp"], r["off"]
    got, ref = [], []
    for d in pick:
        pv, _ = orc.effq_patch(cfg.grid, cfg.physics, seg[d], fp[d])
        ref.append(pv.ravel())
        got.append(r["val"][off[d]:off[d + 1]])
    e = rel_l2(np.concatenate(got), np.concatenate(ref))
    say(f"  rel-L2 sampled patches {e:.2e}")
    assert e < TOL


def test_module_sampled_waveforms(module_run, orc):
    """Waveform samples at the collection peak of pixels under sampled depositions."""
    say("test_module_sampled_waveforms")
    cfg, seg, resp, r = module_run
    g = cfg.grid
    rng = np.random.default_rng(2)
    ofp, ooff, _ = orc.footprints(g, cfg.physics, seg)
    pts = []
    for d in rng.choice(seg.shape[0], 6, replace=False):
        px = int(0.5 * (seg[d, 0] + seg[d, 3]) / W.PITCH)
        py = int(0.5 * (seg[d, 1] + seg[d, 4]) / W.PITCH)
        t0 = int(0.5 * (seg[d, 2] + seg[d, 5]) / cfg.physics.v_drift / W.TICK)
        for dt in (int(0.9 * cfg.kticks) - 3, int(0.9 * cfg.kticks), int(0.5 * cfg.kticks)):
            if 0 <= px < g.npix[0] and 0 <= py < g.npix[1] and t0 + dt < g.nticks + cfg.kticks - 1:
                pts.append((px, py, t0 + dt))
    pts = np.array(pts)
    near = orc.select_near(ofp, g.sub, cfg.kpix, cfg.kticks, pts)
    say(f"  {len(pts)} samples, {len(near)} contributing depositions")
    sub_fp = ofp[near]
    vol = np.prod(np.maximum(sub_fp[:, 3:] - sub_fp[:, :3] + 1, 0), axis=1)
    sub_off = np.concatenate([[0], np.cumsum(vol)]).astype(np.int64)
    sval, _ = orc.effq(g, cfg.physics, seg[near], sub_fp, sub_off)
    ids = pts[:, 0] * g.npix[1] + pts[:, 1]
    ref = orc.waveform_points(g, cfg.kpix, cfg.kticks, resp, sub_fp, sub_off, sval,
                              np.stack([ids, pts[:, 2]], 1))
    slot = np.searchsorted(r["pix"], ids)
    assert (r["pix"][slot] == ids).all()
    got = r["wf"][slot, pts[:, 2]]
    e = rel_l2(got, ref)
    say(f"  rel-L2 sampled waveforms {e:.2e} (|ref| max {np.abs(ref).max():.3e})")
    assert e < TOL


def test_module_whole_waveforms(module_run, orc):
    """Whole waveforms (all nticks + Kt - 1 = 8,297 ticks) of 16 pixels of the module
    event against the oracle's direct sum over every deposition that reaches them:
    four region-edge pixels, four in the output footprint of the last active bin (the
    last key, so the tail workgroup of the paired spatial stage), four holding charge
    in the partial last time bin (ticks 6,144-6,249) and four drawn at random. Every
    pixel holds charge directly (a footprint covers it); pixels whose oracle sum
    would exceed about 1.5e6 reaching cells (3e6 for the late ones) are passed over
    to bound the oracle's time."""
    say("test_module_whole_waveforms")
    cfg, seg, resp, r = module_run
    g, blk = cfg.grid, cfg.blocking
    ofp, ooff, _ = orc.footprints(g, cfg.physics, seg)
    pix = r["pix"]
    npy = g.npix[1]
    L = g.nticks + cfg.kticks - 1
    hx, hy = (cfg.kpix[0] - 1) // 2, (cfg.kpix[1] - 1) // 2
    vol = np.prod(np.maximum(ofp[:, 3:] - ofp[:, :3] + 1, 0), axis=1)
    px0, px1 = ofp[:, 0] // g.sub[0], ofp[:, 3] // g.sub[0]
    py0, py1 = ofp[:, 1] // g.sub[1], ofp[:, 4] // g.sub[1]
    direct = np.zeros(g.npix, bool)
    late = np.zeros(g.npix, bool)
    last_bin = g.nticks // blk.blk_ticks * blk.blk_ticks
    for d in np.nonzero(vol > 0)[0]:
        direct[px0[d]:px1[d] + 1, py0[d]:py1[d] + 1] = True
        if ofp[d, 5] >= last_bin:
            late[px0[d]:px1[d] + 1, py0[d]:py1[d] + 1] = True
    px, py = pix // npy, pix % npy

    def cost(i):
        x, y = px[i], py[i]
        m = (px0 <= x + hx) & (px1 >= x - hx) & (py0 <= y + hy) & (py1 >= y - hy)
        return int(vol[m].sum())

    rng = np.random.default_rng(4)
    sel = []

    def pick(cands, k, cap=1.5e6):
        got = 0
        for i in rng.permutation(cands):
            if got == k:
                break
            if i in sel or not direct[px[i], py[i]] or cost(i) > cap:
                continue
            sel.append(int(i))
            got += 1
        assert got == k

    pick(np.nonzero((px == 0) | (py == 0) | (px == g.npix[0] - 1) | (py == npy - 1))[0], 4)
    kb = r["keys"][-1]
    x0, x1 = kb[0] * blk.blk_pix[0] - hx, kb[0] * blk.blk_pix[0] + blk.blk_pix[0] - 1 + hx
    y0, y1 = kb[1] * blk.blk_pix[1] - hy, kb[1] * blk.blk_pix[1] + blk.blk_pix[1] - 1 + hy
    pick(np.nonzero((px >= x0) & (px <= x1) & (py >= y0) & (py <= y1))[0], 4)
    pick(np.nonzero(late[px, py])[0], 4, cap=3e6)
    pick(np.arange(len(pix)), 4)
    ids = pix[sel]
    near = orc.select_near(ofp, g.sub, cfg.kpix, L,
                           np.stack([ids // npy, ids % npy, np.full(len(ids), L - 1)], 1))
    sfp = ofp[near]
    svol = np.prod(np.maximum(sfp[:, 3:] - sfp[:, :3] + 1, 0), axis=1)
    soff = np.concatenate([[0], np.cumsum(svol)]).astype(np.int64)
    sval, _ = orc.effq(g, cfg.physics, seg[near], sfp, soff)
    ref = orc.waveforms(g, cfg.kpix, cfg.kticks, resp, sfp, soff, sval, ids)
    got = r["wf"][sel]
    assert got.shape == ref.shape == (16, L)
    per = [rel_l2(got[i], ref[i]) for i in range(16)]
    say(f"  {len(near)} depositions reach the 16 pixels; per-pixel rel-L2 "
        + " ".join(f"{e:.1e}" for e in per))
    for name, rows in (("region edge", slice(0, 4)), ("last bin", slice(4, 8)),
                       ("late ticks", slice(8, 12)), ("random", slice(12, 16))):
        e = rel_l2(got[rows], ref[rows])
        say(f"  {name}: rel-L2 {e:.2e}")
        assert e < TOL, name
    e_late = rel_l2(got[8:12, last_bin:], ref[8:12, last_bin:])
    say(f"  ticks >= {last_bin} of the late pixels: rel-L2 {e_late:.2e}")
    assert e_late < TOL
    assert rel_l2(got, ref) < TOL

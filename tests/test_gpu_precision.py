"""GPU parity of the block-direct convolution on BF16 matrix cores against the FP64
oracle, for both operand forms: the hi/lo split (three products, about 16
significant bits per product) and plain BF16 (8 bits). The tolerances are the
targets of the precision study: rel-L2 <= 1e-5 (split) and <= 3e-3 (plain)."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = {True: 1e-5, False: 3e-3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


def max_abs_per_pixel(x, ref):
    """Largest |error| over each pixel's waveform, relative to that waveform's peak."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    peak = np.maximum(np.abs(ref).max(axis=1), 1e-300)
    return float((np.abs(x - ref).max(axis=1) / peak).max())


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


def direct_path(T, g, ph, blk, kpix, kticks, seg, resp, split, batch=16):
    """effq -> binning -> block-direct convolution -> overlap-add, all on the GPU."""
    import torch
    say(f"  direct path: npix={g.npix} sub={g.sub} blk={blk.blk_pix}x{blk.blk_ticks} "
        f"K={kpix}x{kticks} n={seg.shape[0]} split={split}")
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, kpix, sd)
    # the FFT pipeline's buffers and plan give effq, binning and the scatter geometry
    pl = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), seg.shape[0], val_cap, bcap, pix_cap,
                    None, False, 4, row_masks=False)
    pl.run(sd, stop_after="bin")
    dp = T.DirectPlan(g, blk, kpix, kticks, split=split, batch=batch)
    dp.set_response(dev(resp))
    pl.out_blocks.fill_(np.nan)
    T.tred_block_conv_direct(dp, pl.n_active, pl.blocks, pl.out_blocks)
    T.tred_scatter_waveforms(pl.plan, pl.keys, pl.n_active, pl.out_blocks, pl.pix, pl.n_pix,
                             pl.wf, pl.scat_work)
    torch.cuda.synchronize()
    return pl.results()


@pytest.mark.parametrize("split", [True, False])
@pytest.mark.parametrize("name,kw", [
    ("odd-sub", dict()),
    ("sub10", dict(npix=8, sub=10, nticks=300, blk=(4, 4, 128), kpix=(5, 5), kticks=200, n=12,
                   seed=6)),
    ("wide-K-long-bins", dict(npix=12, sub=4, nticks=700, blk=(6, 6, 256), kpix=(9, 7),
                              kticks=300, n=10, seed=13)),
])
def test_direct_small_paths_match_oracle(T, orc, name, kw, split):
    from test_gpu_parity import small_cfg
    say(f"test_direct_small_paths_match_oracle[{name}, split={split}]")
    g, ph, blk, kpix, kticks, fft, seg = small_cfg(**kw)
    # no symmetry needed by the direct form: a generic random response
    rng = np.random.default_rng(21)
    resp = rng.standard_normal((kpix[0], kpix[1], g.sub[0], g.sub[1], kticks)).astype(np.float32)
    r = direct_path(T, g, ph, blk, kpix, kticks, seg, resp, split, batch=3)
    o = orc.simulate(g, ph, blk, kpix, kticks, resp, seg)
    assert np.array_equal(r["keys"], o["keys"])
    assert np.array_equal(r["pix"], o["pix"])
    e = rel_l2(r["wf"], o["wf"])
    m = max_abs_per_pixel(r["wf"], o["wf"])
    say(f"  rel-L2 {e:.2e}, max-abs per pixel waveform / peak {m:.2e}")
    assert e < TOL[split]


@pytest.mark.parametrize("split", [True, False])
def test_direct_plain_small_event(T, orc, split):
    """1,000 segments in 32x32 pixels, 5x5x200 synthetic response, 4x4x128 bins."""
    say(f"test_direct_plain_small_event[split={split}]")
    cfg = W.cfg_plain_small()
    seg = W.gen_segments(cfg)
    resp = W.synthetic_response(cfg.kpix, cfg.grid.sub, cfg.kticks)
    r = direct_path(T, cfg.grid, cfg.physics, cfg.blocking, cfg.kpix, cfg.kticks, seg, resp, split,
                    batch=512)
    o = orc.simulate(cfg.grid, cfg.physics, cfg.blocking, cfg.kpix, cfg.kticks, resp, seg)
    assert np.array_equal(r["pix"], o["pix"])
    e = rel_l2(r["wf"], o["wf"])
    m = max_abs_per_pixel(r["wf"], o["wf"])
    say(f"  rel-L2 {e:.2e}, max-abs per pixel waveform / peak {m:.2e}")
    assert e < TOL[split]


def test_direct_module_sampled_bins(T, orc):
    """Module-scale event: sampled bins through the direct form (both operand forms)
    against the FP64 oracle at sampled output points of each bin, and against the FP32
    FFT path over the bins' whole outputs."""
    import torch
    say("test_direct_module_sampled_bins")
    cfg = W.cfg_module()
    g, ph, blk = cfg.grid, cfg.physics, cfg.blocking
    seg = W.gen_segments(cfg)
    resp = W.synthetic_response(cfg.kpix, g.sub, cfg.kticks)
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, cfg.kpix, sd)
    pl = T.Pipeline(g, ph, blk, cfg.kpix, cfg.kticks, dev(resp), seg.shape[0], val_cap, bcap,
                    pix_cap, cfg.fft, True, 8, row_masks=False)
    pl.run(sd, stop_after="bin")
    torch.cuda.synchronize()
    na = int(pl.n_active.item())
    keys = pl.keys[:na].cpu().numpy()
    fp, off = pl.fp.cpu().numpy(), pl.off.cpu().numpy()
    # bins reached by few depositions keep the FP64 check short
    nmem = np.array([len(orc.bin_members(g, blk, fp, k)) for k in keys])
    rng = np.random.default_rng(3)
    cand = np.nonzero((nmem > 0) & (nmem <= np.percentile(nmem, 30)))[0]
    pick = np.sort(rng.choice(cand, 3, replace=False))
    say(f"  bins {pick.tolist()} with {nmem[pick].tolist()} depositions")
    sub_blocks = pl.blocks[torch.from_numpy(pick).cuda()].contiguous()
    nsub = torch.tensor([len(pick)], dtype=torch.int32, device="cuda")
    vout = pl.out_blocks.shape[1]
    fft_out = torch.empty((len(pick), vout), dtype=torch.float32, device="cuda")
    T.tred_block_conv(pl.plan, nsub, sub_blocks, fft_out)
    res = {}
    for split in (True, False):
        dp = T.DirectPlan(g, blk, cfg.kpix, cfg.kticks, split=split, batch=len(pick))
        dp.set_response(dev(resp))
        out = torch.empty((len(pick), vout), dtype=torch.float32, device="cuda")
        T.tred_block_conv_direct(dp, nsub, sub_blocks, out)
        res[split] = out.cpu().numpy()
        del dp
    fo = fft_out.cpu().numpy()
    box, boy, bot = pl.plan.out_shape
    pts = np.stack([rng.integers(0, box, 40), rng.integers(0, boy, 40),
                    rng.integers(0, bot, 40)], 1)
    # concentrate half the samples near each bin's charge peak (where the signal is)
    for i, b in enumerate(pick):
        mem = orc.bin_members(g, blk, fp, keys[b])
        sub_fp = fp[mem]
        vol = np.prod(np.maximum(sub_fp[:, 3:] - sub_fp[:, :3] + 1, 0), axis=1)
        sub_off = np.concatenate([[0], np.cumsum(vol)]).astype(np.int64)
        sval, _ = orc.effq(g, ph, seg[mem], sub_fp, sub_off)
        bv = orc.block_values(g, blk, sub_fp, sub_off, sval, keys[b])
        o3 = fo[i].reshape(box, boy, bot)
        pk = np.unravel_index(np.argmax(np.abs(o3)), o3.shape)
        near = np.stack([np.clip(pk[0] + rng.integers(-2, 3, 20), 0, box - 1),
                         np.clip(pk[1] + rng.integers(-2, 3, 20), 0, boy - 1),
                         np.clip(pk[2] + rng.integers(-60, 60, 20), 0, bot - 1)], 1)
        P = np.concatenate([pts, near])
        ref = orc.block_output_points(g, blk, cfg.kpix, cfg.kticks, resp, bv, P)
        idx = (P[:, 0] * boy + P[:, 1]) * bot + P[:, 2]
        e_fft = rel_l2(fo[i][idx], ref)
        msg = f"  bin {b}: FFT FP32 rel-L2 {e_fft:.2e}"
        assert e_fft < 1e-5
        for split in (True, False):
            e = rel_l2(res[split][i][idx], ref)
            e_vs_fft = rel_l2(res[split][i], fo[i])
            msg += f" | {'split' if split else 'bf16'} vs oracle {e:.2e}, vs FFT (whole bin) {e_vs_fft:.2e}"
            assert e < TOL[split]
            assert e_vs_fft < TOL[split]
        say(msg)

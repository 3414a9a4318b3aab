"""GPU parity on the cases the smaller sweeps do not reach, against the FP64 oracle.

* Point-like depositions (Sec. II-C, short track segments): an event where a third of
  the segments take the point form, and segments one float32 step on either side of
  the switch (0.1 sigma) on each axis and in both directions; the decision is taken in
  the same binary32 chain on both sides, so it must agree exactly: the two forms differ
  by about 2e-4 (rel-L2) at the threshold, well above the 1e-5 parity bar.
* The spatial-stage instance of the module-scale event (fs 40, 16 inputs per axis,
  two bins per workgroup, four response pieces) with row masks, in full: 16x16-pixel x
  512-tick bins, a 21x21 response of 1,800 ticks (four pieces of a 1,024-point time
  FFT), an odd number of active bins (one workgroup holds a single bin), a partial
  last time bin and charge at the region edges; whole waveforms against the oracle.
* The gradient at the differentiation workload's shapes (fs 40, four pieces, 21x21 x
  2,048 response, 128x128 pixels) against central differences of the oracle.
* The effective-charge gradient on a set with point-like depositions.
* The 64-event batch as the benchmark runs it (chunks through one BatchPipeline):
  per-event bins and pixels bit-exact against the oracle, and sampled waveform points
  of the smallest events against it.
"""
import copy
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


def small_grid(npix=6, sub=3, nticks=200):
    h = W.PITCH / sub
    g = W.Grid(origin=(0.0, 0.0, 0.0), spacing=(h, h, W.TICK), npix=(npix, npix), sub=(sub, sub),
               nticks=nticks)
    return g, W.Physics(sigma_min=(0.5 * h, 0.5 * h, 0.5 * W.TICK))


def threshold_pair(orc, g, ph, base, axis, sign):
    """Two segments that differ only in end-point coordinate `axis`, by one float32
    step: the first takes the point form, the second the line form (the oracle's
    binary32 decision). The segment starts as a point at `base` and grows along
    `axis` in direction `sign`."""
    s = np.asarray(base, np.float32).copy()
    s[3:6] = s[0:3]

    def is_point(v):
        t = s.copy()
        t[3 + axis] = v
        return bool(orc.footprints(g, ph, t[None])[2][0])

    x0 = np.float32(s[axis])
    step = np.float32(1e-6)
    far = np.float32(x0 + sign * step)
    while is_point(far):
        step = np.float32(2 * step)
        far = np.float32(x0 + sign * step)
    # bisection over the float32 values between x0 (point) and far (line)
    lo, hi = x0, far
    while True:
        mid = np.float32(0.5 * (np.float64(lo) + np.float64(hi)))
        if mid == lo or mid == hi:
            break
        if is_point(mid):
            lo = mid
        else:
            hi = mid
    assert np.nextafter(lo, np.float32(sign * np.inf)) == hi
    p, l = s.copy(), s.copy()
    p[3 + axis], l[3 + axis] = lo, hi
    return p, l


def point_event(orc, g, ph, seed=1):
    """12 line segments, 12 short (point-like) segments and 12 at the switch."""
    ext = (g.npix[0] * W.PITCH, g.npix[1] * W.PITCH)
    zmax = g.nticks * W.TICK * ph.v_drift
    a = W.gen_uniform_segments(12, ext, (0.0, zmax), length_range=(0.01, 0.1), seed=seed)
    b = W.gen_uniform_segments(12, ext, (0.0, zmax), length_range=(1e-5, 4e-4), seed=seed + 1)
    rng = np.random.default_rng(seed + 2)
    thr = []
    for axis in range(3):
        for sign in (1, -1):
            base = [rng.uniform(0.3, ext[0] - 0.3), rng.uniform(0.3, ext[1] - 0.3),
                    rng.uniform(0.2 * zmax, 0.8 * zmax), 0, 0, 0, rng.uniform(1e4, 4e4)]
            thr.extend(threshold_pair(orc, g, ph, base, axis, sign))
    return np.concatenate([a, b, np.array(thr, np.float32)]).astype(np.float32), 24


def test_point_like_event_matches_oracle(T, orc):
    """A third of the segments point-like plus 12 at the switch: footprints, offsets,
    bins and pixels bit-exact; patches and waveforms within 1e-5; each switch segment's
    patch within 2e-5 of the oracle's (the other form is 2e-4 away)."""
    from test_gpu_parity import compare_all, gpu_path
    say("test_point_like_event_matches_oracle")
    g, ph = small_grid()
    seg, i_thr = point_event(orc, g, ph)
    blk, kpix, kticks, fft = W.Blocking((2, 2), 64), (3, 5), 100, (8, 8, 256)
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    o = orc.simulate(g, ph, blk, kpix, kticks, resp, seg)
    ip = o["is_point"]
    say(f"  {len(seg)} segments, {int(ip.sum())} point-like; switch pairs "
        f"{ip[i_thr:].tolist()}")
    assert ip.sum() >= len(seg) // 3
    assert ip[i_thr::2].all() and not ip[i_thr + 1::2].any()
    r = gpu_path(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp=True, batch=3)
    compare_all(r, o)
    worst = 0.0
    for d in range(i_thr, len(seg)):
        a, b = o["off"][d], o["off"][d + 1]
        worst = max(worst, rel_l2(r["val"][a:b], o["val"][a:b]))
    say(f"  switch segments: worst patch rel-L2 {worst:.2e}")
    assert worst < 2e-5
    # the two forms are told apart at this tolerance
    for d in range(i_thr, len(seg), 2):
        p, l = seg[d], seg[d + 1]
        vp, _ = orc.effq_patch(g, ph, p, o["fp"][d])
        vl, _ = orc.effq_patch(g, ph, l, o["fp"][d])   # same box: the footprints agree
        assert np.array_equal(o["fp"][d], o["fp"][d + 1])
        assert rel_l2(vl, vp) > 5e-5


def test_effq_gradient_with_point_depositions(T, orc):
    """dL/d(depositions, diff_T, diff_L, lifetime), L = sum c * patch values, on a set of
    line and point-like segments (the point form's transpose) against central
    differences of the oracle that keep every footprint and every form."""
    import torch
    from test_gpu_transpose import compare_grad, grad_cfg
    say("test_effq_gradient_with_point_depositions")
    g, ph, blk, kpix, kticks, fft, seg_l = grad_cfg(n=4)
    ext = (g.npix[0] * W.PITCH, g.npix[1] * W.PITCH)
    zmax = g.nticks * W.TICK * ph.v_drift
    seg_p = W.gen_uniform_segments(4, ext, (0.15 * zmax, 0.7 * zmax), length_range=(2e-4, 2e-3),
                                   seed=77)
    seg = np.concatenate([seg_l, seg_p]).astype(np.float32)
    fp, off, ip = orc.footprints(g, ph, seg)
    say(f"  point-like {ip.tolist()}")
    assert ip[4:].all() and not ip[:4].any()
    nval = int(off[-1])
    c = np.cos(0.013 * np.arange(nval)) * (1.0 + 0.5 * np.sin(0.7 * np.arange(nval)))

    def loss(s, p):
        fps, offs, ips = orc.footprints(g, p, s)
        if not (np.array_equal(fps, fp) and np.array_equal(ips, ip)):
            return np.nan
        val, _ = orc.effq(g, p, s, fps, offs)
        return float(np.dot(val, c))

    n = seg.shape[0]
    ref_seg = np.full((n, 7), np.nan)
    for d in range(n):
        for k in range(7):
            step = 1e-4 * abs(float(seg[d, k])) if k == 6 else 2e-4
            sp, sm = seg.copy(), seg.copy()
            sp[d, k] = np.float32(seg[d, k] + step)
            sm[d, k] = np.float32(seg[d, k] - step)
            ref_seg[d, k] = (loss(sp, ph) - loss(sm, ph)) / (float(sp[d, k]) - float(sm[d, k]))
    ref_phys = np.full(3, np.nan)
    for i, name in enumerate(("diff_T", "diff_L", "lifetime")):
        v = getattr(ph, name)
        pp, pm = copy.copy(ph), copy.copy(ph)
        setattr(pp, name, float(np.float32(v * (1 + 1e-4))))
        setattr(pm, name, float(np.float32(v * (1 - 1e-4))))
        ref_phys[i] = (loss(seg, pp) - loss(seg, pm)) / (getattr(pp, name) - getattr(pm, name))
    sd = dev(seg)
    fpd = torch.empty((n, 6), dtype=torch.int32, device="cuda")
    offd = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    T.tred_effq_windows(g, ph, sd, fpd, offd)
    d_seg = torch.empty((n, 7), dtype=torch.float32, device="cuda")
    d_phys = torch.zeros(3, dtype=torch.float64, device="cuda")
    T.tred_effq_adjoint(g, ph, sd, fpd, offd, dev(c.astype(np.float32)), d_seg, d_phys)
    torch.cuda.synchronize()
    got_seg, got_phys = d_seg.cpu().numpy().astype(np.float64), d_phys.cpu().numpy()
    compare_grad("point-like end points", got_seg[4:, :6], ref_seg[4:, :6], 1e-4)
    compare_grad("point-like charges", got_seg[4:, 6], ref_seg[4:, 6], 1e-4)
    compare_grad("line end points", got_seg[:4, :6], ref_seg[:4, :6], 1e-4)
    compare_grad("diff_T, diff_L, lifetime", got_phys, ref_phys, 1e-4)


# ---------------------------------------------------------------------------
# the module-scale spatial-stage instance, in full


def fs40_event(g, ph, n=15, seed=7):
    """n random segments plus five of 3e4 electrons placed at the four region edges and
    in the last (partial) time bin."""
    ext = (g.npix[0] * W.PITCH, g.npix[1] * W.PITCH)
    zmax = g.nticks * W.TICK * ph.v_drift
    seg = W.gen_uniform_segments(n, ext, (0.0, 0.9 * zmax), length_range=(0.01, 0.1), seed=seed)
    zl = (g.nticks - 12) * W.TICK * ph.v_drift
    extra = [[x, y, z, x + 0.02, y + 0.01, z + 0.01, 3.0e4] for (x, y, z) in [
        (0.003, 0.5 * ext[1], 0.3 * zmax), (ext[0] - 0.003 - 0.02, 0.3 * ext[1], 0.5 * zmax),
        (0.6 * ext[0], 0.004, 0.6 * zmax), (0.2 * ext[0], ext[1] - 0.004 - 0.01, zl),
        (0.45 * ext[0], 0.55 * ext[1], zl)]]
    return np.concatenate([seg, np.array(extra, np.float32)]).astype(np.float32)


@pytest.mark.parametrize("batch", [64, 3])
def test_module_instance_four_pieces_matches_oracle(T, orc, batch):
    """fs 40 / 16 inputs / two bins per workgroup / four pieces, row masks: 48x48 pixels
    x 1,100 ticks (the last 512-tick bin holds 76 ticks), 16x16x512 bins, 21x21x1,800
    response, FFT 40x40x1024; 15 active bins (odd: the last workgroup of a pass holds
    one bin) in one pass, and in passes of 3."""
    from test_gpu_parity import compare_all, gpu_path
    say(f"test_module_instance_four_pieces_matches_oracle[batch={batch}]")
    g = W._grid(48, 1100)
    ph = W._physics(g)
    blk, kpix, kticks, fft = W.Blocking((16, 16), 512), (21, 21), 1800, (40, 40, 1024)
    seg = fs40_event(g, ph)
    resp = W.synthetic_response(kpix, g.sub, kticks)
    o = orc.simulate(g, ph, blk, kpix, kticks, resp, seg)
    keys = o["keys"]
    say(f"  {len(keys)} active bins, {int((keys[:, 2] == 2).sum())} in the partial last bin")
    assert len(keys) % 2 == 1 and (keys[:, 2] == 2).any()
    nfx = g.npix[0] * g.sub[0]
    fp = o["fp"]
    assert (fp[:, 0] == 0).any() and (fp[:, 3] == nfx - 1).any()
    assert (fp[:, 1] == 0).any() and (fp[:, 4] == nfx - 1).any()
    r = gpu_path(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp=True, batch=batch)
    pl_info = T.ConvPlan(g, blk, kpix, kticks, fft, True, 1).info()
    assert pl_info[1] == 4, pl_info
    compare_all(r, o)
    # the partial last bin's ticks and the region-edge pixels on their own
    late = rel_l2(r["wf"][:, 1024:], o["wf"][:, 1024:])
    px, py = o["pix"] // g.npix[1], o["pix"] % g.npix[1]
    edge = (px == 0) | (py == 0) | (px == g.npix[0] - 1) | (py == g.npix[1] - 1)
    e_edge = rel_l2(r["wf"][edge], o["wf"][edge])
    say(f"  rel-L2 ticks >= 1024: {late:.2e}; {int(edge.sum())} region-edge pixels: {e_edge:.2e}")
    assert late < TOL and e_edge < TOL


# ---------------------------------------------------------------------------
# gradient at the differentiation workload's shapes


def test_gradient_at_module_response_shapes(T, orc):
    """Whole-chain gradient (four transposes, row masks) of L = sum_m c_m wf[p_m, t_m]
    over sampled waveform points, on three depositions in the 128x128-pixel region
    with the 21x21 x 2,048-tick response (fs 40, four pieces), against central
    differences of the oracle's path (footprints, effective charge, direct sum at the
    points) in every deposition parameter and in diff_T, diff_L, lifetime."""
    import torch
    from test_gpu_transpose import compare_grad, fd_params
    say("test_gradient_at_module_response_shapes")
    cfg = W.cfg_diff()
    g, ph, blk = cfg.grid, cfg.physics, cfg.blocking
    kpix, kticks, fft = cfg.kpix, cfg.kticks, cfg.fft
    ext = (g.npix[0] * W.PITCH, g.npix[1] * W.PITCH)
    seg = W.gen_uniform_segments(3, (0.5 * ext[0], 0.5 * ext[1]), (20.0, 40.0),
                                 length_range=(0.04, 0.06), seed=5)
    seg[:, [0, 3]] += np.float32(0.25 * ext[0])
    seg[:, [1, 4]] += np.float32(0.25 * ext[1])
    resp = W.synthetic_response(kpix, g.sub, kticks)
    fp, off, ip = orc.footprints(g, ph, seg)
    assert not ip.any()
    # samples: pixels at and around each deposition, ticks over the response's lobes
    rng = np.random.default_rng(3)
    pts = []
    for d in range(3):
        px = int(0.5 * (seg[d, 0] + seg[d, 3]) / W.PITCH)
        py = int(0.5 * (seg[d, 1] + seg[d, 4]) / W.PITCH)
        t0 = int(0.5 * (seg[d, 2] + seg[d, 5]) / ph.v_drift / W.TICK)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for f in (0.5, 0.85, 0.9, 0.95):
                    pts.append(((px + dx) * g.npix[1] + py + dy,
                                t0 + int(f * kticks) + int(rng.integers(-3, 4))))
    pts = np.array(pts, np.int32)
    c = rng.uniform(0.5, 1.5, len(pts)) * np.where(np.arange(len(pts)) % 2 == 0, 1.0, -1.0)

    def loss(s, p):
        fps, offs, _ = orc.footprints(g, p, s)
        val, _ = orc.effq(g, p, s, fps, offs)
        return float(np.dot(orc.waveform_points(g, kpix, kticks, resp, fps, offs, val, pts), c))

    ref_seg, ref_phys = fd_params(orc, g, ph, seg, loss, fp)
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_event(g, ph, blk, kpix, sd)
    pl = T.Pipeline(g, ph, blk, kpix, kticks, dev(resp), 3, val_cap, bcap, pix_cap, fft, True,
                    bcap)
    assert pl.plan.pieces == 4
    pl.run(sd)
    pl.check_capacity()
    npx = int(pl.n_pix.item())
    pix = pl.pix[:npx].cpu().numpy()
    slot = np.searchsorted(pix, pts[:, 0])
    assert (pix[slot] == pts[:, 0]).all()
    d_wf = np.zeros(tuple(pl.wf.shape), np.float32)
    np.add.at(d_wf, (slot, pts[:, 1]), c.astype(np.float32))
    d_seg, d_phys = pl.backward(sd, dev(d_wf))
    torch.cuda.synchronize()
    got_seg, got_phys = d_seg.cpu().numpy().astype(np.float64), d_phys.cpu().numpy()
    say(f"  {int(pl.n_active.item())} bins, {npx} pixels, {len(pts)} loss samples")
    compare_grad("end points", got_seg[:, :6], ref_seg[:, :6], 1e-4)
    compare_grad("charges", got_seg[:, 6], ref_seg[:, 6], 1e-4)
    compare_grad("diff_T, diff_L, lifetime", got_phys, ref_phys, 1e-4)


# ---------------------------------------------------------------------------
# the 64-event batch


def test_event_batch_64_matches_oracle(T, orc):
    """The 64 module-scale events of the batched workload (2.4 M depositions), run as the
    benchmark runs them: events grouped into chunks whose bins fit a 200 GB budget
    (with a 60 GB convolution pass), each chunk through one BatchPipeline (16x16x512
    bins, FFT 40x40x1024) with the chunk's own pixel capacity. Per event, the bins and the pixel set equal the oracle's;
    sampled waveform points of the three smallest events are within 1e-5 of it."""
    import torch
    from paper_2602_12052_amd import autotune
    say("test_event_batch_64_matches_oracle")
    torch.cuda.empty_cache()
    cfg = W.cfg_module()
    g, ph, blk = cfg.grid, cfg.physics, cfg.blocking
    evs = W.gen_event_batch(64, (1_000, 200_000), seed=1)
    sizes = np.array([len(e) for e in evs])
    resp = W.synthetic_response(cfg.kpix, g.sub, cfg.kticks)
    okeys, opix, ofps = [], [], []
    for e in evs:
        fp, off, _ = orc.footprints(g, ph, e)
        k = orc.block_keys(g, blk, fp)
        okeys.append(k)
        opix.append(orc.pix_set(g, blk, cfg.kpix, k))
        ofps.append((fp, off))
    bins = np.array([len(k) for k in okeys])
    # the exact pixel counts the benchmark sizes its chunks by equal the oracle's pixel sets
    for e in np.argsort(sizes)[[0, 1, len(evs) // 2, -1]]:
        got = T.size_event(g, ph, blk, cfg.kpix, dev(evs[e]), exact_pixels=True)
        assert got[1] == bins[e] and got[2] == len(opix[e]), (e, got, bins[e], len(opix[e]))
    fixed, scratch = autotune._bytes_per_bin(g, blk, cfg.kpix, cfg.kticks, cfg.fft, True)
    pass_bins = max(1, int(60e9 // scratch))
    chunk_bins = max(int(bins.max()), int((200e9 - pass_bins * scratch) // fixed))
    chunks, cur, nb = [], [], 0
    for e in range(len(evs)):
        if cur and nb + bins[e] > chunk_bins:
            chunks.append(cur)
            cur, nb = [], 0
        cur.append(e)
        nb += int(bins[e])
    chunks.append(cur)
    say(f"  {int(sizes.sum())} depositions, {int(bins.sum())} (event, bin) pairs, "
        f"{len(chunks)} chunks of <= {chunk_bins} bins, {pass_bins} bins per pass")
    npix = g.npix[0] * g.npix[1]
    per_pix = (blk.blk_pix[0] + cfg.kpix[0] - 1) * (blk.blk_pix[1] + cfg.kpix[1] - 1)
    caps = [(int(sum(ofps[e][1][-1] for e in c)), int(bins[c].sum()),
             int(sum(min(npix, bins[e] * per_pix) for e in c)), int(sizes[c].sum()))
            for c in chunks]
    bp = T.BatchPipeline(g, ph, blk, cfg.kpix, cfg.kticks, dev(resp),
                         max(len(c) for c in chunks), max(x[3] for x in caps),
                         max(x[0] for x in caps), max(x[1] for x in caps),
                         max(x[2] for x in caps), cfg.fft, True,
                         min(pass_bins, max(x[1] for x in caps)))
    small = set(np.argsort(sizes)[:3].tolist())
    checked = 0
    for ci, c in enumerate(chunks):
        n = int(sizes[c].sum())
        eo = np.concatenate([[0], np.cumsum(sizes[c])]).astype(np.int64)
        # each chunk with its own pixel capacity, as the benchmark runs them
        pc = caps[ci][2]
        bp.run(dev(np.concatenate([evs[e] for e in c])), dev(eo), pix_cap=pc)
        torch.cuda.synchronize()
        na, npx = int(bp.n_active.item()), int(bp.n_pix.item())
        assert int(bp.off[n].item()) <= bp.val.numel()
        assert na <= bp.keys.shape[0] and npx <= pc <= bp.pix.shape[0]
        # the rows past the chunk's pixels, up to its capacity, are zero waveforms
        assert npx == pc or float(bp.wf[npx:pc].abs().max()) == 0.0
        keys = bp.keys[:na].cpu().numpy()
        pix = bp.pix[:npx].cpu().numpy()
        for i, e in enumerate(c):
            assert np.array_equal(keys[keys[:, 0] == i][:, 1:], okeys[e]), e
            m = np.nonzero((pix // npix) == i)[0]
            assert np.array_equal(pix[m] - i * npix, opix[e]), e
            if e not in small:
                continue
            fp, off = ofps[e]
            rng = np.random.default_rng(e)
            pts = []
            for d in rng.choice(len(evs[e]), 8, replace=False):
                s = evs[e][d]
                px = int(0.5 * (s[0] + s[3]) / W.PITCH)
                py = int(0.5 * (s[1] + s[4]) / W.PITCH)
                t0 = int(0.5 * (s[2] + s[5]) / ph.v_drift / W.TICK)
                for dt in (int(0.5 * cfg.kticks), int(0.9 * cfg.kticks)):
                    if 0 <= px < g.npix[0] and 0 <= py < g.npix[1] and \
                            t0 + dt < g.nticks + cfg.kticks - 1:
                        pts.append((px, py, t0 + dt))
            pts = np.array(pts)
            near = orc.select_near(fp, g.sub, cfg.kpix, cfg.kticks, pts)
            sfp = fp[near]
            vol = np.prod(np.maximum(sfp[:, 3:] - sfp[:, :3] + 1, 0), axis=1)
            soff = np.concatenate([[0], np.cumsum(vol)]).astype(np.int64)
            sval, _ = orc.effq(g, ph, evs[e][near], sfp, soff)
            ids = pts[:, 0] * g.npix[1] + pts[:, 1]
            ref = orc.waveform_points(g, cfg.kpix, cfg.kticks, resp, sfp, soff, sval,
                                      np.stack([ids, pts[:, 2]], 1))
            k = np.searchsorted(pix[m] - i * npix, ids)
            assert (pix[m][k] - i * npix == ids).all()
            rows = dev(m[k].astype(np.int64))
            got = bp.wf[rows, dev(pts[:, 2].astype(np.int64))].cpu().numpy()
            err = rel_l2(got, ref)
            say(f"  chunk {ci}, event {e}: {sizes[e]} depositions, {len(pts)} samples, "
                f"rel-L2 {err:.2e}")
            assert err < TOL
            checked += 1
    assert checked == 3
    del bp
    torch.cuda.empty_cache()

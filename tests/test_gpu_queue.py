"""GPU tests of batches of events: the (event, bin) pairs of several events go through
one binned tensor and one convolution pass. Per event, bins and pixels must be
bit-exact equal to the single-event path (and to the oracle), waveforms within the
FP32 tolerance; a captured HIP graph of a batch must reproduce the eager run on
every replay."""
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


def small_events(g, ph, sizes, seed):
    zmax = g.nticks * W.TICK * ph.v_drift
    ext = (g.npix[0] * W.PITCH, g.npix[1] * W.PITCH)
    evs = []
    for i, n in enumerate(sizes):
        evs.append(W.gen_uniform_segments(n, ext, (0.0, zmax), seed=seed + i))
    return evs


def run_batch(T, g, ph, blk, kpix, kticks, fft, resp, evs, batch=5):
    import torch
    seg = np.concatenate(evs) if sum(len(e) for e in evs) else np.zeros((0, 7), np.float32)
    ev_off = np.concatenate([[0], np.cumsum([len(e) for e in evs])]).astype(np.int64)
    sd = dev(seg)
    val_cap, bcap, pix_cap = T.size_batch(g, ph, blk, kpix, sd, ev_off)
    bp = T.BatchPipeline(g, ph, blk, kpix, kticks, dev(resp), len(evs), seg.shape[0], val_cap,
                         bcap, pix_cap, fft, True, batch)
    bp.run(sd, dev(ev_off))
    return bp, sd, ev_off, bp.results(seg.shape[0])


def split_by_event(r, n_ev, npix):
    keys, pix, wf = r["keys"], r["pix"], r["wf"]
    out = []
    for e in range(n_ev):
        ke = keys[keys[:, 0] == e][:, 1:]
        m = (pix // npix) == e
        out.append(dict(keys=ke, pix=pix[m] - e * npix, wf=wf[m]))
    return out


def test_batch_equals_single_events_and_oracle(T, orc):
    """Four events of uneven size (one empty, one outside the readout window) batched:
    per event bins/pixels bit-exact vs each event alone and vs the oracle."""
    say("test_batch_equals_single_events_and_oracle")
    from test_gpu_parity import gpu_path, small_cfg
    g, ph, blk, kpix, kticks, fft, _ = small_cfg(npix=8, sub=3, nticks=300, blk=(2, 2, 64),
                                                 kpix=(3, 5), kticks=100, fft=(8, 8, 256))
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    evs = small_events(g, ph, [25, 0, 7, 40], seed=30)
    far = evs[2].copy()
    far[:, 2] += 100.0
    far[:, 5] += 100.0
    evs[2] = far
    bp, sd, ev_off, r = run_batch(T, g, ph, blk, kpix, kticks, fft, resp, evs, batch=5)
    npix = g.npix[0] * g.npix[1]
    per = split_by_event(r, len(evs), npix)
    for e, seg in enumerate(evs):
        o = orc.simulate(g, ph, blk, kpix, kticks, resp, seg)
        assert np.array_equal(per[e]["keys"], o["keys"]), e
        assert np.array_equal(per[e]["pix"], o["pix"]), e
        if len(o["pix"]):
            err = rel_l2(per[e]["wf"], o["wf"])
            say(f"  event {e}: {len(seg)} depositions, {len(o['keys'])} bins, rel-L2 {err:.2e}")
            assert err < TOL
            s = gpu_path(T, g, ph, blk, kpix, kticks, fft, seg, resp, mpcp=True, batch=5)
            assert np.array_equal(s["keys"], per[e]["keys"])
            assert rel_l2(per[e]["wf"], s["wf"]) < 1e-6
        else:
            assert len(per[e]["keys"]) == 0
    # the footprints of the concatenation are the per-event footprints
    ofp, ooff, _ = orc.footprints(g, ph, np.concatenate(evs))
    assert np.array_equal(r["fp"], ofp)


def test_batch_module_events(T):
    """Three module-scale events of uneven size batched vs each alone (bins bit-exact,
    waveforms within FP32 rounding)."""
    say("test_batch_module_events")
    from test_gpu_parity import gpu_path
    cfg = W.cfg_module()
    g, ph, blk = cfg.grid, cfg.physics, cfg.blocking
    resp = W.synthetic_response(cfg.kpix, g.sub, cfg.kticks)
    evs = W.gen_event_batch(3, (2_000, 20_000), seed=5)
    bp, sd, ev_off, r = run_batch(T, g, ph, blk, cfg.kpix, cfg.kticks, cfg.fft, resp, evs,
                                  batch=256)
    per = split_by_event(r, len(evs), g.npix[0] * g.npix[1])
    del bp
    for e, seg in enumerate(evs):
        s = gpu_path(T, g, ph, blk, cfg.kpix, cfg.kticks, cfg.fft, seg, resp, mpcp=True, batch=256)
        assert np.array_equal(s["keys"], per[e]["keys"])
        assert np.array_equal(s["pix"], per[e]["pix"])
        err = rel_l2(per[e]["wf"], s["wf"])
        say(f"  event {e}: {len(seg)} depositions, {len(s['keys'])} bins, batch vs alone {err:.2e}")
        assert err < 1e-6


def test_batch_graph_replays_match_eager(T):
    """A captured graph of one batch replays to the eager result, with eager work
    (another batch through the same buffers) between the replays."""
    import torch
    say("test_batch_graph_replays_match_eager")
    from test_gpu_parity import small_cfg
    g, ph, blk, kpix, kticks, fft, _ = small_cfg(npix=8, sub=3, nticks=300, blk=(2, 2, 64),
                                                 kpix=(3, 5), kticks=100, fft=(8, 8, 256))
    resp = W.random_symmetric_response(kpix, g.sub, kticks, seed=11)
    evs_a = small_events(g, ph, [30, 12, 45], seed=40)
    evs_b = small_events(g, ph, [20, 35], seed=50)
    seg_a, seg_b = np.concatenate(evs_a), np.concatenate(evs_b)
    off_a = np.concatenate([[0], np.cumsum([len(e) for e in evs_a])]).astype(np.int64)
    off_b = np.concatenate([[0], np.cumsum([len(e) for e in evs_b])]).astype(np.int64)
    sa, sb, oa, ob = dev(seg_a), dev(seg_b), dev(off_a), dev(off_b)
    ca = T.size_batch(g, ph, blk, kpix, sa, off_a)
    cb = T.size_batch(g, ph, blk, kpix, sb, off_b)
    caps = [max(x, y) for x, y in zip(ca, cb)]
    bp = T.BatchPipeline(g, ph, blk, kpix, kticks, dev(resp), 3, max(len(seg_a), len(seg_b)),
                         caps[0], caps[1], caps[2], fft, True, 4)
    # each batch with its own pixel capacity (batch a's graph writes rows up to ca[2])
    bp.run(sa, oa, pix_cap=ca[2])
    ref_a = bp.results(len(seg_a), pix_cap=ca[2])
    bp.run(sb, ob, pix_cap=cb[2])
    ref_b = bp.results(len(seg_b), pix_cap=cb[2])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bp.run(sa, oa, pix_cap=ca[2])
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bp.run(sa, oa, pix_cap=ca[2])
    for rep in range(3):
        graph.replay()
        got = bp.results(len(seg_a), pix_cap=ca[2])
        assert got["n_active"] == ref_a["n_active"] and np.array_equal(got["keys"], ref_a["keys"])
        assert np.array_equal(got["pix"], ref_a["pix"])
        err = rel_l2(got["wf"], ref_a["wf"])
        say(f"  replay {rep}: rel-L2 vs eager {err:.2e}")
        assert err < 1e-6
        bp.run(sb, ob, pix_cap=cb[2])   # eager work through the same buffers between replays
        got_b = bp.results(len(seg_b), pix_cap=cb[2])
        assert np.array_equal(got_b["keys"], ref_b["keys"])
        assert rel_l2(got_b["wf"], ref_b["wf"]) < 1e-6

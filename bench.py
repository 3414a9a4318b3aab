"""Benchmark: depositions/s of the whole hot path on one MI355X.

A step is one pass of the path over one synthetic module-scale event (1e5 line
depositions from muon-like tracks and shower blobs in a 256 x 256-pixel region,
21 x 21 x 2048 field response, 16 x 16-pixel x 512-tick bins):

  tred_effq_windows -> tred_effq -> tred_block_bin_rows -> tred_block_conv_rows ->
  tred_scatter_waveforms

Inputs (depositions, response spectra) are resident in HBM before the timed region;
the convolution plan is built once, untimed. Prints one JSON line.
"""
import argparse
import ctypes as C
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 vector: 256 CU x 128 lanes x 2 (FMA) x 2 (dual issue) x 2.4 GHz
BF16_MFMA_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak


class HipEvents:
    """hipEvent_t handles through libamdhip64 (recorded on the launch stream)."""

    def __init__(self, n):
        self.hip = C.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [C.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.ev = []
        for _ in range(n):
            e = C.c_void_p()
            if self.hip.hipEventCreate(C.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev.append(e)

    def record(self, i, stream):
        self.hip.hipEventRecord(self.ev[i], stream)

    def ms(self, a, b):
        self.hip.hipEventSynchronize(self.ev[b])
        out = C.c_float()
        self.hip.hipEventElapsedTime(C.byref(out), self.ev[a], self.ev[b])
        return float(out.value)

    def handles(self, idx):
        return [self.ev[i].value for i in idx]


def fft_flops(n, nnz=None):
    """5 n log2 n for an n-point complex FFT. For a power-of-two n with only nnz
    leading nonzero inputs the first log2(n / nnz') stages (nnz' the next power of
    two) are copies and free; other sizes get no pruning credit."""
    stages = math.log2(n)
    if nnz and n & (n - 1) == 0:
        stages -= math.log2(n / (1 << int(math.ceil(math.log2(max(nnz, 1))))))
    return 5.0 * n * stages


def conv_flops_per_block(blk, sub, kpix, kticks, fft, mpcp):
    """Algorithmic FLOPs of the three convolution stages for one bin: 5 N log2 N per N-point
    complex FFT (pruned inputs credited for power-of-two N), 8 per complex multiply-add."""
    Bx, By, Bt = blk
    fs, ft = fft[0], fft[2]
    nch = (sub[0] * sub[1] + 1) // 2 if mpcp else sub[0] * sub[1]
    ct = ft - Bt
    nc = -(-kticks // ct)
    box, boy = Bx + kpix[0] - 1, By + kpix[1] - 1
    tf = nch * Bx * By * fft_flops(ft, Bt)
    per_f = nch * (By * fft_flops(fs, Bx) + fs * fft_flops(fs, By) + nc * fs * fs * 8) + \
        nc * (fs * fft_flops(fs) + boy * fft_flops(fs))
    sp = ft * per_f
    ti = nc * box * boy * fft_flops(ft)
    return dict(tf=tf, sp=sp, ti=ti, total=tf + sp + ti)


def src_sha(parts):
    """Hash of source text: each part is a path, or (path, first marker, end marker) for
    the lines from the first marker up to the end marker."""
    h = hashlib.sha256()
    for part in parts:
        path, a, b = (part, None, None) if isinstance(part, str) else part
        with open(os.path.join(ROOT, path), "rb") as f:
            text = f.read()
        if a is not None:
            i = text.index(a.encode())
            text = text[i:text.index(b.encode(), i)]
        h.update(text)
    return h.hexdigest()[:16]


# the source of the k_spp kernel: its section of conv.hip and the shared device helpers
KSPP_SOURCE = [("paper_2602_12052_amd/csrc/conv.hip", "// k_spp: the spatial stage",
                "// k_ti: inverse time FFT"), "paper_2602_12052_amd/csrc/tred_internal.hpp"]


def profile_traffic(kernel_key, sha):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they were
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(kernel_key)
        if not e or e.get("source_sha") != sha:
            return None
        return float(e["hbm_bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(cfg, seg, resp, n_sample, seed=0):
    """The FP64 oracle (effective charge, binning, direct convolution) on a random
    sample of the event's depositions, timed on the host cores."""
    import oracle
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(seg.shape[0], n_sample, replace=False))
    sub = seg[pick]
    t = time.perf_counter()
    oracle.simulate(cfg.grid, cfg.physics, cfg.blocking, cfg.kpix, cfg.kticks, resp, sub)
    dt = time.perf_counter() - t
    return dict(value=n_sample / dt, unit="depositions/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"{n_sample} random depositions of the same event (seed {seed}), whole path "
                       f"(effective charge, binning, direct convolution, waveforms): {dt:.1f} s",
                host_cpu=host_cpu_model(), nproc=os.cpu_count(),
                affinity=len(os.sched_getaffinity(0)))


def host_cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo, as lscpu prints it)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_direct(args, split):
    """Block-direct convolution on BF16 matrix cores (hi/lo split or plain) beside the FP32
    FFT convolution on the same bins: the whole 1,000-deposition event and a sample of
    bins of the module-scale event. Prints one JSON line (not the benchmark's main line)."""
    import torch
    import workloads as W
    from paper_2602_12052_amd import tred
    stream = torch.cuda.current_stream().cuda_stream
    ev = HipEvents(4)
    forms = []
    for name, cfg, nbins in (("plain-small-1k", W.cfg_plain_small(args.seed), None),
                             ("module-1e5", W.cfg_module(args.seed), args.direct_bins)):
        seg = W.gen_segments(cfg)
        resp = W.synthetic_response(cfg.kpix, cfg.grid.sub, cfg.kticks)
        sd = torch.from_numpy(seg).cuda()
        dresp = torch.from_numpy(resp).cuda()
        val_cap, bcap, pix_cap = tred.size_event(cfg.grid, cfg.physics, cfg.blocking, cfg.kpix, sd)
        n = bcap if nbins is None else min(nbins, bcap)
        pl = tred.Pipeline(cfg.grid, cfg.physics, cfg.blocking, cfg.kpix, cfg.kticks, dresp,
                           seg.shape[0], val_cap, bcap, pix_cap, cfg.fft, True, n, row_masks=False)
        pl.run(sd, stop_after="bin")
        nact = torch.tensor([n], dtype=torch.int32, device="cuda")
        blocks = pl.blocks[:n]
        dp = tred.DirectPlan(cfg.grid, cfg.blocking, cfg.kpix, cfg.kticks, split=split, batch=n)
        dp.set_response(dresp)
        out_d = torch.empty((n, pl.out_blocks.shape[1]), dtype=torch.float32, device="cuda")
        out_f = torch.empty_like(out_d)

        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                ev.record(0, stream)
                fn()
                ev.record(1, stream)
                ts.append(ev.ms(0, 1))
            return float(np.median(ts))

        reps = max(1, args.steps)
        t_d = timed(lambda: tred.tred_block_conv_direct(dp, nact, blocks, out_d, stream=stream), reps)
        t_f = timed(lambda: tred.tred_block_conv(pl.plan, nact, blocks, out_f, stream), reps)
        torch.cuda.synchronize()
        d, f = out_d.double(), out_f.double()
        err = float(torch.linalg.norm(d - f) / torch.linalg.norm(f))
        Bx, By = cfg.blocking.blk_pix
        S = cfg.grid.sub[0] * cfg.grid.sub[1]
        useful = 2.0 * n * (Bx * By * S * cfg.blocking.blk_ticks) * (cfg.kpix[0] * cfg.kpix[1] * cfg.kticks)
        prods = 3 if split else 1
        forms.append({
            "workload": name, "bins": n, "direct_ms": t_d, "direct_ms_per_bin": t_d / n,
            "fft_fp32_ms": t_f, "fft_fp32_ms_per_bin": t_f / n,
            "mfma_useful_tflop": useful * prods / 1e12,
            "mfma_achieved_tflops": useful * prods / (t_d * 1e-3) / 1e12,
            "mfma_frac_of_bf16_peak": useful * prods / (t_d * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS,
            "rel_l2_vs_fft_fp32": err,
        })
        print(f"# {name}: {forms[-1]}", file=sys.stderr, flush=True)
        del pl, dp, out_d, out_f
        torch.cuda.empty_cache()
    print(json.dumps({
        "metric": "block-direct convolution on BF16 MFMA (%s) beside the FP32 FFT path" %
                  ("hi/lo split, 3 products" if split else "plain BF16"),
        "unit": "ms", "dtype": "bf16x3" if split else "bf16", "data": "synthetic",
        "peak_tflops": BF16_MFMA_PEAK_TFLOPS, "forms": forms}), flush=True)


def bench_adjoint(args):
    """Differentiation workload: 2e4 depositions in a 128x128-pixel region with the
    module-scale response. A step is the forward path (five calls), the gradient of
    the L2 loss against target waveforms made with diff_T +10 %, diff_L -10 % and
    lifetime +20 % (aligned on the simulated pixel list), and the four transposed
    calls back to dL/d(depositions) and dL/d(diff_T, diff_L, lifetime). One JSON line."""
    import copy
    import torch
    import workloads as W
    from paper_2602_12052_amd import tred
    stream = torch.cuda.current_stream().cuda_stream
    cfg = W.cfg_diff(args.seed)
    seg = W.gen_segments(cfg)
    resp = W.synthetic_response(cfg.kpix, cfg.grid.sub, cfg.kticks)
    sd = torch.from_numpy(seg).cuda()
    dresp = torch.from_numpy(resp).cuda()
    g, ph, blk = cfg.grid, cfg.physics, cfg.blocking
    pt = copy.copy(ph)
    pt.diff_T, pt.diff_L, pt.lifetime = ph.diff_T * 1.1, ph.diff_L * 0.9, ph.lifetime * 1.2
    caps = [max(a, b) for a, b in zip(tred.size_event(g, ph, blk, cfg.kpix, sd),
                                      tred.size_event(g, pt, blk, cfg.kpix, sd))]
    pl = tred.Pipeline(g, ph, blk, cfg.kpix, cfg.kticks, dresp, seg.shape[0], caps[0], caps[1],
                       caps[2], cfg.fft, True, caps[1], fused=not args.unfused)
    tgt = tred.Pipeline(g, pt, blk, cfg.kpix, cfg.kticks, dresp, seg.shape[0], caps[0], caps[1],
                        caps[2], cfg.fft, True, caps[1], fused=not args.unfused)
    tgt.run(sd)
    torch.cuda.synchronize()
    nt = int(tgt.n_pix.item())
    tpix, twf = tgt.pix[:nt].clone(), tgt.wf[:nt].clone()
    del tgt
    torch.cuda.empty_cache()
    d_wf = torch.zeros_like(pl.wf)
    ev = HipEvents(3)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")

    def step():
        ev.record(0, stream)
        pl.run(sd)
        ev.record(1, stream)
        n = pl.n_pix                          # device scalar; wf rows past it are zero
        rows = torch.arange(pl.pix.shape[0], device="cuda")
        live = rows < n
        j = torch.searchsorted(tpix, pl.pix).clamp_(max=max(nt - 1, 0))
        hit = live & (tpix[j] == pl.pix) if nt > 0 else torch.zeros_like(live)
        target = torch.where(hit[:, None], twf[j], torch.zeros((), device="cuda"))
        torch.sub(pl.wf, target, out=d_wf)
        d_wf.masked_fill_(~live[:, None], 0.0)
        loss.copy_(0.5 * (d_wf.double() ** 2).sum())
        pl.backward(sd, d_wf)
        ev.record(2, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ts, tf, tb = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - s0))
        tf.append(ev.ms(0, 1))
        tb.append(ev.ms(1, 2))
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / args.steps
    d_seg = pl.d_seg.double()
    print(json.dumps({
        "metric": "depositions/s, forward path + gradient (L2 loss on the waveforms)",
        "value": seg.shape[0] / (ms * 1e-3), "unit": "depositions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "differentiation: 2e4 depositions (tracks + blobs) in 128x128 pixels "
                               "x 6250 ticks, response 21x21 px x 2048 ticks, bins 16x16 px x 512 "
                               "ticks; target waveforms with diff_T +10 %, diff_L -10 %, lifetime "
                               "+20 %", "n_dep": int(seg.shape[0]),
                   "effective_charge": "patches" if args.unfused else "into the bins",
                   "active_bins": int(pl.n_active.item()), "pixels": int(pl.n_pix.item())},
        "step_ms": {"p50": float(np.percentile(ts, 50)), "p99": float(np.percentile(ts, 99))},
        "stage_ms": {"forward": float(np.median(tf)), "loss+gradient": float(np.median(tb))},
        "loss": float(loss.item()),
        "grad": {"d_diff_T": float(pl.d_phys[0]), "d_diff_L": float(pl.d_phys[1]),
                 "d_lifetime": float(pl.d_phys[2]),
                 "rms_d_endpoints": float(torch.sqrt((d_seg[:, :6] ** 2).mean())),
                 "rms_d_charge": float(torch.sqrt((d_seg[:, 6] ** 2).mean()))},
    }), flush=True)


def bench_batched(args):
    """Batched events: n_ev module-scale events of log-uniform size in [1e3, 2e5]. The
    autotuner picks the bin shape and FFT sizes on three events (the quartile sizes);
    events are taken smallest first (by active bins) and grouped into chunks of at most
    --chunk-bins (event, bin) pairs that also fit a memory budget (an event with more
    bins is a chunk of its own); each chunk's whole
    path (effq, binning with the event in the key, one convolution queue over all its
    bins, per-event overlap-add) is captured once in a HIP graph, and the graphs are
    replayed back to back. Reports throughput and the per-event completion latency
    (time from the batch start until the event's chunk is done). One JSON line."""
    import torch
    import workloads as W
    from paper_2602_12052_amd import autotune, tred
    cfg = W.cfg_module(args.seed)
    g, ph = cfg.grid, cfg.physics
    evs = W.gen_event_batch(args.events, (1_000, 200_000), seed=args.seed)
    sizes = np.array([len(e) for e in evs])
    resp = W.synthetic_response(cfg.kpix, g.sub, cfg.kticks)
    dresp = torch.from_numpy(resp).cuda()
    log = lambda m: print("# " + m, file=sys.stderr, flush=True)
    order = np.argsort(sizes, kind="stable")
    picks = [int(order[int(q * (len(sizes) - 1))]) for q in (0.25, 0.5, 0.75)]
    tune = autotune.tune(g, ph, cfg.kpix, cfg.kticks, dresp,
                         [torch.from_numpy(evs[e]).cuda() for e in picks],
                         make_blocking=lambda bp, bt: W.Blocking((bp, bp), bt), log=log,
                         fused=not args.unfused)
    best = tune.best
    blk = W.Blocking((best.blk_pix, best.blk_pix), best.blk_ticks)
    fft = best.fft
    caps = [tred.size_event(g, ph, blk, cfg.kpix, torch.from_numpy(e).cuda(), exact_pixels=True)
            for e in evs]
    bins = np.array([c[1] for c in caps])
    fixed, scratch = autotune._bytes_per_bin(g, blk, cfg.kpix, cfg.kticks, fft, True)
    # one convolution pass per packed chunk unless --pass-gb bounds its scratch (each
    # pass has a fixed cost besides its bins, so a second, small pass is not free)
    pass_bins = (args.chunk_bins if args.pass_gb is None
                 else max(1, int(args.pass_gb * 1e9 // scratch)))
    # packing target of a chunk; an event with more bins than that is a chunk of its own
    # (the pipeline's capacity is the largest chunk, whichever of the two it is)
    chunk_bins = max(1, min(args.chunk_bins,
                            int((args.budget_gb * 1e9 - pass_bins * scratch) // fixed)))
    # smallest events first: the median event completes after a small share of the work
    chunks = autotune.plan_chunks(bins, chunk_bins)
    ccap = [(sum(caps[e][0] for e in c), sum(caps[e][1] for e in c), sum(caps[e][2] for e in c),
             int(sizes[c].sum())) for c in chunks]
    maxc = max(c[1] for c in ccap)
    bp = tred.BatchPipeline(g, ph, blk, cfg.kpix, cfg.kticks, dresp, max(len(c) for c in chunks),
                            max(c[3] for c in ccap), max(c[0] for c in ccap),
                            maxc, max(c[2] for c in ccap), fft, True,
                            min(pass_bins, maxc), fused=not args.unfused)
    segs, offs = [], []
    for c in chunks:
        segs.append(torch.from_numpy(np.concatenate([evs[e] for e in c])).cuda())
        offs.append(torch.from_numpy(np.concatenate([[0], np.cumsum(sizes[c])]).astype(np.int64)).cuda())
    log(f"{len(evs)} events, {int(sizes.sum())} depositions, {int(bins.sum())} active (event, bin) "
        f"pairs in {len(chunks)} chunks (packed to <= {chunk_bins} bins, largest {maxc}), "
        f"{pass_bins} bins per pass")
    # eager warm-up of every chunk, then one captured graph per chunk; each chunk writes
    # waveform rows up to its own pixel capacity (its events' bounds)
    for sg, of, cc in zip(segs, offs, ccap):
        bp.run(sg, of, pix_cap=cc[2])
    torch.cuda.synchronize()
    graphs = []
    for sg, of, cc in zip(segs, offs, ccap):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            bp.run(sg, of, pix_cap=cc[2])
        torch.cuda.current_stream().wait_stream(side)
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            bp.run(sg, of, pix_cap=cc[2])
        graphs.append(gr)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream
    ev = HipEvents(len(graphs) + 1)
    lat, totals = [], []
    for rep in range(args.warmup + args.steps):
        ev.record(0, stream)
        for i, gr in enumerate(graphs):
            gr.replay()
            ev.record(i + 1, stream)
        torch.cuda.synchronize()
        ends = [ev.ms(0, i + 1) for i in range(len(graphs))]
        if rep >= args.warmup:
            totals.append(ends[-1])
            for i, c in enumerate(chunks):
                lat.extend([ends[i]] * len(c))
    total_ms = float(np.median(totals))
    out = {
        "metric": "depositions/s, batched events (HIP graph per chunk of events)",
        "value": float(sizes.sum()) / (total_ms * 1e-3), "unit": "depositions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_batch": total_ms,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(evs)} module-scale events, deposition counts log-uniform in "
                               f"[1e3, 2e5], per-event track/blob mix",
                   "n_dep": int(sizes.sum()), "active_event_bins": int(bins.sum()),
                   "chunks": len(chunks), "chunk_bins": chunk_bins, "chunk_capacity": maxc, "order": "smallest first",
                   "effective_charge": "patches" if args.unfused else "into the bins",
                   "bins_per_pass": min(pass_bins, maxc),
                   "blocking": [best.blk_pix, best.blk_pix, best.blk_ticks], "fft": list(fft)},
        "event_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "autotune": [{"blk": [t.blk_pix, t.blk_pix, t.blk_ticks], "fft": list(t.fft), "ms": t.ms,
                      "bins": t.bins, "note": t.note} for t in tune.trials],
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=140)
    ap.add_argument("--plain", action="store_true", help="complex-of-real packing instead of MPCP")
    ap.add_argument("--unfused", action="store_true",
                    help="effective charge as patches (tred_effq), then tred_block_bin_rows, "
                         "instead of straight into the bins (tred_effq_bin)")
    ap.add_argument("--scratch-gb", type=float, default=None,
                    help="bound on the convolution scratch (sets the bins per pass)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--workload", default="module", choices=["module", "plain-small"],
                    help="module: the benchmark event; plain-small: the 1,000-segment event")
    ap.add_argument("--events", type=int, default=64, help="events of the batched form")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="device memory of a chunk")
    ap.add_argument("--chunk-bins", type=int, default=512,
                    help="(event, bin) pairs per chunk of the batched form (at least one event)")
    ap.add_argument("--pass-gb", type=float, default=None,
                    help="convolution scratch per pass (default: one pass per --chunk-bins)")
    ap.add_argument("--form", default="fft",
                    choices=["fft", "direct-split", "direct-bf16", "batched", "adjoint"],
                    help="fft: the benchmark line; direct-*: block-direct convolution on BF16 "
                         "matrix cores beside the FFT path; batched: 64 events; adjoint: "
                         "forward + gradient on the differentiation workload (separate lines)")
    ap.add_argument("--direct-bins", type=int, default=8,
                    help="module-event bins timed by the direct forms")
    args = ap.parse_args()
    if args.scratch_gb is None:
        from paper_2602_12052_amd import tred as _t
        args.scratch_gb = _t.DEFAULT_CONV_SCRATCH / 1e9

    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the path is "
              f"single-GPU; sharding over several GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        n = 1 << 30
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}))
        return

    if args.form == "batched":
        bench_batched(args)
        return
    if args.form == "adjoint":
        bench_adjoint(args)
        return
    if args.form != "fft":
        bench_direct(args, args.form == "direct-split")
        return

    import workloads as W
    from paper_2602_12052_amd import tred

    cfg = W.cfg_module(args.seed) if args.workload == "module" else W.cfg_plain_small(args.seed)
    seg = W.gen_segments(cfg)
    resp = W.synthetic_response(cfg.kpix, cfg.grid.sub, cfg.kticks)
    dev_seg = torch.from_numpy(seg).cuda()
    dev_resp = torch.from_numpy(resp).cuda()
    mpcp = not args.plain
    val_cap, block_cap, pix_cap = tred.size_event(cfg.grid, cfg.physics, cfg.blocking, cfg.kpix,
                                                  dev_seg)
    Bx, By = cfg.blocking.blk_pix
    Bt = cfg.blocking.blk_ticks
    fs, ft = cfg.fft[0], cfg.fft[2]
    nc = -(-cfg.kticks // (ft - Bt))
    box, boy = Bx + cfg.kpix[0] - 1, By + cfg.kpix[1] - 1
    batch = tred.conv_batch(cfg.grid, cfg.blocking, cfg.kpix, cfg.kticks, cfg.fft, mpcp, block_cap,
                            args.scratch_gb * 1e9)
    fused = not args.unfused
    pl = tred.Pipeline(cfg.grid, cfg.physics, cfg.blocking, cfg.kpix, cfg.kticks, dev_resp,
                       seg.shape[0], val_cap, block_cap, pix_cap, cfg.fft, mpcp, batch,
                       fused=fused)
    stream = torch.cuda.current_stream().cuda_stream
    ev = HipEvents(12)
    pl.plan.set_timing(ev.handles(range(6, 12)))
    print(f"# module event: {seg.shape[0]} depositions, {block_cap} active bins of "
          f"{tred.tred_block_count(cfg.grid, cfg.blocking)}, patch cells {val_cap}, "
          f"bins per conv pass {batch}", file=sys.stderr, flush=True)

    def step(record=False):
        if record:
            ev.record(0, stream)
        tred.tred_effq_windows(pl.grid, pl.phys, dev_seg, pl.fp, pl.off, stream)
        pl.charge_sum.zero_()
        if fused:
            if record:
                ev.record(1, stream)
            tred.tred_effq_bin(pl.grid, pl.phys, pl.blocking, dev_seg, pl.fp, pl.keys, pl.n_active,
                               pl.blocks, pl.rows, pl.bin_work, pl.charge_sum, stream)
        else:
            tred.tred_effq(pl.grid, pl.phys, dev_seg, pl.fp, pl.off, pl.val, pl.charge_sum, stream)
            if record:
                ev.record(1, stream)
            tred.tred_block_bin_rows(pl.grid, pl.blocking, pl.fp, pl.off, pl.val, pl.keys,
                                     pl.n_active, pl.blocks, pl.rows, pl.bin_work, stream)
        if record:
            ev.record(2, stream)
        tred.tred_block_conv_rows(pl.plan, pl.n_active, pl.blocks, pl.rows, pl.out_blocks, stream)
        if record:
            ev.record(3, stream)
        tred.tred_scatter_waveforms(pl.plan, pl.keys, pl.n_active, pl.out_blocks, pl.pix,
                                    pl.n_pix, pl.wf, pl.scat_work, stream)
        if record:
            ev.record(4, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    per_step, stages, conv_stages = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(record=True)
        per_step.append(ev.ms(0, 4))
        stages.append([ev.ms(0, 1), ev.ms(1, 2), ev.ms(2, 3), ev.ms(3, 4)])
        conv_stages.append([ev.ms(6, 7), ev.ms(8, 9), ev.ms(10, 11)])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    n_dep = seg.shape[0]
    n_bins_total = tred.tred_block_count(cfg.grid, cfg.blocking)
    n_act = int(pl.n_active.item())
    n_pix = int(pl.n_pix.item())
    ms_per_step = 1e3 * wall / args.steps
    value = n_dep / (wall / args.steps)
    stages = np.array(stages)
    conv_stages = np.array(conv_stages)

    fl = conv_flops_per_block((Bx, By, Bt), cfg.grid.sub, cfg.kpix, cfg.kticks, cfg.fft, mpcp)
    sp_blocks = min(batch, n_act)
    sp_ms = float(conv_stages[:, 1].mean())
    achieved = fl["sp"] * sp_blocks / (sp_ms * 1e-3) / 1e12
    sha = src_sha(KSPP_SOURCE)
    traffic = profile_traffic("k_spp", sha) if args.workload == "module" else None
    vblk = Bx * cfg.grid.sub[0] * By * cfg.grid.sub[1] * Bt
    vout = box * boy * (Bt + cfg.kticks - 1)
    lwf = cfg.grid.nticks + cfg.kticks - 1
    b_alg = 28 * n_dep + 4 * resp.size + 8 * n_act * vblk + 8 * n_act * vout + 4 * n_pix * lwf

    out = {
        "metric": "depositions/s (effq+block FFT conv) and % HBM roofline; rel-L2 vs FP64 oracle",
        "value": value,
        "unit": "depositions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("module-scale event: 1e5 line depositions (40 tracks at 0.5 mm steps + "
                         "20 shower blobs), 256x256 pixels x 6250 ticks, 10x10 impacts/pixel, "
                         "response 21x21 px x 2048 ticks, bins 16x16 px x 512 ticks"
                         if args.workload == "module" else
                         "1,000 line segments in 32x32 pixels x 6250 ticks, 10x10 impacts/pixel, "
                         "response 5x5 px x 200 ticks, bins 4x4 px x 128 ticks"),
            "n_dep": n_dep, "active_bins": n_act, "bins_total": n_bins_total,
            "active_fraction": n_act / n_bins_total, "pixels": n_pix,
            "fft": list(cfg.fft), "response_pieces": nc,
            "packing": "mirror-pair" if mpcp else "complex-of-real", "bins_per_conv_pass": batch,
            "effective_charge": "into the bins (tred_effq_bin)" if fused else
                                "patches (tred_effq), then tred_block_bin_rows",
        },
        "step_ms": {"p50": float(np.median(per_step)), "p99": float(np.percentile(per_step, 99))},
        "stage_ms": {("effq_windows" if fused else "effq_windows+effq"): float(stages[:, 0].mean()),
                     ("effq_bin" if fused else "block_bin"): float(stages[:, 1].mean()),
                     "block_conv": float(stages[:, 2].mean()), "scatter": float(stages[:, 3].mean()),
                     "conv_time_fwd": float(conv_stages[:, 0].mean()),
                     "conv_space_mac": float(conv_stages[:, 1].mean()),
                     "conv_time_inv": float(conv_stages[:, 2].mean())},
        "roofline": {
            "kernel": ("k_spp<40,8,16,2,4>" if args.workload == "module" else "k_spp<8,8,4,1,2>") +
                      " (spatial transforms + spectral multiply-accumulate)",
            "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
            "flops_per_launch": fl["sp"] * sp_blocks, "avg_launch_ms": sp_ms,
        },
        "hbm": {"algorithmic_bytes_per_step": b_alg,
                "frac_of_peak_per_step": b_alg / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9)},
        "charge_sum_fp64": float(pl.charge_sum.item()),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, seg, resp, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

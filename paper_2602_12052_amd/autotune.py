"""Autotuner for the bin shape and FFT sizes of the convolution.

The paper (Sec. III-B and its bin-size study) chooses the bin shape by measurement:
small bins waste less volume on empty cells but convolve more overlapping output
halos, and the FFT length trades transform work against the number of response
pieces. This tuner times the whole path (effective charge, binning, convolution,
overlap-add) on a sample event for each candidate that fits a memory budget and
returns the fastest. All arithmetic runs in the library; this module only creates
plans, allocates buffers and times calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

from . import tred

# (blk_pix, blk_ticks, fft) candidates; fft = (fs, fs, ft). Spatial sizes 32, 40 and 48
# (the smallest that hold blk_pix + kpix - 1 for a 21-pixel response, and one larger),
# bins of 8 to 28 pixels and of 256, 512 and 1024 ticks with time transforms of 1024 or
# 2048 points.
DEFAULT_CANDIDATES: Tuple[Tuple[int, int, Tuple[int, int, int]], ...] = (
    (16, 512, (40, 40, 1024)),
    (16, 512, (48, 48, 1024)),
    (16, 256, (40, 40, 1024)),
    (16, 1024, (40, 40, 2048)),
    (8, 512, (32, 32, 1024)),
    (8, 256, (40, 40, 1024)),
    (24, 512, (48, 48, 1024)),
    (28, 512, (48, 48, 1024)),
    (24, 1024, (48, 48, 2048)),
)


@dataclass
class Trial:
    blk_pix: int
    blk_ticks: int
    fft: Tuple[int, int, int]
    ms: Optional[float] = None          # median time of the whole path on the sample
    bins: Optional[int] = None
    bytes: Optional[int] = None         # device bytes of blocks, outputs and scratch
    note: str = ""


@dataclass
class TuneResult:
    best: Trial
    trials: List[Trial] = field(default_factory=list)

    def blocking(self, W):
        return W.Blocking((self.best.blk_pix, self.best.blk_pix), self.best.blk_ticks)


def _bytes_per_bin(grid, blocking, kpix, kticks, fft, mpcp):
    g, b = tred.grid_struct(grid), tred.blocking_struct(blocking)
    vblk = b.blk_pix[0] * g.sub[0] * b.blk_pix[1] * g.sub[1] * b.blk_ticks
    vout = (b.blk_pix[0] + kpix[0] - 1) * (b.blk_pix[1] + kpix[1] - 1) * (b.blk_ticks + kticks - 1)
    w1 = tred.plan_workspace_bytes(grid, blocking, kpix, kticks, fft, mpcp, 1 << 16)
    w2 = tred.plan_workspace_bytes(grid, blocking, kpix, kticks, fft, mpcp, 1 << 17)
    return 4 * (vblk + vout), (w2 - w1) // (1 << 16)


def tune(grid, phys, kpix, kticks, resp, seg, mpcp: bool = True,
         candidates: Sequence = DEFAULT_CANDIDATES, budget_bytes: float = 200e9,
         reps: int = 2, make_blocking=None, log=None, fused: bool = True) -> TuneResult:
    """Time each candidate on the sample events `seg` (one device tensor, or a list of
    them: the score is the sum of the events' median times) and return the fastest.
    make_blocking(blk_pix, blk_ticks) builds a blocking object; fused: time the path
    with the effective charge added straight into the bins."""
    import torch
    samples = list(seg) if isinstance(seg, (list, tuple)) else [seg]
    trials = []
    for bp, bt, fft in candidates:
        tr = Trial(bp, bt, tuple(fft))
        trials.append(tr)
        blk = make_blocking(bp, bt)
        try:
            total, nbins, nbytes = 0.0, 0, 0
            for sd in samples:
                val_cap, bcap, pix_cap = tred.size_event(grid, phys, blk, kpix, sd)
                fixed, scratch = _bytes_per_bin(grid, blk, kpix, kticks, fft, mpcp)
                nb = tred.conv_batch(grid, blk, kpix, kticks, fft, mpcp, bcap,
                                     max(scratch, budget_bytes - fixed * bcap))
                nbins += bcap
                nbytes = max(nbytes, fixed * bcap + scratch * nb)
                if fixed * bcap + scratch > budget_bytes:
                    raise MemoryError
                pl = tred.Pipeline(grid, phys, blk, kpix, kticks, resp, sd.shape[0], val_cap, bcap,
                                   pix_cap, fft, mpcp, nb, fused=fused)
                pl.run(sd)
                torch.cuda.synchronize()
                ts = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    pl.run(sd)
                    torch.cuda.synchronize()
                    ts.append(1e3 * (time.perf_counter() - t0))
                total += sorted(ts)[len(ts) // 2]
                del pl
                torch.cuda.empty_cache()
            tr.ms, tr.bins, tr.bytes = total, nbins, nbytes
        except MemoryError:
            tr.note = "over the memory budget"
        except tred.TredError as e:
            tr.note = f"unsupported: {e}"
        if log:
            log(f"autotune: blk {bp}x{bp}x{bt} fft {fft}: "
                + (f"{tr.ms:.1f} ms, {tr.bins} bins" if tr.ms is not None else tr.note))
    ok = [t for t in trials if t.ms is not None]
    if not ok:
        raise RuntimeError("no autotune candidate ran")
    return TuneResult(min(ok, key=lambda t: t.ms), trials)


def plan_chunks(bins: Sequence[int], target: int) -> List[List[int]]:
    """Groups a batch's events into chunks (one HIP graph each) for latency.

    Events are taken smallest first (by active bins; ties keep their order) and a chunk
    closes before the event that would take it past `target` (event, bin) pairs; an
    event with more bins than that is a chunk of its own. An event completes when its
    chunk does, so small chunks of small events let latency follow event size, while
    the chunk target keeps each convolution launch large enough to fill the GPU
    (Sec. III-B batches and chunks events to bound memory; the order is this
    library's). Returns the event indices of each chunk, in the order to run them; the
    pipeline's capacity is the largest chunk's pair count."""
    if target < 1:
        raise ValueError("chunk target must be at least one (event, bin) pair")
    order = sorted(range(len(bins)), key=lambda e: int(bins[e]))
    chunks: List[List[int]] = []
    cur: List[int] = []
    n = 0
    for e in order:
        b = int(bins[e])
        if b < 0:
            raise ValueError("negative bin count")
        if cur and n + b > target:
            chunks.append(cur)
            cur, n = [], 0
        cur.append(e)
        n += b
    if cur:
        chunks.append(cur)
    return chunks

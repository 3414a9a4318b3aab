"""tred_block_bin_rows_noalloc (binning with row masks and no workspace: the library's
static per-device scratch) against tred_block_bin_rows with a caller workspace, on two
calls in a row through the C ABI, the second with a smaller event: keys, the bin count
and the row masks bit-exact, the marked rows of the blocks equal up to the order of the
FP32 atomic sums, and the call rejects a grid with more bins than its scratch holds.
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


def _bin_both(T, g, ph, blk, seg, cap):
    """Effective charge once, then the binning both ways into separate outputs (kept on
    the device)."""
    import torch
    sd = torch.from_numpy(np.ascontiguousarray(seg)).cuda()
    n = seg.shape[0]
    fp = torch.empty((n, 6), dtype=torch.int32, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    T.tred_effq_windows(g, ph, sd, fp, off)
    torch.cuda.synchronize()
    nval = int(off[-1].item())
    val = torch.empty(max(nval, 1), dtype=torch.float32, device="cuda")
    csum = torch.zeros(1, dtype=torch.float64, device="cuda")
    T.tred_effq(g, ph, sd, fp, off, val, csum)
    gs, bs = T.grid_struct(g), T.blocking_struct(blk)
    vblk = bs.blk_pix[0] * gs.sub[0] * bs.blk_pix[1] * gs.sub[1] * bs.blk_ticks
    nrw = T.tred_block_row_words(g, blk)
    out = []
    for noalloc in (False, True):
        keys = torch.full((cap, 3), -7, dtype=torch.int32, device="cuda")
        n_active = torch.full((1,), -7, dtype=torch.int32, device="cuda")
        # blocks pre-filled with NaN: the marked rows compared below must all be written
        blocks = torch.full((cap, vblk), float("nan"), dtype=torch.float32, device="cuda")
        rows = torch.full((cap, nrw), -1, dtype=torch.int32, device="cuda")
        if noalloc:
            T.tred_block_bin_rows_noalloc(g, blk, fp, off, val, keys, n_active, blocks, rows)
        else:
            work = torch.empty(max(4, T.tred_block_bin_workspace(g, blk)), dtype=torch.uint8,
                               device="cuda")
            T.tred_block_bin_rows(g, blk, fp, off, val, keys, n_active, blocks, rows, work)
        torch.cuda.synchronize()
        na = int(n_active.item())
        assert 0 < na <= cap, (na, cap)
        out.append(dict(na=na, keys=keys[:na].cpu().numpy(), rows=rows[:na],
                        blocks=blocks[:na].view(na, -1, bs.blk_ticks)))
    return out


def _compare(ref, got):
    import torch
    assert got["na"] == ref["na"]
    assert np.array_equal(got["keys"], ref["keys"])
    assert torch.equal(got["rows"], ref["rows"])
    na, nrows = ref["blocks"].shape[:2]
    r = torch.arange(nrows, device="cuda")
    marked = ((ref["rows"][:, r // 32] >> (r % 32)) & 1).bool()
    a = ref["blocks"][marked].double()
    b = got["blocks"][marked].double()
    assert bool(torch.isfinite(a).all()) and bool(torch.isfinite(b).all())
    rel = float(torch.linalg.norm(a - b) / torch.linalg.norm(a))
    # same sums, only the order of the FP32 atomic adds differs
    assert rel <= 1e-6, rel
    mx = float((a - b).abs().max())
    assert mx <= 1e-5 * float(a.abs().max()), mx
    return int(marked.sum()), rel


def test_noalloc_binning_matches_workspace_binning(T):
    """64x64 pixels (10x10 impacts) x 2,048 ticks in bins of 8x8 pixels x 128 ticks
    (1,024 bins); module-like events of 2,000 and then 300 depositions."""
    nticks = 2048
    h = W.PITCH / W.SUB
    g = W.Grid(origin=(0.0, 0.0, 0.0), spacing=(h, h, W.TICK), npix=(64, 64),
               sub=(W.SUB, W.SUB), nticks=nticks)
    ph = W.Physics(sigma_min=(0.5 * h, 0.5 * h, 0.5 * W.TICK))
    blk = W.Blocking((8, 8), 128)
    nb = T.tred_block_count(g, blk)
    zmax = nticks * W.TICK * ph.v_drift
    for n in (2000, 300):
        seg = W.gen_module_event(n, (64 * W.PITCH, 64 * W.PITCH), z_max=zmax, n_tracks=6,
                                 n_blobs=4, seed=17 + n)
        say(f"noalloc binning: {n} depositions, 64x64 pixels x {nticks} ticks, {nb} bins of "
            f"8x8 px x 128 ticks")
        ref, got = _bin_both(T, g, ph, blk, seg, cap=nb)
        m, rel = _compare(ref, got)
        say(f"  {ref['na']} active bins, {m} marked rows, blocks rel-L2 {rel:.1e}")
        del ref, got


def test_noalloc_rejects_too_many_bins(T):
    """A grid with more bins than the static scratch holds is refused on the host."""
    import torch
    g = W.Grid(origin=(0.0, 0.0, 0.0), spacing=(0.044, 0.044, W.TICK), npix=(1024, 1024),
               sub=(1, 1), nticks=64 * 64)
    blk = W.Blocking((1, 1), 64)
    assert T.tred_block_count(g, blk) > (1 << 18)
    with pytest.raises(T.TredError, match="static scratch"):
        T.tred_block_bin_rows_noalloc(g, blk, torch.zeros((0, 6), dtype=torch.int32, device="cuda"),
                                      torch.zeros(1, dtype=torch.int64, device="cuda"),
                                      torch.zeros(1, dtype=torch.float32, device="cuda"),
                                      torch.zeros((1, 3), dtype=torch.int32, device="cuda"),
                                      torch.zeros(1, dtype=torch.int32, device="cuda"),
                                      torch.zeros((1, 64), dtype=torch.float32, device="cuda"),
                                      torch.zeros((1, 1), dtype=torch.int32, device="cuda"))

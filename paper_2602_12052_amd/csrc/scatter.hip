// Overlap-add of the block outputs onto unique electrodes (Sec. III-B: reduction of
// overlapping outputs by summation; Fig. 1, "bin & accumulate on unique electrodes").
// Each waveform sample gathers the outputs of the (at most a few) active bins whose
// output footprint covers it, so every sample is written once, without atomics.
#include <algorithm>

#include "tred_internal.hpp"
#include "validate.hpp"

namespace {

struct ScatArgs {
    int32_t npx, npy, Bx, By, Bt, hx, hy, kt;
    int32_t nb[3];
    int32_t box, boy, bot;
    int32_t lwf;        // waveform length nticks + kticks - 1
    int32_t cap, pix_cap;
    int64_t vout;
    int32_t nev, kst;   // events in the batch; key stride (3, or 4 with the event first)
};

__global__ void k_fill(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// per active bin: mark the pixels of its output footprint, record the bin's slot
__global__ __launch_bounds__(256) void k_mark_pix(ScatArgs S, const int32_t* __restrict__ keys,
                                                  const int32_t* __restrict__ n_active,
                                                  int32_t* __restrict__ pmap,
                                                  int32_t* __restrict__ bmap) {
    const int na = min(*n_active, S.cap);
    const int64_t nbins = (int64_t)S.nb[0] * S.nb[1] * S.nb[2];
    const int64_t npix = (int64_t)S.npx * S.npy;
    for (int i = blockIdx.x; i < na; i += gridDim.x) {
        const int32_t* k = keys + (int64_t)S.kst * i;
        const int e = S.kst == 4 ? *k++ : 0;
        const int bx = k[0], by = k[1], bt = k[2];
        if (threadIdx.x == 0) bmap[e * nbins + ((int64_t)bx * S.nb[1] + by) * S.nb[2] + bt] = i;
        const int x0 = max(0, bx * S.Bx - S.hx), x1 = min(S.npx - 1, bx * S.Bx + S.Bx - 1 + S.hx);
        const int y0 = max(0, by * S.By - S.hy), y1 = min(S.npy - 1, by * S.By + S.By - 1 + S.hy);
        const int ny = y1 - y0 + 1;
        const int cnt = (x1 - x0 + 1) * ny;
        for (int c = threadIdx.x; c < cnt; c += blockDim.x)
            pmap[e * npix + (int64_t)(x0 + c / ny) * S.npy + (y0 + c % ny)] = 1;
    }
}

__device__ __forceinline__ int wave_incl_scan_i32(int v, int lane) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// compaction of the marked pixels in id order: pix list, pmap -> slot or -1, n_pix
__global__ __launch_bounds__(1024) void k_compact_pix(ScatArgs S, int32_t* __restrict__ pmap,
                                                      int32_t* __restrict__ pix,
                                                      int32_t* __restrict__ n_pix) {
    __shared__ int wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tot = (int64_t)S.nev * S.npx * S.npy;
    int carry = 0;
    for (int64_t base = 0; base < tot; base += 1024) {
        const int64_t i = base + tid;
        const int f = (i < tot && pmap[i] != 0) ? 1 : 0;
        const int incl = wave_incl_scan_i32(f, lane);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        if (wave == 0) {
            int t = lane < 16 ? wsum[lane] : 0;
            t = wave_incl_scan_i32(t, lane);
            if (lane < 16) wsum[lane] = t;
        }
        __syncthreads();
        const int slot = carry + incl - f + (wave > 0 ? wsum[wave - 1] : 0);
        if (i < tot) {
            if (f && slot < S.pix_cap) pix[slot] = (int32_t)i;
            pmap[i] = (f && slot < S.pix_cap) ? slot : -1;
        }
        carry += wsum[15];
        __syncthreads();
    }
    if (tid == 0) *n_pix = carry;
}

// One workgroup per pixel slot (slots at or past n_pix get a zero waveform). Its threads
// walk the waveform in spans of kGatherSpan ticks (kGatherSpan / 256 per thread), so the
// pixel's bin lookups are made once per span. Per
// sample the covering bins are summed in (bx, by, bt) order. The loads carry no
// branches, so a thread keeps the loads of four bins in flight: each block-output row
// is read through a buffer resource of its own length (ticks outside it read zero),
// and the bin slots of a column are loaded once per wave (one per lane); the active
// ones are found by a ballot and taken with readlane.
#ifndef TRED_GATHER_SPAN
#define TRED_GATHER_SPAN 2048
#endif
constexpr int kGatherSpan = TRED_GATHER_SPAN;

__global__ __launch_bounds__(256) void k_gather(ScatArgs S, const int32_t* __restrict__ pix,
                                                const int32_t* __restrict__ n_pix,
                                                const int32_t* __restrict__ bmap,
                                                const float* __restrict__ outb,
                                                float* __restrict__ wf) {
    const int slot = blockIdx.x;
    if (slot >= min(*n_pix, S.pix_cap)) {
        // slots without a pixel hold a zero waveform, so every row of wf is defined
        float* zrow = wf + (int64_t)slot * S.lwf;
        for (int T = threadIdx.x; T < S.lwf; T += 256) zrow[T] = 0.0f;
        return;
    }
    const int64_t npix = (int64_t)S.npx * S.npy;
    const int e = (int)(pix[slot] / npix);
    const int p = (int)(pix[slot] % npix);
    const int px = p / S.npy, py = p % S.npy;
    const int lane = threadIdx.x & (kWave - 1);
    bmap += e * (int64_t)S.nb[0] * S.nb[1] * S.nb[2];
    // bins whose output footprint contains this pixel: b*B - h <= p <= b*B + B - 1 + h
    const int bx0 = max(0, (px - S.hx - S.Bx + 1 + S.Bx * 4096) / S.Bx - 4096);
    const int bx1 = min(S.nb[0] - 1, (px + S.hx) / S.Bx);
    const int by0 = max(0, (py - S.hy - S.By + 1 + S.By * 4096) / S.By - 4096);
    const int by1 = min(S.nb[1] - 1, (py + S.hy) / S.By);
    constexpr int NJ = kGatherSpan / 256;
    const uint32_t rowb = (uint32_t)S.bot * 4u;
    float* wrow = wf + (int64_t)slot * S.lwf;
    for (int T0 = 0; T0 < S.lwf; T0 += kGatherSpan) {
        // bins whose ticks [bt Bt, bt Bt + bot) meet [T0, T0 + span)
        const int bt0 = max(0, (T0 - S.bot + 1 + S.Bt * 4096) / S.Bt - 4096);
        const int bt1 = min(S.nb[2] - 1, (T0 + kGatherSpan - 1) / S.Bt);
        float acc[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[j] = 0.0f;
        for (int bx = bx0; bx <= bx1; ++bx)
            for (int by = by0; by <= by1; ++by) {
                const int qx = px - bx * S.Bx + S.hx, qy = py - by * S.By + S.hy;
                if (qx < 0 || qx >= S.box || qy < 0 || qy >= S.boy) continue;
                const int32_t* bcol = bmap + ((int64_t)bx * S.nb[1] + by) * S.nb[2];
                const int64_t qoff = ((int64_t)qx * S.boy + qy) * S.bot;
                for (int c0 = bt0; c0 <= bt1; c0 += kWave) {
                    const int nc = min(kWave, bt1 - c0 + 1);
                    const int vb = lane < nc ? bcol[c0 + lane] : -1;
                    // the active bins of the column (lanes with a slot), in bt order, four
                    // at a time: their loads in flight together, then the adds in bin order
                    uint64_t live = __builtin_amdgcn_ballot_w64(vb >= 0);
                    while (live != 0) {
                        float v[4][NJ];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int k = live != 0 ? (int)__builtin_ctzll(live) : 0;
                            const bool use = live != 0;
                            live &= live - 1;   // (no-op once empty)
                            const int b = use ? __builtin_amdgcn_readlane(vb, k) : -1;
                            const auto rr = buf_rsrc(outb + (int64_t)max(b, 0) * S.vout + qoff,
                                                     b < 0 ? 0u : rowb);
                            // tick within the row (negative ticks wrap past the end: zero)
                            const uint32_t tb =
                                (uint32_t)(T0 + (int)threadIdx.x - (c0 + k) * S.Bt) * 4u;
#pragma unroll
                            for (int j = 0; j < NJ; ++j) v[u][j] = buf_f1(rr, tb + 1024u * j, 0u);
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int j = 0; j < NJ; ++j) acc[j] += v[u][j];
                    }
                }
            }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int T = T0 + (int)threadIdx.x + 256 * j;
            if (T < S.lwf) wrow[T] = acc[j];
        }
    }
}

// Transpose of the overlap-add: every block-output sample takes the waveform gradient
// of its pixel and tick; samples of pixels outside the region, of pixels without a
// slot below pix_cap, or past the waveform end get zero. One workgroup per (output
// bin, output pixel).
__global__ __launch_bounds__(256) void k_scatter_adj(ScatArgs S, const int32_t* __restrict__ keys,
                                                     const int32_t* __restrict__ n_active,
                                                     const int32_t* __restrict__ pix,
                                                     const int32_t* __restrict__ n_pix,
                                                     const float* __restrict__ dwf,
                                                     float* __restrict__ dout) {
    const int b = blockIdx.x, q = blockIdx.y;
    if (b >= min(*n_active, S.cap)) return;
    const int32_t* k = keys + (int64_t)S.kst * b;
    const int e = S.kst == 4 ? k[0] : 0;
    const int32_t* kb = k + (S.kst == 4 ? 1 : 0);
    const int qx = q / S.boy, qy = q % S.boy;
    const int px = kb[0] * S.Bx - S.hx + qx, py = kb[1] * S.By - S.hy + qy;
    int slot = -1;
    if (px >= 0 && px < S.npx && py >= 0 && py < S.npy) {
        const int32_t id = (int32_t)(e * ((int64_t)S.npx * S.npy) + (int64_t)px * S.npy + py);
        int lo = 0, hi = min(*n_pix, S.pix_cap) - 1;
        while (lo <= hi) {                       // pix is ascending
            const int mid = (lo + hi) >> 1;
            const int32_t v = pix[mid];
            if (v == id) { slot = mid; break; }
            if (v < id) lo = mid + 1;
            else hi = mid - 1;
        }
    }
    float* row = dout + (int64_t)b * S.vout + (int64_t)q * S.bot;
    const int T0 = kb[2] * S.Bt;
    const float* w = dwf + (int64_t)(slot < 0 ? 0 : slot) * S.lwf;
    for (int t = threadIdx.x; t < S.bot; t += blockDim.x) {
        const int T = T0 + t;
        row[t] = (slot >= 0 && T < S.lwf) ? w[T] : 0.0f;
    }
}

ScatArgs make_sargs(const tred_conv_plan* P) {
    ScatArgs S;
    S.npx = P->grid.npix[0];
    S.npy = P->grid.npix[1];
    S.Bx = P->blk.blk_pix[0];
    S.By = P->blk.blk_pix[1];
    S.Bt = P->blk.blk_ticks;
    S.hx = (P->kpix[0] - 1) / 2;
    S.hy = (P->kpix[1] - 1) / 2;
    S.kt = P->kticks;
    for (int a = 0; a < 3; ++a) S.nb[a] = nblk_axis(&P->grid, &P->blk, a);
    S.box = P->bo[0];
    S.boy = P->bo[1];
    S.bot = P->bo[2];
    S.lwf = P->grid.nticks + P->kticks - 1;
    S.vout = (int64_t)S.box * S.boy * S.bot;
    S.nev = 1;
    S.kst = 3;
    return S;
}

int64_t scatter_workspace(const tred_conv_plan* P, int32_t nev) {
    const int64_t nbt = (int64_t)nblk_axis(&P->grid, &P->blk, 0) * nblk_axis(&P->grid, &P->blk, 1) *
                        nblk_axis(&P->grid, &P->blk, 2);
    return ((int64_t)P->grid.npix[0] * P->grid.npix[1] + nbt) * 4 * nev;
}

tred_status scatter(const tred_conv_plan* P, int32_t nev, int32_t kst, const int32_t* keys,
                    const int32_t* n_active, int32_t cap, const float* out_blocks, int32_t* pix,
                    int32_t* n_pix, float* wf, int32_t pix_cap, void* work, void* stream) {
    TRED_REQUIRE(P && n_active && n_pix && work, "plan/n_active/n_pix/work is NULL");
    TRED_REQUIRE(cap >= 0 && pix_cap >= 0, "capacities must be >= 0");
    TRED_REQUIRE(cap == 0 || (keys && out_blocks), "keys/out_blocks is NULL");
    TRED_REQUIRE(pix_cap == 0 || (pix && wf), "pix/wf is NULL");
    TRED_REQUIRE((int64_t)nev * P->grid.npix[0] * P->grid.npix[1] < INT32_MAX,
                 "too many (event, pixel) pairs");
    hipStream_t st = (hipStream_t)stream;
    ScatArgs S = make_sargs(P);
    S.cap = cap;
    S.pix_cap = pix_cap;
    S.nev = nev;
    S.kst = kst;
    int32_t* pmap = (int32_t*)work;
    const int64_t npix_tot = (int64_t)nev * S.npx * S.npy;
    int32_t* bmap = pmap + npix_tot;
    const int64_t nbt = (int64_t)nev * S.nb[0] * S.nb[1] * S.nb[2];
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>((npix_tot + 255) / 256, 4096)),
                       dim3(256), 0, st, pmap, npix_tot, 0);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>((nbt + 255) / 256, 4096)), dim3(256),
                       0, st, bmap, nbt, -1);
    if (cap > 0)
        hipLaunchKernelGGL(k_mark_pix, dim3((unsigned)std::min(cap, 65536)), dim3(256), 0, st, S,
                           keys, n_active, pmap, bmap);
    hipLaunchKernelGGL(k_compact_pix, dim3(1), dim3(1024), 0, st, S, pmap, pix, n_pix);
    TRED_TRY(tred_check_launch("tred_scatter_waveforms compact"));
    if (pix_cap > 0)
        hipLaunchKernelGGL(k_gather, dim3(pix_cap), dim3(256), 0, st, S, pix, n_pix, bmap,
                           out_blocks, wf);
    return tred_check_launch("tred_scatter_waveforms");
}

}  // namespace

extern "C" int64_t tred_scatter_workspace(const tred_conv_plan* P) {
    if (!P) return -1;
    return scatter_workspace(P, 1);
}

extern "C" tred_status tred_scatter_waveforms(const tred_conv_plan* P, const int32_t* keys,
                                              const int32_t* n_active, int32_t cap,
                                              const float* out_blocks, int32_t* pix, int32_t* n_pix,
                                              float* wf, int32_t pix_cap, void* work,
                                              void* stream) {
    return scatter(P, 1, 3, keys, n_active, cap, out_blocks, pix, n_pix, wf, pix_cap, work, stream);
}

extern "C" tred_status tred_scatter_waveforms_adjoint(const tred_conv_plan* P, const int32_t* keys,
                                                      const int32_t* n_active, int32_t cap,
                                                      const int32_t* pix, const int32_t* n_pix,
                                                      int32_t pix_cap, const float* d_wf,
                                                      float* d_out_blocks, void* stream) {
    TRED_REQUIRE(P && n_active && n_pix, "plan/n_active/n_pix is NULL");
    TRED_REQUIRE(cap >= 0 && pix_cap >= 0, "capacities must be >= 0");
    if (cap == 0) return TRED_OK;
    TRED_REQUIRE(keys && d_out_blocks, "keys/d_out_blocks is NULL");
    TRED_REQUIRE(pix_cap == 0 || (pix && d_wf), "pix/d_wf is NULL");
    ScatArgs S = make_sargs(P);
    S.cap = cap;
    S.pix_cap = pix_cap;
    hipStream_t st = (hipStream_t)stream;
    TRED_REQUIRE(S.box * S.boy <= 65535, "output block of %d pixels", S.box * S.boy);
    hipLaunchKernelGGL(k_scatter_adj, dim3(cap, S.box * S.boy), dim3(256), 0, st, S, keys, n_active,
                       pix, n_pix, d_wf, d_out_blocks);
    return tred_check_launch("tred_scatter_waveforms_adjoint");
}

extern "C" int64_t tred_scatter_events_workspace(const tred_conv_plan* P, int32_t n_ev) {
    if (!P || n_ev <= 0) return -1;
    return scatter_workspace(P, n_ev);
}

extern "C" tred_status tred_scatter_waveforms_events(const tred_conv_plan* P, int32_t n_ev,
                                                     const int32_t* keys, const int32_t* n_active,
                                                     int32_t cap, const float* out_blocks,
                                                     int32_t* pix, int32_t* n_pix, float* wf,
                                                     int32_t pix_cap, void* work, void* stream) {
    TRED_REQUIRE(n_ev > 0, "n_ev must be > 0");
    return scatter(P, n_ev, 4, keys, n_active, cap, out_blocks, pix, n_pix, wf, pix_cap, work,
                   stream);
}

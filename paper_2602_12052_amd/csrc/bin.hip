// Block-sparse binned tensor (Sec. III-B): active bins, their keys and the dense
// charge of each active bin, reduced over overlapping deposition patches. A batch
// of events shares one binned tensor: the event index leads the bin key, so the
// (event, bin) pairs of all events form one list of independent blocks.
#include <mutex>

#include "tred_internal.hpp"
#include "validate.hpp"

// Bin -> slot map of tred_block_bin_rows_noalloc: a fixed array in device memory (one
// copy per device, held until the process ends) instead of a caller workspace. Host
// code never passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): it looks the address up once per device and passes that.
constexpr int64_t kNoallocMaxBins = 1 << 18;  // 1 MiB of int32 slots
static __device__ __align__(256) int32_t scratch[kNoallocMaxBins];

namespace {

constexpr int kMaxDevices = 64;

// device address of `scratch` on the current device (looked up on a device's first call)
tred_status noalloc_scratch(int32_t** out) {
    static std::mutex mu;
    static int32_t* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return tred_fail(TRED_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return tred_fail(TRED_EUNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                         kMaxDevices);
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return tred_fail(TRED_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                             hipGetErrorString(e));
        addr[dev] = (int32_t*)p;
    }
    *out = addr[dev];
    return TRED_OK;
}

struct BinGeom {
    int32_t bf[3];   // bin extent in fine cells
    int32_t nb[3];   // bins per axis
    int64_t vblk;    // cells per bin
    int32_t nev;     // events in the batch
    int32_t kst;     // key stride: 3 (bx, by, bt) or 4 (event, bx, by, bt)
    int64_t nbins;   // bins per event
};

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// every bin touched by a footprint box gets flag 1
__global__ __launch_bounds__(256) void k_mark(BinGeom G, int64_t n, const int32_t* __restrict__ fp,
                                              const int64_t* __restrict__ ev_off,
                                              int32_t* __restrict__ flag) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const int32_t* f = fp + 6 * d;
    if (f[3] < f[0] || f[4] < f[1] || f[5] < f[2]) return;
    flag += (int64_t)event_of(d, ev_off, G.nev) * G.nbins;
    for (int bx = f[0] / G.bf[0]; bx <= f[3] / G.bf[0]; ++bx)
        for (int by = f[1] / G.bf[1]; by <= f[4] / G.bf[1]; ++by)
            for (int bt = f[2] / G.bf[2]; bt <= f[5] / G.bf[2]; ++bt)
                flag[((int64_t)bx * G.nb[1] + by) * G.nb[2] + bt] = 1;
}

__device__ __forceinline__ int wave_incl_scan_i32(int v, int lane) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// Stream compaction of the flags in bin order (one workgroup): flag -> slot or -1,
// keys of active bins in ascending order, count of active bins.
__global__ __launch_bounds__(1024) void k_compact(BinGeom G, int32_t* __restrict__ flag,
                                                  int32_t* __restrict__ keys,
                                                  int32_t* __restrict__ n_active, int32_t cap) {
    __shared__ int wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tot = (int64_t)G.nev * G.nbins;
    int carry = 0;
    for (int64_t base = 0; base < tot; base += 1024) {
        const int64_t i = base + tid;
        const int f = (i < tot && flag[i] != 0) ? 1 : 0;
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
            if (f && slot < cap) {
                const int64_t e = i / G.nbins, b = i % G.nbins;
                int32_t* k = keys + (int64_t)G.kst * slot;
                if (G.kst == 4) *k++ = (int32_t)e;
                k[0] = (int32_t)(b / ((int64_t)G.nb[1] * G.nb[2]));
                k[1] = (int32_t)((b / G.nb[2]) % G.nb[1]);
                k[2] = (int32_t)(b % G.nb[2]);
            }
            flag[i] = (f && slot < cap) ? slot : -1;
        }
        carry += wsum[15];
        __syncthreads();
    }
    if (tid == 0) *n_active = carry;
}

// zero the first min(n_active, cap) bins
__global__ __launch_bounds__(256) void k_zero_blocks(float4* __restrict__ blocks,
                                                     const int32_t* __restrict__ n_active,
                                                     int32_t cap, int64_t vblk) {
    const int64_t na = min(*n_active, cap);
    const int64_t n4 = na * vblk / 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        blocks[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ __launch_bounds__(256) void k_zero_tail(float* __restrict__ blocks,
                                                   const int32_t* __restrict__ n_active,
                                                   int32_t cap, int64_t vblk) {
    const int64_t na = min(*n_active, cap);
    const int64_t n = na * vblk;
    const int64_t i = (n / 4) * 4 + threadIdx.x;
    if (i < n) blocks[i] = 0.f;
}

// Row masks: bit r of bin s (word s * nrw + r / 32) is set when row r = x * bf[1] + y
// (the bf[2] ticks of fine cell (x, y) of the bin) meets a footprint box. One
// workgroup per deposition; a task is one x column of one (bin y, bin t) pair, and
// sets the bits of the column's y range word by word.
__global__ __launch_bounds__(256) void k_mark_rows(BinGeom G, int64_t n, const int32_t* __restrict__ fp,
                                                   const int64_t* __restrict__ ev_off,
                                                   const int32_t* __restrict__ slot_all, int nrw,
                                                   uint32_t* __restrict__ rows) {
    for (int64_t d = blockIdx.x; d < n; d += gridDim.x) {
        const int32_t* f = fp + 6 * d;
        if (f[3] < f[0] || f[4] < f[1] || f[5] < f[2]) continue;
        const int32_t* slot = slot_all + (int64_t)event_of(d, ev_off, G.nev) * G.nbins;
        const int nx = f[3] - f[0] + 1;
        const int by0 = f[1] / G.bf[1], nby = f[4] / G.bf[1] - by0 + 1;
        const int bt0 = f[2] / G.bf[2], nbt = f[5] / G.bf[2] - bt0 + 1;
        for (int i = threadIdx.x; i < nx * nby * nbt; i += blockDim.x) {
            const int ix = i % nx, r = i / nx;
            const int by = by0 + r % nby, bt = bt0 + r / nby;
            const int gx = f[0] + ix, bx = gx / G.bf[0];
            const int s = slot[((int64_t)bx * G.nb[1] + by) * G.nb[2] + bt];
            if (s < 0) continue;
            const int y0 = max(f[1], by * G.bf[1]) - by * G.bf[1];
            const int y1 = min(f[4], by * G.bf[1] + G.bf[1] - 1) - by * G.bf[1];
            const int r0 = (gx - bx * G.bf[0]) * G.bf[1] + y0, r1 = r0 + (y1 - y0);
            uint32_t* w = rows + (int64_t)s * nrw;
            for (int k = r0 >> 5; k <= r1 >> 5; ++k) {
                const int lo = max(r0, k * 32) - k * 32, hi = min(r1, k * 32 + 31) - k * 32;
                const uint32_t m = (hi - lo == 31) ? 0xffffffffu : (((1u << (hi - lo + 1)) - 1u) << lo);
                atomicOr(w + k, m);
            }
        }
    }
}

// zero the marked rows of the first min(n_active, cap) bins: one wave per mask word
__global__ __launch_bounds__(256) void k_zero_rows(float* __restrict__ blocks,
                                                   const uint32_t* __restrict__ rows,
                                                   const int32_t* __restrict__ n_active, int32_t cap,
                                                   int64_t vblk, int nrw, int bt) {
    const int64_t na = min(*n_active, cap);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t w = (int64_t)blockIdx.x * 4 + wv; w < na * nrw; w += (int64_t)gridDim.x * 4) {
        const int64_t s = w / nrw;
        uint32_t bits = rows[w];
        float* base = blocks + s * vblk + (w - s * nrw) * 32 * (int64_t)bt;
        while (bits != 0u) {
            const int b = __builtin_ctz(bits);
            bits &= bits - 1u;
            float* row = base + (int64_t)b * bt;
            for (int k = lane; k < bt; k += kWave) row[k] = 0.0f;
        }
    }
}

// one workgroup per deposition: add its patch into the bins (FP32 atomics; the
// reduction order over overlapping patches is unspecified). A wave takes one patch row
// (fixed x, y: nt cells along t) at a time, so the row's bin column and offsets are
// found once per row; its lanes walk the row's ticks, the t bin advanced as they
// cross bin edges.
__global__ __launch_bounds__(256) void k_accum(BinGeom G, int64_t n, const int32_t* __restrict__ fp,
                                               const int64_t* __restrict__ off,
                                               const float* __restrict__ val, int64_t val_cap,
                                               const int64_t* __restrict__ ev_off,
                                               const int32_t* __restrict__ slot_all,
                                               float* __restrict__ blocks) {
    // the wave index is uniform over the wave: row set-up runs on the scalar unit
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave, nw = blockDim.x / kWave;
    for (int64_t d = blockIdx.x; d < n; d += gridDim.x) {
        const int32_t* f = fp + 6 * d;
        if (f[3] < f[0] || f[4] < f[1] || f[5] < f[2]) continue;
        if (off[d + 1] > val_cap) continue;
        const int32_t* slot = slot_all + (int64_t)event_of(d, ev_off, G.nev) * G.nbins;
        const int ny = f[4] - f[1] + 1, nt = f[5] - f[2] + 1;
        const int nrow = (f[3] - f[0] + 1) * ny;
        const float* v = val + off[d];
        // t bin of this lane's first tick, and the first tick past that bin
        const int bt0 = (f[2] + lane) / G.bf[2];
        const int be0 = (bt0 + 1) * G.bf[2];
        for (int r = wv; r < nrow; r += nw) {
            const int ix = r / ny, iy = r - ix * ny;
            const int gx = f[0] + ix, gy = f[1] + iy;
            const int bx = gx / G.bf[0], by = gy / G.bf[1];
            const int32_t* scol = slot + ((int64_t)bx * G.nb[1] + by) * G.nb[2];
            float* brow = blocks + ((int64_t)(gx - bx * G.bf[0]) * G.bf[1] + (gy - by * G.bf[1])) * G.bf[2];
            const float* vrow = v + (int64_t)r * nt;
            int bt = bt0, be = be0;
            for (int t = lane; t < nt; t += kWave) {
                const int gt = f[2] + t;
                while (gt >= be) {
                    ++bt;
                    be += G.bf[2];
                }
                const float q = vrow[t];
                const int s = scol[bt];
                if (q == 0.0f || s < 0) continue;
                unsafeAtomicAdd(brow + (int64_t)s * G.vblk + (gt - (be - G.bf[2])), q);
            }
        }
    }
}

// Transpose of the binning: the slot of every active bin from the keys, then every
// patch cell takes the gradient of its bin's cell (zero where the bin is not held).
__global__ __launch_bounds__(256) void k_slots(BinGeom G, const int32_t* __restrict__ keys,
                                               const int32_t* __restrict__ n_active, int32_t cap,
                                               int32_t* __restrict__ slot) {
    const int na = min(*n_active, cap);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < na; s += gridDim.x * blockDim.x) {
        const int32_t* k = keys + (int64_t)G.kst * s;
        const int e = G.kst == 4 ? k[0] : 0;
        const int32_t* b = k + (G.kst == 4 ? 1 : 0);
        slot[(int64_t)e * G.nbins + ((int64_t)b[0] * G.nb[1] + b[1]) * G.nb[2] + b[2]] = s;
    }
}

__global__ __launch_bounds__(256) void k_accum_adj(BinGeom G, int64_t n, const int32_t* __restrict__ fp,
                                                   const int64_t* __restrict__ off, int64_t val_cap,
                                                   const int64_t* __restrict__ ev_off,
                                                   const int32_t* __restrict__ slot_all,
                                                   const float* __restrict__ dblocks,
                                                   float* __restrict__ dval) {
    // rows of the patch as in k_accum; cells past val_cap are not written
    // the wave index is uniform over the wave: row set-up runs on the scalar unit
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave, nw = blockDim.x / kWave;
    for (int64_t d = blockIdx.x; d < n; d += gridDim.x) {
        const int32_t* f = fp + 6 * d;
        if (f[3] < f[0] || f[4] < f[1] || f[5] < f[2]) continue;
        const int32_t* slot = slot_all + (int64_t)event_of(d, ev_off, G.nev) * G.nbins;
        const int ny = f[4] - f[1] + 1, nt = f[5] - f[2] + 1;
        const int nrow = (f[3] - f[0] + 1) * ny;
        const int64_t o0 = off[d], o1 = min(off[d + 1], val_cap);
        const bool kept = off[d + 1] <= val_cap;
        const int bt0 = (f[2] + lane) / G.bf[2];
        const int be0 = (bt0 + 1) * G.bf[2];
        for (int r = wv; r < nrow && o0 + (int64_t)r * nt < o1; r += nw) {
            const int ix = r / ny, iy = r - ix * ny;
            const int gx = f[0] + ix, gy = f[1] + iy;
            const int bx = gx / G.bf[0], by = gy / G.bf[1];
            const int32_t* scol = slot + ((int64_t)bx * G.nb[1] + by) * G.nb[2];
            const float* brow =
                dblocks + ((int64_t)(gx - bx * G.bf[0]) * G.bf[1] + (gy - by * G.bf[1])) * G.bf[2];
            float* drow = dval + o0 + (int64_t)r * nt;
            int bt = bt0, be = be0;
            for (int t = lane; t < nt; t += kWave) {
                const int gt = f[2] + t;
                while (gt >= be) {
                    ++bt;
                    be += G.bf[2];
                }
                if (o0 + (int64_t)r * nt + t >= o1) break;
                const int s = scol[bt];
                float g = 0.0f;
                if (kept && s >= 0) g = brow[(int64_t)s * G.vblk + (gt - (be - G.bf[2]))];
                drow[t] = g;
            }
        }
    }
}

// 32-bit words of the row mask of one bin (rows: bin cells along x and y)
int row_words(const BinGeom& G) { return (int)(((int64_t)G.bf[0] * G.bf[1] + 31) / 32); }

BinGeom geom(const tred_grid* g, const tred_blocking* b, int nev, int kst) {
    BinGeom G;
    G.bf[0] = b->blk_pix[0] * g->sub[0];
    G.bf[1] = b->blk_pix[1] * g->sub[1];
    G.bf[2] = b->blk_ticks;
    for (int a = 0; a < 3; ++a) G.nb[a] = nblk_axis(g, b, a);
    G.vblk = (int64_t)G.bf[0] * G.bf[1] * G.bf[2];
    G.nev = nev;
    G.kst = kst;
    G.nbins = (int64_t)G.nb[0] * G.nb[1] * G.nb[2];
    return G;
}

// The effective charge computed inside the binning (instead of patches off/val)
struct FusedEffq {
    const tred_physics* phys;
    const float* seg;
    double* charge_sum;
};

// rows NULL: every bin is zeroed whole; otherwise the row masks are written and only
// the marked rows of each bin are zeroed (the other rows are left as they were).
// fz non-NULL: the effective charge of the depositions is added into the bins by the
// effective-charge kernel itself (off, val and val_cap are not used).
tred_status block_bin(const tred_grid* grid, const tred_blocking* blocking, int32_t n_ev,
                      const int64_t* ev_off, int64_t n_dep, const int32_t* fp, const int64_t* off,
                      const float* val, int64_t val_cap, int32_t* keys, int32_t* n_active,
                      float* blocks, uint32_t* rows, int32_t cap, void* work, void* stream,
                      const FusedEffq* fz = nullptr) {
    TRED_TRY(validate_grid(grid));
    TRED_TRY(validate_blocking(blocking));
    TRED_REQUIRE(n_dep >= 0, "n_dep must be >= 0");
    TRED_REQUIRE(cap >= 0, "cap must be >= 0");
    TRED_REQUIRE(n_active && work, "n_active/work is NULL");
    TRED_REQUIRE(cap == 0 || (keys && blocks), "keys/blocks is NULL");
    if (fz) {
        TRED_TRY(validate_physics(fz->phys));
        TRED_REQUIRE(fz->phys->point_frac > 0.0f, "physics.point_frac must be > 0 for the line form");
        TRED_REQUIRE(n_dep == 0 || (fp && fz->seg), "seg/fp is NULL");
        TRED_REQUIRE((int64_t)blocking->blk_pix[0] * grid->sub[0] * blocking->blk_pix[1] * grid->sub[1] *
                             blocking->blk_ticks <= INT32_MAX,
                     "cells per bin must be below 2^31");
    } else {
        TRED_REQUIRE(n_dep == 0 || (fp && off && val), "fp/off/val is NULL");
    }
    TRED_REQUIRE(tred_block_count(grid, blocking) > 0, "too many bins");
    TRED_REQUIRE((int64_t)n_ev * tred_block_count(grid, blocking) < INT32_MAX,
                 "too many (event, bin) pairs");
    TRED_REQUIRE(((uintptr_t)blocks & 15) == 0, "blocks must be 16-byte aligned");
    const BinGeom G = geom(grid, blocking, n_ev, ev_off ? 4 : 3);
    hipStream_t st = (hipStream_t)stream;
    int32_t* flag = (int32_t*)work;
    const int64_t tot = (int64_t)G.nev * G.nbins;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>((tot + 255) / 256, 4096)),
                       dim3(256), 0, st, flag, tot, 0);
    if (n_dep > 0)
        hipLaunchKernelGGL(k_mark, dim3((unsigned)((n_dep + 255) / 256)), dim3(256), 0, st, G,
                           n_dep, fp, ev_off, flag);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, G, flag, keys, n_active, cap);
    TRED_TRY(tred_check_launch("tred_block_bin compact"));
    if (cap > 0) {
        if (rows) {
            const int nrw = row_words(G);
            const int64_t nw = (int64_t)cap * nrw;
            hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>((nw + 255) / 256, 4096)),
                               dim3(256), 0, st, (int32_t*)rows, nw, 0);
            if (n_dep > 0)
                hipLaunchKernelGGL(k_mark_rows, dim3((unsigned)std::min<int64_t>(n_dep, 1 << 20)),
                                   dim3(256), 0, st, G, n_dep, fp, ev_off, flag, nrw, rows);
            hipLaunchKernelGGL(k_zero_rows, dim3(4096), dim3(256), 0, st, blocks, rows, n_active, cap,
                               G.vblk, nrw, G.bf[2]);
        } else {
            hipLaunchKernelGGL(k_zero_blocks, dim3(2048), dim3(256), 0, st, (float4*)blocks, n_active,
                               cap, G.vblk);
            hipLaunchKernelGGL(k_zero_tail, dim3(1), dim3(4), 0, st, blocks, n_active, cap, G.vblk);
        }
        if (n_dep > 0 && fz == nullptr) {
            unsigned nb = (unsigned)std::min<int64_t>(n_dep, 1 << 20);
            hipLaunchKernelGGL(k_accum, dim3(nb), dim3(256), 0, st, G, n_dep, fp, off, val, val_cap,
                               ev_off, flag, blocks);
        }
    }
    TRED_TRY(tred_check_launch("tred_block_bin"));
    if (fz && n_dep > 0) {   // (with cap 0 every slot is -1: only the charge sum)
        EffqBins B;
        B.blocks = blocks;
        B.slot = flag;
        B.ev_off = ev_off;
        B.nbins = G.nbins;
        B.vblk = G.vblk;
        for (int a = 0; a < 3; ++a) {
            B.bf[a] = G.bf[a];
            B.nb[a] = G.nb[a];
        }
        B.nev = G.nev;
        B.inv_bf2 = 1.0f / (float)G.bf[2];
        TRED_TRY(effq_into_bins(grid, fz->phys, n_dep, fz->seg, fp, B, fz->charge_sum, st));
    }
    return TRED_OK;
}

}  // namespace

extern "C" int32_t tred_block_count(const tred_grid* grid, const tred_blocking* blocking) {
    if (validate_grid(grid) != TRED_OK || validate_blocking(blocking) != TRED_OK) return -1;
    int64_t n = (int64_t)nblk_axis(grid, blocking, 0) * nblk_axis(grid, blocking, 1) *
                nblk_axis(grid, blocking, 2);
    return n > INT32_MAX ? -1 : (int32_t)n;
}

extern "C" int64_t tred_block_bin_workspace(const tred_grid* grid, const tred_blocking* blocking) {
    int32_t n = tred_block_count(grid, blocking);
    return n < 0 ? -1 : (int64_t)n * 4;
}

extern "C" tred_status tred_block_bin(const tred_grid* grid, const tred_blocking* blocking,
                                      int64_t n_dep, const int32_t* fp, const int64_t* off,
                                      const float* val, int64_t val_cap, int32_t* keys,
                                      int32_t* n_active,
                                      float* blocks, int32_t cap, void* work, void* stream) {
    return block_bin(grid, blocking, 1, nullptr, n_dep, fp, off, val, val_cap, keys, n_active,
                     blocks, nullptr, cap, work, stream);
}

extern "C" int32_t tred_block_row_words(const tred_grid* grid, const tred_blocking* blocking) {
    if (validate_grid(grid) != TRED_OK || validate_blocking(blocking) != TRED_OK) return -1;
    const int64_t r = (int64_t)blocking->blk_pix[0] * grid->sub[0] * blocking->blk_pix[1] * grid->sub[1];
    return r > (int64_t)INT32_MAX - 31 ? -1 : (int32_t)((r + 31) / 32);
}

extern "C" tred_status tred_block_bin_rows(const tred_grid* grid, const tred_blocking* blocking,
                                           int64_t n_dep, const int32_t* fp, const int64_t* off,
                                           const float* val, int64_t val_cap, int32_t* keys,
                                           int32_t* n_active, float* blocks, uint32_t* rows,
                                           int32_t cap, void* work, void* stream) {
    TRED_REQUIRE(cap == 0 || rows, "rows is NULL");
    TRED_REQUIRE(((uintptr_t)rows & 3) == 0, "rows must be 4-byte aligned");
    return block_bin(grid, blocking, 1, nullptr, n_dep, fp, off, val, val_cap, keys, n_active,
                     blocks, rows, cap, work, stream);
}

extern "C" tred_status tred_block_bin_rows_noalloc(const tred_grid* grid,
                                                   const tred_blocking* blocking, int64_t n_dep,
                                                   const int32_t* fp, const int64_t* off,
                                                   const float* val, int64_t val_cap,
                                                   int32_t* keys, int32_t* n_active,
                                                   float* blocks, uint32_t* rows, int32_t cap,
                                                   void* stream) {
    TRED_TRY(validate_grid(grid));
    TRED_TRY(validate_blocking(blocking));
    const int32_t nb = tred_block_count(grid, blocking);
    if (nb < 0 || nb > kNoallocMaxBins)
        return tred_fail(TRED_ECAPACITY,
                         "tred_block_bin_rows_noalloc: %d bins exceed the static scratch of %lld "
                         "bins; use tred_block_bin_rows with a workspace",
                         (int)nb, (long long)kNoallocMaxBins);
    TRED_REQUIRE(cap == 0 || rows, "rows is NULL");
    TRED_REQUIRE(((uintptr_t)rows & 3) == 0, "rows must be 4-byte aligned");
    int32_t* work = nullptr;
    TRED_TRY(noalloc_scratch(&work));
    // block_bin clears the map with a fill kernel first, so the previous call's contents
    // do not matter
    return block_bin(grid, blocking, 1, nullptr, n_dep, fp, off, val, val_cap, keys, n_active,
                     blocks, rows, cap, work, stream);
}

extern "C" tred_status tred_effq_bin(const tred_grid* grid, const tred_physics* phys,
                                     const tred_blocking* blocking, int64_t n_dep,
                                     const float* seg, const int32_t* fp, int32_t* keys,
                                     int32_t* n_active, float* blocks, uint32_t* rows, int32_t cap,
                                     double* charge_sum, void* work, void* stream) {
    TRED_REQUIRE(((uintptr_t)rows & 3) == 0, "rows must be 4-byte aligned");
    const FusedEffq fz{phys, seg, charge_sum};
    return block_bin(grid, blocking, 1, nullptr, n_dep, fp, nullptr, nullptr, 0, keys, n_active,
                     blocks, rows, cap, work, stream, &fz);
}

extern "C" tred_status tred_effq_bin_events(const tred_grid* grid, const tred_physics* phys,
                                            const tred_blocking* blocking, int32_t n_ev,
                                            const int64_t* ev_off, int64_t n_dep, const float* seg,
                                            const int32_t* fp, int32_t* keys, int32_t* n_active,
                                            float* blocks, uint32_t* rows, int32_t cap,
                                            double* charge_sum, void* work, void* stream) {
    TRED_REQUIRE(n_ev > 0, "n_ev must be > 0");
    TRED_REQUIRE(ev_off != nullptr, "ev_off is NULL");
    TRED_REQUIRE(((uintptr_t)rows & 3) == 0, "rows must be 4-byte aligned");
    const FusedEffq fz{phys, seg, charge_sum};
    return block_bin(grid, blocking, n_ev, ev_off, n_dep, fp, nullptr, nullptr, 0, keys, n_active,
                     blocks, rows, cap, work, stream, &fz);
}

extern "C" tred_status tred_block_bin_adjoint(const tred_grid* grid, const tred_blocking* blocking,
                                              int64_t n_dep, const int32_t* fp, const int64_t* off,
                                              int64_t val_cap, const int32_t* keys,
                                              const int32_t* n_active, const float* d_blocks,
                                              int32_t cap, float* d_val, void* work, void* stream) {
    TRED_TRY(validate_grid(grid));
    TRED_TRY(validate_blocking(blocking));
    TRED_REQUIRE(n_dep >= 0 && cap >= 0 && val_cap >= 0, "sizes must be >= 0");
    TRED_REQUIRE(n_active && work, "n_active/work is NULL");
    TRED_REQUIRE(cap == 0 || (keys && d_blocks), "keys/d_blocks is NULL");
    TRED_REQUIRE(n_dep == 0 || (fp && off), "fp/off is NULL");
    TRED_REQUIRE(val_cap == 0 || d_val, "d_val is NULL");
    TRED_REQUIRE(tred_block_count(grid, blocking) > 0, "too many bins");
    const BinGeom G = geom(grid, blocking, 1, 3);
    hipStream_t st = (hipStream_t)stream;
    int32_t* slot = (int32_t*)work;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>((G.nbins + 255) / 256, 4096)),
                       dim3(256), 0, st, slot, G.nbins, -1);
    if (cap > 0)
        hipLaunchKernelGGL(k_slots, dim3((unsigned)std::min(((int64_t)cap + 255) / 256, (int64_t)4096)),
                           dim3(256), 0, st, G, keys, n_active, cap, slot);
    if (n_dep > 0 && val_cap > 0) {
        const unsigned nb = (unsigned)std::min<int64_t>(n_dep, 1 << 20);
        hipLaunchKernelGGL(k_accum_adj, dim3(nb), dim3(256), 0, st, G, n_dep, fp, off, val_cap,
                           (const int64_t*)nullptr, slot, d_blocks, d_val);
    }
    return tred_check_launch("tred_block_bin_adjoint");
}

extern "C" int64_t tred_block_bin_events_workspace(const tred_grid* grid,
                                                   const tred_blocking* blocking, int32_t n_ev) {
    int32_t n = tred_block_count(grid, blocking);
    return (n < 0 || n_ev <= 0) ? -1 : (int64_t)n * n_ev * 4;
}

extern "C" tred_status tred_block_bin_events(const tred_grid* grid, const tred_blocking* blocking,
                                             int32_t n_ev, const int64_t* ev_off, int64_t n_dep,
                                             const int32_t* fp, const int64_t* off,
                                             const float* val, int64_t val_cap, int32_t* keys,
                                             int32_t* n_active, float* blocks, int32_t cap,
                                             void* work, void* stream) {
    TRED_REQUIRE(n_ev > 0, "n_ev must be > 0");
    TRED_REQUIRE(ev_off != nullptr, "ev_off is NULL");
    return block_bin(grid, blocking, n_ev, ev_off, n_dep, fp, off, val, val_cap, keys, n_active,
                     blocks, nullptr, cap, work, stream);
}

extern "C" tred_status tred_block_bin_events_rows(const tred_grid* grid,
                                                  const tred_blocking* blocking, int32_t n_ev,
                                                  const int64_t* ev_off, int64_t n_dep,
                                                  const int32_t* fp, const int64_t* off,
                                                  const float* val, int64_t val_cap, int32_t* keys,
                                                  int32_t* n_active, float* blocks, uint32_t* rows,
                                                  int32_t cap, void* work, void* stream) {
    TRED_REQUIRE(n_ev > 0, "n_ev must be > 0");
    TRED_REQUIRE(ev_off != nullptr, "ev_off is NULL");
    TRED_REQUIRE(cap == 0 || rows, "rows is NULL");
    TRED_REQUIRE(((uintptr_t)rows & 3) == 0, "rows must be 4-byte aligned");
    return block_bin(grid, blocking, n_ev, ev_off, n_dep, fp, off, val, val_cap, keys, n_active,
                     blocks, rows, cap, work, stream);
}

// Interlaced convolution of the charge blocks with the field response by FFT
// (Sec. II-D eq. interlaced; Sec. III-A: per-channel transforms, channel sum in the
// frequency domain, one inverse per block; mirror-pair complex packing, eq. multch).
//
// Per block and impact channel j the transform is separable:
//   k_tf : time FFT (length ft) of every (channel, pixel) row   -> T[b][j][p/16][f][p%16]
//   k_sp : per time frequency f, 2-D spatial FFT of each channel (block pixels zero
//          padded to fs x fs), multiply-accumulate with the precomputed response
//          spectra of every response piece, inverse spatial FFT   -> U[b][c][q/8][f][q%8]
//   k_ti : inverse time FFT per output pixel and piece, overlap-add of the pieces
//          into the block's output rows.
// When ft < blk_ticks + kticks - 1 the response is cut into pieces of ct = ft -
// blk_ticks ticks; piece c's linear convolution (length <= ft - 1, no wrap) lands at
// tick offset c * ct.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "tred_internal.hpp"
#include "validate.hpp"

// bins per workgroup of the prime-factor spatial stage with 8-point sub-DFTs
#ifndef TRED_SPP_NB8
#define TRED_SPP_NB8 2
#endif
// XCD-aware workgroup order in the spatial stage (1) or the dispatch order (0)
#ifndef TRED_XCD_REMAP
#define TRED_XCD_REMAP 1
#endif
// transposed spatial stage at L = 8 (fs 24, 40): response-spectrum pieces requested
// ahead of the multiply-adds (register buffers; 2 keeps the kernel within three waves
// per SIMD)
#ifndef TRED_SPP_ADJ_PRE
#define TRED_SPP_ADJ_PRE 2
#endif
// bins per workgroup of the transposed spatial stage at fs = 40
#ifndef TRED_SPP_ADJ_NB
#define TRED_SPP_ADJ_NB 1
#endif
// persistent workgroups of the forward time FFTs (at most)
#ifndef TRED_TF_GRID
#define TRED_TF_GRID 16384
#endif
// forward spatial stage: one barrier per channel, the x pass of the next channel in
// the phase of the current one's y pass and multiply-adds (1: x pass first, 2: after),
// or two phases per channel (0)
#ifndef TRED_SPP_PIPE
#define TRED_SPP_PIPE 1
#endif
// wave-level ordering inside the inverse time FFTs (1) or workgroup barriers (0)
#ifndef TRED_TI_WAVESYNC
#define TRED_TI_WAVESYNC 1
#endif

namespace {

struct ConvArgs {
    int32_t Bx, By, Bt, sx, sy, NYf, S;
    int32_t nch, nc, ct, ft, fs;
    int32_t ppad, qpad, box, boy, bot;
    int32_t mpcp, chx, cap;
    int32_t e1, e2;      // row order of the response spectra: ky = (e1 m + e2 ry) mod fs
    int32_t rpair;       // response spectra stored as row pairs [m / 2][item][m % 2]
    int32_t tskip;       // the spectra of groups flagged all-zero are not written
    int64_t vblk, vout;
    uint8_t* tflag;      // [bin of the pass][nch][ppad / kTile]: 1 = spectra written
    const uint32_t* rows;   // row masks of the bins (NULL: every row is read)
    int32_t nrw;            // mask words per bin
};

// ---------------------------------------------------------------------------
// plan set-up kernels (binary64 arithmetic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 tw64(int64_t k, int64_t n) {
    // exp(-2 pi i k / n) with exact argument reduction
    double s, c;
    sincospi(-2.0 * (double)(k % n) / (double)n, &s, &c);
    return make_double2(c, s);
}

__global__ void k_twiddles(float2* __restrict__ twt, int ft, float2* __restrict__ tws, int fs,
                           double2* __restrict__ twdt, double2* __restrict__ twds) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ft) {
        double2 w = tw64(i, ft);
        twt[i] = make_float2((float)w.x, (float)w.y);
        twdt[i] = w;
    }
    if (i < fs) {
        double2 w = tw64(i, fs);
        tws[i] = make_float2((float)w.x, (float)w.y);
        twds[i] = w;
    }
}

// number of entries violating R[K-1-k][sub-1-j][tau] == R[k][j][tau]
__global__ void k_symcheck(const float* __restrict__ R, int Kx, int Ky, int sx, int sy, int kt,
                           int* __restrict__ bad) {
    int64_t n = (int64_t)Kx * Ky * sx * sy * kt;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i;
        int t = (int)(r % kt); r /= kt;
        int jy = (int)(r % sy); r /= sy;
        int jx = (int)(r % sx); r /= sx;
        int ky = (int)(r % Ky); r /= Ky;
        int kx = (int)r;
        int64_t m = ((((int64_t)(Kx - 1 - kx) * Ky + (Ky - 1 - ky)) * sx + (sx - 1 - jx)) * sy +
                     (sy - 1 - jy)) * kt + t;
        if (R[i] != R[m]) atomicAdd(bad, 1);
    }
}

// PA[ch][c][kx][ky][f] = sum_{tau < ct} R[kx][ky][j][c ct + tau] exp(-2 pi i tau f / ft)
__global__ void k_rhat_time(const float* __restrict__ R, ConvArgs A, int Kx, int Ky, int kt,
                            const double2* __restrict__ twd, double2* __restrict__ PA) {
    const int64_t n = (int64_t)A.nch * A.nc * Kx * Ky * A.ft;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i;
        const int f = (int)(r % A.ft); r /= A.ft;
        const int ky = (int)(r % Ky); r /= Ky;
        const int kx = (int)(r % Kx); r /= Kx;
        const int c = (int)(r % A.nc); r /= A.nc;
        const int ch = (int)r;
        const int jx = ch / A.sy, jy = ch % A.sy;
        const float* row = R + ((((int64_t)kx * Ky + ky) * A.sx + jx) * A.sy + jy) * kt;
        const int t0 = c * A.ct;
        const int len = min(A.ct, kt - t0);
        double re = 0.0, im = 0.0;
        for (int tau = 0; tau < len; ++tau) {
            const double v = (double)row[t0 + tau];
            const double2 w = twd[((int64_t)tau * f) & (A.ft - 1)];
            re += v * w.x;
            im += v * w.y;
        }
        PA[i] = make_double2(re, im);
    }
}

// PB[ch][c][kxf][ky][f] = sum_kx PA[ch][c][kx][ky][f] exp(-2 pi i kx kxf / fs)
__global__ void k_rhat_x(ConvArgs A, int Kx, int Ky, const double2* __restrict__ twd,
                         const double2* __restrict__ PA, double2* __restrict__ PB) {
    const int64_t n = (int64_t)A.nch * A.nc * A.fs * Ky * A.ft;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i;
        const int f = (int)(r % A.ft); r /= A.ft;
        const int ky = (int)(r % Ky); r /= Ky;
        const int kxf = (int)(r % A.fs); r /= A.fs;
        const int64_t cc = r;  // ch * nc + c
        double re = 0.0, im = 0.0;
        for (int kx = 0; kx < Kx; ++kx) {
            const double2 a = PA[((cc * Kx + kx) * Ky + ky) * A.ft + f];
            const double2 w = twd[(kx * kxf) % A.fs];
            re += a.x * w.x - a.y * w.y;
            im += a.x * w.y + a.y * w.x;
        }
        PB[i] = make_double2(re, im);
    }
}

// R̂[ch][f][c][m][item] = scale * sum_ky PB[ch][c][kxf][ky][f] exp(-2 pi i ky kyf / fs),
// item = kxf * RS + ry, kyf = (e1 m + e2 ry) mod fs: the order in which the spatial
// kernels hold spectra (k_sp: kyf = ry + RS m; k_spp: the prime-factor output map),
// so that the nc * L values a thread needs at one frequency lie at fixed offsets.
// With rpair the rows m of one (ch, f, c) are stored in pairs, [m / 2][item][m % 2],
// so that a thread reads two rows with one 16-byte load and a wave's loads are
// contiguous; an odd L is padded with one row (m = L, never read by the kernels).
__global__ void k_rhat_y(ConvArgs A, int Ky, int L, double scale, const double2* __restrict__ twd,
                         const double2* __restrict__ PB, float2* __restrict__ rhat) {
    const int RS = A.fs / L;
    const int TPF = A.fs * RS;
    const int LP = A.rpair ? (L + 1) / 2 * 2 : L;   // rows stored per (ch, f, c)
    const int64_t n = (int64_t)A.nch * A.nc * LP * A.ft * TPF;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i;
        int item, m;
        if (A.rpair) {
            const int e = (int)(r % 2); r /= 2;
            item = (int)(r % TPF); r /= TPF;
            m = 2 * (int)(r % (LP / 2)) + e; r /= LP / 2;
        } else {
            item = (int)(r % TPF); r /= TPF;
            m = (int)(r % L); r /= L;
        }
        const int kxf = item / RS, ry = item % RS;
        const int c = (int)(r % A.nc); r /= A.nc;
        const int f = (int)(r % A.ft); r /= A.ft;
        const int64_t cc = r * A.nc + c;  // ch * nc + c
        const int kyf = (A.e1 * m + A.e2 * ry) % A.fs;
        double re = 0.0, im = 0.0;
        for (int ky = 0; ky < Ky; ++ky) {
            const double2 a = PB[((cc * A.fs + kxf) * Ky + ky) * A.ft + f];
            const double2 w = twd[(ky * kyf) % A.fs];
            re += a.x * w.x - a.y * w.y;
            im += a.x * w.y + a.y * w.x;
        }
        rhat[i] = make_float2((float)(re * scale), (float)(im * scale));
    }
}

// ---------------------------------------------------------------------------
// k_tf: time FFT of the (channel, pixel) rows of a block; one wavefront per row,
// 8 rows (one half of a T tile) per group. Workgroups are persistent: workgroup w
// takes groups w, w + G, w + 2G, ... (G = gridDim.x), and requests the next group's
// rows before the FFT of the current one, so HBM reads overlap the arithmetic.
// Under mirror-pair packing the row is Q_j[p] + i Q_{j'}[B-1-p] with j' = sub-1-j.
// ---------------------------------------------------------------------------
struct TfGroup {
    int bl, ch, pt, half;
};

// LDS of k_tf in floats: the 8 waves' FFT scratch or the staging tile (rows of kTile
// values, no padding), then the twiddles; two workgroups fit in a CU at FT = 1024
template <int FT>
__host__ __device__ constexpr int tf_lds_floats() {
    return 8 * kFftLds<FT> > 2 * FT * kTile ? 8 * kFftLds<FT> : 2 * FT * kTile;
}

// column of pixel c in staging row f: an XOR swizzle by f / 4 spreads a wave's writes
// of one column over all banks (rows are 64 bytes, four rows span the 64 banks)
__device__ __forceinline__ int tf_col(int f, int c) { return c ^ ((f >> 2) & (kTile - 1)); }

// Stores a staged tile ([f][kTile], columns swizzled) as half `half` of a T tile (rows
// of kTileT pixels) with 512 threads: thread t writes pixels c, c + 1
// (c = 2 (t % (kTile / 2))) of rows f = t / (kTile / 2) + R k (R = 512 / (kTile / 2))
// with one 16-byte store. The swizzle XORs c with s = (f / 4) % kTile, the same for all
// of a thread's rows (R is a multiple of 4 kTile), and keeps the two pixels in one
// aligned pair of the staging row, swapped where s is odd.
template <int FT>
__device__ __forceinline__ void tf_store_tile(const float2* stage, __amdgpu_buffer_rsrc_t tr, int half) {
    constexpr int TPR = kTile / 2, R = 512 / TPR;
    static_assert(kTile % 2 == 0 && R % (4 * kTile) == 0 && FT % R == 0, "store loop");
    const int f0 = (int)threadIdx.x / TPR, c = 2 * ((int)threadIdx.x % TPR);
    const int sw = (f0 >> 2) & (kTile - 1);
    const float4* src = (const float4*)(stage + f0 * kTile + ((c ^ sw) & ~1));
    const uint32_t voff = (uint32_t)((f0 * kTileT + half * kTile + c) * 8);
#pragma unroll
    for (int k = 0; k < FT / R; ++k) {
        const float4 p = src[k * R * kTile / 2];
        const float4 v = (sw & 1) ? make_float4(p.z, p.w, p.x, p.y) : p;
        buf_st_f4(v, tr, voff, (uint32_t)(k * R * kTileT * 8));
    }
}

// Group q -> (bin, channel, tile, half). T tiles hold kTileT = 2 kTile pixels per
// frequency (one 128-byte line) and a group transforms the 8 rows of one half.
// Workgroup ids are dealt to the XCDs round-robin; with G a multiple of 2 kXcd the
// two halves of a tile go to groups kXcd apart, i.e. to one XCD (one L2).
__device__ __forceinline__ TfGroup tf_group(const ConvArgs& A, int q) {
    const int nbx = A.ppad / kTile;
    TfGroup g;
    const int x = q % nbx;
    g.ch = (q / nbx) % A.nch;
    g.bl = q / (nbx * A.nch);
    const int ntile = A.ppad / kTileT;
    if (kTileT == kTile) {
        g.pt = x;
        g.half = 0;
    } else if (ntile % (int)kXcd == 0) {
        const int gg = x / (2 * kXcd), r = x % (2 * kXcd);
        g.pt = gg * kXcd + r % kXcd;
        g.half = r / kXcd;
    } else {
        g.pt = x >> 1;
        g.half = x & 1;
    }
    return g;
}

// HALF: the block holds at most FT / 2 ticks, so only the first half of each row is
// loaded (the rest is zero padding).
template <int FT, bool HALF>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(FT <= 1024 ? 4 : 1))) void k_tf(ConvArgs A, int b0, int nbp, const int32_t* __restrict__ n_active,
                                            const float* __restrict__ blocks,
                                            const float2* __restrict__ tw, float2* __restrict__ T) {
    extern __shared__ float lds[];
    constexpr int M = FT / kWave, MB = HALF ? M / 2 : M;
    const int nbin = min(nbp, min(*n_active, A.cap) - b0);
    if (nbin <= 0) return;
    const int total = (A.ppad / kTile) * A.nch * nbin;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int mb = A.Bt / kWave;
    // rows of group q into (ra, rb): Q_j and, under mirror-pair packing, Q_j'; 32-bit
    // offsets within the bin (the host keeps a bin below 2^31 bytes)
    float ra[MB], rb[MB];
    auto load = [&](int q) {
        const TfGroup g = tf_group(A, q);
        const int p = g.pt * kTileT + g.half * kTile + wv;
        const int jx = g.ch / A.sy, jy = g.ch % A.sy;
        const int jb = A.S - 1 - g.ch;
        const bool pair = A.mpcp && jb != g.ch;
        const bool live = p < A.Bx * A.By;
        const auto br = buf_rsrc(blocks + (int64_t)(b0 + g.bl) * A.vblk, (uint32_t)(A.vblk * 4));
        const int px = live ? p / A.By : 0, py = live ? p % A.By : 0;
        const int r0 = (px * A.sx + jx) * A.NYf + (py * A.sy + jy);
        const int jbx = jb / A.sy, jby = jb % A.sy;
        const int r1 = ((A.Bx - 1 - px) * A.sx + jbx) * A.NYf + ((A.By - 1 - py) * A.sy + jby);
        // with row masks, unmarked rows are zero and not read
        bool la = live, lb = live && pair;
        if (A.rows) {
            const uint32_t* rw = A.rows + (int64_t)(b0 + g.bl) * A.nrw;
            la = la && ((rw[r0 >> 5] >> (r0 & 31)) & 1u);
            lb = lb && ((rw[r1 >> 5] >> (r1 & 31)) & 1u);
        }
        const uint32_t o0 = 4u * (uint32_t)(r0 * A.Bt + lane);
        const uint32_t o1 = 4u * (uint32_t)(r1 * A.Bt + lane);
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            ra[m] = (la && m < mb) ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                         br, o0, (uint32_t)(m * kWave * 4), 0))
                                   : 0.0f;
            rb[m] = (lb && m < mb) ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                         br, o1, (uint32_t)(m * kWave * 4), 0))
                                   : 0.0f;
        }
    };
    // twiddle table in LDS after the FFT scratch / staging region
    float2* twl = (float2*)(lds + tf_lds_floats<FT>());
    fft_tw_fill<FT>(twl, tw, threadIdx.x, blockDim.x);
    // per-wave "row pair not all zero", by iteration parity: a wave runs at most one
    // iteration ahead of the others (one barrier per iteration)
    __shared__ int wlive[2][8];
    int q = blockIdx.x;
    if (q < total) load(q);
    __syncthreads();
    for (int it = 0; q < total; q += gridDim.x, ++it) {
        const TfGroup g = tf_group(A, q);
        float2 v[M];
        bool nz = false;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            v[m] = m < MB ? make_float2(ra[m], rb[m]) : make_float2(0.f, 0.f);
            if (m < MB) nz = nz || ra[m] != 0.0f || rb[m] != 0.0f;
        }
        if (q + (int)gridDim.x < total) load(q + gridDim.x);   // in flight during the FFT
        // the transform of zeros is zero: such a wave keeps v
        const bool wlv = __builtin_amdgcn_ballot_w64(nz) != 0;
        if (wlv) wave_fft<FT, true, true>(v, lds + wv * kFftLds<FT>, twl, lane);
        if (lane == 0) wlive[it & 1][wv] = wlv;
        __syncthreads();   // the staging tile overlaps the other waves' FFT scratch
        {
            bool live = false;
#pragma unroll
            for (int w = 0; w < 8; ++w) live = live || wlive[it & 1][w] != 0;
            if (threadIdx.x == 0)
                A.tflag[((int64_t)g.bl * A.nch + g.ch) * (A.ppad / kTile) + g.pt * (kTileT / kTile) + g.half] =
                    live ? 1 : 0;
            if (!live && A.tskip) continue;   // uniform over the workgroup; nothing was staged
        }
        float2* stage = (float2*)lds;   // [f][kTile], columns swizzled
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int f = lane + kWave * m;
            stage[f * kTile + tf_col(f, wv)] = v[m];
        }
        __syncthreads();
        const auto tr = buf_rsrc(T + (((int64_t)g.bl * A.nch + g.ch) * (A.ppad / kTileT) + g.pt) * FT * kTileT,
                                 (uint32_t)(FT * kTileT * sizeof(float2)));
        tf_store_tile<FT>(stage, tr, g.half);
        __syncthreads();   // the next FFT's scratch overlaps the staging tile
    }
}

// ---------------------------------------------------------------------------
// With row masks the live T tiles are known before the transforms: k_tf_tiles lists
// the (bin, channel, tile) whose pixels read a marked row, with the bits of those rows
// (bit half * kTile + wave for Q_j, 16 + that for the mirror row Q_j'), and writes
// the group flags of both halves; k_tf_list transforms the listed tiles only. Row
// groups without a marked row are zero, flagged 0 and never written. The list is in
// no particular order: every tile is written independently of the others.
// ---------------------------------------------------------------------------
__global__ void k_zero_count(int32_t* __restrict__ c) {
    if (threadIdx.x == 0) c[0] = 0;
}

__global__ __launch_bounds__(256) void k_tf_tiles(ConvArgs A, int b0, int nb,
                                                  const int32_t* __restrict__ n_active,
                                                  int2* __restrict__ list, int32_t* __restrict__ count) {
    static_assert(kTileT == 2 * kTile && kTile == 8, "tile bits: two halves of 8 rows");
    const int ntile = A.ppad / kTileT, ng = A.ppad / kTile;
    const int64_t total = (int64_t)nb * A.nch * ntile;
    const int nact = min(*n_active, A.cap) - b0;
    const int lane = threadIdx.x & 63;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < total;
         i0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        uint32_t bits = 0;
        if (i < total) {
            const int pt = (int)(i % ntile);
            const int ch = (int)((i / ntile) % A.nch);
            const int bl = (int)(i / ((int64_t)ntile * A.nch));
            if (bl < nact) {
                const uint32_t* rw = A.rows + (int64_t)(b0 + bl) * A.nrw;
                const int jx = ch / A.sy, jy = ch % A.sy;
                const int jb = A.S - 1 - ch;
                const bool pair = A.mpcp && jb != ch;
                const int jbx = jb / A.sy, jby = jb % A.sy;
                for (int k = 0; k < kTileT; ++k) {
                    const int p = pt * kTileT + k;
                    if (p >= A.Bx * A.By) break;
                    const int px = p / A.By, py = p % A.By;
                    const int r0 = (px * A.sx + jx) * A.NYf + (py * A.sy + jy);
                    const int r1 = ((A.Bx - 1 - px) * A.sx + jbx) * A.NYf + ((A.By - 1 - py) * A.sy + jby);
                    if ((rw[r0 >> 5] >> (r0 & 31)) & 1u) bits |= 1u << k;
                    if (pair && ((rw[r1 >> 5] >> (r1 & 31)) & 1u)) bits |= 1u << (16 + k);
                }
            }
            uint8_t* fl = A.tflag + ((int64_t)bl * A.nch + ch) * ng + 2 * pt;
            fl[0] = (bits & 0x00ff00ffu) != 0;
            fl[1] = (bits & 0xff00ff00u) != 0;
        }
        // one counter update per wave; lanes take consecutive slots in lane order
        const bool live = bits != 0;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(live);
        if (bal != 0) {
            const int leader = __builtin_ctzll(bal);
            int base = 0;
            if (lane == leader) base = atomicAdd(count, __builtin_popcountll(bal));
            base = __shfl(base, leader);
            if (live) {
                const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                list[base + r] = make_int2((int)i, (int)bits);
            }
        }
    }
}

// k_tf_list: the time FFTs of the listed tiles. Iteration q covers half (q / 8) % 2 of
// list entry (q / 16) * 8 + q % 8: the two halves of a tile (one 128-byte line of T per
// frequency) are kXcd apart in q and, with the grid a multiple of 2 kXcd, land on one
// XCD (one L2). Every iteration issues the same vector memory operations in the same
// order (loads and stores it does not need address an empty buffer resource, which
// reads zero and drops stores), so each wait waits for the operation it needs and not
// for the stores still in flight: list entries are requested two iterations before
// their transform and rows one iteration before; the loop starts two iterations early.
template <int FT, bool HALF>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(FT <= 1024 ? 4 : 1))) void k_tf_list(
    ConvArgs A, int b0, const int2* __restrict__ list, const int32_t* __restrict__ count, int32_t lcap,
    const float* __restrict__ blocks, const float2* __restrict__ tw, float2* __restrict__ T) {
    extern __shared__ float lds[];
    constexpr int M = FT / kWave, MB = HALF ? M / 2 : M;
    using u2 = __attribute__((ext_vector_type(2))) unsigned int;
    const int n = min(*count, lcap);
    if (n <= 0) return;
    const int total = 2 * kTile * ((n + kTile - 1) / kTile);
    const int G = (int)gridDim.x;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int mb = A.Bt / kWave;
    const int ntile = A.ppad / kTileT;
    const auto lr = buf_rsrc(list, (uint32_t)n * 8u);
    // list entry of iteration q (q >= 0), requested now and used an iteration later
    u2 en = {0u, 0u};
    bool en_ok = false;
    auto load_entry = [&](int q) {
        const int t = (q >> 4) * kTile + (q & (kTile - 1));
        en_ok = t < n;
        en = __builtin_bit_cast(u2, __builtin_amdgcn_raw_buffer_load_b64(lr, 0u, (uint32_t)min(t, n - 1) * 8u, 0));
    };
    // rows of iteration q's pixel (this wave) of tile `tile` into (ra, rb): Q_j and,
    // under mirror-pair packing, Q_j'; only rows whose bit is set are read (32-bit
    // offsets within the bin: the host keeps a bin below 2^31 bytes)
    float ra[MB], rb[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) ra[m] = rb[m] = 0.0f;
    auto load = [&](int q, int tile, uint32_t bits) {
        const int h = (q >> 3) & 1;
        const int pt = tile % ntile, ch = (tile / ntile) % A.nch, bl = tile / (ntile * A.nch);
        const int p = pt * kTileT + h * kTile + wv;
        const bool la = (bits >> (h * kTile + wv)) & 1u;
        const bool lb = (bits >> (16 + h * kTile + wv)) & 1u;
        const int pc = min(p, A.Bx * A.By - 1);
        const int px = pc / A.By, py = pc % A.By;
        const int jx = ch / A.sy, jy = ch % A.sy;
        const int jb = A.S - 1 - ch;
        const int jbx = jb / A.sy, jby = jb % A.sy;
        const int r0 = (px * A.sx + jx) * A.NYf + (py * A.sy + jy);
        const int r1 = ((A.Bx - 1 - px) * A.sx + jbx) * A.NYf + ((A.By - 1 - py) * A.sy + jby);
        const float* bb = blocks + (int64_t)(b0 + bl) * A.vblk;
        const uint32_t vb = (uint32_t)(A.vblk * 4);
        const auto bra = buf_rsrc(bb, la ? vb : 0u), brb = buf_rsrc(bb, lb ? vb : 0u);
        const uint32_t o0 = 4u * (uint32_t)(r0 * A.Bt + lane);
        const uint32_t o1 = 4u * (uint32_t)(r1 * A.Bt + lane);
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            // ticks past Bt belong to the next row: read tick block mb - 1 again, then zero
            const uint32_t so = (uint32_t)(min(m, mb - 1) * kWave * 4);
            const float xa = buf_f1(bra, o0, so), xb = buf_f1(brb, o1, so);
            ra[m] = m < mb ? xa : 0.0f;
            rb[m] = m < mb ? xb : 0.0f;
        }
    };
    // twiddle table in LDS after the FFT scratch / staging region
    float2* twl = (float2*)(lds + tf_lds_floats<FT>());
    fft_tw_fill<FT>(twl, tw, threadIdx.x, blockDim.x);
    __syncthreads();
    int cur_tile = 0;          // entry of the group this iteration transforms
    uint32_t cur_bits = 0u;
    for (int q = (int)blockIdx.x - 2 * G; q < total; q += G) {
        float2 v[M];
        bool nz = false;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            v[m] = m < MB ? make_float2(ra[m], rb[m]) : make_float2(0.f, 0.f);
            if (m < MB) nz = nz || ra[m] != 0.0f || rb[m] != 0.0f;
        }
        const int tile = cur_tile;
        const uint32_t bits = cur_bits;
        // the next group's rows, in flight during the transform
        cur_tile = (int)__builtin_amdgcn_readfirstlane(en.x);
        cur_bits = en_ok ? __builtin_amdgcn_readfirstlane(en.y) : 0u;
        load(q + G, cur_tile, cur_bits);
        load_entry(q + 2 * G);
        // the transform of zeros is zero: such a wave keeps v
        if (__builtin_amdgcn_ballot_w64(nz) != 0) wave_fft<FT, true, true>(v, lds + wv * kFftLds<FT>, twl, lane);
        __syncthreads();   // the staging tile overlaps the other waves' FFT scratch
        const int h = (q >> 3) & 1;
        const bool wr = q >= 0 && ((bits >> (h * kTile)) & 0xffu | (bits >> (16 + h * kTile)) & 0xffu) != 0;
        float2* stage = (float2*)lds;   // [f][kTile], columns swizzled
        if (wr) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int f = lane + kWave * m;
                stage[f * kTile + tf_col(f, wv)] = v[m];
            }
        }
        __syncthreads();
        const auto tr = buf_rsrc(T + (int64_t)tile * FT * kTileT,
                                 wr ? (uint32_t)(FT * kTileT * sizeof(float2)) : 0u);
        tf_store_tile<FT>(stage, tr, h);
        __syncthreads();   // the next FFT's scratch overlaps the staging tile
    }
}

// ---------------------------------------------------------------------------
// k_sp: spatial transforms and the spectral multiply-accumulate, per time frequency.
// The fs-point transform along an axis with at most B <= 2L nonzero inputs
// (L in {8, 16} divides fs) is split as k = r + RS m (RS = fs / L): for each r an
// L-point DFT of y[n] = sum_t x[n + tL] exp(-2 pi i (n + tL) r / fs) (inputs beyond
// L folded onto the L-periodic kernel). Its inverse with pruned outputs runs the
// split backwards (L-point inverse DFTs, then an RS-point combination).
// A workgroup handles one bin at NF consecutive frequencies; thread (fl, kx, ry)
// owns spectrum column kx, ky = ry + RS m of frequency f0 + fl.
// LDS rows that lanes index with a stride use odd padded strides (bank conflicts).
// ---------------------------------------------------------------------------
struct SpLds {
    int P1, GL, YB;          // padded strides: abuf row (By), inverse rows (L), y rows (boy)
    int zsz, asz, fwd, gsz, g2sz, ysz, y2sz, A, B, total;
};

__host__ __device__ inline SpLds sp_lds(int FS, int L, int NF, int CHX, int By, int ppad, int box,
                                        int boy) {
    SpLds s;
    const int RS = FS / L;
    s.P1 = (By % 2 == 0) ? By + 1 : By;
    s.GL = L + 1;
    s.YB = (boy % 2 == 0) ? boy + 1 : boy;
    s.zsz = CHX * NF * ppad;
    s.asz = CHX * NF * FS * s.P1;
    s.fwd = s.zsz + s.asz;
    s.gsz = NF * FS * RS * s.GL;
    s.g2sz = NF * boy * RS * s.GL;
    s.ysz = NF * FS * s.YB;
    s.y2sz = NF * box * s.YB;
    s.A = s.fwd > s.gsz ? (s.fwd > s.g2sz ? s.fwd : s.g2sz) : (s.gsz > s.g2sz ? s.gsz : s.g2sz);
    s.B = s.ysz > s.y2sz ? s.ysz : s.y2sz;
    s.total = FS + s.A + s.B;
    return s;
}

template <int FS, int L>
struct SpShape {
    static constexpr int RS = FS / L;
    static constexpr int TPF = FS * RS;                       // threads per frequency
    static constexpr int NF = TPF >= 256 ? 1 : (TPF > 128 ? 1 : (TPF > 64 ? 2 : 256 / TPF));
    static constexpr int NT = (NF * TPF + 63) / 64 * 64;      // threads per workgroup
};

// Occupancy target: with 8-point sub-DFTs the accumulators fit 128 VGPRs and four
// waves per SIMD hide the latency of the response-spectrum loads (measured faster than
// three waves without spills); 16-point sub-DFTs keep the compiler's choice.
template <int FS, int L>
__global__ __launch_bounds__((SpShape<FS, L>::NT)) __attribute__((amdgpu_waves_per_eu(L == 8 ? 4 : 1)))
void k_sp(ConvArgs A, int b0, int nbp,
                                                          const int32_t* __restrict__ n_active,
                                                          const float2* __restrict__ T,
                                                          const float2* __restrict__ rhat,
                                                          const float2* __restrict__ tws,
                                                          float2* __restrict__ U) {
    using S = SpShape<FS, L>;
    constexpr int RS = S::RS, TPF = S::TPF, NF = S::NF, NT = S::NT;
    constexpr int FOLD = 2;
    extern __shared__ float2 sm[];
    // bins vary fastest across the grid: the workgroups running at one time share the
    // frequency slab of the response spectra, which then comes from L2 / the last-level
    // cache instead of being streamed from HBM once per bin.
    // Bins of this pass: local index bl < nbp (scratch slots), global b0 + bl < n_active.
    const int na = min(*n_active, A.cap);
    const int bl = blockIdx.x;
    if (bl >= min(nbp, na - b0)) return;
    const int f0 = blockIdx.y * NF;
    const int tid = threadIdx.x;
    const bool active = tid < NF * TPF;      // threads past NF*TPF only help in strided loops
    const int fl = active ? tid / TPF : 0, item = tid % TPF;
    const int kx = item / RS, ry = item % RS;
    const int By = A.By, Bx = A.Bx, CHX = A.chx, ppad = A.ppad, box = A.box, boy = A.boy;
    const int ptiles = ppad / kTileT;
    const SpLds Ls = sp_lds(FS, L, NF, CHX, By, ppad, box, boy);
    const int P1 = Ls.P1, GL = Ls.GL, YB = Ls.YB;
    float2* twl = sm;                        // exp(-2 pi i k / fs)
    float2* regA = sm + FS;
    float2* regB = regA + Ls.A;
    float2* zbuf = regA;                     // [CHX][NF][ppad]
    float2* abuf = regA + Ls.zsz;            // [CHX][NF][FS][P1]
    for (int i = tid; i < FS; i += NT) twl[i] = tws[i];

    float2 acc[4][L];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int m = 0; m < L; ++m) acc[c][m] = make_float2(0.f, 0.f);
    const int nld = CHX * ptiles * NF * kTileT;
    const int nx = CHX * NF * By * RS;
    const int64_t tstride = (int64_t)ptiles * A.ft * kTileT;   // one channel of T
    const float2* Tb = T + (int64_t)bl * A.nch * tstride;
    // response spectra of (channel, frequency): nc * L values per thread at fixed offsets
    const int64_t rstride = (int64_t)A.nc * L * TPF;
    __syncthreads();

    for (int j0 = 0; j0 < A.nch; j0 += CHX) {
        // stage the time spectra of CHX channels at frequencies f0 .. f0+NF-1
        for (int i = tid; i < nld; i += NT) {
            const int pi = i % kTileT;
            int r = i / kTileT;
            const int fl2 = r % NF;
            r /= NF;
            const int pt = r % ptiles;
            const int cx = r / ptiles;
            const int ch = j0 + cx;
            float2 z = make_float2(0.f, 0.f);
            if (ch < A.nch) z = Tb[ch * tstride + (pt * A.ft + f0 + fl2) * kTileT + pi];
            zbuf[(cx * NF + fl2) * ppad + pt * kTileT + pi] = z;
        }
        __syncthreads();
        // x pass: for each (channel, frequency, py, rx): L-point DFT over the folded px
        for (int i = tid; i < nx; i += NT) {
            const int rx = i % RS;
            int r = i / RS;
            const int py = r % By;
            r /= By;
            const int fl2 = r % NF;
            const int cx = r / NF;
            const float2* zr = zbuf + (cx * NF + fl2) * ppad + py;
            float2 s[L];
#pragma unroll
            for (int n = 0; n < L; ++n) {
                s[n] = make_float2(0.f, 0.f);
#pragma unroll
                for (int t = 0; t < FOLD; ++t) {
                    const int px = n + t * L;
                    if (px < Bx) s[n] = cadd(s[n], cmul(zr[px * By], twl[(px * rx) % FS]));
                }
            }
            Dft<L>::run(s);
            float2* ar = abuf + (cx * NF + fl2) * FS * P1 + py;
#pragma unroll
            for (int m = 0; m < L; ++m) ar[(rx + RS * m) * P1] = s[m];
        }
        __syncthreads();
        // y pass and multiply-accumulate, one channel at a time
        if (active) {
            for (int cx = 0; cx < CHX; ++cx) {
                const int ch = j0 + cx;
                if (ch >= A.nch) break;
                const float2* rh = rhat + ((int64_t)ch * A.ft + f0 + fl) * rstride + item;
                const float2* ar = abuf + ((cx * NF + fl) * FS + kx) * P1;
                float2 s[L];
#pragma unroll
                for (int n = 0; n < L; ++n) {
                    s[n] = make_float2(0.f, 0.f);
#pragma unroll
                    for (int t = 0; t < FOLD; ++t) {
                        const int py = n + t * L;
                        if (py < By) s[n] = cadd(s[n], cmul(ar[py], twl[(py * ry) % FS]));
                    }
                }
                Dft<L>::run(s);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c < A.nc) {
                        // one piece at a time: its L loads, then its L multiply-adds
                        // (bounds the loads in flight and the registers they hold)
                        float2 w[L];
#pragma unroll
                        for (int m = 0; m < L; ++m) w[m] = rh[(c * L + m) * TPF];
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int m = 0; m < L; ++m) {
                            acc[c][m].x += s[m].x * w[m].x - s[m].y * w[m].y;
                            acc[c][m].y += s[m].x * w[m].y + s[m].y * w[m].x;
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        }
        __syncthreads();
    }

    // inverse spatial transform of every response piece and the mirror-pair unpacking
    const int qtiles = A.qpad / kTile;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c >= A.nc) break;
        float2* gbuf = regA;    // [NF][FS][RS][GL]
        float2* ybuf = regB;    // [NF][FS][YB]
        if (active) {
            float2 s[L];
#pragma unroll
            for (int m = 0; m < L; ++m) s[m] = cconj(acc[c][m]);
            Dft<L>::run(s);
            float2* gr = gbuf + ((fl * FS + kx) * RS + ry) * GL;
#pragma unroll
            for (int n0 = 0; n0 < L; ++n0) gr[n0] = cmulc(cconj(s[n0]), twl[(n0 * ry) % FS]);
        }
        __syncthreads();
        // combine over ry -> y-inverse at qy = n0 + L n1 < boy
        for (int i = tid; i < NF * FS * L; i += NT) {
            const int n0 = i % L;
            int r = i / L;
            const int kx2 = r % FS;
            const int fl2 = r / FS;
            const float2* gr = gbuf + ((fl2 * FS + kx2) * RS) * GL + n0;
            float2 col[RS];
#pragma unroll
            for (int rr = 0; rr < RS; ++rr) col[rr] = gr[rr * GL];
            float2* yr = ybuf + (fl2 * FS + kx2) * YB;
#pragma unroll
            for (int n1 = 0; n1 < RS; ++n1) {
                const int qy = n0 + L * n1;
                if (qy < boy) {
                    float2 y = col[0];
#pragma unroll
                    for (int rr = 1; rr < RS; ++rr) y = cadd(y, cmulc(col[rr], twl[(n1 * rr * L) % FS]));
                    yr[qy] = y;
                }
            }
        }
        __syncthreads();
        // x-inverse: L-point inverse DFTs over kx = rx + RS m
        float2* g2 = regA;      // [NF][boy][RS][GL]
        for (int i = tid; i < NF * boy * RS; i += NT) {
            const int rx = i % RS;
            int r = i / RS;
            const int qy = r % boy;
            const int fl2 = r / boy;
            const float2* yr = ybuf + (fl2 * FS + rx) * YB + qy;
            float2 s[L];
#pragma unroll
            for (int m = 0; m < L; ++m) s[m] = cconj(yr[RS * m * YB]);
            Dft<L>::run(s);
            float2* gr = g2 + ((fl2 * boy + qy) * RS + rx) * GL;
#pragma unroll
            for (int n0 = 0; n0 < L; ++n0) gr[n0] = cmulc(cconj(s[n0]), twl[(n0 * rx) % FS]);
        }
        __syncthreads();
        float2* y2 = regB;      // [NF][box][YB]
        for (int i = tid; i < NF * boy * L; i += NT) {
            const int n0 = i % L;
            int r = i / L;
            const int qy = r % boy;
            const int fl2 = r / boy;
            const float2* gr = g2 + ((fl2 * boy + qy) * RS) * GL + n0;
            float2 col[RS];
#pragma unroll
            for (int rr = 0; rr < RS; ++rr) col[rr] = gr[rr * GL];
            float2* yr = y2 + fl2 * box * YB + qy;
#pragma unroll
            for (int n1 = 0; n1 < RS; ++n1) {
                const int qx = n0 + L * n1;
                if (qx < box) {
                    float2 y = col[0];
#pragma unroll
                    for (int rr = 1; rr < RS; ++rr) y = cadd(y, cmulc(col[rr], twl[(n1 * rr * L) % FS]));
                    yr[qx * YB] = y;
                }
            }
        }
        __syncthreads();
        // I[q] = Re Y[q] + Im Y[q'] with q' the point reflection within the block output
        // (Re Y(t) + Im Y'(t) = Re(Y(t) - i Y'(t)), taken after the inverse time FFT)
        const int nq = box * boy;
        for (int i = tid; i < qtiles * NF * kTile; i += NT) {
            const int qi = i % kTile;
            int r = i / kTile;
            const int fl2 = r % NF;
            const int qt = r / NF;
            const int q = qt * kTile + qi;
            float2 vq = make_float2(0.f, 0.f);
            if (q < nq) {
                const int qx = q / boy, qy = q % boy;
                const float2* yy = y2 + fl2 * box * YB;
                vq = yy[qx * YB + qy];
                if (A.mpcp) {
                    const float2 yb = yy[(box - 1 - qx) * YB + (boy - 1 - qy)];
                    vq = make_float2(vq.x + yb.y, vq.y - yb.x);
                }
            }
            U[((((int64_t)bl * A.nc + c) * qtiles + qt) * A.ft + f0 + fl2) * kTile + qi] = vq;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_spp: the spatial stage for sizes fs = L * RS with gcd(L, RS) = 1 (8, 16, 24, 40,
// 48), using the prime-factor index maps (Pfa): each L-point sub-DFT gathers its
// inputs with the RS-point phase factors W_RS^(n2 k2) only (RS - 1 distinct values
// per thread, held in registers), and no twiddles sit between the stages. Inputs are
// zero-padded to NIN = L / 2 (sizes 8 and 16), L or 2 L per axis, so every loop is
// unrolled without branches; with NIN = L / 2 half of each sub-DFT's inputs are known
// zeros and their arithmetic is folded away at compile time.
// A workgroup holds NB bins at NF frequencies; thread (fl, kx, k2) owns spectrum
// column kx, rows ky = k_of(k1, k2), of every bin, so each response-spectrum load
// feeds NB multiply-accumulates. The time spectra of the next channel are loaded
// into registers while the current channel is transformed.
// ---------------------------------------------------------------------------
template <int FS, int L, int NIN, int NB>
struct SppShape {
    static constexpr int RS = FS / L;
    static constexpr int TPF = FS * RS;
    static constexpr int NF = TPF >= 128 ? 1 : (TPF > 64 ? 2 : 256 / TPF);
    static constexpr int NT = (NF * TPF + 63) / 64 * 64;
    static constexpr int NZ = NB * NF * NIN * NIN;            // staged inputs
    static constexpr int ZPT = (NZ + NT - 1) / NT;           // per thread
};

struct SppLds {
    int tw, P1, YB, zsz, asz, gsz, g2sz, ysz, y2sz, A, B, C, total;
};

__host__ __device__ inline int even_up(int v) { return (v + 1) & ~1; }

template <int FS, int L, int NIN, int NB, int NF>
__host__ __device__ inline SppLds spp_lds(int box, int boy) {
    constexpr int RS = FS / L;
    SppLds s;
    s.tw = even_up(FS);
    s.P1 = NIN + 2;                                   // even: rows are 16-byte aligned
    s.YB = (boy % 2 == 0) ? boy + 1 : boy;            // odd: strided accesses spread over banks
    s.zsz = NB * NF * NIN * NIN;
    s.asz = NB * NF * FS * s.P1;
    s.gsz = RS > 1 ? NB * NF * FS * L * RS : 0;
    s.g2sz = RS > 1 ? NB * NF * boy * L * RS : 0;
    s.ysz = NB * NF * FS * s.YB;
    s.y2sz = NB * NF * box * s.YB;
    int a = s.zsz + s.asz;
    if (s.gsz > a) a = s.gsz;
    const int a2 = RS > 1 ? s.g2sz : s.y2sz;           // with RS = 1 the x-inverse lands in A
    if (a2 > a) a = a2;
    int b = s.ysz;
    if (RS > 1 && s.y2sz > b) b = s.y2sz;
    // B also holds the forward stage's second staging buffer and, with the channel
    // pipeline, the second x-pass output after it
    if (s.zsz + s.asz > b) b = s.zsz + s.asz;
    // RS > 1: the inverse transforms rotate the k2-inverse output, the x-inverse
    // intermediate and the output of the pieces over B and a third region C
    if (RS > 1 && s.g2sz > b) b = s.g2sz;
    int c = 0;
    if (RS > 1) {
        c = s.ysz;
        if (s.g2sz > c) c = s.g2sz;
        if (s.y2sz > c) c = s.y2sz;
    }
    s.A = even_up(a);
    s.B = even_up(b);
    s.C = even_up(c);
    s.total = s.tw + s.A + s.B + s.C;
    return s;
}

// NC: response pieces the accumulators hold (the plan's piece count rounded up to 2 or 4)
template <int FS, int L, int NIN, int NB, int NC>
__global__ __launch_bounds__((SppShape<FS, L, NIN, NB>::NT)) __attribute__((amdgpu_waves_per_eu(FS == 36 ? 3 : 2))) void k_spp(
    ConvArgs A, int b0, int nbp, const int32_t* __restrict__ n_active,
    const float2* __restrict__ T, const float2* __restrict__ rhat,
    const float2* __restrict__ tws, float2* __restrict__ U) {
    using S = SppShape<FS, L, NIN, NB>;
    using P = Pfa<L, S::RS>;
    constexpr int RS = S::RS, TPF = S::TPF, NF = S::NF, NT = S::NT, NZ = S::NZ, ZPT = S::ZPT;
    static_assert(NIN % 2 == 0 && NIN <= 2 * L, "input padding");
    extern __shared__ float4 sm4[];
    float2* sm = (float2*)sm4;
    // Bins vary fastest in the logical order (response spectra shared through L2).
    // Workgroup ids are dealt round-robin to the XCDs; the logical index is remapped so
    // that each XCD walks a contiguous range of frequencies and the response-spectrum
    // slab of a frequency is fetched into one XCD's L2 only.
    const unsigned nbg = gridDim.x, total = gridDim.x * gridDim.y;
    const unsigned wid = blockIdx.y * nbg + blockIdx.x;
    unsigned lid = wid;
    if (TRED_XCD_REMAP && total % kXcd == 0) lid = (wid % kXcd) * (total / kXcd) + wid / kXcd;
    const int na = min(*n_active, A.cap);
    const int nloc = min(nbp, na - b0);
    const int bl0 = (int)(lid % nbg) * NB;
    if (bl0 >= nloc) return;
    const int nbv = min(NB, nloc - bl0);
    const int f0 = (int)(lid / nbg) * NF;
    const int tid = threadIdx.x;
    // threads past the NF * TPF work items repeat the last item's work in the channel
    // loop (keeps that loop free of branches, so loads can be waited for precisely);
    // only active threads write results
    const bool active = tid < NF * TPF;
    const int tw_ = active ? tid : NF * TPF - 1;
    const int fl = tw_ / TPF, item = tw_ % TPF;
    const int kx = item / RS, k2 = item % RS;
    const int Bx = A.Bx, By = A.By, box = A.box, boy = A.boy;
    const SppLds Ls = spp_lds<FS, L, NIN, NB, NF>(box, boy);
    const int P1 = Ls.P1, YB = Ls.YB;
    float2* twl = sm;                       // exp(-2 pi i k / fs)
    float2* regA = sm + Ls.tw;
    float2* regB = regA + Ls.A;
    // staged time spectra [NB][NF][NIN px][NIN py] of channels ch (even, odd) in two
    // buffers: the next channel's are staged while this one's are transformed
    // (an offset, not a choice between two pointers: a pointer pair indexed by the
    // channel parity ends up in scratch memory)
    const int zdelta = Ls.A;                // regB - regA
    auto zbs = [&](int ch) { return regA + (ch & 1) * zdelta; };
    float2* abuf = regA + Ls.zsz;           // [NB][NF][FS kx][P1 py]
    for (int i = tid; i < FS; i += NT) twl[i] = tws[i];

    const int ptiles = A.ppad / kTileT;
    const int64_t tstride = (int64_t)ptiles * A.ft * kTileT;   // one channel of T
    const float2* Tb = T + (int64_t)bl0 * A.nch * tstride;
    // Staged time spectra of one channel: element i of zbuf (py fastest, then px, fl,
    // bin) comes from T at a fixed per-thread offset plus the channel stride. The
    // loads are unconditional, so that no wait for them is forced before the
    // arithmetic that follows: elements outside the bins and elements of row groups
    // that the time FFT flagged empty (their spectra were not written) take an offset
    // past the end of the buffer resource, which reads zero without touching memory.
    // (byte offsets from channel ch of bin bl0; the host keeps NB channels' worth of
    // bins below 2^31 bytes)
    constexpr uint32_t kOob = 0xfffffff0u;
    const int ng = A.ppad / kTile;
    uint32_t zoff[ZPT], zfo[ZPT];
    bool zval[ZPT];
#pragma unroll
    for (int k = 0; k < ZPT; ++k) {
        const int i = tid + k * NT;
        const int py = i % NIN;
        int r = i / NIN;
        const int px = r % NIN;
        r /= NIN;
        const int fl2 = r % NF;
        const int b = r / NF;
        zval[k] = i < NZ && b < nbv && px < Bx && py < By;
        const int p = px * By + py;
        zoff[k] = (uint32_t)(8 * (zval[k] ? ((int64_t)b * A.nch) * tstride +
                                                ((int64_t)(p / kTileT) * A.ft + f0 + fl2) * kTileT +
                                                p % kTileT
                                          : (int64_t)f0 * kTileT));
        zfo[k] = zval[k] ? (uint32_t)(b * A.nch * ng + p / kTile) : 0u;
    }
    // the flags of this workgroup's bins, [b][ch][group], staged in LDS once
    uint8_t* zflag = reinterpret_cast<uint8_t*>(sm + Ls.total);
    for (int i = tid; i < NB * A.nch * ng; i += NT)
        zflag[i] = i < nbv * A.nch * ng ? A.tflag[(int64_t)bl0 * A.nch * ng + i] : 0;
    __syncthreads();
    // the flag bytes of channel ch's elements, read one channel ahead of their loads
    // (unconditional LDS reads: the element's own group, or group 0 of bin 0)
    uint32_t zfb[ZPT];
    auto flags = [&](int ch) {
#pragma unroll
        for (int k = 0; k < ZPT; ++k) zfb[k] = zflag[zfo[k] + ch * ng];
    };
    float2 zpre[ZPT];
    auto load_T = [&](int ch) {   // with zfb read for channel ch
        const auto tr = buf_rsrc(Tb + (int64_t)ch * tstride,
                                 (uint32_t)(((int64_t)nbv * A.nch - ch) * tstride * 8));
#pragma unroll
        for (int k = 0; k < ZPT; ++k)
            zpre[k] = buf_f2(tr, (zval[k] & (zfb[k] != 0u)) ? zoff[k] : kOob, 0u);
    };
    auto store_T = [&](float2* zbuf) {
#pragma unroll
        for (int k = 0; k < ZPT; ++k) {
            const int i = tid + k * NT;
            if (i < NZ) zbuf[i] = zpre[k];
        }
    };

    static_assert(NC == 2 || NC == 4, "pieces");
    float2 acc[NB][NC][L];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int m = 0; m < L; ++m) acc[b][c][m] = make_float2(0.f, 0.f);
    flags(0);
    load_T(0);
    flags(min(1, A.nch - 1));
    float2 wy[RS];   // W_RS^(j k2) of this thread's rows
#pragma unroll
    for (int j = 0; j < RS; ++j) wy[j] = twl[((j * k2) % RS) * L];
    store_T(zbs(0));
    load_T(min(1, A.nch - 1));
    flags(min(2, A.nch - 1));
    __syncthreads();
    constexpr int LP = (L + 1) / 2 * 2;                 // rows stored (odd L: one pad row)
    const int64_t rstride = (int64_t)A.nc * LP * TPF;   // nc * LP * TPF values per (ch, f)
    // response spectra of (ch, f0 .. f0 + NF - 1) as row pairs [c][m / 2][item][m % 2]
    const uint32_t rbytes = (uint32_t)(NF * rstride * 8);
    const uint32_t rvoff = (uint32_t)(fl * rstride * 8 + item * 16);

    // x pass: for each (bin, frequency, py, k2x) an L-point DFT over the gathered px.
    // With at most one item per thread its phase factors are read once, here (not at
    // fs 36, whose three waves per SIMD cap the registers at 168).
    constexpr bool XONE = NB * NF * NIN * RS <= NT && FS != 36;
    float2 wx[RS];
#pragma unroll
    for (int j = 0; j < RS; ++j) wx[j] = twl[((j * (tid % RS)) % RS) * L];
    auto xpass = [&](const float2* zbuf, float2* ab) {
        for (int i = tid; i < NB * NF * NIN * RS; i += NT) {
            const int kk = i % RS;
            int r = i / RS;
            const int py = r % NIN;
            const int bf = r / NIN;   // b * NF + fl2
            float2 t[L];
            if (py < By) {
                const float2* zr = zbuf + bf * NIN * NIN + py;
                float2 x[NIN];
#pragma unroll
                for (int px = 0; px < NIN; ++px) x[px] = zr[px * NIN];
                float2 w[RS];
#pragma unroll
                for (int j = 0; j < RS; ++j) w[j] = XONE ? wx[j] : twl[((j * kk) % RS) * L];
                pfa_gather<L, RS, NIN>(x, w, t);
                Dft<L>::run(t);
            } else {
#pragma unroll
                for (int m = 0; m < L; ++m) t[m] = make_float2(0.f, 0.f);
            }
            float2* ar = ab + bf * FS * P1 + py;
#pragma unroll
            for (int m = 0; m < L; ++m) ar[P::k_of(m, kk) * P1] = t[m];
        }
    };
    // y pass and multiply-accumulate with the response spectra of every piece, for
    // channel ch from the x-pass output ab. The spectra of piece 0 are requested before
    // the y pass and those of piece c + 1 before the multiply-adds of piece c (two or
    // three register buffers), so L2 latency is covered by arithmetic. Vector loads
    // complete in issue order, so a wait for response spectra also waits for every
    // time-spectra load issued before them: the time spectra of channel ch + AH + 1 are
    // requested after the last piece's response spectra, which leaves the rest of this
    // channel and what follows before any wait depends on them, and those of channel
    // ch + AH (requested AH channels ago) are staged after the y pass. Everything is
    // unconditional: pieces past nc load piece nc - 1 again and accumulate into slots
    // that are never read, the last channels request the last channel again.
    auto ymac = [&](int ch, const float2* ab, int AH) {
        const auto rr = buf_rsrc(rhat + ((int64_t)ch * A.ft + f0) * rstride, rbytes);
        auto load_w = [&](float2* wv, int c) {
#pragma unroll
            for (int mp = 0; mp < LP / 2; ++mp) {
                const float4 v = buf_f4(rr, rvoff, (uint32_t)((c * LP + 2 * mp) * TPF * 8));
                wv[2 * mp] = make_float2(v.x, v.y);
                wv[2 * mp + 1] = make_float2(v.z, v.w);
            }
        };
        const int clast = A.nc - 1;
        // WB register buffers: piece c + WB - 1 is requested before the multiply-adds of
        // c (three where the registers allow it)
        constexpr int WB = (RS == 5 || FS == 8) ? 3 : 2;
        float2 w[WB][LP];
        load_w(w[0], 0);
        if (WB == 3) load_w(w[1], min(1, clast));
        __builtin_amdgcn_sched_barrier(0);
        float2 s[NB][L];
        if (active) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float4* ar4 = (const float4*)(ab + ((b * NF + fl) * FS + kx) * P1);
                float2 x[NIN];
#pragma unroll
                for (int q = 0; q < NIN / 2; ++q) {
                    const float4 v = ar4[q];
                    x[2 * q] = make_float2(v.x, v.y);
                    x[2 * q + 1] = make_float2(v.z, v.w);
                }
                pfa_gather<L, RS, NIN>(x, wy, s[b]);
                Dft<L>::run(s[b]);
            }
        }
        // channel ch + AH into its buffer (the x pass that last read that buffer ended
        // before this phase)
        store_T(zbs(ch + AH));
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c + WB - 1 < NC) load_w(w[(c + WB - 1) % WB], min(c + WB - 1, clast));
            if (c == (NC > WB ? NC - WB : 0)) {   // after the last piece's request (and store_T)
                __builtin_amdgcn_sched_barrier(0);   // vector loads complete in issue order
                load_T(min(ch + AH + 1, A.nch - 1));
                flags(min(ch + AH + 2, A.nch - 1));
            }
            __builtin_amdgcn_sched_barrier(0);
            if (active) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int m = 0; m < L; ++m)
                        acc[b][c][m] = cfma(s[b][m], w[c % WB][m], acc[b][c][m]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    if constexpr (TRED_SPP_PIPE != 0) {
        // channel pipeline: the x pass of channel ch + 1 and the y pass and
        // multiply-adds of channel ch share one phase (one barrier per channel); the
        // x-pass output is double-buffered after the staged time spectra of the same
        // channel parity
        auto abufs = [&](int ch) { return zbs(ch) + Ls.zsz; };
        xpass(zbs(0), abufs(0));
        store_T(zbs(1));
        load_T(min(2, A.nch - 1));
        flags(min(3, A.nch - 1));
        __syncthreads();
        for (int ch = 0; ch < A.nch; ++ch) {
            if (TRED_SPP_PIPE == 1 && ch + 1 < A.nch) xpass(zbs(ch + 1), abufs(ch + 1));
            __builtin_amdgcn_sched_barrier(0);
            ymac(ch, abufs(ch), 2);
            __builtin_amdgcn_sched_barrier(0);
            if (TRED_SPP_PIPE == 2 && ch + 1 < A.nch) xpass(zbs(ch + 1), abufs(ch + 1));
            __syncthreads();
        }
    } else {
        for (int ch = 0; ch < A.nch; ++ch) {
            xpass(zbs(ch), abuf);
            __syncthreads();
            ymac(ch, abuf, 1);
            __syncthreads();
        }
    }

    // inverse spatial transforms of every response piece and the mirror-pair unpacking.
    // Per piece: the k1 inverse from the accumulators (M), the k2 inverse (Y, RS > 1),
    // the x inverse over k1 (X) and over k2 (R, RS > 1), then the unpacking and stores
    // of U (S). S of piece c - 1 reads y2 while M of piece c writes the other LDS
    // region, so the two share a phase (four barriers per piece). Between the stages the
    // values are kept conjugated where that saves sign flips: Y and R store their DFTs
    // as computed (the conjugates of the inverses), X transforms Y's output as read, and
    // S folds the last conjugation into the unpacking.
    const int qtiles = A.qpad / kTile;
    float2* gbuf = regA;                    // [NB][NF][FS kx][L n1][RS k2]
    float2* ybuf = regB;                    // [NB][NF][FS kx][YB qy]
    float2* g2 = regA;                      // [NB][NF][boy qy][L n1][RS k2]
    float2* y2 = RS > 1 ? regB : regA;      // [NB][NF][box qx][YB qy], conjugated
    // S items of this thread, the same for every piece: i = tid + NT k over [b][qt][fl2][qi];
    // the y2 offsets of Y[q] and of its mirror Y[q'] (16 bits each; bit 31: q >= nq,
    // stores zero) and the byte offset in piece c's part of this workgroup's bins of U
    // (past the buffer resource for items outside the bins: dropped)
    constexpr int QTM = (FS * FS + kTile - 1) / kTile;
    constexpr int IS = (NB * QTM * NF * kTile + NT - 1) / NT;
    static_assert(NB * NF * FS * (FS + 1) < 32768, "packed y2 offsets");
    const int nq = box * boy;
    const int nst = NB * qtiles * NF * kTile;
    uint32_t s_src[IS], s_off[IS];
#pragma unroll
    for (int k = 0; k < IS; ++k) {
        const int i = tid + NT * k;
        const int qi = i % kTile;
        int r = i / kTile;
        const int fl2 = r % NF;
        r /= NF;
        const int qt = r % qtiles;
        const int b = r / qtiles;
        const int q = qt * kTile + qi;
        const bool ok = i < nst && b < nbv;
        uint32_t sp = 0x80000000u;
        if (ok && q < nq) {
            const int qx = q / boy, qy = q % boy;
            const int base = (b * NF + fl2) * box * YB;
            sp = (uint32_t)(base + qx * YB + qy) | ((uint32_t)(base + (box - 1 - qx) * YB + (boy - 1 - qy)) << 16);
        }
        s_src[k] = sp;
        s_off[k] = ok ? (uint32_t)(8 * ((((int64_t)b * A.nc * qtiles + qt) * A.ft + f0 + fl2) * kTile + qi))
                      : 0xfffffff0u;
    }
    const int64_t upiece = (int64_t)qtiles * A.ft * kTile;   // elements of one piece of a bin
    float2* Ub = U + (int64_t)bl0 * A.nc * upiece;
    const int64_t ubytes = (int64_t)nbv * A.nc * upiece * 8;   // below 2^31 (host check)
    auto store_piece = [&](int c, const float2* y2c) {
        const auto ur = buf_rsrc(Ub + (int64_t)c * upiece, (uint32_t)(ubytes - (int64_t)c * upiece * 8));
#pragma unroll
        for (int k = 0; k < IS; ++k) {
            const uint32_t sp = s_src[k];
            const float2 a = y2c[sp & 0xffffu], m = y2c[(sp >> 16) & 0x7fffu];
            // y2 holds conj(Y): I[q] = Re Y[q] + Im Y[q'] (mirror pair) or Y[q]
            float2 vq = A.mpcp ? make_float2(a.x - m.y, -a.y - m.x) : make_float2(a.x, -a.y);
            if (sp >> 31) vq = make_float2(0.f, 0.f);
            buf_st_f2(vq, ur, s_off[k], 0u);
        }
    };
    // M: y-inverse, L-point stage over k1 (conj(DFT(conj .)) = inverse DFT) of piece c
    // (called from fully unrolled loops, so c indexes the accumulators at compile
    // time); RS > 1: into gbuf, else into ybuf
    auto stage_m = [&](int c) {
        if (active) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                float2 t[L];
#pragma unroll
                for (int m = 0; m < L; ++m) t[m] = cconj(acc[b][c][m]);
                Dft<L>::run(t);
                const int bf = b * NF + fl;
                if constexpr (RS == 1) {
                    float2* yr = ybuf + (bf * FS + kx) * YB;   // conjugated
#pragma unroll
                    for (int n = 0; n < L; ++n)
                        if (n < boy) yr[n] = t[n];
                } else {
                    float2* gr = gbuf + ((bf * FS + kx) * L) * RS + k2;
#pragma unroll
                    for (int n = 0; n < L; ++n) gr[n * RS] = t[n];   // conjugated partial sums
                }
            }
        }
    };
    // Y: y-inverse, RS-point stage over k2 -> qy = n_of(n1, n2) < boy (conjugated)
    auto stage_y = [&](float2* yb) {
        for (int i = tid; i < NB * NF * FS * L; i += NT) {
            const int n1 = i % L;
            const int r = i / L;   // bf * FS + kx
            const float2* gr = gbuf + (r * L + n1) * RS;
            float2 t[RS];
#pragma unroll
            for (int k = 0; k < RS; ++k) t[k] = gr[k];
            Dft<RS>::run(t);
            float2* yr = yb + r * YB;
            int qy = (RS * n1) % FS;   // n_of(n1, n2), stepping n2 by L (mod FS)
#pragma unroll
            for (int n2 = 0; n2 < RS; ++n2) {
                if (qy < boy) yr[qy] = t[n2];
                qy += L;
                qy = qy >= FS ? qy - FS : qy;
            }
        }
    };
    // X: x-inverse, L-point stage over kx = k_of(k1, k2x) for every qy (the conjugated
    // y inverse is the DFT's input as stored). Items run over qy < FS (a compile-time
    // bound, so that their decomposition is shifts and multiplies by constants); rows
    // qy >= boy are skipped. RS > 1: into g2 [bf][boy qy][L n1][RS kk], else into y2.
    auto stage_x = [&](const float2* yb, float2* dst) {
        for (int i = tid; i < NB * NF * FS * RS; i += NT) {
            const int kk = i % RS;
            const int r = i / RS;     // bf * FS + qy
            const int qy = r % FS, bf = r / FS;
            if (qy >= boy) continue;
            const float2* yr = yb + bf * FS * YB + qy;
            float2 t[L];
            const int kb = (Pfa<L, RS>::k_of(0, 1) * kk) % FS;   // k_of(0, kk)
#pragma unroll
            for (int m = 0; m < L; ++m) {
                int kxm = kb + P::k_of(m, 0);
                kxm = kxm >= FS ? kxm - FS : kxm;
                t[m] = yr[kxm * YB];
            }
            Dft<L>::run(t);
            if constexpr (RS == 1) {
#pragma unroll
                for (int n = 0; n < L; ++n)
                    if (n < box) dst[(bf * box + n) * YB + qy] = t[n];
            } else {
                float2* gr = dst + ((bf * boy + qy) * L) * RS + kk;
#pragma unroll
                for (int n = 0; n < L; ++n) gr[n * RS] = t[n];
            }
        }
    };
    // R: x-inverse, RS-point stage -> qx = n_of(n1, n2) < box (conjugated); items over
    // qy < FS as in X
    auto stage_r = [&](const float2* g2c, float2* y2c) {
        for (int i = tid; i < NB * NF * FS * L; i += NT) {
            const int n1 = i % L;
            const int r = i / L;  // bf * FS + qy
            const int qy = r % FS, bf = r / FS;
            if (qy >= boy) continue;
            const float2* gr = g2c + ((bf * boy + qy) * L + n1) * RS;
            float2 t[RS];
#pragma unroll
            for (int k = 0; k < RS; ++k) t[k] = gr[k];
            Dft<RS>::run(t);
            float2* yc = y2c + bf * box * YB + qy;
            int qx = (RS * n1) % FS;   // n_of(n1, n2)
#pragma unroll
            for (int n2 = 0; n2 < RS; ++n2) {
                if (qx < box) yc[qx * YB] = t[n2];
                qx += L;
                qx = qx >= FS ? qx - FS : qx;
            }
        }
    };
    if constexpr (RS > 1) {
        // Three phases per piece: {M(c), R(c - 1)}, {Y(c), S(c - 1)}, {X(c)}. M writes
        // gbuf (region A); the k2-inverse output, the x-inverse intermediate and the
        // output of piece c lie in (B, C, B) for even c and (C, B, C) for odd c, so no
        // phase writes a buffer that another of its stages reads, and every buffer is
        // read before the phase that overwrites it.
        auto yb_of = [&](int c) { return regB + (c & 1) * Ls.B; };          // y and y2
        auto g2_of = [&](int c) { return regB + ((c & 1) ^ 1) * Ls.B; };    // g2
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c >= A.nc) break;
            stage_m(c);
            if (c > 0) stage_r(g2_of(c - 1), yb_of(c - 1));
            __syncthreads();
            stage_y(yb_of(c));
            if (c > 0) store_piece(c - 1, yb_of(c - 1));
            __syncthreads();
            stage_x(yb_of(c), g2_of(c));
            __syncthreads();
        }
        stage_r(g2_of(A.nc - 1), yb_of(A.nc - 1));
        __syncthreads();
        store_piece(A.nc - 1, yb_of(A.nc - 1));
    } else {
        // two phases per piece: {M(c) into ybuf, S(c - 1) from y2 (region A)}, {X(c)}
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c >= A.nc) break;
            stage_m(c);
            if (c > 0) store_piece(c - 1, y2);
            __syncthreads();
            stage_x(ybuf, y2);
            __syncthreads();
        }
        store_piece(A.nc - 1, y2);
    }
}

// ---------------------------------------------------------------------------
// k_ti: inverse time FFT of each output pixel and response piece; the real part of
// piece c lands at tick offset c * ct. The lane that owns tick a in piece c owned
// it in every earlier piece (ct is a multiple of 64), so the overlap is added in
// program order by one thread.
// ---------------------------------------------------------------------------
// Four waves per SIMD (two 8-wave workgroups per CU; the compiler's choice of 145
// registers at ft = 1024 leaves one) for a spill of a few registers.
template <int FT, bool CARRY>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(FT <= 1024 ? 4 : 1))) void k_ti(ConvArgs A, int b0, const int32_t* __restrict__ n_active,
                                            const float2* __restrict__ U,
                                            const float2* __restrict__ tw, float* __restrict__ out) {
    extern __shared__ float lds[];
    constexpr int M = FT / kWave;
    const int bl = blockIdx.y, b = b0 + bl;
    if (b >= min(*n_active, A.cap)) return;
    const int qt = blockIdx.x;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = qt * kTile + wv;
    const bool valid = q < A.box * A.boy;
    const int qtiles = A.qpad / kTile;
    float* orow = out + (int64_t)b * A.vout + (int64_t)(valid ? q : 0) * A.bot;
    // CARRY (pieces of half the transform length, ct = Bt = FT / 2): the second half of
    // piece c overlaps only the first half of piece c + 1, so it is carried in
    // registers and every output tick is written once; otherwise overlaps are added
    // in memory
    constexpr int MH = M / 2;
    float carry[MH];
#pragma unroll
    for (int m = 0; m < MH; ++m) carry[m] = 0.0f;
    // twiddle table in LDS after the FFT scratch / staging region
    float2* twl = (float2*)(lds + tf_lds_floats<FT>());
    fft_tw_fill<FT>(twl, tw, threadIdx.x, blockDim.x);
    for (int c = 0; c < A.nc; ++c) {
        const float2* s2 = U + ((((int64_t)bl * A.nc + c) * qtiles + qt) * FT) * kTile;
        float2* stage = (float2*)lds;   // [f][kTile], columns swizzled (tf_col)
        // the tile is requested in groups of four 16-byte loads (two pixels of one
        // frequency each) that are in flight together before their LDS writes
        constexpr int NLD = FT * kTile / 2 / 512, G = NLD < 4 ? NLD : 4;
        static_assert(FT * kTile % 1024 == 0 && kTile % 2 == 0 && NLD % G == 0, "tile loads");
        const auto ur = buf_rsrc(s2, (uint32_t)(FT * kTile * sizeof(float2)));
#pragma unroll
        for (int k0 = 0; k0 < NLD; k0 += G) {
            float4 ld[G];
#pragma unroll
            for (int k = 0; k < G; ++k)
                ld[k] = buf_f4(ur, threadIdx.x * 16u, (uint32_t)((k0 + k) * 512 * 16));
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int i = 2 * ((int)threadIdx.x + 512 * (k0 + k));
                const int f = i / kTile, c = i % kTile;
                stage[f * kTile + tf_col(f, c)] = make_float2(ld[k].x, ld[k].y);
                stage[f * kTile + tf_col(f, c + 1)] = make_float2(ld[k].z, ld[k].w);
            }
        }
        __syncthreads();
        float2 v[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int f = lane + kWave * m;
            v[m] = cconj(stage[f * kTile + tf_col(f, wv)]);
        }
        __syncthreads();
        wave_fft<FT, TRED_TI_WAVESYNC, true>(v, lds + wv * kFftLds<FT>, twl, lane);
        __syncthreads();   // the next piece's tile overlaps the other waves' FFT scratch
        if (valid) {
            if constexpr (CARRY) {
                const bool last = c == A.nc - 1;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int a = c * A.ct + lane + kWave * m;
                    const float r = v[m].x;   // Re conj(.) = Re(.)
                    if (m < MH) {
                        if (a < A.bot) orow[a] = r + carry[m];
                    } else if (last) {
                        if (a < A.bot) orow[a] = r;
                    } else {
                        carry[m - MH] = r;
                    }
                }
            } else {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int t = lane + kWave * m;
                    const int a = c * A.ct + t;
                    if (a < A.bot) {
                        const float r = v[m].x;
                        if (c > 0 && t < A.Bt) orow[a] += r;
                        else orow[a] = r;
                    }
                }
            }
        }
    }
}

// ===========================================================================
// Transpose of the convolution (gradients, Sec. V-C). For one bin the forward map is
//   out = OLA_c Re F_t^H Unpack Crop F_xy^H ( sum_ch Rhat[ch][c] F_xy F_t Pack(Q_ch) )
// with F the unnormalised DFT (the 1/N factors live in Rhat). Its transpose (real
// inner products) runs the same stages backwards:
//   dQ = Pack^T Crop_Bt F_t^H ( Crop_B F_xy^H sum_c conj(Rhat[ch][c]) F_xy Unpack^H F_t Seg_c(dout) )
// k_ti_adj: F_t of each output-gradient piece segment -> dU (layout of U);
// k_spp_adj: per frequency, Unpack^H and F_xy of the pieces, the conjugate multiply-
//            accumulate into every channel, F_xy^H pruned to the bin -> dT (layout of T);
// k_tf_adj:  F_t^H of every (channel, pixel) row cropped to Bt, Pack^T -> d blocks.
// ===========================================================================

// k_ti_adj: per (output-pixel tile, piece, bin); wave wv handles pixel qt * 8 + wv.
template <int FT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(FT <= 1024 ? 4 : 1))) void k_ti_adj(
    ConvArgs A, int b0, const int32_t* __restrict__ n_active, const float* __restrict__ dout,
    const float2* __restrict__ tw, float2* __restrict__ dU) {
    extern __shared__ float lds[];
    constexpr int M = FT / kWave;
    const int qt = blockIdx.x, c = blockIdx.y, bl = blockIdx.z, b = b0 + bl;
    if (b >= min(*n_active, A.cap)) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = qt * kTile + wv;
    const bool valid = q < A.box * A.boy;
    float2* twl = (float2*)(lds + tf_lds_floats<FT>());
    fft_tw_fill<FT>(twl, tw, threadIdx.x, blockDim.x);
    const float* row = dout + (int64_t)b * A.vout + (int64_t)(valid ? q : 0) * A.bot;
    float2 v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int a = c * A.ct + lane + kWave * m;   // output tick of piece sample t
        v[m] = make_float2(valid && a < A.bot ? row[a] : 0.0f, 0.0f);
    }
    __syncthreads();
    wave_fft<FT, true, true>(v, lds + wv * kFftLds<FT>, twl, lane);
    __syncthreads();
    float2* stage = (float2*)lds;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int f = lane + kWave * m;
        stage[f * kTile + tf_col(f, wv)] = v[m];
    }
    __syncthreads();
    const int qtiles = A.qpad / kTile;
    float2* d2 = dU + ((((int64_t)bl * A.nc + c) * qtiles + qt) * FT) * kTile;
    // the tile is contiguous: thread t writes elements i, i + 1 (i = 2 (t + 512 k), so
    // pixels cc, cc + 1 of one row, one aligned LDS pair under the swizzle, swapped
    // where the swizzle flips bit 0) with one 16-byte store
    {
        static_assert(FT * kTile % 1024 == 0 && kTile % 2 == 0, "tile stores");
        const auto dr = buf_rsrc(d2, (uint32_t)(FT * kTile * sizeof(float2)));
#pragma unroll
        for (int k = 0; k < FT * kTile / 1024; ++k) {
            const int i = 2 * ((int)threadIdx.x + 512 * k);
            const int f = i / kTile, cc = i % kTile;
            const int sw = (f >> 2) & (kTile - 1);
            const float4 p = *(const float4*)(stage + f * kTile + ((cc ^ sw) & ~1));
            buf_st_f4((sw & 1) ? make_float4(p.z, p.w, p.x, p.y) : p, dr, (uint32_t)(i * 8), 0u);
        }
    }
}

// Row groups of the time transforms that hold a marked row (its own or the mirror
// row of the pair): tflag[bin][ch][p / kTile] = 1, else 0. Used by the transposed
// convolution with row masks, whose outputs are needed on the marked rows only.
__global__ __launch_bounds__(256) void k_group_need(ConvArgs A, int b0, int nb,
                                                    const int32_t* __restrict__ n_active) {
    const int ng = A.ppad / kTile;
    const int64_t total = (int64_t)nb * A.nch * ng;
    const int nact = min(*n_active, A.cap) - b0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)(i % ng);
        const int ch = (int)((i / ng) % A.nch);
        const int bl = (int)(i / ((int64_t)ng * A.nch));
        uint8_t need = 0;
        if (bl < nact) {
            const uint32_t* rw = A.rows + (int64_t)(b0 + bl) * A.nrw;
            const int jx = ch / A.sy, jy = ch % A.sy;
            const int jb = A.S - 1 - ch;
            const bool pair = A.mpcp && jb != ch;
            const int jbx = jb / A.sy, jby = jb % A.sy;
            for (int w = 0; w < kTile; ++w) {
                const int p = g * kTile + w;
                if (p >= A.Bx * A.By) break;
                const int px = p / A.By, py = p % A.By;
                const int r0 = (px * A.sx + jx) * A.NYf + (py * A.sy + jy);
                const int r1 = ((A.Bx - 1 - px) * A.sx + jbx) * A.NYf + ((A.By - 1 - py) * A.sy + jby);
                if ((rw[r0 >> 5] >> (r0 & 31)) & 1u) need = 1;
                if (pair && ((rw[r1 >> 5] >> (r1 & 31)) & 1u)) need = 1;
            }
        }
        A.tflag[i] = need;
    }
}

// k_tf_adj: the transpose of the time FFT per group (bin, channel, half T tile): F^H of
// the group's 8 rows of T-layout gradients (wave wv: pixel wv of the half tile),
// cropped to Bt ticks and unpacked from the mirror pair into the rows of d blocks.
// Workgroups are persistent (groups q = w, w + G, ..., with tf_group's order, so the
// two halves of a tile go to one XCD) and request a group's half tile one iteration
// before its transform and its need flag (row masks) two iterations before, so the
// reads of the spectra overlap the transforms. Every iteration issues the same vector
// memory operations in the same order (as in k_tf_list): a group that is not needed
// (no marked row or mirror row), a row that is not marked and the ticks past Bt
// address an empty buffer resource or an offset past its end, which reads zero and
// drops stores, so each wait is for the operation it needs.
template <int FT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(FT <= 1024 ? 4 : 1))) void k_tf_adj(
    ConvArgs A, int b0, int nb, const int32_t* __restrict__ n_active, const float2* __restrict__ dT,
    const float2* __restrict__ tw, float* __restrict__ dblocks) {
    extern __shared__ float lds[];
    constexpr int M = FT / kWave;
    constexpr int SPT = FT * kTile / 512;   // staged half-tile values per thread
    constexpr uint32_t kOob = 0xfffffff0u;
    const int nact = min(min(*n_active, A.cap) - b0, nb);
    if (nact <= 0) return;
    const int nbx = A.ppad / kTile;
    const int total = nact * A.nch * nbx;   // groups (the host keeps nb * nch * nbx < 2^31)
    const int G = (int)gridDim.x;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int ntile = A.ppad / kTileT;
    const int mb = A.Bt / kWave;
    float2* twl = (float2*)(lds + tf_lds_floats<FT>());
    fft_tw_fill<FT>(twl, tw, threadIdx.x, blockDim.x);
    const auto fr = buf_rsrc(A.tflag, A.rows ? (uint32_t)total : 0u);
    // need flag of group q (requested now, read an iteration later); 1 without row masks
    auto load_flag = [&](int q) -> uint32_t {
        const int qc = min(q, total - 1);
        const TfGroup g = tf_group(A, qc);
        const uint32_t idx = (uint32_t)(qc - qc % nbx + g.pt * (kTileT / kTile) + g.half);
        const uint32_t f = buf_u8(fr, idx, 0u);
        return A.rows ? f : 1u;
    };
    // half tile of group q: thread t holds columns t % kTile of rows f = t / kTile +
    // (512 / kTile) k, read from the tile's [f][kTileT] layout
    float2 pre[SPT];
    auto load = [&](int q, bool need) {
        const int qc = min(q, total - 1);
        const TfGroup g = tf_group(A, qc);
        const float2* s2 = dT + (((int64_t)g.bl * A.nch + g.ch) * ntile + g.pt) * FT * kTileT +
                           g.half * kTile;
        const auto r = buf_rsrc(s2, need && q < total ? (uint32_t)((FT * kTileT - g.half * kTile) * 8) : 0u);
        const int f0 = (int)threadIdx.x / kTile, cc = (int)threadIdx.x % kTile;
        const uint32_t voff = (uint32_t)((f0 * kTileT + cc) * 8);
#pragma unroll
        for (int k = 0; k < SPT; ++k)
            pre[k] = buf_f2(r, voff, (uint32_t)(k * (512 / kTile) * kTileT * 8));
    };
    __syncthreads();
    int q = (int)blockIdx.x;
    uint32_t need = __builtin_amdgcn_readfirstlane(load_flag(q));
    load(q, need != 0u);
    uint32_t fnext = load_flag(q + G);
    for (; q < total; q += G) {
        const TfGroup g = tf_group(A, q);
        // stage the half tile [f][kTile] (columns swizzled) and take this wave's column
        float2* stage = (float2*)lds;
        {
            const int f0 = (int)threadIdx.x / kTile, cc = (int)threadIdx.x % kTile;
#pragma unroll
            for (int k = 0; k < SPT; ++k) {
                const int f = f0 + (512 / kTile) * k;
                stage[f * kTile + tf_col(f, cc)] = pre[k];
            }
        }
        __syncthreads();
        float2 v[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int f = lane + kWave * m;
            v[m] = cconj(stage[f * kTile + tf_col(f, wv)]);
        }
        __syncthreads();   // the staging tile overlaps the FFT scratch
        const bool cur = need != 0u;
        // the next group's half tile and the flag after it, in flight during the transform
        need = __builtin_amdgcn_readfirstlane(fnext);
        load(q + G, need != 0u);
        fnext = load_flag(q + 2 * G);
        if (cur) wave_fft<FT, true, true>(v, lds + wv * kFftLds<FT>, twl, lane);   // F^H = conj F conj
        // rows of pixel p: Q_j (real part) and, under mirror-pair packing, Q_j' of the
        // mirrored pixel (imaginary part); with row masks only marked rows are written
        const int p = g.pt * kTileT + g.half * kTile + wv;
        const bool pv = cur && p < A.Bx * A.By;
        const int pc = min(p, A.Bx * A.By - 1);
        const int jx = g.ch / A.sy, jy = g.ch % A.sy;
        const int jb = A.S - 1 - g.ch;
        const bool pair = A.mpcp && jb != g.ch;
        const int px = pc / A.By, py = pc % A.By;
        const int jbx = jb / A.sy, jby = jb % A.sy;
        const int q0 = (px * A.sx + jx) * A.NYf + (py * A.sy + jy);
        const int q1 = ((A.Bx - 1 - px) * A.sx + jbx) * A.NYf + ((A.By - 1 - py) * A.sy + jby);
        bool w0 = pv, w1 = pv && pair;
        if (A.rows) {
            const uint32_t* rw = A.rows + (int64_t)(b0 + g.bl) * A.nrw;
            w0 = w0 && ((rw[q0 >> 5] >> (q0 & 31)) & 1u);
            w1 = w1 && ((rw[q1 >> 5] >> (q1 & 31)) & 1u);
        }
        float* blk = dblocks + (int64_t)(b0 + g.bl) * A.vblk;
        const uint32_t vb = (uint32_t)(A.vblk * 4);   // a bin is below 2^31 bytes
        const auto r0 = buf_rsrc(blk, w0 ? vb : 0u), r1 = buf_rsrc(blk, w1 ? vb : 0u);
        const uint32_t o0 = 4u * (uint32_t)(q0 * A.Bt + lane), o1 = 4u * (uint32_t)(q1 * A.Bt + lane);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float2 z = cconj(v[m]);
            const uint32_t so = (uint32_t)(m * kWave * 4);
            buf_st_f1(z.x, r0, m < mb ? o0 : kOob, m < mb ? so : 0u);
            buf_st_f1(z.y, r1, m < mb ? o1 : kOob, m < mb ? so : 0u);
        }
        __syncthreads();   // the next staging tile overlaps this transform's scratch
    }
}

// k_spp_adj: the transpose of k_spp for one group of NB bins at NF frequencies.
// Phase A (per piece): dU of the output pixels -> Unpack^H (dY[q] = dU[q] + i dU[q'])
// -> forward 2-D DFT with the box x boy inputs zero-padded to fs -> dacc[b][c][k1] in
// registers of thread (kx, k2), the layout of the forward accumulators.
// Phase B (per channel): s = sum_c conj(Rhat[ch][c]) dacc[c] -> inverse 2-D DFT with
// outputs pruned to the bin's Bx x By pixels -> dT[ch] (layout of T).
template <int FS, int L, int NIN, int NB>
struct SppAdjLds {
    int tw, P2, YB, du, a2, gb, yb, g2, ob, A, B, total;
};

template <int FS, int L, int NIN, int NB, int NF>
__host__ __device__ inline SppAdjLds<FS, L, NIN, NB> spp_adj_lds(int box, int boy, int Bx, int By) {
    constexpr int RS = FS / L;
    SppAdjLds<FS, L, NIN, NB> s;
    s.tw = even_up(FS);
    s.P2 = even_up(FS) + 2;                    // even: 16-byte rows for the column reads
    s.YB = (By % 2 == 0) ? By + 1 : By;
    s.du = NB * NF * boy * s.P2;                // output-gradient rows qy of P2 (qx fastest)
    s.a2 = NB * NF * FS * s.P2;
    s.gb = RS > 1 ? NB * NF * FS * L * RS : 0;
    s.yb = NB * NF * FS * s.YB;
    s.g2 = RS > 1 ? NB * NF * NIN * L * RS : 0;
    s.ob = NB * NF * Bx * By;
    s.A = even_up(s.du + s.a2);
    // the pipelined channel loop (RS > 1) holds the four stage buffers apart
    int bb = s.gb > s.g2 + s.ob ? s.gb : s.g2 + s.ob;
    s.B = RS > 1 ? even_up(s.gb + s.yb + s.g2 + s.ob) : even_up(bb + s.yb);
    s.total = s.tw + (s.A > s.B ? s.A : s.B);
    return s;
}

template <int FS, int L, int NIN, int NB>
__global__ __launch_bounds__((SppShape<FS, L, NIN, NB>::NT)) __attribute__((amdgpu_waves_per_eu(2))) void k_spp_adj(
    ConvArgs A, int b0, int nbp, const int32_t* __restrict__ n_active,
    const float2* __restrict__ dU, const float2* __restrict__ rhat,
    const float2* __restrict__ tws, float2* __restrict__ dT) {
    using S = SppShape<FS, L, NIN, NB>;
    using P = Pfa<L, S::RS>;
    constexpr int RS = S::RS, TPF = S::TPF, NF = S::NF, NT = S::NT;
    constexpr bool kPipe = RS > 1 && L <= 8;   // pipelined channel loop
    extern __shared__ float4 sm4[];
    float2* sm = (float2*)sm4;
    // bins fastest in the logical order; each XCD walks a contiguous range of
    // frequencies (as in k_spp), so a response-spectrum slab is fetched into one L2
    const unsigned nbg = gridDim.x, total = gridDim.x * gridDim.y;
    const unsigned wid = blockIdx.y * nbg + blockIdx.x;
    unsigned lid = wid;
    if (TRED_XCD_REMAP && total % kXcd == 0) lid = (wid % kXcd) * (total / kXcd) + wid / kXcd;
    const int na = min(*n_active, A.cap);
    const int nloc = min(nbp, na - b0);
    const int bl0 = (int)(lid % nbg) * NB;
    if (bl0 >= nloc) return;
    const int nbv = min(NB, nloc - bl0);
    const int f0 = (int)(lid / nbg) * NF;
    const int tid = threadIdx.x;
    const bool active = tid < NF * TPF;
    const int tw_ = active ? tid : NF * TPF - 1;
    const int fl = tw_ / TPF, item = tw_ % TPF;
    const int kx = item / RS, k2 = item % RS;
    const int Bx = A.Bx, By = A.By, box = A.box, boy = A.boy;
    const auto Ls = spp_adj_lds<FS, L, NIN, NB, NF>(box, boy, Bx, By);
    const int P2 = Ls.P2, YB = Ls.YB;
    float2* twl = sm;
    float2* reg = sm + Ls.tw;
    float2* du = reg;                  // [NB][NF][boy qy][P2 qx], zero past qx = box
    float2* a2 = reg + Ls.du;          // [NB][NF][FS kx][P2 qy]
    float2* gbuf = reg;                // [NB][NF][FS kx][L n1][RS k2]
    float2* g2 = reg;                  // [NB][NF][By py][L n1][RS kk]
    float2* ob = reg + Ls.g2;          // [NB][NF][Bx px][By py]
    float2* yb = reg + (Ls.gb > Ls.g2 + Ls.ob ? Ls.gb : Ls.g2 + Ls.ob);   // [NB][NF][FS kx][YB py]
    for (int i = tid; i < FS; i += NT) twl[i] = tws[i];
    // the staging rows are read whole (FS entries, unconditionally): the entries past the
    // output footprint (qx >= box, qy >= boy) are zero, written once here and never after
    for (int i = tid; i < Ls.A; i += NT) reg[i] = make_float2(0.f, 0.f);
    __syncthreads();
    float2 wy[RS];
#pragma unroll
    for (int j = 0; j < RS; ++j) wy[j] = twl[((j * k2) % RS) * L];
    const int qtiles = A.qpad / kTile;
    const int nq = box * boy;

    float2 dacc[NB][4][L];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c < A.nc) {
            // output-pixel gradients of piece c at the group's frequencies
            for (int i = tid; i < NB * NF * nq; i += NT) {
                const int q = i % nq;
                const int r = i / nq;   // b * NF + fl2
                const int fl2 = r % NF, b = r / NF;
                float2 u = make_float2(0.f, 0.f);
                if (b < nbv)
                    u = dU[((((int64_t)(bl0 + b) * A.nc + c) * qtiles + q / kTile) * A.ft + f0 + fl2) *
                               kTile + q % kTile];
                du[(r * boy + q % boy) * P2 + q / boy] = u;
            }
            __syncthreads();
            if (A.mpcp) {
                // dY[q] = dU[q] + i dU[q'] for the mirror pair (q, q'), in place
                const int npair = (nq + 1) / 2;
                for (int i = tid; i < NB * NF * npair; i += NT) {
                    const int q = i % npair, r = i / npair;
                    const int qm = nq - 1 - q;
                    float2* yy = du + r * boy * P2;
                    const int ia = (q % boy) * P2 + q / boy, ib = (qm % boy) * P2 + qm / boy;
                    const float2 u = yy[ia], w = yy[ib];
                    yy[ia] = make_float2(u.x - w.y, u.y + w.x);
                    if (ib != ia) yy[ib] = make_float2(w.x - u.y, w.y + u.x);
                }
                __syncthreads();
            }
            // x stage: for each (b, qy, kk) an L-point DFT over the gathered qx (zero past box)
            for (int i = tid; i < NB * NF * boy * RS; i += NT) {
                const int kk = i % RS;
                const int r = i / RS;   // bf * boy + qy
                const int qy = r % boy, bf = r / boy;
                const float4* dr4 = (const float4*)(du + r * P2);
                float2 x[FS];
#pragma unroll
                for (int q = 0; q < FS / 2; ++q) {
                    const float4 v = dr4[q];
                    x[2 * q] = make_float2(v.x, v.y);
                    x[2 * q + 1] = make_float2(v.z, v.w);
                }
                float2 w[RS];
#pragma unroll
                for (int j = 0; j < RS; ++j) w[j] = twl[((j * kk) % RS) * L];
                float2 t[L];
                pfa_gather<L, RS, FS>(x, w, t);
                Dft<L>::run(t);
                float2* ar = a2 + bf * FS * P2 + qy;
#pragma unroll
                for (int m = 0; m < L; ++m) ar[P::k_of(m, kk) * P2] = t[m];
            }
            __syncthreads();
            // y stage: thread (kx, k2) over the gathered qy (zero past boy)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float4* ar4 = (const float4*)(a2 + ((b * NF + fl) * FS + kx) * P2);
                float2 x[FS];
#pragma unroll
                for (int q = 0; q < FS / 2; ++q) {
                    const float4 v = ar4[q];
                    x[2 * q] = make_float2(v.x, v.y);
                    x[2 * q + 1] = make_float2(v.z, v.w);
                }
                pfa_gather<L, RS, FS>(x, wy, dacc[b][c]);
                Dft<L>::run(dacc[b][c]);
                if constexpr (kPipe) {   // held conjugated by the pipelined channel loop
#pragma unroll
                    for (int m = 0; m < L; ++m) dacc[b][c][m] = cconj(dacc[b][c][m]);
                }
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int m = 0; m < L; ++m) dacc[b][c][m] = make_float2(0.f, 0.f);
        }
    }

    const int64_t rstride = (int64_t)A.nc * L * TPF;
    const uint32_t rbytes = (uint32_t)(NF * rstride * 8);
    const uint32_t rvoff = (uint32_t)(fl * rstride * 8 + item * 16);
    const int ptiles = A.ppad / kTileT;
    const int64_t tstride = (int64_t)ptiles * A.ft * kTileT;   // one channel of T
    // output items of this thread (b, fl2, p): LDS source and byte offset in channel ch of
    // bin bl0 (the host keeps NB channels' worth of bins below 2^31 bytes)
    constexpr int IT5 = (NB * NF * NIN * NIN + NT - 1) / NT;
    int o_src[IT5];
    uint32_t o_off[IT5], o_fo[IT5];
    bool o_ok[IT5];
    // with row masks: the need flags of this workgroup's groups, [b][ch][group], in LDS;
    // the stores of groups without a marked row go past the end of the buffer resource
    // (dropped)
    const int ng = A.ppad / kTile;
    uint8_t* gflag = reinterpret_cast<uint8_t*>(sm + Ls.total);
    if (A.rows) {
        for (int i = tid; i < NB * A.nch * ng; i += NT)
            gflag[i] = i < nbv * A.nch * ng ? A.tflag[(int64_t)bl0 * A.nch * ng + i] : 0;
    }
    {
        const int npx = Bx * By;
#pragma unroll
        for (int k = 0; k < IT5; ++k) {
            const int i = tid + k * NT;
            const int p = i % npx;
            const int r = i / npx;   // b * NF + fl2
            const int fl2 = r % NF, b = r / NF;
            o_ok[k] = i < NB * NF * npx && b < nbv;
            o_src[k] = o_ok[k] ? r * npx + p : 0;
            o_off[k] = o_ok[k] ? (uint32_t)(8 * ((int64_t)b * A.nch * tstride +
                                                  ((int64_t)(p / kTileT) * A.ft + f0 + fl2) * kTileT +
                                                  p % kTileT))
                               : 0u;
            o_fo[k] = o_ok[k] ? (uint32_t)(b * A.nch * ng + p / kTile) : 0u;
        }
    }
    if constexpr (kPipe) {
        // Channel pipeline, two barriers per channel. Stages of channel ch:
        //   M  conjugate multiply-add over the pieces, L-point inverse over k1 -> gq
        //   Y  RS-point inverse over k2, rows py < By -> yq
        //   X  L-point inverse over kx = k_of(k1, kk) for every py < By -> g2q
        //   R  RS-point inverse, columns px < Bx -> obq
        //   S  stores of obq into dT
        // Interval A of step k runs M(k), X(k - 1) and S(k - 2); interval B runs Y(k) and
        // R(k - 1). Every stage has a buffer of its own, written in one interval and read
        // in the next, so one barrier closes each interval. The response spectra of the
        // first PRE pieces of M(k) are requested at the start of interval A, ahead of the
        // X and S work, and piece c + PRE after the multiply-adds of piece c (a ring of
        // PRE register buffers; the last piece is requested again where c + PRE >= nc).
        // The inverse transforms are forward DFTs of conjugates, and the values between
        // stages are kept conjugated so that no stage flips signs: the accumulators hold
        // conj(dacc), so M sums conj(dacc) Rhat = conj(sum dacc conj(Rhat)) and its DFT is
        // the conjugated k1 inverse; Y's DFT is the conjugate of the k2 inverse, which X
        // transforms as read; R conjugates its outputs once.
        float2* gq = reg;                  // [NB][NF][FS kx][L n1][RS k2]
        float2* yq = gq + Ls.gb;           // [NB][NF][FS kx][YB py]
        float2* g2q = yq + Ls.yb;          // [NB][NF][NIN py][L n1][RS kk]
        float2* obq = g2q + Ls.g2;         // [NB][NF][Bx px][By py]
        constexpr int PRE = TRED_SPP_ADJ_PRE;   // pieces requested ahead (registers)
        static_assert(PRE >= 1 && PRE <= 4, "pieces requested ahead");
        const int clast = A.nc - 1;
        auto stage_y = [&]() {
            for (int i = tid; i < NB * NF * FS * L; i += NT) {
                const int n1 = i % L;
                const int r = i / L;   // bf * FS + kx
                const float2* gr = gq + (r * L + n1) * RS;
                float2 t[RS];
#pragma unroll
                for (int k = 0; k < RS; ++k) t[k] = gr[k];
                Dft<RS>::run(t);
                float2* yr = yq + r * YB;   // conjugated (stage X reads it so)
                int py = (RS * n1) % FS;   // n_of(n1, n2), stepping n2 by L (mod FS)
#pragma unroll
                for (int n2 = 0; n2 < RS; ++n2) {
                    if (py < By) yr[py] = t[n2];
                    py += L;
                    py = py >= FS ? py - FS : py;
                }
            }
        };
        auto stage_x = [&]() {
#pragma unroll
            for (int it = 0; it < (NB * NF * NIN * RS + NT - 1) / NT; ++it) {
                const int i = tid + it * NT;
                const int kk = i % RS;
                const int r = i / RS;     // bf * NIN + py
                const int py = r % NIN, bf = r / NIN;
                if (i >= NB * NF * NIN * RS || py >= By) continue;
                const float2* yr = yq + bf * FS * YB + py;
                float2 t[L];
                const int kb = (Pfa<L, RS>::k_of(0, 1) * kk) % FS;   // k_of(0, kk)
#pragma unroll
                for (int m = 0; m < L; ++m) {
                    int kxm = kb + P::k_of(m, 0);
                    kxm = kxm >= FS ? kxm - FS : kxm;
                    t[m] = yr[kxm * YB];
                }
                Dft<L>::run(t);
                float2* gr = g2q + ((bf * NIN + py) * L) * RS + kk;
#pragma unroll
                for (int n = 0; n < L; ++n) gr[n * RS] = t[n];
            }
        };
        // stage R runs in the interval of stage Y, whose items past the first NT fall
        // to the first threads: R's items start after those threads
        constexpr int YX = (NB * NF * FS * L) % NT;
        const int rrot = tid >= YX ? tid - YX : tid + NT - YX;
        auto stage_r = [&]() {
#pragma unroll
            for (int it = 0; it < (NB * NF * NIN * L + NT - 1) / NT; ++it) {
                const int i = rrot + it * NT;
                const int n1 = i % L;
                const int r = i / L;  // bf * NIN + py
                const int py = r % NIN, bf = r / NIN;
                if (i >= NB * NF * NIN * L || py >= By) continue;
                const float2* gr = g2q + (r * L + n1) * RS;
                float2 t[RS];
#pragma unroll
                for (int k = 0; k < RS; ++k) t[k] = gr[k];
                Dft<RS>::run(t);
                int px = (RS * n1) % FS;   // n_of(n1, n2)
#pragma unroll
                for (int n2 = 0; n2 < RS; ++n2) {
                    if (px < Bx) obq[(bf * Bx + px) * By + py] = cconj(t[n2]);
                    px += L;
                    px = px >= FS ? px - FS : px;
                }
            }
        };
        auto stage_s = [&](int ch) {
            const auto tr = buf_rsrc(dT + ((int64_t)bl0 * A.nch + ch) * tstride,
                                     (uint32_t)(((int64_t)nbv * A.nch - ch) * tstride * 8));
#pragma unroll
            for (int k = 0; k < IT5; ++k) {
                const bool need = !A.rows || gflag[o_fo[k] + ch * ng] != 0;
                if (o_ok[k]) buf_st_f2(obq[o_src[k]], tr, need ? o_off[k] : 0xfffffff0u, 0u);
            }
        };
        for (int k = 0; k < A.nch + 2; ++k) {
            const bool doM = k < A.nch;
            const auto rr = buf_rsrc(rhat + ((int64_t)min(k, A.nch - 1) * A.ft + f0) * rstride, rbytes);
            auto load_w = [&](float2* wv, int c) {
#pragma unroll
                for (int mp = 0; mp < L / 2; ++mp) {
                    const float4 v = buf_f4(rr, rvoff, (uint32_t)((c * L + 2 * mp) * TPF * 8));
                    wv[2 * mp] = make_float2(v.x, v.y);
                    wv[2 * mp + 1] = make_float2(v.z, v.w);
                }
            };
            float2 w[PRE][L];
            if (doM) {
#pragma unroll
                for (int c = 0; c < PRE; ++c) load_w(w[c], min(c, clast));
            }
            __builtin_amdgcn_sched_barrier(0);
            if (k >= 2) stage_s(k - 2);
            if (k >= 1 && k <= A.nch) stage_x();
            __builtin_amdgcn_sched_barrier(0);
            if (doM) {
                float2 t[NB][L];   // set by piece 0 (nc >= 1); read by active threads only
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c < A.nc && active) {
#pragma unroll
                        for (int b = 0; b < NB; ++b)
#pragma unroll
                            for (int m = 0; m < L; ++m) {
                                const float2 d = dacc[b][c][m], r = w[c % PRE][m];
                                if (c == 0) {   // the sum from zero, as cfma's steps
                                    t[b][m].x = fmaf(-d.y, r.y, d.x * r.x);
                                    t[b][m].y = fmaf(d.y, r.x, d.x * r.y);
                                } else {
                                    t[b][m] = cfma(d, r, t[b][m]);
                                }
                            }
                    }
                    if (c + PRE < 4) load_w(w[c % PRE], min(c + PRE, clast));
                }
                if (active) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        Dft<L>::run(t[b]);
                        float2* gr = gq + (((b * NF + fl) * FS + kx) * L) * RS + k2;
#pragma unroll
                        for (int n = 0; n < L; ++n) gr[n * RS] = t[b][n];
                    }
                }
            }
            __syncthreads();
            if (k < A.nch) stage_y();
            if (k >= 1 && k <= A.nch) stage_r();
            __syncthreads();
        }
    } else {
        for (int ch = 0; ch < A.nch; ++ch) {
            const auto rr = buf_rsrc(rhat + ((int64_t)ch * A.ft + f0) * rstride, rbytes);
            // conjugate multiply-accumulate over the pieces and the L-point inverse over k1
            if (active) {
    #pragma unroll
                for (int b = 0; b < NB; ++b) {
                    float2 t[L];
    #pragma unroll
                    for (int m = 0; m < L; ++m) t[m] = make_float2(0.f, 0.f);
    #pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (c < A.nc) {
    #pragma unroll
                            for (int mp = 0; mp < L / 2; ++mp) {
                                const float4 v = buf_f4(rr, rvoff, (uint32_t)((c * L + 2 * mp) * TPF * 8));
                                t[2 * mp] = cfma(dacc[b][c][2 * mp], make_float2(v.x, -v.y), t[2 * mp]);
                                t[2 * mp + 1] = cfma(dacc[b][c][2 * mp + 1], make_float2(v.z, -v.w), t[2 * mp + 1]);
                            }
                        }
                    }
    #pragma unroll
                    for (int m = 0; m < L; ++m) t[m] = cconj(t[m]);
                    Dft<L>::run(t);
                    const int bf = b * NF + fl;
                    if constexpr (RS == 1) {
                        float2* yr = yb + (bf * FS + kx) * YB;
    #pragma unroll
                        for (int n = 0; n < L; ++n)
                            if (n < By) yr[n] = cconj(t[n]);
                    } else {
                        float2* gr = gbuf + ((bf * FS + kx) * L) * RS + k2;
    #pragma unroll
                        for (int n = 0; n < L; ++n) gr[n * RS] = t[n];
                    }
                }
            }
            __syncthreads();
            if constexpr (RS > 1) {
                for (int i = tid; i < NB * NF * FS * L; i += NT) {
                    const int n1 = i % L;
                    const int r = i / L;   // bf * FS + kx
                    const float2* gr = gbuf + (r * L + n1) * RS;
                    float2 t[RS];
    #pragma unroll
                    for (int k = 0; k < RS; ++k) t[k] = gr[k];
                    Dft<RS>::run(t);
                    float2* yr = yb + r * YB;
                    int py = (RS * n1) % FS;   // n_of(n1, n2), stepping n2 by L (mod FS)
    #pragma unroll
                    for (int n2 = 0; n2 < RS; ++n2) {
                        if (py < By) yr[py] = cconj(t[n2]);
                        py += L;
                        py = py >= FS ? py - FS : py;
                    }
                }
                __syncthreads();
            }
            // x inverse: L-point stage over kx = k_of(k1, kk) for every py. Items run over
            // py < NIN (a compile-time bound) so that their decomposition is shifts and
            // multiplies by constants; rows py >= By are skipped.
    #pragma unroll
            for (int it = 0; it < (NB * NF * NIN * RS + NT - 1) / NT; ++it) {
                const int i = tid + it * NT;
                const int kk = i % RS;
                const int r = i / RS;     // bf * NIN + py
                const int py = r % NIN, bf = r / NIN;
                if (i >= NB * NF * NIN * RS || py >= By) continue;
                const float2* yr = yb + bf * FS * YB + py;
                float2 t[L];
                const int kb = (Pfa<L, RS>::k_of(0, 1) * kk) % FS;   // k_of(0, kk)
    #pragma unroll
                for (int m = 0; m < L; ++m) {
                    int kxm = kb + P::k_of(m, 0);
                    kxm = kxm >= FS ? kxm - FS : kxm;
                    t[m] = cconj(yr[kxm * YB]);
                }
                Dft<L>::run(t);
                if constexpr (RS == 1) {
    #pragma unroll
                    for (int n = 0; n < L; ++n)
                        if (n < Bx) ob[(bf * Bx + n) * By + py] = cconj(t[n]);
                } else {
                    float2* gr = g2 + ((bf * NIN + py) * L) * RS + kk;   // [bf][py][n1][kk]
    #pragma unroll
                    for (int n = 0; n < L; ++n) gr[n * RS] = t[n];
                }
            }
            __syncthreads();
            if constexpr (RS > 1) {
    #pragma unroll
                for (int it = 0; it < (NB * NF * NIN * L + NT - 1) / NT; ++it) {
                    const int i = tid + it * NT;
                    const int n1 = i % L;
                    const int r = i / L;  // bf * NIN + py
                    const int py = r % NIN, bf = r / NIN;
                    if (i >= NB * NF * NIN * L || py >= By) continue;
                    const float2* gr = g2 + (r * L + n1) * RS;
                    float2 t[RS];
    #pragma unroll
                    for (int k = 0; k < RS; ++k) t[k] = gr[k];
                    Dft<RS>::run(t);
                    int px = (RS * n1) % FS;   // n_of(n1, n2)
    #pragma unroll
                    for (int n2 = 0; n2 < RS; ++n2) {
                        if (px < Bx) ob[(bf * Bx + px) * By + py] = cconj(t[n2]);
                        px += L;
                        px = px >= FS ? px - FS : px;
                    }
                }
                __syncthreads();
            }
            // dT[b][ch][p / kTileT][f][p % kTileT] for the bin's pixels p = px * By + py, with
            // the per-thread offsets computed before the channel loop
            {
                const auto tr = buf_rsrc(dT + ((int64_t)bl0 * A.nch + ch) * tstride,
                                         (uint32_t)(((int64_t)nbv * A.nch - ch) * tstride * 8));
    #pragma unroll
                for (int k = 0; k < IT5; ++k) {
                    const bool need = !A.rows || gflag[o_fo[k] + ch * ng] != 0;
                    if (o_ok[k]) buf_st_f2(ob[o_src[k]], tr, need ? o_off[k] : 0xfffffff0u, 0u);
                }
            }
            __syncthreads();
        }
    }
}

int pow2_at_least(int v, int lo) {
    int p = lo;
    while (p < v) p <<= 1;
    return p;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// supported spatial transform sizes and the length of their register sub-DFTs
int spatial_sub_length(int fs) {
    switch (fs) {
        case 8: case 24: case 40: return 8;
        case 16: case 32: case 48: case 64: return 16;
        case 36: return 9;
        default: return 0;
    }
}

int spatial_size_at_least(int n) {
    const int sizes[] = {8, 16, 24, 32, 40, 48, 64};
    for (int s : sizes)
        if (s >= n) return s;
    return 128;  // rejected by the caller
}

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

ConvArgs make_args(const tred_conv_plan* P) {
    ConvArgs A;
    const tred_grid& g = P->grid;
    A.Bx = P->blk.blk_pix[0];
    A.By = P->blk.blk_pix[1];
    A.Bt = P->blk.blk_ticks;
    A.sx = g.sub[0];
    A.sy = g.sub[1];
    A.NYf = A.By * A.sy;
    A.S = A.sx * A.sy;
    A.nch = P->nch;
    A.nc = P->nc;
    A.ct = P->ct;
    A.ft = P->ft;
    A.fs = P->fs;
    A.ppad = (A.Bx * A.By + kTileT - 1) / kTileT * kTileT;
    A.qpad = P->qpad;
    A.box = P->bo[0];
    A.boy = P->bo[1];
    A.bot = P->bo[2];
    A.mpcp = P->mpcp;
    A.chx = std::max(1, A.fs / A.By);
    A.cap = 0;
    const int L = P->ls, RS = P->fs / P->ls;
    if (P->pfa) {
        // prime-factor output map k = (RS (RS^-1 mod L) k1 + L (L^-1 mod RS) k2) mod fs
        int rsi = 0, li = 0;
        for (int x = 0; x < L; ++x)
            if ((RS * x) % L == 1 % L) { rsi = x; break; }
        for (int x = 0; x < RS; ++x)
            if ((L * x) % RS == 1 % RS) { li = x; break; }
        A.e1 = (RS * rsi) % P->fs;
        A.e2 = RS > 1 ? (L * li) % P->fs : 0;
        A.rpair = 1;   // k_spp reads rows in pairs (an odd L is padded with one row)
    } else {
        A.e1 = RS;
        A.e2 = 1;
        A.rpair = 0;
    }
    A.vblk = (int64_t)A.Bx * A.sx * A.NYf * A.Bt;
    A.vout = (int64_t)A.box * A.boy * A.bot;
    A.tskip = 0;
    A.tflag = nullptr;
    A.rows = nullptr;
    A.nrw = (int32_t)(((int64_t)A.Bx * A.sx * A.NYf + 31) / 32);
    return A;
}

// Permit dynamic LDS above the 64 KiB default (gfx950 has 160 KiB per CU). The
// attribute is set once per kernel and size, so that launches recorded into a graph
// are not interleaved with attribute calls.
template <typename K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return;
    static std::mutex mu;
    static std::unordered_map<const void*, size_t> done;
    std::lock_guard<std::mutex> lock(mu);
    size_t& have = done[(const void*)kernel];
    if (bytes <= have) return;
    if (hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes) == hipSuccess)
        have = bytes;
}

// list: workspace for the live-tile list (row masks with skipped groups) or NULL
template <int FT>
tred_status launch_time_fwd(const ConvArgs& A, int b0, int nb, const int32_t* na, const float* blocks,
                            const float2* tw, float2* T, int2* list, int32_t* count, hipStream_t st) {
    const size_t lds = (size_t)tf_lds_floats<FT>() * sizeof(float) + (size_t)FT * sizeof(float2);
    if (A.vblk * 4 > INT32_MAX)
        return tred_fail(TRED_EUNSUPPORTED, "time forward: %lld B per bin", (long long)(A.vblk * 4));
    if (list && A.rows && A.tskip) {
        // live tiles listed first; the transforms run over the list
        const int64_t tiles = (int64_t)(A.ppad / kTileT) * A.nch * nb;
        if (tiles <= 0) return TRED_OK;
        if (tiles > INT32_MAX / 2)
            return tred_fail(TRED_EUNSUPPORTED, "time forward: %lld tiles per pass", (long long)tiles);
        hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, st, count);
        hipLaunchKernelGGL(k_tf_tiles, dim3((unsigned)std::min<int64_t>((tiles + 255) / 256, 8192)), dim3(256),
                           0, st, A, b0, nb, na, list, count);
        const int64_t qs = 2 * tiles;
        const int64_t G = std::min<int64_t>(TRED_TF_GRID, (qs + 2 * kXcd - 1) / (2 * kXcd) * (2 * kXcd));
        if (2 * A.Bt <= FT) {
            allow_lds(k_tf_list<FT, true>, lds);
            hipLaunchKernelGGL((k_tf_list<FT, true>), dim3((unsigned)G), dim3(512), lds, st, A, b0, list, count,
                               (int32_t)tiles, blocks, tw, T);
        } else {
            allow_lds(k_tf_list<FT, false>, lds);
            hipLaunchKernelGGL((k_tf_list<FT, false>), dim3((unsigned)G), dim3(512), lds, st, A, b0, list, count,
                               (int32_t)tiles, blocks, tw, T);
        }
        return tred_check_launch("tred_block_conv time forward (listed tiles)");
    }
    // persistent workgroups: a multiple of 2 kXcd (tile halves on one XCD), a few per CU
    const int64_t groups = (int64_t)(A.ppad / kTile) * A.nch * nb;
    const int64_t cap = TRED_TF_GRID;
    const int64_t G = std::min(cap, (groups + 2 * kXcd - 1) / (2 * kXcd) * (2 * kXcd));
    if (G <= 0) return TRED_OK;
    if (2 * A.Bt <= FT) {
        allow_lds(k_tf<FT, true>, lds);
        hipLaunchKernelGGL((k_tf<FT, true>), dim3((unsigned)G), dim3(512), lds, st, A, b0, nb, na,
                           blocks, tw, T);
    } else {
        allow_lds(k_tf<FT, false>, lds);
        hipLaunchKernelGGL((k_tf<FT, false>), dim3((unsigned)G), dim3(512), lds, st, A, b0, nb, na,
                           blocks, tw, T);
    }
    return tred_check_launch("tred_block_conv time forward");
}

template <int FT>
tred_status launch_time_inv(const ConvArgs& A, int b0, int nb, const int32_t* na, const float2* U,
                            const float2* tw, float* out, hipStream_t st) {
    const size_t lds = (size_t)tf_lds_floats<FT>() * sizeof(float) + (size_t)FT * sizeof(float2);
    if (A.ct == A.Bt && 2 * A.ct == FT) {
        allow_lds(k_ti<FT, true>, lds);
        hipLaunchKernelGGL((k_ti<FT, true>), dim3(A.qpad / kTile, nb), dim3(512), lds, st, A, b0, na,
                           U, tw, out);
    } else {
        allow_lds(k_ti<FT, false>, lds);
        hipLaunchKernelGGL((k_ti<FT, false>), dim3(A.qpad / kTile, nb), dim3(512), lds, st, A, b0, na,
                           U, tw, out);
    }
    return tred_check_launch("tred_block_conv time inverse");
}

template <int FS, int L>
tred_status launch_space(const ConvArgs& A0, int b0, int nb, const int32_t* na, const float2* T,
                         const float2* rhat, const float2* tws, float2* U, hipStream_t st) {
    using S = SpShape<FS, L>;
    constexpr int MAXIT = 2;   // per-thread staging / x-pass items the kernel unrolls
    ConvArgs A = A0;
    const int per_ch_ld = A.ppad * S::NF;
    const int per_ch_x = S::NF * A.By * S::RS;
    A.chx = std::min(std::max(1, FS / A.By),
                     std::min(MAXIT * S::NT / per_ch_ld, MAXIT * S::NT / per_ch_x));
    if (A.chx < 1) return tred_fail(TRED_EUNSUPPORTED, "bin too large for the spatial stage");
    const SpLds Ls = sp_lds(FS, L, S::NF, A.chx, A.By, A.ppad, A.box, A.boy);
    const size_t lds = (size_t)Ls.total * sizeof(float2);
    if (lds > 160 * 1024) return tred_fail(TRED_EUNSUPPORTED, "spatial stage needs %zu B of LDS", lds);
    allow_lds(k_sp<FS, L>, lds);
    hipLaunchKernelGGL((k_sp<FS, L>), dim3(nb, A.ft / S::NF), dim3(S::NT), lds, st, A, b0, nb, na, T,
                       rhat, tws, U);
    return tred_check_launch("tred_block_conv space");
}

template <int FS, int L, int NIN, int NB, int NC>
tred_status launch_spp_nc(const ConvArgs& A, int b0, int nb, const int32_t* na, const float2* T,
                          const float2* rhat, const float2* tws, float2* U, hipStream_t st) {
    using S = SppShape<FS, L, NIN, NB>;
    const SppLds Ls = spp_lds<FS, L, NIN, NB, S::NF>(A.box, A.boy);
    // + the row-group flags of NB bins
    const size_t lds = (size_t)Ls.total * sizeof(float2) + ((size_t)NB * A.nch * (A.ppad / kTile) + 15) / 16 * 16;
    if (lds > 160 * 1024) return tred_fail(TRED_EUNSUPPORTED, "spatial stage needs %zu B of LDS", lds);
    const int64_t tbytes = (int64_t)NB * A.nch * (A.ppad / kTileT) * A.ft * kTileT * 8;
    if (tbytes > INT32_MAX)
        return tred_fail(TRED_EUNSUPPORTED, "spatial stage: %lld B of time spectra per workgroup",
                         (long long)tbytes);
    // the stores of U address NB bins' pieces with 32-bit offsets
    const int64_t ubytes = (int64_t)NB * A.nc * (A.qpad / kTile) * A.ft * kTile * 8;
    if (ubytes > INT32_MAX)
        return tred_fail(TRED_EUNSUPPORTED, "spatial stage: %lld B of output spectra per workgroup",
                         (long long)ubytes);
    allow_lds(k_spp<FS, L, NIN, NB, NC>, lds);
    hipLaunchKernelGGL((k_spp<FS, L, NIN, NB, NC>), dim3((nb + NB - 1) / NB, A.ft / S::NF), dim3(S::NT),
                       lds, st, A, b0, nb, na, T, rhat, tws, U);
    return tred_check_launch("tred_block_conv space");
}

template <int FS, int L, int NIN, int NB>
tred_status launch_spp(const ConvArgs& A, int b0, int nb, const int32_t* na, const float2* T,
                       const float2* rhat, const float2* tws, float2* U, hipStream_t st) {
    return A.nc <= 2 ? launch_spp_nc<FS, L, NIN, NB, 2>(A, b0, nb, na, T, rhat, tws, U, st)
                     : launch_spp_nc<FS, L, NIN, NB, 4>(A, b0, nb, na, T, rhat, tws, U, st);
}
template <int FS, int L, int NIN, int NB>
tred_status launch_spp_adj(const ConvArgs& A, int b0, int nb, const int32_t* na, const float2* dU,
                           const float2* rhat, const float2* tws, float2* dT, hipStream_t st) {
    using S = SppShape<FS, L, NIN, NB>;
    const auto Ls = spp_adj_lds<FS, L, NIN, NB, S::NF>(A.box, A.boy, A.Bx, A.By);
    // + the need flags of NB bins (row masks)
    const size_t lds = (size_t)Ls.total * sizeof(float2) +
                       (A.rows ? ((size_t)NB * A.nch * (A.ppad / kTile) + 15) / 16 * 16 : 0);
    if (lds > 160 * 1024)
        return tred_fail(TRED_EUNSUPPORTED, "adjoint spatial stage needs %zu B of LDS", lds);
    const int64_t tbytes = (int64_t)NB * A.nch * (A.ppad / kTileT) * A.ft * kTileT * 8;
    if (tbytes > INT32_MAX)
        return tred_fail(TRED_EUNSUPPORTED, "adjoint spatial stage: %lld B of spectra per workgroup",
                         (long long)tbytes);
    allow_lds(k_spp_adj<FS, L, NIN, NB>, lds);
    hipLaunchKernelGGL((k_spp_adj<FS, L, NIN, NB>), dim3((nb + NB - 1) / NB, A.ft / S::NF),
                       dim3(S::NT), lds, st, A, b0, nb, na, dU, rhat, tws, dT);
    return tred_check_launch("tred_block_conv_adjoint space");
}

tred_status launch_space_adj(const tred_conv_plan* P, const ConvArgs& A, int b0, int nb,
                             const int32_t* na, const float2* dU, const float2* rhat,
                             const float2* tws, float2* dT, hipStream_t st) {
    if (!P->pfa)
        return tred_fail(TRED_EUNSUPPORTED, "adjoint: spatial size %d (sizes 8, 16, 24, 40, 48 only)",
                         P->fs);
    const bool two = P->nin == 2 * P->ls;
    switch (P->fs) {
        case 8: return launch_spp_adj<8, 8, 8, 1>(A, b0, nb, na, dU, rhat, tws, dT, st);
        case 16: return launch_spp_adj<16, 16, 16, 1>(A, b0, nb, na, dU, rhat, tws, dT, st);
        case 24:
            return two ? launch_spp_adj<24, 8, 16, 1>(A, b0, nb, na, dU, rhat, tws, dT, st)
                       : launch_spp_adj<24, 8, 8, 1>(A, b0, nb, na, dU, rhat, tws, dT, st);
        case 40:
            return two ? launch_spp_adj<40, 8, 16, TRED_SPP_ADJ_NB>(A, b0, nb, na, dU, rhat, tws, dT, st)
                       : launch_spp_adj<40, 8, 8, TRED_SPP_ADJ_NB>(A, b0, nb, na, dU, rhat, tws, dT, st);
        case 48:
            return two ? launch_spp_adj<48, 16, 32, 1>(A, b0, nb, na, dU, rhat, tws, dT, st)
                       : launch_spp_adj<48, 16, 16, 1>(A, b0, nb, na, dU, rhat, tws, dT, st);
        default: return tred_fail(TRED_EUNSUPPORTED, "adjoint: spatial size %d", P->fs);
    }
}

template <int FT>
tred_status launch_time_adj(const ConvArgs& A, int b0, int nb, const int32_t* na, const float* dout,
                            const float2* tw, float2* dU, float2* dT, float* dblocks, int stage,
                            hipStream_t st) {
    const size_t lds = (size_t)tf_lds_floats<FT>() * sizeof(float) + (size_t)FT * sizeof(float2);
    if (stage == 0) {
        allow_lds(k_ti_adj<FT>, lds);
        hipLaunchKernelGGL((k_ti_adj<FT>), dim3(A.qpad / kTile, A.nc, nb), dim3(512), lds, st, A, b0,
                           na, dout, tw, dU);
    } else {
        // persistent workgroups: a multiple of 2 kXcd (tile halves on one XCD)
        const int64_t groups = (int64_t)(A.ppad / kTile) * A.nch * nb;
        if (groups > INT32_MAX / 4)
            return tred_fail(TRED_EUNSUPPORTED, "adjoint time stage: %lld row groups per pass",
                             (long long)groups);
        const int64_t G = std::min<int64_t>(TRED_TF_GRID, (groups + 2 * kXcd - 1) / (2 * kXcd) * (2 * kXcd));
        if (G <= 0) return TRED_OK;
        allow_lds(k_tf_adj<FT>, lds);
        hipLaunchKernelGGL((k_tf_adj<FT>), dim3((unsigned)G), dim3(512), lds, st, A, b0, nb, na, dT, tw,
                           dblocks);
    }
    return tred_check_launch("tred_block_conv_adjoint time");
}

tred_status launch_space_any(const tred_conv_plan* P, const ConvArgs& A, int b0, int nb,
                             const int32_t* na, const float2* T, const float2* rhat,
                             const float2* tws, float2* U, hipStream_t st) {
    constexpr int NB8 = TRED_SPP_NB8;
    if (P->pfa) {
        const bool two = P->nin == 2 * P->ls;
        const bool half = 2 * P->nin == P->ls;
        switch (P->fs) {
            case 8:
                return half ? launch_spp<8, 8, 4, 1>(A, b0, nb, na, T, rhat, tws, U, st)
                            : launch_spp<8, 8, 8, 1>(A, b0, nb, na, T, rhat, tws, U, st);
            case 16:
                return half ? launch_spp<16, 16, 8, 1>(A, b0, nb, na, T, rhat, tws, U, st)
                            : launch_spp<16, 16, 16, 1>(A, b0, nb, na, T, rhat, tws, U, st);
            case 24:
                return two ? launch_spp<24, 8, 16, NB8>(A, b0, nb, na, T, rhat, tws, U, st)
                           : launch_spp<24, 8, 8, NB8>(A, b0, nb, na, T, rhat, tws, U, st);
            case 36:
                return P->nin == 16 ? launch_spp<36, 9, 16, 1>(A, b0, nb, na, T, rhat, tws, U, st)
                                    : launch_spp<36, 9, 8, 1>(A, b0, nb, na, T, rhat, tws, U, st);
            case 40:
                return two ? launch_spp<40, 8, 16, NB8>(A, b0, nb, na, T, rhat, tws, U, st)
                           : launch_spp<40, 8, 8, NB8>(A, b0, nb, na, T, rhat, tws, U, st);
            case 48:
                return two ? launch_spp<48, 16, 32, 1>(A, b0, nb, na, T, rhat, tws, U, st)
                           : launch_spp<48, 16, 16, 1>(A, b0, nb, na, T, rhat, tws, U, st);
            default: return tred_fail(TRED_EUNSUPPORTED, "spatial size %d", P->fs);
        }
    }
    switch (P->fs) {
        case 32: return launch_space<32, 16>(A, b0, nb, na, T, rhat, tws, U, st);
        case 64: return launch_space<64, 16>(A, b0, nb, na, T, rhat, tws, U, st);
        default: return tred_fail(TRED_EUNSUPPORTED, "spatial size %d", P->fs);
    }
}

template <typename F>
tred_status dispatch_ft(int ft, F&& f) {
    switch (ft) {
        case 256: return f(std::integral_constant<int, 256>{});
        case 512: return f(std::integral_constant<int, 512>{});
        case 1024: return f(std::integral_constant<int, 1024>{});
        case 2048: return f(std::integral_constant<int, 2048>{});
        default: return tred_fail(TRED_EUNSUPPORTED, "time FFT size %d", ft);
    }
}

}  // namespace

extern "C" tred_status tred_conv_plan_create(const tred_grid* grid, const tred_blocking* blocking,
                                             const int32_t kpix[2], int32_t kticks,
                                             const int32_t fft[3], uint32_t flags, int32_t batch,
                                             tred_conv_plan** plan, int64_t* workspace_bytes) {
    TRED_TRY(validate_grid(grid));
    TRED_TRY(validate_blocking(blocking));
    TRED_REQUIRE(kpix && plan && workspace_bytes, "kpix/plan/workspace_bytes is NULL");
    TRED_REQUIRE(kpix[0] > 0 && kpix[1] > 0 && (kpix[0] & 1) && (kpix[1] & 1),
                 "kpix must be positive and odd");
    TRED_REQUIRE(kticks > 0, "kticks must be > 0");
    TRED_REQUIRE(batch > 0, "batch must be > 0");
    TRED_REQUIRE((flags & ~TRED_CONV_MPCP) == 0, "unknown flags");
    *plan = nullptr;
    tred_conv_plan* P = new tred_conv_plan();
    P->grid = *grid;
    P->blk = *blocking;
    P->kpix[0] = kpix[0];
    P->kpix[1] = kpix[1];
    P->kticks = kticks;
    P->mpcp = (flags & TRED_CONV_MPCP) ? 1 : 0;
    P->batch = batch;
    const int Bx = blocking->blk_pix[0], By = blocking->blk_pix[1], Bt = blocking->blk_ticks;
    P->bo[0] = Bx + kpix[0] - 1;
    P->bo[1] = By + kpix[1] - 1;
    P->bo[2] = Bt + kticks - 1;
    int fsx = fft && fft[0] ? fft[0] : spatial_size_at_least(P->bo[0]);
    int fsy = fft && fft[1] ? fft[1] : spatial_size_at_least(P->bo[1]);
    int ft = fft && fft[2] ? fft[2] : pow2_at_least(P->bo[2], 256);
    auto bad = [&](tred_status s, const char* msg) {
        delete P;
        return tred_fail(s, "%s", msg);
    };
    if (fsx < P->bo[0] || fsy < P->bo[1])
        return bad(TRED_EINVAL, "spatial FFT sizes must be >= blk_pix + kpix - 1");
    if (fsx != fsy || spatial_sub_length(fsx) == 0)
        return bad(TRED_EUNSUPPORTED,
                   "spatial FFT sizes must be equal and in {8,16,24,32,36,40,48,64}");
    const int L = spatial_sub_length(fsx);
    // inputs per axis of the prime-factor stage: L / 2 (sizes 8 and 16 only), L or 2 L;
    // size 36 (L = 9) takes 8 or 16 (an even count)
    const int nin = fsx == 36 ? (std::max(Bx, By) <= 8 ? 8 : 16)
                              : (fsx <= 16 && std::max(Bx, By) <= L / 2)
                                    ? L / 2
                                    : (std::max(Bx, By) <= L ? L : 2 * L);
    if (Bx > nin || By > nin || Bx > 2 * L || By > 2 * L)
        return bad(TRED_EUNSUPPORTED, "blk_pix too large for this FFT size");
    if (Bt % 64 != 0) return bad(TRED_EUNSUPPORTED, "blk_ticks must be a multiple of 64");
    if (!is_pow2(ft)) return bad(TRED_EINVAL, "time FFT size must be a power of two");
    if (ft < 256 || ft > 2048) return bad(TRED_EUNSUPPORTED, "time FFT size must be in [256, 2048]");
    if (ft < Bt + 64) return bad(TRED_EINVAL, "time FFT size must be >= blk_ticks + 64");
    P->fs = fsx;
    P->ls = L;
    P->pfa = (fsx % 32) != 0;   // 8, 16, 24, 36, 40, 48: L and fs / L coprime
    P->nin = nin;
    P->spp_nb = L == 8 ? TRED_SPP_NB8 : 1;
    P->ft = ft;
    P->ct = ft - Bt;
    P->nc = (kticks + P->ct - 1) / P->ct;
    if (P->nc > 4) return bad(TRED_EUNSUPPORTED, "more than 4 response pieces; raise fft[2]");
    const int S = grid->sub[0] * grid->sub[1];
    P->nch = P->mpcp ? (S + 1) / 2 : S;
    P->qpad = (P->bo[0] * P->bo[1] + kTile - 1) / kTile * kTile;
    const int64_t ppad = (Bx * By + kTileT - 1) / kTileT * kTileT;
    // workspace layout
    int64_t o = 0;
    P->off_tw_t = o;
    o = align256(o + (int64_t)ft * 8);
    P->off_tw_s = o;
    o = align256(o + (int64_t)P->fs * 8);
    P->off_chan = o;
    P->off_rhat = o;
    // response spectra: fs * fs values per (ch, c, f), or (L + 1) * fs * fs / L with the
    // pad row of an odd L
    const int64_t rsp = (int64_t)(L + (L & 1)) * (P->fs / L) * P->fs;
    o = align256(o + (int64_t)P->nch * P->nc * rsp * ft * 8);
    P->off_scratch_t = o;
    const int64_t tbytes = align256((int64_t)batch * P->nch * ppad * ft * 8);
    const int64_t ubytes = align256((int64_t)batch * P->nc * P->qpad * ft * 8);
    // set-up scratch (binary64): PA, PB and two twiddle tables
    const int64_t pa = (int64_t)P->nch * P->nc * kpix[0] * kpix[1] * ft * 16;
    const int64_t pb = (int64_t)P->nch * P->nc * P->fs * kpix[1] * ft * 16;
    const int64_t setup = align256(pa) + align256(pb) + align256((int64_t)(ft + P->fs) * 16) + 256;
    const int64_t scr = std::max(tbytes + ubytes, setup);
    P->off_scratch_u = o + tbytes;
    o += scr;
    P->off_tflag = o;
    o = align256(o + (int64_t)batch * P->nch * (ppad / kTile));
    P->off_tlist = o;   // live T tiles of a pass (row masks)
    o = align256(o + (int64_t)batch * P->nch * (ppad / kTileT) * 8);
    P->off_tcount = o;
    o = align256(o + 4);
    P->ws_bytes = o;
    P->ws = nullptr;
    P->ready = 0;
    *plan = P;
    *workspace_bytes = o;
    return TRED_OK;
}

extern "C" tred_status tred_conv_plan_info(const tred_conv_plan* P, int32_t fft[3], int32_t* pieces,
                                           int32_t* channels, int32_t out[3]) {
    TRED_REQUIRE(P != nullptr, "plan is NULL");
    if (fft) {
        fft[0] = P->fs;
        fft[1] = P->fs;
        fft[2] = P->ft;
    }
    if (pieces) *pieces = P->nc;
    if (channels) *channels = P->nch;
    if (out)
        for (int a = 0; a < 3; ++a) out[a] = P->bo[a];
    return TRED_OK;
}

extern "C" tred_status tred_conv_plan_set_response(tred_conv_plan* P, const float* resp,
                                                   void* workspace, void* stream) {
    TRED_REQUIRE(P && resp && workspace, "plan/resp/workspace is NULL");
    TRED_REQUIRE(((uintptr_t)workspace & 255) == 0, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    const int Kx = P->kpix[0], Ky = P->kpix[1], kt = P->kticks;
    const int sx = P->grid.sub[0], sy = P->grid.sub[1];
    char* scr = ws + P->off_scratch_t;
    int64_t o = 0;
    double2* PA = (double2*)(scr + o);
    o += align256((int64_t)P->nch * P->nc * Kx * Ky * P->ft * 16);
    double2* PB = (double2*)(scr + o);
    o += align256((int64_t)P->nch * P->nc * P->fs * Ky * P->ft * 16);
    double2* twdt = (double2*)(scr + o);
    double2* twds = twdt + P->ft;
    o += align256((int64_t)(P->ft + P->fs) * 16);
    int* bad = (int*)(scr + o);
    if (P->mpcp) {
        if (hipMemsetAsync(bad, 0, sizeof(int), st) != hipSuccess)
            return tred_fail(TRED_EDEVICE, "memset failed");
        hipLaunchKernelGGL(k_symcheck, dim3(1024), dim3(256), 0, st, resp, Kx, Ky, sx, sy, kt, bad);
        TRED_TRY(tred_check_launch("symmetry check"));
        int hbad = 0;
        if (hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return tred_fail(TRED_EDEVICE, "symmetry check readback failed");
        if (hbad != 0)
            return tred_fail(TRED_EINVAL,
                             "mirror-pair packing needs R[K-1-k][sub-1-j][t] == R[k][j][t] "
                             "(%d entries differ)", hbad);
    }
    ConvArgs A = make_args(P);
    const int mx = std::max(P->ft, P->fs);
    hipLaunchKernelGGL(k_twiddles, dim3((mx + 255) / 256), dim3(256), 0, st,
                       (float2*)(ws + P->off_tw_t), P->ft, (float2*)(ws + P->off_tw_s), P->fs, twdt,
                       twds);
    hipLaunchKernelGGL(k_rhat_time, dim3(8192), dim3(256), 0, st, resp, A, Kx, Ky, kt, twdt, PA);
    hipLaunchKernelGGL(k_rhat_x, dim3(8192), dim3(256), 0, st, A, Kx, Ky, twds, PA, PB);
    const int L = P->ls;
    const double scale = 1.0 / ((double)P->fs * P->fs * P->ft);
    hipLaunchKernelGGL(k_rhat_y, dim3(8192), dim3(256), 0, st, A, Ky, L, scale, twds, PB,
                       (float2*)(ws + P->off_rhat));
    TRED_TRY(tred_check_launch("response spectra"));
    if (hipStreamSynchronize(st) != hipSuccess)
        return tred_fail(TRED_EDEVICE, "response spectra: %s", hipGetErrorString(hipGetLastError()));
    P->ws = workspace;
    P->ready = 1;
    return TRED_OK;
}

namespace {
tred_status block_conv(const tred_conv_plan* P, const int32_t* n_active, int32_t cap,
                       const float* blocks, const uint32_t* rows, float* out_blocks, void* stream) {
    TRED_REQUIRE(P && n_active, "plan/n_active is NULL");
    TRED_REQUIRE(P->ready, "plan has no response (call tred_conv_plan_set_response)");
    TRED_REQUIRE(cap >= 0, "cap must be >= 0");
    if (cap == 0) return TRED_OK;
    TRED_REQUIRE(blocks && out_blocks, "blocks/out_blocks is NULL");
    TRED_REQUIRE(((uintptr_t)blocks & 15) == 0 && ((uintptr_t)out_blocks & 3) == 0,
                 "blocks must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    ConvArgs A = make_args(P);
    A.cap = cap;
    char* ws = (char*)P->ws;
    const float2* twt = (const float2*)(ws + P->off_tw_t);
    const float2* tws = (const float2*)(ws + P->off_tw_s);
    const float2* rhat = (const float2*)(ws + P->off_rhat);
    float2* T = (float2*)(ws + P->off_scratch_t);
    float2* U = (float2*)(ws + P->off_scratch_u);
    // the prime-factor spatial stage reads the group flags: groups of all-zero rows
    // (most of a block-sparse event) skip their transform and spectra
    A.tskip = P->pfa;
    A.tflag = (uint8_t*)(ws + P->off_tflag);
    A.rows = rows;
    int2* tlist = (int2*)(ws + P->off_tlist);
    int32_t* tcount = (int32_t*)(ws + P->off_tcount);
    auto mark = [&](int b0, int k) {
        if (P->timing && b0 == 0) (void)hipEventRecord(P->ev[k], st);
    };
    const int pass = std::min(P->batch, 65535);   // bins per pass (a grid dimension)
    for (int b0 = 0; b0 < cap; b0 += pass) {
        const int nb = std::min(pass, cap - b0);
        mark(b0, 0);
        TRED_TRY(dispatch_ft(P->ft, [&](auto ftc) {
            return launch_time_fwd<decltype(ftc)::value>(A, b0, nb, n_active, blocks, twt, T, tlist, tcount, st);
        }));
        mark(b0, 1);
        mark(b0, 2);
        TRED_TRY(launch_space_any(P, A, b0, nb, n_active, T, rhat, tws, U, st));
        mark(b0, 3);
        mark(b0, 4);
        TRED_TRY(dispatch_ft(P->ft, [&](auto ftc) {
            return launch_time_inv<decltype(ftc)::value>(A, b0, nb, n_active, U, twt, out_blocks, st);
        }));
        mark(b0, 5);
    }
    return TRED_OK;
}
}  // namespace

extern "C" tred_status tred_block_conv(const tred_conv_plan* P, const int32_t* n_active,
                                       int32_t cap, const float* blocks, float* out_blocks,
                                       void* stream) {
    return block_conv(P, n_active, cap, blocks, nullptr, out_blocks, stream);
}

extern "C" tred_status tred_block_conv_rows(const tred_conv_plan* P, const int32_t* n_active,
                                            int32_t cap, const float* blocks, const uint32_t* rows,
                                            float* out_blocks, void* stream) {
    TRED_REQUIRE(cap == 0 || rows, "rows is NULL");
    TRED_REQUIRE(((uintptr_t)rows & 3) == 0, "rows must be 4-byte aligned");
    return block_conv(P, n_active, cap, blocks, rows, out_blocks, stream);
}

namespace {
tred_status block_conv_adjoint(const tred_conv_plan* P, const int32_t* n_active, int32_t cap,
                               const float* d_out_blocks, const uint32_t* rows, float* d_blocks,
                               void* stream) {
    TRED_REQUIRE(P && n_active, "plan/n_active is NULL");
    TRED_REQUIRE(P->ready, "plan has no response (call tred_conv_plan_set_response)");
    TRED_REQUIRE(cap >= 0, "cap must be >= 0");
    if (cap == 0) return TRED_OK;
    TRED_REQUIRE(d_out_blocks && d_blocks, "d_out_blocks/d_blocks is NULL");
    hipStream_t st = (hipStream_t)stream;
    ConvArgs A = make_args(P);
    A.cap = cap;
    char* ws = (char*)P->ws;
    const float2* twt = (const float2*)(ws + P->off_tw_t);
    const float2* tws = (const float2*)(ws + P->off_tw_s);
    const float2* rhat = (const float2*)(ws + P->off_rhat);
    float2* T = (float2*)(ws + P->off_scratch_t);
    float2* U = (float2*)(ws + P->off_scratch_u);
    A.rows = rows;
    A.tflag = (uint8_t*)(ws + P->off_tflag);
    const int pass = std::min(P->batch, 65535);   // bins per pass (a grid dimension)
    for (int b0 = 0; b0 < cap; b0 += pass) {
        const int nb = std::min(pass, cap - b0);
        if (rows) {
            const int64_t ngr = (int64_t)nb * A.nch * (A.ppad / kTile);
            hipLaunchKernelGGL(k_group_need, dim3((unsigned)std::min<int64_t>((ngr + 255) / 256, 8192)),
                               dim3(256), 0, st, A, b0, nb, n_active);
        }
        TRED_TRY(dispatch_ft(P->ft, [&](auto ftc) {
            return launch_time_adj<decltype(ftc)::value>(A, b0, nb, n_active, d_out_blocks, twt, U,
                                                         T, d_blocks, 0, st);
        }));
        TRED_TRY(launch_space_adj(P, A, b0, nb, n_active, U, rhat, tws, T, st));
        TRED_TRY(dispatch_ft(P->ft, [&](auto ftc) {
            return launch_time_adj<decltype(ftc)::value>(A, b0, nb, n_active, d_out_blocks, twt, U,
                                                         T, d_blocks, 1, st);
        }));
    }
    return TRED_OK;
}
}  // namespace

extern "C" tred_status tred_block_conv_adjoint(const tred_conv_plan* P, const int32_t* n_active,
                                               int32_t cap, const float* d_out_blocks,
                                               float* d_blocks, void* stream) {
    return block_conv_adjoint(P, n_active, cap, d_out_blocks, nullptr, d_blocks, stream);
}

extern "C" tred_status tred_block_conv_adjoint_rows(const tred_conv_plan* P,
                                                    const int32_t* n_active, int32_t cap,
                                                    const float* d_out_blocks, const uint32_t* rows,
                                                    float* d_blocks, void* stream) {
    TRED_REQUIRE(cap == 0 || rows, "rows is NULL");
    TRED_REQUIRE(((uintptr_t)rows & 3) == 0, "rows must be 4-byte aligned");
    return block_conv_adjoint(P, n_active, cap, d_out_blocks, rows, d_blocks, stream);
}

extern "C" tred_status tred_conv_plan_set_timing(tred_conv_plan* P, void* const* events) {
    TRED_REQUIRE(P != nullptr, "plan is NULL");
    if (!events) {
        P->timing = 0;
        return TRED_OK;
    }
    for (int k = 0; k < 6; ++k) {
        TRED_REQUIRE(events[k] != nullptr, "events[%d] is NULL", k);
        P->ev[k] = (hipEvent_t)events[k];
    }
    P->timing = 1;
    return TRED_OK;
}

extern "C" void tred_conv_plan_destroy(tred_conv_plan* P) { delete P; }

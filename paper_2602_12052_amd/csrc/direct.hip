// Block-direct interlaced convolution on the matrix cores (Sec. II-D eq. interlaced,
// evaluated without transforms): for every active bin
//   out[p + k][t'] = sum_{j, tau} Q_j[p][t' - tau] R_j[k][tau]
// with p the bin's pixels, k the response's pixel offsets (kx, ky), j the impact
// positions and tau the response ticks. Per bin this is one dense contraction
//   C[(p, t')][k] = sum_{(tau, j)} A[(p, t')][(tau, j)] B[(tau, j)][k],
//   A[(p, t')][(tau, j)] = Q_j[p][t' - tau],   B[(tau, j)][k] = R_j[k][tau],
// run on BF16 MFMA (v_mfma_f32_32x32x16_bf16) with FP32 accumulation, either plain
// (operands rounded to BF16) or with the hi/lo split x = hi + lo (hi = bf16(x),
// lo = bf16(x - hi)) and the three products hi*hi + hi*lo + lo*hi.
// Operands are laid out with the impact position fastest in groups of 8, so each
// lane's 8-element MFMA operand is one 16-byte load:
//   Rt[tau][k][j]   (k padded to tiles of 32, j padded to jpad = 16 * ceil(S / 16))
//   Qt[bin][p][t][j] with a zero margin of PAD ticks on both sides of the bin.
#include <algorithm>
#include <cstdint>

#include "tred_internal.hpp"
#include "validate.hpp"

struct tred_direct_plan {
    tred_grid grid;
    tred_blocking blk;
    int32_t kpix[2], kticks;
    int32_t split;          // hi/lo split products
    int32_t batch;          // bins per pass (bounds the operand scratch)
    int32_t S, jpad, nk, kpad, npix, tq;
    int32_t bo[3];
    int64_t off_rhi, off_rlo, off_qhi, off_qlo, ws_bytes;
    void* ws;
    int ready;
};

namespace {

constexpr int kPad = 32;    // zero ticks on each side of a bin in Qt (>= 2 TT - 2)
#ifndef TRED_DIRECT_TT
#define TRED_DIRECT_TT 16
#endif
constexpr int kDirTT = TRED_DIRECT_TT;   // output ticks per wave of the matrix-core kernel
static_assert(2 * kDirTT - 2 <= kPad, "charge margin");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// binary32 -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct DirArgs {
    int32_t Bx, By, Bt, sx, sy, NYf, S, jpad;
    int32_t Kx, Ky, kt, nk, kpad;
    int32_t npix, tq, box, boy, bot;
    int32_t cap;
    int64_t vblk, vout;
};

// Rt hi/lo from resp[kx][ky][jx][jy][tau]
__global__ void k_direct_resp(DirArgs A, const float* __restrict__ R, uint16_t* __restrict__ rhi,
                              uint16_t* __restrict__ rlo) {
    const int64_t n = (int64_t)A.kt * A.kpad * A.jpad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % A.jpad);
        const int64_t r = i / A.jpad;
        const int k = (int)(r % A.kpad);
        const int tau = (int)(r / A.kpad);
        float x = 0.0f;
        if (k < A.nk && j < A.S) {
            const int kx = k / A.Ky, ky = k % A.Ky, jx = j / A.sy, jy = j % A.sy;
            x = R[((((int64_t)kx * A.Ky + ky) * A.sx + jx) * A.sy + jy) * A.kt + tau];
        }
        const uint16_t h = bf16_rne(x);
        rhi[i] = h;
        rlo[i] = bf16_rne(x - bf16_to_f32(h));
    }
}

// Qt hi/lo of the bins of one pass from blocks[bin][x fine][y fine][t]
__global__ void k_direct_charge(DirArgs A, int b0, int nb, const int32_t* __restrict__ n_active,
                                const float* __restrict__ blocks, uint16_t* __restrict__ qhi,
                                uint16_t* __restrict__ qlo) {
    const int na = min(*n_active, A.cap);
    const int64_t n = (int64_t)nb * A.npix * A.tq * A.jpad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % A.jpad);
        int64_t r = i / A.jpad;
        const int t = (int)(r % A.tq) - kPad;
        r /= A.tq;
        const int p = (int)(r % A.npix);
        const int bl = (int)(r / A.npix);
        float x = 0.0f;
        if (b0 + bl < na && j < A.S && t >= 0 && t < A.Bt) {
            const int px = p / A.By, py = p % A.By, jx = j / A.sy, jy = j % A.sy;
            x = blocks[(int64_t)(b0 + bl) * A.vblk +
                       ((int64_t)(px * A.sx + jx) * A.NYf + (py * A.sy + jy)) * A.Bt + t];
        }
        const uint16_t h = bf16_rne(x);
        qhi[i] = h;
        qlo[i] = bf16_rne(x - bf16_to_f32(h));
    }
}

__global__ void k_direct_zero(DirArgs A, int b0, int nb, const int32_t* __restrict__ n_active,
                              float* __restrict__ out) {
    const int na = min(*n_active, A.cap);
    const int nbv = min(nb, na - b0);
    if (nbv <= 0) return;
    const int64_t n = (int64_t)nbv * A.vout;
    float* o = out + (int64_t)b0 * A.vout;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        o[i] = 0.0f;
}

__device__ __forceinline__ bf16x8 ld8(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0u, 0));
}

// One wave per tile of 32 pixels p (rows) x 32 response offsets k (columns) x TT output
// ticks t' (one accumulator tile per tick); a workgroup holds 2 x 2 such tiles (two
// pixel tiles, two offset tiles) at the same ticks. For response tick tau and impact
// positions j = 16 s .. 16 s + 15 the product is A[p][j] = Q_j[p][t' - tau] times
// B[j][k] = R_j[k][tau]: a charge fragment (tick u = t' - tau) serves the TT output
// ticks at TT consecutive tau, so the tau loop is unrolled by TT and the fragments sit in
// a ring of TT registers (slot u mod TT, with tau walked in groups aligned to t0), one new
// fragment and one response fragment per tau (one wave per SIMD, the accumulators in
// the AGPRs). Loads go through buffer resources: ticks
// before 0 or past the response, and pixels past the bin, read zero. Lane l holds
// A[row l % 32][8 (l / 32) .. + 7] and B[8 (l / 32) .. + 7][col l % 32] of each
// 32 x 16 x 32 step, and accumulator element i of C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
template <bool SPLIT, int TT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1))) void k_direct_mma(
    DirArgs A, int b0, int nb, const int32_t* __restrict__ n_active,
    const uint16_t* __restrict__ qhi, const uint16_t* __restrict__ qlo,
    const uint16_t* __restrict__ rhi, const uint16_t* __restrict__ rlo, float* __restrict__ out) {
    const int na = min(*n_active, A.cap);
    const int npt = (A.npix + 31) / 32, nkt = A.kpad / 32;
    const int cpx = (npt + 1) / 2, ckx = (nkt + 1) / 2;
    static_assert((TT & (TT - 1)) == 0, "ticks per wave: a power of two");
    // bins vary fastest: workgroups running together share the response slab of their
    // ticks and offsets
    int64_t w = blockIdx.x;
    const int bl = (int)(w % nb);
    w /= nb;
    const int pc = (int)(w % cpx);
    w /= cpx;
    const int kc = (int)(w % ckx);
    const int tt = (int)(w / ckx);
    if (b0 + bl >= na) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int pt = 2 * pc + (wv & 1), kt = 2 * kc + (wv >> 1);
    if (pt >= npt || kt >= nkt) return;
    const int row = lane & 31, half = lane >> 5;
    const int p0 = pt * 32, k0 = kt * 32, t0 = tt * TT;
    // response ticks that reach some output tick of the tile from inside the bin
    const int tlo = max(0, t0 - (A.Bt - 1)), thi = min(A.kt - 1, t0 + TT - 1);
    if (tlo > thi) return;
    const int tb0 = t0 - TT * ((t0 - tlo + TT - 1) / TT);   // <= tlo, congruent to t0 mod TT
    const int jb = A.jpad * 2;                      // bytes per (pixel, tick) or (tau, k) row
    const uint32_t qbytes = (uint32_t)((int64_t)A.npix * A.tq * jb);
    const uint32_t rbytes = (uint32_t)((int64_t)A.kt * A.kpad * jb);
    const int64_t qbin = (int64_t)bl * A.npix * A.tq * A.jpad;
    const auto qh = buf_rsrc(qhi + qbin, qbytes), rh = buf_rsrc(rhi, rbytes);
    const auto ql = buf_rsrc(qlo + qbin, qbytes), rl = buf_rsrc(rlo, rbytes);
    // byte offsets: A(u) = Q[p0 + row][u] at qa + u * jb (margin kPad ticks before the bin);
    // B(tau) = R[tau][k0 + row] at ra + tau * kpad * jb (negative tau wraps past the range)
    const int qa = ((p0 + row) * A.tq + kPad) * jb + 16 * half;
    const int ra = (k0 + row) * jb + 16 * half;
    const int rstep = A.kpad * jb;
    const int jsteps = A.jpad / 16;
    constexpr int M = TT - 1;
    f32x16 acc[TT];
#pragma unroll
    for (int i = 0; i < TT; ++i) acc[i] = (f32x16){};
    for (int s = 0; s < jsteps; ++s) {
        // hi (and lo) fragments; each tau's charge and response fragments are requested
        // just before their multiplies, which the TT (x 3 with the split) products cover
        bf16x8 fh[TT], fl[SPLIT ? TT : 1];
#pragma unroll
        for (int i = 1; i < TT; ++i) {
            const uint32_t o = (uint32_t)(qa + (t0 - tb0 + i) * jb + 32 * s);
            fh[i] = ld8(qh, o);
            if constexpr (SPLIT) fl[i] = ld8(ql, o);
        }
        for (int tb = tb0; tb <= thi; tb += TT) {
#pragma unroll
            for (int d = 0; d < TT; ++d) {
                const int tau = tb + d;
                const int sl = (TT - d) & M;
                const uint32_t oq = (uint32_t)(qa + (t0 - tau) * jb + 32 * s);
                const uint32_t orr = (uint32_t)(ra + tau * rstep + 32 * s);
                fh[sl] = ld8(qh, oq);
                const bf16x8 bh = ld8(rh, orr);
                bf16x8 blo;
                if constexpr (SPLIT) {
                    fl[sl] = ld8(ql, oq);
                    blo = ld8(rl, orr);
                }
#pragma unroll
                for (int i = 0; i < TT; ++i) {
                    const int q = (i - d) & M;
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh[q], bh, acc[i], 0, 0, 0);
                    if constexpr (SPLIT) {
                        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fh[q], blo, acc[i], 0, 0, 0);
                        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fl[q], bh, acc[i], 0, 0, 0);
                    }
                }
            }
        }
    }
    // scatter-add C[p][k] of tick t' into out[p + k][t']
    const int k = k0 + row;
    if (k >= A.nk) return;
    const int kx = k / A.Ky, ky = k % A.Ky;
    float* ob = out + (int64_t)(b0 + bl) * A.vout;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int p = p0 + 8 * (e / 4) + 4 * half + (e % 4);
        if (p >= A.npix) continue;
        const int px = p / A.By, py = p % A.By;
        float* o = ob + ((int64_t)(px + kx) * A.boy + (py + ky)) * A.bot + t0;
#pragma unroll
        for (int i = 0; i < TT; ++i)
            if (t0 + i < A.bot) atomicAdd(o + i, acc[i][e]);
    }
}

DirArgs make_dargs(const tred_direct_plan* P) {
    DirArgs A;
    A.Bx = P->blk.blk_pix[0];
    A.By = P->blk.blk_pix[1];
    A.Bt = P->blk.blk_ticks;
    A.sx = P->grid.sub[0];
    A.sy = P->grid.sub[1];
    A.NYf = A.By * A.sy;
    A.S = P->S;
    A.jpad = P->jpad;
    A.Kx = P->kpix[0];
    A.Ky = P->kpix[1];
    A.kt = P->kticks;
    A.nk = P->nk;
    A.kpad = P->kpad;
    A.npix = P->npix;
    A.tq = P->tq;
    A.box = P->bo[0];
    A.boy = P->bo[1];
    A.bot = P->bo[2];
    A.cap = 0;
    A.vblk = (int64_t)A.Bx * A.sx * A.NYf * A.Bt;
    A.vout = (int64_t)A.box * A.boy * A.bot;
    return A;
}

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

}  // namespace

extern "C" tred_status tred_direct_plan_create(const tred_grid* grid, const tred_blocking* blocking,
                                               const int32_t kpix[2], int32_t kticks, uint32_t flags,
                                               int32_t batch, tred_direct_plan** plan,
                                               int64_t* workspace_bytes) {
    TRED_TRY(validate_grid(grid));
    TRED_TRY(validate_blocking(blocking));
    TRED_REQUIRE(kpix && plan && workspace_bytes, "kpix/plan/workspace_bytes is NULL");
    TRED_REQUIRE(kpix[0] > 0 && kpix[1] > 0 && (kpix[0] & 1) && (kpix[1] & 1),
                 "kpix must be positive and odd");
    TRED_REQUIRE(kticks > 0, "kticks must be > 0");
    TRED_REQUIRE(batch > 0 && batch <= 65535, "batch must be in [1, 65535]");
    TRED_REQUIRE((flags & ~TRED_DIRECT_SPLIT) == 0, "unknown flags");
    *plan = nullptr;
    tred_direct_plan* P = new tred_direct_plan();
    P->grid = *grid;
    P->blk = *blocking;
    P->kpix[0] = kpix[0];
    P->kpix[1] = kpix[1];
    P->kticks = kticks;
    P->split = (flags & TRED_DIRECT_SPLIT) ? 1 : 0;
    P->batch = batch;
    P->S = grid->sub[0] * grid->sub[1];
    P->jpad = (P->S + 15) / 16 * 16;
    P->nk = kpix[0] * kpix[1];
    P->kpad = (P->nk + 31) / 32 * 32;
    P->npix = blocking->blk_pix[0] * blocking->blk_pix[1];
    P->tq = blocking->blk_ticks + 2 * kPad;
    P->bo[0] = blocking->blk_pix[0] + kpix[0] - 1;
    P->bo[1] = blocking->blk_pix[1] + kpix[1] - 1;
    P->bo[2] = blocking->blk_ticks + kticks - 1;
    const int64_t rsz = align256((int64_t)kticks * P->kpad * P->jpad * 2);
    const int64_t qsz = align256((int64_t)batch * P->npix * P->tq * P->jpad * 2);
    P->off_rhi = 0;
    P->off_rlo = rsz;
    P->off_qhi = 2 * rsz;
    P->off_qlo = 2 * rsz + qsz;
    P->ws_bytes = 2 * rsz + 2 * qsz;
    P->ws = nullptr;
    P->ready = 0;
    *plan = P;
    *workspace_bytes = P->ws_bytes;
    return TRED_OK;
}

extern "C" tred_status tred_direct_plan_set_response(tred_direct_plan* P, const float* resp,
                                                     void* workspace, void* stream) {
    TRED_REQUIRE(P && resp && workspace, "plan/resp/workspace is NULL");
    TRED_REQUIRE(((uintptr_t)workspace & 255) == 0, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    DirArgs A = make_dargs(P);
    const int64_t n = (int64_t)A.kt * A.kpad * A.jpad;
    hipLaunchKernelGGL(k_direct_resp, dim3(grid_for(n)), dim3(256), 0, st, A, resp,
                       (uint16_t*)(ws + P->off_rhi), (uint16_t*)(ws + P->off_rlo));
    TRED_TRY(tred_check_launch("direct response operands"));
    if (hipStreamSynchronize(st) != hipSuccess)
        return tred_fail(TRED_EDEVICE, "direct response operands: %s",
                         hipGetErrorString(hipGetLastError()));
    P->ws = workspace;
    P->ready = 1;
    return TRED_OK;
}

extern "C" tred_status tred_block_conv_direct(const tred_direct_plan* P, const int32_t* n_active,
                                              int32_t cap, const float* blocks, float* out_blocks,
                                              void* stream) {
    TRED_REQUIRE(P && n_active, "plan/n_active is NULL");
    TRED_REQUIRE(P->ready, "plan has no response (call tred_direct_plan_set_response)");
    TRED_REQUIRE(cap >= 0, "cap must be >= 0");
    if (cap == 0) return TRED_OK;
    TRED_REQUIRE(blocks && out_blocks, "blocks/out_blocks is NULL");
    hipStream_t st = (hipStream_t)stream;
    DirArgs A = make_dargs(P);
    A.cap = cap;
    char* ws = (char*)P->ws;
    const uint16_t* rhi = (const uint16_t*)(ws + P->off_rhi);
    const uint16_t* rlo = (const uint16_t*)(ws + P->off_rlo);
    uint16_t* qhi = (uint16_t*)(ws + P->off_qhi);
    uint16_t* qlo = (uint16_t*)(ws + P->off_qlo);
    const int npt = (A.npix + 31) / 32, nkt = A.kpad / 32;
    const int64_t combos = (int64_t)((npt + 1) / 2) * ((nkt + 1) / 2) * ((A.bot + kDirTT - 1) / kDirTT);
    if (combos * P->batch > 0x7fffffff || (int64_t)A.npix * A.tq * A.jpad * 2 > 0x7fffffff ||
        (int64_t)A.kt * A.kpad * A.jpad * 2 > 0x7fffffff)
        return tred_fail(TRED_EUNSUPPORTED, "bin too large for the direct path");
    for (int b0 = 0; b0 < cap; b0 += P->batch) {
        const int nb = std::min(P->batch, cap - b0);
        const int64_t nq = (int64_t)nb * A.npix * A.tq * A.jpad;
        hipLaunchKernelGGL(k_direct_charge, dim3(grid_for(nq)), dim3(256), 0, st, A, b0, nb, n_active,
                           blocks, qhi, qlo);
        hipLaunchKernelGGL(k_direct_zero, dim3(grid_for((int64_t)nb * A.vout)), dim3(256), 0, st, A, b0,
                           nb, n_active, out_blocks);
        const unsigned nwg = (unsigned)(combos * nb);
        if (P->split)
            hipLaunchKernelGGL((k_direct_mma<true, kDirTT>), dim3(nwg), dim3(256), 0, st, A, b0, nb,
                               n_active, qhi, qlo, rhi, rlo, out_blocks);
        else
            hipLaunchKernelGGL((k_direct_mma<false, kDirTT>), dim3(nwg), dim3(256), 0, st, A, b0, nb,
                               n_active, qhi, qlo, rhi, rlo, out_blocks);
        TRED_TRY(tred_check_launch("tred_block_conv_direct"));
    }
    return TRED_OK;
}

extern "C" void tred_direct_plan_destroy(tred_direct_plan* P) { delete P; }

// Internal helpers of the gfx950 library: status handling, complex arithmetic,
// in-register DFT codelets and the per-wavefront Stockham FFT used on the time axis.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tred.h"

// ---------------------------------------------------------------------------
// host-side status helpers (api.cpp)
// ---------------------------------------------------------------------------
tred_status tred_fail(tred_status s, const char* fmt, ...);
tred_status tred_check_launch(const char* what);

#define TRED_REQUIRE(cond, ...)                                      \
    do {                                                             \
        if (!(cond)) return tred_fail(TRED_EINVAL, __VA_ARGS__);     \
    } while (0)

constexpr int kWave = 64;
constexpr unsigned kXcd = 8;   // XCDs of an MI355X; workgroup ids are dealt to them round-robin

// ---------------------------------------------------------------------------
// effective charge added straight into the bins (effq.hip computes, bin.hip lays
// out the bins): the binning's bin -> slot map (slot, or -1 for a bin that is not
// held) and the geometry needed to address a fine cell inside its bin
// ---------------------------------------------------------------------------
struct EffqBins {
    float* blocks;
    const int32_t* slot;     // [nev][nbins]
    const int64_t* ev_off;   // event bounds over the depositions; NULL: one event
    int64_t nbins;           // bins per event
    int64_t vblk;            // cells per bin
    int32_t bf[3];           // bin extent in fine cells
    int32_t nb[3];           // bins per axis
    int32_t nev;
    float inv_bf2;           // 1 / bf[2] (binary32; bin index corrected by +-1)
};

// event of deposition d: ev_off[e] <= d < ev_off[e + 1] (ev_off NULL: one event)
__device__ __forceinline__ int event_of(int64_t d, const int64_t* __restrict__ ev_off, int nev) {
    if (ev_off == nullptr) return 0;
    int lo = 0, hi = nev - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ev_off[mid] <= d) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// (effq.hip) the effective charge of every deposition added into the bins of B
// (FP32 atomics), as tred_effq followed by the accumulation of the binning
tred_status effq_into_bins(const tred_grid* grid, const tred_physics* phys, int64_t n_dep,
                           const float* seg, const int32_t* fp, const EffqBins& B,
                           double* charge_sum, hipStream_t st);

// ---------------------------------------------------------------------------
// complex arithmetic on float2
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }
// multiply by +i
__device__ __forceinline__ float2 cmul_pi(float2 a) { return make_float2(-a.y, a.x); }

// ---------------------------------------------------------------------------
// Forward DFT codelets in registers, natural order in and out:
// X[k] = sum_n x[n] exp(-2 pi i n k / R).
// Twiddle constants are the correctly rounded binary32 values of cos/sin of
// multiples of pi/8.
// ---------------------------------------------------------------------------
namespace cst {
constexpr float r2 = 0.70710678118654752f;   // cos(pi/4)
constexpr float c8 = 0.92387953251128676f;   // cos(pi/8)
constexpr float s8 = 0.38268343236508977f;   // sin(pi/8)
}  // namespace cst

// multiply by exp(-2 pi i k / R) for compile-time k, R (R divides 16)
template <int R, int K>
__device__ __forceinline__ float2 wconst(float2 a) {
    constexpr int k16 = ((K * (16 / R)) % 16 + 16) % 16;  // angle in units of 2 pi / 16
    if constexpr (k16 == 0) return a;
    else if constexpr (k16 == 4) return cmul_mi(a);
    else if constexpr (k16 == 8) return make_float2(-a.x, -a.y);
    else if constexpr (k16 == 12) return cmul_pi(a);
    else if constexpr (k16 == 2) return make_float2(cst::r2 * (a.x + a.y), cst::r2 * (a.y - a.x));
    else if constexpr (k16 == 6) return make_float2(cst::r2 * (a.y - a.x), -cst::r2 * (a.x + a.y));
    else if constexpr (k16 == 10) return make_float2(-cst::r2 * (a.x + a.y), cst::r2 * (a.x - a.y));
    else if constexpr (k16 == 14) return make_float2(cst::r2 * (a.x - a.y), cst::r2 * (a.x + a.y));
    else {
        // generic: cos(2 pi k/16), sin(2 pi k/16) for odd k
        constexpr float cs[16] = {1.f, cst::c8, cst::r2, cst::s8, 0.f, -cst::s8, -cst::r2, -cst::c8,
                                  -1.f, -cst::c8, -cst::r2, -cst::s8, 0.f, cst::s8, cst::r2, cst::c8};
        constexpr float sn[16] = {0.f, cst::s8, cst::r2, cst::c8, 1.f, cst::c8, cst::r2, cst::s8,
                                  0.f, -cst::s8, -cst::r2, -cst::c8, -1.f, -cst::c8, -cst::r2, -cst::s8};
        // exp(-i theta) = cos - i sin
        return cmul(a, make_float2(cs[k16], -sn[k16]));
    }
}

template <int R>
struct Dft;

template <>
struct Dft<1> {
    __device__ __forceinline__ static void run(float2*) {}
};

template <>
struct Dft<2> {
    __device__ __forceinline__ static void run(float2* x) {
        float2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};

template <>
struct Dft<4> {
    __device__ __forceinline__ static void run(float2* x) {
        float2 s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
        float2 s13 = cadd(x[1], x[3]), d13 = csub(x[1], x[3]);
        x[0] = cadd(s02, s13);
        x[2] = csub(s02, s13);
        x[1] = cadd(d02, cmul_mi(d13));
        x[3] = csub(d02, cmul_mi(d13));
    }
};

// 3- and 5-point DFTs (the odd factors of the prime-factor spatial transforms);
// constants are the correctly rounded binary32 values of cos/sin of 2 pi k / R.
namespace cst {
constexpr float h3 = 0.86602540378443865f;   // sin(2 pi / 3)
constexpr float c51 = 0.30901699437494742f;  // cos(2 pi / 5)
constexpr float c52 = -0.80901699437494742f; // cos(4 pi / 5)
constexpr float s51 = 0.95105651629515357f;  // sin(2 pi / 5)
constexpr float s52 = 0.58778525229247313f;  // sin(4 pi / 5)
constexpr float c91 = 0.76604444311897801f;  // cos(2 pi / 9)
constexpr float s91 = 0.64278760968653925f;  // sin(2 pi / 9)
constexpr float c92 = 0.17364817766693041f;  // cos(4 pi / 9)
constexpr float s92 = 0.98480775301220802f;  // sin(4 pi / 9)
constexpr float c94 = -0.93969262078590832f; // cos(8 pi / 9)
constexpr float s94 = 0.34202014332566888f;  // sin(8 pi / 9)
}  // namespace cst

template <>
struct Dft<3> {
    __device__ __forceinline__ static void run(float2* x) {
        const float2 s = cadd(x[1], x[2]), d = csub(x[1], x[2]);
        const float2 m = make_float2(x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y);
        x[0] = cadd(x[0], s);
        x[1] = make_float2(m.x + cst::h3 * d.y, m.y - cst::h3 * d.x);
        x[2] = make_float2(m.x - cst::h3 * d.y, m.y + cst::h3 * d.x);
    }
};

template <>
struct Dft<5> {
    __device__ __forceinline__ static void run(float2* x) {
        const float2 a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
        const float2 a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
        const float2 x0 = x[0];
        // real-coefficient parts and the quadrature parts (multiplied by -i below)
        const float2 r1 = make_float2(x0.x + cst::c51 * a1.x + cst::c52 * a2.x,
                                      x0.y + cst::c51 * a1.y + cst::c52 * a2.y);
        const float2 r2 = make_float2(x0.x + cst::c52 * a1.x + cst::c51 * a2.x,
                                      x0.y + cst::c52 * a1.y + cst::c51 * a2.y);
        const float2 q1 = make_float2(cst::s51 * b1.x + cst::s52 * b2.x, cst::s51 * b1.y + cst::s52 * b2.y);
        const float2 q2 = make_float2(cst::s52 * b1.x - cst::s51 * b2.x, cst::s52 * b1.y - cst::s51 * b2.y);
        x[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
        x[1] = cadd(r1, cmul_mi(q1));
        x[4] = csub(r1, cmul_mi(q1));
        x[2] = cadd(r2, cmul_mi(q2));
        x[3] = csub(r2, cmul_mi(q2));
    }
};

// 9-point DFT as 3 x 3: n = 3 n1 + n2, k = k1 + 3 k2; 3-point DFTs over n1, the
// twiddles W9^(n2 k1), 3-point DFTs over n2.
template <>
struct Dft<9> {
    __device__ __forceinline__ static void run(float2* x) {
        float2 y[3][3];
#pragma unroll
        for (int n2 = 0; n2 < 3; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 3; ++n1) y[n2][n1] = x[3 * n1 + n2];
            Dft<3>::run(y[n2]);
        }
        // exp(-2 pi i k / 9) for k = n2 k1 in {1, 2, 4}
        y[1][1] = cmul(y[1][1], make_float2(cst::c91, -cst::s91));
        y[1][2] = cmul(y[1][2], make_float2(cst::c92, -cst::s92));
        y[2][1] = cmul(y[2][1], make_float2(cst::c92, -cst::s92));
        y[2][2] = cmul(y[2][2], make_float2(cst::c94, -cst::s94));
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
            float2 z[3] = {y[0][k1], y[1][k1], y[2][k1]};
            Dft<3>::run(z);
#pragma unroll
            for (int k2 = 0; k2 < 3; ++k2) x[k1 + 3 * k2] = z[k2];
        }
    }
};

// radix-2 split of an R-point DFT into two R/2-point DFTs (R = 8, 16)
template <int R>
struct Dft {
    template <int K>
    __device__ __forceinline__ static void comb(float2* x, const float2* e, const float2* o) {
        if constexpr (K < R / 2) {
            float2 t = wconst<R, K>(o[K]);
            x[K] = cadd(e[K], t);
            x[K + R / 2] = csub(e[K], t);
            comb<K + 1>(x, e, o);
        }
    }
    __device__ __forceinline__ static void run(float2* x) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = x[2 * i];
            o[i] = x[2 * i + 1];
        }
        Dft<R / 2>::run(e);
        Dft<R / 2>::run(o);
        comb<0>(x, e, o);
    }
};

// c + a * b as four fused multiply-adds
// Raw buffer loads: a 128-bit resource (base, size in bytes) held in scalar registers,
// a 32-bit per-lane byte offset and a wave-uniform byte offset. Offsets at or past
// the size read zero. Address arithmetic stays 32-bit, and a uniform part of the
// offset costs no vector instruction.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ float buf_f1(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ float2 buf_f2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ float4 buf_f4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
// Streaming stores of data read only by a later kernel (larger than the L2) may carry
// the non-temporal cache policy (TRED_NT_STORE).
#ifndef TRED_NT_STORE
#define TRED_NT_STORE 1
#endif
__device__ __forceinline__ void buf_st_f2(float2 v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                          uint32_t soff) {
    using u2 = __attribute__((ext_vector_type(2))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff,
                                          TRED_NT_STORE ? 2 : 0);
}

__device__ __forceinline__ void buf_st_f4(float4 v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                          uint32_t soff) {
    using u4 = __attribute__((ext_vector_type(4))) unsigned int;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, voff, soff,
                                           TRED_NT_STORE ? 2 : 0);
}

__device__ __forceinline__ void buf_st_f1(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                          uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}
__device__ __forceinline__ uint32_t buf_u8(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, voff, soff, 0);
}

__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
    c.x = fmaf(a.x, b.x, c.x);
    c.x = fmaf(-a.y, b.y, c.x);
    c.y = fmaf(a.x, b.y, c.y);
    c.y = fmaf(a.y, b.x, c.y);
    return c;
}

// ---------------------------------------------------------------------------
// Prime-factor (Good-Thomas) index maps of an FS-point DFT with FS = L * RS and
// gcd(L, RS) = 1. Input n <-> (n1, n2) with n = (RS n1 + L n2) mod FS; output
// k <-> (k1, k2) = (k mod L, k mod RS). Then
//   X[k] = sum_n1 W_L^(n1 k1) sum_n2 W_RS^(n2 k2) x[n(n1, n2)]
// with no twiddle factors between the L- and RS-point stages.
// ---------------------------------------------------------------------------
template <int L, int RS>
struct Pfa {
    static constexpr int FS = L * RS;
    static constexpr int inv(int a, int m) {
        for (int x = 0; x < m; ++x)
            if ((a * x) % m == 1 % m) return x;
        return -1;
    }
    static constexpr int RSi = inv(RS % L, L);            // RS^-1 mod L
    static constexpr int Li = RS > 1 ? inv(L % RS, RS) : 0;  // L^-1 mod RS
    static_assert(RSi >= 0 && Li >= 0, "L and RS must be coprime");
    __host__ __device__ static constexpr int n1(int n) { return (n * RSi) % L; }
    __host__ __device__ static constexpr int n2(int n) { return RS > 1 ? (n * Li) % RS : 0; }
    __host__ __device__ static constexpr int n_of(int a, int b) { return (RS * a + L * b) % FS; }
    __host__ __device__ static constexpr int k_of(int k1, int k2) {
        return (RS * RSi * k1 + L * Li * k2) % FS;
    }
};

// t[n1] = sum over inputs n < NIN with n1(n) = n1 of x[n] W_RS^(n2(n) k2), where
// w[j] = W_RS^(j k2) (w[0] = 1). The inputs n < L meet distinct n1; with NIN < L the
// classes that receive no input are zero (known to the compiler, so the DFT that
// follows folds them away).
template <int L, int RS, int NIN>
__device__ __forceinline__ void pfa_gather(const float2* x, const float2* w, float2* t) {
    using P = Pfa<L, RS>;
    if constexpr (NIN < L) {
#pragma unroll
        for (int a = 0; a < L; ++a) t[a] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int n = 0; n < NIN; ++n) {
        const int a = P::n1(n), b = P::n2(n);
        if (n < L) t[a] = b == 0 ? x[n] : cmul(x[n], w[b]);
        else t[a] = b == 0 ? cadd(t[a], x[n]) : cfma(x[n], w[b], t[a]);
    }
}

// ---------------------------------------------------------------------------
// Per-wavefront Stockham FFT of length N = 64 * M (M in {4, 8, 16, 32, 64}).
// On entry lane l holds x[l + 64 m] in v[m]; on exit X[l + 64 m] (forward DFT,
// natural order). `buf` is the wave's private LDS scratch of kFftLds<N> floats;
// `tw` is a table of exp(-2 pi i k / N), k < N, in device memory, or (TWL) the
// per-stage tables of FftTw<N> in LDS.
// Radix sequence: N = R1 * R2 * ... with every radix <= 16. The scratch is private
// to the wave (no workgroup barrier inside).
// Stage (radix R, Ns = product of earlier radices): butterfly j reads
// in[j + r N/R], multiplies by exp(-2 pi i r (j mod Ns) / (Ns R)), takes an
// R-point DFT and writes out[(j / Ns) Ns R + j mod Ns + r Ns].
// ---------------------------------------------------------------------------
template <int N>
struct FftPlan;
template <> struct FftPlan<256>  { static constexpr int R[4] = {4, 4, 4, 4}; static constexpr int S = 4; };
template <> struct FftPlan<512>  { static constexpr int R[4] = {8, 8, 8, 1}; static constexpr int S = 3; };
template <> struct FftPlan<1024> { static constexpr int R[4] = {16, 16, 4, 1}; static constexpr int S = 3; };
template <> struct FftPlan<2048> { static constexpr int R[4] = {16, 16, 8, 1}; static constexpr int S = 3; };
template <> struct FftPlan<4096> { static constexpr int R[4] = {16, 16, 16, 1}; static constexpr int S = 3; };

// Per-stage twiddle tables for LDS: stage s (radix R, Ns = product of the earlier
// radices, Ns > 1) holds W_N^(r j (N / (Ns R))) at [r - 1][j], r = 1 .. R-1, j < Ns, so
// the lanes of a wave (consecutive j) read consecutive words. The tables of all stages
// take fewer than N entries.
template <int N>
struct FftTw {
    using P = FftPlan<N>;
    static constexpr int ns(int s) {
        int v = 1;
        for (int t = 0; t < s; ++t) v *= P::R[t];
        return v;
    }
    static constexpr int size(int s) { return s == 0 ? 0 : ns(s) * (P::R[s] - 1); }
    static constexpr int off(int s) {
        int o = 0;
        for (int t = 0; t < s; ++t) o += size(t);
        return o;
    }
    static constexpr int stage_of(int nsv) {
        for (int t = 0; t < P::S; ++t)
            if (ns(t) == nsv) return t;
        return -1;
    }
    static constexpr int total() { return off(P::S); }
    static_assert(total() <= N, "stage twiddles exceed the table");
};

// fill the per-stage tables at dst (LDS) from the N-entry table tw (device memory)
template <int N>
__device__ __forceinline__ void fft_tw_fill(float2* dst, const float2* __restrict__ tw, int tid,
                                            int nthreads) {
    using F = FftTw<N>;
    for (int s = 1; s < F::P::S; ++s) {
        const int nsv = F::ns(s), R = F::P::R[s];
        for (int i = tid; i < F::size(s); i += nthreads) {
            const int r = i / nsv + 1, j = i % nsv;
            dst[F::off(s) + i] = tw[r * j * (N / (nsv * R))];
        }
    }
}

// Ordering of LDS accesses within one wavefront: the wave's LDS operations execute
// in issue order, so it suffices to keep the compiler from moving accesses across
// this point (the buffers of wave_fft are private to the wave).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// padded LDS index: one pad word per 16 (keeps stride-16 accesses conflict free)
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
template <int N>
constexpr int kFftLds = 2 * (N + N / 16);

// WS: the scratch is private to the wave and only wave-level ordering is needed;
// otherwise the stages are separated by workgroup barriers.
template <bool WS>
__device__ __forceinline__ void fft_sync() {
    if constexpr (WS) wave_lds_sync();
    else __syncthreads();
}

// TWL: the per-stage twiddle tables (FftTw) are in LDS and read where they are used (LDS loads leave the
// vector-memory counter alone, so loads in flight from before the FFT are not waited
// for); otherwise it is in device memory, read through a buffer resource (32-bit
// offsets), and a stage requests all its twiddles before its first butterfly.
template <int N, int R, int NS, bool FIRST, bool WS, bool TWL>
__device__ __forceinline__ void fft_stage(float2* v, float* buf, const float2* tw, int lane) {
    constexpr int M = N / kWave;
    constexpr int NB = N / R;            // butterflies in this stage
    constexpr int PER = NB / kWave;      // butterflies per lane
    static_assert(PER >= 1 && PER * R == M, "radix does not match the lane data");
    float* re = buf;
    float* im = buf + (N + N / 16);
    constexpr int NW = (NS > 1 && !TWL) ? R : 1;
    float2 w[PER][NW];
    if constexpr (NS > 1 && !TWL) {
        const auto twr = buf_rsrc(tw, (uint32_t)(N * sizeof(float2)));
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int jm = (lane + kWave * i) % NS;
#pragma unroll
            for (int r = 1; r < R; ++r)
                w[i][r] = buf_f2(twr, (uint32_t)(r * jm * (N / (NS * R))) * 8u, 0u);
        }
    }
    float2 u[M];
    if constexpr (FIRST) {
        // inputs in[j + r N/R] with j = lane + 64 i: register i + r * PER
#pragma unroll
        for (int m = 0; m < M; ++m) u[m] = v[m];
    } else {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            int j = lane + kWave * i;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                int idx = lpad(j + r * NB);
                u[i * R + r] = make_float2(re[idx], im[idx]);
            }
        }
    }
    fft_sync<WS>();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        int j = lane + kWave * i;
        float2 x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = FIRST ? u[i + r * PER] : u[i * R + r];
        if constexpr (NS > 1) {
            if constexpr (TWL) {
                // one base per butterfly, the radix index in the immediate offset
                const float2* twb = tw + FftTw<N>::off(FftTw<N>::stage_of(NS)) + j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) x[r] = cmul(x[r], twb[(r - 1) * NS]);
            } else {
#pragma unroll
                for (int r = 1; r < R; ++r) x[r] = cmul(x[r], w[i][NW > 1 ? r : 0]);
            }
        }
        Dft<R>::run(x);
        int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int idx = lpad(base + r * NS);
            re[idx] = x[r].x;
            im[idx] = x[r].y;
        }
    }
    fft_sync<WS>();
}

template <int N, bool WS, bool TWL = false>
__device__ __forceinline__ void wave_fft(float2* v, float* buf, const float2* tw, int lane) {
    using P = FftPlan<N>;
    constexpr int R0 = P::R[0], R1 = P::R[1], R2 = P::R[2], R3 = P::R[3];
    fft_stage<N, R0, 1, true, WS, TWL>(v, buf, tw, lane);
    fft_stage<N, R1, R0, false, WS, TWL>(v, buf, tw, lane);
    if constexpr (P::S >= 3) fft_stage<N, R2, R0 * R1, false, WS, TWL>(v, buf, tw, lane);
    if constexpr (P::S >= 4) fft_stage<N, R3, R0 * R1 * R2, false, WS, TWL>(v, buf, tw, lane);
    constexpr int M = N / kWave;
    const float* re = buf;
    const float* im = buf + (N + N / 16);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        int idx = lpad(lane + kWave * m);
        v[m] = make_float2(re[idx], im[idx]);
    }
    fft_sync<WS>();
}

// ---------------------------------------------------------------------------
// Plan object (host side)
// ---------------------------------------------------------------------------
struct tred_conv_plan {
    tred_grid grid;
    tred_blocking blk;
    int32_t kpix[2];
    int32_t kticks;
    int32_t fs;          // spatial FFT size (square)
    int32_t ls;          // length of the register sub-DFTs of the spatial transform
    int32_t pfa;         // spatial stage by prime-factor maps (fs = ls * RS, coprime)
    int32_t nin;         // inputs per axis of the prime-factor stage (ls / 2, ls or 2 ls)
    int32_t spp_nb;      // bins per workgroup of the prime-factor stage
    int32_t ft;          // time FFT size
    int32_t ct;          // response ticks per piece
    int32_t nc;          // response pieces
    int32_t nch;         // transformed channels (pairs under MPCP)
    int32_t mpcp;
    int32_t batch;
    int32_t bo[3];       // output block extent
    int32_t qpad;        // output pixels per block padded to the tile of 8
    // workspace layout (byte offsets)
    int64_t off_tw_t, off_tw_s, off_rhat, off_chan, off_scratch_t, off_scratch_u;
    int64_t off_tflag;   // liveness of the time-FFT row groups (one byte each)
    int64_t off_tlist, off_tcount;   // live T tiles of a pass (int2 each) and their count
    int64_t ws_bytes;
    void* ws;            // bound by set_response
    int ready;
    hipEvent_t ev[6];    // optional stage timing
    int timing;
};

constexpr int kTile = 8;   // pixels per interleaved tile of the spectral scratch
constexpr int kTileP = kTile + 1;   // LDS row stride of a staged tile (odd: no bank conflicts)
// pixels per frequency in a tile of the time spectra T: 16 (one 128-byte line) or 8
#ifndef TRED_TTILE
#define TRED_TTILE 16
#endif
constexpr int kTileT = TRED_TTILE;

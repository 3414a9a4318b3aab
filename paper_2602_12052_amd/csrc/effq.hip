// Transport, quadrature windows and effective charge of line-segment depositions
// (Sec. II-A; Sec. II-C eqs. cub, trilinear, eff_q, qline and the point-like limit).
#include <cmath>

#include "tred_internal.hpp"
#include "validate.hpp"

// threads per deposition and LDS floats of a tile of the effective-charge kernel
#ifndef TRED_EFFQ_NT
#define TRED_EFFQ_NT 256
#endif
#ifndef TRED_EFFQ_CAP
#define TRED_EFFQ_CAP 9984   // 39 KiB: four workgroups per CU (160 KiB of LDS)
#endif

namespace {

// ---------------------------------------------------------------------------
// Discrete decisions: a fixed chain of correctly rounded binary32 operations.
// Division and square root are evaluated in binary64 and rounded once to
// binary32, which equals the correctly rounded binary32 result (53 >= 2*24 + 2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float div_rn(float a, float b) { return (float)((double)a / (double)b); }
__device__ __forceinline__ float sqrt_rn(float a) { return (float)sqrt((double)a); }

__device__ __forceinline__ int32_t floor_to_int(float v) {
    float f = floorf(v);
    f = fminf(fmaxf(f, -16777216.0f), 16777216.0f);
    return (int32_t)f;
}

struct Win {
    int32_t lo[3], hi[3];
    int point;
};

__device__ Win window_f32(const tred_grid& g, const tred_physics& ph, const float* s) {
#pragma clang fp contract(off)
    Win w;
    const float v = ph.v_drift;
    const float t0 = div_rn(s[2], v);
    const float t1 = div_rn(s[5], v);
    float tm = (t0 + t1) * 0.5f;
    if (tm < 0.0f) tm = 0.0f;
    const float sT = sqrt_rn((2.0f * ph.diff_T) * tm);
    const float sL = div_rn(sqrt_rn((2.0f * ph.diff_L) * tm), v);
    const float sg[3] = {fmaxf(sT, ph.sigma_min[0]), fmaxf(sT, ph.sigma_min[1]),
                         fmaxf(sL, ph.sigma_min[2])};
    const float P0[3] = {s[0], s[1], t0};
    const float P1[3] = {s[3], s[4], t1};
    int point = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float h = g.spacing[a];
        float u0 = div_rn(P0[a] - g.origin[a], h);
        float u1 = div_rn(P1[a] - g.origin[a], h);
        if (a == 2) {
            u0 = u0 + 0.5f;
            u1 = u1 + 0.5f;
        }
        const float e = ph.n_sigma * div_rn(sg[a], h);
        const float umin = u0 < u1 ? u0 : u1;
        const float umax = u0 < u1 ? u1 : u0;
        w.lo[a] = floor_to_int(umin - e);
        w.hi[a] = floor_to_int(umax + e);
        const float dd = fabsf(P1[a] - P0[a]);
        if (!(dd < ph.point_frac * sg[a])) point = 0;
    }
    w.point = point;
    return w;
}

__device__ __forceinline__ int nfine(const tred_grid& g, int a) {
    return a == 0 ? g.npix[0] * g.sub[0] : a == 1 ? g.npix[1] * g.sub[1] : g.nticks;
}

__global__ __launch_bounds__(256) void k_windows(tred_grid g, tred_physics ph, int64_t n,
                                                 const float* __restrict__ seg,
                                                 int32_t* __restrict__ fp,
                                                 int64_t* __restrict__ off) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d == 0) off[0] = 0;
    if (d >= n) return;
    float s[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) s[k] = seg[7 * d + k];
    Win w = window_f32(g, ph, s);
    int64_t vol = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int32_t N = nfine(g, a);
        int32_t lo = max(w.lo[a] - 1, 0);
        int32_t hi = min(w.hi[a] + 1, N - 1);
        fp[6 * d + a] = lo;
        fp[6 * d + 3 + a] = hi;
        vol = hi < lo ? 0 : vol * (int64_t)(hi - lo + 1);
    }
    off[d + 1] = vol;
}

// In-place inclusive scan of a[1..n] by one workgroup of 1024 threads.
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int64_t u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

__global__ __launch_bounds__(1024) void k_scan_inplace(int64_t* __restrict__ a, int64_t n) {
    constexpr int PER = 16;
    __shared__ int64_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += 1024 * PER) {
        int64_t v[PER];
        int64_t s = 0;
        const int64_t i0 = base + (int64_t)tid * PER;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            v[k] = (i0 + k < n) ? a[1 + i0 + k] : 0;
            s += v[k];
        }
        int64_t incl = wave_incl_scan(s, lane);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        if (wave == 0) {
            int64_t t = lane < 16 ? wsum[lane] : 0;
            t = wave_incl_scan(t, lane);
            if (lane < 16) wsum[lane] = t;
        }
        __syncthreads();
        int64_t run = carry + incl - s + (wave > 0 ? wsum[wave - 1] : 0);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            run += v[k];
            if (i0 + k < n) a[1 + i0 + k] = run;
        }
        carry += wsum[15];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Effective charge
// ---------------------------------------------------------------------------
struct EffqParams {
    tred_grid g;
    tred_physics ph;
    float xi[8];   // Gauss-Legendre nodes on [-1,1], ascending
    float w[8];    // weights
    float u[16];   // per-axis spread weights over the node stencil of one grid point
};

// exp(x) for x <= 0 on the hardware base-2 exponential: exp2(x log2 e). The rounded
// product costs a relative error of about |x| 2^-24 (below 1e-6 for the Gaussians of
// a quadrature window); results under 2^-126 flush to zero.
__device__ __forceinline__ float exp_neg(float x) {
    return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}

// exp(-e / 2) for e >= 0, the factor -log2(e) / 2 folded into one product
__device__ __forceinline__ float exp_neg_half(float e) {
    return __builtin_amdgcn_exp2f(e * -0.72134752044448170f);
}

// erfc(z) for z >= 0 in the form t exp(-z^2 + P(t)), t = 1 / (1 + z / 2) (the Chebyshev
// form of Numerical Recipes' erfcc); P is a degree-9 least-squares fit made for this
// library (erfc_fit.py: relative error below 6e-7 on [0, 2], below 7e-6 up to z = 9).
__device__ __forceinline__ float erfc_pos(float z) {
    constexpr float c[10] = {-1.265481591e+00f, 9.994024634e-01f,  3.792311549e-01f,
                             7.404764742e-02f,  -1.270266324e-01f, 1.849500537e-01f,
                             -1.046039343e+00f, 1.441537738e+00f,  -8.111995459e-01f,
                             1.705782861e-01f};
    constexpr float l2e = 1.44269504088896341f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, z, 1.0f));
    // P(t) log2(e) by Horner on the coefficients times log2(e) (binary32 products,
    // folded at compile time)
    float p = c[9] * l2e;
#pragma unroll
    for (int k = 8; k >= 0; --k) p = fmaf(p, t, c[k] * l2e);
    return t * __builtin_amdgcn_exp2f(fmaf(-z * l2e, z, p));
}

// erf(b) - erf(a) for a <= b from erfc(|a|) and erfc(|b|): erfc(a) - erfc(b) when both
// are >= 0, erfc(|b|) - erfc(|a|) when both are <= 0 (no cancellation of the tails),
// 2 - erfc(|a|) - erfc(|b|) across zero. Branch free.
__device__ __forceinline__ float erf_diff(float b, float a) {
    const float ea = erfc_pos(fabsf(a)), eb = erfc_pos(fabsf(b));
    // all three forms, then selects (no divergent branches)
    const float pos = ea - eb, neg = eb - ea, across = (2.0f - ea) - eb;
    const float r = b <= 0.0f ? neg : across;
    return a >= 0.0f ? pos : r;
}

// Small 3-D index iterator advancing by a fixed stride (avoids per-element divisions).
struct Idx3 {
    int i, j, k;        // k fastest
    int nj, nk;
    int di, dj, dk;     // decomposition of the stride
    __device__ void init(int start, int stride, int nj_, int nk_) {
        nj = nj_;
        nk = nk_;
        k = start % nk;
        int r = start / nk;
        j = r % nj;
        i = r / nj;
        dk = stride % nk;
        r = stride / nk;
        dj = r % nj;
        di = r / nj;
    }
    __device__ void next() {
        k += dk;
        int c = 0;
        if (k >= nk) { k -= nk; c = 1; }
        j += dj + c;
        c = 0;
        if (j >= nj) { j -= nj; c = 1; }
        i += di + c;
    }
};

// One workgroup of NT threads per deposition (grid-stride over depositions). Every
// Gauss-Legendre node of the window cells is evaluated once, by the thread that owns
// its (x-node, y-node) column: the thread walks the column along t and applies the t
// part of the trilinear spread in registers (the nodes of cells g-1, g and g+1 reach
// grid point g), writing A[y-node][t][x-node]; the x and y parts follow in one pass in
// which every footprint cell sums the S x S stencil columns from LDS (per y node, the
// S x nodes are consecutive and read in pairs). The footprint is cut into tiles (the
// whole x-y extent when it fits, as many ticks as fit); between t tiles a column's
// sliding state (the node charges of the two cells the next tile still needs) is kept
// in LDS, so no node is evaluated twice along t. Only columns of window cells are
// stored; per-tile tables give every footprint cell's stencil its weights, zero for
// nodes outside the window (those reads land on other finite values of the tile).
// (four waves per SIMD for the 2-point rule: four 256-thread workgroups per CU)
// BIN: the cells are added into the bins of B (FP32 atomics) instead of being written
// as patches; off, val and val_cap are not used.
template <int NGL, int CAP, int NT, bool BIN>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NGL <= 2 ? 4 : 1))) void k_effq(
    EffqParams P, int64_t n_dep, const float* __restrict__ seg, const int32_t* __restrict__ fp,
    const int64_t* __restrict__ off, float* __restrict__ val, int64_t val_cap,
    double* __restrict__ charge_sum, EffqBins B) {
    constexpr int NPOS = NGL / 2;                 // nodes with xi > 0 in a cell
    constexpr int S = NGL + 2 * NPOS;             // stencil nodes per axis
    constexpr int NST = NPOS + NGL;               // sliding state of a column
    constexpr int TX = (S + 1 + 3) / 4 * 4;       // x table row: first node, S weights
    // y table row: S offsets, S weights (BIN: and the y parts of the bin index and of
    // the cell offset in its bin; the x table row holds the x parts after its weights)
    constexpr int TY = 2 * S + (BIN ? 2 : 0);
    constexpr int NW = NT / kWave;
    __shared__ __align__(16) float sm[CAP];
    __shared__ double red[NW];
    __shared__ float sxi[8], sw[8];
    const int tid = threadIdx.x;
    const tred_grid& g = P.g;
    if (tid < 8) {
        sxi[tid] = P.xi[tid];
        sw[tid] = P.w[tid];
    }
    float su[S];
#pragma unroll
    for (int k = 0; k < S; ++k) su[k] = P.u[k];
    // every float of the tile memory holds a finite value from here on (the gather reads
    // a few floats beyond a row with weight zero)
    for (int i = tid; i < CAP; i += NT) sm[i] = 0.0f;
    __syncthreads();

    for (int64_t d = blockIdx.x; d < n_dep; d += gridDim.x) {
        const int32_t* f = fp + 6 * d;
        int F0[3] = {f[0], f[1], f[2]}, F1[3] = {f[3], f[4], f[5]};
        if (F1[0] < F0[0] || F1[1] < F0[1] || F1[2] < F0[2]) continue;
        int64_t o0 = 0;
        const int32_t* slotp = nullptr;   // BIN: the slot map of this deposition's event
        if constexpr (BIN) {
            slotp = B.slot + (int64_t)event_of(d, B.ev_off, B.nev) * B.nbins;
        } else {
            const int64_t o1 = off[d + 1];
            o0 = off[d];
            // patches past val_cap, or of 2^31 cells or more (32-bit offsets), are skipped
            if (o1 > val_cap || o1 - o0 > INT32_MAX) continue;
        }
        float s[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) s[k] = seg[7 * d + k];
        const Win W = window_f32(g, P.ph, s);

        // transport (binary64 per deposition, Sec. II-A)
        const double v = P.ph.v_drift;
        const double t0 = (double)s[2] / v, t1 = (double)s[5] / v;
        double tm = 0.5 * (t0 + t1);
        if (tm < 0.0) tm = 0.0;
        const double Qp = (double)s[6] * exp(-tm / (double)P.ph.lifetime);
        const double sT = sqrt(2.0 * (double)P.ph.diff_T * tm);
        const double sg[3] = {fmax(sT, (double)P.ph.sigma_min[0]), fmax(sT, (double)P.ph.sigma_min[1]),
                              fmax(sqrt(2.0 * (double)P.ph.diff_L * tm) / v, (double)P.ph.sigma_min[2])};
        const double h[3] = {g.spacing[0], g.spacing[1], g.spacing[2]};
        const double D[3] = {(double)s[3] - (double)s[0], (double)s[4] - (double)s[1], t1 - t0};
        // node coordinates relative to the segment start (line) or midpoint (point):
        // r_a = base_a + ((c - lo_a) + xi/2) h_a
        double base[3];
        base[0] = (double)g.origin[0] + ((double)W.lo[0] + 0.5) * h[0] - (double)s[0];
        base[1] = (double)g.origin[1] + ((double)W.lo[1] + 0.5) * h[1] - (double)s[1];
        base[2] = (double)g.origin[2] + (double)W.lo[2] * h[2] - t0;
        const bool point = W.point != 0;
        float fb[3], fh[3], fd[3], isg2[3], gvec[3];
        float inv_alpha = 0.f, kq = 0.f, pref;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            fb[a] = (float)(point ? base[a] - 0.5 * D[a] : base[a]);
            fh[a] = (float)h[a];
            fd[a] = (float)D[a];
            isg2[a] = (float)(1.0 / (sg[a] * sg[a]));
            gvec[a] = 0.f;
        }
        // the rule's Jacobian h_x h_y tick / 8 is folded into the prefactor
        const double jac = h[0] * h[1] * h[2] / 8.0;
        if (point) {
            pref = (float)(jac * Qp * pow(2.0 * M_PI, -1.5) / (sg[0] * sg[1] * sg[2]));
        } else {
            double alpha = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                gvec[a] = (float)(D[a] / (sg[a] * sg[a]));
                alpha += D[a] * D[a] / (sg[a] * sg[a]);
            }
            inv_alpha = (float)(1.0 / alpha);
            kq = (float)sqrt(0.5 * alpha);
            // Q / (4 pi Delta) with Delta = sigma_x sigma_y sigma_t sqrt(alpha)
            pref = (float)(jac * Qp / (4.0 * M_PI * sg[0] * sg[1] * sg[2] * sqrt(alpha)));
        }

        // cells whose nodes are evaluated: the quadrature window (intersected with F +- 1)
        int C0[3], C1[3], Fs[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C0[a] = max(W.lo[a], F0[a] - 1);
            C1[a] = min(W.hi[a], F1[a] + 1);
            Fs[a] = F1[a] - F0[a] + 1;
        }
        // tiles. LDS: the stencil tables of the tile's x and y cells, A[y node][t][x node]
        // (window columns; rows of PX = ncx | 1 floats, odd so that the columns' rows
        // start in distinct banks) between two guard bands of S floats, and the
        // columns' sliding state
        const int nwx = C1[0] - C0[0] + 1, nwy = C1[1] - C0[1] + 1;
        auto ncols = [&](int t, int nw) { return max(0, min(t + 2, nw)) * NGL; };
        auto fixed = [&](int t0, int t1) {   // floats besides the ticks of A
            const int cx = ncols(t0, nwx), cy = ncols(t1, nwy);
            return t0 * TX + t1 * TY + 2 * S + cx * cy * NST;
        };
        auto per_tick = [&](int t0, int t1) { return ncols(t1, nwy) * (ncols(t0, nwx) | 1); };
        int T[3] = {Fs[0], Fs[1], Fs[2]};
        {
            const int tmin = min(Fs[2], 5);
            while (fixed(T[0], T[1]) + tmin * per_tick(T[0], T[1]) > CAP && (T[0] > 1 || T[1] > 1)) {
                if (T[0] >= T[1]) T[0] = (T[0] + 1) / 2;
                else T[1] = (T[1] + 1) / 2;
            }
            const int pt = per_tick(T[0], T[1]);
            if (pt > 0) T[2] = max(1, min(Fs[2], (CAP - fixed(T[0], T[1])) / pt));
        }
        // patch of this deposition (its cell count, FX FY FT, is below 2^31: 32-bit offsets)
        const int FY = Fs[1], FT = Fs[2];
        float* vd = BIN ? nullptr : val + o0;
        double nsum = 0.0;

        for (int X0 = F0[0]; X0 <= F1[0]; X0 += T[0])
            for (int Y0 = F0[1]; Y0 <= F1[1]; Y0 += T[1]) {
                const int X1 = min(X0 + T[0] - 1, F1[0]);
                const int Y1 = min(Y0 + T[1] - 1, F1[1]);
                // window cells among x in X0-1 .. X1+1, y in Y0-1 .. Y1+1
                const int ex0 = max(X0 - 1, C0[0]), ex1 = min(X1 + 1, C1[0]);
                const int ey0 = max(Y0 - 1, C0[1]), ey1 = min(Y1 + 1, C1[1]);
                const int ncx = max(0, ex1 - ex0 + 1) * NGL, ncy = max(0, ey1 - ey0 + 1) * NGL;
                const int ncw = ncx * ncy;
                const int PX = ncx | 1, PY = T[2] * PX;
                // cells whose nodes this x-y tile counts in the charge sum (x, y tiles share
                // their edge cells; along t every cell is counted once)
                const int ox0 = max(X0 == F0[0] ? X0 - 1 : X0, C0[0]);
                const int ox1 = min(X1 == F1[0] ? X1 + 1 : X1, C1[0]);
                const int oy0 = max(Y0 == F0[1] ? Y0 - 1 : Y0, C0[1]);
                const int oy1 = min(Y1 == F1[1] ? Y1 + 1 : Y1, C1[1]);
                const int nx = X1 - X0 + 1, ny = Y1 - Y0 + 1;
                float* tabx = sm;                               // [nx][TX]: x0 node, S weights
                float* taby = sm + T[0] * TX;                   // [ny][TY]: S offsets, S weights
                float* A = taby + T[1] * TY + S;                // [ncy][T2][PX]
                float* ST = A + ncy * PY + S;                   // [ncw][NST]
                // stencil tables: cell g of the tile gathers nodes x0 .. x0 + S - 1 (node
                // NGL - NPOS of cell g - 1 onwards); those outside the window weigh zero
                for (int i = tid; i < nx + ny; i += NT) {
                    if (i < nx) {
                        const int x0 = (X0 + i - 1 - ex0) * NGL + (NGL - NPOS);
                        tabx[i * TX] = __int_as_float(x0);
#pragma unroll
                        for (int a = 0; a < S; ++a)
                            tabx[i * TX + 1 + a] = (x0 + a >= 0 && x0 + a < ncx) ? su[a] : 0.0f;
                        if constexpr (BIN) {
                            const int gx = X0 + i, bx = gx / B.bf[0];
                            tabx[i * TX + S + 1] = __int_as_float(bx * B.nb[1] * B.nb[2]);
                            tabx[i * TX + S + 2] = __int_as_float((gx - bx * B.bf[0]) * B.bf[1] * B.bf[2]);
                        }
                    } else {
                        const int y = i - nx;
                        const int y0 = (Y0 + y - 1 - ey0) * NGL + (NGL - NPOS);
#pragma unroll
                        for (int b = 0; b < S; ++b) {
                            const bool ok = y0 + b >= 0 && y0 + b < ncy;
                            taby[y * TY + b] = __int_as_float((ok ? y0 + b : 0) * PY);
                            taby[y * TY + S + b] = ok ? su[b] : 0.0f;
                        }
                        if constexpr (BIN) {
                            const int gy = Y0 + y, by = gy / B.bf[1];
                            taby[y * TY + 2 * S] = __int_as_float(by * B.nb[2]);
                            taby[y * TY + 2 * S + 1] = __int_as_float((gy - by * B.bf[1]) * B.bf[2]);
                        }
                    }
                }
                for (int Z0 = F0[2]; Z0 <= F1[2]; Z0 += T[2]) {
                    const int Z1 = min(Z0 + T[2] - 1, F1[2]);
                    const int nz = Z1 - Z0 + 1;
                    const bool first = Z0 == F0[2], last = Z1 == F1[2];
                    // 1) columns: node charges along t, t part of the spread
                    const int c0t = __builtin_amdgcn_readfirstlane(C0[2]);
                    const int c1t = __builtin_amdgcn_readfirstlane(C1[2]);
                    for (int c = tid; c < ncw; c += NT) {
                        const int yn = c / ncx, xn = c - yn * ncx;
                        const int cx = ex0 + xn / NGL, lx = xn % NGL;
                        const int cy = ey0 + yn / NGL, ly = yn % NGL;
                        float xx, xy, wxy;
                        if constexpr (NGL == 2) {
                            constexpr float xi2 = 0.57735026918962576f;   // nodes -+1/sqrt(3)
                            xx = lx ? xi2 : -xi2;
                            xy = ly ? xi2 : -xi2;
                            wxy = 1.0f;
                        } else {
                            xx = sxi[lx];
                            xy = sxi[ly];
                            wxy = sw[lx] * sw[ly];
                        }
                        const float rx = fb[0] + ((float)(cx - W.lo[0]) + 0.5f * xx) * fh[0];
                        const float ry = fb[1] + ((float)(cy - W.lo[1]) + 0.5f * xy) * fh[1];
                        const bool cnt = cx >= ox0 && cx <= ox1 && cy >= oy0 && cy <= oy1;
                        const float bxy = rx * gvec[0] + ry * gvec[1];
                        const float exy = rx * rx * isg2[0] + ry * ry * isg2[1];
                        // w * q of the NGL nodes of cell ct (zero outside the window); the
                        // column's nodes are summed in binary32 (csum: at most the T2 + 2
                        // cells of this tile) and the sum joins the binary64 total once
                        float csum = 0.0f;
                        auto cell = [&](int ct, float* q) {
                            // ct is the same for every column of the tile: the cells
                            // outside the window (two at each end of a column) are
                            // skipped by the whole workgroup
                            const int cts = __builtin_amdgcn_readfirstlane(ct);
                            if (cts < c0t || cts > c1t) {
#pragma unroll
                                for (int l = 0; l < NGL; ++l) q[l] = 0.0f;
                                return;
                            }
                            const float ctf = (float)(ct - W.lo[2]);
#pragma unroll
                            for (int l = 0; l < NGL; ++l) {
                                float xt, wt;
                                if constexpr (NGL == 2) {
                                    constexpr float xi2 = 0.57735026918962576f;
                                    xt = l ? xi2 : -xi2;
                                    wt = wxy;
                                } else {
                                    xt = sxi[l];
                                    wt = wxy * sw[l];
                                }
                                const float rt = fb[2] + (ctf + 0.5f * xt) * fh[2];
                                float v;
                                if (point) {
                                    v = pref * exp_neg_half(fmaf(rt * isg2[2], rt, exy));
                                } else {
                                    const float sst = fmaf(rt, gvec[2], bxy) * inv_alpha;   // closest point on the line
                                    const float px = rx - sst * fd[0], py = ry - sst * fd[1], pt = rt - sst * fd[2];
                                    const float e = px * px * isg2[0] + py * py * isg2[1] + pt * pt * isg2[2];
                                    v = pref * exp_neg_half(e) * erf_diff(kq * (1.0f - sst), -kq * sst);
                                }
                                q[l] = wt * v;
                                csum += q[l];
                            }
                        };
                        float hold[NPOS > 0 ? NPOS : 1], cur[NGL], nxt[NGL];
                        float* stc = ST + c * NST;
                        if (first) {
                            // cells F0t - 1 and F0t: every node counted once
                            cell(Z0 - 1, nxt);
#pragma unroll
                            for (int k = 0; k < NPOS; ++k) hold[k] = nxt[NGL - NPOS + k];
                            cell(Z0, cur);
                        } else {
#pragma unroll
                            for (int k = 0; k < NPOS; ++k) hold[k] = stc[k];
#pragma unroll
                            for (int k = 0; k < NGL; ++k) cur[k] = stc[NPOS + k];
                        }
                        float* arow = A + yn * PY + xn;
                        for (int j = 0; j < nz; ++j) {
                            cell(Z0 + j + 1, nxt);
                            float a = 0.0f;
#pragma unroll
                            for (int k = 0; k < NPOS; ++k) a = fmaf(su[k], hold[k], a);
#pragma unroll
                            for (int k = 0; k < NGL; ++k) a = fmaf(su[NPOS + k], cur[k], a);
#pragma unroll
                            for (int k = 0; k < NPOS; ++k) a = fmaf(su[NPOS + NGL + k], nxt[k], a);
                            arow[j * PX] = a;
#pragma unroll
                            for (int k = 0; k < NPOS; ++k) hold[k] = cur[NGL - NPOS + k];
#pragma unroll
                            for (int k = 0; k < NGL; ++k) cur[k] = nxt[k];
                        }
                        if (!last) {
#pragma unroll
                            for (int k = 0; k < NPOS; ++k) stc[k] = hold[k];
#pragma unroll
                            for (int k = 0; k < NGL; ++k) stc[NPOS + k] = cur[k];
                        }
                        if (cnt) nsum += (double)csum;
                    }
                    __syncthreads();
                    // 2) x and y parts of the spread: each footprint cell of the tile sums the
                    //    S x S stencil columns with the tables' weights
                    {
                        const int count = nx * ny * nz;
                        Idx3 it;
                        it.init(tid, NT, ny, nz);
                        for (int k = tid; k < count; k += NT, it.next()) {
                            const float* tx = tabx + it.i * TX;
                            const float* ty = taby + it.j * TY;
                            const float* ab = A + it.k * PX + __float_as_int(tx[0]);
                            float acc = 0.0f;
#pragma unroll
                            for (int b = 0; b < S; ++b) {
                                const float* r = ab + __float_as_int(ty[b]);
                                float ax = 0.0f;
#pragma unroll
                                for (int a = 0; a < S; ++a) ax = fmaf(tx[1 + a], r[a], ax);
                                acc = fmaf(ty[S + b], ax, acc);
                            }
                            if constexpr (BIN) {
                                // t bin of the cell (the binary32 quotient is within one of it)
                                const int gt = Z0 + it.k;
                                int bt = (int)((float)gt * B.inv_bf2);
                                bt -= bt * B.bf[2] > gt ? 1 : 0;
                                bt += (bt + 1) * B.bf[2] <= gt ? 1 : 0;
                                const int sl = slotp[__float_as_int(tx[S + 1]) + __float_as_int(ty[2 * S]) + bt];
                                if (sl >= 0 && acc != 0.0f)
                                    unsafeAtomicAdd(B.blocks + (int64_t)sl * B.vblk +
                                                        (__float_as_int(tx[S + 2]) + __float_as_int(ty[2 * S + 1]) +
                                                         (gt - bt * B.bf[2])),
                                                    acc);
                            } else {
                                vd[((X0 + it.i - F0[0]) * FY + (Y0 + it.j - F0[1])) * FT + (Z0 + it.k - F0[2])] = acc;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
        if (charge_sum) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) nsum += __shfl_down(nsum, o, kWave);
            if ((tid & 63) == 0) red[tid >> 6] = nsum;
            __syncthreads();
            if (tid == 0) {
                double tsum = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) tsum += red[w];
                atomicAdd(charge_sum, tsum);
            }
            __syncthreads();
        }
    }
}

// Gauss-Legendre rule by Newton iteration on P_n (three-term recurrence).
void gl_rule(int n, double* xi, double* w) {
    for (int i = 0; i < n; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double p = 0, pm = 0, dp = 0;
        for (int it = 0; it < 100; ++it) {
            p = 1.0;
            pm = 0.0;
            for (int k = 0; k < n; ++k) {
                double pn = ((2.0 * k + 1.0) * x * p - k * pm) / (k + 1.0);
                pm = p;
                p = pn;
            }
            dp = n * (pm - x * p) / (1.0 - x * x);
            double dx = p / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        p = 1.0;
        pm = 0.0;
        for (int k = 0; k < n; ++k) {
            double pn = ((2.0 * k + 1.0) * x * p - k * pm) / (k + 1.0);
            pm = p;
            p = pn;
        }
        dp = n * (pm - x * p) / (1.0 - x * x);
        xi[n - 1 - i] = x;
        w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

template <int NGL, bool BIN>
void launch_effq(const EffqParams& P, int64_t n_dep, const float* seg, const int32_t* fp,
                 const int64_t* off, float* val, int64_t val_cap, double* cs, const EffqBins& B,
                 hipStream_t st) {
    // LDS floats of a tile: at least the tables and window columns of one x-y cell and
    // its neighbours, one tick each, and their sliding state
    constexpr int S = NGL + 2 * (NGL / 2);
    constexpr int TX = (S + 1 + 3) / 4 * 4, TY = 2 * S + (BIN ? 2 : 0);
    constexpr int CMIN = 9 * NGL * NGL * (NGL + NGL / 2) + 3 * NGL * (3 * NGL + 1) + TX + TY + 2 * S;
    constexpr int CAP = TRED_EFFQ_CAP > CMIN ? TRED_EFFQ_CAP : CMIN;
    constexpr int NT = TRED_EFFQ_NT;
    int64_t grid = n_dep < (1 << 20) ? n_dep : (1 << 20);
    hipLaunchKernelGGL((k_effq<NGL, CAP, NT, BIN>), dim3((unsigned)grid), dim3(NT), 0, st, P, n_dep,
                       seg, fp, off, val, val_cap, cs, B);
}

// kernel parameters of the rule with n_gl nodes: nodes, weights and the stencil
// weights u of one grid point (nodes with xi > 0 of cell g-1 (weight |xi|/2), all
// nodes of cell g (1 - |xi|/2), nodes with xi < 0 of cell g+1 (|xi|/2))
EffqParams effq_params(const tred_grid* grid, const tred_physics* phys) {
    EffqParams P;
    P.g = *grid;
    P.ph = *phys;
    double xi[8], w[8];
    const int n = phys->n_gl;
    gl_rule(n, xi, w);
    for (int i = 0; i < 8; ++i) {
        P.xi[i] = i < n ? (float)xi[i] : 0.f;
        P.w[i] = i < n ? (float)w[i] : 0.f;
    }
    const int npos = n / 2;
    int k = 0;
    for (int l = n - npos; l < n; ++l) P.u[k++] = (float)(std::fabs(xi[l]) / 2.0);
    for (int l = 0; l < n; ++l) P.u[k++] = (float)(1.0 - std::fabs(xi[l]) / 2.0);
    for (int l = 0; l < npos; ++l) P.u[k++] = (float)(std::fabs(xi[l]) / 2.0);
    for (; k < 16; ++k) P.u[k] = 0.f;
    return P;
}

template <bool BIN>
void launch_effq_rule(const EffqParams& P, int64_t n_dep, const float* seg, const int32_t* fp,
                      const int64_t* off, float* val, int64_t val_cap, double* cs,
                      const EffqBins& B, hipStream_t st) {
    switch (P.ph.n_gl) {
        case 1: launch_effq<1, BIN>(P, n_dep, seg, fp, off, val, val_cap, cs, B, st); break;
        case 2: launch_effq<2, BIN>(P, n_dep, seg, fp, off, val, val_cap, cs, B, st); break;
        case 3: launch_effq<3, BIN>(P, n_dep, seg, fp, off, val, val_cap, cs, B, st); break;
        case 4: launch_effq<4, BIN>(P, n_dep, seg, fp, off, val, val_cap, cs, B, st); break;
        case 5: launch_effq<5, BIN>(P, n_dep, seg, fp, off, val, val_cap, cs, B, st); break;
        case 6: launch_effq<6, BIN>(P, n_dep, seg, fp, off, val, val_cap, cs, B, st); break;
        case 7: launch_effq<7, BIN>(P, n_dep, seg, fp, off, val, val_cap, cs, B, st); break;
        default: launch_effq<8, BIN>(P, n_dep, seg, fp, off, val, val_cap, cs, B, st); break;
    }
}

// waves per SIMD the effective-charge gradient is compiled for (register bound)
#ifndef TRED_EFFQ_ADJ_WAVES
#define TRED_EFFQ_ADJ_WAVES 2
#endif

// ---------------------------------------------------------------------------
// Gradient of the effective charge (Sec. V-C), in closed form. The node charge is
// q = Qp g(r, D, sigma) with r the node's offset from the segment start (from the
// midpoint for a point charge), D the segment vector and sigma the widths. With
// I_a = 1 / sigma_a^2, alpha = sum D_a^2 I_a, s = (sum r_a D_a I_a) / alpha the
// parameter of the closest point, p = r - s D the offset from it, k = sqrt(alpha / 2)
// and the erf limits A = -k s, B = k (1 - s), the line charge is
//   g = N (erf B - erf A),  N = exp(-sum p_a^2 I_a / 2) / (4 pi sigma_x sigma_y sigma_t sqrt(alpha)).
// Differentiating through alpha, s and the limits, with gA, gB the erf derivatives
// (2 / sqrt(pi)) exp(-A^2), exp(-B^2), phi = N k (gB - gA) / alpha and
// psi = N (gB (1 - s) + gA s) / (2 k):
//   dg/dr_a     = I_a (-g p_a - phi D_a)
//   dg/dD_a     = I_a ((g s - phi) p_a + (phi s + psi - g / alpha) D_a)
//   dg/dsigma_a = (I_a / sigma_a) (g p_a^2 + 2 phi p_a D_a + (g / alpha - psi) D_a^2) - g / sigma_a
// (point charge: phi = psi = 0, no alpha terms). The per-deposition factors (I_a, D_a,
// alpha, sigma_a) come out of the sums over nodes, so each node adds G_n w_n times
// g, g p_a, g p_a^2, g s p_a, phi, phi p_a, phi s and psi into sixteen binary64 sums,
// G_n = sum over the grid points c whose stencil holds n of u(c, n) dL/dV_c being the
// transposed trilinear spread. Writing the gradient in p rather than r keeps the terms
// of a long segment (|r| up to its length, |p| a few widths) free of cancellation.
// The sums then go through the chain rule of the transport (t = z / v, t_mid, the
// widths and Qp = Q exp(-t_mid / lifetime)) once per deposition.
// ---------------------------------------------------------------------------
template <int NGL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TRED_EFFQ_ADJ_WAVES))) void k_effq_adj(EffqParams P, int64_t n_dep,
                                                  const float* __restrict__ seg,
                                                  const int32_t* __restrict__ fp,
                                                  const int64_t* __restrict__ off,
                                                  const float* __restrict__ dval, int64_t val_cap,
                                                  float* __restrict__ dseg,
                                                  double* __restrict__ dphys) {
    constexpr int NT = 256, NW = NT / kWave;
    // sums over nodes: g, g p (3), g p^2 (3), g s p (3), phi, phi p (3), phi s, psi
    enum { SG = 0, SGP = 1, SGP2 = 4, SGSP = 7, SPHI = 10, SPHP = 11, SPHS = 14, SPSI = 15, NA = 16 };
    constexpr int CAPA = 12288;   // patch cells staged in LDS (larger patches read memory)
    __shared__ double red[NW][NA];
    __shared__ float sdv[CAPA];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const tred_grid& g = P.g;
    // Node j of a dual cell, for the ascending Gauss-Legendre nodes (the first NH
    // negative, the last NH positive, a middle one zero): j < NH lies in cell c + 1 at
    // xi_j, j >= NH in cell c. Offset from the centre of cell c in cell widths, and
    // spread weights onto c and c + 1 times the quadrature weight w_j.
    constexpr int NH = NGL / 2;
    __shared__ float stq[3][8];   // offset, weight onto c, weight onto c + 1 (x and y axes)
    float tqo[NGL], tq0[NGL], tq1[NGL];   // the same, in registers (t axis)
#pragma unroll
    for (int j = 0; j < NGL; ++j) {
        const float x = P.xi[j], wq = P.w[j], ax = 0.5f * fabsf(x);
        tqo[j] = j < NH ? 1.0f + 0.5f * x : 0.5f * x;
        tq0[j] = wq * (j < NH ? ax : 1.0f - ax);
        tq1[j] = wq * (j < NH ? 1.0f - ax : ax);
        if (tid == j) {
            stq[0][j] = tqo[j];
            stq[1][j] = tq0[j];
            stq[2][j] = tq1[j];
        }
    }
    __syncthreads();
    for (int64_t d = blockIdx.x; d < n_dep; d += gridDim.x) {
        const int32_t* f = fp + 6 * d;
        const int F0[3] = {f[0], f[1], f[2]}, F1[3] = {f[3], f[4], f[5]};
        const bool empty = F1[0] < F0[0] || F1[1] < F0[1] || F1[2] < F0[2] || off[d + 1] > val_cap;
        float s[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) s[k] = seg[7 * d + k];
        const Win W = window_f32(g, P.ph, s);
        // transport, as the forward kernel
        const double v = P.ph.v_drift;
        const double t0 = (double)s[2] / v, t1 = (double)s[5] / v;
        const double tm_raw = 0.5 * (t0 + t1);
        const double tm = tm_raw < 0.0 ? 0.0 : tm_raw;
        const double att = exp(-tm / (double)P.ph.lifetime);
        const double Qp = (double)s[6] * att;
        const double sT = sqrt(2.0 * (double)P.ph.diff_T * tm);
        const double sLr = sqrt(2.0 * (double)P.ph.diff_L * tm) / v;
        const bool fl[3] = {!(sT >= (double)P.ph.sigma_min[0]), !(sT >= (double)P.ph.sigma_min[1]),
                            !(sLr >= (double)P.ph.sigma_min[2])};
        const double sg[3] = {fl[0] ? (double)P.ph.sigma_min[0] : sT, fl[1] ? (double)P.ph.sigma_min[1] : sT,
                              fl[2] ? (double)P.ph.sigma_min[2] : sLr};
        const double h[3] = {g.spacing[0], g.spacing[1], g.spacing[2]};
        const double D[3] = {(double)s[3] - (double)s[0], (double)s[4] - (double)s[1], t1 - t0};
        double base[3];
        base[0] = (double)g.origin[0] + ((double)W.lo[0] + 0.5) * h[0] - (double)s[0];
        base[1] = (double)g.origin[1] + ((double)W.lo[1] + 0.5) * h[1] - (double)s[1];
        base[2] = (double)g.origin[2] + (double)W.lo[2] * h[2] - t0;
        const bool point = W.point != 0;
        // per-deposition factors in binary32, as the nodes use them
        float fb[3], fh[3], Df[3], Is[3];
        float alf = 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            fb[a] = (float)(point ? base[a] - 0.5 * D[a] : base[a]);
            fh[a] = (float)h[a];
            Df[a] = point ? 0.0f : (float)D[a];
            const float sf = (float)sg[a];
            Is[a] = 1.0f / (sf * sf);
            alf = fmaf(Df[a] * Df[a], Is[a], alf);
        }
        const double ssp = (double)(float)sg[0] * (double)(float)sg[1] * (double)(float)sg[2];
        // (2 pi)^(-3/2) / (sigma_x sigma_y sigma_t), or 1 / (4 pi sigma_x sigma_y sigma_t sqrt(alpha))
        const float pref = point ? (float)(0.0634936359342409697 / ssp)
                                 : (float)(0.0795774715459476679 / (ssp * sqrt((double)alf)));
        const float ial = point ? 0.0f : 1.0f / alf;
        const float kq = sqrtf(0.5f * alf);
        const float kia = kq * ial, hik = point ? 0.0f : 0.5f / kq;
        const double jac = h[0] * h[1] * h[2] / 8.0;   // node volume, applied to the sums
        // Dual cells: the nodes between grid points c and c + 1 of an axis (those of cell
        // c with xi >= 0 and those of cell c + 1 with xi < 0) spread onto c and c + 1
        // only, so a dual cell reads the patch gradient at 2 x 2 x 2 grid points and the
        // transposed spread of its nodes is separable. Dual cells c = F0 - 1 .. F1 hold
        // every node whose spread reaches the footprint.
        int nd[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) nd[a] = empty ? 0 : F1[a] - F0[a] + 2;
        const int FY = F1[1] - F0[1] + 1, FTt = F1[2] - F0[2] + 1;
        const int ostr[3] = {FY * FTt, FTt, 1};
        const float* dv = dval + (empty ? 0 : off[d]);
        const int64_t cnt = empty ? 0 : off[d + 1] - off[d];
        const bool staged = cnt <= CAPA;
        if (staged) {
            for (int64_t k = tid; k < cnt; k += NT) sdv[k] = dv[k];
            __syncthreads();
        }
        double acc[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) acc[k] = 0.0;
        float ot[NGL];   // node offsets along t (from the centre of cell c)
#pragma unroll
        for (int j = 0; j < NGL; ++j) ot[j] = tqo[j] * fh[2];
        const int64_t total = (int64_t)nd[0] * nd[1] * nd[2];
        Idx3 itc;
        itc.init(tid, NT, max(nd[1], 1), max(nd[2], 1));
        auto run = [&](auto node) {
            for (int64_t i = tid; i < total; i += NT, itc.next()) {
                const int c[3] = {F0[0] - 1 + itc.i, F0[1] - 1 + itc.j, F0[2] - 1 + itc.k};
                // patch gradient at c and c + 1 per axis (zero outside the footprint)
                int o[3][2];
                bool v[3][2], wl[3][2];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    v[a][0] = c[a] >= F0[a];
                    v[a][1] = c[a] + 1 <= F1[a];
                    o[a][0] = v[a][0] ? (c[a] - F0[a]) * ostr[a] : 0;
                    o[a][1] = v[a][1] ? (c[a] + 1 - F0[a]) * ostr[a] : 0;
                    // nodes j >= NH lie in cell c, nodes j < NH in cell c + 1; either
                    // cell may lie outside the quadrature window
                    wl[a][0] = c[a] >= W.lo[a] && c[a] <= W.hi[a];
                    wl[a][1] = c[a] + 1 >= W.lo[a] && c[a] + 1 <= W.hi[a];
                }
                float Dv[2][2][2];
#pragma unroll
                for (int bx = 0; bx < 2; ++bx)
#pragma unroll
                    for (int by = 0; by < 2; ++by)
#pragma unroll
                        for (int bt = 0; bt < 2; ++bt) {
                            const bool ok = v[0][bx] && v[1][by] && v[2][bt];
                            const int at = o[0][bx] + o[1][by] + o[2][bt];
                            const float x = staged ? sdv[at] : dv[at];
                            Dv[bx][by][bt] = ok ? x : 0.0f;
                        }
                // spread weights along t folded in: St[bx][by][jt]
                float St[2][2][NGL];
#pragma unroll
                for (int jt = 0; jt < NGL; ++jt) {
                    const bool okt = jt < NH ? wl[2][1] : wl[2][0];
                    const float a0 = okt ? tq0[jt] : 0.0f, a1 = okt ? tq1[jt] : 0.0f;
#pragma unroll
                    for (int bx = 0; bx < 2; ++bx)
#pragma unroll
                        for (int by = 0; by < 2; ++by)
                            St[bx][by][jt] = fmaf(a0, Dv[bx][by][0], a1 * Dv[bx][by][1]);
                }
                const float rbx = fb[0] + (float)(c[0] - W.lo[0]) * fh[0];
                const float rby = fb[1] + (float)(c[1] - W.lo[1]) * fh[1];
                const float rbt = fb[2] + (float)(c[2] - W.lo[2]) * fh[2];
#pragma unroll 1
                for (int jx = 0; jx < NGL; ++jx) {
                    const bool okx = jx < NH ? wl[0][1] : wl[0][0];
                    const float ax0 = okx ? stq[1][jx] : 0.0f, ax1 = okx ? stq[2][jx] : 0.0f;
                    const float rx = fmaf(stq[0][jx], fh[0], rbx);
                    // binary32 sums over the NGL^2 nodes of this x slice
                    float fs[NA];
#pragma unroll
                    for (int k = 0; k < NA; ++k) fs[k] = 0.0f;
#pragma unroll 1
                    for (int jy = 0; jy < NGL; ++jy) {
                        const bool oky = jy < NH ? wl[1][1] : wl[1][0];
                        const float ay0 = oky ? stq[1][jy] : 0.0f, ay1 = oky ? stq[2][jy] : 0.0f;
                        const float ry = fmaf(stq[0][jy], fh[1], rby);
                        const float w00 = ax0 * ay0, w01 = ax0 * ay1, w10 = ax1 * ay0, w11 = ax1 * ay1;
#pragma unroll
                        for (int jt = 0; jt < NGL; ++jt) {
                            const float w = fmaf(w00, St[0][0][jt],
                                                 fmaf(w01, St[0][1][jt], fmaf(w10, St[1][0][jt], w11 * St[1][1][jt])));
                            const float r[3] = {rx, ry, rbt + ot[jt]};
                            node(w, r, fs);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < NA; ++k) acc[k] += (double)fs[k];
                }
            }
        };
        if (point) {
            run([&](float w, const float* r, float* fs) {
                const float e = r[0] * r[0] * Is[0] + r[1] * r[1] * Is[1] + r[2] * r[2] * Is[2];
                const float wg = w * (pref * exp_neg(-0.5f * e));
                fs[SG] += wg;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    fs[SGP + a] = fmaf(wg, r[a], fs[SGP + a]);
                    fs[SGP2 + a] = fmaf(wg * r[a], r[a], fs[SGP2 + a]);
                }
            });
        } else {
            run([&](float w, const float* r, float* fs) {
                const float sst = (r[0] * Df[0] * Is[0] + r[1] * Df[1] * Is[1] + r[2] * Df[2] * Is[2]) * ial;
                float p[3], e = 0.0f;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    p[a] = r[a] - sst * Df[a];
                    e = fmaf(p[a] * p[a], Is[a], e);
                }
                const float N = pref * exp_neg(-0.5f * e);
                const float A1 = -kq * sst, B1 = kq - kq * sst;
                const float gb = 1.12837916709551257f * exp_neg(-B1 * B1);   // 2 / sqrt(pi)
                const float ga = 1.12837916709551257f * exp_neg(-A1 * A1);
                const float wg = w * (N * erf_diff(B1, A1));
                const float wph = w * (N * (gb - ga) * kia);
                const float wps = w * (N * fmaf(gb, 1.0f - sst, ga * sst) * hik);
                fs[SG] += wg;
                fs[SPHI] += wph;
                fs[SPHS] = fmaf(wph, sst, fs[SPHS]);
                fs[SPSI] += wps;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    fs[SGP + a] = fmaf(wg, p[a], fs[SGP + a]);
                    fs[SGP2 + a] = fmaf(wg * p[a], p[a], fs[SGP2 + a]);
                    fs[SGSP + a] = fmaf(wg * sst, p[a], fs[SGSP + a]);
                    fs[SPHP + a] = fmaf(wph, p[a], fs[SPHP + a]);
                }
            });
        }
        // workgroup reduction of the sums
#pragma unroll
        for (int k = 0; k < NA; ++k) {
            double x = acc[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
            if (lane == 0) red[wave][k] = x;
        }
        __syncthreads();
        if (tid < NA) {   // thread k totals sum k over the waves (in place, column k)
            double x = red[0][tid];
            for (int w = 1; w < NW; ++w) x += red[w][tid];
            red[0][tid] = x * jac;
        }
        __syncthreads();
        if (tid == 0) {
            double S[NA];
#pragma unroll
            for (int k = 0; k < NA; ++k) S[k] = red[0][k];
            // A[0..2]: d/dr, A[3..5]: d/dD, A[6..8]: d/dsigma (each times Qp), A[9]: d/dQp
            double A[10];
            const double sgS = S[SG], ia = point ? 0.0 : 1.0 / (double)alf;
            for (int a = 0; a < 3; ++a) {
                const double I = (double)Is[a], Da = (double)Df[a], sa = (double)(float)sg[a];
                A[a] = Qp * I * (-S[SGP + a] - Da * S[SPHI]);
                A[3 + a] = Qp * I * (S[SGSP + a] - S[SPHP + a] + Da * (S[SPHS] + S[SPSI] - sgS * ia));
                A[6 + a] = Qp * ((I / sa) * (S[SGP2 + a] + 2.0 * Da * S[SPHP + a] +
                                             Da * Da * (sgS * ia - S[SPSI])) - sgS / sa);
            }
            A[9] = sgS;
            double dP0[3], dP1[3];
            for (int a = 0; a < 3; ++a) {
                if (point) {
                    dP0[a] = -0.5 * A[a];
                    dP1[a] = -0.5 * A[a];
                } else {
                    dP0[a] = -A[a] - A[3 + a];
                    dP1[a] = A[3 + a];
                }
            }
            const double tau = P.ph.lifetime, DT = P.ph.diff_T, DL = P.ph.diff_L;
            const double dsx = fl[0] || sT <= 0.0 ? 0.0 : DT / sT;
            const double dsy = fl[1] || sT <= 0.0 ? 0.0 : DT / sT;
            const double dst = fl[2] || sLr <= 0.0 ? 0.0 : DL / (v * v * sLr);
            const double dtm = tm_raw < 0.0 ? 0.0 : 0.5;   // d t_mid / d t0 = d t_mid / d t1
            const double Stm = A[6] * dsx + A[7] * dsy + A[8] * dst - A[9] * Qp / tau;
            dP0[2] += dtm * Stm;
            dP1[2] += dtm * Stm;
            float* o = dseg + 7 * d;
            o[0] = empty ? 0.f : (float)dP0[0];
            o[1] = empty ? 0.f : (float)dP0[1];
            o[2] = empty ? 0.f : (float)(dP0[2] / v);
            o[3] = empty ? 0.f : (float)dP1[0];
            o[4] = empty ? 0.f : (float)dP1[1];
            o[5] = empty ? 0.f : (float)(dP1[2] / v);
            o[6] = empty ? 0.f : (float)(A[9] * att);
            if (dphys && !empty) {
                const double gT = (fl[0] || sT <= 0.0 ? 0.0 : A[6] * tm / sT) +
                                  (fl[1] || sT <= 0.0 ? 0.0 : A[7] * tm / sT);
                const double gL = fl[2] || sLr <= 0.0 ? 0.0 : A[8] * tm / (v * v * sLr);
                const double gTau = A[9] * Qp * tm / (tau * tau);
                atomicAdd(dphys + 0, gT);
                atomicAdd(dphys + 1, gL);
                atomicAdd(dphys + 2, gTau);
            }
        }
        __syncthreads();
    }
}

}  // namespace

extern "C" tred_status tred_effq_windows(const tred_grid* grid, const tred_physics* phys,
                                         int64_t n_dep, const float* seg, int32_t* fp,
                                         int64_t* off, void* stream) {
    TRED_TRY(validate_grid(grid));
    TRED_TRY(validate_physics(phys));
    TRED_REQUIRE(n_dep >= 0, "n_dep must be >= 0");
    TRED_REQUIRE(off != nullptr, "off is NULL");
    TRED_REQUIRE(n_dep == 0 || (seg != nullptr && fp != nullptr), "seg/fp is NULL");
    hipStream_t st = (hipStream_t)stream;
    int64_t nb = (n_dep + 255) / 256;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_windows, dim3((unsigned)nb), dim3(256), 0, st, *grid, *phys, n_dep, seg,
                       fp, off);
    TRED_TRY(tred_check_launch("tred_effq_windows"));
    if (n_dep > 0) {
        hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, st, off, n_dep);
        TRED_TRY(tred_check_launch("tred_effq_windows scan"));
    }
    return TRED_OK;
}

extern "C" tred_status tred_effq_adjoint(const tred_grid* grid, const tred_physics* phys,
                                         int64_t n_dep, const float* seg, const int32_t* fp,
                                         const int64_t* off, const float* d_val, int64_t val_cap,
                                         float* d_seg, double* d_phys, void* stream) {
    TRED_TRY(validate_grid(grid));
    TRED_TRY(validate_physics(phys));
    TRED_REQUIRE(phys->point_frac > 0.0f, "physics.point_frac must be > 0 for the line form");
    TRED_REQUIRE(n_dep >= 0, "n_dep must be >= 0");
    TRED_REQUIRE(val_cap >= 0, "val_cap must be >= 0");
    if (n_dep == 0) return TRED_OK;
    TRED_REQUIRE(seg && fp && off && d_seg, "seg/fp/off/d_seg is NULL");
    TRED_REQUIRE(d_val != nullptr || val_cap == 0, "d_val is NULL");
    EffqParams P;
    P.g = *grid;
    P.ph = *phys;
    double xi[8], w[8];
    const int n = phys->n_gl;
    gl_rule(n, xi, w);
    for (int i = 0; i < 8; ++i) {
        P.xi[i] = i < n ? (float)xi[i] : 0.f;
        P.w[i] = i < n ? (float)w[i] : 0.f;
    }
    for (int k = 0; k < 16; ++k) P.u[k] = 0.f;
    hipStream_t st = (hipStream_t)stream;
    const unsigned nb = (unsigned)std::min<int64_t>(n_dep, 1 << 20);
    auto launch = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, st, P, n_dep, seg, fp, off, d_val, val_cap,
                           d_seg, d_phys);
    };
    switch (n) {
        case 1: launch(k_effq_adj<1>); break;
        case 2: launch(k_effq_adj<2>); break;
        case 3: launch(k_effq_adj<3>); break;
        case 4: launch(k_effq_adj<4>); break;
        case 5: launch(k_effq_adj<5>); break;
        case 6: launch(k_effq_adj<6>); break;
        case 7: launch(k_effq_adj<7>); break;
        default: launch(k_effq_adj<8>); break;
    }
    return tred_check_launch("tred_effq_adjoint");
}

extern "C" tred_status tred_effq(const tred_grid* grid, const tred_physics* phys, int64_t n_dep,
                                 const float* seg, const int32_t* fp, const int64_t* off,
                                 float* val, int64_t val_cap, double* charge_sum, void* stream) {
    TRED_TRY(validate_grid(grid));
    TRED_TRY(validate_physics(phys));
    TRED_REQUIRE(phys->point_frac > 0.0f, "physics.point_frac must be > 0 for the line form");
    TRED_REQUIRE(n_dep >= 0, "n_dep must be >= 0");
    TRED_REQUIRE(val_cap >= 0, "val_cap must be >= 0");
    if (n_dep == 0) return TRED_OK;
    TRED_REQUIRE(seg && fp && off, "seg/fp/off is NULL");
    TRED_REQUIRE(val != nullptr || val_cap == 0, "val is NULL");
    const EffqParams P = effq_params(grid, phys);
    launch_effq_rule<false>(P, n_dep, seg, fp, off, val, val_cap, charge_sum, EffqBins{},
                            (hipStream_t)stream);
    return tred_check_launch("tred_effq");
}

// (the binning has laid out the bins: slot map, zeroed rows; validated by the caller)
tred_status effq_into_bins(const tred_grid* grid, const tred_physics* phys, int64_t n_dep,
                           const float* seg, const int32_t* fp, const EffqBins& B,
                           double* charge_sum, hipStream_t st) {
    if (n_dep == 0) return TRED_OK;
    const EffqParams P = effq_params(grid, phys);
    launch_effq_rule<true>(P, n_dep, seg, fp, nullptr, nullptr, 0, charge_sum, B, st);
    return tred_check_launch("effective charge into the bins");
}

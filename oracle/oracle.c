/*
 * FP64 CPU oracle for the pixel-TPC signal-formation hot path.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference against which
 * the GPU library is checked. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it. It shares no code, header, table or
 * helper with the GPU library.
 *
 * Every function follows the paper (arXiv 2602.12052) step by step, in its
 * notation, and cites the section / equation it implements:
 *   - transport:            Sec. II-A (drift, attachment, diffusion), Sec. II-C
 *   - Gauss-Legendre rule:  Sec. II-C (N-point rule on [-1,1])
 *   - line charge q(x):     Sec. II-C, eq. (qline), with exponent -B/(2 Delta^2)
 *   - point charge:         Sec. II-C, short-segment limit
 *   - effective charge:     Sec. II-C, eqs. (cub), (trilinear), (eff_q)
 *   - block-sparse binning: Sec. III-B (block-sparse binned tensor)
 *   - induced current:      Sec. II-D, eq. (interlaced) with eq. (firstapprox);
 *                           computed as a direct (non-FFT) sum.
 *
 * Discrete decisions (window bounds, point-like switch) are replayed in IEEE
 * binary32 with correctly rounded + - * / sqrt and no contraction (this file
 * must be compiled with -ffp-contract=off), so that integer outputs are unique.
 * Everything else is binary64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    float origin[3];   /* x, y of lower edge of pixel (0,0) [cm]; t of tick 0 [us] */
    float spacing[3];  /* h_x, h_y [cm]; tick [us] */
    int32_t npix[2];
    int32_t sub[2];
    int32_t nticks;
} o_grid;

typedef struct {
    float v_drift;      /* cm/us */
    float lifetime;     /* us */
    float diff_T;       /* cm^2/us */
    float diff_L;       /* cm^2/us */
    float sigma_min[3]; /* cm, cm, us */
    float n_sigma;
    float point_frac;
    int32_t n_gl;
} o_physics;

typedef struct {
    int32_t blk_pix[2];
    int32_t blk_ticks;
} o_blocking;

static int o_nfine(const o_grid* g, int a) {
    return a == 0 ? g->npix[0] * g->sub[0] : a == 1 ? g->npix[1] * g->sub[1] : g->nticks;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule (Sec. II-C): nodes xi_i and weights w_i of the N-point
 * rule on [-1, 1], from Newton iteration on the Legendre polynomial P_N using
 * the three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.
 * Weights w_i = 2 / ((1 - xi^2) P_N'(xi)^2). Nodes returned ascending.       */
int oracle_gl_rule(int n, double* xi, double* w) {
    if (n < 1 || n > 64) return 1;
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double pn = 0.0, pnm1 = 0.0, dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            /* P_N(x) and P_{N-1}(x) by the recurrence */
            pnm1 = 1.0;
            pn = x;
            for (int k = 1; k < n; ++k) {
                double pnext = ((2.0 * k + 1.0) * x * pn - k * pnm1) / (k + 1.0);
                pnm1 = pn;
                pn = pnext;
            }
            if (n == 1) { pn = x; pnm1 = 1.0; }
            /* P_N'(x) = N (x P_N - P_{N-1}) / (x^2 - 1) */
            dp = n * (x * pn - pnm1) / (x * x - 1.0);
            double dx = pn / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        pnm1 = 1.0;
        pn = x;
        for (int k = 1; k < n; ++k) {
            double pnext = ((2.0 * k + 1.0) * x * pn - k * pnm1) / (k + 1.0);
            pnm1 = pn;
            pn = pnext;
        }
        dp = n * (x * pn - pnm1) / (x * x - 1.0);
        xi[n - 1 - i] = x; /* cos(...) decreases with i: store ascending */
        w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Transport (Sec. II-A; one diffusion width per axis per segment, Sec. II-C).
 * Drift time t = z / v. Attachment: the whole segment is attenuated by
 * exp(-t_mid / tau_e) at its mid drift time. Diffusion: sigma_T = sqrt(2 D_T t_mid),
 * sigma_t = sqrt(2 D_L t_mid) / v, each floored at the minimum diffusion scale
 * (Sec. V-A). out = { t0, t1, t_mid, Q', sigma_x, sigma_y, sigma_t }.        */
void oracle_transport(const o_physics* ph, const float* seg, double* out) {
    double v = ph->v_drift;
    double t0 = (double)seg[2] / v, t1 = (double)seg[5] / v;
    double tm = 0.5 * (t0 + t1);
    if (tm < 0.0) tm = 0.0;
    double q = (double)seg[6] * exp(-tm / (double)ph->lifetime);
    double sT = sqrt(2.0 * (double)ph->diff_T * tm);
    double sL = sqrt(2.0 * (double)ph->diff_L * tm) / v;
    out[0] = t0;
    out[1] = t1;
    out[2] = tm;
    out[3] = q;
    out[4] = fmax(sT, (double)ph->sigma_min[0]);
    out[5] = fmax(sT, (double)ph->sigma_min[1]);
    out[6] = fmax(sL, (double)ph->sigma_min[2]);
}

/* ------------------------------------------------------------------------ */
/* Discrete decisions in binary32 (integer outputs must be unique).
 * Window per axis: grid coordinate u = (P - o)/h of each endpoint (for time,
 * u = (t - origin_t)/tick + 1/2 so that cell n covers [(n-1/2), (n+1/2)) ticks),
 * lo = floor(min(u0,u1) - n_sigma*sigma/h), hi = floor(max(u0,u1) + n_sigma*sigma/h).
 * Point-like switch (Sec. II-C): all |p1 - p0| components < point_frac * sigma.    */
static int32_t o_floor_to_int(float v) {
    float f = floorf(v);
    if (f < -16777216.0f) f = -16777216.0f;
    if (f > 16777216.0f) f = 16777216.0f;
    return (int32_t)f;
}

void oracle_window_f32(const o_grid* g, const o_physics* ph, const float* seg,
                       int32_t* lo, int32_t* hi, int32_t* is_point) {
    float v = ph->v_drift;
    float t0 = seg[2] / v;
    float t1 = seg[5] / v;
    float tm = (t0 + t1) * 0.5f;
    if (tm < 0.0f) tm = 0.0f;
    float vT = (2.0f * ph->diff_T) * tm;
    float sT = sqrtf(vT);
    float s[3];
    s[0] = fmaxf(sT, ph->sigma_min[0]);
    s[1] = fmaxf(sT, ph->sigma_min[1]);
    float vL = (2.0f * ph->diff_L) * tm;
    float sL = sqrtf(vL) / v;
    s[2] = fmaxf(sL, ph->sigma_min[2]);
    float P0[3] = {seg[0], seg[1], t0};
    float P1[3] = {seg[3], seg[4], t1};
    for (int a = 0; a < 3; ++a) {
        float h = g->spacing[a];
        float u0, u1;
        if (a < 2) {
            u0 = (P0[a] - g->origin[a]) / h;
            u1 = (P1[a] - g->origin[a]) / h;
        } else {
            u0 = (P0[a] - g->origin[a]) / h + 0.5f;
            u1 = (P1[a] - g->origin[a]) / h + 0.5f;
        }
        float e = ph->n_sigma * (s[a] / h);
        float umin = u0 < u1 ? u0 : u1;
        float umax = u0 < u1 ? u1 : u0;
        lo[a] = o_floor_to_int(umin - e);
        hi[a] = o_floor_to_int(umax + e);
    }
    int pt = 1;
    for (int a = 0; a < 3; ++a) {
        float d = fabsf(P1[a] - P0[a]);
        if (!(d < ph->point_frac * s[a])) pt = 0;
    }
    *is_point = pt;
}

/* Footprint of the effective charge: window dilated by the one-cell trilinear
 * stencil (Sec. II-C, eq. trilinear), cropped to the region. fp = lo[3], hi[3]
 * inclusive (lo > hi on some axis means empty). Returns the cell count.     */
int64_t oracle_footprint(const o_grid* g, const o_physics* ph, const float* seg, int32_t* fp,
                         int32_t* is_point) {
    int32_t lo[3], hi[3];
    oracle_window_f32(g, ph, seg, lo, hi, is_point);
    int64_t vol = 1;
    for (int a = 0; a < 3; ++a) {
        int32_t N = o_nfine(g, a);
        int32_t l = lo[a] - 1, h = hi[a] + 1;
        if (l < 0) l = 0;
        if (h > N - 1) h = N - 1;
        fp[a] = l;
        fp[3 + a] = h;
        if (h < l) vol = 0;
        else vol *= (int64_t)(h - l + 1);
    }
    return vol;
}

/* All depositions: footprints, point flags and exclusive prefix sum of volumes. */
void oracle_footprints(const o_grid* g, const o_physics* ph, int64_t n, const float* seg,
                       int32_t* fp, int64_t* off, int32_t* is_point) {
    off[0] = 0;
    for (int64_t d = 0; d < n; ++d) {
        int64_t vol = oracle_footprint(g, ph, seg + 7 * d, fp + 6 * d, is_point + d);
        off[d + 1] = off[d] + vol;
    }
}

/* ------------------------------------------------------------------------ */
/* Difference erf(b) - erf(a), using erfc when both arguments share a sign so
 * that tails do not cancel.                                                 */
static double o_erf_diff(double b, double a) {
    if (a >= 0.0 && b >= 0.0) return erfc(a) - erfc(b);
    if (a <= 0.0 && b <= 0.0) return erfc(-b) - erfc(-a);
    return erf(b) - erf(a);
}

/* Line-charge density, Sec. II-C eq. (qline): a uniform line charge Q from p0 to
 * p1 convolved with an anisotropic Gaussian (sigma_x, sigma_y, sigma_z), in the
 * paper's notation (Delta^2, A1, A2, B); the drift coordinate z is time here.
 * The exponent is -B/(2 Delta^2): the printed -B/Delta^2 lacks the factor 1/2
 * that the derivation (and the paper's own symbolic form) carries.           */
double oracle_q_line(double x, double y, double z, const double* p0, const double* p1,
                     const double* sig, double Q) {
    double x0 = p0[0], y0 = p0[1], z0 = p0[2];
    double x1 = p1[0], y1 = p1[1], z1 = p1[2];
    double sx2 = sig[0] * sig[0], sy2 = sig[1] * sig[1], sz2 = sig[2] * sig[2];
    double D2 = sy2 * sz2 * (x0 - x1) * (x0 - x1) + sz2 * sx2 * (y0 - y1) * (y0 - y1) +
                sx2 * sy2 * (z0 - z1) * (z0 - z1);
    double D = sqrt(D2);
    double A1 = sy2 * sz2 * (x - x0) * (x0 - x1) + sz2 * sx2 * (y - y0) * (y0 - y1) +
                sx2 * sy2 * (z - z0) * (z0 - z1);
    double A2 = sy2 * sz2 * (x - x1) * (x0 - x1) + sz2 * sx2 * (y - y1) * (y0 - y1) +
                sx2 * sy2 * (z - z1) * (z0 - z1);
    double b1 = x * (z0 - z1) + (z1 * x0 - z0 * x1) - z * (x0 - x1);
    double b2 = y * (x0 - x1) + (x1 * y0 - x0 * y1) - x * (y0 - y1);
    double b3 = y * (z0 - z1) + (z1 * y0 - z0 * y1) - z * (y0 - y1);
    double B = sy2 * b1 * b1 + sz2 * b2 * b2 + sx2 * b3 * b3;
    double kappa = sqrt(2.0) * D * sig[0] * sig[1] * sig[2];
    return Q * exp(-B / (2.0 * D2)) / (4.0 * M_PI * D) * o_erf_diff(A2 / kappa, A1 / kappa);
}

/* Point-like limit of eq. (qline) (Sec. II-C, short segments): a Gaussian of
 * total charge Q centred at the segment midpoint m.                          */
double oracle_q_point(double x, double y, double z, const double* m, const double* sig,
                      double Q) {
    double ex = (x - m[0]) / sig[0], ey = (y - m[1]) / sig[1], ez = (z - m[2]) / sig[2];
    return Q * pow(2.0 * M_PI, -1.5) / (sig[0] * sig[1] * sig[2]) *
           exp(-0.5 * (ex * ex + ey * ey + ez * ez));
}

/* Ionization charge density of one deposition after transport, at (x, y, t). */
double oracle_q_seg(const o_physics* ph, const float* seg, double x, double y, double t) {
    double tr[7];
    oracle_transport(ph, seg, tr);
    int32_t lo[3], hi[3], ipt;
    /* the point/line choice is a discrete decision: binary32 replay */
    o_grid dummy;
    memset(&dummy, 0, sizeof dummy);
    dummy.spacing[0] = dummy.spacing[1] = dummy.spacing[2] = 1.0f;
    oracle_window_f32(&dummy, ph, seg, lo, hi, &ipt);
    double p0[3] = {seg[0], seg[1], tr[0]};
    double p1[3] = {seg[3], seg[4], tr[1]};
    double sig[3] = {tr[4], tr[5], tr[6]};
    if (ipt) {
        double m[3] = {0.5 * (p0[0] + p1[0]), 0.5 * (p0[1] + p1[1]), tr[2]};
        return oracle_q_point(x, y, t, m, sig, tr[3]);
    }
    return oracle_q_line(x, y, t, p0, p1, sig, tr[3]);
}

/* ------------------------------------------------------------------------ */
/* Effective charge of one deposition (Sec. II-C, eqs. cub, trilinear, eff_q).
 *
 * Cells C of the window [lo, hi] (the cuboids of the fine grid, centred on grid
 * points: x_i = origin_x + (i + 1/2) h_x, t_n = origin_t + n * tick) each carry
 * n_gl^3 Gauss-Legendre nodes at centre + xi * h / 2 per axis, with weight
 * w_l w_m w_n * (h_x/2)(h_y/2)(tick/2) (the rule mapped from [-1,1] to the cell).
 * The node charge w * q(node) is spread to grid points by the trilinear
 * interpolation coefficients u of the node inside the cell: along each axis the
 * node at xi gives 1 - |xi|/2 to the cell's own grid point and |xi|/2 to the
 * neighbour on the node's side; the 3-D coefficient is the product.
 * Targets outside the region are dropped.
 *
 * val: the deposition's footprint box fp (x-major, then y, then t fastest).
 * node_sum (optional): the sum of w*q over all evaluated nodes.
 * Returns 0.                                                                 */
int oracle_effq_patch(const o_grid* g, const o_physics* ph, const float* seg, const int32_t* fp,
                      double* val, double* node_sum) {
    int32_t lo[3], hi[3], ipt;
    oracle_window_f32(g, ph, seg, lo, hi, &ipt);
    double tr[7];
    oracle_transport(ph, seg, tr);
    double p0[3] = {seg[0], seg[1], tr[0]};
    double p1[3] = {seg[3], seg[4], tr[1]};
    double sig[3] = {tr[4], tr[5], tr[6]};
    double mid[3] = {0.5 * (p0[0] + p1[0]), 0.5 * (p0[1] + p1[1]), tr[2]};
    double xi[64], w[64];
    int n = ph->n_gl;
    oracle_gl_rule(n, xi, w);
    double h[3] = {g->spacing[0], g->spacing[1], g->spacing[2]};
    double jac = (h[0] / 2.0) * (h[1] / 2.0) * (h[2] / 2.0);
    int32_t F0[3] = {fp[0], fp[1], fp[2]};
    int32_t F1[3] = {fp[3], fp[4], fp[5]};
    int64_t ny = (int64_t)(F1[1] - F0[1] + 1), nt = (int64_t)(F1[2] - F0[2] + 1);
    int empty = 0;
    for (int a = 0; a < 3; ++a)
        if (F1[a] < F0[a]) empty = 1;
    if (!empty) memset(val, 0, sizeof(double) * (size_t)((F1[0] - F0[0] + 1) * ny * nt));
    double total = 0.0;
    /* cells whose pushes can reach the region: c in [lo,hi] and c in [-1, N] */
    int32_t c0[3], c1[3];
    for (int a = 0; a < 3; ++a) {
        int32_t N = o_nfine(g, a);
        c0[a] = lo[a] > -1 ? lo[a] : -1;
        c1[a] = hi[a] < N ? hi[a] : N;
    }
    for (int32_t cx = c0[0]; cx <= c1[0]; ++cx)
        for (int32_t cy = c0[1]; cy <= c1[1]; ++cy)
            for (int32_t ct = c0[2]; ct <= c1[2]; ++ct) {
                double xc = (double)g->origin[0] + (cx + 0.5) * h[0];
                double yc = (double)g->origin[1] + (cy + 0.5) * h[1];
                double tc = (double)g->origin[2] + ct * h[2];
                for (int l = 0; l < n; ++l)
                    for (int m = 0; m < n; ++m)
                        for (int k = 0; k < n; ++k) {
                            double x = xc + xi[l] * h[0] / 2.0;
                            double y = yc + xi[m] * h[1] / 2.0;
                            double t = tc + xi[k] * h[2] / 2.0;
                            double q = ipt ? oracle_q_point(x, y, t, mid, sig, tr[3])
                                           : oracle_q_line(x, y, t, p0, p1, sig, tr[3]);
                            double v = w[l] * w[m] * w[k] * jac * q;
                            total += v;
                            /* trilinear spread to the 2x2x2 grid points on the node's octant */
                            double ux[2] = {1.0 - fabs(xi[l]) / 2.0, fabs(xi[l]) / 2.0};
                            double uy[2] = {1.0 - fabs(xi[m]) / 2.0, fabs(xi[m]) / 2.0};
                            double ut[2] = {1.0 - fabs(xi[k]) / 2.0, fabs(xi[k]) / 2.0};
                            int sx = xi[l] > 0 ? 1 : -1, sy = xi[m] > 0 ? 1 : -1,
                                st = xi[k] > 0 ? 1 : -1;
                            for (int a = 0; a < 2; ++a) {
                                if (a == 1 && xi[l] == 0.0) continue;
                                int32_t gx = cx + a * sx;
                                if (gx < F0[0] || gx > F1[0]) continue;
                                for (int b = 0; b < 2; ++b) {
                                    if (b == 1 && xi[m] == 0.0) continue;
                                    int32_t gy = cy + b * sy;
                                    if (gy < F0[1] || gy > F1[1]) continue;
                                    for (int c = 0; c < 2; ++c) {
                                        if (c == 1 && xi[k] == 0.0) continue;
                                        int32_t gt = ct + c * st;
                                        if (gt < F0[2] || gt > F1[2]) continue;
                                        val[((int64_t)(gx - F0[0]) * ny + (gy - F0[1])) * nt +
                                            (gt - F0[2])] += v * ux[a] * uy[b] * ut[c];
                                    }
                                }
                            }
                        }
            }
    if (node_sum) *node_sum = total;
    return 0;
}

/* Effective charge of all depositions into their patches val[off[d] .. off[d+1]). */
void oracle_effq(const o_grid* g, const o_physics* ph, int64_t n, const float* seg,
                 const int32_t* fp, const int64_t* off, double* val, double* node_sums) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t d = 0; d < n; ++d) {
        double s = 0.0;
        oracle_effq_patch(g, ph, seg + 7 * d, fp + 6 * d, val + off[d], &s);
        if (node_sums) node_sums[d] = s;
    }
}

/* Per-cell node sums before the trilinear spread (sum over the cell's nodes of
 * w * q): the Gauss-Legendre estimate of the charge inside each cuboid
 * (Sec. II-C, eq. cub with I = 1). Cells: the box [c0, c1] (inclusive). */
void oracle_cell_sums(const o_grid* g, const o_physics* ph, const float* seg, const int32_t* c0,
                      const int32_t* c1, double* out) {
    double tr[7];
    oracle_transport(ph, seg, tr);
    int32_t lo[3], hi[3], ipt;
    oracle_window_f32(g, ph, seg, lo, hi, &ipt);
    double p0[3] = {seg[0], seg[1], tr[0]};
    double p1[3] = {seg[3], seg[4], tr[1]};
    double sig[3] = {tr[4], tr[5], tr[6]};
    double mid[3] = {0.5 * (p0[0] + p1[0]), 0.5 * (p0[1] + p1[1]), tr[2]};
    double xi[64], w[64];
    int n = ph->n_gl;
    oracle_gl_rule(n, xi, w);
    double h[3] = {g->spacing[0], g->spacing[1], g->spacing[2]};
    double jac = (h[0] / 2.0) * (h[1] / 2.0) * (h[2] / 2.0);
    int64_t idx = 0;
    for (int32_t cx = c0[0]; cx <= c1[0]; ++cx)
        for (int32_t cy = c0[1]; cy <= c1[1]; ++cy)
            for (int32_t ct = c0[2]; ct <= c1[2]; ++ct) {
                double xc = (double)g->origin[0] + (cx + 0.5) * h[0];
                double yc = (double)g->origin[1] + (cy + 0.5) * h[1];
                double tc = (double)g->origin[2] + ct * h[2];
                double s = 0.0;
                for (int l = 0; l < n; ++l)
                    for (int m = 0; m < n; ++m)
                        for (int k = 0; k < n; ++k) {
                            double x = xc + xi[l] * h[0] / 2.0;
                            double y = yc + xi[m] * h[1] / 2.0;
                            double t = tc + xi[k] * h[2] / 2.0;
                            double q = ipt ? oracle_q_point(x, y, t, mid, sig, tr[3])
                                           : oracle_q_line(x, y, t, p0, p1, sig, tr[3]);
                            s += w[l] * w[m] * w[k] * jac * q;
                        }
                out[idx++] = s;
            }
}

/* ------------------------------------------------------------------------ */
/* Block-sparse binning (Sec. III-B): the region is partitioned into bins of
 * blk_pix * sub fine cells in x and y and blk_ticks ticks in t, aligned to the
 * region origin; a bin is kept iff some deposition's footprint has a cell in
 * it. keys: (bx, by, bt) of kept bins, ascending by (bx, by, bt).
 * Returns the number of kept bins (keys beyond cap are not written).        */
int32_t oracle_block_keys(const o_grid* g, const o_blocking* b, int64_t n, const int32_t* fp,
                          int32_t* keys, int32_t cap) {
    int32_t Bf[3] = {b->blk_pix[0] * g->sub[0], b->blk_pix[1] * g->sub[1], b->blk_ticks};
    int32_t NB[3];
    for (int a = 0; a < 3; ++a) NB[a] = (o_nfine(g, a) + Bf[a] - 1) / Bf[a];
    int64_t tot = (int64_t)NB[0] * NB[1] * NB[2];
    uint8_t* mark = (uint8_t*)calloc((size_t)tot, 1);
    for (int64_t d = 0; d < n; ++d) {
        const int32_t* f = fp + 6 * d;
        if (f[3] < f[0] || f[4] < f[1] || f[5] < f[2]) continue;
        for (int32_t bx = f[0] / Bf[0]; bx <= f[3] / Bf[0]; ++bx)
            for (int32_t by = f[1] / Bf[1]; by <= f[4] / Bf[1]; ++by)
                for (int32_t bt = f[2] / Bf[2]; bt <= f[5] / Bf[2]; ++bt)
                    mark[((int64_t)bx * NB[1] + by) * NB[2] + bt] = 1;
    }
    int32_t na = 0;
    for (int64_t i = 0; i < tot; ++i) {
        if (!mark[i]) continue;
        if (na < cap) {
            keys[3 * na + 0] = (int32_t)(i / ((int64_t)NB[1] * NB[2]));
            keys[3 * na + 1] = (int32_t)((i / NB[2]) % NB[1]);
            keys[3 * na + 2] = (int32_t)(i % NB[2]);
        }
        ++na;
    }
    free(mark);
    return na;
}

/* Values of one bin: the sum of all deposition patches restricted to the bin
 * (overlapping contributions reduced by summation, Sec. III-B).             */
void oracle_block_values(const o_grid* g, const o_blocking* b, int64_t n, const int32_t* fp,
                         const int64_t* off, const double* val, const int32_t* key,
                         double* out) {
    int32_t Bf[3] = {b->blk_pix[0] * g->sub[0], b->blk_pix[1] * g->sub[1], b->blk_ticks};
    int32_t L0[3], L1[3];
    for (int a = 0; a < 3; ++a) {
        L0[a] = key[a] * Bf[a];
        L1[a] = L0[a] + Bf[a] - 1;
    }
    memset(out, 0, sizeof(double) * (size_t)Bf[0] * Bf[1] * Bf[2]);
    for (int64_t d = 0; d < n; ++d) {
        const int32_t* f = fp + 6 * d;
        int32_t lo[3], hi[3], skip = 0;
        for (int a = 0; a < 3; ++a) {
            lo[a] = f[a] > L0[a] ? f[a] : L0[a];
            hi[a] = f[3 + a] < L1[a] ? f[3 + a] : L1[a];
            if (hi[a] < lo[a]) skip = 1;
        }
        if (skip) continue;
        int64_t ny = f[4] - f[1] + 1, nt = f[5] - f[2] + 1;
        const double* v = val + off[d];
        for (int32_t x = lo[0]; x <= hi[0]; ++x)
            for (int32_t y = lo[1]; y <= hi[1]; ++y)
                for (int32_t t = lo[2]; t <= hi[2]; ++t)
                    out[((int64_t)(x - L0[0]) * Bf[1] + (y - L0[1])) * Bf[2] + (t - L0[2])] +=
                        v[((int64_t)(x - f[0]) * ny + (y - f[1])) * nt + (t - f[2])];
    }
}

/* ------------------------------------------------------------------------ */
/* Induced current (Sec. II-D, eq. interlaced; Sec. II-B eq. firstapprox).
 * The fine index splits into (sub-pixel j, pixel p); a unit charge at fine cell
 * (ix, iy) and tick n contributes R[k][j][tau] to pixel p + k - (K-1)/2 at tick
 * n + tau (cross-correlation in the pixel plane folded into the response
 * orientation R[k] = i[-k]; convolution in time). Direct sum over every patch
 * cell, by linearity of the reduction over depositions (Sec. III-B).
 * resp: [Kx][Ky][sx][sy][Kt]. pix: list of n_pix pixel ids (px * npix_y + py).
 * wf: [n_pix][nticks + Kt - 1], zeroed here.                                 */
void oracle_waveforms(const o_grid* g, const int32_t* kpix, int32_t kt, const float* resp,
                      int64_t n, const int32_t* fp, const int64_t* off, const double* val,
                      int64_t n_pix, const int32_t* pix, double* wf) {
    int32_t sx = g->sub[0], sy = g->sub[1];
    int32_t hx = (kpix[0] - 1) / 2, hy = (kpix[1] - 1) / 2;
    int64_t L = (int64_t)g->nticks + kt - 1;
    memset(wf, 0, sizeof(double) * (size_t)(n_pix * L));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ip = 0; ip < n_pix; ++ip) {
        int32_t P[2] = {pix[ip] / g->npix[1], pix[ip] % g->npix[1]};
        double* out = wf + ip * L;
        for (int64_t d = 0; d < n; ++d) {
            const int32_t* f = fp + 6 * d;
            if (f[3] < f[0] || f[4] < f[1] || f[5] < f[2]) continue;
            /* charge pixels that reach P: px in [P - hx, P + hx] */
            int32_t x0 = (P[0] - hx) * sx, x1 = (P[0] + hx + 1) * sx - 1;
            int32_t y0 = (P[1] - hy) * sy, y1 = (P[1] + hy + 1) * sy - 1;
            if (x0 < f[0]) x0 = f[0];
            if (x1 > f[3]) x1 = f[3];
            if (y0 < f[1]) y0 = f[1];
            if (y1 > f[4]) y1 = f[4];
            if (x1 < x0 || y1 < y0) continue;
            int64_t ny = f[4] - f[1] + 1, nt = f[5] - f[2] + 1;
            const double* v = val + off[d];
            for (int32_t ix = x0; ix <= x1; ++ix) {
                int32_t px = ix / sx, jx = ix % sx, kx = P[0] - px + hx;
                for (int32_t iy = y0; iy <= y1; ++iy) {
                    int32_t py = iy / sy, jy = iy % sy, ky = P[1] - py + hy;
                    const float* r =
                        resp + ((((int64_t)kx * kpix[1] + ky) * sx + jx) * sy + jy) * kt;
                    const double* q = v + ((int64_t)(ix - f[0]) * ny + (iy - f[1])) * nt;
                    for (int32_t it = f[2]; it <= f[5]; ++it) {
                        double qv = q[it - f[2]];
                        if (qv == 0.0) continue;
                        double* o = out + it;
                        for (int32_t tau = 0; tau < kt; ++tau) o[tau] += qv * (double)r[tau];
                    }
                }
            }
        }
    }
}

/* The same sum evaluated at isolated output samples (pixel id, tick). */
void oracle_waveform_points(const o_grid* g, const int32_t* kpix, int32_t kt, const float* resp,
                            int64_t n, const int32_t* fp, const int64_t* off, const double* val,
                            int64_t n_pts, const int32_t* pts, double* out) {
    int32_t sx = g->sub[0], sy = g->sub[1];
    int32_t hx = (kpix[0] - 1) / 2, hy = (kpix[1] - 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ip = 0; ip < n_pts; ++ip) {
        int32_t P[2] = {pts[2 * ip] / g->npix[1], pts[2 * ip] % g->npix[1]};
        int32_t T = pts[2 * ip + 1];
        double acc = 0.0;
        for (int64_t d = 0; d < n; ++d) {
            const int32_t* f = fp + 6 * d;
            if (f[3] < f[0] || f[4] < f[1] || f[5] < f[2]) continue;
            int32_t x0 = (P[0] - hx) * sx, x1 = (P[0] + hx + 1) * sx - 1;
            int32_t y0 = (P[1] - hy) * sy, y1 = (P[1] + hy + 1) * sy - 1;
            int32_t t0 = T - kt + 1, t1 = T;
            if (x0 < f[0]) x0 = f[0];
            if (x1 > f[3]) x1 = f[3];
            if (y0 < f[1]) y0 = f[1];
            if (y1 > f[4]) y1 = f[4];
            if (t0 < f[2]) t0 = f[2];
            if (t1 > f[5]) t1 = f[5];
            if (x1 < x0 || y1 < y0 || t1 < t0) continue;
            int64_t ny = f[4] - f[1] + 1, nt = f[5] - f[2] + 1;
            const double* v = val + off[d];
            for (int32_t ix = x0; ix <= x1; ++ix) {
                int32_t px = ix / sx, jx = ix % sx, kx = P[0] - px + hx;
                for (int32_t iy = y0; iy <= y1; ++iy) {
                    int32_t py = iy / sy, jy = iy % sy, ky = P[1] - py + hy;
                    const float* r =
                        resp + ((((int64_t)kx * kpix[1] + ky) * sx + jx) * sy + jy) * kt;
                    const double* q = v + ((int64_t)(ix - f[0]) * ny + (iy - f[1])) * nt;
                    for (int32_t it = t0; it <= t1; ++it)
                        acc += q[it - f[2]] * (double)r[T - it];
                }
            }
        }
        out[ip] = acc;
    }
}

/*
 * Driver for the sanitizer build of the oracle (TEST INFRASTRUCTURE ONLY).
 *
 * The test suite compiles this file together with oracle.c under the host address
 * and undefined-behaviour sanitizers and runs it on one small event. It reads the
 * inputs from a binary file, calls every oracle entry point (Gauss-Legendre rule,
 * line/point densities, footprints, effective charge, cell sums, bin keys and
 * values, waveforms, waveform samples) and writes their outputs to another file,
 * which the test compares with the regular build's outputs.
 *
 * Input file layout (little endian):
 *   grid (o_grid), physics (o_physics), blocking (o_blocking),
 *   int32 kpix[2], int32 kticks, int64 n, float seg[n][7], float resp[...],
 *   int64 n_pts, int32 pts[n_pts][2]
 * Output file: int64 n_keys, int32 keys[n_keys][3], int32 fp[n][6], int64 off[n+1],
 *   int32 is_point[n], double val[off[n]], double node_sums[n],
 *   double block_values[n_keys][Vblk], int64 n_pix, int32 pix[n_pix],
 *   double wf[n_pix][nticks + kticks - 1], double pts_out[n_pts],
 *   double cell_sums[27] (3x3x3 cells around the first deposition's window centre),
 *   double gl[2][8] (nodes and weights of the 8-point rule), double q[2] (line and
 *   point densities of the first deposition at its midpoint).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float origin[3];
    float spacing[3];
    int32_t npix[2];
    int32_t sub[2];
    int32_t nticks;
} o_grid;

typedef struct {
    float v_drift, lifetime, diff_T, diff_L;
    float sigma_min[3];
    float n_sigma, point_frac;
    int32_t n_gl;
} o_physics;

typedef struct {
    int32_t blk_pix[2];
    int32_t blk_ticks;
} o_blocking;

int oracle_gl_rule(int n, double* xi, double* w);
void oracle_transport(const o_physics* ph, const float* seg, double* out);
void oracle_window_f32(const o_grid* g, const o_physics* ph, const float* seg, int32_t* lo,
                       int32_t* hi, int32_t* is_point);
void oracle_footprints(const o_grid* g, const o_physics* ph, int64_t n, const float* seg,
                       int32_t* fp, int64_t* off, int32_t* is_point);
double oracle_q_line(double x, double y, double z, const double* p0, const double* p1,
                     const double* sig, double Q);
double oracle_q_point(double x, double y, double z, const double* m, const double* sig, double Q);
void oracle_effq(const o_grid* g, const o_physics* ph, int64_t n, const float* seg,
                 const int32_t* fp, const int64_t* off, double* val, double* node_sums);
void oracle_cell_sums(const o_grid* g, const o_physics* ph, const float* seg, const int32_t* c0,
                      const int32_t* c1, double* out);
int32_t oracle_block_keys(const o_grid* g, const o_blocking* b, int64_t n, const int32_t* fp,
                          int32_t* keys, int32_t cap);
void oracle_block_values(const o_grid* g, const o_blocking* b, int64_t n, const int32_t* fp,
                         const int64_t* off, const double* val, const int32_t* key, double* out);
void oracle_waveforms(const o_grid* g, const int32_t* kpix, int32_t kt, const float* resp,
                      int64_t n, const int32_t* fp, const int64_t* off, const double* val,
                      int64_t n_pix, const int32_t* pix, double* wf);
void oracle_waveform_points(const o_grid* g, const int32_t* kpix, int32_t kt, const float* resp,
                            int64_t n, const int32_t* fp, const int64_t* off, const double* val,
                            int64_t n_pts, const int32_t* pts, double* out);

static void* xmalloc(size_t bytes) {
    /* exact sizes, so that the address sanitizer sees every overrun */
    void* p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static void rd(void* p, size_t size, size_t n, FILE* f) {
    if (n && fread(p, size, n, f) != n) {
        fprintf(stderr, "short input file\n");
        exit(2);
    }
}

static void wr(const void* p, size_t size, size_t n, FILE* f) {
    if (n && fwrite(p, size, n, f) != n) {
        fprintf(stderr, "write failed\n");
        exit(2);
    }
}

int main(int argc, char** argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 2;
    }
    FILE* in = fopen(argv[1], "rb");
    if (!in) return 2;
    o_grid g;
    o_physics ph;
    o_blocking b;
    int32_t kpix[2], kt;
    int64_t n, n_pts;
    rd(&g, sizeof g, 1, in);
    rd(&ph, sizeof ph, 1, in);
    rd(&b, sizeof b, 1, in);
    rd(kpix, sizeof(int32_t), 2, in);
    rd(&kt, sizeof kt, 1, in);
    rd(&n, sizeof n, 1, in);
    float* seg = (float*)xmalloc(sizeof(float) * 7 * (size_t)n);
    rd(seg, sizeof(float), 7 * (size_t)n, in);
    size_t nresp = (size_t)kpix[0] * kpix[1] * g.sub[0] * g.sub[1] * kt;
    float* resp = (float*)xmalloc(sizeof(float) * nresp);
    rd(resp, sizeof(float), nresp, in);
    rd(&n_pts, sizeof n_pts, 1, in);
    int32_t* pts = (int32_t*)xmalloc(sizeof(int32_t) * 2 * (size_t)n_pts);
    rd(pts, sizeof(int32_t), 2 * (size_t)n_pts, in);
    fclose(in);

    int32_t* fp = (int32_t*)xmalloc(sizeof(int32_t) * 6 * (size_t)n);
    int64_t* off = (int64_t*)xmalloc(sizeof(int64_t) * ((size_t)n + 1));
    int32_t* ip = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n);
    oracle_footprints(&g, &ph, n, seg, fp, off, ip);
    double* val = (double*)xmalloc(sizeof(double) * (size_t)off[n]);
    double* ns = (double*)xmalloc(sizeof(double) * (size_t)n);
    oracle_effq(&g, &ph, n, seg, fp, off, val, ns);

    int32_t nb[3] = {(g.npix[0] * g.sub[0] + b.blk_pix[0] * g.sub[0] - 1) / (b.blk_pix[0] * g.sub[0]),
                     (g.npix[1] * g.sub[1] + b.blk_pix[1] * g.sub[1] - 1) / (b.blk_pix[1] * g.sub[1]),
                     (g.nticks + b.blk_ticks - 1) / b.blk_ticks};
    int32_t cap = nb[0] * nb[1] * nb[2];
    int32_t* keys = (int32_t*)xmalloc(sizeof(int32_t) * 3 * (size_t)cap);
    int32_t nk = oracle_block_keys(&g, &b, n, fp, keys, cap);
    size_t vblk = (size_t)b.blk_pix[0] * g.sub[0] * b.blk_pix[1] * g.sub[1] * b.blk_ticks;
    double* bv = (double*)xmalloc(sizeof(double) * vblk * (size_t)nk);
    for (int32_t k = 0; k < nk; ++k) oracle_block_values(&g, &b, n, fp, off, val, keys + 3 * k, bv + vblk * k);

    /* every pixel of the region */
    int64_t n_pix = (int64_t)g.npix[0] * g.npix[1];
    int32_t* pix = (int32_t*)xmalloc(sizeof(int32_t) * (size_t)n_pix);
    for (int64_t i = 0; i < n_pix; ++i) pix[i] = (int32_t)i;
    size_t lwf = (size_t)g.nticks + kt - 1;
    double* wf = (double*)xmalloc(sizeof(double) * lwf * (size_t)n_pix);
    oracle_waveforms(&g, kpix, kt, resp, n, fp, off, val, n_pix, pix, wf);
    double* po = (double*)xmalloc(sizeof(double) * (size_t)n_pts);
    oracle_waveform_points(&g, kpix, kt, resp, n, fp, off, val, n_pts, pts, po);

    double cs[27];
    memset(cs, 0, sizeof cs);
    double gl[16], q[2] = {0.0, 0.0};
    oracle_gl_rule(8, gl, gl + 8);
    if (n > 0) {
        int32_t lo[3], hi[3], pt, c0[3], c1[3];
        oracle_window_f32(&g, &ph, seg, lo, hi, &pt);
        for (int a = 0; a < 3; ++a) {
            c0[a] = (lo[a] + hi[a]) / 2 - 1;
            c1[a] = c0[a] + 2;
        }
        oracle_cell_sums(&g, &ph, seg, c0, c1, cs);
        double tr[7];
        oracle_transport(&ph, seg, tr);
        double p0[3] = {seg[0], seg[1], tr[0]}, p1[3] = {seg[3], seg[4], tr[1]};
        double sig[3] = {tr[4], tr[5], tr[6]};
        double m[3] = {0.5 * (p0[0] + p1[0]), 0.5 * (p0[1] + p1[1]), tr[2]};
        q[0] = oracle_q_line(m[0], m[1], m[2], p0, p1, sig, tr[3]);
        q[1] = oracle_q_point(m[0], m[1], m[2], m, sig, tr[3]);
    }

    FILE* out = fopen(argv[2], "wb");
    if (!out) return 2;
    int64_t nk64 = nk;
    wr(&nk64, sizeof nk64, 1, out);
    wr(keys, sizeof(int32_t), 3 * (size_t)nk, out);
    wr(fp, sizeof(int32_t), 6 * (size_t)n, out);
    wr(off, sizeof(int64_t), (size_t)n + 1, out);
    wr(ip, sizeof(int32_t), (size_t)n, out);
    wr(val, sizeof(double), (size_t)off[n], out);
    wr(ns, sizeof(double), (size_t)n, out);
    wr(bv, sizeof(double), vblk * (size_t)nk, out);
    wr(&n_pix, sizeof n_pix, 1, out);
    wr(pix, sizeof(int32_t), (size_t)n_pix, out);
    wr(wf, sizeof(double), lwf * (size_t)n_pix, out);
    wr(po, sizeof(double), (size_t)n_pts, out);
    wr(cs, sizeof(double), 27, out);
    wr(gl, sizeof(double), 16, out);
    wr(q, sizeof(double), 2, out);
    fclose(out);
    free(seg); free(resp); free(pts); free(fp); free(off); free(ip); free(val); free(ns);
    free(keys); free(bv); free(pix); free(wf); free(po);
    return 0;
}

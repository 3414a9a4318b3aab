/*
 * tred.h - C ABI of the MI355X (gfx950) library for the signal-formation hot path
 * of pixelated LArTPC simulation (arXiv 2602.12052):
 *
 *   depositions --(transport, effective charge)--> per-deposition charge patches
 *               --(block-sparse binning)---------> dense charge blocks on active bins
 *               --(interlaced FFT convolution)---> induced-current blocks
 *               --(overlap-add)------------------> per-pixel current waveforms
 *
 * Conventions for every call
 *   - Array arguments are DEVICE pointers owned by the caller; the library never
 *     allocates, frees or retains them (a conv plan keeps the workspace pointer
 *     given to tred_conv_plan_set_response until the plan is destroyed).
 *   - `stream` is a hipStream_t (NULL = the null stream). Calls are asynchronous:
 *     they enqueue kernels and return. Argument errors are detected on the host
 *     before anything is enqueued; launch failures return TRED_EDEVICE; faults
 *     inside kernels surface at the caller's next synchronisation.
 *   - Counts that depend on the data (off[n_dep], *n_active, *n_pix) are written
 *     to device memory; kernels never write past the given capacity, and a count
 *     larger than its capacity reports truncation. Every capacity has a
 *     host-computable bound (tred_block_count, npix[0]*npix[1], and
 *     n_dep * the largest footprint) so that no host synchronisation is needed.
 *   - Axis order is x, y, t everywhere; t varies fastest in every array.
 *   - Integer outputs are deterministic. Floating-point sums (over depositions,
 *     blocks, impact channels) are taken in an unspecified order.
 *   - NaN or infinite inputs give undefined (but memory-safe) results.
 */
#ifndef TRED_H
#define TRED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRED_ABI_VERSION 1

typedef enum {
    TRED_OK = 0,
    TRED_EINVAL = 1,       /* null pointer, non-positive size, out-of-range parameter     */
    TRED_ECAPACITY = 2,    /* a host-visible capacity is too small for a static bound     */
    TRED_EDEVICE = 3,      /* a HIP call or kernel launch failed                          */
    TRED_EUNSUPPORTED = 4  /* valid request outside what the kernels implement            */
} tred_status;

/* Static description of a status code. */
const char* tred_status_string(int status);
/* Detail of the last non-OK status returned on the calling host thread ("" if none). */
const char* tred_last_error(void);
int tred_abi_version(void);
/* Identity of the build: the hex SHA-256 of the sources (every file of csrc/ and
 * this header), compiler flags and defines it was compiled from ("unversioned"
 * when built without one). A binding compares it with its source tree. */
const char* tred_build_id(void);

/* Fine sampling grid of the field response (Sec. II-B, II-C): each pixel of
 * pitch a is divided into sub[0] x sub[1] impact cells of size
 * spacing[0..1] = a / sub; time is sampled in ticks of spacing[2].
 * Grid point (i, j, n) sits at (origin_x + (i+1/2) h_x, origin_y + (j+1/2) h_y,
 * origin_t + n * tick); its cell spans +-h/2 around it. Fine index i splits into
 * pixel i / sub[0] and impact position i % sub[0] (Sec. II-D). */
typedef struct {
    float origin[3];   /* x, y of the lower edge of pixel (0,0) [cm]; t of tick 0 [us] */
    float spacing[3];  /* h_x, h_y [cm]; tick [us]                                      */
    int32_t npix[2];   /* pixels along x, y                                             */
    int32_t sub[2];    /* impact positions per pixel along x, y                         */
    int32_t nticks;    /* ticks in the readout window                                   */
} tred_grid;

/* Transport and quadrature (Sec. II-A, II-C, V-A). A segment (x0,y0,z0)-(x1,y1,z1)
 * with z the drift distance [cm] arrives at t = z / v_drift. With t_mid the mid
 * arrival time, its charge becomes Q exp(-t_mid / lifetime) and its diffusion
 * widths sigma_x = sigma_y = max(sqrt(2 diff_T t_mid), sigma_min[0..1]) and
 * sigma_t = max(sqrt(2 diff_L t_mid) / v_drift, sigma_min[2]). The quadrature
 * window spans n_sigma widths beyond the segment's end points on each axis. A
 * segment whose end points differ by less than point_frac * sigma on every axis is
 * treated as a point charge at its midpoint. n_gl Gauss-Legendre nodes per axis
 * per cell, 1 <= n_gl <= 8; tred_effq requires point_frac > 0 (a segment of zero
 * length must take the point form). */
typedef struct {
    float v_drift;      /* cm/us                          */
    float lifetime;     /* us                             */
    float diff_T;       /* cm^2/us                        */
    float diff_L;       /* cm^2/us                        */
    float sigma_min[3]; /* floor of the widths: cm, cm, us */
    float n_sigma;
    float point_frac;
    int32_t n_gl;
} tred_physics;

/* Bins of the block-sparse binned tensor (Sec. III-B): blk_pix pixels (i.e.
 * blk_pix * sub fine cells) along x and y, blk_ticks ticks along t, aligned to
 * the region origin. Bin (bx, by, bt) covers fine cells
 * [bx*blk_pix[0]*sub[0], (bx+1)*blk_pix[0]*sub[0]) and the same for y, t. */
typedef struct {
    int32_t blk_pix[2];
    int32_t blk_ticks;
} tred_blocking;

/* ------------------------------------------------------------------------- */
/* Transport and footprints (Sec. II-A; Sec. II-C line/point switch and the
 * one-cell trilinear stencil).
 *
 * seg [n_dep][7]: x0, y0, z0, x1, y1, z1 [cm], Q [electrons after recombination].
 * fp  [n_dep][6] out: footprint of the deposition's effective charge, inclusive
 *     cell bounds lo[3], hi[3] of (quadrature window dilated by one cell) cropped to
 *     the region; lo > hi on some axis means the deposition misses the region.
 * off [n_dep+1] out: off[0] = 0, off[d+1] = off[d] + cell count of fp[d].
 * The window bounds and the point/line decision are computed by a fixed chain of
 * correctly rounded binary32 operations (no contraction), so they are unique:
 *   t_a = z_a / v; t_mid = (t0 + t1) * 0.5; sT = sqrt((2 diff_T) t_mid);
 *   sL = sqrt((2 diff_L) t_mid) / v; sigma = max(., sigma_min);
 *   u_a = (P_a - origin) / h (+ 0.5 on t); e = n_sigma * (sigma / h);
 *   lo = floor(min(u0, u1) - e); hi = floor(max(u0, u1) + e).
 * n_dep = 0 is valid (writes off[0] = 0). */
tred_status tred_effq_windows(const tred_grid* grid, const tred_physics* phys, int64_t n_dep,
                              const float* seg, int32_t* fp, int64_t* off, void* stream);

/* Effective charge (Sec. II-C, eqs. cub, trilinear, eff_q; line charge eq. qline
 * with exponent -B/(2 Delta^2), or its point-like limit). For every cell of the
 * quadrature window, n_gl^3 Gauss-Legendre nodes carry w * q(node) (rule mapped to
 * the cell); each node's charge is spread to the grid points of the 2x2x2 cells on
 * its side with trilinear coefficients. Patch d is val[off[d] .. off[d+1]) over
 * the cells of fp[d] (x-major, then y, t fastest), summed over that deposition
 * only. Grid points outside the region are dropped.
 * val_cap: length of val; depositions whose patch would end past val_cap are
 * skipped (the caller detects this from off[n_dep] > val_cap), and so are patches of
 * 2^31 cells or more (off[d+1] - off[d] > INT32_MAX; their values are not written).
 * charge_sum (may be NULL): sum over all evaluated nodes of w * q (binary32 along
 * one column of nodes within a tile of cells, binary64 over columns),
 * accumulated (not overwritten) by this call. */
tred_status tred_effq(const tred_grid* grid, const tred_physics* phys, int64_t n_dep,
                      const float* seg, const int32_t* fp, const int64_t* off, float* val,
                      int64_t val_cap, double* charge_sum, void* stream);

/* ------------------------------------------------------------------------- */
/* Block-sparse binning (Sec. III-B): the active bins are the bins that contain a
 * cell of some footprint; blocks hold the sum of all patches restricted to the bin.
 *
 * keys   [cap][3] out: (bx, by, bt) of active bins, ascending lexicographically.
 * n_active out (device scalar): number of active bins (may exceed cap).
 * blocks [cap][blk_pix[0]*sub[0]][blk_pix[1]*sub[1]][blk_ticks] out: dense FP32
 *        charge of each active bin (zero where no patch reaches); 16-byte aligned.
 * val_cap: length of val; patches ending past it are ignored (as in tred_effq).
 * work: device workspace of tred_block_bin_workspace() bytes. */
int32_t tred_block_count(const tred_grid* grid, const tred_blocking* blocking);
int64_t tred_block_bin_workspace(const tred_grid* grid, const tred_blocking* blocking);
tred_status tred_block_bin(const tred_grid* grid, const tred_blocking* blocking, int64_t n_dep,
                           const int32_t* fp, const int64_t* off, const float* val,
                           int64_t val_cap, int32_t* keys, int32_t* n_active, float* blocks,
                           int32_t cap, void* work, void* stream);

/* Block-sparse binning with row masks: as tred_block_bin, and additionally marks the
 * rows of each active bin that can hold charge, so that only those are written. A
 * row is the blk_ticks cells of one fine (x, y) cell of the bin, r = x * (blk_pix[1] *
 * sub[1]) + y; it is marked when it meets some footprint box.
 * rows [cap][tred_block_row_words()] out: bit (r % 32) of word r / 32 of bin s is set
 *      for the marked rows of bin s (4-byte aligned).
 * blocks: marked rows hold the binned charge; the other rows are NOT written (their
 *      contents are whatever the buffer held) and are zero in the binned tensor. Pass
 *      both to tred_block_conv_rows. */
int32_t tred_block_row_words(const tred_grid* grid, const tred_blocking* blocking);
tred_status tred_block_bin_rows(const tred_grid* grid, const tred_blocking* blocking,
                                int64_t n_dep, const int32_t* fp, const int64_t* off,
                                const float* val, int64_t val_cap, int32_t* keys,
                                int32_t* n_active, float* blocks, uint32_t* rows, int32_t cap,
                                void* work, void* stream);

/* tred_block_bin_rows for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * outputs as tred_block_bin_rows, with the workspace replaced by a static array in the
 * library's device memory (1 MiB, one copy per device, held until the process ends;
 * found on a device's first call, which must have that device current). The call
 * allocates nothing and frees nothing.
 * Returns TRED_ECAPACITY if tred_block_count() exceeds 262,144 bins (the array's
 * size); use tred_block_bin_rows with a workspace then.
 * Every call on one device shares that device's array: calls that overlap on one
 * device (other streams, other host threads) race and give undefined outputs; calls
 * ordered on one stream are safe (each call clears the array before using it). */
tred_status tred_block_bin_rows_noalloc(const tred_grid* grid, const tred_blocking* blocking,
                                        int64_t n_dep, const int32_t* fp, const int64_t* off,
                                        const float* val, int64_t val_cap, int32_t* keys,
                                        int32_t* n_active, float* blocks, uint32_t* rows,
                                        int32_t cap, void* stream);

/* Effective charge straight into the bins (Sec. II-C eq. eff_q, Sec. III-B): the
 * outputs of tred_effq followed by tred_block_bin_rows (rows non-NULL) or
 * tred_block_bin (rows NULL), without the patches. The bins are laid out from the
 * footprints fp of tred_effq_windows (keys, n_active, rows, zeroed rows or bins),
 * then the effective-charge kernel adds every footprint cell of every deposition
 * into its bin with an FP32 atomic, so no patch buffer is written or read. Blocks
 * equal those of the two-call path up to the order of the FP32 additions; cells of
 * bins beyond cap are dropped as there. charge_sum (may be NULL) accumulates the
 * node sum of tred_effq. The patch-size limits of tred_effq do not apply.
 * Requires physics.point_frac > 0 and fewer than 2^31 cells per bin (TRED_EINVAL).
 * work: tred_block_bin_workspace() bytes. */
tred_status tred_effq_bin(const tred_grid* grid, const tred_physics* phys,
                          const tred_blocking* blocking, int64_t n_dep, const float* seg,
                          const int32_t* fp, int32_t* keys, int32_t* n_active, float* blocks,
                          uint32_t* rows, int32_t cap, double* charge_sum, void* work,
                          void* stream);

/* ------------------------------------------------------------------------- */
/* Interlaced convolution with the field response (Sec. II-D, eq. interlaced),
 * evaluated per active bin by FFT with the channel sum in the frequency domain
 * (Sec. III-A): Y = IFFT( sum_j FFT(R_j) FFT(Q_j) ), with FFT(R_j) precomputed.
 *
 * resp [kpix[0]][kpix[1]][sub[0]][sub[1]][kticks]: R[k][j][tau] is the current on
 * the pixel at offset k - (kpix-1)/2 from the pixel holding a unit charge at impact
 * position j, tau ticks after the charge's arrival time.
 * Output of bin (bx, by, bt): out[qx][qy][t'] for qx < blk_pix[0] + kpix[0] - 1,
 * qy < blk_pix[1] + kpix[1] - 1, t' < blk_ticks + kticks - 1, i.e. pixel
 * (bx*blk_pix[0] - (kpix[0]-1)/2 + qx, by*blk_pix[1] - (kpix[1]-1)/2 + qy) at tick
 * bt*blk_ticks + t'.
 *
 * fft: FFT sizes (x, y, t). Spatial sizes must be equal, taken from
 * {8,16,24,32,36,40,48,64}, with fft[a] >= blk_pix[a] + kpix[a] - 1 (0 selects the
 * smallest of {8,16,24,32,40,48,64}). The
 * time size is a power of two in [256, 2048] with fft[2] >= blk_ticks + 64 (0 selects
 * the smallest power of two >= blk_ticks + kticks - 1); when fft[2] is shorter
 * than blk_ticks + kticks - 1 the response is split into ceil(kticks /
 * (fft[2] - blk_ticks)) <= 4 consecutive pieces whose outputs are overlap-added.
 * Kernel limits (TRED_EUNSUPPORTED otherwise): blk_pix[a] <= 2 L with L = 8 for
 * spatial sizes 8, 24, 40 and L = 16 for 16, 32, 48, 64, blk_pix[a] <= 16 for size 36
 * (the gradient calls do not take size 36); blk_ticks a multiple of 64;
 * kpix must be odd (TRED_EINVAL).
 * flags: TRED_CONV_MPCP pairs impact channels j and its mirror (sub-1-j) into one
 * complex transform (Sec. III-A, eq. multch); it requires the exact point symmetry
 * R[kpix-1-k][sub-1-j][tau] == R[k][j][tau], checked by set_response.
 * batch: bins transformed per pass; bounds the scratch in the workspace.
 * workspace_bytes out: device bytes the caller provides to set_response.
 * A plan's scratch is shared: calls using one plan must be serialised. */
typedef struct tred_conv_plan tred_conv_plan;
#define TRED_CONV_MPCP 1u

tred_status tred_conv_plan_create(const tred_grid* grid, const tred_blocking* blocking,
                                  const int32_t kpix[2], int32_t kticks, const int32_t fft[3],
                                  uint32_t flags, int32_t batch, tred_conv_plan** plan,
                                  int64_t* workspace_bytes);
/* Precompute the response spectra into `workspace` (binary64 arithmetic, stored
 * binary32). Synchronises `stream`. Returns TRED_EINVAL if MPCP was requested
 * and resp lacks the point symmetry. */
tred_status tred_conv_plan_set_response(tred_conv_plan* plan, const float* resp,
                                        void* workspace, void* stream);
/* Query the plan's resolved parameters: fft[3], number of response pieces,
 * number of transformed channels, output block extent out[3]. Any pointer may be NULL. */
tred_status tred_conv_plan_info(const tred_conv_plan* plan, int32_t fft[3], int32_t* pieces,
                                int32_t* channels, int32_t out[3]);
/* Optional stage timing (profiling aid, not part of the computation): events points
 * to six hipEvent_t created by the caller; tred_block_conv then records events[2s]
 * and events[2s+1] on its stream before and after the launches of stage s in its
 * first pass over the bins (s = 0: time-axis forward transforms; 1: spatial
 * transforms and spectral multiply-accumulate; 2: time-axis inverse transforms and
 * overlap-add of the response pieces). With batch >= cap each stage is one launch.
 * events = NULL switches timing off. */
tred_status tred_conv_plan_set_timing(tred_conv_plan* plan, void* const* events);
/* out_blocks [cap][blk_pix[0]+kpix[0]-1][blk_pix[1]+kpix[1]-1][blk_ticks+kticks-1]. */
tred_status tred_block_conv(const tred_conv_plan* plan, const int32_t* n_active, int32_t cap,
                            const float* blocks, float* out_blocks, void* stream);
/* As tred_block_conv on blocks whose unmarked rows (rows from tred_block_bin_rows)
 * are zero: only the marked rows of `blocks` are read. */
tred_status tred_block_conv_rows(const tred_conv_plan* plan, const int32_t* n_active,
                                 int32_t cap, const float* blocks, const uint32_t* rows,
                                 float* out_blocks, void* stream);

/* ------------------------------------------------------------------------- */
/* Overlap-add onto unique electrodes (Sec. III-B): the waveform of every pixel in
 * the union of the active bins' output footprints (cropped to the region) is the
 * sum of all block outputs covering it.
 * pix [pix_cap] out: pixel ids px * npix[1] + py, ascending; n_pix out (device).
 * wf  [pix_cap][nticks + kticks - 1] out: current waveform of pix[i], tick 0 first
 *     (ticks past the end of the readout window carry the response tail); rows
 *     i >= *n_pix are set to zero, so every row of wf is defined after the call.
 * work: device workspace of tred_scatter_workspace() bytes. */
int64_t tred_scatter_workspace(const tred_conv_plan* plan);
tred_status tred_scatter_waveforms(const tred_conv_plan* plan, const int32_t* keys,
                                   const int32_t* n_active, int32_t cap, const float* out_blocks,
                                   int32_t* pix, int32_t* n_pix, float* wf, int32_t pix_cap,
                                   void* work, void* stream);

void tred_conv_plan_destroy(tred_conv_plan* plan);

/* ------------------------------------------------------------------------- */
/* Batches of events (one binned tensor for many events). The depositions of n_ev
 * events are concatenated: event e owns depositions [ev_off[e], ev_off[e+1]) with
 * ev_off a DEVICE int64 array of n_ev + 1 non-decreasing offsets (ev_off[0] = 0,
 * ev_off[n_ev] = n_dep). tred_effq_windows / tred_effq run unchanged on the
 * concatenation (they are per deposition). The active (event, bin) pairs of all
 * events form one list of bins, so one tred_block_conv pass convolves the bins of
 * every event together (Sec. III-B, batching over the outer dimensions).
 * keys [cap][4] out: (event, bx, by, bt), ascending lexicographically.
 * pix  [pix_cap] out: ids event * npix[0] * npix[1] + px * npix[1] + py, ascending.
 * Per event, bins, pixels and waveforms are those of tred_block_bin and
 * tred_scatter_waveforms run on that event alone. Workspaces scale with n_ev. */
int64_t tred_block_bin_events_workspace(const tred_grid* grid, const tred_blocking* blocking,
                                        int32_t n_ev);
tred_status tred_block_bin_events(const tred_grid* grid, const tred_blocking* blocking,
                                  int32_t n_ev, const int64_t* ev_off, int64_t n_dep,
                                  const int32_t* fp, const int64_t* off, const float* val,
                                  int64_t val_cap, int32_t* keys, int32_t* n_active, float* blocks,
                                  int32_t cap, void* work, void* stream);
/* As tred_block_bin_events with the row masks of tred_block_bin_rows (rows
 * [cap][tred_block_row_words()]); convolve with tred_block_conv_rows. */
tred_status tred_block_bin_events_rows(const tred_grid* grid, const tred_blocking* blocking,
                                       int32_t n_ev, const int64_t* ev_off, int64_t n_dep,
                                       const int32_t* fp, const int64_t* off, const float* val,
                                       int64_t val_cap, int32_t* keys, int32_t* n_active,
                                       float* blocks, uint32_t* rows, int32_t cap, void* work,
                                       void* stream);
/* tred_effq_bin over a batch of events (keys [cap][4] as tred_block_bin_events;
 * work: tred_block_bin_events_workspace() bytes). */
tred_status tred_effq_bin_events(const tred_grid* grid, const tred_physics* phys,
                                 const tred_blocking* blocking, int32_t n_ev,
                                 const int64_t* ev_off, int64_t n_dep, const float* seg,
                                 const int32_t* fp, int32_t* keys, int32_t* n_active,
                                 float* blocks, uint32_t* rows, int32_t cap, double* charge_sum,
                                 void* work, void* stream);
int64_t tred_scatter_events_workspace(const tred_conv_plan* plan, int32_t n_ev);
tred_status tred_scatter_waveforms_events(const tred_conv_plan* plan, int32_t n_ev,
                                          const int32_t* keys, const int32_t* n_active,
                                          int32_t cap, const float* out_blocks, int32_t* pix,
                                          int32_t* n_pix, float* wf, int32_t pix_cap, void* work,
                                          void* stream);

/* ------------------------------------------------------------------------- */
/* Block-direct interlaced convolution on the matrix cores: the same operation and
 * output as tred_block_conv (Sec. II-D eq. interlaced), evaluated per bin as the
 * dense contraction out[p + k][t'] = sum_{j, tau} Q_j[p][t' - tau] R_j[k][tau]
 * on BF16 matrix instructions with FP32 accumulation (no transforms).
 * flags: TRED_DIRECT_SPLIT represents each operand x as hi + lo with hi = bf16(x),
 * lo = bf16(x - hi) and accumulates hi*hi + hi*lo + lo*hi (about 16 significant
 * bits per product); without it the operands are rounded to BF16 (8 bits).
 * batch: bins per pass (1 <= batch <= 65535); bounds the operand scratch.
 * workspace_bytes out: device bytes for set_response (BF16 response operands and
 * the charge operands of one pass). Outputs are accumulated with atomic adds, so
 * float sums are in an unspecified order; out_blocks rows of the active bins are
 * overwritten. The response may be of any shape (no symmetry needed); kpix odd.
 * Output rows are [cap][blk_pix[0]+kpix[0]-1][blk_pix[1]+kpix[1]-1][blk_ticks+kticks-1]
 * as for tred_block_conv, so tred_scatter_waveforms (with a tred_conv_plan of the
 * same geometry, which needs no response) forms the waveforms. */
typedef struct tred_direct_plan tred_direct_plan;
#define TRED_DIRECT_SPLIT 1u

tred_status tred_direct_plan_create(const tred_grid* grid, const tred_blocking* blocking,
                                    const int32_t kpix[2], int32_t kticks, uint32_t flags,
                                    int32_t batch, tred_direct_plan** plan,
                                    int64_t* workspace_bytes);
/* Convert the response to BF16 operands in `workspace` (256-byte aligned; kept by
 * the plan). Synchronises `stream`. */
tred_status tred_direct_plan_set_response(tred_direct_plan* plan, const float* resp,
                                          void* workspace, void* stream);
tred_status tred_block_conv_direct(const tred_direct_plan* plan, const int32_t* n_active,
                                   int32_t cap, const float* blocks, float* out_blocks,
                                   void* stream);
void tred_direct_plan_destroy(tred_direct_plan* plan);

/* ------------------------------------------------------------------------- */
/* Gradients (Sec. V-C: the simulation is differentiable, e.g. to fit the electron
 * lifetime). Each call is the transpose of the forward call of the same name for
 * the same inputs, plan, keys, pixel list and capacities: given dL/d(its outputs)
 * it returns dL/d(its inputs). Chained backwards they give dL/d(depositions) and
 * dL/d(transport parameters) for a loss L on the waveforms; the effective charge is
 * recomputed, not stored.
 *
 * tred_scatter_waveforms_adjoint: d_wf [pix_cap][nticks + kticks - 1] in,
 *   d_out_blocks [cap][..] out (every sample of the active bins written: the
 *   gradient of its pixel's waveform at its tick, zero for pixels outside the region,
 *   pixels without a slot below pix_cap and ticks past the waveform end). */
tred_status tred_scatter_waveforms_adjoint(const tred_conv_plan* plan, const int32_t* keys,
                                           const int32_t* n_active, int32_t cap,
                                           const int32_t* pix, const int32_t* n_pix,
                                           int32_t pix_cap, const float* d_wf,
                                           float* d_out_blocks, void* stream);
/* tred_block_conv_adjoint: d_out_blocks in, d_blocks [cap][..] out (every cell of the
 *   active bins written). The correlation with the response by the same transforms:
 *   conj(FFT(R_j)) in the channel fan-out. Supported for spatial sizes 8, 16, 24, 40
 *   and 48 (TRED_EUNSUPPORTED otherwise); uses the plan's scratch like tred_block_conv. */
tred_status tred_block_conv_adjoint(const tred_conv_plan* plan, const int32_t* n_active,
                                    int32_t cap, const float* d_out_blocks, float* d_blocks,
                                    void* stream);
/* tred_block_conv_adjoint_rows: as tred_block_conv_adjoint, writing only the rows of
 * d_blocks marked in `rows` (row masks of tred_block_bin_rows; the other rows are left
 * as they were). tred_block_bin_adjoint reads d_blocks at patch cells only, which lie
 * in marked rows. */
tred_status tred_block_conv_adjoint_rows(const tred_conv_plan* plan, const int32_t* n_active,
                                         int32_t cap, const float* d_out_blocks,
                                         const uint32_t* rows, float* d_blocks, void* stream);
/* tred_block_bin_adjoint: d_blocks in, d_val [val_cap] out (each patch cell gets the
 *   gradient of its bin cell; zero for cells of bins beyond cap and for patches that
 *   end past val_cap). work: tred_block_bin_workspace() bytes (overwritten). */
tred_status tred_block_bin_adjoint(const tred_grid* grid, const tred_blocking* blocking,
                                   int64_t n_dep, const int32_t* fp, const int64_t* off,
                                   int64_t val_cap, const int32_t* keys, const int32_t* n_active,
                                   const float* d_blocks, int32_t cap, float* d_val, void* work,
                                   void* stream);
/* tred_effq_adjoint: d_val in; d_seg [n_dep][7] out: dL/d(x0, y0, z0, x1, y1, z1, Q) of
 *   every deposition (zero for depositions that miss the region or whose patch ends
 *   past val_cap); d_phys (may be NULL) [3] binary64, ACCUMULATED: dL/d(diff_T, diff_L,
 *   lifetime). The quadrature windows and the point/line decision are held fixed
 *   (they are piecewise constant in the inputs); widths at their floor sigma_min do
 *   not depend on t_mid or the diffusion constants. The node sums are binary64. */
tred_status tred_effq_adjoint(const tred_grid* grid, const tred_physics* phys, int64_t n_dep,
                              const float* seg, const int32_t* fp, const int64_t* off,
                              const float* d_val, int64_t val_cap, float* d_seg, double* d_phys,
                              void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TRED_H */

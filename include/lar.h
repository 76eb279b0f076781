/*
 * lar.h -- C ABI of the MI355X (gfx950) LArTPC signal-simulation hot path.
 *
 * The library computes the signal term of the LArTPC measurement model,
 * paper arXiv:2203.02479 Sec. 2.1 Eq. (1):  M = R (*) S, per wire plane on
 * the 2D (drift time x wire pitch) space, with the three tasks named in
 * Sec. 2.2 -- Raster (bin each diffused ionization group as a Gaussian
 * patch), Scatter-add (sum the patches into one dense grid, Sec. 2.3) and
 * Convolution (Sec. 2.2 Eq. (2): FT of the grid, product with the response
 * spectrum, inverse FT).
 *
 * Conventions shared by every call:
 *  - All array pointers are DEVICE pointers owned by the caller.  Structs
 *    (lar_plane, lar_depos, lar_fluct) are read from host memory during the
 *    call only.  `stream` is a hipStream_t (NULL = the null stream).
 *  - Calls are asynchronous on `stream`, never synchronise, never allocate
 *    device memory; scratch comes from a caller-provided workspace whose
 *    size the matching *_workspace() call reports.  The workspace must not
 *    be used by overlapping calls.
 *  - Return value: LAR_OK (0) or a negative LAR_E* code; on error nothing
 *    is launched, except LAR_EHIP (a launch failed; lar_last_hip_error()
 *    gives the hipError_t).
 *  - Grid layout: S[m][j], m = w*n_imp + k (impact row k of wire w; row m
 *    covers pitch [x0 - pitch/2 + m*d, +d) with d = pitch/n_imp), j = tick
 *    (covers [t0 + j*tick, +tick)); row-major, ticks contiguous,
 *    n_wires*n_imp rows of n_ticks floats.
 *  - Response spectrum layout: resp[k][p][f] complex (interleaved re, im
 *    float32), k < n_imp, p < nw_fft, f <= nt_fft/2: the 2D DFT over
 *    (nw_fft, nt_fft) of the response of impact offset k.
 *  - Waveforms: wave[w][j], n_wires rows of n_ticks floats.
 *  - Units: time and sigma_t in microseconds, x, pitch and sigma_x in mm,
 *    charge in electrons.
 */
#ifndef LAR_H
#define LAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LAR_OK = 0,
    LAR_EINVAL = -1,     /* null pointer, negative count, bad enum */
    LAR_ESIZE = -2,      /* FFT length not 2^a 3^b, too short, or beyond the kernel limits */
    LAR_EWORKSPACE = -3, /* workspace missing or smaller than required */
    LAR_EHIP = -4        /* a HIP launch failed; see lar_last_hip_error() */
};

/* Geometry of one wire plane and its FFT sizes (paper Sec. 2.1: each plane
 * is simulated on its own drift-time x wire-pitch space).
 * nt_fft: time FFT length Tf, even, 2^a 3^b, n_ticks <= Tf <= 16384; the
 *         convolution is circular over Tf (ticks n_ticks..Tf-1 hold zero).
 * nw_fft: wire FFT length Wf, 2^a 3^b, n_wires <= Wf <= 1024; circular over
 *         Wf, so Wf >= n_wires + 2H gives a linear convolution for a
 *         response spanning +-H wires. */
typedef struct lar_plane {
    int32_t n_wires;
    int32_t n_imp;      /* impact positions per pitch, >= 1 */
    int32_t n_ticks;
    int32_t nt_fft;
    int32_t nw_fft;
    float pitch;        /* wire pitch (mm) */
    float x0;           /* pitch coordinate of wire 0's centre (mm) */
    float tick;         /* sampling period (us) */
    float t0;           /* start time of tick 0 (us) */
} lar_plane;

/* Drifted, diffused depositions as a structure of arrays (paper Sec. 2.3:
 * SoA data objects, parallel over ionization groups).  n >= 0 entries each;
 * sigma_t is the longitudinal width in time units.  A depo with any
 * non-finite field is skipped; sigma < 1e-6 bin widths is a point charge. */
typedef struct lar_depos {
    const float *q, *t, *x, *sigma_t, *sigma_x;
    int64_t n;
} lar_depos;

/* The optional counter of skipped depos: *count (device, one int64, 8-byte
 * aligned, written on `stream`, not accumulated) = the number of depos with
 * a non-finite field, the ones every raster call skips.  Stream-ordered and
 * allocation-free (no memset node: a graph may capture it).  LAR_EINVAL for
 * a null depos, a null or misaligned count, or a depos that lar_raster would
 * reject (LAR_ESIZE above 2^32 depos). */
int lar_depos_nonfinite(const lar_depos *depos, int64_t *count, void *stream);

/* Charge fluctuation (paper Sec. 3.1: the reference code draws binomial
 * electron counts, the GPU port a normal approximation).  mode 0: mean
 * patch q*wt*wx; 1: Binomial(rint|q|, p) per bin; 2: Poisson(|q| p) per
 * bin; 3: the normal approximation of mode 1, rint(n p + sqrt(n p (1-p)) z)
 * clipped to [0, n], n = rint|q|, z = sqrt(-2 log u1) cos(2 pi u2) from the
 * bin's first two uniforms; p = wt*wx, sign(q) restored.  Draws
 * use Philox4x32-10 with key = seed and counter (depo index, event,
 * m*n_ticks + j, plane*2^24 + draw), so results are reproducible for any
 * launch shape.  NULL = mode 0.  plane < 256; with mode != 0 the grid's
 * n_wires*n_imp*n_ticks must not exceed 2^32 - 1 (the bin word), else
 * LAR_ESIZE. */
typedef struct lar_fluct {
    int32_t mode;
    uint32_t event;
    uint32_t plane;
    uint32_t reserved;
    uint64_t seed;
} lar_fluct;

const char *lar_status_str(int status);
int lar_last_hip_error(void);

/* Raster + scatter-add (paper Sec. 2.2 "Raster" and "Scatter-add").  For
 * every depo: the bins intersecting mu +- nsigma*sigma on each axis, the
 * Gaussian bin integrals Phi(z_{j+1}) - Phi(z_j) (no renormalisation), the
 * patch q*wt[j]*wx[m] (or its fluctuated counts) ADDED into grid.
 * grid: [n_wires*n_imp][n_ticks] float, accumulated (+=), not cleared.
 * nsigma > 0.  Float atomics: the summation order, and so the last bits of
 * the grid, depend on scheduling (fluctuated counts are integers and sum
 * exactly below 2^24).
 * Workspace: none for the mean patch (ws may be NULL); a fluctuated raster
 * queues in it (16 bytes each) the rejection-regime bins that the first
 * try's immediate acceptance does not decide, and draws them in later
 * kernels.  lar_raster_workspace gives the recommended size for n_depos
 * (room for 48 such bins per depo); any size of
 * at least the size it gives for n_depos = depos->n with a queue of zero
 * (the sum of a 256-byte header and one byte per 16 depos, rounded up to
 * 256) is accepted and gives the same counts, a smaller queue only moves
 * work to a slower path (mode 3 queues nothing: the header and flags are
 * all it needs).  The workspace must be 256-byte aligned. */
int lar_raster_workspace(const lar_plane *plane, int64_t n_depos, const lar_fluct *fluct,
                         size_t *bytes);
int lar_raster(const lar_plane *plane, const lar_depos *depos, float nsigma,
               const lar_fluct *fluct, float *grid, void *workspace, size_t ws_bytes,
               void *stream);

/* Convolution of a grid with the response spectra (paper Sec. 2.2 Eq. (2)):
 * wave = crop_{n_wires x n_ticks} IFT2( sum_k resp[k] * FT2(S_k) ), where
 * S_k[w][j] = grid[w*n_imp + k][j] zero-padded to (nw_fft, nt_fft), FT2 is
 * a real FFT over time then a complex FFT over wires (unnormalised), and
 * IFT2 the inverse (1/(nw_fft*nt_fft)) whose real inverse in time takes the
 * real part of the DC and Nyquist columns.  wave is overwritten. */
int lar_fftconv_workspace(const lar_plane *plane, size_t *bytes);
int lar_fftconv(const lar_plane *plane, const float *grid, const float *resp, float *wave,
                void *workspace, size_t ws_bytes, void *stream);

/* lar_fftconv for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result as lar_fftconv, with the spectra held in a
 * fixed device array of lar_fftconv_noalloc_max_bytes() bytes (256 MiB,
 * one per GPU the library runs on, kept until the process ends) instead of
 * a workspace.  A plane whose lar_fftconv workspace exceeds that size gets
 * LAR_ESIZE (n_wires * n_imp + n_wires rows of (nt_fft/2 + 1, rounded up to
 * 16) complex64 must fit: e.g. 8000 + 800 rows at nt_fft = 6144).  Nothing
 * is allocated; the array's address is looked up on the first call on each
 * device.  Every call on one GPU shares the array: calls that overlap on
 * one GPU (several streams or threads) race and must be serialised by the
 * caller.  The array holds the last call's spectra; nothing in it needs to
 * start at zero. */
size_t lar_fftconv_noalloc_max_bytes(void);
int lar_fftconv_noalloc(const lar_plane *plane, const float *grid, const float *resp, float *wave,
                        void *stream);

/* One plane end to end: clear an internal grid, lar_raster, lar_fftconv.
 * The workspace covers the grid, the raster's queue for n_depos depos and
 * the convolution's buffers. */
int lar_sim_plane_workspace(const lar_plane *plane, int64_t n_depos, const lar_fluct *fluct,
                            size_t *bytes);
int lar_sim_plane(const lar_plane *plane, const lar_depos *depos, float nsigma,
                  const lar_fluct *fluct, const float *resp, float *wave,
                  void *workspace, size_t ws_bytes, void *stream);

/* Adjoint of lar_fftconv (gradients of a loss L through wave = conv(grid,
 * resp); no paper counterpart, the transpose of Eq. (2)).  With G =
 * dL/dwave [n_wires][n_ticks] and FT2/IFT2 as in lar_fftconv:
 *  grid_grad[w*n_imp + k][j] = crop IFT2( conj(resp[k]) * FT2(G) )
 *      (OVERWRITTEN; exact for any resp),
 *  resp_grad[k][p][f] += c_f/(nw_fft*nt_fft) * FT2(G)[p][f] * conj(FT2(S_k)[p][f])
 *      (ACCUMULATED, as d/dRe + i d/dIm; c_f = 1 at f = 0 and nt_fft/2, else 2).
 * Either output may be NULL; grid may be NULL when resp_grad is. */
int lar_fftconv_backward_workspace(const lar_plane *plane, size_t *bytes);
int lar_fftconv_backward(const lar_plane *plane, const float *grid, const float *resp,
                         const float *wave_grad, float *grid_grad, float *resp_grad,
                         void *workspace, size_t ws_bytes, void *stream);

/* lar_fftconv_backward with the grid given by its time spectrum: after
 * lar_fftconv returns, its workspace begins with grid_spec, the real FFT
 * over ticks of every grid row, [n_wires*n_imp][ld] complex64 (float
 * pairs), ld = nt_fft/2 + 1 rounded up to a multiple of 16.  Keeping that
 * workspace for the backward pass saves the transform of the grid.
 * grid_spec is only read, so the same spectrum serves any number of
 * backward calls.  resp_accumulate != 0: resp_grad += gradient, as in
 * lar_fftconv_backward; 0: resp_grad = gradient.  Workspace
 * (lar_fftconv_backward_spec_workspace): the FT of wave_grad and the
 * grid-gradient spectrum. */
int lar_fftconv_backward_spec_workspace(const lar_plane *plane, size_t *bytes);
int lar_fftconv_backward_spec(const lar_plane *plane, const void *grid_spec, const float *resp,
                              const float *wave_grad, float *grid_grad, float *resp_grad,
                              int32_t resp_accumulate, void *workspace, size_t ws_bytes,
                              void *stream);

/* Adjoint of the mean raster (no paper counterpart): for every depo the
 * gradient of L = sum grid_grad * S with respect to q, t, x, sigma_t,
 * sigma_x, windows held fixed (the patch is recomputed, not stored):
 *  dq = sum G wt wx, dt = q sum G (dwt/dt) wx, dsigma_t = q sum G (dwt/dsigma_t) wx,
 *  and likewise for x and sigma_x, with dw/dmu = -(phi(z_b) - phi(z_a))/sigma and
 *  dw/dsigma = -(z_b phi(z_b) - z_a phi(z_a))/sigma.  Point axes and skipped
 * depos get zero.  Outputs: n floats each, OVERWRITTEN.  No workspace. */
int lar_raster_backward(const lar_plane *plane, const lar_depos *depos, float nsigma,
                        const float *grid_grad, float *dq, float *dt, float *dx,
                        float *dsigma_t, float *dsigma_x, void *stream);

/* Response spectrum from a time-domain response (detector response R of
 * Eq. (1), paper Sec. 2.1): r_time[k][dw + half_w][tau], k < n_imp,
 * |dw| <= half_w, tau < n_rt, placed at wire index dw mod nw_fft and tick
 * tau, then resp = FT2 (as in lar_fftconv).  resp is overwritten. */
int lar_response_spectrum_workspace(const lar_plane *plane, int32_t half_w, int32_t n_rt,
                                    size_t *bytes);
int lar_response_spectrum(const lar_plane *plane, const float *r_time, int32_t half_w,
                          int32_t n_rt, float *resp, void *workspace, size_t ws_bytes,
                          void *stream);

/* The per-bin sampler of lar_raster on injected inputs (same device code):
 * out[i] = sign(q[i]) * n with n ~ Binomial(rint|q[i]|, p[i]) (mode 1),
 * Poisson(|q[i]| p[i]) (mode 2) or the normal approximation of the
 * binomial (mode 3), counter (ctr3[3i], ctr3[3i+1], ctr3[3i+2],
 * plane*2^24 + draw), key = seed.  p is double (the sampler's precision). */
int lar_sample_counts(int32_t mode, int64_t n, const float *q, const double *p,
                      const uint32_t *ctr3, uint32_t plane, uint64_t seed, float *out,
                      void *stream);

/* ---------------------------------------------------------------- drift
 * The drift of ionization groups to the anode, upstream of the raster
 * (paper Sec. 2.2: a group is diffused while it drifts, so it reaches the
 * wires as a 2D Gaussian over drift time and wire pitch).  Per group, in
 * FP64 from the float32 inputs, each output rounded once to float32:
 *   td = max(xd, 0) / speed                      (drift time, us)
 *   q  = q0 * exp(-td / lifetime)                (lifetime <= 0: q = q0)
 *   t  = t0 + td,  sigma_t = sqrt(2 diff_l td) / speed  (time units),
 *   sigma_x = sqrt(2 diff_t td),
 *   x[p] = z * proj[p].cos + y * proj[p].sin + proj[p].offset
 * for each of the n_planes wire planes (the pitch coordinate on plane p).
 * Units: mm, us, electrons.  The outputs form the lar_depos of each plane
 * (q, t, x[p], sigma_t, sigma_x). */
typedef struct lar_drift_params {
    float speed;      /* drift speed v (mm/us), > 0 */
    float diff_l;     /* longitudinal diffusion constant D_L (mm^2/us), >= 0 */
    float diff_t;     /* transverse diffusion constant D_T (mm^2/us), >= 0 */
    float lifetime;   /* electron lifetime (us); <= 0 means no attenuation */
} lar_drift_params;

typedef struct lar_plane_proj {
    float cos_a, sin_a, offset;   /* x = z cos_a + y sin_a + offset (mm) */
} lar_plane_proj;

/* Inputs (device, n floats each): q0 (electrons at creation), t0 (creation
 * time, us), xd (distance to the anode along the drift, mm), y, z (mm).
 * proj: n_planes entries in HOST memory, 0 <= n_planes <= 8.  Outputs
 * (device, OVERWRITTEN): q, t, sigma_t, sigma_x (n floats each) and x
 * ([n_planes][n] floats; may be NULL when n_planes = 0).  No workspace. */
int lar_drift(const lar_drift_params *prm, const float *q0, const float *t0, const float *xd,
              const float *y, const float *z, int64_t n, const lar_plane_proj *proj,
              int32_t n_planes, float *q, float *t, float *sigma_t, float *sigma_x, float *x,
              void *stream);

/* Adjoint of lar_drift (no paper counterpart): gradients of
 * L = sum(gq q + gt t + gsigma_t sigma_t + gsigma_x sigma_x + sum_p gx[p] x[p])
 * with respect to the inputs (dq0, dt0, dxd, dy, dz: n floats each,
 * OVERWRITTEN, each may be NULL) and to the four parameters (dparams: 4
 * floats (speed, diff_l, diff_t, lifetime), OVERWRITTEN, may be NULL),
 * summed over the groups in a fixed order (deterministic).  Where xd <= 0,
 * or a width is zero, the derivative terms through td or through that
 * width's square root are zero.  gx: [n_planes][n] (may be NULL when
 * n_planes = 0).  Workspace (for dparams): lar_drift_backward_workspace. */
int lar_drift_backward_workspace(int64_t n, size_t *bytes);
int lar_drift_backward(const lar_drift_params *prm, const float *q0, const float *xd, int64_t n,
                       const lar_plane_proj *proj, int32_t n_planes, const float *gq,
                       const float *gt, const float *gsigma_t, const float *gsigma_x,
                       const float *gx, float *dq0, float *dt0, float *dxd, float *dy, float *dz,
                       float *dparams, void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- noise, ADC
 * The noise term N(t,x) of Eq. (1) (paper Sec. 2.1; Sec. 2.2 leaves it out
 * of the port) and the digitisation downstream of the convolution.
 * lar_noise: per wire w < n_wires a random half spectrum
 *   X[w][f] = amp[f] (g_re + i g_im),  f <= nt_fft/2,
 * with (g_re, g_im) the Box-Muller cosine and sine normals of the two
 * uniforms of Philox4x32-10 block (w, event, f, plane*2^24 + 2^23), key =
 * seed (bit 23 of the last word keeps it apart from the raster's draws);
 * the DC and Nyquist bins are real.  noise = the inverse real FFT over
 * nt_fft (1/nt_fft) cropped to [n_wires][n_ticks], OVERWRITTEN.  amp:
 * nt_fft/2 + 1 floats (device).  plane < 256.  Workspace:
 * lar_noise_workspace. */
int lar_noise_workspace(const lar_plane *plane, size_t *bytes);
int lar_noise(const lar_plane *plane, const float *amp, uint64_t seed, uint32_t event,
              uint32_t plane_id, float *noise, void *workspace, size_t ws_bytes, void *stream);

/* ADC codes: adc[i] = clip(rint(gain * v + baseline), 0, 2^bits - 1) with
 * v = wave[i] + noise[i] (noise may be NULL), each operation a float32
 * operation rounded on its own (no fused multiply-add), rint ties to even,
 * a NaN voltage gives 0.  1 <= bits <= 16.  n >= 0 elements. */
int lar_digitize(const float *wave, const float *noise, int64_t n, float gain, float baseline,
                 int32_t bits, uint16_t *adc, void *stream);

/* ---------------------------------------------------------------- batching
 * Many (event, plane) items in few launches (no paper counterpart: the
 * paper raises throughput by running independent processes per GPU,
 * Sec. 3.3).  Items are grouped by plane type; each type's items run in
 * waves of at most K items, K the largest that the given workspace holds:
 * per wave one raster launch over the wave's items (their table is built on
 * the device by a prefix sum of their depo sub-chunks) and one launch per
 * FFT stage, the response spectrum of the type shared by the wave's items.
 * Each item's waveforms equal those of lar_sim_plane on the same depos with
 * fluct {mode, event, plane, seed} (fluctuated counts exactly; mean grids up
 * to float summation order). */
typedef struct lar_batch_item {
    int32_t plane_type;     /* index into planes[] and resp[] */
    uint32_t event;         /* fluctuation counter words of this item */
    uint32_t plane;         /* < 256 */
    int32_t reserved;
    int64_t depo_offset;    /* first depo of the item in the concatenated arrays */
    int64_t n_depos;
    int64_t wave_offset;    /* first float of the item's [n_wires][n_ticks] waveforms */
} lar_batch_item;

typedef struct lar_batch lar_batch;    /* opaque plan */

/* Workspace for waves of at most max_wave items per plane type (0: every
 * item of a type in one wave, the most the plan can use): item tables,
 * one wave's grids, time spectra and wire-pass outputs (an arena shared by
 * every wave), with more than one wave a second region of one wave's grids
 * (waves alternate between the two, so that a wave's FFT stages overlap the
 * next wave's raster), and the raster queue of the largest wave (fluct
 * only).
 * lar_batch_workspace(...) = lar_batch_workspace_waves(..., 0, ...).
 * n_items < 2^27 (LAR_ESIZE otherwise). */
int lar_batch_workspace_waves(const lar_plane *planes, int32_t n_types, const lar_batch_item *items,
                              int32_t n_items, const lar_fluct *fluct, int32_t max_wave,
                              size_t *bytes);
int lar_batch_workspace(const lar_plane *planes, int32_t n_types, const lar_batch_item *items,
                        int32_t n_items, const lar_fluct *fluct, size_t *bytes);

/* Build a plan for these exact device buffers: depos holds all items'
 * depos (concatenated), resp[t] the spectrum of plane type t, wave the
 * output.  The waves are as large as ws_bytes allows (every type in one
 * wave when that fits; LAR_EWORKSPACE when not even one item per wave
 * fits).  Uploads the tables to the workspace (a synchronous copy) and, with
 * use_graph, captures the whole sequence into a hipGraph.  The contents of
 * depos / resp may change between runs; their addresses and the item
 * counts may not.  Setup call: it allocates host memory, the graph, the
 * events that order the plan's two streams and (without use_graph) the
 * second stream, all released by lar_batch_destroy. */
int lar_batch_create(const lar_plane *planes, int32_t n_types, const float *const *resp,
                     const lar_depos *depos, float nsigma, const lar_fluct *fluct,
                     const lar_batch_item *items, int32_t n_items, float *wave, void *workspace,
                     size_t ws_bytes, int32_t use_graph, lar_batch **plan);
/* The plan's wave count and largest wave (either pointer may be NULL). */
int lar_batch_waves(const lar_batch *plan, int32_t *n_waves, int32_t *max_items);
/* Run the plan on `stream` (one graph launch with use_graph).  The FFT
 * stages run on a second stream forked from `stream` and joined back before
 * the call's work on `stream` ends, so later work on `stream` sees the
 * waveforms. */
int lar_batch_run(lar_batch *plan, void *stream);

/* Backward of a mean-path plan (fluct NULL or mode 0; LAR_EINVAL
 * otherwise), the batched form of lar_fftconv_backward + lar_raster_backward
 * (no paper counterpart): for L with dL/dwave = wave_grad (the layout of
 * wave), per wave of items, last wave first: the grids and their time
 * spectra are recomputed (patches are not stored) -- except for the last
 * wave when lar_batch_run was the plan's previous call (its spectra are
 * still in the workspace; both calls on the same stream) --, the waveform
 * gradients transformed,
 * the adjoint wire pass runs over the wave's items with the response
 * gradient of each tile summed over the items in registers, then the grid
 * gradients and the depo gradients.
 *   resp_grad[t] ([n_imp][nw_fft][nt_fft/2+1] complex, as resp) =
 *       the sum over the items of type t of their response gradients,
 *       OVERWRITTEN (types without items untouched); resp_grad or any
 *       entry may be NULL;
 *   dq, dt, dx, dsigma_t, dsigma_x: the layout of the depo arrays, each
 *       item's depos OVERWRITTEN with their gradients; all five or none.
 * Uses the plan's workspace (do not overlap with lar_batch_run); eager
 * launches on `stream`. */
int lar_batch_backward(lar_batch *plan, const float *wave_grad, float *const *resp_grad, float *dq,
                       float *dt, float *dx, float *dsigma_t, float *dsigma_x, void *stream);
int lar_batch_destroy(lar_batch *plan);

/* ---------------------------------------------------------------- streams
 * Independent plane simulations sharing one GPU through several HIP
 * streams (the single-GPU form of the paper's several processes per GPU,
 * Sec. 3.3 and Fig. 4): item i (a lar_batch_item record) runs as
 * lar_sim_plane on its depos (depo_offset, n_depos) with fluct {mode,
 * item.event, item.plane, seed}, writing [n_wires][n_ticks] floats at
 * wave + wave_offset, on streams[i mod n_streams] with workspace slice
 * i mod n_streams.  The worker streams first wait for the work already on
 * `stream`, and `stream` then waits for them, so the call is ordered like
 * any other call on `stream`.  streams: 1..64 distinct hipStream_t, none
 * equal to `stream`, created by the caller (default priority).  Results
 * equal per-item lar_sim_plane calls (fluctuated counts exactly).
 * Workspace: lar_sim_streams_workspace (n_streams slices of the largest
 * item's lar_sim_plane workspace).  Events are created on the first call
 * of each host thread and kept. */
int lar_sim_streams_workspace(const lar_plane *planes, int32_t n_types, const lar_batch_item *items,
                              int32_t n_items, const lar_fluct *fluct, int32_t n_streams, size_t *bytes);
int lar_sim_streams(const lar_plane *planes, int32_t n_types, const float *const *resp,
                    const lar_depos *depos, float nsigma, const lar_fluct *fluct,
                    const lar_batch_item *items, int32_t n_items, float *wave, void *const *streams,
                    int32_t n_streams, void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- schedules
 * Launch schedule of the FFT convolution and of the raster for one plane
 * shape (no paper counterpart: a tuning knob of this implementation).  Every valid schedule
 * computes the same transform up to float rounding; which one is fastest
 * depends on the shape.  Schedules are keyed by (n_wires, n_imp, n_ticks,
 * nt_fft, nw_fft), process-wide, and read when a call launches its kernels
 * (lar_batch_create reads them once).  Radix orders 0..5 pick the order of
 * the radix-8/6/4/3/2 passes of a transform:
 *   0: 8s (then one 4 or 2), then 3s   1: 4s, 3s, then one 2
 *   2: 3s, then 8s (then one 4 or 2)  3: the reverse of 0
 *   4: 8s, then each remaining 2 paired with a 3 as a 6, then the rest
 *   5: radix 6 first and last (needs 36 | n); between them 8s, a 4 or 2,
 *      6s, then 3s (864: 6 4 6 6) */
typedef struct lar_schedule {
    int32_t row_threads;    /* threads per time-axis row workgroup: 256, 384, 512, 768, 1024 */
    int32_t row_order;      /* radix order of the nt_fft/2-point plan */
    int32_t wire_cols;      /* time-frequency columns per wire-pass tile: 4, 8, 16 */
    int32_t wire_threads;   /* threads per wire-pass workgroup: 256, 512, 1024
                               (cols 4: 256/512; cols 16: 512/1024), or 576 with
                               cols 4 and the nw_fft = 864 plan 6 4 6 6 (order 5) */
    int32_t wire_order;     /* radix order of the nw_fft-point plan */
    int32_t raster_tile;    /* floats of a raster wave's LDS tile: 384, 512, 640, 768
                               (0 in lar_schedule_set: the built-in 512).  A wave sums
                               the patches of its 16 depos there when their bounding
                               box fits, else adds them straight to the grid; larger
                               tiles take more LDS per workgroup */
} lar_schedule;

/* The built-in schedule of a shape / the one in effect (registered or
 * built-in).  LAR_ESIZE if the shape has no valid FFT plan. */
int lar_schedule_default(const lar_plane *plane, lar_schedule *out);
int lar_schedule_get(const lar_plane *plane, lar_schedule *out);
/* Register sched for this shape (NULL: back to the built-in one).
 * LAR_EINVAL if a field is outside the lists above or a thread holds more
 * than 8 values of a transform (ceil(nt_fft/2 / row_threads) > 8,
 * ceil(nw_fft * wire_cols / wire_threads) > 8) or the wire tile exceeds the
 * 160 KB LDS of a CU.  Thread-safe; calls that overlap a change may launch
 * with either schedule. */
int lar_schedule_set(const lar_plane *plane, const lar_schedule *sched);
/* Valid schedules to time: the built-in one first, then every other row
 * choice with the built-in wire pass, then every other wire choice with the
 * built-in rows (radix orders that repeat an earlier order's plan are left
 * out), then every other raster tile with the built-in FFT choices.  Writes up to cap entries
 * and sets *n to the full count. */
int lar_schedule_candidates(const lar_plane *plane, lar_schedule *out, int32_t cap, int32_t *n);

/* Profiling aid (no paper counterpart): when events is non-NULL, the calls
 * on this host thread record events[i] (each a hipEvent_t created by the
 * caller) on their stream right after kernel stage i: 0 grid clear,
 * 1 raster main kernel, 2 rest of the raster (deferred draws, overflow,
 * wide depos), 3 time-axis real FFT, 4 wire pass, 5 time-axis inverse real
 * FFT (lar_raster records 1-2, lar_fftconv 3-5).  n_events must be >= 6;
 * pass NULL to stop.  Recording adds no synchronisation. */
int lar_set_stage_events(void *const *events, int32_t n_events);

/* Measurement aid (no paper counterpart): the peak rate of the global float
 * atomics the raster's tile flushes issue, for comparing the mean raster,
 * which they bound, against it.  Adds 1.0f to n_segments segments of 64
 * consecutive floats of buf (device, n_floats >= 64, 256-byte aligned), one
 * wave per segment, at segment slots spread over the buffer by a hash; buf
 * keeps the sums.  Asynchronous on stream.  LAR_EINVAL for a null or
 * misaligned buf, n_floats < 64 or n_segments < 0. */
int lar_atomic_probe(float *buf, int64_t n_floats, int64_t n_segments, void *stream);

/* Measurement aid (no paper counterpart): the rate of the raster's per-bin
 * draw, one Philox4x32-10 block and its 52-bit uniform, for comparing the
 * raster kernels against it.  n_threads threads (a positive multiple of 256)
 * draw the blocks of counters (i, 0x5EED, i >> 32, 0), i < n_blocks, under
 * a fixed key, thread t taking i = t, t + n_threads, ...; out[t] (device,
 * n_threads doubles) receives the sum of thread t's first uniforms.
 * Asynchronous on stream.  LAR_EINVAL for a null or misaligned out,
 * n_threads not a positive multiple of 256, or n_blocks < 0. */
int lar_philox_probe(double *out, int64_t n_threads, int64_t n_blocks, void *stream);

/* Measurement aid (no paper counterpart): the memory floor of the time
 * R2C's access pattern, for comparing that transform against it.  Copies
 * n_rows rows with the transform's persistent grid (blocks_per_cu
 * workgroups of 384 threads per compute unit, 1..16) and loads: input row
 * r (device, n_in floats at in + r*ld_in; n_in even, 2..6144) is read as
 * n_in/2 float pairs, and output row r (device, n_out complex values of 8
 * bytes at out + r*ld_out complex; n_out 1..3073) receives pair k at
 * element k for k < n_in/2, the last pair at the elements after it.  Both
 * buffers 8-byte aligned, ld_in even, ld_in >= n_in, ld_out >= n_out.
 * Asynchronous on stream.  LAR_EINVAL for arguments outside these ranges;
 * nothing is launched for n_rows == 0. */
int lar_row_copy_probe(const float *in, int64_t ld_in, int32_t n_in, int32_t n_rows, void *out, int64_t ld_out,
                       int32_t n_out, int32_t blocks_per_cu, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LAR_H */

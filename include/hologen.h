/*
 * hologen.h -- C ABI of the MI355X (gfx950) iterative Fourier-transform
 * hologram library: Gerchberg-Saxton and One-Step Phase-Retrieval holograms,
 * Fourier or Fresnel, phase-only, multi-level or binary SLMs.
 *
 * The calls follow the way the paper's algorithm objects receive a problem:
 * an algorithm object stores the target, illumination and starting images and
 * the common parameters, moves them to the GPU, and runs the iterations in
 * RunIterations() (Sec. 4, Algorithm Interface; Sec. 7.3, AlgorithmCuda).  The
 * plan descriptor carries the SLM resolution and type (Sec. 3.2, the
 * SLMResolutionX / SLMTypeOption / MultiAmpSLM options), the Fourier or
 * Fresnel propagation (Abstract keywords) and the quantiser levels (Sec. 7.3,
 * QuantiserCuda).
 *
 * Conventions shared by every call
 *   - Arrays are row-major [height][width]; width is the contiguous axis.
 *   - Complex arrays are interleaved complex64 (float re, float im).
 *   - SLM-plane arrays (phase, levels, illumination) are in natural pixel
 *     order.  Replay-plane arrays (targets, OSPR subframe phases, OSPR
 *     intensity, Fresnel output fields) are in centred image order: the
 *     optical axis sits at (height/2, width/2) (integer division).
 *   - Forward transform: X[k] = sum_n x[n] exp(-2 pi i n k / N), unnormalised;
 *     inverse: exp(+2 pi i n k / N) scaled by 1/N.  2D = rows then columns.
 *   - Every pointer argument except the plan descriptor and out-parameters is
 *     a DEVICE pointer owned by the caller; the library never frees it.  The
 *     plan owns only small tables (twiddles, chirps, level values).
 *   - Calls validate all host-visible arguments first and return a status
 *     without enqueueing anything when validation fails.  On success the work
 *     is enqueued on `stream` (0 = the null stream) and the results are valid
 *     once the stream has been synchronised.  Launch failures return
 *     HG_ERR_DEVICE; hg_error() then gives the HIP error text.
 *   - A plan is immutable after creation and may be used from several host
 *     threads and streams at once if every concurrent call has its own
 *     workspace.  Using a plan after hg_plan_destroy is undefined.
 */
#ifndef HOLOGEN_H
#define HOLOGEN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hg_plan_s* hg_plan;

typedef enum {
  HG_OK = 0,
  HG_ERR_INVALID_ARGUMENT = 1, /* null pointer, bad enum, non-finite optics, ... */
  HG_ERR_UNSUPPORTED_SIZE = 2, /* a dimension with no compiled transform        */
  HG_ERR_OUT_OF_MEMORY = 3,    /* plan tables could not be allocated            */
  HG_ERR_DEVICE = 4,           /* a HIP call or kernel launch failed            */
  HG_ERR_INTERNAL = 5
} hg_status;

enum { HG_FOURIER = 0, HG_FRESNEL = 1, HG_ANGULAR = 2 };                               /* propagation */
enum { HG_PHASE = 0, HG_PHASE_QUANTISED = 1, HG_BINARY_PHASE = 2,
       HG_AMPLITUDE = 3 };                                        /* SLM modulation */
enum { HG_FORWARD = 1 /* SLM -> replay */, HG_INVERSE = -1 /* replay -> SLM */ };

typedef struct {
  int32_t width, height;   /* SLM resolution in pixels; each must be a compiled
                              transform length (hg_length_supported): 16, 24,
                              32, 60, 64, 90, 120, 128, 256, 512, 1024, 1080,
                              1280, 1536, 1920, 2048, 2160, 3840, 4096, 8192;
                              any other value returns HG_ERR_UNSUPPORTED_SIZE
                              (HG_ERR_INVALID_ARGUMENT outside [2, 8192])      */
  int32_t propagation;     /* HG_FOURIER, HG_FRESNEL or HG_ANGULAR               */
  double wavelength;       /* metres; Fresnel, angular: finite and > 0           */
  double pixel_pitch;      /* metres; Fresnel, angular: finite and > 0; angular
                              also needs pixel_pitch > wavelength / sqrt(2), so
                              that no sampled plane wave is evanescent          */
  double distance;         /* metres; Fresnel: finite and > 0; angular: finite
                              (negative propagates backwards)                   */
  int32_t modulation;      /* HG_PHASE, HG_PHASE_QUANTISED, HG_BINARY_PHASE or
                              HG_AMPLITUDE (continuous amplitude-only SLM: the
                              SLM-plane constraint is the nearest non-negative
                              real value, see hg_gs_iterate)                    */
  int32_t levels;          /* 0 for HG_PHASE and HG_AMPLITUDE; 2..256 for
                              HG_PHASE_QUANTISED; 2 for HG_BINARY_PHASE          */
} hg_plan_desc;

/* Create a plan on the current HIP device: validates the descriptor, builds
 * the FP64 twiddle, chirp and level tables, rounds them to FP32 and copies
 * them to the device (synchronously).  *out is set only on HG_OK. */
hg_status hg_plan_create(const hg_plan_desc* desc, hg_plan* out);

/* Free the plan's device tables.  The caller must make sure no enqueued work
 * still uses the plan.  NULL is accepted and ignored. */
hg_status hg_plan_destroy(hg_plan plan);

/* Bytes of device workspace every hg_propagate / hg_gs_iterate / hg_ospr call
 * on this plan needs (a complex64 field plus reduction scratch).  0 for NULL. */
size_t hg_workspace_bytes(hg_plan plan);

/* 1 if the library compiles a transform of length n (usable as a width or a
 * height), else 0. */
int32_t hg_length_supported(int32_t n);

/* Propagate one complex64 field between the SLM and replay planes.
 *   HG_FOURIER: forward = 2D FFT, inverse = 2D inverse FFT (x 1/(H W)); both
 *               in FFT index order (the raw transform).
 *   HG_FRESNEL: the single-FFT Fresnel transform and its exact inverse:
 *       U_z = c Q2 fftshift(FFT2(ifftshift(Q1 U_0))),
 *       Q1 = exp(i pi (xi^2 + eta^2)/(lambda z)) at xi = (n - W/2) p,
 *       Q2 = exp(i pi (x^2 + y^2)/(lambda z)) at x = (k - W/2) lambda z/(W p),
 *       c  = exp(i 2 pi z / lambda) / (i lambda z) * p^2;
 *     SLM field in natural order, replay field in centred order.
 *   HG_ANGULAR: angular-spectrum propagation on the SLM's own grid, a
 *     method variant added here (the transfer-function form of scalar
 *     diffraction: Goodman, Introduction to Fourier Optics, the angular
 *     spectrum of plane waves and its propagation); the
 *     paper itself names only Fourier and Fresnel holograms:
 *       U_z = IFFT2(FFT2(U_0) T),  T = exp(i 2 pi z sqrt(1/lambda^2 - fx^2 - fy^2))
 *     at fx = kx / (W p) for FFT index kx (kx - W from kx >= (W + 1) / 2 on),
 *     fy likewise; the inverse uses conj(T).  Both planes in natural order.
 * in and out may be the same buffer.  workspace may be NULL (unused). */
hg_status hg_propagate(hg_plan plan, const void* in_c64, void* out_c64, int32_t direction,
                       void* workspace, hipStream_t stream);

/* Gerchberg-Saxton error reduction (Sec. 7.3, HoloGenAlgGSCuda):
 *   T_f = ifftshift(target_amp);  H_0 = A exp(i C(phase_in))
 *   for k = 0..iterations:
 *     R_k = FFT2(Q1 H_k)            (Q1 = 1 for HG_FOURIER, the source chirp
 *                                    above for HG_FRESNEL)
 *     nmse[k] = NMSE(|R_k|^2, T_f^2); stop at k = iterations
 *     H_{k+1} = A P(conj(Q1) IFFT2(T_f R_k / |R_k|))
 * For a HG_ANGULAR plan R_k = AS_z(H_k), H_{k+1} = A P(AS_-z(T_f R_k / |R_k|))
 * with the angular-spectrum operator of hg_propagate and T_f = target_amp
 * (no shift: the replay plane keeps the SLM's natural order).
 * with P = phase-only projection G/|G| (HG_PHASE) or the uniform quantiser
 * l = floor(mod(arg G, 2 pi) L / (2 pi) + 1/2) mod L, value exp(2 pi i l / L)
 * (HG_PHASE_QUANTISED, and HG_BINARY_PHASE with L = 2); C is the identity or
 * the same quantiser applied to the starting phase.
 *   NMSE(I, T) = sum (I/sum I - T/sum T)^2 / sum (T/sum T)^2, full frame, with
 *   sum I = H W sum A^2 (Parseval).
 * target_amp   [H][W] float, centred, >= 0, not all zero.      (required)
 * illumination [H][W] float SLM amplitude A; NULL means A = 1.
 * phase        [H][W] float: in = starting phase (radians, finite), out =
 *              phase of H_iterations in [0, 2 pi).             (required)
 * levels       [H][W] uint8 level index of H_iterations (0 in HG_PHASE mode);
 *              NULL to skip.
 * nmse         [iterations + 1] float; NULL to skip the error metric.
 * iterations   >= 0.
 * workspace    hg_workspace_bytes(plan) bytes of device memory.  (required)
 *
 * HG_AMPLITUDE plans (HG_FOURIER or HG_FRESNEL; no illumination): an
 * amplitude-only SLM, whose SLM types the paper names without defining them
 * (Sec. 3.2, SLMTypeOption, MultiAmpSLM).  Read here as the continuous
 * amplitude modulator under uniform illumination: H = a with a real a >= 0,
 * and P(G) = max(Re G, 0), the nearest such value (Fienup 1982).  `phase`
 * then holds the SLM amplitude instead of a phase: in = starting amplitude
 * a_0 (finite; negative values constrain to 0), out = a_n of the last state
 * at the scale of the normalised inverse transform (a_0 itself when
 * iterations = 0); levels receives 0.  The field energy changes between
 * states, so sum I is summed rather than taken from Parseval. */
hg_status hg_gs_iterate(hg_plan plan, const float* target_amp, const float* illumination, float* phase,
                        uint8_t* levels, float* nmse, int32_t iterations, void* workspace,
                        hipStream_t stream);

/* Gerchberg-Saxton with a signal window in the replay plane: the target is
 * imposed only inside the window, the rest of the replay plane keeps the light
 * the hologram sends there, and the error is measured inside the window.  The
 * paper's application lets a user draw masks over its images (Sec. 7.1,
 * HoloGenUIMask; Sec. 7.2, HoloGenMaskOptions) without saying how a mask
 * enters the iteration; this is the signal-window form of error reduction
 * (Fienup 1982; Wyrowski & Bryngdahl 1988):
 *   M = ifftshift(window) != 0;  c = sqrt(H W sum A^2 / sum_M T_f^2)
 *   R_k = FFT2(Q1 H_k);  nmse[k] = NMSE over M of (|R_k|^2, T_f^2)
 *   R'_k = c T_f R_k / |R_k| on M,  R_k off M;  H_{k+1} = A P(conj(Q1) IFFT2(R'_k))
 * with NMSE over M = sum_M (I/sum_M I - T/sum_M T)^2 / sum_M (T/sum_M T)^2
 * (1 when no light reaches the window).  c puts the window's target at the
 * field's energy, so each step is a nearest-point projection; a window
 * covering the frame gives the iterates of hg_gs_iterate (up to rounding).
 * window [H][W] uint8, centred like target_amp, nonzero inside (required);
 * the target must not vanish on the whole window (else the error and c are
 * not finite).  HG_FOURIER and HG_FRESNEL plans; other arguments, outputs and
 * the workspace (hg_workspace_bytes) as hg_gs_iterate. */
hg_status hg_gs_iterate_window(hg_plan plan, const float* target_amp, const uint8_t* window, const float* illumination,
                               float* phase, uint8_t* levels, float* nmse, int32_t iterations, void* workspace,
                               hipStream_t stream);

/* hg_gs_iterate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, bitwise the same results, with the workspace taken
 * from a static device array of HG_NOALLOC_WORKSPACE_MAX bytes that the
 * library holds on every device it runs on until the process ends.  The
 * caller passes inputs and outputs only; the call allocates nothing (its
 * first call on a device looks up that device's array).  Every call on one
 * device shares that array and overwrites it, so calls that overlap on one
 * device (other streams, other host threads) race: serialise them.  The
 * passes write every workspace byte they read, so nothing needs clearing
 * between calls.  Errors: HG_ERR_UNSUPPORTED_SIZE when hg_workspace_bytes(plan)
 * exceeds HG_NOALLOC_WORKSPACE_MAX (every frame up to 2048 x 2048 fits);
 * other arguments and errors as hg_gs_iterate. */
#define HG_NOALLOC_WORKSPACE_MAX (64u << 20)
hg_status hg_gs_iterate_noalloc(hg_plan plan, const float* target_amp, const float* illumination, float* phase,
                                uint8_t* levels, float* nmse, int32_t iterations, hipStream_t stream);

/* Gerchberg-Saxton on a batch of same-shape holograms in one launch per pass:
 * exactly hg_gs_iterate applied to each item b < batch (bitwise the same
 * results), with every pass launched once over all items, so that many small
 * holograms fill the GPU together.  Holograms of several shapes run as one
 * call per shape on one stream.  Item b uses target_amp + b H W,
 * phase + b H W, levels + b H W and nmse + b (iterations + 1); the
 * illumination (or NULL) is shared.  1 <= batch <= 65535 and
 * batch H Wt < 2^32 (Wt = W rounded up to a multiple of the plan's field
 * tile width, at most 8).  workspace: hg_workspace_bytes_batched(plan, batch)
 * bytes (the fields of all items are resident together).  HG_FOURIER and
 * HG_FRESNEL plans only (HG_ANGULAR: HG_ERR_INVALID_ARGUMENT). */
size_t hg_workspace_bytes_batched(hg_plan plan, int32_t batch);
hg_status hg_gs_iterate_batched(hg_plan plan, int32_t batch, const float* target_amp, const float* illumination,
                                float* phase, uint8_t* levels, float* nmse, int32_t iterations, void* workspace,
                                hipStream_t stream);

/* One-Step Phase-Retrieval, binary phase (Sec. 7.3, HoloGenAlgOSPRCuda), on a
 * HG_FOURIER plan:
 *   for n < n_sub: G_n = IFFT2(ifftshift(target_amp exp(i sub_phase[n])));
 *                  h_n = +1 (level 0) if Re G_n >= 0 else -1 (level 1);
 *                  I_n = |FFT2(h_n)|^2
 *   intensity = fftshift(mean_n I_n),  nmse[0] = NMSE(intensity, target_amp^2).
 * target_amp [H][W] float centred (required); sub_phase [n_sub][H][W] float
 * centred (required); holograms [n_sub][H][W] uint8 levels or NULL; intensity
 * [H][W] float centred (required); nmse [1] float or NULL; n_sub >= 1. */
hg_status hg_ospr(hg_plan plan, const float* target_amp, const float* sub_phase, int32_t n_sub,
                  uint8_t* holograms, float* intensity, float* nmse, void* workspace, hipStream_t stream);

/* Multi-plane Gerchberg-Saxton, one replay plane after another: each of the
 * `iterations` iterations runs one GS step per plane j = 0..n_planes-1 on
 * the same SLM state,
 *   R_j = FFT2(Q1_j H);  H = A P(conj(Q1_j) IFFT2(T_j R_j / |R_j|)),
 * with Q1_j the source chirp of plans[j] (1 for a HG_FOURIER plan; no
 * HG_ANGULAR plans) and P and the start constraint as in hg_gs_iterate.  All
 * plans share width, height, modulation and levels.  target_amp [n_planes][H][W] centred; phase, levels
 * and illumination as in hg_gs_iterate.  nmse [iterations * n_planes +
 * n_planes] or NULL: the error of every step (plane j of iteration k at
 * k n_planes + j), then of the final state at every plane.
 * workspace: hg_multiplane_workspace_bytes(plans[0], n_planes) bytes. */
size_t hg_multiplane_workspace_bytes(hg_plan plan, int32_t n_planes);
hg_status hg_gs_multiplane(const hg_plan* planes, int32_t n_planes, const float* target_amp,
                            const float* illumination, float* phase, uint8_t* levels, float* nmse,
                            int32_t iterations, void* workspace, hipStream_t stream);

/* Multi-plane GS on a batch of same-shape problems in one launch per pass:
 * exactly hg_gs_multiplane applied to each problem b < batch (bitwise the
 * same results), every pass launched once over all problems.  Problem b uses
 * target_amp + b n_planes H W ([batch][n_planes][H][W]), phase + b H W,
 * levels + b H W and nmse + b (iterations n_planes + n_planes); the
 * illumination (or NULL) is shared.  1 <= batch <= 65535 and batch H Wt <
 * 2^32 (Wt as for hg_gs_iterate_batched).  workspace:
 * hg_multiplane_workspace_bytes_batched(plans[0], n_planes, batch) bytes
 * (0 for arguments out of range).  Errors as hg_gs_multiplane. */
size_t hg_multiplane_workspace_bytes_batched(hg_plan plan, int32_t n_planes, int32_t batch);
hg_status hg_gs_multiplane_batched(const hg_plan* planes, int32_t n_planes, int32_t batch,
                                    const float* target_amp, const float* illumination, float* phase,
                                    uint8_t* levels, float* nmse, int32_t iterations, void* workspace,
                                    hipStream_t stream);

/* OSPR with real and imaginary subframe pairs, binary phase, on a HG_FOURIER
 * plan: one inverse transform per pair gives two subframes,
 *   G_n = IFFT2(ifftshift(target_amp exp(i sub_phase[n]))),
 *   h_2n = sign(Re G_n), h_2n+1 = sign(Im G_n)   (>= 0 -> +1 / level 0),
 *   intensity = fftshift(mean over the 2 n_pairs subframes of |FFT2 h|^2),
 *   nmse[0] = NMSE(intensity, target_amp^2).
 * Both subframes of a pair share one forward transform of h_2n + i h_2n+1;
 * their intensities are separated through the Hermitian symmetry of real
 * holograms.  holograms [2 n_pairs][H][W] uint8 or NULL; other arguments as
 * hg_ospr; n_pairs >= 1. */
hg_status hg_ospr_pairs(hg_plan plan, const float* target_amp, const float* sub_phase, int32_t n_pairs,
                        uint8_t* holograms, float* intensity, float* nmse, void* workspace, hipStream_t stream);

/* Single-pixel search on a HG_PHASE_QUANTISED or HG_BINARY_PHASE plan,
 * HG_FOURIER or HG_FRESNEL (Sec. 7.3: direct binary search HoloGenAlgDSCuda, simulated annealing
 * HoloGenAlgSACuda, single-pixel replay updates FFTUpdaterCuda).  The state
 * is the level map `levels` [H][W] uint8 (in: start, out: result; values
 * < L).  E = NMSE(|FFT2(Q1 exp(2 pi i l / L))|^2, ifftshift(target_amp)^2).
 * Trial k (device array trials [n_trials][2] int32) moves pixel
 * trials[k][0] = y W + x to level trials[k][1]; with dE the resulting change
 * of E it is accepted iff dE < 0 (direct search, temperature == uniform ==
 * NULL) or, annealing, iff dE < 0 or uniform[k] < exp(-dE / temperature[k])
 * (device float arrays [n_trials], temperature > 0 in NMSE units).  The
 * replay field is computed once per call and then updated in place by one
 * pass per trial.  A trial whose pixel or level is out of range (or whose
 * pixel holds a level >= L) is rejected without effect.
 * accepted [n_trials] uint8 or NULL; nmse [n_trials + 1] float or NULL: E of
 * the start state, then after each trial.
 * workspace: hg_search_workspace_bytes(plan) bytes. */
size_t hg_search_workspace_bytes(hg_plan plan);
hg_status hg_pixel_search(hg_plan plan, const float* target_amp, uint8_t* levels, const int32_t* trials,
                          int32_t n_trials, const float* temperature, const float* uniform, uint8_t* accepted,
                          float* nmse, void* workspace, hipStream_t stream);

/* Gradient-descent hologram optimisation: the method added beyond the
 * paper's library, whose further algorithms are left to future work (Sec. 8).
 * The parameter is the continuous SLM phase phi; each of the n_planes replay
 * planes j is given by its own plan (all of one width and height; HG_FOURIER
 * or HG_FRESNEL at its own distance, not HG_ANGULAR; modulation and levels
 * are ignored):
 *   V_j = Q1_j exp(i phi),  U_j = FFT2(V_j),  I_j = |U_j|^2
 *   L   = sum_j NMSE(I_j, ifftshift(target_amp_j)^2)   (NMSE as in hg_gs_iterate,
 *         sum I_j = (H W)^2 by Parseval)
 *   dL/dphi = sum_j 2 Im(conj(V_j) F^H(dL/dI_j * U_j)),  F^H = H W IFFT2,
 *   dL/dI_j = 2 (I_j/sum I_j - T_j/sum T_j) / (sum I_j sum (T_j/sum T_j)^2).
 * V_j is recomputed from phi in the adjoint pass, never stored.  A state
 * costs two launches whatever n_planes: one column pass over every plane and
 * one row pass that sums the planes' gradients in registers.
 * planes     [n_planes] plans, 1 <= n_planes <= 16.                 (required)
 * target_amp [n_planes][H][W] float, centred, >= 0, each not all zero.  (required)
 * workspace  hg_grad_workspace_bytes(planes[0], n_planes) bytes.    (required)
 * Invalid arguments return HG_ERR_INVALID_ARGUMENT before anything is enqueued. */
size_t hg_grad_workspace_bytes(hg_plan plan, int32_t n_planes);

/* One evaluation at phase [H][W] (read only): grad [H][W] float receives
 * dL/dphi, loss [1] float receives L; either may be NULL (both NULL: no work). */
hg_status hg_grad(const hg_plan* planes, int32_t n_planes, const float* target_amp, const float* phase,
                  float* grad, float* loss, void* workspace, hipStream_t stream);

/* `steps` Adam steps (Kingma & Ba 2015) on phase [H][W], in place:
 *   g = dL/dphi; m = beta1 m + (1 - beta1) g; v = beta2 v + (1 - beta2) g^2;
 *   phi -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 * t = first_step, first_step + 1, ...  adam_m and adam_v [H][W] float hold the
 * moments across calls (zero them before t = 1).  loss [steps + 1] float or
 * NULL: loss[k] = L of the phase before step k + 1, loss[steps] = L of the
 * returned phase.  steps >= 0, first_step >= 1, lr > 0, beta1 and beta2 in
 * [0, 1), eps > 0. */
hg_status hg_grad_adam(const hg_plan* planes, int32_t n_planes, const float* target_amp, float* phase,
                       float* adam_m, float* adam_v, int32_t steps, int32_t first_step, float lr, float beta1,
                       float beta2, float eps, float* loss, void* workspace, hipStream_t stream);

/* The gradient method on `batch` same-shape problems side by side: every
 * pass is one launch over all problems (grid.y = problem), and each
 * problem's results are bitwise those of the single-problem call.  Problem b
 * uses target_amp + b n_planes H W (its n_planes targets), phase, grad,
 * adam_m and adam_v + b H W, and loss + b (hg_grad_batched: one value) or
 * loss + b (steps + 1) (hg_grad_adam_batched); the planes are shared.
 * 1 <= batch, batch n_planes <= 65535 and batch n_planes H W' < 2^32 (W' = W
 * rounded up to the field's column-tile width).  workspace:
 * hg_grad_workspace_bytes_batched(planes[0], n_planes, batch) bytes (one
 * field per plane of every problem, resident together).  Other arguments and
 * errors as hg_grad / hg_grad_adam. */
size_t hg_grad_workspace_bytes_batched(hg_plan plan, int32_t n_planes, int32_t batch);
hg_status hg_grad_batched(const hg_plan* planes, int32_t n_planes, int32_t batch, const float* target_amp,
                          const float* phase, float* grad, float* loss, void* workspace, hipStream_t stream);
hg_status hg_grad_adam_batched(const hg_plan* planes, int32_t n_planes, int32_t batch, const float* target_amp,
                               float* phase, float* adam_m, float* adam_v, int32_t steps, int32_t first_step,
                               float lr, float beta1, float beta2, float eps, float* loss, void* workspace,
                               hipStream_t stream);

/* Diagnostics: per-kernel timing with HIP events.
 * hg_timing_begin makes every later launch of `kernel` made by calls on this
 * plan a timed launch on the call's stream, until hg_timing_end.
 * repeats == 1: the launch goes through hipExtLaunchKernel with a start/stop
 *   hipEvent pair that the runtime stamps from the dispatch itself.  Results
 *   are unchanged, but attaching the events costs the timed kernel about
 *   0.5-1 us of its own and shifts cache write-back work between it and the
 *   next kernel, so this mode overstates short kernels.
 * repeats > 1: the kernel is launched `repeats` times back to back with
 *   identical arguments, one hipEventRecord before the first and one after
 *   the last, so the average is the kernel's duration plus the small gap
 *   between back-to-back dispatches, with nothing attached to any launch.
 *   Every repeat rewrites the kernel's outputs from its inputs, so the
 *   numbers a call returns in this mode are not its results: use it for
 *   timing only.
 * hg_timing_end waits for the last event, returns the summed kernel time and
 * the number of kernel executions it covers (launches x repeats), and
 * switches timing off.  A plan in timing mode must be used from one host
 * thread.  Errors: HG_ERR_INVALID_ARGUMENT for an unknown kernel id or
 * repeats outside 1..1000.
 * kernel: HG_KERNEL_GS_REPLAY (column pass of GS: FFT, NMSE, amplitude
 * replacement, inverse FFT), HG_KERNEL_GS_SLM (row pass of GS: inverse FFT,
 * SLM constraint, FFT), HG_KERNEL_OSPR_A / _B / _C (the three OSPR passes),
 * HG_KERNEL_PROP_ROW / _COL (hg_propagate passes). */
enum { HG_KERNEL_GS_REPLAY = 1, HG_KERNEL_GS_SLM = 2, HG_KERNEL_OSPR_A = 3, HG_KERNEL_OSPR_B = 4,
       HG_KERNEL_OSPR_C = 5, HG_KERNEL_PROP_ROW = 6, HG_KERNEL_PROP_COL = 7 };
hg_status hg_timing_begin(hg_plan plan, int32_t kernel, int32_t repeats);
hg_status hg_timing_end(hg_plan plan, double* total_ms, int64_t* launches);

/* Static text for a status.  If s equals the calling thread's last non-OK
 * status, the text also carries that call's detail (argument name, HIP
 * error).  Never NULL; the pointer stays valid until this thread's next
 * library call. */
const char* hg_error(hg_status s);

#ifdef __cplusplus
}
#endif

#endif /* HOLOGEN_H */

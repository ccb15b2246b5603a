/*
 * msl.h -- C ABI of libmsl, the MI355X (gfx950) multislice library for
 * coherent surface scattering imaging in reflection geometry
 * (Myint et al., "Multislice forward modeling of Coherent Surface Scattering
 * Imaging on surface and interfacial structures", arXiv 2212.01253).
 *
 * What is computed (paper passages in brackets):
 *   - the multislice recurrence of Eq. (1) [Sec. 1]: for every slice s the
 *     complex field is multiplied by the slice transmission
 *     T_s = exp(i k dx (delta_s + i beta_s)), Fourier transformed, multiplied
 *     by the Fresnel propagator and inverse transformed; the exit wave of one
 *     slice enters the next [Sec. 1; Fig. 1 caption];
 *   - the far-field detector intensity: Fourier transform of the final exit
 *     wave, squared [Sec. 1; Fig. 1 caption];
 *   - the amplitude loss of Eq. (4) [Sec. 4.1] and its gradient with respect
 *     to every slice's delta and beta, which the paper obtains by automatic
 *     differentiation [Sec. 1, Sec. 3, Sec. 4] and this library by an explicit
 *     adjoint sweep with checkpoints.
 *
 * Conventions (the complex conjugate of the paper's exp(+ikZ) form; every
 * detector intensity is identical to the paper-convention one):
 *   transmission   T = exp(i k dx (delta + i beta)), k = 2 pi / lambda
 *   propagator     paraxial H = exp(+i dx (ky^2 + kz^2) / 2k)      [Eq. 1]
 *                  exact    H = exp(+i dx kp^2 / (k + sqrt(k^2 - kp^2)))
 *                  (kp >= k: exp(-dx sqrt(kp^2 - k^2)) exp(i k dx))
 *   the global carrier exp(i k dx) of Eq. (1) is dropped (one phase per slice);
 *   default probe  psi0[j][l] = exp(+i k sin(alpha_i) * j * dy), a plane wave
 *                  tilted toward row 0 (incidence enters as a beam tilt in the
 *                  sample frame instead of the object rotation of Eq. 2-3);
 *   far field      A = sum_j psi_j exp(+2 pi i (u jy / Ny + v jz / Nz)),
 *                  I = |A|^2 / (Ny Nz), fftshifted: row Ny/2 is the horizon.
 *
 * Coordinates (paper lab frame -> this library): the beam axis Z of the paper
 * is x here (slice index s, thickness dx); the surface normal Y is y (rows,
 * index j, row 0 is the deepest substrate row); the horizontal transverse
 * axis X is z (columns, index l).
 *
 * Layouts: every field is complex64 [ny][nz] row-major (interleaved re, im);
 * slice stacks (delta, beta and their gradients) are float32 [n_slices][ny][nz];
 * intensities and measured amplitudes are float32 [ny][nz] in fftshifted order.
 *
 * Memory and ownership: every array argument is DEVICE memory owned by the
 * caller.  The library allocates no device memory; it builds its tables (FFT
 * twiddles, propagator, probe) in the caller's workspace on every call, so it
 * keeps no data between calls and calls on different streams with different
 * workspaces may overlap.  Calls that share a workspace or an output must be
 * ordered by the caller.  Process-wide are only the execution settings
 * (msl_set_schedule, msl_set_tuning) and, per device, the helper streams and
 * events the adjoint and the batched forward create on first use.
 *
 * Asynchrony: every call only enqueues work on `hip_stream` (a hipStream_t
 * passed as void*, NULL = the null stream) and returns.  Faults during
 * execution surface at the caller's next synchronisation.
 *
 * Errors: arguments are validated on the host before anything is enqueued;
 * on a non-OK status nothing was enqueued and outputs are untouched, and
 * msl_last_error() returns a description.  A failing HIP launch returns
 * MSL_ERR_HIP with HIP's error string.
 */
#ifndef MSL_H
#define MSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSL_ABI_VERSION 6

typedef struct { float re, im; } msl_c64;

typedef enum {
  MSL_OK = 0,
  MSL_ERR_ARG = -1,          /* null/misaligned pointer, bad size or parameter */
  MSL_ERR_UNSUPPORTED = -2,  /* valid request outside what the library implements */
  MSL_ERR_WORKSPACE = -3,    /* workspace missing, misaligned or too small */
  MSL_ERR_HIP = -4           /* a HIP runtime call or launch failed */
} msl_status;

typedef enum { MSL_PROP_PARAXIAL = 0, MSL_PROP_EXACT = 1 } msl_propagator;

/* Execution schedule of the slice loop (msl_set_schedule). */
typedef enum {
  MSL_SCHED_AUTO = 0,        /* library choice */
  MSL_SCHED_PER_PASS = 1,    /* one kernel launch per line pass */
  MSL_SCHED_PERSISTENT = 2   /* one cooperative launch per phase, grid barriers between passes
                                (square grids, ny == nz; other shapes run per pass) */
} msl_schedule;

typedef struct {
  int32_t ny, nz;            /* rows (y) and columns (z): powers of two in [16, 1024] */
  int32_t n_slices;          /* Ns >= 1 */
  double  dy_nm, dz_nm;      /* transverse pixel pitch (nm), > 0 */
  double  dx_nm;             /* slice thickness along the beam (nm), > 0 */
  double  wavelength_nm;     /* lambda > 0 */
  double  alpha_i_rad;       /* incidence angle (rad), |alpha| < pi/2 */
  int32_t propagator;        /* msl_propagator */
} msl_geometry;

/* ABI version of the loaded library (MSL_ABI_VERSION). */
int32_t msl_abi_version(void);

/* Bytes of workspace every entry point below needs for geometry g when
 * checkpoints are taken every `ckpt_every` slices (0 = no checkpoints; the
 * adjoint needs ckpt_every >= 1).  Returns 0 if g is invalid. */
size_t msl_workspace_bytes(const msl_geometry* g, int32_t ckpt_every);

/* Number of checkpoint fields msl_forward writes: ceil(Ns / ckpt_every). */
int32_t msl_checkpoint_count(const msl_geometry* g, int32_t ckpt_every);

/* Forward multislice [Eq. 1; Sec. 1; Fig. 1 caption].
 *   delta, beta  float32 [Ns][ny][nz]: slice-averaged refractive index
 *                decrement and absorption index of every slice (the slice
 *                integral of Eq. 1 is dx times these averages).
 *   probe        complex64 [ny][nz] entrance field, or NULL for the tilted
 *                plane wave above.
 *   field_out    complex64 [ny][nz]: exit wave psi_Ns after the last slice
 *                (including its propagation).  Used as scratch while running.
 *   ckpt         NULL (then ckpt_every must be 0) or complex64
 *                [msl_checkpoint_count][ny][nz]: ckpt[c] receives the
 *                entrance field of slice c * ckpt_every (ckpt[0] = probe).
 *   flags        0 or MSL_REUSE_SLICE_PACK (below); unknown bits are an error.
 *   workspace    device memory, 256-byte aligned, >= msl_workspace_bytes. */
msl_status msl_forward(const msl_geometry* g, const float* delta, const float* beta,
                       const msl_c64* probe, msl_c64* field_out,
                       msl_c64* ckpt, int32_t ckpt_every, uint32_t flags,
                       void* workspace, size_t ws_bytes, void* hip_stream);

/* Forward without allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Computes exactly what msl_forward computes (same
 * arguments and outputs, no workspace, no flags) and enqueues the same kind of
 * work, but its tables (FFT twiddles, propagator) live in a fixed device array
 * of MSL_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends; the call allocates and frees nothing.  It builds no slice
 * pack: every pass evaluates its transmission from delta and beta directly
 * (the same arithmetic; more work per pass, and strided reads in the column
 * passes).
 * Limits: the exact propagator's table must fit, i.e. ny * nz <= 512 * 512
 * with MSL_PROP_EXACT (any valid paraxial geometry fits); a larger request
 * returns MSL_ERR_UNSUPPORTED before anything is enqueued.  All calls on one
 * GPU share its array, which keeps the last call's tables: calls that overlap
 * on one GPU (other streams, other host threads) race and must be ordered by
 * the caller.  The schedule setting is ignored (always one launch per pass). */
#define MSL_NOALLOC_SCRATCH_BYTES ((size_t)(4 * 64 * 1024 * 8 + 2 * 512 * 512 * 8))
msl_status msl_forward_noalloc(const msl_geometry* g, const float* delta, const float* beta,
                               const msl_c64* probe, msl_c64* field_out,
                               msl_c64* ckpt, int32_t ckpt_every, void* hip_stream);

/* Far-field detector intensity of a field [Sec. 1; Fig. 1 caption]:
 * intensity[r][c] = |A|^2 / (ny nz) at fftshifted position (r, c), float32. */
msl_status msl_far_field(const msl_geometry* g, const msl_c64* field, float* intensity,
                         void* workspace, size_t ws_bytes, void* hip_stream);

/* Amplitude loss of Eq. (4) [Sec. 4.1], summed (not averaged) over pixels:
 *   loss_out[0]     (double, device) = sum (sqrt(I) - m)^2, accumulated in FP64;
 *   grad_intensity  float32 [ny][nz] (may be NULL) = dL/dI = 1 - m / sqrt(I),
 *                   0 where I = 0.
 * intensity and meas_amp are float32 [ny][nz] in the same (fftshifted) order. */
msl_status msl_amp_loss(const msl_geometry* g, const float* intensity, const float* meas_amp,
                        double* loss_out, float* grad_intensity,
                        void* workspace, size_t ws_bytes, void* hip_stream);

/* Cotangent of a field from the cotangent of its far-field intensity:
 * grad_field = FFT2(2 * gI * A / (ny nz)) with A the unshifted backward DFT
 * of `field` and gI = grad_intensity moved back to unshifted order.
 * Complex cotangents use dL = Re sum conj(g) dz (PyTorch's convention). */
msl_status msl_far_field_adjoint(const msl_geometry* g, const msl_c64* field,
                                 const float* grad_intensity, msl_c64* grad_field,
                                 void* workspace, size_t ws_bytes, void* hip_stream);

/* Flag of msl_forward and msl_adjoint: the workspace already holds the slice
 * pack (below) for this geometry's wavelength and dx and these delta and
 * beta, written by msl_pack_slices or by an earlier msl_forward / msl_adjoint
 * call on the same workspace, and delta and beta are unchanged since; the
 * call skips rebuilding it.  Without the flag every call rebuilds it. */
#define MSL_REUSE_SLICE_PACK 1u

/* Slice pack: with the paraxial propagator every line pass that transmits
 * reads the transmission T - 1 = exp(i k dx (delta + i beta)) - 1 of its
 * slice precomputed ([Ns][ny][nz] complex64 in 2x2 tiles of 32 bytes, in the
 * workspace): the pass then spends no arithmetic on it, and row and column
 * passes alike read whole tiles.  This call writes it (a no-op for the exact
 * propagator, which needs none).  It depends on delta, beta, the wavelength
 * and dx, not on the incidence angle or the probe. */
msl_status msl_pack_slices(const msl_geometry* g, const float* delta, const float* beta,
                           void* workspace, size_t ws_bytes, void* hip_stream);

/* Gradient of a real loss through the multislice recurrence (reverse sweep
 * of Eq. 1 with checkpoint recomputation).
 *   delta, beta, probe, ckpt, ckpt_every: exactly as given to / produced by
 *                msl_forward (ckpt is required, ckpt_every >= 1).
 *   grad_field   complex64 [ny][nz]: cotangent of psi_Ns.
 *   grad_delta, grad_beta  float32 [Ns][ny][nz] (either may be NULL):
 *                overwritten with dL/d delta and dL/d beta.
 *   grad_probe   NULL or complex64 [ny][nz]: cotangent of the probe.
 *   flags        0 or MSL_REUSE_SLICE_PACK (see above); unknown bits are an error. */
msl_status msl_adjoint(const msl_geometry* g, const float* delta, const float* beta,
                       const msl_c64* probe, const msl_c64* ckpt, int32_t ckpt_every,
                       const msl_c64* grad_field, float* grad_delta, float* grad_beta,
                       msl_c64* grad_probe, uint32_t flags,
                       void* workspace, size_t ws_bytes, void* hip_stream);

/* Select the slice-loop schedule for later calls from this process
 * (process-wide; not synchronised with calls running on other threads).
 * Returns the previous setting, or MSL_ERR_ARG for an unknown value. */
int32_t msl_set_schedule(int32_t schedule);

/* Outcome of the last msl_forward, msl_far_field, msl_far_field_adjoint or
 * msl_adjoint call on `workspace` (each of them restarts it): waits for
 * hip_stream, then returns MSL_OK, or MSL_ERR_HIP if a grid barrier of the
 * persistent schedule gave up waiting.  That wait is bounded (it polls at most
 * the spin limit below, then raises an error word and lets the grid drain);
 * the call's results are then not valid, and its working field is overwritten
 * with NaN.  Errors of the per-pass schedule surface as HIP errors instead. */
msl_status msl_workspace_status(void* workspace, size_t ws_bytes, void* hip_stream);

/* Polls the persistent schedule's barrier makes before it gives up
 * (process-wide, default 2^22, far beyond any healthy wait; >= 0).  Returns the
 * previous value, or MSL_ERR_ARG.  A small value forces the failure path. */
int32_t msl_set_barrier_spin_limit(int32_t polls);

/* ---- launch shape and its autotuner ----
 * The line passes run as workgroups of several neighbouring lines each, every
 * line held by N / P lanes at P points per lane.
 * Entry e of points_per_lane is P for 2^e-point lines: 4 (radix-4 stages,
 * e >= 4) or 8 (radix-8 stages, e >= 6); 0 = the library default (8 from 512
 * points up, 4 below); other entries must be 0.  P changes the order of the
 * FFT's float32 operations, so results differ in the last bits between
 * settings (both within the parity tolerances).  The persistent schedule
 * (MSL_SCHED_PERSISTENT) always uses the default.
 * Entry e of lines_per_group is the number of 2^e-point lines per workgroup
 * (e = 4..10; 0 = the library default: one 64-lane wavefront's worth of
 * lanes and at least two lines; other entries must be 0).  Allowed values are
 * powers of two up to the limit set by the 256-thread workgroup (the
 * workgroup's LDS exchange buffers stay within 64 KiB at every allowed
 * value): at 8 points per lane
 * 2^e = 64: 32, 128: 16, 256: 8, 512: 4, 1024: 2; at 4 points per lane
 * 2^e = 16: 64, 32: 32, 64: 16, 128: 8, 256: 4, 512: 2, 1024: 1.
 * The lines per workgroup only deal lines to the hardware: at one P every
 * allowed value gives bit-identical results.
 * batch_streams: how many grid-size groups msl_forward_batch runs side by side
 * (1..4; 0 = 4).  The setting is process-wide, applies to later calls, and is
 * not synchronised with calls running on other threads. */
#define MSL_TUNE_SLOTS 11
typedef struct {
  int32_t lines_per_group[MSL_TUNE_SLOTS];
  int32_t points_per_lane[MSL_TUNE_SLOTS];
  int32_t batch_streams;
} msl_tuning;

/* Validate and apply a launch shape (nothing changes on an error). */
msl_status msl_set_tuning(const msl_tuning* t);
/* The launch shape in effect. */
msl_status msl_get_tuning(msl_tuning* t);

/* Autotuner of the launch shape for one geometry: times msl_forward (no
 * probe, no checkpoints) on the caller's delta and beta (device
 * [Ns][ny][nz] f32) for every allowed (points per lane, lines per workgroup)
 * pair of the nz-point slot, keeps the fastest, then the same for the ny-point slot
 * (when ny != nz).  Each candidate runs once untimed and then `reps` times
 * (1..1000) between two HIP events on hip_stream; the call blocks until the
 * search ends.  field_scratch: device complex64 [ny][nz], overwritten.
 * workspace: as for msl_forward (at least msl_workspace_bytes(g, 0)).  On
 * success the fastest shape stays in effect and is copied to *best (may be
 * NULL), its mean forward time in ms to *best_ms (may be NULL); on an error
 * the previous shape is restored. */
msl_status msl_autotune_forward(const msl_geometry* g, const float* delta, const float* beta,
                                msl_c64* field_scratch, void* workspace, size_t ws_bytes, int32_t reps,
                                void* hip_stream, msl_tuning* best, float* best_ms);

/* Thread-local text for the last non-OK status returned on this thread. */
const char* msl_last_error(void);

/* ------------------------------------------------------------------------
 * Batched forward: many independent instances (own grid, slice count,
 * wavelength, incidence angle, probe) in one call, each computing the Eq. (1)
 * recurrence and its far field as msl_forward and msl_far_field do.  The line
 * passes of all instances of one grid size that are at the same slice run as
 * one launch, so a batch fills the GPU where one small instance cannot.
 *
 * Slice stacks are compact: a pool of the instance's distinct slices plus the
 * pool index of every slice (elongated samples repeat slices for long runs
 * along the beam; a dense stack of a large batch would not fit in memory). */
typedef struct {
  msl_geometry g;              /* propagator must be MSL_PROP_PARAXIAL */
  int32_t n_pool;              /* distinct slices, >= 1 */
  const float* pool_delta;     /* device float32 [n_pool][ny][nz] */
  const float* pool_beta;      /* device float32 [n_pool][ny][nz] */
  const int32_t* slice_index;  /* device int32 [n_slices]: pool slice of every slice;
                                  values outside [0, n_pool) are clamped */
  const msl_c64* probe;        /* device [ny][nz] entrance field, or NULL: tilted plane wave */
  msl_c64* field_out;          /* device [ny][nz]: exit wave (also the working field) */
  float* intensity_out;        /* device [ny][nz] fftshifted far field, or NULL */
} msl_instance;

/* Workspace bytes msl_forward_batch needs for these instances (0 if any is invalid). */
size_t msl_batch_workspace_bytes(const msl_instance* inst, int32_t n);

/* Runs every instance of the host array inst[0..n-1] (read during the call
 * only).  Instances must not share output buffers.  Errors as above; an
 * exact-propagator instance is MSL_ERR_UNSUPPORTED. */
msl_status msl_forward_batch(const msl_instance* inst, int32_t n, void* workspace, size_t ws_bytes,
                             void* hip_stream);

/* Launch-shape autotuner for a batch, as msl_autotune_forward (msl_set_tuning): times
 * msl_forward_batch over inst[0..n) for every batch_streams value (1..4), keeps the fastest,
 * then every allowed (points per lane, lines per workgroup) pair of each line length the instances use, one
 * length at a time.  The instances' outputs are overwritten by the timed runs; workspace as
 * for msl_forward_batch; blocks until the search ends. */
msl_status msl_autotune_batch(const msl_instance* inst, int32_t n, void* workspace, size_t ws_bytes, int32_t reps,
                              void* hip_stream, msl_tuning* best, float* best_ms);

/* ------------------------------------------------------------------------
 * Object rotation [Eq. 2-3; Sec. 2]: the paper rotates the sample's index
 * volume into the lab frame (pitch by the incidence angle about the
 * horizontal axis, yaw by the in-plane angle about the surface normal) and
 * propagates a straight beam through it.  This library's default reading
 * tilts the beam instead (see the probe above); this call builds the literal
 * lab-frame stack for comparison or for angles the tilt does not cover.
 *
 * Axes in library order (slice axis a = the paper's Z, row y = Y, column
 * z = X).  A lab voxel (s, j, l) sits at u = (s dx, j dy, l dz) - lab_pivot;
 * its sample-frame position is v = M u + sample_pivot with M the product of
 * the paper's pitch and yaw matrices in this axis order,
 *   a' =  cos(p) cos(w) a + sin(p) y - cos(p) sin(w) z
 *   y' = -sin(p) cos(w) a + cos(p) y + sin(p) sin(w) z
 *   z' =  sin(w) a                   + cos(w) z
 * (p = pitch, w = yaw; with p > 0 the sample surface rises along the beam),
 * and delta, beta there are trilinear interpolates of the sample volume
 * (voxel (i, j, k) of the sample at (i da, j dy, k dz); zero outside it). */
typedef struct {
  int32_t na, ny, nz;                /* sample voxels along a (beam-wise length), y (normal), z */
  double da_nm, dy_nm, dz_nm;        /* sample voxel pitch (nm), > 0 */
  double pivot_a_nm, pivot_y_nm, pivot_z_nm;  /* sample pivot, nm from voxel (0, 0, 0) */
} msl_sample_grid;

/* delta, beta float32 [g->n_slices][g->ny][g->nz] (lab frame, written) from
 * delta_s, beta_s float32 [s->na][s->ny][s->nz] (sample frame). */
msl_status msl_rotate_object(const msl_geometry* g, double lab_pivot_a_nm, double lab_pivot_y_nm,
                             double lab_pivot_z_nm, const msl_sample_grid* s, double pitch_rad, double yaw_rad,
                             const float* delta_s, const float* beta_s, float* delta, float* beta,
                             void* hip_stream);

/* ------------------------------------------------------------------------
 * Reconstruction support [Sec. 4.1]: the paper refines a 3-D object by
 * minimising the amplitude loss of Eq. (4) with gradients and the ADAM
 * optimiser (Kingma and Ba, 2014).  The unknowns here are the delta values of
 * the voxels in one box of the slice stack, with beta tied to delta by a
 * fixed ratio (beta = beta_over_delta * delta); everything outside the box is
 * known and left untouched. */

/* Box of unknown voxels: slices [s0, s0 + ns), rows [y0, y0 + ny), columns
 * [z0, z0 + nz) of the [n_slices][ny][nz] stack.  Parameters theta are
 * float32 [ns][ny][nz] (row-major over the box). */
typedef struct {
  int32_t s0, ns, y0, ny, z0, nz;
  float beta_over_delta;
} msl_region;

/* ADAM hyper-parameters; each updated theta is clamped to [lo, hi]. */
typedef struct {
  float lr, beta1, beta2, eps, lo, hi;
} msl_adam;

/* delta[box] = theta, beta[box] = beta_over_delta * theta. */
msl_status msl_region_scatter(const msl_geometry* g, const msl_region* r, const float* theta,
                              float* delta, float* beta, void* hip_stream);

/* One ADAM step on theta from the stack gradients of the loss, then the
 * scatter above with the new theta.  With the box gradient
 *   gr = grad_scale * (grad_delta[box] + beta_over_delta * grad_beta[box])
 * (grad_scale rescales a loss that was evaluated up to a constant factor)
 * and step count t >= 1:
 *   m = beta1 m + (1 - beta1) gr;  v = beta2 v + (1 - beta2) gr^2;
 *   theta = clamp(theta - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps), lo, hi).
 * theta, m, v are float32 [ns][ny][nz] (m = v = 0 before the first step);
 * grad_delta, grad_beta as written by msl_adjoint (both required). */
/* Nearest-value filter [Sec. 4.1: after some epochs the paper maps every
 * voxel parameter to the nearest refractive index of the materials present]:
 * theta[i] = the entry of levels[0 .. n_levels) nearest to theta[i] (distances
 * in float32; on a tie the lower index wins), then the scatter above.
 * levels is HOST memory, 1 <= n_levels <= MSL_MAX_LEVELS. */
#define MSL_MAX_LEVELS 16
msl_status msl_region_snap(const msl_geometry* g, const msl_region* r, const float* levels, int32_t n_levels,
                           float* theta, float* delta, float* beta, void* hip_stream);

/* Shrink-wrap support [Sec. 4.1, with Marchesini et al. 2003]: the box
 * parameters are blurred with a separable Gaussian (standard deviations
 * sigma_a, sigma_y, sigma_z in voxels, >= 0; kernel truncated at
 * radius floor(3 sigma + 1/2), normalised, zero outside the box), every
 * parameter whose blurred |theta| is not above threshold times the largest
 * blurred value is set to 0, and the result is scattered as above.
 * scratch: float32, 2 * ns * ny * nz + 1024 values (device). */
msl_status msl_region_shrinkwrap(const msl_geometry* g, const msl_region* r, float sigma_a, float sigma_y,
                                 float sigma_z, float threshold, float* theta, float* scratch, float* delta,
                                 float* beta, void* hip_stream);

msl_status msl_region_adam_step(const msl_geometry* g, const msl_region* r, const msl_adam* a,
                                int32_t t, float grad_scale,
                                const float* grad_delta, const float* grad_beta,
                                float* theta, float* m, float* v,
                                float* delta, float* beta, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MSL_H */

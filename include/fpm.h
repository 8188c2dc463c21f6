/*
 * fpm.h -- C ABI of the MI355X (gfx950) Fourier ptychographic reconstruction
 * library (libfpm.so).
 *
 * The method is the one of Zhou et al., "Parallel Fourier Ptychography
 * reconstruction": alternating projections between the spatial modulus
 * constraint and the frequency support constraint (Sec. 1, Sec. 2.1),
 * run independently per overlapping sub-region with its own illumination
 * angles and defocus (Sec. 2.2, Sec. 3.1), and across groups of LEDs whose
 * spectrum regions do not overlap (Sec. 3.2), on FFT/IFFT kernels written
 * for the GPU (Sec. 3.3).
 *
 * Conventions shared by every entry point
 *  - Complex data are interleaved float pairs (complex64), row-major.
 *  - Spectra are centred: index u is frequency (u - size/2) / (n * pixel_um).
 *  - LED index j = r * led_cols + c is the board (grid) index, row-major;
 *    it is not the processing order.
 *  - Multi-tile arrays are the per-tile arrays concatenated in plan order;
 *    tile t of a plan starts at the element offset the plan reports.
 *  - Ownership: the caller owns every buffer it passes; buffers must stay
 *    valid until the call returns (fpm_submit: until fpm_poll has returned
 *    a status other than FPM_PENDING).  The library owns plans, servers and
 *    all device-resident state it allocates.
 *  - Device pointers and streams: FPM_MEM_DEVICE pointers are HIP device
 *    addresses on the current device; `hip_stream` is a hipStream_t cast to
 *    void* (NULL = the default stream).
 *  - Errors: every call returns an fpm_status; nothing is thrown across the
 *    ABI (a host allocation or thread start that fails inside a call
 *    returns FPM_E_NOMEM).  fpm_last_error() gives a thread-local message
 *    for the last non-OK status.  A call rejected before it enqueues work
 *    (FPM_E_ARG, FPM_E_GEOMETRY, FPM_E_STATE, FPM_E_UNSUPPORTED) writes no
 *    output buffer; after FPM_E_NOMEM, FPM_E_DIVERGED or FPM_E_DEVICE the
 *    outputs' contents are unspecified (FPM_E_DIVERGED is found once they
 *    are written).
 */
#ifndef FPM_H
#define FPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FPM_OK = 0,
  FPM_PENDING = 1,        /* fpm_poll: the request has not finished          */
  FPM_E_ARG = -1,         /* invalid argument (NULL, size, non-finite data)   */
  FPM_E_GEOMETRY = -2,    /* a crop window leaves the high-resolution grid    */
  FPM_E_NOMEM = -3,       /* device or host allocation failed                 */
  FPM_E_DEVICE = -4,      /* a HIP call failed                                */
  FPM_E_DIVERGED = -5,    /* a residual became non-finite                     */
  FPM_E_CANCELLED = -6,   /* the request was cancelled                        */
  FPM_E_UNSUPPORTED = -7, /* tile size or precision the library does not run */
  FPM_E_STATE = -8        /* call out of order (online session open/closed)   */
} fpm_status;

/* Arithmetic of the two n x n transforms of every update.  The MFMA forms
 * compute them as dense products with centred DFT matrices on the matrix
 * cores with FP32 accumulation (tile sides 64, 96, 128; FPM_E_UNSUPPORTED
 * for 256); the plan, the update rule and every other step are unchanged. */
typedef enum {
  FPM_PREC_FP32_FFT = 0,     /* FP32 FFTs in LDS and registers (default)    */
  FPM_PREC_MFMA_BF16X3 = 1,  /* dense DFT on MFMA, three-term split bf16    */
  FPM_PREC_MFMA_FP16 = 2     /* dense DFT on MFMA, scaled fp16              */
} fpm_precision;

typedef enum {
  FPM_SCHED_SEQUENTIAL = 0,  /* one LED at a time, ascending illumination NA */
  FPM_SCHED_LED_GROUPS = 1,  /* Sec. 3.2: members of a non-overlapping LED
                                group run concurrently from the group-start
                                state; the pupil takes their mean increment  */
  FPM_SCHED_GROUP_ORDER = 2, /* one LED at a time, in the grouped order      */
  FPM_SCHED_PIPELINED = 3    /* Sec. 3.2 Fig. 6b/d: the sequential NA-order
                                sweep with its updates over all iterations
                                level-scheduled -- an update runs once every
                                earlier update whose spectrum window overlaps
                                it has run, so iteration k+1 starts on the
                                inner LEDs while iteration k finishes the outer
                                ones.  Same result as SEQUENTIAL (bitwise);
                                with pupil recovery every update depends on the
                                previous one and the levels are the sequence. */
} fpm_schedule;

typedef enum { FPM_MEM_HOST = 0, FPM_MEM_DEVICE = 1 } fpm_mem;

/* One tile = one independent reconstruction (Sec. 3.1).  The fields are the
 * paper's problem statement: LED board geometry and height (Sec. 2.2,
 * Sec. 4), wavelength and objective NA (Sec. 2.1), effective pixel size
 * (Sec. 4), the sub-region's position and defocus (Sec. 2.2), iterations
 * (Sec. 2.1, Sec. 4.1), plus the upsampling factor of the synthesised grid.
 *
 * Geometry (all FP64, evaluated left to right as written):
 *   LED (r, c):  x = (c - (led_cols-1)/2) * led_pitch_um + led_origin_x_um
 *                y = (r - (led_rows-1)/2) * led_pitch_um + led_origin_y_um
 *   rho  = sqrt((x - tile_x)^2 + (y - tile_y)^2 + led_height^2)
 *   dcol = floor((x - tile_x)/rho * n * pixel_um / wavelength_um + 0.5)
 *   drow = floor((y - tile_y)/rho * n * pixel_um / wavelength_um + 0.5)
 *   support radius r = na_obj * n * pixel_um / wavelength_um (bins);
 *   D0 = {(u,v) : (u - n/2)^2 + (v - n/2)^2 <= r^2}.
 *   LED j's window in the N x N spectrum (N = n * upsample): rows
 *   [N/2 + drow - n/2, +n), cols [N/2 + dcol - n/2, +n); |drow|, |dcol| must
 *   not exceed (N - n)/2, else FPM_E_GEOMETRY. */
typedef struct {
  int32_t n;              /* LR tile side in pixels: 64, 96, 128 or 256       */
  int32_t upsample;       /* HR side N = n * upsample                         */
  int32_t led_rows, led_cols;
  double led_pitch_um, led_height_um;
  double led_origin_x_um, led_origin_y_um;
  double wavelength_um, na_obj, pixel_um;  /* pixel_um: sample-plane LR pixel */
  double tile_x_um, tile_y_um;             /* tile centre w.r.t. optical axis */
  double defocus_um;                       /* tile defocus z                  */
  int32_t iterations;
  int32_t pupil_update;                    /* 0 or 1                          */
  int32_t precision;                       /* fpm_precision                   */
  int32_t schedule;                        /* fpm_schedule                    */
} fpm_tile_desc;

/* Per-tile facts a plan derives (fpm_plan_tile_info). */
typedef struct {
  int32_t n, N, L;             /* LR side, HR side, LED count               */
  int32_t support_count;       /* |D0|                                       */
  int32_t ngroups;             /* non-overlapping LED groups (Sec. 3.2)      */
  int32_t max_group;           /* largest group                              */
  int32_t steps;               /* dependent update steps per iteration       */
  int32_t iterations;
  double min_tie_distance;     /* min |frac(offset) - 0.5| over LEDs/axes    */
  int64_t intensity_offset;    /* element offset of this tile's [L][n][n]    */
  int64_t object_offset;       /* complex offset of this tile's [N][N]       */
  int64_t pupil_offset;        /* complex offset of this tile's [n][n]       */
  int64_t residual_offset;     /* offset of this tile's [iterations] doubles */
  int32_t levels;              /* dependent launches of the whole sweep      */
  int32_t reserved;
} fpm_tile_info;

typedef struct fpm_plan_s fpm_plan_t;
typedef struct fpm_server_s fpm_server_t;

/* Build a plan for `ntiles` independent tiles (Sec. 3.1).  Host-only FP64
 * geometry: integer spectrum offsets per LED (Sec. 2.2), the processing
 * order (ascending illumination NA; Sec. 3.2 Fig. 6a), the non-overlapping
 * LED groups (greedy first fit over that order; Sec. 3.2), the support D0
 * and the initial pupil D0 * exp(i phi_z) with the tile's defocus phase.
 * Device memory is allocated on first use, on the current device.
 * Errors: FPM_E_ARG (NULL, ntiles < 1, unsupported field values),
 * FPM_E_GEOMETRY (a window outside the HR grid), FPM_E_UNSUPPORTED. */
fpm_status fpm_plan(const fpm_tile_desc *tiles, int32_t ntiles, fpm_plan_t **out);
void fpm_plan_destroy(fpm_plan_t *plan);

fpm_status fpm_plan_tile_info(const fpm_plan_t *plan, int32_t tile, fpm_tile_info *info);

/* Host copies of tile `tile`'s integer tables, each optional (NULL skips):
 * offsets [L][2] (drow, dcol) per grid LED; order [L] (grid indices in
 * ascending illumination NA); group_of [L] (group of each grid LED);
 * sweep [L] (groups concatenated, members in order). */
fpm_status fpm_plan_tables(const fpm_plan_t *plan, int32_t tile, int32_t *offsets,
                           int32_t *order, int32_t *group_of, int32_t *sweep);

/* Device bytes the plan holds once fpm_reconstruct has run (state, scratch,
 * work lists; excluding caller buffers). */
fpm_status fpm_plan_device_bytes(const fpm_plan_t *plan, size_t *bytes);

/* Forward model (Sec. 2.1, Fig. 1): for every tile and grid LED j,
 * I_j = |IFFT_n(shift(P * W_j(S)))|^2 with S = shift(FFT_N(object)) / up^2.
 *   object    complex64 [tile][N][N], spatial domain.
 *   pupil     complex64 [tile][n][n] centred, or NULL for the plan's initial
 *             pupil; only its values on D0 are used.
 *   intensity float [tile][L][n][n] output.
 * `where` applies to all three buffers.  Device mode enqueues on
 * `hip_stream` and returns; host mode copies and synchronises. */
fpm_status fpm_forward(fpm_plan_t *plan, const void *object, const void *pupil,
                       float *intensity, fpm_mem where, void *hip_stream);

/* Reconstruction (Sec. 2.1 Fig. 2 with embedded pupil recovery; Sec. 3.1
 * tiles; Sec. 3.2 LED groups).  Per tile, from the initial guess
 * S = 0 except the centred n x n window = shift(FFT_n(sqrt I_j0)) (j0 the
 * first LED of the sweep; an intensity carries no illumination tilt, so its
 * spectrum sits at zero frequency), P = P_init, for each iteration and each
 * LED j of the schedule:
 *   X = W_j(S), Phi = P X, psi = IFFT_n(shift Phi),
 *   psi' = sqrt(I_j) psi / |psi|, Phi' = shift FFT_n(psi'), D = Phi' - Phi,
 *   W_j(S) <- X + conj(P) D / max|P|^2          on D0,
 *   P      <- P + conj(X) D / max|S|^2          on D0 (pupil_update),
 * where max|S|^2 is taken over the whole spectrum at the start of the
 * iteration; LED groups read the group-start state and average their pupil
 * increments.  After each iteration: residual = sum (|psi| - sqrt I)^2 /
 * sum I (FP64), and, with pupil_update, the pupil energy is normalised to
 * |D0| (P <- sP, S <- S/s; the product P*S is unchanged).
 *   intensity     float [tile][L][n][n] (grid LED order), finite, >= 0.
 *   object_out    complex64 [tile][N][N]: up^2 * IFFT_N(shift S); may be NULL.
 *   pupil_out     complex64 [tile][n][n]; may be NULL.
 *   residual_out  double [tile][iterations]; may be NULL.
 * `where` applies to all four buffers.  FPM_MEM_HOST: the intensities are
 * validated (FPM_E_ARG on NaN, Inf or a negative value), copied, and the call
 * synchronises; FPM_E_DIVERGED if a residual is not finite.  On either error
 * no output is written.  FPM_MEM_DEVICE: enqueued on `hip_stream`, returns
 * without waiting; the intensities are checked on the device before the
 * sweep and the residuals after it, and if either check fails the outputs
 * are not written; fpm_plan_status reports the outcome (FPM_E_ARG or
 * FPM_E_DIVERGED) once the work has run.
 * The plan's tiles run as independent chains on streams of the library's
 * own, forked from `hip_stream` and joined back into it with events, so the
 * work is ordered on `hip_stream` as one operation; FPM_CHAINS=1..4 sets the
 * number of chains.  Calls on one plan share its device state: a call on a
 * stream other than the previous call's first waits (on the device, through
 * an event) for that call's work, so calls on one plan never overlap,
 * whatever streams they come on; a call on the previous call's stream waits
 * for nothing. */
fpm_status fpm_reconstruct(fpm_plan_t *plan, const float *intensity, fpm_mem where,
                           void *object_out, void *pupil_out, double *residual_out,
                           void *hip_stream);

/* Online reconstruction (Sec. 3.4, Fig. 7a): the images of one LED arrive
 * at a time, and each arrival runs that LED's update on every tile at once,
 * so the first iteration proceeds while the next LED pattern is set up.
 * Every tile of the plan must use FPM_SCHED_SEQUENTIAL and the same L
 * (FPM_E_ARG otherwise).
 *   fpm_online_begin: opens a session on `plan` (device state, tuning and
 *     the first-iteration work lists are set up here, not in the pushes).
 *     While it is open, fpm_forward, fpm_reconstruct and
 *     fpm_profile_reconstruct on the plan return FPM_E_STATE; begin again
 *     restarts the session.
 *   fpm_online_push: `intensity` float [tile][n][n], the tiles' images for
 *     LED `led` (grid index), in plan tile order (each tile its own n).
 *     Each LED once, any order (FPM_E_ARG for a repeat or out of range).  The
 *     first pushed image is the initial guess (its LED plays j0 of
 *     fpm_reconstruct); each push then runs the update of Fig. 2 for `led`
 *     on every tile, in arrival order.  After the L-th push the first
 *     iteration's residual and normalisation follow.  FPM_MEM_HOST: the
 *     image is validated and copied into pinned staging, the call returns
 *     without waiting for the GPU (it waits only for the previous push's
 *     copy to leave the staging); FPM_MEM_DEVICE: the buffer must stay valid
 *     until the stream has run the push.  Enqueued on `hip_stream`.
 *   fpm_online_finish: once all L LEDs are pushed (FPM_E_STATE before),
 *     runs iterations 2.. in the plan's sweep order over the whole stack and
 *     writes the outputs as fpm_reconstruct does (same layouts and `where`
 *     rules); closes the session and synchronises the stream.
 *   fpm_online_abort: closes an open session without outputs (synchronises
 *     the device); a no-op when none is open.
 * With pushes in the plan's sweep order the result is bitwise that of
 * fpm_reconstruct.  All calls of one session go to one stream. */
fpm_status fpm_online_begin(fpm_plan_t *plan, void *hip_stream);
fpm_status fpm_online_push(fpm_plan_t *plan, int32_t led, const float *intensity,
                           fpm_mem where, void *hip_stream);
fpm_status fpm_online_finish(fpm_plan_t *plan, fpm_mem where, void *object_out,
                             void *pupil_out, double *residual_out, void *hip_stream);
fpm_status fpm_online_abort(fpm_plan_t *plan);

/* Defocus distance of each sub-region, estimated before its reconstruction
 * from its bright-field images (Sec. 3.4 Fig. 7b offline strategy, at least
 * nine bright-field images; Sec. 2.2: each sub-region has its own defocus).
 * Per tile: the bright-field LEDs are those whose window's zero-frequency
 * bin (n/2 - drow, n/2 - dcol) lies in the support disc D0 (FPM_E_GEOMETRY
 * if fewer than nine); the search runs on the smallest centred block of the
 * LED grid that holds them all (rows and columns of the grid's parity).
 * For each candidate z = z_lo + k z_step <= z_hi the block is reconstructed
 * with the pupil fixed at D0 H_z, LED groups, `iterations` iterations, and
 * scored by its last residual; all candidates of all tiles run as one
 * batched reconstruction.  z is the vertex of the parabola through the best
 * score and its two neighbours (the grid point at an end of the grid or
 * where the three scores are not convex).
 *   tiles      ntiles descriptors; defocus_um, iterations, pupil_update,
 *              schedule and precision are not used.
 *   intensity  float [tile][L][n][n] (grid LED order), `where` host or
 *              device; host data are validated (FPM_E_ARG on NaN, Inf or a
 *              negative value).
 *   z_out      double [ntiles], host.
 *   scores_out double [ntiles][scores_per_tile], host, may be NULL: the
 *              candidates' scores (scores_per_tile >= the candidate count).
 * Synchronises `hip_stream` before returning.  Errors: FPM_E_ARG (NULL,
 * z_step <= 0, z_hi < z_lo, iterations outside 1..1000, more than 4096
 * candidates, scores_out too short), FPM_E_GEOMETRY, FPM_E_DIVERGED (a
 * score not finite), FPM_E_NOMEM, FPM_E_DEVICE; z_out is untouched then. */
fpm_status fpm_estimate_defocus(const fpm_tile_desc *tiles, int32_t ntiles,
                                const float *intensity, fpm_mem where, double z_lo, double z_hi,
                                double z_step, int32_t iterations, double *z_out,
                                double *scores_out, int32_t scores_per_tile, void *hip_stream);

/* Stitch reconstructed tiles into one field of view (Sec. 3.1, Eq. (1)).
 *   tiles  complex64 [rows][cols][side][side]: the tile objects on their grid,
 *          row-major, neighbours sharing `overlap` pixels (stride
 *          side - overlap along both axes).
 *   out    complex64 [H][W], H = rows (side - overlap) + overlap, W likewise
 *          with cols.
 * Each row of tiles is merged left to right, then the merged rows top to
 * bottom: f1 is kept up to the middle of the overlap (width - overlap/2),
 * after it f2 scaled by mu1 / mu2, the complex means of the two images over
 * their shared overlap strip (FP64); with overlap 0 the tiles are
 * concatenated.  `where` applies to both buffers; the call returns once `out`
 * is written.  Errors: FPM_E_ARG (NULL, rows or cols < 1, overlap outside
 * [0, side/2]), FPM_E_NOMEM, FPM_E_DEVICE. */
fpm_status fpm_stitch(const void *tiles, int32_t rows, int32_t cols, int32_t side,
                      int32_t overlap, void *out, fpm_mem where, void *hip_stream);

/* fpm_stitch without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same layout, arithmetic and result bits as fpm_stitch,
 * device memory only: `tiles` and `out` are device pointers the caller owns.
 * The strip sums and factors live in a fixed scratch array of each device,
 * sized for at most 4096 tiles (rows * cols) and held until the process
 * ends; it allocates, frees and synchronises nothing, and returns once the
 * kernels are enqueued on hip_stream (`out` is written when the stream
 * reaches them).  All calls on one device share that scratch: calls whose
 * work overlaps on one device (different streams, no ordering between them)
 * race and must be ordered by the caller.  Errors: FPM_E_ARG (NULL, grid,
 * side or overlap out of range, more than 4096 tiles), FPM_E_DEVICE (the
 * scratch lookup or a launch failed); `out` is untouched on error. */
fpm_status fpm_stitch_noalloc(const void *tiles, int32_t rows, int32_t cols, int32_t side,
                              int32_t overlap, void *out, void *hip_stream);

/* Outcome of the plan's last device-mode fpm_reconstruct (or online
 * session): waits until that call's work has run, then sets *status to
 * FPM_OK, FPM_E_ARG (a negative or non-finite intensity) or FPM_E_DIVERGED
 * (a residual that is not finite); in both error cases the call wrote no
 * output, and fpm_last_error says which.  Host-mode calls report their own
 * errors and leave FPM_OK here.  Returns FPM_E_ARG for NULL arguments,
 * FPM_E_DEVICE if the wait or the read fails. */
fpm_status fpm_plan_status(fpm_plan_t *plan, fpm_status *status);

/* Per-kind kernel timing of one reconstruction (profiling aid). */
typedef enum {
  FPM_KERNEL_UPDATE = 0,      /* fused LED-tile update (the hot loop)          */
  FPM_KERNEL_PUPIL_MEAN = 1,  /* mean pupil increment of an LED group          */
  FPM_KERNEL_ITER_END = 2,    /* FP64 residual + pupil-energy normalisation    */
  FPM_KERNEL_SPEC_MAX = 3,    /* max |S|^2 for the next iteration's pupil step */
  FPM_KERNEL_INIT = 4,        /* initial state and its FFT                      */
  FPM_KERNEL_KINDS = 5
} fpm_kernel_kind;

typedef struct {
  int32_t launches;   /* kernel launches of this kind                      */
  int32_t pad;
  int64_t items;      /* FPM_KERNEL_UPDATE: LED-tile updates processed      */
  double total_ms;    /* sum of per-launch durations (HIP events)           */
  double busy_ms;     /* time at least one launch of this kind ran (the
                         union of the launch intervals; chains overlap)    */
} fpm_kernel_time;

/* Run the reconstruction sweep of `plan` once, eagerly (no graph), with a
 * HIP event pair around every launch on the stream it runs on (the chains
 * of tiles concurrently, as in fpm_reconstruct, forked from and joined back
 * into `hip_stream`); synchronise; fill out[FPM_KERNEL_KINDS].  Same kernels
 * and launch shapes as fpm_reconstruct; the state it leaves is that of a
 * reconstruction.  `intensity` as in fpm_reconstruct with FPM_MEM_DEVICE. */
fpm_status fpm_profile_reconstruct(fpm_plan_t *plan, const float *intensity,
                                   fpm_kernel_time *out, void *hip_stream);

/* ------------------------------------------------------------ serving */

typedef struct {
  double submit_s;      /* seconds since server start, taken on entry to
                           fpm_submit                                     */
  double admit_s;       /* admitted (device memory granted)               */
  double finish_s;      /* outputs ready                                  */
  int64_t updates;      /* LED-tile updates the request ran               */
  int32_t status;       /* final fpm_status of the request                */
} fpm_request_stats;

/* A request loop on its own host thread: requests are admitted while their
 * device footprint fits `hbm_budget_bytes` and fewer than `max_slots` run;
 * every admitted request keeps its spectrum and pupil resident; each
 * scheduler tick runs one iteration of every admitted request, step s of all
 * of them in the same launches (continuous batching), and requests join and
 * leave between ticks.  The whole budget is allocated as one device slab
 * when the server is created (FPM_E_NOMEM if it cannot be), and requests
 * take first-fit pieces of it: the request loop allocates and frees no
 * device memory, except the tick's work lists for batches beyond 441 LED
 * updates per slot, and 256 MiB of transpose scratch the first time a
 * 256-px request runs (held until the server is destroyed).
 * Errors: FPM_E_ARG, FPM_E_NOMEM, FPM_E_DEVICE. */
fpm_status fpm_server_create(size_t hbm_budget_bytes, int32_t max_slots, fpm_server_t **out);
void fpm_server_destroy(fpm_server_t *server);

/* Enqueue one tile reconstruction.  `intensity` is float [L][n][n] in host
 * or device memory per `where`; it must stay valid until fpm_poll returns
 * non-PENDING.  Returns at once with a request id. */
fpm_status fpm_submit(fpm_server_t *server, const fpm_tile_desc *tile, const float *intensity,
                      fpm_mem where, uint64_t *id);

/* FPM_PENDING while the request runs; else its final status, having copied
 * the outputs (host memory; each may be NULL) and released the request. */
fpm_status fpm_poll(fpm_server_t *server, uint64_t id, void *object_out, void *pupil_out,
                    double *residual_out, fpm_request_stats *stats);

/* Wait until request `id` is no longer pending (or `timeout_s` passes), then
 * behave as fpm_poll. */
fpm_status fpm_wait(fpm_server_t *server, uint64_t id, double timeout_s, void *object_out,
                    void *pupil_out, double *residual_out, fpm_request_stats *stats);

/* Cancel a request: frees its slot; other requests are unaffected. */
fpm_status fpm_cancel(fpm_server_t *server, uint64_t id);

/* Thread-local text of the last non-OK status on this thread. */
const char *fpm_last_error(void);
/* Library version string. */
const char *fpm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FPM_H */

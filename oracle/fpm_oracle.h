/*
 * FP64 CPU oracle for Fourier ptychographic (FPM) reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library: it is a plain, slow,
 * step-by-step statement of what the reconstruction computes, in double
 * precision, so that a reader can check it against the paper by eye.
 *
 * The paper (Zhou et al., "Parallel Fourier Ptychography reconstruction")
 * describes the method in words only:
 *   - Sec. 1 / Sec. 2.1: alternating projections between a spatial modulus
 *     constraint (amplitude consistent with each low-resolution intensity
 *     image) and a frequency support constraint (a circular low-pass filter
 *     set by the objective NA and the wavelength);
 *   - Sec. 2.2 (Figs. 3-4): the illumination angle of each sub-region comes
 *     from the LED position on the board and the LED-to-sample height, and
 *     each sub-region carries its own defocus distance;
 *   - Sec. 3.1: sub-regions are independent problems;
 *   - Sec. 3.2: the update sequence may be rearranged so that concurrently
 *     processed sub-spectrum regions do not affect each other.
 * The update equations (Fig. 2) are not printed; this oracle follows the
 * standard FPM alternating-projection scheme with embedded pupil recovery
 * (spectrum and pupil both updated from the same exit-wave difference), as
 * the readings listed in the design notes state.
 *
 * Conventions: complex arrays are interleaved (re, im) doubles, row-major.
 * FFT is unnormalised with exp(-2 pi i jk/n); the inverse carries 1/n.
 * Spectra are stored centred: index u is frequency (u - size/2) * dk.
 */
#ifndef FPM_ORACLE_H
#define FPM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n;            /* low-resolution tile side (pixels)              */
  int32_t up;           /* upsampling; high-resolution side N = up * n    */
  int32_t led_rows, led_cols;
  double led_pitch_um, led_height_um;
  double led_x0_um, led_y0_um;   /* LED-grid centre w.r.t. optical axis   */
  double wavelength_um, na, pixel_um;
  double tile_x_um, tile_y_um;   /* tile centre w.r.t. optical axis       */
  double defocus_um;
} orc_geom;

enum { ORC_SEQUENTIAL = 0, ORC_LED_GROUPS = 1, ORC_GROUP_ORDER = 2 };

/* 1-D / 2-D mixed-radix (2, 3, 5, other primes by direct sums) FFT, in place.
 * sign = -1 forward (unnormalised), +1 inverse (scaled by 1/size). */
void orc_fft1(double *z, int32_t n, int32_t sign);
void orc_fft2(double *z, int32_t rows, int32_t cols, int32_t sign);
/* Threads for the independent line transforms of orc_fft2 (default 1; the
 * results do not depend on it). */
void orc_set_threads(int32_t k);

/* Frequency support of the objective: returns |D0|, fills mask[n*n]. */
int32_t orc_support(const orc_geom *g, uint8_t *mask);
/* Initial pupil: support times defocus phase, complex [n][n]. */
void orc_pupil_init(const orc_geom *g, double *pupil);
/* Integer spectrum offsets (drow, dcol) per LED in grid order, [L][2].
 * Returns 0, or -2 if a crop window leaves the high-resolution grid. */
int32_t orc_offsets(const orc_geom *g, int32_t *off);
/* LED processing order (grid indices), ascending illumination NA. */
void orc_order(const orc_geom *g, int32_t *order);
/* Non-overlapping LED groups (greedy first fit over `order`).
 * group_of[L]: group of each LED (grid index).  sweep[L]: groups
 * concatenated.  gstart[L+1]: group g holds sweep[gstart[g] .. gstart[g+1]).
 * Returns the number of groups. */
int32_t orc_groups(const orc_geom *g, const int32_t *off, const int32_t *order,
                   int32_t *group_of, int32_t *sweep, int32_t *gstart);

/* Object (complex [N][N]) <-> scaled centred spectrum S (complex [N][N]). */
void orc_object_to_spectrum(const orc_geom *g, const double *obj, double *S);
void orc_spectrum_to_object(const orc_geom *g, const double *S, double *obj);

/* Forward model: I[L][n][n] (grid LED order) from spectrum S and pupil P. */
void orc_forward(const orc_geom *g, const double *S, const double *P, double *I);

/* Reconstruction.  I: float intensities [L][n][n] in grid LED order.
 * S_out: complex [N][N] scaled centred spectrum; P_out: complex [n][n];
 * residual: [iterations].  S_in / P_in: optional starting state (NULL =
 * the standard initial guess).  Returns 0, or -1 on bad arguments, -2 on
 * bad geometry. */
int32_t orc_reconstruct(const orc_geom *g, const float *I, int32_t iterations,
                        int32_t pupil_update, int32_t schedule,
                        const double *S_in, const double *P_in,
                        double *S_out, double *P_out, double *residual);

/* Online reconstruction (Sec. 3.4, Fig. 7a), sequential schedule: the images
 * arrive one LED at a time in `arrival` (a permutation of the L grid
 * indices); the first arrival gives the initial guess, the first iteration
 * updates in arrival order, later iterations in ascending-NA order.  Equal
 * to orc_reconstruct(SEQUENTIAL) when `arrival` is that order.  Returns 0,
 * -1 (bad arguments or `arrival` not a permutation), -2 (bad geometry). */
int32_t orc_reconstruct_online(const orc_geom *g, const float *I, int32_t iterations,
                               int32_t pupil_update, const int32_t *arrival,
                               double *S_out, double *P_out, double *residual);

#ifdef __cplusplus
}
#endif
#endif

/*
 * FP64 CPU oracle for Fourier ptychographic reconstruction.
 * TEST INFRASTRUCTURE ONLY -- see fpm_oracle.h for scope and conventions.
 *
 * Every function states the passage of the paper (or the reading of it) that
 * it follows.  Nothing here is blocked, fused or reordered beyond the plain
 * definition of the step; the FFT is a textbook recursive Cooley-Tukey.
 */
#include "fpm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ FFT */
/* Sec. 3.3: the reconstruction is built from 2-D FFT/IFFT and pointwise
 * complex products.  Decimation in time on the smallest prime factor p of
 * n = p*m:  X[k + m s] = sum_r W_n^{r (k + m s)} Y_r[k], with Y_r the
 * length-m DFT of x[p i + r].  W_n^e = exp(sign * 2 pi i e / n). */

static int smallest_factor(int n) {
  for (int p = 2; p * p <= n; ++p)
    if (n % p == 0) return p;
  return n;
}

static void fft_rec(const double *in, int istride, double *out, int n,
                    const double *w, int wstep, int wn) {
  if (n == 1) {
    out[0] = in[0];
    out[1] = in[1];
    return;
  }
  int p = smallest_factor(n);
  int m = n / p;
  for (int r = 0; r < p; ++r)
    fft_rec(in + 2 * r * istride, istride * p, out + 2 * r * m, m, w, wstep * p, wn);
  /* the p outputs of one butterfly; small radices (every size used here
   * factors into 2, 3 and 5) stay on the stack */
  double tmp_small[2 * 8];
  double *tmp = p <= 8 ? tmp_small : (double *)malloc(sizeof(double) * 2 * p);
  for (int k = 0; k < m; ++k) {
    for (int s = 0; s < p; ++s) {
      double ar = 0.0, ai = 0.0;
      for (int r = 0; r < p; ++r) {
        /* exponent of W_n: r (k + m s) mod n, with r (k + m s) < p n; the
         * table holds W_wn^j and W_n = W_wn^wstep (wstep * n = wn) */
        long e = (long)r * (long)(k + m * s);
        while (e >= n) e -= n;
        const double *t = w + 2 * (e * wstep);
        double yr = out[2 * (r * m + k)], yi = out[2 * (r * m + k) + 1];
        ar += yr * t[0] - yi * t[1];
        ai += yr * t[1] + yi * t[0];
      }
      tmp[2 * s] = ar;
      tmp[2 * s + 1] = ai;
    }
    for (int s = 0; s < p; ++s) {
      out[2 * (k + m * s)] = tmp[2 * s];
      out[2 * (k + m * s) + 1] = tmp[2 * s + 1];
    }
  }
  if (tmp != tmp_small) free(tmp);
}

static double *twiddles(int n, int sign) {
  double *w = (double *)malloc(sizeof(double) * 2 * n);
  for (int j = 0; j < n; ++j) {
    double a = 2.0 * PI * (double)j / (double)n;
    w[2 * j] = cos(a);
    w[2 * j + 1] = sign * sin(a);
  }
  return w;
}

static void fft_line(double *z, int n, int sign, const double *w, double *buf) {
  memcpy(buf, z, sizeof(double) * 2 * n);
  fft_rec(buf, 1, z, n, w, 1, n);
  if (sign > 0) {
    double s = 1.0 / (double)n;
    for (int j = 0; j < 2 * n; ++j) z[j] *= s;
  }
}

void orc_fft1(double *z, int32_t n, int32_t sign) {
  double *w = twiddles(n, sign < 0 ? -1 : 1);
  double *buf = (double *)malloc(sizeof(double) * 2 * n);
  fft_line(z, n, sign, w, buf);
  free(buf);
  free(w);
}

/* Worker threads for the line transforms of orc_fft2 (default 1).  The
 * lines of a 2-D transform are independent, and each line is computed the
 * same way whichever thread runs it, so the result does not depend on this
 * count. */
static int g_threads = 1;

void orc_set_threads(int32_t k) { g_threads = k < 1 ? 1 : k; }

void orc_fft2(double *z, int32_t rows, int32_t cols, int32_t sign) {
  int sg = sign < 0 ? -1 : 1;
  int mx = rows > cols ? rows : cols;
  double *wc = twiddles(cols, sg);
  double *wr = twiddles(rows, sg);
  /* rows first, then columns */
#pragma omp parallel num_threads(g_threads) if (g_threads > 1)
  {
    double *buf = (double *)malloc(sizeof(double) * 2 * mx);
    double *line = (double *)malloc(sizeof(double) * 2 * mx);
#pragma omp for schedule(static)
    for (int r = 0; r < rows; ++r) fft_line(z + 2 * (size_t)r * cols, cols, sign, wc, buf);
#pragma omp for schedule(static)
    for (int c = 0; c < cols; ++c) {
      for (int r = 0; r < rows; ++r) {
        line[2 * r] = z[2 * ((size_t)r * cols + c)];
        line[2 * r + 1] = z[2 * ((size_t)r * cols + c) + 1];
      }
      fft_line(line, rows, sign, wr, buf);
      for (int r = 0; r < rows; ++r) {
        z[2 * ((size_t)r * cols + c)] = line[2 * r];
        z[2 * ((size_t)r * cols + c) + 1] = line[2 * r + 1];
      }
    }
    free(line);
    free(buf);
  }
  free(wr);
  free(wc);
}

/* Centring shift by half the size on both axes (even sizes: its own inverse). */
static void shift2(const double *in, double *out, int rows, int cols) {
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) {
      int rr = (r + rows / 2) % rows, cc = (c + cols / 2) % cols;
      out[2 * ((size_t)rr * cols + cc)] = in[2 * ((size_t)r * cols + c)];
      out[2 * ((size_t)rr * cols + cc) + 1] = in[2 * ((size_t)r * cols + c) + 1];
    }
}

/* ------------------------------------------------------------- geometry */

/* Sec. 1 / Sec. 2.1: the frequency-domain constraint is a circular low-pass
 * filter fixed by the objective NA and the wavelength.  Cutoff NA/lambda in
 * cycles/um; with bin spacing dk = 1/(n dx) the radius in bins is
 * r = NA * n * dx / lambda.  D0 = {(u,v): (u-n/2)^2 + (v-n/2)^2 <= r^2}. */
static double support_radius(const orc_geom *g) {
  return g->na * (double)g->n * g->pixel_um / g->wavelength_um;
}

int32_t orc_support(const orc_geom *g, uint8_t *mask) {
  int n = g->n;
  double r = support_radius(g);
  double r2 = r * r;
  int32_t count = 0;
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v) {
      double du = (double)(u - n / 2), dv = (double)(v - n / 2);
      int in = (du * du + dv * dv) <= r2;
      mask[u * n + v] = (uint8_t)in;
      count += in;
    }
  return count;
}

/* Sec. 2.2: each sub-region has its own defocus distance z.  Modelled as the
 * angular-spectrum propagation phase with the piston term removed:
 * phi = 2 pi z (sqrt(1/lambda^2 - k^2) - 1/lambda), written in the
 * cancellation-free form -2 pi z k^2 / (1/lambda + sqrt(1/lambda^2 - k^2)).
 * P_init = exp(i phi) on D0, 0 elsewhere. */
void orc_pupil_init(const orc_geom *g, double *P) {
  int n = g->n;
  uint8_t *mask = (uint8_t *)malloc((size_t)n * n);
  orc_support(g, mask);
  double dk = 1.0 / ((double)n * g->pixel_um);
  double il = 1.0 / g->wavelength_um;
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v) {
      size_t i = (size_t)u * n + v;
      if (!mask[i]) {
        P[2 * i] = 0.0;
        P[2 * i + 1] = 0.0;
        continue;
      }
      double ku = (double)(u - n / 2) * dk, kv = (double)(v - n / 2) * dk;
      double k2 = ku * ku + kv * kv;
      double phi = -2.0 * PI * g->defocus_um * k2 / (il + sqrt(il * il - k2));
      P[2 * i] = cos(phi);
      P[2 * i + 1] = sin(phi);
    }
  free(mask);
}

/* Sec. 2.2 (Figs. 3-4): the illumination angle of a sub-region is set by the
 * LED position on the board, the LED-to-sample height and the sub-region's
 * own position.  For LED (r, c) at board position (x, y) and tile centre
 * (xt, yt): sin(theta_x) = (x - xt)/rho, rho = |(x - xt, y - yt, H)|.  The
 * tilt shifts the object spectrum; the crop centre sits at
 * sin(theta)/lambda, i.e. sin(theta) * n * dx / lambda bins, rounded half up.
 * Window rows [N/2 + drow - n/2, +n), cols [N/2 + dcol - n/2, +n). */
int32_t orc_offsets(const orc_geom *g, int32_t *off) {
  int rows = g->led_rows, cols = g->led_cols;
  int n = g->n, N = g->n * g->up;
  int lim = (N - n) / 2;
  int32_t status = 0;
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) {
      double x = ((double)c - (double)(cols - 1) / 2.0) * g->led_pitch_um + g->led_x0_um;
      double y = ((double)r - (double)(rows - 1) / 2.0) * g->led_pitch_um + g->led_y0_um;
      double ddx = x - g->tile_x_um, ddy = y - g->tile_y_um;
      double h = g->led_height_um;
      double rho = sqrt(ddx * ddx + ddy * ddy + h * h);
      double sx = ddx / rho, sy = ddy / rho;
      int32_t dcol = (int32_t)floor(sx * (double)n * g->pixel_um / g->wavelength_um + 0.5);
      int32_t drow = (int32_t)floor(sy * (double)n * g->pixel_um / g->wavelength_um + 0.5);
      int j = r * cols + c;
      off[2 * j] = drow;
      off[2 * j + 1] = dcol;
      if (abs(drow) > lim || abs(dcol) > lim) status = -2;
    }
  return status;
}

/* Sec. 3.2 (Fig. 6a): the usual sweep goes outward from the centre of the
 * spectrum.  Order = ascending nominal illumination NA of the on-axis board,
 * key (2r - (rows-1))^2 + (2c - (cols-1))^2, ties by grid index
 * (insertion sort on (key, index); no shared state, safe across threads). */
void orc_order(const orc_geom *g, int32_t *order) {
  int rows = g->led_rows, cols = g->led_cols, L = rows * cols;
  long *key = (long *)malloc(sizeof(long) * (size_t)L);
  for (int j = 0; j < L; ++j) {
    long a = 2 * (j / cols) - (rows - 1), b = 2 * (j % cols) - (cols - 1);
    key[j] = a * a + b * b;
  }
  for (int k = 0; k < L; ++k) {
    int j = k, pos = k;
    while (pos > 0 && (key[order[pos - 1]] > key[j] ||
                       (key[order[pos - 1]] == key[j] && order[pos - 1] > j))) {
      order[pos] = order[pos - 1];
      --pos;
    }
    order[pos] = j;
  }
  free(key);
}

/* Sec. 3.2: rearrange the update sequence so that concurrently processed
 * sub-spectrum regions do not affect each other.  Two LEDs conflict when the
 * high-resolution pixels under their supports intersect.  Each LED, in
 * order, joins the first group none of whose members it conflicts with
 * (checked here by stamping pixels), else opens a new group. */
int32_t orc_groups(const orc_geom *g, const int32_t *off, const int32_t *order,
                   int32_t *group_of, int32_t *sweep, int32_t *gstart) {
  int n = g->n, N = g->n * g->up, L = g->led_rows * g->led_cols;
  uint8_t *mask = (uint8_t *)malloc((size_t)n * n);
  orc_support(g, mask);
  uint8_t **stamp = (uint8_t **)calloc((size_t)L, sizeof(uint8_t *));
  int32_t *count = (int32_t *)calloc((size_t)L, sizeof(int32_t));
  int32_t **members = (int32_t **)calloc((size_t)L, sizeof(int32_t *));
  int ng = 0;
  for (int oi = 0; oi < L; ++oi) {
    int j = order[oi];
    int wy = N / 2 + off[2 * j] - n / 2, wx = N / 2 + off[2 * j + 1] - n / 2;
    int chosen = -1;
    for (int gi = 0; gi < ng && chosen < 0; ++gi) {
      int hit = 0;
      for (int u = 0; u < n && !hit; ++u)
        for (int v = 0; v < n; ++v)
          if (mask[u * n + v] && stamp[gi][(size_t)(wy + u) * N + (wx + v)]) {
            hit = 1;
            break;
          }
      if (!hit) chosen = gi;
    }
    if (chosen < 0) {
      chosen = ng++;
      stamp[chosen] = (uint8_t *)calloc((size_t)N * N, 1);
      members[chosen] = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    }
    for (int u = 0; u < n; ++u)
      for (int v = 0; v < n; ++v)
        if (mask[u * n + v]) stamp[chosen][(size_t)(wy + u) * N + (wx + v)] = 1;
    members[chosen][count[chosen]++] = j;
    group_of[j] = chosen;
  }
  int pos = 0;
  for (int gi = 0; gi < ng; ++gi) {
    gstart[gi] = pos;
    for (int k = 0; k < count[gi]; ++k) sweep[pos++] = members[gi][k];
    free(stamp[gi]);
    free(members[gi]);
  }
  gstart[ng] = pos;
  free(stamp);
  free(members);
  free(count);
  free(mask);
  return ng;
}

/* ----------------------------------------------------- state and model */

/* Scaled centred spectrum S = shift(FFT_N(o)) / up^2, so that a unit object
 * under on-axis light yields unit low-resolution intensity. */
void orc_object_to_spectrum(const orc_geom *g, const double *obj, double *S) {
  int N = g->n * g->up;
  size_t nn = (size_t)N * N;
  double *t = (double *)malloc(sizeof(double) * 2 * nn);
  memcpy(t, obj, sizeof(double) * 2 * nn);
  orc_fft2(t, N, N, -1);
  shift2(t, S, N, N);
  double s = 1.0 / ((double)g->up * (double)g->up);
  for (size_t i = 0; i < 2 * nn; ++i) S[i] *= s;
  free(t);
}

/* Object = up^2 * IFFT_N(shift(S)). */
void orc_spectrum_to_object(const orc_geom *g, const double *S, double *obj) {
  int N = g->n * g->up;
  size_t nn = (size_t)N * N;
  shift2(S, obj, N, N);
  orc_fft2(obj, N, N, +1);
  double s = (double)g->up * (double)g->up;
  for (size_t i = 0; i < 2 * nn; ++i) obj[i] *= s;
}

static void window_origin(const orc_geom *g, const int32_t *off, int j, int *wy, int *wx) {
  int n = g->n, N = g->n * g->up;
  *wy = N / 2 + off[2 * j] - n / 2;
  *wx = N / 2 + off[2 * j + 1] - n / 2;
}

/* Sec. 2.1 (Fig. 1): the low-resolution image under LED j is the intensity
 * of the objective-filtered, tilt-shifted object field:
 * I_j = |IFFT_n(shift(P * W_j(S)))|^2. */
void orc_forward(const orc_geom *g, const double *S, const double *P, double *I) {
  int n = g->n, N = g->n * g->up, L = g->led_rows * g->led_cols;
  size_t nn = (size_t)n * n;
  int32_t *off = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)L);
  orc_offsets(g, off);
  double *phi = (double *)malloc(sizeof(double) * 2 * nn);
  double *psi = (double *)malloc(sizeof(double) * 2 * nn);
  for (int j = 0; j < L; ++j) {
    int wy, wx;
    window_origin(g, off, j, &wy, &wx);
    for (int u = 0; u < n; ++u)
      for (int v = 0; v < n; ++v) {
        size_t i = (size_t)u * n + v;
        const double *x = S + 2 * ((size_t)(wy + u) * N + (wx + v));
        phi[2 * i] = P[2 * i] * x[0] - P[2 * i + 1] * x[1];
        phi[2 * i + 1] = P[2 * i] * x[1] + P[2 * i + 1] * x[0];
      }
    shift2(phi, psi, n, n);
    orc_fft2(psi, n, n, +1);
    for (size_t i = 0; i < nn; ++i)
      I[(size_t)j * nn + i] = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
  }
  free(psi);
  free(phi);
  free(off);
}

/* ------------------------------------------------------- reconstruction */

typedef struct {
  const orc_geom *g;
  const uint8_t *mask;
  int n, N;
  double *phi, *psi, *tmp, *X;   /* n*n complex work arrays */
  double e, ref;                 /* FP64 residual accumulators */
} orc_work;

/* One alternating-projection step for LED j (Sec. 2.1 / Fig. 2, with the
 * embedded pupil update; readings in the design notes):
 *   X = W_j(S_read);  Phi = P X;  psi = IFFT(shift Phi)
 *   e += sum (|psi| - sqrt I)^2;  ref += sum I
 *   psi' = sqrt(I) psi/|psi|  (sqrt(I) where psi = 0)
 *   Phi' = shift FFT(psi');  D = Phi' - Phi
 *   X' = X + conj(P) D / max|P|^2  on D0      -> written to S_write
 *   dP = conj(X) D / smax2         on D0      -> added to dP_out
 * Both increments use the pre-update X and P.  Each step size is normalised
 * by the largest squared magnitude of the whole other factor: the whole
 * pupil for the spectrum step, the whole high-resolution spectrum for the
 * pupil step (smax2, taken at the start of the iteration). */
static void ap_step(orc_work *w, const int32_t *off, int j, const float *Ij,
                    const double *Sread, double *Swrite, const double *P, double smax2,
                    double *dP_out) {
  const orc_geom *g = w->g;
  int n = w->n, N = w->N;
  size_t nn = (size_t)n * n;
  int wy, wx;
  window_origin(g, off, j, &wy, &wx);
  double pmax2 = 0.0;
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v) {
      size_t i = (size_t)u * n + v;
      const double *x = Sread + 2 * ((size_t)(wy + u) * N + (wx + v));
      w->X[2 * i] = x[0];
      w->X[2 * i + 1] = x[1];
      w->phi[2 * i] = P[2 * i] * x[0] - P[2 * i + 1] * x[1];
      w->phi[2 * i + 1] = P[2 * i] * x[1] + P[2 * i + 1] * x[0];
      double p2 = P[2 * i] * P[2 * i] + P[2 * i + 1] * P[2 * i + 1];
      if (p2 > pmax2) pmax2 = p2;
    }
  shift2(w->phi, w->psi, n, n);
  orc_fft2(w->psi, n, n, +1);
  for (size_t i = 0; i < nn; ++i) {
    double I = (double)Ij[i];
    double m = sqrt(I > 0.0 ? I : 0.0);
    double a = hypot(w->psi[2 * i], w->psi[2 * i + 1]);
    w->e += (a - m) * (a - m);
    w->ref += I;
    if (a > 0.0) {
      w->psi[2 * i] *= m / a;
      w->psi[2 * i + 1] *= m / a;
    } else {
      w->psi[2 * i] = m;
      w->psi[2 * i + 1] = 0.0;
    }
  }
  orc_fft2(w->psi, n, n, -1);
  shift2(w->psi, w->tmp, n, n);   /* tmp = Phi' */
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v) {
      size_t i = (size_t)u * n + v;
      if (!w->mask[i]) continue;
      double dr = w->tmp[2 * i] - w->phi[2 * i], di = w->tmp[2 * i + 1] - w->phi[2 * i + 1];
      double pr = P[2 * i], pi = P[2 * i + 1];
      double xr = w->X[2 * i], xi = w->X[2 * i + 1];
      double *xo = Swrite + 2 * ((size_t)(wy + u) * N + (wx + v));
      if (pmax2 > 0.0) {
        /* conj(P) * D / pmax2 */
        xo[0] = xr + (pr * dr + pi * di) / pmax2;
        xo[1] = xi + (pr * di - pi * dr) / pmax2;
      }
      if (dP_out && smax2 > 0.0) {
        dP_out[2 * i] += (xr * dr + xi * di) / smax2;
        dP_out[2 * i + 1] += (xr * di - xi * dr) / smax2;
      }
    }
}

/* `first`: NULL for the offline sweep; else the order in which the L images
 * arrive (online strategy, Sec. 3.4 Fig. 7a): the first arrival gives the
 * initial guess and the first iteration updates in arrival order; later
 * iterations follow the schedule's order over the complete stack. */
static int32_t reconstruct(const orc_geom *g, const float *I, int32_t iterations,
                           int32_t pupil_update, int32_t schedule, const int32_t *first,
                           const double *S_in, const double *P_in, double *S_out,
                           double *P_out, double *residual) {
  if (!g || !I || !S_out || !P_out || iterations < 0 || g->n <= 0 || g->n % 2 || g->up < 1 ||
      schedule < 0 || schedule > 2 || (first && schedule != ORC_SEQUENTIAL))
    return -1;
  int n = g->n, N = g->n * g->up, L = g->led_rows * g->led_cols;
  size_t nn = (size_t)n * n, NN = (size_t)N * N;
  int32_t *off = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)L);
  if (orc_offsets(g, off) != 0) {
    free(off);
    return -2;
  }
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
  int32_t *group_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
  int32_t *sweep = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
  int32_t *gstart = (int32_t *)malloc(sizeof(int32_t) * (size_t)(L + 1));
  orc_order(g, order);
  int ng = orc_groups(g, off, order, group_of, sweep, gstart);
  uint8_t *mask = (uint8_t *)malloc(nn);
  int32_t nd0 = orc_support(g, mask);

  orc_work w;
  w.g = g;
  w.mask = mask;
  w.n = n;
  w.N = N;
  w.phi = (double *)malloc(sizeof(double) * 2 * nn);
  w.psi = (double *)malloc(sizeof(double) * 2 * nn);
  w.tmp = (double *)malloc(sizeof(double) * 2 * nn);
  w.X = (double *)malloc(sizeof(double) * 2 * nn);
  double *S = S_out, *P = P_out;

  /* Initial guess (reading: the paper does not state one): S = 0 except the
   * centred n x n window, which takes shift(FFT_n(sqrt I_j0)) of the first
   * LED's image; P = P_init.  The intensity keeps no trace of the
   * illumination tilt (Sec. 2.2: the tilt only shifts the spectrum, and the
   * modulus drops the resulting phase ramp), so sqrt(I_j0) estimates |o| and
   * its spectrum is centred on the object's zero frequency. */
  if (S_in) {
    memcpy(S, S_in, sizeof(double) * 2 * NN);
  } else {
    memset(S, 0, sizeof(double) * 2 * NN);
    int j0 = first ? first[0] : order[0];
    for (size_t i = 0; i < nn; ++i) {
      double v = (double)I[(size_t)j0 * nn + i];
      w.phi[2 * i] = sqrt(v > 0.0 ? v : 0.0);
      w.phi[2 * i + 1] = 0.0;
    }
    orc_fft2(w.phi, n, n, -1);
    shift2(w.phi, w.tmp, n, n);
    const int wy = N / 2 - n / 2, wx = N / 2 - n / 2;
    for (int u = 0; u < n; ++u)
      for (int v = 0; v < n; ++v) {
        double *xo = S + 2 * ((size_t)(wy + u) * N + (wx + v));
        xo[0] = w.tmp[2 * ((size_t)u * n + v)];
        xo[1] = w.tmp[2 * ((size_t)u * n + v) + 1];
      }
  }
  if (P_in)
    memcpy(P, P_in, sizeof(double) * 2 * nn);
  else
    orc_pupil_init(g, P);

  double *dP = (double *)malloc(sizeof(double) * 2 * nn);
  double *S0 = (schedule == ORC_LED_GROUPS) ? (double *)malloc(sizeof(double) * 2 * NN) : NULL;
  double *P0 = (double *)malloc(sizeof(double) * 2 * nn);

  for (int it = 0; it < iterations; ++it) {
    w.e = 0.0;
    w.ref = 0.0;
    double smax2 = 0.0;
    for (size_t i = 0; i < NN; ++i) {
      double a = S[2 * i] * S[2 * i] + S[2 * i + 1] * S[2 * i + 1];
      if (a > smax2) smax2 = a;
    }
    if (schedule == ORC_SEQUENTIAL || schedule == ORC_GROUP_ORDER) {
      const int32_t *seq = (schedule == ORC_SEQUENTIAL) ? (first && it == 0 ? first : order)
                                                         : sweep;
      for (int k = 0; k < L; ++k) {
        int j = seq[k];
        memset(dP, 0, sizeof(double) * 2 * nn);
        ap_step(&w, off, j, I + (size_t)j * nn, S, S, P, smax2, pupil_update ? dP : NULL);
        if (pupil_update)
          for (size_t i = 0; i < 2 * nn; ++i) P[i] += dP[i];
      }
    } else {
      /* Sec. 3.2: members of one group all read the state as it stands at
       * the start of the group; each writes only its own support pixels; the
       * pupil takes the mean of the members' increments. */
      for (int gi = 0; gi < ng; ++gi) {
        memcpy(S0, S, sizeof(double) * 2 * NN);
        memcpy(P0, P, sizeof(double) * 2 * nn);
        memset(dP, 0, sizeof(double) * 2 * nn);
        int cnt = gstart[gi + 1] - gstart[gi];
        for (int k = gstart[gi]; k < gstart[gi + 1]; ++k) {
          int j = sweep[k];
          ap_step(&w, off, j, I + (size_t)j * nn, S0, S, P0, smax2, pupil_update ? dP : NULL);
        }
        if (pupil_update)
          for (size_t i = 0; i < 2 * nn; ++i) P[i] = P0[i] + dP[i] / (double)cnt;
      }
    }
    if (residual) residual[it] = w.ref > 0.0 ? w.e / w.ref : 0.0;
    /* Reading: pupil energy fixed once per iteration (gauge of the P*S
     * product): s = sqrt(|D0| / sum|P|^2), P <- s P, S <- S / s. */
    if (pupil_update) {
      double E = 0.0;
      for (size_t i = 0; i < nn; ++i)
        if (mask[i]) E += P[2 * i] * P[2 * i] + P[2 * i + 1] * P[2 * i + 1];
      if (E > 0.0) {
        double s = sqrt((double)nd0 / E);
        for (size_t i = 0; i < 2 * nn; ++i) P[i] *= s;
        for (size_t i = 0; i < 2 * NN; ++i) S[i] /= s;
      }
    }
  }

  free(P0);
  free(S0);
  free(dP);
  free(w.phi);
  free(w.psi);
  free(w.tmp);
  free(w.X);
  free(mask);
  free(gstart);
  free(sweep);
  free(group_of);
  free(order);
  free(off);
  return 0;
}

int32_t orc_reconstruct(const orc_geom *g, const float *I, int32_t iterations,
                        int32_t pupil_update, int32_t schedule, const double *S_in,
                        const double *P_in, double *S_out, double *P_out, double *residual) {
  return reconstruct(g, I, iterations, pupil_update, schedule, NULL, S_in, P_in, S_out, P_out,
                     residual);
}

int32_t orc_reconstruct_online(const orc_geom *g, const float *I, int32_t iterations,
                               int32_t pupil_update, const int32_t *arrival, double *S_out,
                               double *P_out, double *residual) {
  if (!arrival) return -1;
  const int L = g ? g->led_rows * g->led_cols : 0;
  char *seen = (char *)calloc((size_t)(L > 0 ? L : 1), 1);
  for (int k = 0; k < L; ++k) {
    if (arrival[k] < 0 || arrival[k] >= L || seen[arrival[k]]) {
      free(seen);
      return -1;
    }
    seen[arrival[k]] = 1;
  }
  free(seen);
  return reconstruct(g, I, iterations, pupil_update, ORC_SEQUENTIAL, arrival, NULL, NULL, S_out,
                     P_out, residual);
}

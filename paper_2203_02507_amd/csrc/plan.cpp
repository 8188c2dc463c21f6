// Host FP64 plan: per-tile geometry, processing order and LED groups.
//
// Everything here is integer or FP64 host arithmetic evaluated in the exact
// expression order documented in include/fpm.h, so that the integer tables
// are reproducible bit for bit by any other FP64 implementation of the same
// formulas.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "fpm_internal.h"

namespace fpm {

namespace {

constexpr double kPi = 3.14159265358979323846;

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Sec. 1 / Sec. 2.1: the frequency support is a disc of radius NA/lambda,
// i.e. r = NA * n * dx / lambda bins on an n-point grid of spacing 1/(n dx).
void build_support(TilePlan& tp) {
  const int n = tp.n;
  const double r = tp.d.na_obj * (double)n * tp.d.pixel_um / tp.d.wavelength_um;
  const double r2 = r * r;
  tp.mask.assign((size_t)n * n, 0);
  tp.nd0 = 0;
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v) {
      const double du = (double)(u - n / 2), dv = (double)(v - n / 2);
      const bool in = (du * du + dv * dv) <= r2;
      tp.mask[(size_t)u * n + v] = in;
      tp.nd0 += in;
    }
  // column chords: the rows of D0 in column kx form one interval (convex set)
  tp.chord.assign((size_t)2 * n, 0);
  int first = -1, last = -1;
  for (int v = 0; v < n; ++v) {
    int lo = n, hi = -1;
    for (int u = 0; u < n; ++u)
      if (tp.mask[(size_t)u * n + v]) {
        lo = std::min(lo, u);
        hi = std::max(hi, u);
      }
    tp.chord[2 * v] = lo;
    tp.chord[2 * v + 1] = hi;
    if (hi >= lo) {
      if (first < 0) first = v;
      last = v;
    }
  }
  tp.kx0 = first < 0 ? 0 : first;
  tp.nd = first < 0 ? 0 : last - first + 1;
}

// Sec. 2.2: the defocus of the sub-region enters as the angular-spectrum
// propagation phase without its piston, evaluated in the cancellation-free
// form phi = -2 pi z k^2 / (1/lambda + sqrt(1/lambda^2 - k^2)).
void build_pupil(TilePlan& tp) {
  const int n = tp.n;
  const double dk = 1.0 / ((double)n * tp.d.pixel_um);
  const double il = 1.0 / tp.d.wavelength_um;
  tp.pupil0.assign((size_t)2 * n * n, 0.0f);
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v) {
      const size_t i = (size_t)u * n + v;
      if (!tp.mask[i]) continue;
      const double ku = (double)(u - n / 2) * dk, kv = (double)(v - n / 2) * dk;
      const double k2 = ku * ku + kv * kv;
      const double phi = -2.0 * kPi * tp.d.defocus_um * k2 / (il + std::sqrt(il * il - k2));
      tp.pupil0[2 * i] = (float)std::cos(phi);
      tp.pupil0[2 * i + 1] = (float)std::sin(phi);
    }
}

// Sec. 2.2 (Figs. 3-4): LED position and height give the sub-region's
// illumination angle; the tilt shifts the spectrum by sin(theta)/lambda.
bool build_offsets(TilePlan& tp, std::string& err) {
  const fpm_tile_desc& d = tp.d;
  const int rows = d.led_rows, cols = d.led_cols, n = tp.n, N = tp.N;
  const int lim = (N - n) / 2;
  tp.off.assign((size_t)2 * tp.L, 0);
  tp.min_tie = 1.0;
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) {
      const double x = ((double)c - (double)(cols - 1) / 2.0) * d.led_pitch_um + d.led_origin_x_um;
      const double y = ((double)r - (double)(rows - 1) / 2.0) * d.led_pitch_um + d.led_origin_y_um;
      const double ex = x - d.tile_x_um, ey = y - d.tile_y_um;
      const double h = d.led_height_um;
      const double rho = std::sqrt(ex * ex + ey * ey + h * h);
      const double sx = ex / rho, sy = ey / rho;
      const double vx = sx * (double)n * d.pixel_um / d.wavelength_um;
      const double vy = sy * (double)n * d.pixel_um / d.wavelength_um;
      const int dcol = (int)std::floor(vx + 0.5);
      const int drow = (int)std::floor(vy + 0.5);
      const int j = r * cols + c;
      tp.off[2 * j] = drow;
      tp.off[2 * j + 1] = dcol;
      tp.min_tie = std::min(tp.min_tie, std::fabs(vx - std::floor(vx) - 0.5));
      tp.min_tie = std::min(tp.min_tie, std::fabs(vy - std::floor(vy) - 0.5));
      if (std::abs(drow) > lim || std::abs(dcol) > lim) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "LED (%d,%d) crop offset (%d,%d) exceeds (N-n)/2 = %d; raise upsample", r,
                      c, drow, dcol, lim);
        err = buf;
        return false;
      }
    }
  return true;
}

// Sec. 3.2 (Fig. 6a): outward sweep = ascending nominal illumination NA.
void build_order(TilePlan& tp) {
  const int rows = tp.d.led_rows, cols = tp.d.led_cols;
  tp.order.resize(tp.L);
  for (int j = 0; j < tp.L; ++j) tp.order[j] = j;
  auto key = [&](int j) {
    const long a = 2L * (j / cols) - (rows - 1), b = 2L * (j % cols) - (cols - 1);
    return a * a + b * b;
  };
  std::stable_sort(tp.order.begin(), tp.order.end(), [&](int a, int b) {
    const long ka = key(a), kb = key(b);
    return ka != kb ? ka < kb : a < b;
  });
}

// Sec. 3.2: rearrange the sweep so that concurrently updated sub-spectra do
// not interact.  LEDs j, k conflict iff their support discs, placed at their
// offsets, share a high-resolution pixel, i.e. iff the offset difference
// (dr, dc) lies in the difference set D0 - D0.  Row u1 of D0 (columns
// [a1, b1]) meets row u1 + dr (columns [a2, b2]) under a column shift dc iff
// a2 - b1 <= dc <= b2 - a1; the stencil marks every such (dr, dc).
// Groups: greedy first fit over the processing order.
// Conflict relation of two LEDs: their windows on the high-resolution grid
// share a support pixel, i.e. the offset difference lies in D0 - D0 (Sec.
// 3.2).  D0 - D0 as a (2n-1)^2 stencil built from the row intervals of D0.
struct Conflicts {
  int n = 0, W = 0;
  std::vector<uint8_t> stencil;
  const TilePlan* tp = nullptr;
  bool operator()(int j, int k) const {
    const int dr = tp->off[2 * k] - tp->off[2 * j], dc = tp->off[2 * k + 1] - tp->off[2 * j + 1];
    if (dr <= -n || dr >= n || dc <= -n || dc >= n) return false;
    return stencil[(size_t)(dr + n - 1) * W + (dc + n - 1)] != 0;
  }
};
Conflicts make_conflicts(const TilePlan& tp);

void build_groups(TilePlan& tp) {
  const Conflicts conflict = make_conflicts(tp);
  std::vector<std::vector<int>> groups;
  tp.group_of.assign(tp.L, -1);
  for (int j : tp.order) {
    int chosen = -1;
    for (size_t g = 0; g < groups.size() && chosen < 0; ++g) {
      bool ok = true;
      for (int k : groups[g])
        if (conflict(j, k)) {
          ok = false;
          break;
        }
      if (ok) chosen = (int)g;
    }
    if (chosen < 0) {
      chosen = (int)groups.size();
      groups.emplace_back();
    }
    groups[chosen].push_back(j);
    tp.group_of[j] = chosen;
  }
  tp.ngroups = (int)groups.size();
  tp.sweep.clear();
  tp.gstart.clear();
  tp.max_group = 0;
  for (auto& g : groups) {
    tp.gstart.push_back((int)tp.sweep.size());
    tp.sweep.insert(tp.sweep.end(), g.begin(), g.end());
    tp.max_group = std::max(tp.max_group, (int)g.size());
  }
  tp.gstart.push_back((int)tp.sweep.size());
}

Conflicts make_conflicts(const TilePlan& tp) {
  Conflicts c;
  const int n = tp.n, W = 2 * n - 1;
  c.n = n;
  c.W = W;
  c.tp = &tp;
  std::vector<int> rlo(n, n), rhi(n, -1);
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v)
      if (tp.mask[(size_t)u * n + v]) {
        rlo[u] = std::min(rlo[u], v);
        rhi[u] = std::max(rhi[u], v);
      }
  c.stencil.assign((size_t)W * W, 0);
  // pixel of j at window offset a equals pixel of k at offset b: a - b = off_k - off_j
  for (int dr = -(n - 1); dr <= n - 1; ++dr)
    for (int u1 = 0; u1 < n; ++u1) {
      const int u2 = u1 + dr;
      if (u2 < 0 || u2 >= n || rhi[u1] < rlo[u1] || rhi[u2] < rlo[u2]) continue;
      const int lo = rlo[u2] - rhi[u1], hi = rhi[u2] - rlo[u1];
      for (int dc = lo; dc <= hi; ++dc) c.stencil[(size_t)(dr + n - 1) * W + (dc + n - 1)] = 1;
    }
  return c;
}

// The whole sweep as levels of independent updates.  Iteration-aligned
// schedules: level = one step of one iteration, the iteration ends after its
// last step.  PIPELINED (Sec. 3.2 Fig. 6b/d): the updates (k, j) of the
// sequential NA-order sweep, iterations unrolled, each at 1 + the highest
// level of an earlier update it conflicts with (its own LED's previous
// update included); with pupil recovery every update shares the pupil, so
// each depends on the one before it.
void build_program(TilePlan& tp) {
  tp.prog_led.clear();
  tp.prog_iter.clear();
  tp.prog_beg.assign(1, 0);
  tp.prog_end.clear();
  const int K = tp.d.iterations;
  if (tp.d.schedule != FPM_SCHED_PIPELINED) {
    for (int k = 0; k < K; ++k)
      for (int s = 0; s < tp.nsteps; ++s) {
        for (int m = tp.step_beg[s]; m < tp.step_beg[s + 1]; ++m) {
          tp.prog_led.push_back(tp.step_leds[m]);
          tp.prog_iter.push_back(k);
        }
        tp.prog_beg.push_back((int)tp.prog_led.size());
        tp.prog_end.push_back(s + 1 == tp.nsteps ? k : -1);
      }
    tp.nlevels = (int)tp.prog_end.size();
    return;
  }
  const Conflicts conflict = make_conflicts(tp);
  std::vector<std::vector<int>> conf(tp.L);
  for (int j = 0; j < tp.L; ++j)
    for (int k = 0; k < tp.L; ++k)
      if (conflict(j, k)) conf[j].push_back(k);
  std::vector<int> last(tp.L, 0);  // level of each LED's latest update (0: none yet)
  std::vector<int> lvl_of;         // level of update (k, position in order)
  std::vector<int> iter_end(K, 0);
  int top = 0;
  for (int k = 0; k < K; ++k)
    for (int j : tp.order) {
      int lv = 0;
      if (tp.d.pupil_update) {
        lv = top + 1;
      } else {
        for (int c : conf[j]) lv = std::max(lv, last[c]);
        lv += 1;
      }
      last[j] = lv;
      top = std::max(top, lv);
      iter_end[k] = std::max(iter_end[k], lv);
      lvl_of.push_back(lv);
    }
  tp.nlevels = top;
  // bucket the updates by level, in sweep order within a level
  std::vector<int> count(top + 2, 0);
  for (int lv : lvl_of) ++count[lv];
  std::vector<int> start(top + 2, 0);
  for (int g = 1; g <= top; ++g) start[g + 1] = start[g] + count[g];
  tp.prog_led.assign(lvl_of.size(), 0);
  tp.prog_iter.assign(lvl_of.size(), 0);
  std::vector<int> fill(start);
  for (size_t u = 0; u < lvl_of.size(); ++u) {
    const int at = fill[lvl_of[u]]++;
    tp.prog_led[at] = tp.order[u % tp.L];
    tp.prog_iter[at] = (int)(u / tp.L);
  }
  tp.prog_beg.clear();
  tp.prog_end.assign(top, -1);
  for (int g = 1; g <= top + 1; ++g) tp.prog_beg.push_back(start[g]);
  for (int k = 0; k < K; ++k) tp.prog_end[iter_end[k] - 1] = k;
}

void build_steps(TilePlan& tp) {
  tp.step_leds.clear();
  tp.step_beg.clear();
  switch (tp.d.schedule) {
    case FPM_SCHED_LED_GROUPS:
      tp.step_leds = tp.sweep;
      tp.step_beg = tp.gstart;
      break;
    case FPM_SCHED_GROUP_ORDER:
      tp.step_leds = tp.sweep;
      for (int s = 0; s <= tp.L; ++s) tp.step_beg.push_back(s);
      break;
    default:
      tp.step_leds = tp.order;
      for (int s = 0; s <= tp.L; ++s) tp.step_beg.push_back(s);
      break;
  }
  tp.nsteps = (int)tp.step_beg.size() - 1;
}

}  // namespace

fpm_status build_tile_plan(const fpm_tile_desc& d, TilePlan& tp, std::string& err) {
  tp = TilePlan{};
  tp.d = d;
  if (d.n != 64 && d.n != 96 && d.n != 128 && d.n != 256) {
    err = "tile side n must be 64, 96, 128 or 256";
    return FPM_E_UNSUPPORTED;
  }
  if (d.n == 256 && d.precision != FPM_PREC_FP32_FFT) {
    err = "the MFMA precision variant runs tile sides 64, 96 and 128";
    return FPM_E_UNSUPPORTED;
  }
  if (d.upsample < 1 || d.upsample > 8 || d.led_rows < 1 || d.led_cols < 1 ||
      d.led_rows * d.led_cols > 4096 || d.iterations < 0 || d.iterations > 100000 ||
      (d.pupil_update != 0 && d.pupil_update != 1) || d.schedule < 0 || d.schedule > 3 ||
      d.precision < 0 || d.precision > 2) {
    err = "tile descriptor field out of range";
    return FPM_E_ARG;
  }
  if (!finite_pos(d.led_pitch_um) || !finite_pos(d.led_height_um) ||
      !finite_pos(d.wavelength_um) || !finite_pos(d.na_obj) || !finite_pos(d.pixel_um) ||
      !std::isfinite(d.led_origin_x_um) || !std::isfinite(d.led_origin_y_um) ||
      !std::isfinite(d.tile_x_um) || !std::isfinite(d.tile_y_um) ||
      !std::isfinite(d.defocus_um)) {
    err = "tile geometry must be finite (and positive for pitch, height, lambda, NA, pixel)";
    return FPM_E_ARG;
  }
  if (d.na_obj >= d.wavelength_um / (2.0 * d.pixel_um)) {
    err = "support radius reaches the Nyquist edge (need NA < lambda / (2 pixel))";
    return FPM_E_ARG;
  }
  if (d.upsample == 7) {
    err = "upsample must have no prime factor above 5 (1-6 or 8)";
    return FPM_E_ARG;
  }
  tp.n = d.n;
  tp.N = d.n * d.upsample;
  tp.L = d.led_rows * d.led_cols;
  build_support(tp);
  if (tp.nd0 == 0) {
    err = "empty frequency support";
    return FPM_E_ARG;
  }
  if (!build_offsets(tp, err)) return FPM_E_GEOMETRY;
  build_order(tp);
  build_groups(tp);
  build_pupil(tp);
  build_steps(tp);
  build_program(tp);
  return FPM_OK;
}

}  // namespace fpm

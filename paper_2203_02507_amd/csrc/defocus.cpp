// Defocus-distance estimation of sub-regions before their reconstruction
// (Sec. 3.4 Fig. 7b, offline strategy: the defocus of each sub-region is
// found from its bright-field images, at least nine, before the HR
// reconstruction; Sec. 2.2: every sub-region has its own defocus).
//
// Per tile: the bright-field LEDs are those whose window's zero-frequency bin
// (n/2 - drow, n/2 - dcol) lies in the support disc D0.  The search runs on
// the smallest centred block of the LED grid holding all of them.  Every
// candidate z of the grid z_lo, z_lo + step, ... <= z_hi becomes one tile of
// a single plan: the block's LEDs and images, the pupil fixed at D0 H_z (no
// pupil recovery), LED groups, `iterations` iterations.  All candidates of
// all tiles run as one batched reconstruction on the GPU (Sec. 3.1: the
// problems are independent), and a candidate's score is its last residual:
// the right defocus pupil makes the images most consistent with one
// spectrum.  z is the vertex of the parabola through the best score and its
// two neighbours (the grid point itself at an end of the grid or where the
// three scores are not convex).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fpm_internal.h"
#include "runtime.h"

using namespace fpm;

namespace {

constexpr int kMinBrightField = 9;

// smallest centred run [start, start + m) of 0..total-1, m of total's
// parity, holding every index in `used`
void centred_span(int total, const std::vector<int>& used, int* start, int* m) {
  for (int k = 2 - total % 2; k <= total; k += 2) {
    const int s = (total - k) / 2;
    bool all = true;
    for (int u : used) all &= u >= s && u < s + k;
    if (all) {
      *start = s;
      *m = k;
      return;
    }
  }
  *start = 0;
  *m = total;
}

struct Block {
  int r0 = 0, c0 = 0, rows = 0, cols = 0, bright = 0;
};

fpm_status search_block(const fpm_tile_desc& d, Block* b, std::string& err) {
  TilePlan tp;
  const fpm_status st = build_tile_plan(d, tp, err);
  if (st != FPM_OK) return st;
  std::vector<int> rows, cols;
  const int n = tp.n;
  for (int j = 0; j < tp.L; ++j) {
    const int u = n / 2 - tp.off[2 * j], v = n / 2 - tp.off[2 * j + 1];
    if (u < 0 || u >= n || v < 0 || v >= n || !tp.mask[(size_t)u * n + v]) continue;
    rows.push_back(j / d.led_cols);
    cols.push_back(j % d.led_cols);
  }
  b->bright = (int)rows.size();
  if (b->bright < kMinBrightField) {
    err = std::to_string(b->bright) + " bright-field LEDs; the estimate needs at least " +
          std::to_string(kMinBrightField);
    return FPM_E_GEOMETRY;
  }
  centred_span(d.led_rows, rows, &b->r0, &b->rows);
  centred_span(d.led_cols, cols, &b->c0, &b->cols);
  return FPM_OK;
}

double vertex(const std::vector<double>& zs, const double* s, int best) {
  const int K = (int)zs.size();
  if (best <= 0 || best >= K - 1) return zs[best];
  const double a = s[best - 1], c0 = s[best], c = s[best + 1];
  const double curv = a - 2.0 * c0 + c;
  if (!(curv > 0.0)) return zs[best];
  return zs[best] + 0.5 * (zs[1] - zs[0]) * (a - c) / curv;
}

}  // namespace

extern "C" {

fpm_status fpm_estimate_defocus(const fpm_tile_desc* tiles, int32_t ntiles, const float* intensity,
                                fpm_mem where, double z_lo, double z_hi, double z_step,
                                int32_t iterations, double* z_out, double* scores_out,
                                int32_t scores_per_tile, void* hip_stream) try {
  if (!tiles || !intensity || !z_out || ntiles < 1 ||
      (where != FPM_MEM_HOST && where != FPM_MEM_DEVICE))
    return fail(FPM_E_ARG, "fpm_estimate_defocus: NULL argument, ntiles < 1 or bad memory kind");
  if (!(z_step > 0.0) || !(z_hi >= z_lo) || !std::isfinite(z_lo) || !std::isfinite(z_hi) ||
      iterations < 1 || iterations > 1000)
    return fail(FPM_E_ARG, "fpm_estimate_defocus: need z_step > 0, z_hi >= z_lo, 1 <= iterations "
                           "<= 1000");
  const int K = (int)std::floor((z_hi - z_lo) / z_step + 1e-6) + 1;
  if (K > 4096) return fail(FPM_E_ARG, "fpm_estimate_defocus: more than 4096 candidates");
  if (scores_out && scores_per_tile < K)
    return fail(FPM_E_ARG, "fpm_estimate_defocus: scores_out holds " +
                               std::to_string(scores_per_tile) + " per tile, " +
                               std::to_string(K) + " candidates");
  std::vector<double> zs(K);
  for (int k = 0; k < K; ++k) zs[k] = z_lo + z_step * k;

  // the block of every tile, and the candidate tiles of one batched plan
  std::vector<Block> blk(ntiles);
  std::vector<fpm_tile_desc> cand;
  cand.reserve((size_t)ntiles * K);
  int64_t in_floats = 0, blk_floats = 0;
  for (int t = 0; t < ntiles; ++t) {
    std::string err;
    const fpm_status st = search_block(tiles[t], &blk[t], err);
    if (st != FPM_OK) return fail(st, "fpm_estimate_defocus: tile " + std::to_string(t) + ": " + err);
    const fpm_tile_desc& d = tiles[t];
    in_floats += (int64_t)d.led_rows * d.led_cols * d.n * d.n;
    blk_floats += (int64_t)K * blk[t].rows * blk[t].cols * d.n * d.n;
    for (int k = 0; k < K; ++k) {
      fpm_tile_desc c = d;
      c.led_rows = blk[t].rows;
      c.led_cols = blk[t].cols;
      c.defocus_um = zs[k];
      c.iterations = iterations;
      c.pupil_update = 0;
      c.schedule = FPM_SCHED_LED_GROUPS;
      c.precision = FPM_PREC_FP32_FFT;
      cand.push_back(c);
    }
  }
  fpm_plan_t* plan = nullptr;
  fpm_status st = fpm_plan(cand.data(), (int32_t)cand.size(), &plan);
  if (st != FPM_OK) return st;
  struct PlanGuard {
    fpm_plan_t* p;
    ~PlanGuard() { fpm_plan_destroy(p); }
  } guard{plan};

  // the block images of each tile, once per candidate, on the device
  hipStream_t s = (hipStream_t)hip_stream;
  DevBuf in_stage, stack, res;
  const float* src = intensity;
  if (where == FPM_MEM_HOST) {
    for (int64_t i = 0; i < in_floats; ++i)
      if (!(intensity[i] >= 0.0f) || !std::isfinite(intensity[i]))
        return fail(FPM_E_ARG, "fpm_estimate_defocus: intensity " + std::to_string(i) +
                                   " is negative or not finite");
    if (!hip_ok(in_stage.alloc(sizeof(float) * in_floats), "hipMalloc(defocus input)", &st) ||
        !hip_ok(hipMemcpyAsync(in_stage.p, intensity, sizeof(float) * in_floats,
                               hipMemcpyHostToDevice, s),
                "H2D intensity", &st))
      return st;
    src = (const float*)in_stage.p;
  }
  if (!hip_ok(stack.alloc(sizeof(float) * blk_floats), "hipMalloc(defocus stack)", &st) ||
      !hip_ok(res.alloc(sizeof(double) * (size_t)ntiles * K * iterations), "hipMalloc(residuals)",
              &st))
    return st;
  {
    float* dst = (float*)stack.p;
    const float* tile_src = src;
    for (int t = 0; t < ntiles; ++t) {
      const fpm_tile_desc& d = tiles[t];
      const size_t img = (size_t)d.n * d.n;
      const Block& b = blk[t];
      float* first = dst;
      for (int r = 0; r < b.rows; ++r) {
        // one run of b.cols consecutive LEDs of the grid row r0 + r
        const size_t j0 = (size_t)(b.r0 + r) * d.led_cols + b.c0;
        if (!hip_ok(hipMemcpyAsync(dst, tile_src + j0 * img, sizeof(float) * img * b.cols,
                                   hipMemcpyDeviceToDevice, s),
                    "gather block images", &st))
          return st;
        dst += img * b.cols;
      }
      const size_t blk_bytes = sizeof(float) * img * b.rows * b.cols;
      for (int k = 1; k < K; ++k, dst += img * b.rows * b.cols)
        if (!hip_ok(hipMemcpyAsync(dst, first, blk_bytes, hipMemcpyDeviceToDevice, s),
                    "replicate block images", &st))
          return st;
      tile_src += img * d.led_rows * d.led_cols;
    }
  }
  st = fpm_reconstruct(plan, (const float*)stack.p, FPM_MEM_DEVICE, nullptr, nullptr,
                       (double*)res.p, hip_stream);
  if (st != FPM_OK) return st;
  std::vector<double> r((size_t)ntiles * K * iterations);
  if (!hip_ok(hipMemcpyAsync(r.data(), res.p, sizeof(double) * r.size(), hipMemcpyDeviceToHost, s),
              "D2H residuals", &st) ||
      !hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize", &st))
    return st;
  std::vector<double> score(K);
  for (int t = 0; t < ntiles; ++t) {
    int best = 0;
    for (int k = 0; k < K; ++k) {
      score[k] = r[((size_t)t * K + k) * iterations + iterations - 1];
      if (!std::isfinite(score[k]))
        return fail(FPM_E_DIVERGED, "fpm_estimate_defocus: tile " + std::to_string(t) +
                                        ": residual not finite at z = " + std::to_string(zs[k]));
      if (score[k] < score[best]) best = k;
    }
    z_out[t] = vertex(zs, score.data(), best);
    if (scores_out) std::memcpy(scores_out + (size_t)t * scores_per_tile, score.data(), sizeof(double) * K);
  }
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_estimate_defocus")

}  // extern "C"

// C ABI entry points for plans (include/fpm.h).  No exception crosses the
// boundary; every failure becomes an fpm_status plus a thread-local message.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "fpm_internal.h"
#include "runtime.h"

struct fpm_plan_s {
  std::vector<fpm::TilePlan> tiles;
  int device = -1;
  fpm::Executor exec;
  std::mutex mu;
  // completion of the last call's device work and the stream it ran on: a
  // call on another stream waits for it first (calls share the plan's state)
  hipEvent_t done_ev = nullptr;
  hipStream_t done_stream = nullptr;
  bool done_armed = false;
};

namespace fpm {
namespace {

bool use_graphs() {
  const char* v = std::getenv("FPM_NO_GRAPH");
  return !(v && v[0] == '1');
}

// Make the plan's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  DeviceGuard(fpm_plan_t* p) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (p->device < 0) p->device = prev;
    if (p->device != prev && hipSetDevice(p->device) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    if (ok && prev >= 0) (void)hipSetDevice(prev);
  }
};

fpm_status ensure_setup(fpm_plan_t* p) {
  if (p->exec.ready) return FPM_OK;
  return p->exec.setup(p->tiles);
}

// A call's device work goes after the previous call's: device-mode calls
// return without waiting, and the next one may come on another stream while
// the first still runs on the plan's state and staging buffers.  A call on
// the same stream as the previous one is ordered already and waits for
// nothing (no cross-stream dependency enters a caller's capture).
fpm_status order_after_previous(fpm_plan_t* p, hipStream_t s) {
  fpm_status st = FPM_OK;
  if (p->done_armed && p->done_stream != s &&
      !hip_ok(hipStreamWaitEvent(s, p->done_ev, 0), "hipStreamWaitEvent(previous call)", &st))
    return st;
  return FPM_OK;
}
fpm_status mark_done(fpm_plan_t* p, hipStream_t s) {
  fpm_status st = FPM_OK;
  if (!p->done_ev &&
      !hip_ok(hipEventCreateWithFlags(&p->done_ev, hipEventDisableTiming), "hipEventCreate", &st))
    return st;
  if (!hip_ok(hipEventRecord(p->done_ev, s), "hipEventRecord(call done)", &st)) return st;
  p->done_stream = s;
  p->done_armed = true;
  return FPM_OK;
}

// The plan's device status word, allocated on first use and cleared for
// this call.
fpm_status clear_status(Executor& ex, hipStream_t s) {
  fpm_status st = FPM_OK;
  if (!hip_ok(ex.status_d.alloc(16), "hipMalloc(status)", &st) ||
      !hip_ok(launch_status_clear((int*)ex.status_d.p, s), "clear status", &st))
    return st;
  return FPM_OK;
}

// Object (finalised), pupil and residual history of every tile into the
// caller's buffers, and nothing of them when the call failed.
//   Host mode: the residuals come back first; if one is not finite the call
//   returns FPM_E_DIVERGED with no output written, else the outputs are
//   copied and the stream synchronised.
//   Device mode: the residuals are checked on the device into the plan's
//   status word (with the intensity check run before the sweep), and every
//   output is copied by a kernel that writes nothing when that word is set;
//   fpm_plan_status reports it once the work has run.
fpm_status collect_outputs(fpm_plan_t* plan, fpm_mem where, void* object_out, void* pupil_out,
                           double* residual_out, hipStream_t s) {
  Executor& ex = plan->exec;
  fpm_status st = FPM_OK;
  const TileDev* tab = (const TileDev*)ex.table.p;
  int* status = (int*)ex.status_d.p;
  if (!hip_ok(ex.res_stage.alloc(sizeof(double) * std::max<int64_t>(1, ex.total_res)), "hipMalloc",
              &st) ||
      !hip_ok(launch_gather(tab, ex.ntiles, ex.res_stage.p, (const int64_t*)ex.r_off_d.p, 3,
                            ex.n_max, s),
              "gather residual", &st))
    return st;
  if (where == FPM_MEM_HOST) {
    std::vector<double> res_host(std::max<int64_t>(1, ex.total_res));
    if (!hip_ok(hipMemcpyAsync(res_host.data(), ex.res_stage.p, sizeof(double) * ex.total_res,
                               hipMemcpyDeviceToHost, s),
                "D2H residual", &st) ||
        !hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize", &st))
      return st;
    for (int64_t i = 0; i < ex.total_res; ++i)
      if (!std::isfinite(res_host[i]))
        return fail(FPM_E_DIVERGED, "fpm_reconstruct: residual became non-finite");
    if (object_out) {
      if (!hip_ok(ex.enqueue_finalize(s), "finalise", &st) ||
          !hip_ok(hipMemcpyAsync(object_out, ex.obj_stage.p, sizeof(float2) * ex.total_obj,
                                 hipMemcpyDeviceToHost, s),
                  "copy object", &st))
        return st;
    }
    if (pupil_out) {
      if (!hip_ok(ex.pupil_stage.alloc(sizeof(float2) * ex.total_pupil), "hipMalloc", &st) ||
          !hip_ok(launch_gather(tab, ex.ntiles, ex.pupil_stage.p, (const int64_t*)ex.p_off_d.p, 1,
                                ex.n_max, s),
                  "gather pupil", &st) ||
          !hip_ok(hipMemcpyAsync(pupil_out, ex.pupil_stage.p, sizeof(float2) * ex.total_pupil,
                                 hipMemcpyDeviceToHost, s),
                  "copy pupil", &st))
        return st;
    }
    if (residual_out) std::memcpy(residual_out, res_host.data(), sizeof(double) * ex.total_res);
    if (!hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize", &st)) return st;
    return FPM_OK;
  }
  if (!hip_ok(launch_check_residuals(tab, ex.ntiles, status, s), "check residuals", &st))
    return st;
  if (object_out) {
    if (!hip_ok(ex.enqueue_finalize(s), "finalise", &st) ||
        !hip_ok(launch_copy_if_ok(object_out, ex.obj_stage.p,
                                  (int64_t)sizeof(float2) * ex.total_obj, status, s),
                "copy object", &st))
      return st;
  }
  if (pupil_out) {
    if (!hip_ok(ex.pupil_stage.alloc(sizeof(float2) * ex.total_pupil), "hipMalloc", &st) ||
        !hip_ok(launch_gather(tab, ex.ntiles, ex.pupil_stage.p, (const int64_t*)ex.p_off_d.p, 1,
                              ex.n_max, s),
                "gather pupil", &st) ||
        !hip_ok(launch_copy_if_ok(pupil_out, ex.pupil_stage.p,
                                  (int64_t)sizeof(float2) * ex.total_pupil, status, s),
                "copy pupil", &st))
      return st;
  }
  if (residual_out &&
      !hip_ok(launch_copy_if_ok(residual_out, ex.res_stage.p,
                                (int64_t)sizeof(double) * ex.total_res, status, s),
              "copy residual", &st))
    return st;
  return FPM_OK;
}

// Host intensities -> ex.I_stage, validated on the way: chunks are checked
// and copied into one of two pinned buffers by host threads, and each chunk's
// upload overlaps the checking of the next.  FPM_E_ARG names the first bad
// value; nothing is launched on the stack then.
fpm_status stage_host_intensities(Executor& ex, const float* src, hipStream_t s) {
  constexpr int64_t kChunk = (int64_t)32 << 20;  // floats per chunk (128 MiB)
  fpm_status st = FPM_OK;
  for (int k = 0; k < 2; ++k) {
    if (!ex.host_pin[k] &&
        !hip_ok(hipHostMalloc(&ex.host_pin[k], sizeof(float) * kChunk, hipHostMallocDefault),
                "hipHostMalloc(intensity staging)", &st))
      return st;
    if (!ex.host_pin_ev[k] &&
        !hip_ok(hipEventCreateWithFlags(&ex.host_pin_ev[k], hipEventDisableTiming),
                "hipEventCreate", &st))
      return st;
  }
  constexpr int kMaxThreads = 16;
  const unsigned hw = std::thread::hardware_concurrency();
  const int nthreads = (int)std::max(1u, std::min((unsigned)kMaxThreads, hw ? hw : 1u));
  bool armed[2] = {false, false};
  for (int64_t c0 = 0, c = 0; c0 < ex.total_I; c0 += kChunk, ++c) {
    const int k = (int)(c & 1);
    const int64_t len = std::min(kChunk, ex.total_I - c0);
    if (armed[k] && !hip_ok(hipEventSynchronize(ex.host_pin_ev[k]), "hipEventSynchronize", &st))
      return st;
    float* dst = (float*)ex.host_pin[k];
    std::array<int64_t, kMaxThreads> bad;
    bad.fill(-1);
    const int64_t part = (len + nthreads - 1) / nthreads;
    auto check = [&](int w) {
      const int64_t b = w * part, e = std::min(len, b + part);
      for (int64_t i = b; i < e; ++i) {
        const float v = src[c0 + i];
        if (!(v >= 0.0f) || !std::isfinite(v)) {
          bad[w] = c0 + i;
          return;
        }
        dst[i] = v;
      }
    };
    // parts 1.. on helper threads, part 0 here; a part whose thread cannot be
    // started also runs here, so no exception leaves the C ABI
    std::vector<std::thread> pool;
    int started = 0;
    try {
      pool.reserve(nthreads - 1);
      for (int w = 1; w < nthreads; ++w) {
        pool.emplace_back(check, w);
        ++started;
      }
    } catch (const std::exception&) {
    }
    check(0);
    for (int w = started + 1; w < nthreads; ++w) check(w);
    for (auto& th : pool) th.join();
    for (int64_t b : bad)
      if (b >= 0) {
        // let the copies already queued finish before the caller reuses anything
        (void)hipStreamSynchronize(s);
        return fail(FPM_E_ARG, "fpm_reconstruct: intensity " + std::to_string(b) +
                                   " is negative or not finite");
      }
    if (!hip_ok(hipMemcpyAsync((float*)ex.I_stage.p + c0, dst, sizeof(float) * len,
                               hipMemcpyHostToDevice, s),
                "H2D intensity", &st) ||
        !hip_ok(hipEventRecord(ex.host_pin_ev[k], s), "hipEventRecord", &st))
      return st;
    armed[k] = true;
  }
  return FPM_OK;
}

}  // namespace
}  // namespace fpm

using namespace fpm;

extern "C" {

const char* fpm_last_error(void) { return g_last_error.c_str(); }

const char* fpm_version(void) { return "fpm-mi355x 0.1 (gfx950)"; }

fpm_status fpm_plan(const fpm_tile_desc* tiles, int32_t ntiles, fpm_plan_t** out) try {
  if (!tiles || !out || ntiles < 1 || ntiles > (1 << 20))
    return fail(FPM_E_ARG, "fpm_plan: NULL argument or ntiles out of range");
  *out = nullptr;
  std::unique_ptr<fpm_plan_t> p(new (std::nothrow) fpm_plan_t());
  if (!p) return fail(FPM_E_NOMEM, "fpm_plan: host allocation failed");
  p->tiles.resize(ntiles);
  int64_t io = 0, oo = 0, po = 0, ro = 0;
  for (int t = 0; t < ntiles; ++t) {
    std::string err;
    const fpm_status s = build_tile_plan(tiles[t], p->tiles[t], err);
    if (s != FPM_OK) return fail(s, "tile " + std::to_string(t) + ": " + err);
    TilePlan& tp = p->tiles[t];
    tp.i_off = io;
    tp.o_off = oo;
    tp.p_off = po;
    tp.r_off = ro;
    io += (int64_t)tp.L * tp.n * tp.n;
    oo += (int64_t)tp.N * tp.N;
    po += (int64_t)tp.n * tp.n;
    ro += tp.d.iterations;
  }
  *out = p.release();
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_plan")

void fpm_plan_destroy(fpm_plan_t* plan) {
  if (!plan) return;
  if (plan->device >= 0) {  // device state exists only once a call has run
    DeviceGuard g(plan);
    (void)hipDeviceSynchronize();
    if (plan->done_ev) (void)hipEventDestroy(plan->done_ev);
    plan->exec.~Executor();
    new (&plan->exec) Executor();
  }
  delete plan;
}

fpm_status fpm_plan_tile_info(const fpm_plan_t* plan, int32_t tile, fpm_tile_info* info) try {
  if (!plan || !info || tile < 0 || tile >= (int)plan->tiles.size())
    return fail(FPM_E_ARG, "fpm_plan_tile_info: bad argument");
  const TilePlan& tp = plan->tiles[tile];
  info->n = tp.n;
  info->N = tp.N;
  info->L = tp.L;
  info->support_count = tp.nd0;
  info->ngroups = tp.ngroups;
  info->max_group = tp.max_group;
  info->steps = tp.nsteps;
  info->iterations = tp.d.iterations;
  info->min_tie_distance = tp.min_tie;
  info->intensity_offset = tp.i_off;
  info->object_offset = tp.o_off;
  info->pupil_offset = tp.p_off;
  info->residual_offset = tp.r_off;
  info->levels = tp.nlevels;
  info->reserved = 0;
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_plan_tile_info")

fpm_status fpm_plan_tables(const fpm_plan_t* plan, int32_t tile, int32_t* offsets, int32_t* order,
                           int32_t* group_of, int32_t* sweep) try {
  if (!plan || tile < 0 || tile >= (int)plan->tiles.size())
    return fail(FPM_E_ARG, "fpm_plan_tables: bad argument");
  const TilePlan& tp = plan->tiles[tile];
  if (offsets) std::memcpy(offsets, tp.off.data(), sizeof(int32_t) * 2 * tp.L);
  if (order) std::memcpy(order, tp.order.data(), sizeof(int32_t) * tp.L);
  if (group_of) std::memcpy(group_of, tp.group_of.data(), sizeof(int32_t) * tp.L);
  if (sweep) std::memcpy(sweep, tp.sweep.data(), sizeof(int32_t) * tp.L);
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_plan_tables")

fpm_status fpm_plan_device_bytes(const fpm_plan_t* plan, size_t* bytes) try {
  if (!plan || !bytes) return fail(FPM_E_ARG, "fpm_plan_device_bytes: bad argument");
  *bytes = plan->exec.device_bytes();
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_plan_device_bytes")

fpm_status fpm_stitch(const void* tiles, int32_t rows, int32_t cols, int32_t side,
                      int32_t overlap, void* out, fpm_mem where, void* hip_stream) try {
  if (!tiles || !out || (where != FPM_MEM_HOST && where != FPM_MEM_DEVICE))
    return fail(FPM_E_ARG, "fpm_stitch: NULL argument or bad memory kind");
  if (rows < 1 || cols < 1 || side < 2 || side > 65536 || overlap < 0 || 2 * overlap > side ||
      (int64_t)rows * cols > (1 << 20))
    return fail(FPM_E_ARG, "fpm_stitch: grid, side or overlap out of range (0 <= overlap <= side/2)");
  const int64_t W = (int64_t)cols * (side - overlap) + overlap;
  const int64_t H = (int64_t)rows * (side - overlap) + overlap;
  if (W * H > ((int64_t)1 << 34)) return fail(FPM_E_ARG, "fpm_stitch: output too large");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t tile_bytes = (size_t)rows * cols * side * side * sizeof(float2);
  const size_t out_bytes = (size_t)W * H * sizeof(float2);
  fpm_status st = FPM_OK;
  DevBuf scratch, tin, tout;
  if (!hip_ok(scratch.alloc(stitch_scratch_bytes(rows, cols)), "hipMalloc(stitch scratch)", &st))
    return st;
  const float2* src = (const float2*)tiles;
  float2* dst = (float2*)out;
  if (where == FPM_MEM_HOST) {
    if (!hip_ok(tin.alloc(tile_bytes), "hipMalloc(stitch input)", &st) ||
        !hip_ok(tout.alloc(out_bytes), "hipMalloc(stitch output)", &st) ||
        !hip_ok(hipMemcpyAsync(tin.p, tiles, tile_bytes, hipMemcpyHostToDevice, s), "H2D tiles",
                &st))
      return st;
    src = (const float2*)tin.p;
    dst = (float2*)tout.p;
  }
  if (!hip_ok(launch_stitch(src, rows, cols, side, overlap, dst, scratch.p, s), "stitch kernels",
              &st))
    return st;
  if (where == FPM_MEM_HOST &&
      !hip_ok(hipMemcpyAsync(out, dst, out_bytes, hipMemcpyDeviceToHost, s), "D2H stitched", &st))
    return st;
  // the scratch (and staging) buffers are freed on return
  if (!hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize", &st)) return st;
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_stitch")

fpm_status fpm_stitch_noalloc(const void* tiles, int32_t rows, int32_t cols, int32_t side,
                              int32_t overlap, void* out, void* hip_stream) try {
  if (!tiles || !out) return fail(FPM_E_ARG, "fpm_stitch_noalloc: NULL argument");
  if (rows < 1 || cols < 1 || side < 2 || side > 65536 || overlap < 0 || 2 * overlap > side)
    return fail(FPM_E_ARG,
                "fpm_stitch_noalloc: grid, side or overlap out of range (0 <= overlap <= side/2)");
  if ((int64_t)rows * cols > kStitchNoAllocMaxTiles)
    return fail(FPM_E_ARG, "fpm_stitch_noalloc: more than " +
                               std::to_string(kStitchNoAllocMaxTiles) +
                               " tiles (the fixed scratch holds at most that many); use fpm_stitch");
  const int64_t W = (int64_t)cols * (side - overlap) + overlap;
  const int64_t H = (int64_t)rows * (side - overlap) + overlap;
  if (W * H > ((int64_t)1 << 34)) return fail(FPM_E_ARG, "fpm_stitch_noalloc: output too large");
  if (stitch_scratch_bytes(rows, cols) > kStitchNoAllocBytes)
    return fail(FPM_E_ARG, "fpm_stitch_noalloc: scratch too small for the grid");
  void* scratch = nullptr;
  fpm_status st = FPM_OK;
  if (!hip_ok(stitch_noalloc_scratch(&scratch), "hipGetSymbolAddress(stitch scratch)", &st))
    return st;
  // every scratch word a call reads is written earlier in the same call, so
  // nothing needs clearing between calls
  if (!hip_ok(launch_stitch((const float2*)tiles, rows, cols, side, overlap, (float2*)out,
                            scratch, (hipStream_t)hip_stream),
              "stitch kernels", &st))
    return st;
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_stitch_noalloc")

fpm_status fpm_forward(fpm_plan_t* plan, const void* object, const void* pupil, float* intensity,
                       fpm_mem where, void* hip_stream) try {
  if (!plan || !object || !intensity || (where != FPM_MEM_HOST && where != FPM_MEM_DEVICE))
    return fail(FPM_E_ARG, "fpm_forward: NULL argument or bad memory kind");
  std::lock_guard<std::mutex> lk(plan->mu);
  if (plan->exec.online_count >= 0)
    return fail(FPM_E_STATE, "fpm_forward: an online session holds the plan");
  DeviceGuard g(plan);
  if (!g.ok) return fail(FPM_E_DEVICE, "fpm_forward: cannot select the plan's device");
  fpm_status st = ensure_setup(plan);
  if (st != FPM_OK) return st;
  Executor& ex = plan->exec;
  hipStream_t s = (hipStream_t)hip_stream;
  if ((st = order_after_previous(plan, s)) != FPM_OK) return st;
  const size_t obj_bytes = sizeof(float2) * ex.total_obj;
  const size_t pup_bytes = sizeof(float2) * ex.total_pupil;
  const size_t int_bytes = sizeof(float) * ex.total_I;
  const hipMemcpyKind h2d = where == FPM_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  const float2* src = (const float2*)object;
  if (where == FPM_MEM_HOST) {
    if (!hip_ok(hipMemcpyAsync(ex.obj_stage.p, object, obj_bytes, h2d, s), "H2D object", &st))
      return st;
    src = (const float2*)ex.obj_stage.p;
  }
  if (pupil) {
    if (!hip_ok(hipMemcpyAsync(ex.fwd_P.p, pupil, pup_bytes, h2d, s), "copy pupil", &st)) return st;
  } else if (!hip_ok(launch_gather((const TileDev*)ex.table.p, ex.ntiles, ex.fwd_P.p,
                                   (const int64_t*)ex.p_off_d.p, 2, ex.n_max, s),
                     "gather initial pupil", &st)) {
    return st;
  }
  float* out = intensity;
  if (where == FPM_MEM_HOST) {
    if (!hip_ok(ex.I_stage.alloc(int_bytes), "hipMalloc(intensity stage)", &st)) return st;
    out = (float*)ex.I_stage.p;
  }
  if (!hip_ok(ex.enqueue_forward(src, out, s), "forward kernels", &st)) return st;
  if (where == FPM_MEM_HOST) {
    if (!hip_ok(hipMemcpyAsync(intensity, out, int_bytes, hipMemcpyDeviceToHost, s), "D2H", &st) ||
        !hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize", &st))
      return st;
  }
  return mark_done(plan, s);
}
FPM_ABI_GUARD("fpm_forward")

fpm_status fpm_reconstruct(fpm_plan_t* plan, const float* intensity, fpm_mem where,
                           void* object_out, void* pupil_out, double* residual_out,
                           void* hip_stream) try {
  if (!plan || !intensity || (where != FPM_MEM_HOST && where != FPM_MEM_DEVICE))
    return fail(FPM_E_ARG, "fpm_reconstruct: NULL argument or bad memory kind");
  std::lock_guard<std::mutex> lk(plan->mu);
  if (plan->exec.online_count >= 0)
    return fail(FPM_E_STATE, "fpm_reconstruct: an online session holds the plan");
  DeviceGuard g(plan);
  if (!g.ok) return fail(FPM_E_DEVICE, "fpm_reconstruct: cannot select the plan's device");
  fpm_status st = ensure_setup(plan);
  if (st != FPM_OK) return st;
  Executor& ex = plan->exec;
  hipStream_t s = (hipStream_t)hip_stream;
  if ((st = order_after_previous(plan, s)) != FPM_OK) return st;
  if ((st = clear_status(ex, s)) != FPM_OK) return st;
  const size_t int_bytes = sizeof(float) * ex.total_I;
  const float* I = intensity;
  if (where == FPM_MEM_HOST) {
    if (!hip_ok(ex.I_stage.alloc(int_bytes), "hipMalloc(intensity stage)", &st)) return st;
    if ((st = stage_host_intensities(ex, intensity, s)) != FPM_OK) return st;
    I = (const float*)ex.I_stage.p;
  } else if (!hip_ok(launch_validate_intensity(intensity, ex.total_I, (int*)ex.status_d.p, s),
                     "validate intensity", &st)) {
    return st;
  }
  if (!hip_ok(launch_set_intensity((TileDev*)ex.table.p, ex.ntiles, I,
                                   (const int64_t*)ex.i_off_d.p, s),
              "set intensity", &st))
    return st;
  if (!hip_ok(ex.run(s, use_graphs()), "reconstruction sweep", &st)) return st;
  st = collect_outputs(plan, where, object_out, pupil_out, residual_out, s);
  const fpm_status md = mark_done(plan, s);
  return st != FPM_OK ? st : md;
}
FPM_ABI_GUARD("fpm_reconstruct")

fpm_status fpm_online_begin(fpm_plan_t* plan, void* hip_stream) try {
  if (!plan) return fail(FPM_E_ARG, "fpm_online_begin: NULL plan");
  std::lock_guard<std::mutex> lk(plan->mu);
  const int L = plan->tiles[0].L;
  for (size_t t = 0; t < plan->tiles.size(); ++t) {
    const TilePlan& tp = plan->tiles[t];
    if (tp.d.schedule != FPM_SCHED_SEQUENTIAL)
      return fail(FPM_E_ARG, "fpm_online_begin: tile " + std::to_string(t) +
                                 " is not FPM_SCHED_SEQUENTIAL (one image, one update)");
    if (tp.L != L)
      return fail(FPM_E_ARG, "fpm_online_begin: tiles differ in LED count (" +
                                 std::to_string(tp.L) + " vs " + std::to_string(L) + ")");
  }
  DeviceGuard g(plan);
  if (!g.ok) return fail(FPM_E_DEVICE, "fpm_online_begin: cannot select the plan's device");
  fpm_status st = ensure_setup(plan);
  if (st != FPM_OK) return st;
  Executor& ex = plan->exec;
  hipStream_t s = (hipStream_t)hip_stream;
  if ((st = order_after_previous(plan, s)) != FPM_OK) return st;
  if (!ex.tuned) {
    // variant timing scribbles on state that the first push initialises
    if (!hip_ok(ex.tune(s), "update-kernel tuning", &st)) return st;
    ex.tuned = true;
  }
  if (ex.online_launch.empty() && (st = ex.online_setup(plan->tiles)) != FPM_OK) return st;
  if (!hip_ok(launch_set_intensity((TileDev*)ex.table.p, ex.ntiles, (const float*)ex.online_I.p,
                                   (const int64_t*)ex.i_off_d.p, s),
              "bind online stack", &st))
    return st;
  if ((st = clear_status(ex, s)) != FPM_OK) return st;
  ex.online_pushed.assign(L, 0);
  ex.online_count = 0;
  return mark_done(plan, s);
}
FPM_ABI_GUARD("fpm_online_begin")

fpm_status fpm_online_push(fpm_plan_t* plan, int32_t led, const float* intensity, fpm_mem where,
                           void* hip_stream) try {
  if (!plan || !intensity || (where != FPM_MEM_HOST && where != FPM_MEM_DEVICE))
    return fail(FPM_E_ARG, "fpm_online_push: NULL argument or bad memory kind");
  std::lock_guard<std::mutex> lk(plan->mu);
  Executor& ex = plan->exec;
  if (ex.online_count < 0) return fail(FPM_E_STATE, "fpm_online_push: no online session");
  const int L = (int)ex.online_pushed.size();
  if (led < 0 || led >= L)
    return fail(FPM_E_ARG, "fpm_online_push: LED " + std::to_string(led) + " out of range");
  if (ex.online_pushed[led])
    return fail(FPM_E_ARG, "fpm_online_push: LED " + std::to_string(led) + " already pushed");
  DeviceGuard g(plan);
  if (!g.ok) return fail(FPM_E_DEVICE, "fpm_online_push: cannot select the plan's device");
  hipStream_t s = (hipStream_t)hip_stream;
  fpm_status st = FPM_OK;
  if ((st = order_after_previous(plan, s)) != FPM_OK) return st;
  const size_t bytes = sizeof(float) * ex.online_push_floats;
  const float* src = intensity;
  if (where == FPM_MEM_HOST) {
    for (int64_t i = 0; i < ex.online_push_floats; ++i) {
      const float v = intensity[i];
      if (!(v >= 0.0f) || !std::isfinite(v))
        return fail(FPM_E_ARG, "fpm_online_push: intensity " + std::to_string(i) +
                                   " is negative or not finite");
    }
    // the pinned staging buffer is free once the previous push's copy has run
    if (ex.online_ev_armed &&
        !hip_ok(hipEventSynchronize(ex.online_ev), "hipEventSynchronize", &st))
      return st;
    std::memcpy(ex.online_pin, intensity, bytes);
    if (!hip_ok(hipMemcpyAsync(ex.online_stage.p, ex.online_pin, bytes, hipMemcpyHostToDevice, s),
                "H2D image", &st) ||
        !hip_ok(hipEventRecord(ex.online_ev, s), "hipEventRecord", &st))
      return st;
    ex.online_ev_armed = true;
    src = (const float*)ex.online_stage.p;
  } else if (!hip_ok(launch_validate_intensity(intensity, ex.online_push_floats,
                                               (int*)ex.status_d.p, s),
                     "validate image", &st)) {
    return st;
  }
  TileDev* tab = (TileDev*)ex.table.p;
  if (!hip_ok(launch_online_scatter(tab, ex.ntiles, src, (const int64_t*)ex.online_src_off_d.p,
                                    (float*)ex.online_I.p, (const int64_t*)ex.i_off_d.p, led, s),
              "scatter image", &st))
    return st;
  if (ex.online_count == 0) {
    // the first image is the initial guess (Sec. 2.1 step 1): its LED plays j0
    if (!hip_ok(launch_set_j0(tab, ex.ntiles, led, s), "set first LED", &st) ||
        !hip_ok(ex.enqueue_range(0, 1, s), "initial state", &st))
      return st;
  }
  for (int c = 0; c < ex.online_classes; ++c) {
    const Launch& l = ex.online_launch[(size_t)led * ex.online_classes + c];
    if (l.count > 0 &&
        !hip_ok(launch_update_class(l, tab, (const Item*)ex.online_items_d.p + l.off, s),
                "update", &st))
      return st;
  }
  ex.online_pushed[led] = 1;
  if (++ex.online_count == L) {
    // iteration 0 is complete: its residual, and the spectrum maximum the
    // next iteration's pupil steps divide by (each chain's own launches)
    for (size_t p = 0; p < ex.parts.size(); ++p) {
      const std::vector<int>& first = ex.part_iter_first[p];
      if (first.empty()) continue;
      const size_t end0 = first.size() > 1 ? (size_t)first[1] : (size_t)ex.parts[p].second;
      for (size_t li = (size_t)first[0]; li < end0; ++li) {
        const Launch::Kind k = ex.launches[li].kind;
        if ((k == Launch::ITER_END || k == Launch::SMAX) &&
            !hip_ok(ex.enqueue_range(li, li + 1, s), "iteration end", &st))
          return st;
      }
    }
  }
  return mark_done(plan, s);
}
FPM_ABI_GUARD("fpm_online_push")

fpm_status fpm_online_finish(fpm_plan_t* plan, fpm_mem where, void* object_out, void* pupil_out,
                             double* residual_out, void* hip_stream) try {
  if (!plan || (where != FPM_MEM_HOST && where != FPM_MEM_DEVICE))
    return fail(FPM_E_ARG, "fpm_online_finish: NULL plan or bad memory kind");
  std::lock_guard<std::mutex> lk(plan->mu);
  Executor& ex = plan->exec;
  if (ex.online_count < 0) return fail(FPM_E_STATE, "fpm_online_finish: no online session");
  if (ex.online_count < (int)ex.online_pushed.size())
    return fail(FPM_E_STATE, "fpm_online_finish: " + std::to_string(ex.online_count) + " of " +
                                 std::to_string(ex.online_pushed.size()) + " LEDs pushed");
  DeviceGuard g(plan);
  if (!g.ok) return fail(FPM_E_DEVICE, "fpm_online_finish: cannot select the plan's device");
  hipStream_t s = (hipStream_t)hip_stream;
  fpm_status st = FPM_OK;
  if ((st = order_after_previous(plan, s)) != FPM_OK) return st;
  // iterations 1.. over the whole stack, in the plan's order, chain by chain
  for (size_t p = 0; p < ex.parts.size(); ++p)
    if (ex.part_iter_first[p].size() > 1 &&
        !hip_ok(ex.enqueue_range((size_t)ex.part_iter_first[p][1], (size_t)ex.parts[p].second, s),
                "remaining iterations", &st))
      return st;
  ex.online_count = -1;
  st = collect_outputs(plan, where, object_out, pupil_out, residual_out, s);
  // the plan's own first LED again for later fpm_reconstruct calls
  fpm_status st2 = FPM_OK;
  if (!hip_ok(hipMemcpyAsync(ex.table.p, ex.host_tiles.data(),
                             sizeof(TileDev) * ex.host_tiles.size(), hipMemcpyHostToDevice, s),
              "restore tile table", &st2) ||
      !hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize", &st2))
    return st != FPM_OK ? st : st2;
  plan->done_armed = false;  // everything has completed
  return st;
}
FPM_ABI_GUARD("fpm_online_finish")

fpm_status fpm_online_abort(fpm_plan_t* plan) try {
  if (!plan) return fail(FPM_E_ARG, "fpm_online_abort: NULL plan");
  std::lock_guard<std::mutex> lk(plan->mu);
  Executor& ex = plan->exec;
  if (ex.online_count < 0) return FPM_OK;
  DeviceGuard g(plan);
  if (!g.ok) return fail(FPM_E_DEVICE, "fpm_online_abort: cannot select the plan's device");
  fpm_status st = FPM_OK;
  ex.online_count = -1;
  if (!hip_ok(hipDeviceSynchronize(), "hipDeviceSynchronize", &st) ||
      !hip_ok(hipMemcpy(ex.table.p, ex.host_tiles.data(), sizeof(TileDev) * ex.host_tiles.size(),
                        hipMemcpyHostToDevice),
              "restore tile table", &st))
    return st;
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_online_abort")

fpm_status fpm_plan_status(fpm_plan_t* plan, fpm_status* status) try {
  if (!plan || !status) return fail(FPM_E_ARG, "fpm_plan_status: NULL argument");
  std::lock_guard<std::mutex> lk(plan->mu);
  *status = FPM_OK;
  if (plan->device < 0 || !plan->exec.status_d.p) return FPM_OK;  // nothing has run
  DeviceGuard g(plan);
  if (!g.ok) return fail(FPM_E_DEVICE, "fpm_plan_status: cannot select the plan's device");
  fpm_status st = FPM_OK;
  if (plan->done_armed &&
      !hip_ok(hipEventSynchronize(plan->done_ev), "hipEventSynchronize(last call)", &st))
    return st;
  int word = 0;
  if (!hip_ok(hipMemcpy(&word, plan->exec.status_d.p, sizeof word, hipMemcpyDeviceToHost),
              "read status", &st))
    return st;
  if (word & 1) {
    *status = FPM_E_ARG;
    g_last_error = "device-mode call: an intensity is negative or not finite (no output written)";
  } else if (word & 2) {
    *status = FPM_E_DIVERGED;
    g_last_error = "device-mode call: a residual became non-finite (no output written)";
  }
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_plan_status")

fpm_status fpm_profile_reconstruct(fpm_plan_t* plan, const float* intensity,
                                   fpm_kernel_time* out, void* hip_stream) try {
  if (!plan || !intensity || !out) return fail(FPM_E_ARG, "fpm_profile_reconstruct: NULL argument");
  std::lock_guard<std::mutex> lk(plan->mu);
  if (plan->exec.online_count >= 0)
    return fail(FPM_E_STATE, "fpm_profile_reconstruct: an online session holds the plan");
  DeviceGuard g(plan);
  if (!g.ok) return fail(FPM_E_DEVICE, "fpm_profile_reconstruct: cannot select the plan's device");
  fpm_status st = ensure_setup(plan);
  if (st != FPM_OK) return st;
  Executor& ex = plan->exec;
  hipStream_t s = (hipStream_t)hip_stream;
  if ((st = order_after_previous(plan, s)) != FPM_OK) return st;
  if (!hip_ok(launch_set_intensity((TileDev*)ex.table.p, ex.ntiles, intensity,
                                   (const int64_t*)ex.i_off_d.p, s),
              "set intensity", &st) ||
      !hip_ok(ex.profile(s, out), "profiled sweep", &st))
    return st;
  return mark_done(plan, s);
}
FPM_ABI_GUARD("fpm_profile_reconstruct")

}  // extern "C"

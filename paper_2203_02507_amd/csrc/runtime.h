// Executor: device state and the launch sequence of a reconstruction.
#pragma once

#include <exception>
#include <string>
#include <vector>

#include "fpm_internal.h"

namespace fpm {

extern thread_local std::string g_last_error;
fpm_status fail(fpm_status s, const std::string& msg);
bool hip_ok(hipError_t e, const char* what, fpm_status* st);

// Handler of the function-try-block around each C ABI entry point that returns
// a status: an exception thrown by host code (an allocation, a thread start)
// becomes FPM_E_NOMEM with its message instead of leaving the C boundary.
#define FPM_ABI_GUARD(name)                                                         \
  catch (const std::exception& e) {                                                 \
    return ::fpm::fail(FPM_E_NOMEM, std::string(name) + ": host failure: " + e.what()); \
  }                                                                                 \
  catch (...) {                                                                     \
    return ::fpm::fail(FPM_E_NOMEM, std::string(name) + ": host failure");          \
  }

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  hipError_t alloc(size_t n);  // (re)allocate to at least n bytes; contents undefined
};

struct Launch {
  enum Kind { INIT, UPDATE, REDUCE, ITER_END, SMAX } kind = INIT;
  int n = 0, nd_max = 0;   // UPDATE, REDUCE: tile side, largest support-column count
  int prec = 0;            // UPDATE: fpm_precision of every item of the launch
  int box_max = 0;         // UPDATE, MFMA: largest support box
  const uint16_t* tabE = nullptr;  // UPDATE, MFMA: DFT tables
  const uint16_t* tabF = nullptr;
  float2* big_scratch = nullptr;   // UPDATE, n = 256: transpose slots
  int roff = -1, rcount = 0;       // UPDATE, group-sequential form: range list slice
  int off = 0, count = 0;  // range in the item / step-tile / tile-id lists
  int iter = 0;            // ITER_END
};

// Launch one update class: the FP32 FFT kernel (prec 0, autotuned variant)
// or the MFMA DFT kernel (prec 1, 2).
// `ranges`: device range list of the group-sequential launches (l.roff >= 0).
hipError_t launch_update_class(const Launch& l, const TileDev* tiles, const Item* items,
                               hipStream_t st, const int2* ranges = nullptr);
// Group-sequential form for a launch with `groups` tile groups (one
// workgroup per group, no group-mean launch): FPM_GROUP_SEQ=1 selects it.
bool use_group_seq(int groups);

// Process-wide choice of update-kernel variant per tile size (autotuned on
// first use; FPM_UPDATE_VARIANT=k forces one).
// The variant used where nothing has been tuned (the server): the four-round
// 8-lane form, the fastest measured at n = 128 (n = 256 runs its 16-lane
// kernel for every variant but 1).
constexpr int kDefaultUpdateVariant = 7;
int update_variant(int n);
void set_update_variant(int n, int v);
bool update_variant_known(int n);

// independent launch sequences (chains of tiles) of one plan
constexpr int kMaxChains = 4;

struct LineLaunch {
  int off = 0, count = 0, len = 0, max_lines = 0, inverse = 0;
};

// Everything one plan needs on the device to run the sweep of all its tiles:
// per-tile state (spectrum, pupil, scratch, residual partials), the work
// lists of every launch, and the captured graph that replays them.
struct Executor {
  bool ready = false;
  bool tuned = false;
  int ntiles = 0;
  int64_t NN_max = 0;
  int64_t total_updates = 0;
  DevBuf state, table, items_d, steps_d, ids_d, jobs_d, ranges_d;
  std::vector<TileDev> host_tiles;
  std::vector<Launch> launches;
  std::vector<LineLaunch> init_line_launches;
  Launch init_ids;
  // concatenated-array offsets per tile (device copies): intensity, object,
  // pupil, residual
  DevBuf i_off_d, o_off_d, p_off_d, r_off_d;
  int64_t total_I = 0, total_obj = 0, total_pupil = 0, total_res = 0;
  int n_max = 0;
  // object finalise / forward staging: complex [total_obj], pupil [total_pupil]
  DevBuf obj_stage, fwd_P, fwd_table, fwd_items, I_stage, res_stage, pupil_stage;
  DevBuf status_d;  // int: status word of the last device-mode call (see launch_status_clear)
  DevBuf big_scratch;  // transpose slots of the n = 256 kernels (allocated if used)
  std::vector<LineLaunch> fin_line_launches, fwd_line_launches;
  struct FwdLaunch {
    int n, nd_max, off, count;
  };
  std::vector<FwdLaunch> fwd_launches;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;

  // launches[0] initialises every tile; chain p (tiles of its own, on a
  // stream of its own) runs launches [parts[p].first, parts[p].second), and
  // part_iter_first[p][k] is its first launch of iteration k
  std::vector<std::pair<int, int>> parts;
  std::vector<std::vector<int>> part_iter_first;
  hipStream_t chain_stream[kMaxChains] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kMaxChains] = {};
  // online reconstruction (one LED's images at a time): the stack the pushes
  // fill, per-(LED, class) update launches of iteration 0 over every tile
  DevBuf online_I, online_items_d, online_src_off_d, online_stage;
  std::vector<Launch> online_launch;  // [led][class]
  int online_classes = 0;
  int64_t online_push_floats = 0;     // floats of one push: sum over tiles of n^2
  std::vector<char> online_pushed;
  int online_count = -1;  // -1: no online session
  // host-buffer reconstructions: two pinned staging chunks and their copy events
  void* host_pin[2] = {nullptr, nullptr};
  hipEvent_t host_pin_ev[2] = {nullptr, nullptr};
  // host pushes: pinned staging, reused once the previous copy has left it
  void* online_pin = nullptr;
  hipEvent_t online_ev = nullptr;
  bool online_ev_armed = false;

  ~Executor();
  fpm_status setup(const std::vector<TilePlan>& tiles);
  // the whole sweep: initialisation on `s`, then the chains on their streams
  // (forked from and joined back into `s`; also under graph capture)
  hipError_t enqueue_sweep(hipStream_t s);
  // launches [begin, end) of the sweep, eagerly
  hipError_t enqueue_range(size_t begin, size_t end, hipStream_t s);
  // online session: per-(LED, class) launches over all tiles (iteration 0)
  fpm_status online_setup(const std::vector<TilePlan>& tiles);
  hipError_t run(hipStream_t s, bool use_graph);
  // time every update-kernel variant on this plan's largest launch of each
  // tile size (before the state is initialised) and keep the fastest
  hipError_t tune(hipStream_t s);
  std::vector<float> tune_ms;  // [n class][variant] mean launch time of the last tuning
  // eager sweep with an event pair around each launch; per-kind totals
  hipError_t profile(hipStream_t s, fpm_kernel_time* out);
  // object_stage <- up^2 IFFT_N(shift(sigma S)) for every tile
  hipError_t enqueue_finalize(hipStream_t s);
  // intensities for every (tile, LED) from obj_stage spectra and fwd_P
  hipError_t enqueue_forward(const float2* obj_src, float* out, hipStream_t s);
  size_t device_bytes() const;
};

}  // namespace fpm

// Serving: a request loop with continuous batching.
//
// Requests are single-tile reconstructions (Sec. 3.1: tiles are independent
// problems).  A host thread admits waiting requests while their device
// footprint fits the budget and a slot is free, keeps every admitted
// request's spectrum and pupil resident, and on each tick runs one whole
// iteration of every admitted request: its dependent steps (one LED, or one
// LED group, Sec. 3.2) go to the stream in order, step s of all requests in
// the same kernels, with one host synchronisation per tick; requests are
// admitted and retired between ticks.  Each request's arithmetic is independent of
// what it is batched with (one workgroup per update, per-tile reductions in
// fixed order), so a result is bitwise the same alone and in a mix.
//
// Device memory: the whole budget is one slab allocated when the server is
// created; requests take first-fit pieces of it and give them back, so the
// request loop itself never calls hipMalloc or hipFree (the tick's work
// lists are sized at creation too and grow only for unusually large
// batches).  The worker holds the server's mutex only to move requests
// between queues and to publish results: the device work of an admission
// (uploads, initial state) and of a retirement (object, copies back) runs
// outside it, so callers submitting or polling are never held up by it.
#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "fpm_internal.h"
#include "runtime.h"

using namespace fpm;

namespace {

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Request {
  uint64_t id = 0;
  TilePlan plan;
  const float* I_user = nullptr;
  fpm_mem where = FPM_MEM_HOST;
  fpm_status status = FPM_PENDING;
  bool cancelled = false;
  fpm_request_stats stats{};
  // device state (one allocation) and the request's table slot
  void* dev = nullptr;
  size_t dev_bytes = 0;
  TileDev td{};
  int slot = -1;
  int slot_id = -1;  // host source of the admission's slot-id upload
  LineJob jobs_host[4] = {};  // host source of the admission's line-job upload
  float2* obj_stage = nullptr;
  float* I_copy = nullptr;
  // progress
  int iter = 0;  // completed iterations (a tick runs one)
  // results (host)
  std::vector<float2> obj, pupil;
  std::vector<double> residual;
  // why the request failed: set by the worker thread, reported by fpm_poll/fpm_wait
  // (the worker's own last-error message is not visible to the caller's thread)
  std::string err;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t footprint(const TilePlan& tp, fpm_mem where) {
  const size_t nn = (size_t)tp.n * tp.n, NN = (size_t)tp.N * tp.N;
  const bool grouped = tp.d.schedule == FPM_SCHED_LED_GROUPS && tp.d.pupil_update;
  size_t b = 0;
  b += align256(NN * 8);                                  // S
  b += align256(nn * 8);                                  // P
  b += align256((grouped ? tp.max_group : 1) * nn * 8);   // dP
  b += 2 * align256((size_t)tp.L * 8);                    // e, i partials
  b += 2 * align256(8);                                   // sigma, smax
  b += align256((size_t)tp.n * 8);                        // chord
  b += align256(nn * 8);                                  // P0
  b += align256((size_t)std::max(1, tp.d.iterations) * 8);
  b += align256(NN * 8);                                  // object stage
  if (where == FPM_MEM_HOST) b += align256((size_t)tp.L * nn * 4);
  b += align256(4 * sizeof(LineJob));
  return b;
}

// First-fit allocator over one device slab.  Pieces are 256-byte aligned;
// free pieces are kept by offset and merged with their neighbours when given
// back.  Host bookkeeping only: giving a piece back does not wait for the
// device, so the caller gives back only memory no queued work still uses.
struct Slab {
  char* base = nullptr;
  size_t size = 0, used = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
  hipError_t init(size_t bytes) {
    size = align256(bytes);
    hipError_t e = hipMalloc(&base, size);
    if (e != hipSuccess) {
      base = nullptr;
      return e;
    }
    free_[0] = size;
    return hipSuccess;
  }
  ~Slab() {
    if (base) (void)hipFree(base);
  }
  void* take(size_t bytes) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      used += bytes;
      return base + off;
    }
    return nullptr;
  }
  void give(void* p, size_t bytes) {
    bytes = align256(bytes);
    size_t off = (size_t)((char*)p - base);
    used -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
};

}  // namespace

// LED updates per slot the tick's work lists are sized for at creation
constexpr size_t kListLedsPerSlot = 441;

struct fpm_server_s {
  size_t budget = 0;
  Slab slab;  // the whole budget, allocated at creation
  int max_slots = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t stream2 = nullptr;  // second half of each tick's batch
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> waiting;
  std::vector<Request*> active;
  std::map<uint64_t, std::unique_ptr<Request>> all;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  // device tables rebuilt per tick
  DevBuf table, items, steps, ids, jobs;
  DevBuf items2, steps2, ids2;  // work lists of the second half
  // host copies of the halves' work lists: they stay alive until the tick's
  // synchronisation, so the asynchronous uploads never read freed memory
  std::vector<Item> host_items[2];
  std::vector<StepTile> host_steps[2];
  std::vector<int> host_ids[2];
  // transpose slots of the n = 256 kernel, one set per half, allocated on first use
  DevBuf big_scratch;
  std::vector<int> free_slots;
  std::vector<TileDev> host_table;
  const int64_t zero_off = 0;  // host source of the retirement's offset upload
  fpm_status fatal = FPM_OK;

  void run();
  bool reserve(Request* r);
  hipError_t admit(Request* r);
  void release(Request* r);
  hipError_t tick(std::vector<Request*>& batch);
  hipError_t tick_part(std::vector<Request*>& batch, int part);
  hipError_t finish(Request* r);
};

// Under the server's mutex: a piece of the slab and a table slot for r, or
// false (nothing taken) when either is missing.
bool fpm_server_s::reserve(Request* r) {
  if (free_slots.empty()) return false;
  const size_t bytes = footprint(r->plan, r->where);
  void* p = slab.take(bytes);
  if (!p) return false;
  r->dev = p;
  r->dev_bytes = bytes;
  r->slot = free_slots.back();
  free_slots.pop_back();
  return true;
}

// Outside the mutex: the request's device state in its reserved piece and
// slot, and its initial state, enqueued on the first stream (the caller
// synchronises once for all requests admitted together).
hipError_t fpm_server_s::admit(Request* r) {
  const TilePlan& tp = r->plan;
  const size_t nn = (size_t)tp.n * tp.n, NN = (size_t)tp.N * tp.N;
  if (tp.d.precision != FPM_PREC_FP32_FFT) {
    const uint16_t *E = nullptr, *F = nullptr;  // built once per process and size
    const hipError_t e = dft_tables(tp.n, tp.d.precision, &E, &F);
    if (e != hipSuccess) return e;
  }
  char* p = (char*)r->dev;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += align256(bytes);
    return q;
  };
  const bool grouped = tp.d.schedule == FPM_SCHED_LED_GROUPS && tp.d.pupil_update;
  TileDev& d = r->td;
  d.S = (float2*)take(NN * 8);
  d.P = (float2*)take(nn * 8);
  d.dP = (float2*)take((grouped ? tp.max_group : 1) * nn * 8);
  d.e_part = (double*)take((size_t)tp.L * 8);
  d.i_part = (double*)take((size_t)tp.L * 8);
  d.sigma = (double*)take(8);
  d.smax = (unsigned*)take(8);
  d.chord = (const int2*)take((size_t)tp.n * 8);
  d.P0 = (const float2*)take(nn * 8);
  d.residual = (double*)take((size_t)std::max(1, tp.d.iterations) * 8);
  r->obj_stage = (float2*)take(NN * 8);
  if (r->where == FPM_MEM_HOST) r->I_copy = (float*)take((size_t)tp.L * nn * 4);
  LineJob* jobs_dev = (LineJob*)take(4 * sizeof(LineJob));
  d.I = r->where == FPM_MEM_HOST ? r->I_copy : r->I_user;
  d.N = tp.N;
  d.L = tp.L;
  d.n = tp.n;
  d.kx0 = tp.kx0;
  d.nd = tp.nd;
  d.nd0 = tp.nd0;
  d.up = tp.d.upsample;
  d.j0 = tp.step_leds.empty() ? 0 : tp.step_leds[0];
  d.wy0_j0 = tp.N / 2 - tp.n / 2;
  d.wx0_j0 = tp.N / 2 - tp.n / 2;
  d.mode = !tp.d.pupil_update ? 0 : (grouped ? 2 : 1);
  d.iters = tp.d.iterations;
  d.e_stride = 0;  // iterations run one at a time: one set of residual partials
  hipError_t e = hipSuccess;
  if (r->where == FPM_MEM_HOST)
    e = hipMemcpyAsync(r->I_copy, r->I_user, (size_t)tp.L * nn * 4, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync((void*)d.chord, tp.chord.data(), (size_t)tp.n * 8, hipMemcpyHostToDevice,
                       stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync((void*)d.P0, tp.pupil0.data(), nn * 8, hipMemcpyHostToDevice, stream);
  // line-FFT jobs: initial window rows/cols (forward), object rows/cols
  // (inverse); the host copy lives in the request until the upload has run
  LineJob* hj = r->jobs_host;
  for (int pass = 0; pass < 2; ++pass) {
    LineJob& j = hj[pass];
    j = LineJob{};
    j.base = d.S + (size_t)d.wy0_j0 * d.N + d.wx0_j0;
    j.line_stride = pass == 0 ? d.N : 1;
    j.elem_stride = pass == 0 ? 1 : d.N;
    j.nlines = d.n;
    j.scale = 1.0f;
    LineJob& f = hj[2 + pass];
    f = LineJob{};
    f.base = r->obj_stage;
    f.line_stride = pass == 0 ? d.N : 1;
    f.elem_stride = pass == 0 ? 1 : d.N;
    f.nlines = d.N;
    f.scale = 1.0f;
    f.modulate = pass == 1;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(jobs_dev, hj, sizeof r->jobs_host, hipMemcpyHostToDevice, stream);
  // the table slot (reserved under the mutex; only the worker writes slots)
  host_table[r->slot] = d;
  TileDev* tab = (TileDev*)table.p;
  if (e == hipSuccess)
    e = hipMemcpyAsync(tab + r->slot, &host_table[r->slot], sizeof(TileDev), hipMemcpyHostToDevice,
                       stream);
  // initial state; the slot id is read from the table entry's own copy, which
  // stays put until the caller's synchronisation
  r->slot_id = r->slot;
  int* ids_d = (int*)r->td.residual;  // scratch until the first iteration ends
  if (e == hipSuccess)
    e = hipMemcpyAsync(ids_d, &r->slot_id, sizeof(int), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = launch_init_state(tab, ids_d, 1, d.n, d.N, stream);
  if (e == hipSuccess) e = launch_line_fft(jobs_dev, 1, d.n, d.n, 0, stream);
  if (e == hipSuccess) e = launch_line_fft(jobs_dev + 1, 1, d.n, d.n, 0, stream);
  if (e == hipSuccess) e = launch_smax(tab, ids_d, 1, d.N * d.N, stream);
  return e;
}

// Under the mutex, with no queued work left on r's memory: its piece of the
// slab and its slot go back.
void fpm_server_s::release(Request* r) {
  if (r->dev) {
    slab.give(r->dev, r->dev_bytes);
    r->dev = nullptr;
  }
  if (r->slot >= 0) {
    free_slots.push_back(r->slot);
    r->slot = -1;
  }
}

// Outside the mutex: the request's object, pupil and residuals, enqueued on
// the first stream into its host vectors (the caller synchronises once for
// all requests retired together).
hipError_t fpm_server_s::finish(Request* r) {
  // object = up^2 IFFT_N(shift(sigma S)): scale into the stage, two passes of line IFFTs
  const TilePlan& tp = r->plan;
  const size_t NN = (size_t)tp.N * tp.N, nn = (size_t)tp.n * tp.n;
  TileDev* tab = (TileDev*)table.p;
  const LineJob* jobs_dev = (const LineJob*)((char*)r->obj_stage + align256(NN * 8) +
                                             (r->where == FPM_MEM_HOST
                                                  ? align256((size_t)tp.L * nn * 4)
                                                  : 0));
  hipError_t e = hipMemcpyAsync(ids.p, &zero_off, sizeof zero_off, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = launch_scale_spectrum(tab + r->slot, 1, r->obj_stage, (const int64_t*)ids.p, tp.N, stream);
  if (e == hipSuccess) e = launch_line_fft(jobs_dev + 2, 1, tp.N, tp.N, 1, stream);
  if (e == hipSuccess) e = launch_line_fft(jobs_dev + 3, 1, tp.N, tp.N, 1, stream);
  r->obj.resize(NN);
  r->pupil.resize(nn);
  r->residual.resize(std::max(1, tp.d.iterations));
  if (e == hipSuccess)
    e = hipMemcpyAsync(r->obj.data(), r->obj_stage, NN * 8, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(r->pupil.data(), r->td.P, nn * 8, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(r->residual.data(), r->td.residual, r->residual.size() * 8,
                       hipMemcpyDeviceToHost, stream);
  return e;
}

// One scheduler tick: one whole iteration of every admitted request, and one
// host synchronisation.  The batch is split in two halves, balanced by update
// work, each on its own stream, so that one half's partial last waves and
// short launches overlap the other half's updates; a request's own launches
// keep their order, so its result does not depend on the split.
hipError_t fpm_server_s::tick(std::vector<Request*>& batch) {
  std::vector<Request*> half[2];
  {
    std::vector<Request*> ord = batch;
    auto cost = [](const Request* r) { return (double)r->plan.L * r->plan.n * r->plan.n; };
    std::stable_sort(ord.begin(), ord.end(),
                     [&](const Request* a, const Request* b) { return cost(a) > cost(b); });
    double load[2] = {0.0, 0.0};
    // split only while a step's launches leave the GPU short of work (fewer
    // than two workgroups per CU on average): then the halves overlap; with
    // more work per step, twice the launches only add their fixed costs
    double items = 0.0;
    int steps_max = 1;
    for (const Request* r : batch) {
      items += r->plan.L;
      steps_max = std::max(steps_max, r->plan.nsteps);
    }
    const char* one = std::getenv("FPM_SERVER_ONE_STREAM");  // 1: never split (comparisons)
    const bool split = !(one && one[0] == '1') && items / steps_max < 160.0;
    for (Request* r : ord) {
      const int p = split && load[1] < load[0] ? 1 : 0;
      half[p].push_back(r);
      load[p] += cost(r);
    }
  }
  hipError_t e = hipSuccess;
  for (int p = 0; p < 2 && e == hipSuccess; ++p)
    if (!half[p].empty()) e = tick_part(half[p], p);
  const hipError_t e0 = hipStreamSynchronize(stream), e1 = hipStreamSynchronize(stream2);
  return e != hipSuccess ? e : (e0 != hipSuccess ? e0 : e1);
}

// One half of a tick on its own stream: the dependent LED-group steps in
// stream order (step s of every request in one launch per (size, precision)
// class, then the group means of step s), then the iteration ends.
hipError_t fpm_server_s::tick_part(std::vector<Request*>& batch, int part) {
  const hipStream_t stream = part ? stream2 : this->stream;
  DevBuf& items = part ? items2 : this->items;
  DevBuf& steps = part ? steps2 : this->steps;
  DevBuf& ids = part ? ids2 : this->ids;
  struct ClassLaunch {
    std::pair<int, int> cls;  // (n, precision)
    size_t off, count;
    int nd_max, box_max;
  };
  int max_steps = 0, n_max = 0;
  for (Request* r : batch) {
    max_steps = std::max(max_steps, r->plan.nsteps);
    n_max = std::max(n_max, r->plan.n);
  }
  std::vector<Item>& flat = host_items[part];
  std::vector<StepTile>& st = host_steps[part];
  flat.clear();
  st.clear();
  std::vector<std::vector<ClassLaunch>> step_launches(max_steps);
  std::vector<std::pair<size_t, size_t>> step_means(max_steps);  // StepTile range per step
  for (int s = 0; s < max_steps; ++s) {
    std::map<std::pair<int, int>, std::vector<Item>> by_cls;
    std::map<std::pair<int, int>, std::pair<int, int>> mx;  // max nd, max MFMA box
    const size_t st0 = st.size();
    for (Request* r : batch) {
      const TilePlan& tp = r->plan;
      if (s >= tp.nsteps) continue;
      const std::pair<int, int> cls{tp.n, tp.d.precision};
      for (int m = tp.step_beg[s]; m < tp.step_beg[s + 1]; ++m) {
        const int j = tp.step_leds[m];
        Item it{};
        it.tile = r->slot;
        it.led = j;
        it.wy0 = tp.N / 2 + tp.off[2 * j] - tp.n / 2;
        it.wx0 = tp.N / 2 + tp.off[2 * j + 1] - tp.n / 2;
        it.slot = m - tp.step_beg[s];
        it.gsize = tp.step_beg[s + 1] - tp.step_beg[s];
        by_cls[cls].push_back(it);
      }
      auto& x = mx[cls];
      x.first = std::max(x.first, tp.nd);
      x.second = std::max(x.second, mfma_box(tp.kx0, tp.nd));
      if (r->td.mode == 2) st.push_back(StepTile{r->slot, tp.step_beg[s + 1] - tp.step_beg[s]});
    }
    step_means[s] = {st0, st.size() - st0};
    for (auto& kv : by_cls) {
      step_launches[s].push_back(
          ClassLaunch{kv.first, flat.size(), kv.second.size(), mx[kv.first].first,
                      mx[kv.first].second});
      flat.insert(flat.end(), kv.second.begin(), kv.second.end());
    }
  }
  hipError_t e = items.alloc(std::max<size_t>(1, flat.size()) * sizeof(Item));
  if (e == hipSuccess) e = steps.alloc(std::max<size_t>(1, st.size()) * sizeof(StepTile));
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(items.p, flat.data(), flat.size() * sizeof(Item), hipMemcpyHostToDevice,
                     stream);
  if (e == hipSuccess && !st.empty())
    e = hipMemcpyAsync(steps.p, st.data(), st.size() * sizeof(StepTile), hipMemcpyHostToDevice,
                       stream);
  const TileDev* tab = (const TileDev*)table.p;
  for (int s = 0; s < max_steps && e == hipSuccess; ++s) {
    for (const ClassLaunch& cl : step_launches[s]) {
      if (e != hipSuccess) break;
      Launch l{};
      l.kind = Launch::UPDATE;
      l.n = cl.cls.first;
      l.prec = cl.cls.second;
      // one update variant per size for the whole process: if no plan has
      // tuned this size yet, the server fixes the default, so served and
      // planned results stay bitwise equal
      if (!update_variant_known(l.n)) set_update_variant(l.n, kDefaultUpdateVariant);
      l.nd_max = cl.nd_max;
      l.box_max = cl.box_max;
      l.count = (int)cl.count;
      if (l.prec != FPM_PREC_FP32_FFT) e = dft_tables(l.n, l.prec, &l.tabE, &l.tabF);
      if (e == hipSuccess && l.n == 256) {
        e = big_scratch.alloc(2 * big_scratch_bytes(256));
        l.big_scratch = (float2*)((char*)big_scratch.p + (size_t)part * big_scratch_bytes(256));
      }
      if (e == hipSuccess) e = launch_update_class(l, tab, (const Item*)items.p + cl.off, stream);
    }
    if (e == hipSuccess && step_means[s].second > 0)
      e = launch_pupil_reduce(tab, (const StepTile*)steps.p + step_means[s].first,
                              (int)step_means[s].second, n_max, stream);
  }
  // iteration ends (residual + normalisation) and the spectrum max for the
  // next iteration, one launch per distinct iteration index
  if (e == hipSuccess) {
    std::map<int, std::vector<int>> by_iter;
    for (Request* r : batch) by_iter[r->iter].push_back(r->slot);
    std::vector<int>& flat_ids = host_ids[part];
    flat_ids.clear();
    for (auto& kv : by_iter) flat_ids.insert(flat_ids.end(), kv.second.begin(), kv.second.end());
    e = hipMemcpyAsync(ids.p, flat_ids.data(), flat_ids.size() * sizeof(int),
                       hipMemcpyHostToDevice, stream);
    size_t off = 0;
    for (auto& kv : by_iter) {
      if (e != hipSuccess) break;
      e = launch_iter_end(tab, (const int*)ids.p + off, (int)kv.second.size(), kv.first, stream);
      if (e == hipSuccess) {
        int nmax = 0;
        for (Request* r : batch) nmax = std::max(nmax, r->plan.N);
        e = launch_smax(tab, (const int*)ids.p + off, (int)kv.second.size(), nmax * nmax, stream);
      }
      off += kv.second.size();
    }
  }
  return e;
}
void fpm_server_s::run() {
  (void)hipSetDevice(device);
  while (true) {
    std::vector<Request*> batch, admitting, retiring;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !waiting.empty() || !active.empty(); });
      if (stop) break;
      // drop cancelled requests (no work of theirs is queued between ticks)
      for (auto it = active.begin(); it != active.end();) {
        if ((*it)->cancelled) {
          release(*it);
          (*it)->status = FPM_E_CANCELLED;
          (*it)->stats.finish_s = now_s(t0);
          it = active.erase(it);
          cv_done.notify_all();
        } else {
          ++it;
        }
      }
      // admission by device footprint and free slots (first come, first
      // served): a piece of the slab and a slot are reserved here, the
      // device work runs below without the mutex
      while (!waiting.empty()) {
        Request* r = waiting.front();
        if (r->cancelled) {
          waiting.pop_front();
          r->status = FPM_E_CANCELLED;
          r->stats.finish_s = now_s(t0);
          cv_done.notify_all();
          continue;
        }
        if (!reserve(r)) break;
        waiting.pop_front();
        admitting.push_back(r);
      }
      batch = active;
    }
    // admissions: every new request's initial state, one synchronisation
    if (!admitting.empty()) {
      std::vector<hipError_t> err(admitting.size(), hipSuccess);
      for (size_t k = 0; k < admitting.size(); ++k) err[k] = admit(admitting[k]);
      const hipError_t se = hipStreamSynchronize(stream);
      const double t_adm = now_s(t0);
      std::lock_guard<std::mutex> lk(mu);
      for (size_t k = 0; k < admitting.size(); ++k) {
        Request* r = admitting[k];
        const hipError_t e = err[k] != hipSuccess ? err[k] : se;
        r->stats.admit_s = t_adm;
        if (e != hipSuccess) {
          release(r);
          r->status = FPM_E_DEVICE;
          r->err = std::string("admission: ") + hipGetErrorString(e);
          cv_done.notify_all();
        } else if (r->plan.d.iterations == 0) {
          retiring.push_back(r);
        } else {
          active.push_back(r);
          batch.push_back(r);
        }
      }
    }
    if (!batch.empty()) {
      hipError_t e;
      try {
        e = tick(batch);
      } catch (const std::exception&) {  // host allocation of the tick's work lists
        e = hipErrorOutOfMemory;
      }
      std::lock_guard<std::mutex> lk(mu);
      if (e != hipSuccess) {
        for (Request* r : batch) {
          release(r);
          r->status = FPM_E_DEVICE;
          r->err = std::string("server tick: ") + hipGetErrorString(e);
        }
        active.clear();
        fatal = FPM_E_DEVICE;
        cv_done.notify_all();
        continue;
      }
      for (auto it = active.begin(); it != active.end();) {
        Request* r = *it;
        r->stats.updates += r->plan.L;  // a tick runs one whole iteration
        if (++r->iter == r->plan.d.iterations) {
          retiring.push_back(r);
          it = active.erase(it);
        } else {
          ++it;
        }
      }
    }
    // retirements: objects and copies back for every finished request, one
    // synchronisation, then the results are published
    if (!retiring.empty()) {
      std::vector<hipError_t> err(retiring.size(), hipSuccess);
      for (size_t k = 0; k < retiring.size(); ++k) err[k] = finish(retiring[k]);
      const hipError_t se = hipStreamSynchronize(stream);
      const double t_fin = now_s(t0);
      std::lock_guard<std::mutex> lk(mu);
      for (size_t k = 0; k < retiring.size(); ++k) {
        Request* r = retiring[k];
        const hipError_t fe = err[k] != hipSuccess ? err[k] : se;
        bool finite = true;
        for (double v : r->residual) finite &= std::isfinite(v);
        release(r);
        r->status = fe != hipSuccess ? FPM_E_DEVICE : (finite ? FPM_OK : FPM_E_DIVERGED);
        if (fe != hipSuccess)
          r->err = std::string("result copy: ") + hipGetErrorString(fe);
        else if (!finite)
          r->err = "residual became non-finite";
        r->stats.finish_s = t_fin;
      }
      cv_done.notify_all();
    }
  }
}

extern "C" {

fpm_status fpm_server_create(size_t hbm_budget_bytes, int32_t max_slots, fpm_server_t** out) try {
  if (!out || max_slots < 1 || max_slots > 65536 || hbm_budget_bytes == 0)
    return fail(FPM_E_ARG, "fpm_server_create: bad argument");
  *out = nullptr;
  std::unique_ptr<fpm_server_s> s(new (std::nothrow) fpm_server_s());
  if (!s) return fail(FPM_E_NOMEM, "fpm_server_create: host allocation failed");
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->t0 = std::chrono::steady_clock::now();
  fpm_status st = FPM_OK;
  // on failure: the streams made so far are destroyed (device buffers free themselves)
  auto undo = [&](fpm_status code) {
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->stream2) (void)hipStreamDestroy(s->stream2);
    return code;
  };
  if (!hip_ok(hipGetDevice(&s->device), "hipGetDevice", &st) ||
      !hip_ok(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate", &st) ||
      !hip_ok(hipStreamCreateWithFlags(&s->stream2, hipStreamNonBlocking), "hipStreamCreate",
              &st) ||
      !hip_ok(s->table.alloc(sizeof(TileDev) * max_slots), "hipMalloc(table)", &st) ||
      !hip_ok(s->ids.alloc(sizeof(int64_t) * std::max(2, max_slots)), "hipMalloc(ids)", &st) ||
      !hip_ok(s->ids2.alloc(sizeof(int64_t) * std::max(2, max_slots)), "hipMalloc(ids)", &st) ||
      // work lists of a tick, sized for every slot holding a 21 x 21 board
      !hip_ok(s->items.alloc(sizeof(Item) * kListLedsPerSlot * max_slots), "hipMalloc(items)",
              &st) ||
      !hip_ok(s->items2.alloc(sizeof(Item) * kListLedsPerSlot * max_slots), "hipMalloc(items)",
              &st) ||
      !hip_ok(s->steps.alloc(sizeof(StepTile) * kListLedsPerSlot * max_slots),
              "hipMalloc(steps)", &st) ||
      !hip_ok(s->steps2.alloc(sizeof(StepTile) * kListLedsPerSlot * max_slots),
              "hipMalloc(steps)", &st) ||
      !hip_ok(s->slab.init(hbm_budget_bytes), "hipMalloc(server slab)", &st))
    return undo(st);
  try {
    s->host_table.assign(max_slots, TileDev{});
    s->free_slots.reserve(max_slots);
    for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    fpm_server_s* raw = s.get();
    s->worker = std::thread([raw] { raw->run(); });
  } catch (const std::exception&) {
    return undo(fail(FPM_E_NOMEM, "fpm_server_create: host allocation or worker start failed"));
  }
  *out = s.release();
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_server_create")

void fpm_server_destroy(fpm_server_t* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamSynchronize(s->stream2);
  for (auto& kv : s->all) s->release(kv.second.get());
  (void)hipStreamDestroy(s->stream);
  (void)hipStreamDestroy(s->stream2);
  delete s;
}

fpm_status fpm_submit(fpm_server_t* s, const fpm_tile_desc* tile, const float* intensity,
                      fpm_mem where, uint64_t* id) try {
  if (!s || !tile || !intensity || !id || (where != FPM_MEM_HOST && where != FPM_MEM_DEVICE))
    return fail(FPM_E_ARG, "fpm_submit: bad argument");
  // the request's latency clock starts when the call is made
  const double t_arrive = now_s(s->t0);
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return fail(FPM_E_NOMEM, "fpm_submit: host allocation failed");
  std::string err;
  const fpm_status ps = build_tile_plan(*tile, r->plan, err);
  if (ps != FPM_OK) return fail(ps, "fpm_submit: " + err);
  if (where == FPM_MEM_HOST) {
    const size_t cnt = (size_t)r->plan.L * r->plan.n * r->plan.n;
    for (size_t i = 0; i < cnt; ++i)
      if (!(intensity[i] >= 0.0f) || !std::isfinite(intensity[i]))
        return fail(FPM_E_ARG, "fpm_submit: intensity " + std::to_string(i) +
                                   " is negative or not finite");
  }
  if (footprint(r->plan, where) > s->budget)
    return fail(FPM_E_NOMEM, "fpm_submit: request footprint exceeds the server budget");
  r->I_user = intensity;
  r->where = where;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fatal != FPM_OK) return fail(s->fatal, "fpm_submit: server stopped after a device error");
  r->id = s->next_id++;
  r->stats.submit_s = t_arrive;
  r->stats.status = FPM_PENDING;
  *id = r->id;
  s->waiting.push_back(r.get());
  s->all[r->id] = std::move(r);
  s->cv_work.notify_all();
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_submit")

static fpm_status collect(fpm_server_t* s, std::unique_lock<std::mutex>& lk, uint64_t id,
                          void* object_out, void* pupil_out, double* residual_out,
                          fpm_request_stats* stats) {
  auto it = s->all.find(id);
  if (it == s->all.end()) return fail(FPM_E_ARG, "fpm_poll: unknown request id");
  Request* r = it->second.get();
  if (r->status == FPM_PENDING) {
    if (stats) {
      *stats = r->stats;
      stats->status = FPM_PENDING;
    }
    return FPM_PENDING;
  }
  const fpm_status st = r->status;
  if (st == FPM_OK) {
    if (object_out) std::memcpy(object_out, r->obj.data(), r->obj.size() * 8);
    if (pupil_out) std::memcpy(pupil_out, r->pupil.data(), r->pupil.size() * 8);
    if (residual_out)
      std::memcpy(residual_out, r->residual.data(), (size_t)r->plan.d.iterations * 8);
  }
  if (stats) {
    *stats = r->stats;
    stats->status = st;
  }
  const std::string why = st == FPM_E_CANCELLED ? std::string("request cancelled")
                                                : "request failed: " + r->err;
  s->all.erase(it);  // frees *r
  (void)lk;
  if (st != FPM_OK) return fail(st, why);
  return FPM_OK;
}

fpm_status fpm_poll(fpm_server_t* s, uint64_t id, void* object_out, void* pupil_out,
                    double* residual_out, fpm_request_stats* stats) try {
  if (!s) return fail(FPM_E_ARG, "fpm_poll: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  return collect(s, lk, id, object_out, pupil_out, residual_out, stats);
}
FPM_ABI_GUARD("fpm_poll")

fpm_status fpm_wait(fpm_server_t* s, uint64_t id, double timeout_s, void* object_out,
                    void* pupil_out, double* residual_out, fpm_request_stats* stats) try {
  if (!s) return fail(FPM_E_ARG, "fpm_wait: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                            std::chrono::duration<double>(std::max(0.0, timeout_s)));
  s->cv_done.wait_until(lk, deadline, [&] {
    auto it = s->all.find(id);
    return it == s->all.end() || it->second->status != FPM_PENDING;
  });
  return collect(s, lk, id, object_out, pupil_out, residual_out, stats);
}
FPM_ABI_GUARD("fpm_wait")

fpm_status fpm_cancel(fpm_server_t* s, uint64_t id) try {
  if (!s) return fail(FPM_E_ARG, "fpm_cancel: NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return fail(FPM_E_ARG, "fpm_cancel: unknown request id");
  it->second->cancelled = true;
  s->cv_work.notify_all();
  return FPM_OK;
}
FPM_ABI_GUARD("fpm_cancel")

}  // extern "C"

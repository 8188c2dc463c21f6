// Executor and C ABI for plans: device state, work lists, hipGraph capture
// and replay of the reconstruction sweep, the forward model.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fpm_internal.h"
#include "runtime.h"

namespace fpm {

thread_local std::string g_last_error;

fpm_status fail(fpm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

bool hip_ok(hipError_t e, const char* what, fpm_status* st) {
  if (e == hipSuccess) return true;
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  *st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? FPM_E_NOMEM : FPM_E_DEVICE;
  return false;
}

// ------------------------------------------------------ variant cache
namespace {
std::mutex g_variant_mu;
std::map<int, int> g_variant;
}  // namespace

int update_variant(int n) {
  // FPM_UPDATE_VARIANT_<n> (one tile size), then FPM_UPDATE_VARIANT (all)
  const std::string one = "FPM_UPDATE_VARIANT_" + std::to_string(n);
  for (const char* name : {one.c_str(), "FPM_UPDATE_VARIANT"})
    if (const char* v = std::getenv(name)) {
      const int k = std::atoi(v);
      if (k >= 0 && k < kUpdateVariants) return k;
    }
  std::lock_guard<std::mutex> lk(g_variant_mu);
  auto it = g_variant.find(n);
  return it == g_variant.end() ? kDefaultUpdateVariant : it->second;
}
void set_update_variant(int n, int v) {
  std::lock_guard<std::mutex> lk(g_variant_mu);
  g_variant[n] = v;
}
bool update_variant_known(int n) {
  if (std::getenv("FPM_UPDATE_VARIANT") ||
      std::getenv(("FPM_UPDATE_VARIANT_" + std::to_string(n)).c_str()))
    return true;
  std::lock_guard<std::mutex> lk(g_variant_mu);
  return g_variant.count(n) != 0;
}

hipError_t launch_update_class(const Launch& l, const TileDev* tiles, const Item* items,
                               hipStream_t st, const int2* ranges) {
  if (l.prec == FPM_PREC_FP32_FFT)
    return launch_update(l.n, tiles, items, l.count, l.nd_max, update_variant(l.n), l.big_scratch,
                         st, l.roff >= 0 ? ranges + l.roff : nullptr, l.rcount);
  return launch_update_mfma(l.n, l.prec, tiles, items, l.count, l.box_max, l.tabE, l.tabF, st);
}

bool use_group_seq(int groups) {
  // Opt-in: it removes the group-mean launch and its pupil-increment traffic,
  // but a step then takes as long as its largest group (one workgroup per
  // group), and group sizes differ between tiles; on the full field that
  // costs more than the group-mean launch saves.
  if (const char* v = std::getenv("FPM_GROUP_SEQ")) return std::atoi(v) != 0 && groups > 0;
  return false;
}

// ------------------------------------------------------------- DevBuf
DevBuf::~DevBuf() {
  if (p) hipFree(p);
}
hipError_t DevBuf::alloc(size_t n) {
  if (p && bytes >= n) return hipSuccess;
  if (p) hipFree(p);
  p = nullptr;
  bytes = 0;
  if (n == 0) return hipSuccess;
  hipError_t e = hipMalloc(&p, n);
  if (e == hipSuccess) bytes = n;
  return e;
}

// ------------------------------------------------------------ Executor
Executor::~Executor() {
  if (graph_exec) hipGraphExecDestroy(graph_exec);
  if (cap_stream) hipStreamDestroy(cap_stream);
  for (int p = 0; p < kMaxChains; ++p) {
    if (chain_stream[p]) hipStreamDestroy(chain_stream[p]);
    if (join_ev[p]) hipEventDestroy(join_ev[p]);
  }
  if (fork_ev) hipEventDestroy(fork_ev);
  if (online_ev) hipEventDestroy(online_ev);
  if (online_pin) hipHostFree(online_pin);
  for (int k = 0; k < 2; ++k) {
    if (host_pin_ev[k]) hipEventDestroy(host_pin_ev[k]);
    if (host_pin[k]) hipHostFree(host_pin[k]);
  }
}

namespace {
int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }
bool piped(const TilePlan& tp) { return tp.d.schedule == FPM_SCHED_PIPELINED; }
}  // namespace

fpm_status Executor::setup(const std::vector<TilePlan>& tiles) {
  fpm_status st = FPM_OK;
  const int T = (int)tiles.size();
  // ---- persistent per-tile state, one allocation
  struct Lay {
    int64_t S, P, dP, e, i, sig, smax, chord, P0, res;
  };
  std::vector<Lay> lay(T);
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    int64_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  for (int t = 0; t < T; ++t) {
    const TilePlan& tp = tiles[t];
    const int64_t nn = (int64_t)tp.n * tp.n, NN = (int64_t)tp.N * tp.N;
    const bool grouped = tp.d.schedule == FPM_SCHED_LED_GROUPS && tp.d.pupil_update;
    lay[t].S = take(NN * 8);
    lay[t].P = take(nn * 8);
    lay[t].dP = take((grouped ? tp.max_group : 1) * nn * 8);
    // residual partials: per iteration for pipelined tiles (iterations overlap)
    const int64_t eparts = (int64_t)tp.L * (piped(tp) ? std::max(1, tp.d.iterations) : 1);
    lay[t].e = take(eparts * 8);
    lay[t].i = take(eparts * 8);
    lay[t].sig = take(8);
    lay[t].smax = take(4);
    lay[t].chord = take((int64_t)tp.n * 8);
    lay[t].P0 = take(nn * 8);
    lay[t].res = take((int64_t)std::max(1, tp.d.iterations) * 8);
  }
  if (!hip_ok(state.alloc((size_t)off), "hipMalloc(state)", &st)) return st;
  char* base = (char*)state.p;
  host_tiles.assign(T, TileDev{});
  for (int t = 0; t < T; ++t) {
    const TilePlan& tp = tiles[t];
    TileDev& d = host_tiles[t];
    d.S = (float2*)(base + lay[t].S);
    d.P = (float2*)(base + lay[t].P);
    d.I = nullptr;
    d.dP = (float2*)(base + lay[t].dP);
    d.e_part = (double*)(base + lay[t].e);
    d.i_part = (double*)(base + lay[t].i);
    d.sigma = (double*)(base + lay[t].sig);
    d.smax = (unsigned*)(base + lay[t].smax);
    d.chord = (const int2*)(base + lay[t].chord);
    d.P0 = (const float2*)(base + lay[t].P0);
    d.residual = (double*)(base + lay[t].res);
    d.N = tp.N;
    d.L = tp.L;
    d.n = tp.n;
    d.kx0 = tp.kx0;
    d.nd = tp.nd;
    d.nd0 = tp.nd0;
    d.up = tp.d.upsample;
    const int j0 = tp.step_leds.empty() ? 0 : tp.step_leds[0];
    d.j0 = j0;
    d.wy0_j0 = tp.N / 2 - tp.n / 2;  // initial spectrum: the centred window
    d.wx0_j0 = tp.N / 2 - tp.n / 2;
    d.mode = !tp.d.pupil_update ? 0 : (tp.d.schedule == FPM_SCHED_LED_GROUPS ? 2 : 1);
    d.iters = tp.d.iterations;
    d.e_stride = piped(tp) ? tp.L : 0;
    // static tables
    if (!hip_ok(hipMemcpy((void*)d.chord, tp.chord.data(), (size_t)tp.n * 8, hipMemcpyHostToDevice),
                "hipMemcpy(chord)", &st))
      return st;
    if (!hip_ok(hipMemcpy((void*)d.P0, tp.pupil0.data(), (size_t)tp.n * tp.n * 8,
                          hipMemcpyHostToDevice),
                "hipMemcpy(P0)", &st))
      return st;
  }
  if (!hip_ok(table.alloc(sizeof(TileDev) * T), "hipMalloc(table)", &st)) return st;

  // ---- work lists
  std::vector<Item> items;
  std::vector<int2> ranges;
  std::vector<StepTile> steptiles;
  std::vector<int> ids;
  launches.clear();
  int max_iter = 0, max_steps = 0;
  // update classes: (n, precision) -> max support-column count, max MFMA box
  std::map<std::pair<int, int>, std::pair<int, int>> uclass;
  std::map<int, int> nclass;  // n -> max nd
  for (const TilePlan& tp : tiles) {
    max_iter = std::max(max_iter, tp.d.iterations);
    max_steps = std::max(max_steps, tp.nsteps);
    nclass[tp.n] = std::max(nclass[tp.n], tp.nd);
    auto& u = uclass[{tp.n, tp.d.precision}];
    u.first = std::max(u.first, tp.nd);
    u.second = std::max(u.second, mfma_box(tp.kx0, tp.nd));
  }
  // number of chains of tiles (see below): four for a plan of one FP32 class
  // of tiles up to 128 px (more of each chain's group-mean and iteration-end
  // launches then overlap other chains' updates), otherwise two (a mixed
  // plan puts its size classes on chains of their own first)
  int P = T >= 2 ? 2 : 1;
  if (uclass.size() == 1 && uclass.begin()->first.first <= 128 &&
      uclass.begin()->first.second == FPM_PREC_FP32_FFT)
    P = std::min(4, T);
  if (const char* v = std::getenv("FPM_CHAINS")) {
    const int k = std::atoi(v);
    if (k >= 1 && k <= kMaxChains) P = std::min(k, T);
  }
  // transpose slots of the n = 256 kernels, one set per chain (chains run concurrently)
  if (nclass.count(256) &&
      !hip_ok(big_scratch.alloc((size_t)P * big_scratch_bytes(256)), "hipMalloc(transpose slots)",
              &st))
    return st;
  std::map<std::pair<int, int>, std::pair<const uint16_t*, const uint16_t*>> utabs;
  for (auto& kv : uclass) {
    if (kv.first.second == FPM_PREC_FP32_FFT) continue;
    const uint16_t *E = nullptr, *F = nullptr;
    if (!hip_ok(dft_tables(kv.first.first, kv.first.second, &E, &F), "DFT tables", &st)) return st;
    utabs[kv.first] = {E, F};
  }
  int maxN = 0;
  for (const TilePlan& tp : tiles) maxN = std::max(maxN, tp.N);
  NN_max = maxN * maxN;

  auto id_range = [&](const std::vector<int>& v) {
    Launch r{};
    r.off = (int)ids.size();
    r.count = (int)v.size();
    ids.insert(ids.end(), v.begin(), v.end());
    return r;
  };
  // init
  {
    std::vector<int> all(T);
    for (int t = 0; t < T; ++t) all[t] = t;
    Launch l = id_range(all);
    l.kind = Launch::INIT;
    launches.push_back(l);
    init_ids = l;
  }
  // Chains: the tiles are split into independent launch sequences that run on
  // streams of their own; one chain's partial last wave of workgroups and its
  // short group-mean launches then overlap the other chain's updates.  A
  // tile's own launches keep their order, so the results do not depend on
  // the split.
  std::vector<int> part_of(T, 0);
  {
    std::vector<int> ord(T);
    for (int t = 0; t < T; ++t) ord[t] = t;
    auto cost = [&](int t) {
      return (double)tiles[t].L * tiles[t].d.iterations * tiles[t].n * tiles[t].n;
    };
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<double> load(P, 0.0);
    // Whole (n, precision) classes go to chains of their own, largest class
    // first: a class's launches then never wait behind another class's in
    // stream order, and the sizes run side by side.  Chains left over after
    // every class has one take tiles of the classes with the most work per
    // chain, balanced by update count, so a single-class plan still splits
    // over P chains.
    std::map<std::pair<int, int>, double> ccost;
    std::map<std::pair<int, int>, int> ccount;
    for (int t = 0; t < T; ++t) {
      ccost[{tiles[t].n, tiles[t].d.precision}] += cost(t);
      ++ccount[{tiles[t].n, tiles[t].d.precision}];
    }
    std::vector<std::pair<double, std::pair<int, int>>> cs;
    for (auto& kv : ccost) cs.push_back({kv.second, kv.first});
    std::stable_sort(cs.begin(), cs.end(),
                     [](const auto& a, const auto& b) { return a.first > b.first; });
    const int C = (int)cs.size();
    std::map<std::pair<int, int>, std::vector<int>> chains_of;
    const bool whole_classes = C >= P;
    if (whole_classes) {
      for (const auto& c : cs) {
        const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        chains_of[c.second] = {q};
        load[q] += c.first;
      }
    } else {
      // one chain per class, the rest to the classes with the most work per chain
      // (never more chains than a class has tiles)
      std::vector<int> nch(C, 1);
      for (int extra = P - C; extra > 0; --extra) {
        int best = -1;
        for (int i = 0; i < C; ++i)
          if (nch[i] < ccount[cs[i].second] &&
              (best < 0 || cs[i].first / nch[i] > cs[best].first / nch[best]))
            best = i;
        if (best < 0) break;
        ++nch[best];
      }
      int next = 0;
      for (int i = 0; i < C; ++i)
        for (int k = 0; k < nch[i]; ++k) chains_of[cs[i].second].push_back(next++);
      P = next;
      load.assign(P, 0.0);
    }
    for (int t : ord) {  // by cost, over the class's chains
      const auto& mine = chains_of[{tiles[t].n, tiles[t].d.precision}];
      int q = mine[0];
      for (int c : mine)
        if (load[c] < load[q] || (load[c] == load[q] && c < q)) q = c;
      part_of[t] = q;
      if (!whole_classes) load[q] += cost(t);
    }
  }
  parts.clear();
  part_iter_first.assign(P, {});
  for (int p = 0; p < P; ++p) {
    float2* chain_scratch =
        big_scratch.p ? (float2*)((char*)big_scratch.p + (size_t)p * big_scratch_bytes(256))
                      : nullptr;
    const int part_begin = (int)launches.size();
    std::vector<int> prev_active;
    int reuse_from = -1;  // first launch index of the previous iteration body
    for (int k = 0; k < max_iter; ++k) {
      std::vector<int> active;
      for (int t = 0; t < T; ++t)
        if (part_of[t] == p && tiles[t].d.iterations > k && !piped(tiles[t])) active.push_back(t);
      const int body_start = (int)launches.size();
      part_iter_first[p].push_back(body_start);
      if (k > 0 && active == prev_active && reuse_from >= 0) {
        // identical work lists: replay the previous iteration's launches
        const int body_len = body_start - reuse_from;
        for (int i = 0; i < body_len; ++i) {
          Launch l = launches[reuse_from + i];
          if (l.kind == Launch::ITER_END) l.iter = k;
          if (l.kind == Launch::SMAX && k + 1 >= max_iter) {
            bool any = false;
            for (int t : active) any |= tiles[t].d.iterations > k + 1;
            if (!any) continue;
          }
          launches.push_back(l);
        }
        reuse_from = body_start;
        prev_active = active;
        continue;
      }
      for (int s = 0; s < max_steps; ++s) {
        std::vector<char> seq_done(T, 0);  // tiles whose group mean runs inside the update
        for (auto& kv : uclass) {
          Launch l{};
          l.kind = Launch::UPDATE;
          l.n = kv.first.first;
          l.prec = kv.first.second;
          l.nd_max = kv.second.first;
          l.box_max = kv.second.second;
          if (l.n == 256) l.big_scratch = chain_scratch;
          if (l.prec != FPM_PREC_FP32_FFT) {
            l.tabE = utabs[kv.first].first;
            l.tabF = utabs[kv.first].second;
          }
          l.off = (int)items.size();
          for (int t : active) {
            const TilePlan& tp = tiles[t];
            if (tp.n != l.n || tp.d.precision != l.prec || s >= tp.nsteps) continue;
            for (int m = tp.step_beg[s]; m < tp.step_beg[s + 1]; ++m) {
              const int j = tp.step_leds[m];
              Item it{};
              it.tile = t;
              it.led = j;
              it.wy0 = tp.N / 2 + tp.off[2 * j] - tp.n / 2;
              it.wx0 = tp.N / 2 + tp.off[2 * j + 1] - tp.n / 2;
              it.slot = m - tp.step_beg[s];
              it.gsize = tp.step_beg[s + 1] - tp.step_beg[s];
              items.push_back(it);
            }
          }
          l.count = (int)items.size() - l.off;
          if (l.count > 0 && l.prec == FPM_PREC_FP32_FFT && l.n <= 128) {
            // items of one tile are contiguous and in slot order
            std::vector<int2> rg;
            for (int i = l.off; i < l.off + l.count;) {
              int j = i;
              while (j < l.off + l.count && items[j].tile == items[i].tile) ++j;
              rg.push_back(make_int2(i - l.off, j - i));
              i = j;
            }
            if (use_group_seq((int)rg.size())) {
              l.roff = (int)ranges.size();
              l.rcount = (int)rg.size();
              ranges.insert(ranges.end(), rg.begin(), rg.end());
              for (const int2& r : rg) seq_done[items[l.off + r.x].tile] = 1;
            }
          }
          if (l.count > 0) launches.push_back(l);
        }
        // pupil means of the groups that ran in this step
        Launch r{};
        r.kind = Launch::REDUCE;
        r.off = (int)steptiles.size();
        int nmax = 0, ndmax = 0;
        for (int t : active) {
          const TilePlan& tp = tiles[t];
          if (host_tiles[t].mode != 2 || s >= tp.nsteps || seq_done[t]) continue;
          steptiles.push_back(StepTile{t, tp.step_beg[s + 1] - tp.step_beg[s]});
          nmax = std::max(nmax, tp.n);
          ndmax = std::max(ndmax, tp.nd);
        }
        r.count = (int)steptiles.size() - r.off;
        r.n = nmax;
        r.nd_max = ndmax;
        if (r.count > 0) launches.push_back(r);
      }
      if (!active.empty()) {
        Launch e = id_range(active);
        e.kind = Launch::ITER_END;
        e.iter = k;
        launches.push_back(e);
      }
      std::vector<int> next;
      for (int t : active)
        if (tiles[t].d.iterations > k + 1) next.push_back(t);
      if (!next.empty()) {
        Launch m = id_range(next);
        m.kind = Launch::SMAX;
        launches.push_back(m);
      }
      reuse_from = body_start;
      prev_active = active;
    }
    // pipelined tiles: their level programs, level g of every such tile in one
    // launch per (n, precision) class, iteration ends where a program has them
    {
      int max_levels = 0;
      for (int t = 0; t < T; ++t)
        if (part_of[t] == p && piped(tiles[t]))
          max_levels = std::max(max_levels, tiles[t].nlevels);
      for (int g = 0; g < max_levels; ++g) {
        for (auto& kv : uclass) {
          Launch l{};
          l.kind = Launch::UPDATE;
          l.n = kv.first.first;
          l.prec = kv.first.second;
          l.nd_max = kv.second.first;
          l.box_max = kv.second.second;
          if (l.n == 256) l.big_scratch = chain_scratch;
          if (l.prec != FPM_PREC_FP32_FFT) {
            l.tabE = utabs[kv.first].first;
            l.tabF = utabs[kv.first].second;
          }
          l.off = (int)items.size();
          for (int t = 0; t < T; ++t) {
            const TilePlan& tp = tiles[t];
            if (part_of[t] != p || !piped(tp) || tp.n != l.n || tp.d.precision != l.prec ||
                g >= tp.nlevels)
              continue;
            const int b = tp.prog_beg[g], e = tp.prog_beg[g + 1];
            for (int m = b; m < e; ++m) {
              const int j = tp.prog_led[m];
              Item it{};
              it.tile = t;
              it.led = j;
              it.wy0 = tp.N / 2 + tp.off[2 * j] - tp.n / 2;
              it.wx0 = tp.N / 2 + tp.off[2 * j + 1] - tp.n / 2;
              it.slot = m - b;
              it.gsize = e - b;
              it.iter = tp.prog_iter[m];
              items.push_back(it);
            }
          }
          l.count = (int)items.size() - l.off;
          if (l.count > 0) launches.push_back(l);
        }
        std::map<int, std::vector<int>> ends;  // iteration -> tiles ending it after level g
        for (int t = 0; t < T; ++t) {
          const TilePlan& tp = tiles[t];
          if (part_of[t] == p && piped(tp) && g < tp.nlevels && tp.prog_end[g] >= 0)
            ends[tp.prog_end[g]].push_back(t);
        }
        for (auto& kv : ends) {
          Launch e = id_range(kv.second);
          e.kind = Launch::ITER_END;
          e.iter = kv.first;
          launches.push_back(e);
          std::vector<int> next;
          for (int t : kv.second)
            if (tiles[t].d.iterations > kv.first + 1) next.push_back(t);
          if (!next.empty()) {
            Launch m = id_range(next);
            m.kind = Launch::SMAX;
            launches.push_back(m);
          }
        }
      }
    }
    parts.emplace_back(part_begin, (int)launches.size());
  }
  total_updates = 0;
  for (const TilePlan& tp : tiles) total_updates += (int64_t)tp.d.iterations * tp.L;
  // the chains' streams and fork / join events, before any graph capture
  if (parts.size() > 1 && !fork_ev &&
      !hip_ok(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming), "hipEventCreate", &st))
    return st;
  for (size_t p = 1; p < parts.size(); ++p) {
    if (!chain_stream[p] &&
        !hip_ok(hipStreamCreateWithFlags(&chain_stream[p], hipStreamNonBlocking), "hipStreamCreate",
                &st))
      return st;
    if (!join_ev[p] &&
        !hip_ok(hipEventCreateWithFlags(&join_ev[p], hipEventDisableTiming), "hipEventCreate", &st))
      return st;
  }

  if (!hip_ok(items_d.alloc(std::max<size_t>(1, items.size()) * sizeof(Item)), "hipMalloc(items)",
              &st))
    return st;
  if (!items.empty() &&
      !hip_ok(hipMemcpy(items_d.p, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice),
              "hipMemcpy(items)", &st))
    return st;
  if (!hip_ok(ranges_d.alloc(std::max<size_t>(1, ranges.size()) * sizeof(int2)),
              "hipMalloc(ranges)", &st))
    return st;
  if (!ranges.empty() &&
      !hip_ok(hipMemcpy(ranges_d.p, ranges.data(), ranges.size() * sizeof(int2),
                        hipMemcpyHostToDevice),
              "hipMemcpy(ranges)", &st))
    return st;
  if (!hip_ok(steps_d.alloc(std::max<size_t>(1, steptiles.size()) * sizeof(StepTile)),
              "hipMalloc(steps)", &st))
    return st;
  if (!steptiles.empty() &&
      !hip_ok(hipMemcpy(steps_d.p, steptiles.data(), steptiles.size() * sizeof(StepTile),
                        hipMemcpyHostToDevice),
              "hipMemcpy(steps)", &st))
    return st;
  if (!hip_ok(ids_d.alloc(std::max<size_t>(1, ids.size()) * sizeof(int)), "hipMalloc(ids)", &st))
    return st;
  if (!ids.empty() &&
      !hip_ok(hipMemcpy(ids_d.p, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice),
              "hipMemcpy(ids)", &st))
    return st;

  // ---- line-FFT jobs for the initial window (rows, then columns), per n
  std::vector<LineJob> jobs;
  init_line_launches.clear();
  for (auto& kv : nclass) {
    for (int pass = 0; pass < 2; ++pass) {
      LineLaunch ll{};
      ll.off = (int)jobs.size();
      ll.len = kv.first;
      ll.inverse = 0;
      for (int t = 0; t < T; ++t) {
        if (tiles[t].n != kv.first) continue;
        const TileDev& d = host_tiles[t];
        LineJob j{};
        j.base = d.S + (size_t)d.wy0_j0 * d.N + d.wx0_j0;
        j.line_stride = pass == 0 ? d.N : 1;
        j.elem_stride = pass == 0 ? 1 : d.N;
        j.nlines = d.n;
        j.scale = 1.0f;
        j.modulate = 0;
        jobs.push_back(j);
      }
      ll.count = (int)jobs.size() - ll.off;
      ll.max_lines = kv.first;
      init_line_launches.push_back(ll);
    }
  }

  // ---- concatenated-array offsets
  {
    std::vector<int64_t> io(T), oo(T), po(T), ro(T);
    total_I = total_obj = total_pupil = total_res = 0;
    n_max = 0;
    for (int t = 0; t < T; ++t) {
      const TilePlan& tp = tiles[t];
      io[t] = total_I;
      oo[t] = total_obj;
      po[t] = total_pupil;
      ro[t] = total_res;
      total_I += (int64_t)tp.L * tp.n * tp.n;
      total_obj += (int64_t)tp.N * tp.N;
      total_pupil += (int64_t)tp.n * tp.n;
      total_res += tp.d.iterations;
      n_max = std::max(n_max, tp.n);
    }
    for (auto* pr : {&i_off_d, &o_off_d, &p_off_d, &r_off_d})
      if (!hip_ok(pr->alloc(sizeof(int64_t) * T), "hipMalloc(offsets)", &st)) return st;
    if (!hip_ok(hipMemcpy(i_off_d.p, io.data(), 8 * T, hipMemcpyHostToDevice), "hipMemcpy", &st) ||
        !hip_ok(hipMemcpy(o_off_d.p, oo.data(), 8 * T, hipMemcpyHostToDevice), "hipMemcpy", &st) ||
        !hip_ok(hipMemcpy(p_off_d.p, po.data(), 8 * T, hipMemcpyHostToDevice), "hipMemcpy", &st) ||
        !hip_ok(hipMemcpy(r_off_d.p, ro.data(), 8 * T, hipMemcpyHostToDevice), "hipMemcpy", &st))
      return st;
    if (!hip_ok(obj_stage.alloc(sizeof(float2) * total_obj), "hipMalloc(object stage)", &st) ||
        !hip_ok(fwd_P.alloc(sizeof(float2) * total_pupil), "hipMalloc(pupil stage)", &st))
      return st;
    // finalise (inverse, on obj_stage) and forward (forward, on obj_stage) line jobs per N
    std::map<int, std::vector<int>> byN;
    for (int t = 0; t < T; ++t) byN[tiles[t].N].push_back(t);
    float2* ob = (float2*)obj_stage.p;
    for (int inv = 1; inv >= 0; --inv) {
      auto& dstl = inv ? fin_line_launches : fwd_line_launches;
      dstl.clear();
      for (auto& kv : byN) {
        for (int pass = 0; pass < 2; ++pass) {
          LineLaunch ll{};
          ll.off = (int)jobs.size();
          ll.len = kv.first;
          ll.inverse = inv;
          ll.max_lines = kv.first;
          for (int t : kv.second) {
            LineJob j{};
            j.base = ob + oo[t];
            j.line_stride = pass == 0 ? kv.first : 1;
            j.elem_stride = pass == 0 ? 1 : kv.first;
            j.nlines = kv.first;
            j.scale = 1.0f;
            j.modulate = (inv && pass == 1) ? 1 : 0;
            jobs.push_back(j);
          }
          ll.count = (int)jobs.size() - ll.off;
          dstl.push_back(ll);
        }
      }
    }
    // forward-model table: spectrum in obj_stage, pupil in fwd_P
    std::vector<TileDev> ft = host_tiles;
    for (int t = 0; t < T; ++t) {
      ft[t].S = ob + oo[t];
      ft[t].P = (float2*)fwd_P.p + po[t];
    }
    if (!hip_ok(fwd_table.alloc(sizeof(TileDev) * T), "hipMalloc(fwd table)", &st) ||
        !hip_ok(hipMemcpy(fwd_table.p, ft.data(), sizeof(TileDev) * T, hipMemcpyHostToDevice),
                "hipMemcpy(fwd table)", &st))
      return st;
    std::vector<Item> fi;
    fwd_launches.clear();
    for (auto& kv : nclass) {
      FwdLaunch fl{kv.first, kv.second, (int)fi.size(), 0};
      for (int t = 0; t < T; ++t) {
        const TilePlan& tp = tiles[t];
        if (tp.n != kv.first) continue;
        for (int j = 0; j < tp.L; ++j) {
          Item it{};
          it.tile = t;
          it.led = j;
          it.wy0 = tp.N / 2 + tp.off[2 * j] - tp.n / 2;
          it.wx0 = tp.N / 2 + tp.off[2 * j + 1] - tp.n / 2;
          fi.push_back(it);
        }
      }
      fl.count = (int)fi.size() - fl.off;
      fwd_launches.push_back(fl);
    }
    if (!hip_ok(fwd_items.alloc(sizeof(Item) * std::max<size_t>(1, fi.size())), "hipMalloc", &st) ||
        !hip_ok(hipMemcpy(fwd_items.p, fi.data(), sizeof(Item) * fi.size(), hipMemcpyHostToDevice),
                "hipMemcpy(fwd items)", &st))
      return st;
  }
  if (!hip_ok(hipMemcpy(table.p, host_tiles.data(), sizeof(TileDev) * T, hipMemcpyHostToDevice),
              "hipMemcpy(table)", &st))
    return st;
  if (!hip_ok(jobs_d.alloc(std::max<size_t>(1, jobs.size()) * sizeof(LineJob)), "hipMalloc(jobs)",
              &st))
    return st;
  if (!jobs.empty() &&
      !hip_ok(hipMemcpy(jobs_d.p, jobs.data(), jobs.size() * sizeof(LineJob), hipMemcpyHostToDevice),
              "hipMemcpy(jobs)", &st))
    return st;
  ntiles = T;
  ready = true;
  return FPM_OK;
}

hipError_t Executor::profile(hipStream_t s, fpm_kernel_time* out) {
  for (int k = 0; k < FPM_KERNEL_KINDS; ++k) out[k] = fpm_kernel_time{};
  const size_t nl = launches.size();
  std::vector<hipEvent_t> ev(2 * nl, nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if ((e = hipEventCreate(&x)) != hipSuccess) break;
  // launch i on its chain's stream, bracketed by events on that stream
  auto timed = [&](size_t i, hipStream_t st) {
    hipError_t r = hipEventRecord(ev[2 * i], st);
    if (r == hipSuccess) r = enqueue_range(i, i + 1, st);
    if (r == hipSuccess) r = hipEventRecord(ev[2 * i + 1], st);
    return r;
  };
  if (e == hipSuccess && nl > 0) e = timed(0, s);  // initial state
  if (e == hipSuccess && parts.size() > 1) e = hipEventRecord(fork_ev, s);
  for (size_t p = 1; p < parts.size() && e == hipSuccess; ++p) {
    e = hipStreamWaitEvent(chain_stream[p], fork_ev, 0);
    for (int i = parts[p].first; i < parts[p].second && e == hipSuccess; ++i)
      e = timed((size_t)i, chain_stream[p]);
    if (e == hipSuccess) e = hipEventRecord(join_ev[p], chain_stream[p]);
  }
  if (!parts.empty())
    for (int i = parts[0].first; i < parts[0].second && e == hipSuccess; ++i) e = timed((size_t)i, s);
  for (size_t p = 1; p < parts.size() && e == hipSuccess; ++p)
    e = hipStreamWaitEvent(s, join_ev[p], 0);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  // intervals relative to the first event; per kind: count, items, summed
  // durations and the union of the intervals
  std::vector<std::vector<std::pair<float, float>>> iv(FPM_KERNEL_KINDS);
  for (size_t i = 0; e == hipSuccess && i < nl; ++i) {
    float t0 = 0.0f, t1 = 0.0f;
    e = hipEventElapsedTime(&t0, ev[0], ev[2 * i]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t1, ev[0], ev[2 * i + 1]);
    if (e != hipSuccess) break;
    const Launch& l = launches[i];
    const int kind = l.kind == Launch::UPDATE     ? FPM_KERNEL_UPDATE
                     : l.kind == Launch::REDUCE   ? FPM_KERNEL_PUPIL_MEAN
                     : l.kind == Launch::ITER_END ? FPM_KERNEL_ITER_END
                     : l.kind == Launch::SMAX     ? FPM_KERNEL_SPEC_MAX
                                                  : FPM_KERNEL_INIT;
    fpm_kernel_time& k = out[kind];
    k.launches += 1;
    k.items += l.kind == Launch::UPDATE ? l.count : 0;
    k.total_ms += t1 - t0;
    iv[kind].emplace_back(t0, t1);
  }
  for (int k = 0; e == hipSuccess && k < FPM_KERNEL_KINDS; ++k) {
    std::sort(iv[k].begin(), iv[k].end());
    double busy = 0.0, lo = 0.0, hi = -1.0;
    for (const auto& x : iv[k]) {
      if (x.first > hi) {
        if (hi > lo) busy += hi - lo;
        lo = x.first;
        hi = x.second;
      } else if (x.second > hi) {
        hi = x.second;
      }
    }
    if (hi > lo) busy += hi - lo;
    out[k].busy_ms = busy;
  }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  return e;
}

hipError_t Executor::enqueue_sweep(hipStream_t s) {
  hipError_t e = enqueue_range(0, 1, s);  // initial state of every tile
  if (e != hipSuccess || parts.empty()) return e;
  if (parts.size() == 1) return enqueue_range(parts[0].first, parts[0].second, s);
  if ((e = hipEventRecord(fork_ev, s)) != hipSuccess) return e;
  for (size_t p = 1; p < parts.size(); ++p) {
    if ((e = hipStreamWaitEvent(chain_stream[p], fork_ev, 0)) != hipSuccess ||
        (e = enqueue_range(parts[p].first, parts[p].second, chain_stream[p])) != hipSuccess ||
        (e = hipEventRecord(join_ev[p], chain_stream[p])) != hipSuccess)
      return e;
  }
  if ((e = enqueue_range(parts[0].first, parts[0].second, s)) != hipSuccess) return e;
  for (size_t p = 1; p < parts.size(); ++p)
    if ((e = hipStreamWaitEvent(s, join_ev[p], 0)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t Executor::enqueue_range(size_t begin, size_t end, hipStream_t s) {
  const TileDev* tab = (const TileDev*)table.p;
  const Item* it = (const Item*)items_d.p;
  const StepTile* stp = (const StepTile*)steps_d.p;
  const int* ids = (const int*)ids_d.p;
  const LineJob* jobs = (const LineJob*)jobs_d.p;
  hipError_t e = hipSuccess;
  for (size_t li = begin; li < end && li < launches.size(); ++li) {
    const Launch& l = launches[li];
    switch (l.kind) {
      case Launch::INIT: {
        e = launch_init_state(tab, ids + l.off, l.count, 0, (int)std::sqrt((double)NN_max), s);
        for (const LineLaunch& ll : init_line_launches) {
          if (e != hipSuccess) break;
          e = launch_line_fft(jobs + ll.off, ll.count, ll.len, ll.max_lines, ll.inverse, s);
        }
        if (e == hipSuccess) e = launch_smax(tab, ids + l.off, l.count, (int)NN_max, s);
        break;
      }
      case Launch::UPDATE:
        e = launch_update_class(l, tab, it + l.off, s, (const int2*)ranges_d.p);
        break;
      case Launch::REDUCE:
        e = launch_pupil_reduce(tab, stp + l.off, l.count, l.nd_max > 0 ? l.nd_max : l.n, s);
        break;
      case Launch::ITER_END:
        e = launch_iter_end(tab, ids + l.off, l.count, l.iter, s);
        break;
      case Launch::SMAX:
        e = launch_smax(tab, ids + l.off, l.count, (int)NN_max, s);
        break;
    }
    if (e != hipSuccess) return e;
  }
  return e;
}

hipError_t Executor::tune(hipStream_t s) {
  const TileDev* tab = (const TileDev*)table.p;
  const Item* it = (const Item*)items_d.p;
  std::map<int, const Launch*> biggest;
  for (const Launch& l : launches)
    if (l.kind == Launch::UPDATE && l.prec == FPM_PREC_FP32_FFT && l.n != 256 &&
        (!biggest.count(l.n) || biggest[l.n]->count < l.count))
      biggest[l.n] = &l;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  tune_ms.clear();
  for (auto& kv : biggest) {
    if (e != hipSuccess) break;
    if (update_variant_known(kv.first)) continue;
    const Launch& l = *kv.second;
    int best = 0;
    float best_ms = 1e30f;
    // only the 8-lane family (variants 4-7): its variants differ in layout
    // alone and give the same bits, so a reconstruction's result does not
    // depend on which of them the timing picks (the 4-lane family rounds
    // differently and is selectable through FPM_UPDATE_VARIANT only)
    for (int v = kTuneFirst; v <= kTuneLast && e == hipSuccess; ++v) {
      const int2* rg = l.roff >= 0 ? (const int2*)ranges_d.p + l.roff : nullptr;
      e = launch_update(l.n, tab, it + l.off, l.count, l.nd_max, v, nullptr, s, rg,
                        l.rcount);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int r = 0; r < 3 && e == hipSuccess; ++r)
        e = launch_update(l.n, tab, it + l.off, l.count, l.nd_max, v, nullptr, s, rg, l.rcount);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      tune_ms.push_back(ms / 3.0f);
      if (e == hipSuccess && ms < best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    if (e == hipSuccess) set_update_variant(kv.first, best);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

hipError_t Executor::run(hipStream_t s, bool use_graph) {
  if (!tuned) {
    // the tuning launches only scribble on state that the sweep initialises
    const hipError_t te = tune(s);
    if (te != hipSuccess) return te;
    tuned = true;
  }
  if (!use_graph) return enqueue_sweep(s);
  if (!graph_exec) {
    hipError_t e;
    if (!cap_stream) {
      e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = enqueue_sweep(cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap_stream, &g);
    if (le != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return le;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      graph_exec = nullptr;
      return e;
    }
  }
  return hipGraphLaunch(graph_exec, s);
}

}  // namespace fpm

namespace fpm {

fpm_status Executor::online_setup(const std::vector<TilePlan>& tiles) {
  fpm_status st = FPM_OK;
  const int T = (int)tiles.size();
  const int L = tiles[0].L;
  // update classes in a fixed order, as in the sweep
  std::map<std::pair<int, int>, std::pair<int, int>> ucls;
  for (const TilePlan& tp : tiles) {
    auto& u = ucls[{tp.n, tp.d.precision}];
    u.first = std::max(u.first, tp.nd);
    u.second = std::max(u.second, mfma_box(tp.kx0, tp.nd));
  }
  online_classes = (int)ucls.size();
  std::vector<Item> items;
  online_launch.clear();
  for (int j = 0; j < L; ++j)
    for (auto& kv : ucls) {
      Launch l{};
      l.kind = Launch::UPDATE;
      l.n = kv.first.first;
      l.prec = kv.first.second;
      l.nd_max = kv.second.first;
      l.box_max = kv.second.second;
      if (l.n == 256) l.big_scratch = (float2*)big_scratch.p;
      if (l.prec != FPM_PREC_FP32_FFT &&
          !hip_ok(dft_tables(l.n, l.prec, &l.tabE, &l.tabF), "DFT tables", &st))
        return st;
      l.off = (int)items.size();
      for (int t = 0; t < T; ++t) {
        const TilePlan& tp = tiles[t];
        if (tp.n != l.n || tp.d.precision != l.prec) continue;
        Item it{};
        it.tile = t;
        it.led = j;
        it.wy0 = tp.N / 2 + tp.off[2 * j] - tp.n / 2;
        it.wx0 = tp.N / 2 + tp.off[2 * j + 1] - tp.n / 2;
        it.slot = 0;
        it.gsize = 1;
        it.iter = 0;
        items.push_back(it);
      }
      l.count = (int)items.size() - l.off;
      online_launch.push_back(l);
    }
  if (!hip_ok(online_items_d.alloc(sizeof(Item) * std::max<size_t>(1, items.size())),
              "hipMalloc(online items)", &st) ||
      !hip_ok(hipMemcpy(online_items_d.p, items.data(), sizeof(Item) * items.size(),
                        hipMemcpyHostToDevice),
              "hipMemcpy(online items)", &st))
    return st;
  // where each tile's image sits in one push: tiles in order, n^2 floats each
  std::vector<int64_t> src_off(T);
  online_push_floats = 0;
  for (int t = 0; t < T; ++t) {
    src_off[t] = online_push_floats;
    online_push_floats += (int64_t)tiles[t].n * tiles[t].n;
  }
  if (!hip_ok(online_src_off_d.alloc(sizeof(int64_t) * T), "hipMalloc(online offsets)", &st) ||
      !hip_ok(hipMemcpy(online_src_off_d.p, src_off.data(), sizeof(int64_t) * T,
                        hipMemcpyHostToDevice),
              "hipMemcpy(online offsets)", &st) ||
      !hip_ok(online_I.alloc(sizeof(float) * total_I), "hipMalloc(online stack)", &st) ||
      !hip_ok(online_stage.alloc(sizeof(float) * online_push_floats), "hipMalloc(online stage)",
              &st))
    return st;
  if (!online_pin &&
      !hip_ok(hipHostMalloc(&online_pin, sizeof(float) * online_push_floats, hipHostMallocDefault),
              "hipHostMalloc(online stage)", &st))
    return st;
  if (!online_ev && !hip_ok(hipEventCreateWithFlags(&online_ev, hipEventDisableTiming),
                            "hipEventCreate", &st))
    return st;
  return FPM_OK;
}

hipError_t Executor::enqueue_finalize(hipStream_t s) {
  const TileDev* tab = (const TileDev*)table.p;
  const LineJob* jobs = (const LineJob*)jobs_d.p;
  const int Nmax = (int)std::lround(std::sqrt((double)NN_max));
  hipError_t e = launch_scale_spectrum(tab, ntiles, (float2*)obj_stage.p, (const int64_t*)o_off_d.p,
                                       Nmax, s);
  for (const LineLaunch& ll : fin_line_launches) {
    if (e != hipSuccess) return e;
    e = launch_line_fft(jobs + ll.off, ll.count, ll.len, ll.max_lines, ll.inverse, s);
  }
  return e;
}

hipError_t Executor::enqueue_forward(const float2* obj_src, float* out, hipStream_t s) {
  const TileDev* ft = (const TileDev*)fwd_table.p;
  const LineJob* jobs = (const LineJob*)jobs_d.p;
  const int Nmax = (int)std::lround(std::sqrt((double)NN_max));
  hipError_t e = launch_object_to_spectrum(ft, ntiles, obj_src, (const int64_t*)o_off_d.p, Nmax, s);
  for (const LineLaunch& ll : fwd_line_launches) {
    if (e != hipSuccess) return e;
    e = launch_line_fft(jobs + ll.off, ll.count, ll.len, ll.max_lines, ll.inverse, s);
  }
  for (const FwdLaunch& fl : fwd_launches) {
    if (e != hipSuccess) return e;
    e = launch_forward_leds(fl.n, ft, (const Item*)fwd_items.p + fl.off, fl.count, out,
                            (const int64_t*)i_off_d.p, fl.nd_max, (float2*)big_scratch.p, s);
  }
  return e;
}

size_t Executor::device_bytes() const {
  const DevBuf* all[] = {&state, &table, &items_d, &ranges_d, &steps_d, &ids_d, &jobs_d, &i_off_d, &o_off_d,
                         &p_off_d, &r_off_d, &obj_stage, &fwd_P, &fwd_table, &fwd_items,
                         &I_stage, &res_stage, &pupil_stage, &big_scratch, &online_I,
                         &online_items_d, &online_src_off_d, &online_stage};
  size_t b = 0;
  for (const DevBuf* d : all) b += d->bytes;
  return b;
}

}  // namespace fpm

// Internal declarations shared by the host plan, the executor and the HIP
// kernels of libfpm.  Not part of the C ABI (include/fpm.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fpm.h"

namespace fpm {

// ----------------------------------------------------------------- plan
// Everything a tile needs that is fixed by its geometry (Sec. 2.2, Sec. 3.2).
struct TilePlan {
  fpm_tile_desc d{};
  int n = 0, N = 0, L = 0;
  int nd0 = 0;                       // |D0|
  int kx0 = 0, nd = 0;               // support columns [kx0, kx0 + nd)
  std::vector<uint8_t> mask;         // [n][n]
  std::vector<int32_t> chord;        // [n][2]: rows [lo, hi] of column kx (lo > hi: empty)
  std::vector<int32_t> off;          // [L][2] (drow, dcol)
  std::vector<int32_t> order;        // [L] ascending illumination NA
  std::vector<int32_t> group_of;     // [L]
  std::vector<int32_t> sweep;        // [L] groups concatenated
  std::vector<int32_t> gstart;       // [ngroups + 1]
  int ngroups = 0, max_group = 0;
  double min_tie = 0.0;
  std::vector<float> pupil0;         // [n][n][2] complex64 initial pupil
  // derived schedule: step s of an iteration updates LEDs steps[sbeg[s] .. sbeg[s+1])
  std::vector<int32_t> step_leds, step_beg;
  int nsteps = 0;
  // the whole sweep as dependent launches ("levels"): level g updates the
  // (iteration prog_iter[i], LED prog_led[i]) for i in [prog_beg[g],
  // prog_beg[g+1]); iteration prog_end[g] (or -1) ends after level g
  std::vector<int32_t> prog_led, prog_iter, prog_beg, prog_end;
  int nlevels = 0;
  int64_t i_off = 0, o_off = 0, p_off = 0, r_off = 0;  // offsets in concatenated arrays
};

fpm_status build_tile_plan(const fpm_tile_desc& d, TilePlan& tp, std::string& err);

// ------------------------------------------------------- device structures
// Per-tile device view used by every kernel.  Plain pointers, no torch.
struct TileDev {
  float2* S;          // [N][N]  stored spectrum (true spectrum = sigma * S)
  float2* P;          // [n][n]  pupil
  const float* I;     // [L][n][n] intensities
  float2* dP;         // [max_group][n][n] pupil increments of the current group
  double* e_part;     // residual numerator per (iteration, LED): [iter * e_stride + LED]
  double* i_part;     // sum of I per (iteration, LED), same indexing
  double* sigma;      // [1] lazy spectrum scale
  unsigned* smax;     // [1] bits of max |S|^2 (stored scale) at iteration start
  const int2* chord;  // [n] (lo, hi) per support column
  const float2* P0;   // [n][n] initial pupil
  double* residual;   // [iterations]
  int N, L, n, kx0, nd, nd0, j0, up;
  int wy0_j0, wx0_j0;  // window of the initial spectrum (the centred window)
  int mode;            // 0 spectrum only, 1 pupil in place, 2 pupil increments to dP
  int iters;           // iterations of this tile
  int e_stride;        // L (partials kept per iteration) or 0 (one iteration at a time)
};

struct Item {      // one (tile, LED) update
  int tile, led, wy0, wx0;
  int slot;        // member index within the tile's group of this step
  int gsize;       // members of that group
  int iter;        // iteration the update belongs to
};

struct StepTile {  // a tile that ran a group in this step
  int tile, count;
};

// Kernel launchers (kernels.hip).  All enqueue on `st` and return the HIP
// status of the launch.
// `variant` selects the lanes per line Q, the LDS row padding of the
// transpose buffer and the lines per workgroup: 0..3 Q = 4 with padding 16,
// 1, 8, 32 complex elements; 4, 5 Q = 8 with padding 1, 16; 6, 7 Q = 8,
// padding 1, every line of a phase in 2 or 4 rounds of a smaller workgroup
// (two workgroups per CU; their cross-lane steps are fused DPP multiply-adds);
// 8 Q = 4, padding 1, in 2 rounds.  Every variant computes the same FFTs; the
// Q = 4 and Q = 8 forms differ in the order of their floating-point steps,
// and the variants of one Q give the same bits.
constexpr int kUpdateVariants = 9;
// the variants the autotuner times: the 8-lane family, whose members give
// identical bits (the default, variant 7, is one of them)
constexpr int kTuneFirst = 4, kTuneLast = 7;
// n = 256 runs a persistent kernel whose workgroups keep their transposes in
// `big_scratch`: kBigSlots slots of n * n complex values (kBigSlots * 512 KiB);
// ignored for n <= 128.
constexpr int kBigSlots = 256;
constexpr size_t big_scratch_bytes(int n) { return (size_t)kBigSlots * n * n * 8; }
// ranges (n <= 128 only): group-sequential form, workgroup b runs the items
// ranges[b].x .. + ranges[b].y - 1 in order (one tile's LED group, slot
// order) and applies the group's pupil mean itself; no pupil_reduce launch.
hipError_t launch_update(int n, const TileDev* tiles, const Item* items, int count, int nd_max,
                         int variant, float2* big_scratch, hipStream_t st,
                         const int2* ranges = nullptr, int nranges = 0);
hipError_t launch_forward_leds(int n, const TileDev* tiles, const Item* items, int count,
                               float* out, const int64_t* out_off, int nd_max,
                               float2* big_scratch, hipStream_t st);
// rows: workgroups per tile, at least every listed tile's support-row count
// (the tile side n always is)
hipError_t launch_pupil_reduce(const TileDev* tiles, const StepTile* steps, int count, int rows,
                               hipStream_t st);
hipError_t launch_iter_end(const TileDev* tiles, const int* tile_ids, int count, int iter,
                           hipStream_t st);
hipError_t launch_smax(const TileDev* tiles, const int* tile_ids, int count, int NN_max,
                       hipStream_t st);
hipError_t launch_init_state(const TileDev* tiles, const int* tile_ids, int count, int n,
                             int N_max, hipStream_t st);
// batched line FFTs over per-tile base pointers (see kernels.hip)
struct LineJob {
  float2* base;       // first element of line 0
  int64_t line_stride, elem_stride;
  int nlines;
  float scale;        // applied to the output
  int modulate;       // multiply output element (line l, elem e) by (-1)^(l+e)
  int pad;
};
hipError_t launch_line_fft(const LineJob* jobs, int njobs, int len, int max_lines, int inverse,
                           hipStream_t st);
// dst[off[t] + i] = sigma * S * up^2 / N^2 for every tile (object finalise)
hipError_t launch_scale_spectrum(const TileDev* tiles, int count, float2* dst, const int64_t* off,
                                 int N_max, hipStream_t st);
// obj_stage[t] = (-1)^(x+y) * object[t] / up^2 (ahead of the forward line FFTs)
hipError_t launch_object_to_spectrum(const TileDev* tiles, int count, const float2* src_base,
                                     const int64_t* src_off, int N_max, hipStream_t st);
// table[t].I = base + i_off[t]   (kernel argument, so no host buffer outlives the call)
hipError_t launch_set_intensity(TileDev* table, int count, const float* base,
                                const int64_t* i_off, hipStream_t st);
// stack[i_off[t] + led n_t^2 ...] <- src[src_off[t] ...], n_t^2 floats per tile
hipError_t launch_online_scatter(const TileDev* table, int count, const float* src,
                                 const int64_t* src_off, float* stack, const int64_t* i_off,
                                 int led, hipStream_t st);
// table[t].j0 = j0 for every tile (the first LED of an online session)
hipError_t launch_set_j0(TileDev* table, int count, int j0, hipStream_t st);
// dst[off[t] + i] = tile t's pupil (which = 1), initial pupil (which = 2) or
// residual history (which = 3, doubles)
// Device-mode status word (bit 0: a negative or non-finite intensity, bit 1:
// a residual that is not finite): cleared by a kernel, set by the checks;
// copy_if_ok copies `bytes` only while the word is 0.
hipError_t launch_status_clear(int* status, hipStream_t st);
hipError_t launch_validate_intensity(const float* I, int64_t count, int* status, hipStream_t st);
hipError_t launch_check_residuals(const TileDev* tiles, int count, int* status, hipStream_t st);
hipError_t launch_copy_if_ok(void* dst, const void* src, int64_t bytes, const int* status,
                             hipStream_t st);
hipError_t launch_gather(const TileDev* tiles, int count, void* dst, const int64_t* off,
                         int which, int n_max, hipStream_t st);

}  // namespace fpm

namespace fpm {
// MFMA precision variant (mfma.hip).  Tables of the centred DFT matrices per
// (device, n, precision), built on first use and kept for the process.
hipError_t dft_tables(int n, int prec, const uint16_t** E, const uint16_t** F);
// side of the square support box the MFMA kernel covers for a support of
// rows/columns [kx0, kx0 + nd)
int mfma_box(int kx0, int nd);
hipError_t launch_update_mfma(int n, int prec, const TileDev* tiles, const Item* items, int count,
                              int box_max, const uint16_t* E, const uint16_t* F, hipStream_t st);
}  // namespace fpm

namespace fpm {
// Stitching (stitch.hip): scratch bytes for a rows x cols grid, and the
// launches (strip sums, factor chains, composition) on `st`.
size_t stitch_scratch_bytes(int rows, int cols);
hipError_t launch_stitch(const float2* tiles, int rows, int cols, int side, int overlap,
                         float2* out, void* scratch, hipStream_t st);
// The allocation-free stitch keeps its scratch in a fixed device array of
// kStitchNoAllocBytes per device (enough for kStitchNoAllocMaxTiles tiles:
// 88 bytes per tile plus 256); stitch_noalloc_scratch returns the current
// device's copy, looked up on the first call on that device.
constexpr int kStitchNoAllocMaxTiles = 4096;
constexpr size_t kStitchNoAllocBytes = (size_t)kStitchNoAllocMaxTiles * 88 + 256;
constexpr int kMaxDevices = 64;
hipError_t stitch_noalloc_scratch(void** ptr);
}  // namespace fpm

// Stitching of reconstructed tiles into one field of view (Sec. 3.1,
// Eq. (1)).
//
// Tiles sit on a rows x cols grid with stride s = side - overlap; every pixel
// of the result is taken from one tile, the owner, scaled by that tile's
// complex factor:
//   along x, tile c owns strip columns [c s + ov/2, (c+1) s + ov/2) (the first
//   from 0, the last to its end), i.e. f1 up to the middle of the overlap and
//   f2 after it; along y the same with rows;
//   merging a row left to right, tile c gets h_c = h_{c-1} mu1/mu2 with mu1
//   the mean of the strip's last `overlap` columns (tile c-1's, scaled by
//   h_{c-1}) and mu2 the mean of tile c's first `overlap` columns; merging the
//   strips top to bottom, strip r gets v_r = v_{r-1} mu1/mu2 over the bottom
//   rows of strip r-1 and the top rows of strip r.  Equal pixel counts make
//   the ratio of means a ratio of sums.
// Sums and factors are FP64; the result is complex64.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "fpm_internal.h"

namespace fpm {

namespace {

constexpr int kSumThreads = 256;

struct D2 {
  double x, y;
};

__device__ __forceinline__ void owned_range(int c, int C, int side, int ov, int& lo, int& hi) {
  lo = c > 0 ? ov / 2 : 0;
  hi = c < C - 1 ? side - ov + ov / 2 : side;
}

// block (tile, which): which 0 = first `ov` columns (all rows), 1 = last `ov`
// columns, 2 = first `ov` rows over the owned columns, 3 = last `ov` rows
// over the owned columns
__global__ __launch_bounds__(kSumThreads) void strip_sums_kernel(const float2* __restrict__ tiles,
                                                                 int R, int C, int side, int ov,
                                                                 D2* __restrict__ sums) {
  const int t = blockIdx.x, which = blockIdx.y;
  const int c = t % C;
  const float2* tile = tiles + (size_t)t * side * side;
  int x0 = 0, x1 = side, y0 = 0, y1 = side;
  if (which == 0) {
    x1 = ov;
  } else if (which == 1) {
    x0 = side - ov;
  } else {
    owned_range(c, C, side, ov, x0, x1);
    if (which == 2)
      y1 = ov;
    else
      y0 = side - ov;
  }
  const int w = x1 - x0, count = w * (y1 - y0);
  double sx = 0.0, sy = 0.0;
  for (int i = threadIdx.x; i < count; i += kSumThreads) {
    const int y = y0 + i / w, x = x0 + i % w;
    const float2 v = tile[(size_t)y * side + x];
    sx += v.x;
    sy += v.y;
  }
  __shared__ double rx[kSumThreads], ry[kSumThreads];
  rx[threadIdx.x] = sx;
  ry[threadIdx.x] = sy;
  __syncthreads();
  for (int o = kSumThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      rx[threadIdx.x] += rx[threadIdx.x + o];
      ry[threadIdx.x] += ry[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[(size_t)t * 4 + which] = D2{rx[0], ry[0]};
}

__device__ __forceinline__ D2 dmul(D2 a, D2 b) { return D2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ D2 ddiv(D2 a, D2 b) {
  const double d = b.x * b.x + b.y * b.y;
  if (!(d > 0.0)) return D2{1.0, 0.0};  // an all-zero overlap carries no phase: keep the scale
  return D2{(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

// one thread: the chains of ratios in merge order
__global__ void stitch_factors_kernel(const D2* __restrict__ sums, int R, int C, int ov,
                                      D2* __restrict__ hfac, float2* __restrict__ fac) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int r = 0; r < R; ++r) {
    D2 h{1.0, 0.0};
    hfac[(size_t)r * C] = h;
    for (int c = 1; c < C; ++c) {
      if (ov > 0) h = dmul(h, ddiv(sums[((size_t)r * C + c - 1) * 4 + 1], sums[((size_t)r * C + c) * 4 + 0]));
      hfac[(size_t)r * C + c] = h;
    }
  }
  D2 v{1.0, 0.0};
  for (int r = 0; r < R; ++r) {
    if (r > 0 && ov > 0) {
      D2 bottom{0.0, 0.0}, top{0.0, 0.0};
      for (int c = 0; c < C; ++c) {
        const D2 hb = dmul(hfac[(size_t)(r - 1) * C + c], sums[((size_t)(r - 1) * C + c) * 4 + 3]);
        const D2 ht = dmul(hfac[(size_t)r * C + c], sums[((size_t)r * C + c) * 4 + 2]);
        bottom.x += hb.x;
        bottom.y += hb.y;
        top.x += ht.x;
        top.y += ht.y;
      }
      v = dmul(v, ddiv(bottom, top));
    }
    for (int c = 0; c < C; ++c) {
      const D2 f = dmul(v, hfac[(size_t)r * C + c]);
      fac[(size_t)r * C + c] = make_float2((float)f.x, (float)f.y);
    }
  }
}

__device__ __forceinline__ int owner(int p, int stride, int ov, int count) {
  if (p < ov / 2) return 0;
  const int k = (p - ov / 2) / stride;
  return k < count - 1 ? k : count - 1;
}

// one thread per output pixel, rows of the output along blockIdx.y
__global__ __launch_bounds__(256) void stitch_compose_kernel(const float2* __restrict__ tiles,
                                                             const float2* __restrict__ fac,
                                                             int R, int C, int side, int ov,
                                                             int W, float2* __restrict__ out) {
  const int X = blockIdx.x * 256 + threadIdx.x, Y = blockIdx.y;
  if (X >= W) return;
  const int s = side - ov;
  const int r = owner(Y, s, ov, R), c = owner(X, s, ov, C);
  const float2 f = fac[(size_t)r * C + c];
  const float2 v = tiles[((size_t)r * C + c) * side * side + (size_t)(Y - r * s) * side + (X - c * s)];
  out[(size_t)Y * W + X] = make_float2(f.x * v.x - f.y * v.y, f.x * v.y + f.y * v.x);
}

// Scratch of the allocation-free stitch (fpm_stitch_noalloc): the strip
// sums, row factors and tile factors of at most kStitchNoAllocMaxTiles tiles,
// in one array per device that lives until the process ends.  Host code
// never uses this name as an address: stitch_noalloc_scratch() looks up each
// device's copy once and hands that pointer to the kernels.
static_assert(4 * sizeof(D2) + sizeof(D2) + sizeof(float2) == 88,
              "per-tile scratch bytes of the allocation-free stitch");
static __device__ __align__(256) unsigned char scratch[kStitchNoAllocBytes];

}  // namespace

size_t stitch_scratch_bytes(int rows, int cols) {
  return (size_t)rows * cols * (4 * sizeof(D2) + sizeof(D2) + sizeof(float2)) + 256;
}

hipError_t stitch_noalloc_scratch(void** ptr) {
  static std::mutex mu;
  static void* per_device[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!per_device[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    per_device[dev] = p;
  }
  *ptr = per_device[dev];
  return hipSuccess;
}

hipError_t launch_stitch(const float2* tiles, int rows, int cols, int side, int overlap,
                         float2* out, void* scratch, hipStream_t st) {
  const int T = rows * cols;
  D2* sums = (D2*)scratch;
  D2* hfac = sums + (size_t)T * 4;
  float2* fac = (float2*)(hfac + T);
  if (overlap > 0) {
    hipLaunchKernelGGL(strip_sums_kernel, dim3(T, 4), dim3(kSumThreads), 0, st, tiles, rows, cols,
                       side, overlap, sums);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(stitch_factors_kernel, dim3(1), dim3(1), 0, st, sums, rows, cols, overlap,
                     hfac, fac);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int W = cols * (side - overlap) + overlap, H = rows * (side - overlap) + overlap;
  hipLaunchKernelGGL(stitch_compose_kernel, dim3((W + 255) / 256, H), dim3(256), 0, st, tiles, fac,
                     rows, cols, side, overlap, W, out);
  return hipGetLastError();
}

}  // namespace fpm

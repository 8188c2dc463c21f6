// MFMA precision variant of the LED update (gfx950 matrix cores).
//
// The two n x n transforms of one (tile, LED) update are computed as dense
// products with centred DFT matrices instead of FFTs:
//   IFFT   psi  = E Phi E^T,      E[r][a] = exp(+2 pi i (a - n/2) r / n)
//   FFT    Phi' = F psi' F^T,     F[a][r] = exp(-2 pi i (a - n/2) r / n)
// where Phi = sigma P X lives on the support disc, so only the support rows /
// columns a in [ub, ub + box) of E and F take part.  The centring shifts of
// the method are part of E and F, so no (-1)^(x+y) bookkeeping is needed.
// Each complex product runs on v_mfma_f32_32x32x16 in one of two forms:
//   precision 1  split BF16: x = hi + lo (both bf16), products hi*hi + hi*lo
//                + lo*hi accumulated in FP32 (three MFMA terms);
//   precision 2  FP16 with power-of-two scaling of every operand stage into
//                the FP16 range (one MFMA term), FP32 accumulation.
// One workgroup of n/32 waves per (tile, LED); wave w owns LR columns
// [32w, 32w + 32) through the inverse transform, the modulus projection and
// the first forward stage, so those stages need no data from other waves:
//   stage 1  M1 = E_w Phi^T    (rows c of block w, all support a)
//   stage 2  psi = E M1^T      (all rows r, columns of block w)
//   modulus  psi' = sqrt(I) psi/|psi| in registers, residual partials
//   stage 3  V = F psi'        (support rows a, columns of block w); the
//            accumulator registers of psi' are the B operand as they stand,
//            with the K order of F permuted to match the accumulator layout
//   stage 4  Phi'^T = F V^T    (support x support output tiles over waves)
//   update   S and P on the support pixels, as in the FP32 kernel.
// Operand layouts of v_mfma_f32_32x32x16 (lane l, h = l / 32):
//   A[i][k]: lane i%32 + 32h holds k = 8h .. 8h+7;
//   B[k][j]: lane j%32 + 32h holds k = 8h .. 8h+7;
//   C[i][j]: lane j + 32h, register q holds i = 8(q/4) + 4h + q%4.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>

#include "fpm_internal.h"
#include "xcd_order.h"

namespace fpm {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// LDS written by a wave and read back by other lanes of the same wave
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// power of two s with s * amax <= 1 (1 for amax = 0 or not finite)
__device__ __forceinline__ float pow2_below(float amax) {
  if (!(amax > 0.0f) || !(amax < 3.0e38f)) return 1.0f;
  int ex;
  (void)frexpf(amax, &ex);  // amax = f 2^ex, f in [0.5, 1)
  return ldexpf(1.0f, -ex);
}

// ------------------------------------------------------------ operands
template <int PREC>
struct Op;
template <>
struct Op<1> {  // split bf16: hi, lo of re and im (+ negated im for the real part)
  bf8 rh, rl, ih, il, nih, nil;
};
template <>
struct Op<2> {  // fp16
  h8 r, i, ni;
};

__device__ __forceinline__ bf8 as_bf8(u4 v) { return __builtin_bit_cast(bf8, v); }
__device__ __forceinline__ h8 as_h8(u4 v) { return __builtin_bit_cast(h8, v); }
__device__ __forceinline__ u4 neg_bits(u4 v) { return v ^ 0x80008000u; }

// table operand: 8 consecutive K entries per plane at element offset `off`
template <int PREC>
__device__ __forceinline__ Op<PREC> load_tab(const uint16_t* __restrict__ tab, size_t plane,
                                              size_t off) {
  Op<PREC> o;
  const u4* p = reinterpret_cast<const u4*>(tab + off);
  const size_t ps = plane / 8;  // plane stride in u4
  if constexpr (PREC == 1) {
    o.rh = as_bf8(p[0]);
    o.rl = as_bf8(p[ps]);
    o.ih = as_bf8(p[2 * ps]);
    o.il = as_bf8(p[3 * ps]);
  } else {
    o.r = as_h8(p[0]);
    o.i = as_h8(p[ps]);
  }
  return o;
}

// data operand from 8 FP32 complex values, multiplied by the power of two s
template <int PREC>
__device__ __forceinline__ Op<PREC> make_data(const float (&re)[8], const float (&im)[8], float s) {
  Op<PREC> o;
  if constexpr (PREC == 1) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const __bf16 rh = (__bf16)re[e], ih = (__bf16)im[e];
      o.rh[e] = rh;
      o.ih[e] = ih;
      o.rl[e] = (__bf16)(re[e] - (float)rh);
      o.il[e] = (__bf16)(im[e] - (float)ih);
    }
    o.nih = as_bf8(neg_bits(__builtin_bit_cast(u4, o.ih)));
    o.nil = as_bf8(neg_bits(__builtin_bit_cast(u4, o.il)));
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      o.r[e] = (_Float16)(re[e] * s);
      o.i[e] = (_Float16)(im[e] * s);
    }
    o.ni = as_h8(neg_bits(__builtin_bit_cast(u4, o.i)));
  }
  return o;
}

// (cr + i ci) += A (table) * B (data), complex, 32x32 output tile, K = 16
template <int PREC>
__device__ __forceinline__ void cmac(f16v& cr, f16v& ci, const Op<PREC>& a, const Op<PREC>& b) {
  if constexpr (PREC == 1) {
    cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.rl, b.rh, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.rl, b.ih, ci, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.rh, b.rl, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.rh, b.il, ci, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.il, b.nih, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.il, b.rh, ci, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.ih, b.nil, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.ih, b.rl, ci, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.rh, b.rh, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.rh, b.ih, ci, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.ih, b.nih, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.ih, b.rh, ci, 0, 0, 0);
  } else {
    cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.r, b.r, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.r, b.i, ci, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.i, b.ni, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.i, b.r, ci, 0, 0, 0);
  }
}

__device__ __forceinline__ void ld8(const float* p0, const float* p1, float (&v)[8]) {
  const float4 a = *reinterpret_cast<const float4*>(p0);
  const float4 b = *reinterpret_cast<const float4*>(p1);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = a.z;
  v[3] = a.w;
  v[4] = b.x;
  v[5] = b.y;
  v[6] = b.z;
  v[7] = b.w;
}

// elements per thread per batch of the support-box loops
constexpr int kFill = 8;

// precision 2 transforms the modulus correction psi' - psi forward
template <int PREC>
constexpr bool kDelta = PREC == 2;

// K position p (0..15) of a 16-deep step whose B operand is taken straight
// from accumulator registers maps to accumulator row perm(p) of that step
__host__ __device__ constexpr int acc_perm(int p) { return 8 * ((p % 8) / 4) + 4 * (p / 8) + p % 4; }

template <int n>
struct Geo {
  static constexpr int W = n / 32;        // waves per workgroup
  static constexpr int NT = 64 * W;       // threads
  static constexpr int MT = n / 32;       // 32-row tiles of the LR field
  static constexpr int KS = n / 16;       // 16-deep K steps over the LR field
  static constexpr int EP = n + 16;       // E table pitch (support columns may run past n)
  static constexpr int FR = n + 32;       // F table rows (support tiles may run past n)
  static constexpr size_t EPL = (size_t)n * EP;  // elements per E plane
  static constexpr size_t FPL = (size_t)FR * n;  // elements per F plane
};

}  // namespace

// ========================================================= the MFMA kernel
// MS: compile-time bound on the 32-wide support tiles (box <= 32 MS)
template <int n, int MS, int PREC>
__global__ __launch_bounds__(2 * n) void mfma_update_kernel(const TileDev* __restrict__ tiles,
                                                            const Item* __restrict__ items,
                                                            const uint16_t* __restrict__ tabE,
                                                            const uint16_t* __restrict__ tabF,
                                                            int count) {
  using G = Geo<n>;
  constexpr int W = G::W, NT = G::NT, MT = G::MT, KS = G::KS;
  constexpr int T4W = (MS * MS + W - 1) / W;  // stage-4 output tiles per wave
  extern __shared__ float lds[];
  __shared__ float red_p[W], red_f[W], red_v[W];
  __shared__ double red_e[W], red_i[W];

  const int ii = xcd_item((int)blockIdx.x, count);
  if (ii < 0) return;  // the whole workgroup: past the last item
  const Item it = items[ii];
  const TileDev t = tiles[it.tile];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6, h = lane >> 5, c32 = lane & 31;
  const int N = t.N;
  const int ub = t.kx0 & ~7;                       // first support row/column, 8-aligned
  const int nk = (t.kx0 + t.nd - ub + 15) >> 4;    // 16-deep steps over the support
  const int box = nk << 4;
  const int mt = (box + 31) >> 5;                  // 32-wide tiles over the support
  const int p1 = box + 4;                          // Phi / M1 row pitch (floats)
  const int pv = n + 4;                            // V row pitch
  const int pp = box + 1;                          // Phi' row pitch
  const float sig = (float)*t.sigma;
  float2* __restrict__ Sw = t.S + (size_t)it.wy0 * N + it.wx0;
  float2* __restrict__ Pp = t.P;
  const int2* __restrict__ chord = t.chord;
  const float rbox = 1.0f / (float)box;

  // ---- Phi = sigma P X on the support box (zero off the disc), max |P|^2
  {
    float* PhR = lds;
    float* PhI = lds + box * p1;
    float pm = 0.0f, fm = 0.0f;
    // batches of kFill elements per thread: every load of a batch is issued
    // before the first is used (one wave per SIMD hides little latency)
    for (int e0 = 0; e0 < box * box; e0 += kFill * NT) {
      float2 xs[kFill], ps[kFill];
      int off[kFill];
#pragma unroll
      for (int j = 0; j < kFill; ++j) {
        const int e = e0 + j * NT + tid;
        const int ar = (int)(((float)e + 0.5f) * rbox);
        const int br = e - ar * box;
        const int a = ub + ar, b = ub + br;
        bool in = e < box * box && a < n && b < n;
        if (in) {
          const int2 ch = chord[b];
          in = a >= ch.x && a <= ch.y;
        }
        off[j] = in ? ar * p1 + br : -1 - (e < box * box ? ar * p1 + br : 0);
        xs[j] = in ? Sw[(size_t)a * N + b] : make_float2(0.0f, 0.0f);
        ps[j] = in ? Pp[a * n + b] : make_float2(0.0f, 0.0f);
      }
#pragma unroll
      for (int j = 0; j < kFill; ++j) {
        const int e = e0 + j * NT + tid;
        if (e >= box * box) continue;
        pm = fmaxf(pm, cabs2(ps[j]));
        const float2 v = cscale(cmul(ps[j], xs[j]), sig);
        fm = fmaxf(fm, cabs2(v));
        const int o = off[j] >= 0 ? off[j] : -1 - off[j];
        PhR[o] = v.x;
        PhI[o] = v.y;
      }
    }
    pm = wave_max(pm);
    fm = wave_max(fm);
    if (lane == 0) {
      red_p[w] = pm;
      red_f[w] = fm;
    }
  }
  lds_barrier();
  float pmax2 = red_p[0], fmax2 = red_f[0];
#pragma unroll
  for (int v = 1; v < W; ++v) {
    pmax2 = fmaxf(pmax2, red_p[v]);
    fmax2 = fmaxf(fmax2, red_f[v]);
  }
  const float s1 = PREC == 2 ? pow2_below(__builtin_sqrtf(fmax2)) : 1.0f;

  // ---- stage 1: M1[c][a] = sum_b E[c][b] Phi[a][b], c in block w
  f16v a1r[MS], a1i[MS];
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    a1r[j] = f16v{};
    a1i[j] = f16v{};
  }
  {
    const float* PhR = lds;
    const float* PhI = lds + box * p1;
#pragma unroll
    for (int k = 0; k < 2 * MS; ++k) {
      if (k >= nk) break;
      const Op<PREC> A =
          load_tab<PREC>(tabE, G::EPL, (size_t)(32 * w + c32) * G::EP + ub + 16 * k + 8 * h);
#pragma unroll
      for (int j = 0; j < MS; ++j) {
        if (j < mt) {
          const int ar = min(32 * j + c32, box - 1);
          const int o = ar * p1 + 16 * k + 8 * h;
          float re[8], im[8];
          ld8(PhR + o, PhR + o + 4, re);
          ld8(PhI + o, PhI + o + 4, im);
          cmac<PREC>(a1r[j], a1i[j], A, make_data<PREC>(re, im, s1));
        }
      }
    }
  }
  lds_barrier();  // Phi consumed; the space becomes the per-wave M1 regions

  // ---- M1 to this wave's LDS region as [c][a]
  float* M1R = lds + w * (2 * 32 * p1);
  float* M1I = M1R + 32 * p1;
  float gm = 0.0f;
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    const int ar = 32 * j + c32;
    if (j < mt && ar < box) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int cl = 8 * (q / 4) + 4 * h + (q % 4);
        M1R[cl * p1 + ar] = a1r[j][q];
        M1I[cl * p1 + ar] = a1i[j][q];
        gm = fmaxf(gm, a1r[j][q] * a1r[j][q] + a1i[j][q] * a1i[j][q]);
      }
    }
  }
  wave_lds_sync();
  const float s2 = PREC == 2 ? pow2_below(__builtin_sqrtf(wave_max(gm))) : 1.0f;

  // ---- stage 2: psi[r][c] = sum_a E[r][a] M1[c][a] (times n^2 s1 s2)
  f16v a2r[MT], a2i[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    a2r[i] = f16v{};
    a2i[i] = f16v{};
  }
#pragma unroll
  for (int k = 0; k < 2 * MS; ++k) {
    if (k >= nk) break;
    const int o = c32 * p1 + 16 * k + 8 * h;
    float re[8], im[8];
    ld8(M1R + o, M1R + o + 4, re);
    ld8(M1I + o, M1I + o + 4, im);
    const Op<PREC> B = make_data<PREC>(re, im, s2);
#pragma unroll
    for (int i = 0; i < MT; ++i) {
      const Op<PREC> A =
          load_tab<PREC>(tabE, G::EPL, (size_t)(32 * i + c32) * G::EP + ub + 16 * k + 8 * h);
      cmac<PREC>(a2r[i], a2i[i], A, B);
    }
  }

  // ---- modulus projection and residual partials, psi' kept in a2
  float e_acc = 0.0f, i_acc = 0.0f, mmax = 0.0f;
  {
    const float* __restrict__ Ip = t.I + (size_t)it.led * n * n;
    const float inv_scale = 1.0f / ((float)(n * n) * s1 * s2);
    const int c = 32 * w + c32;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int r = 32 * i + 8 * (q / 4) + 4 * h + (q % 4);
        const float I = Ip[r * n + c];
        const float m = __builtin_amdgcn_sqrtf(fmaxf(I, 0.0f));
        // |psi| through the hardware reciprocal square root, which flushes
        // denormal inputs: fields with |psi|^2 below 2^-100 are scaled by
        // 2^100 first (exact), so every nonzero psi keeps its phase
        const float2 v = make_float2(a2r[i][q], a2i[i][q]);
        const float p2 = cabs2(v);
        const bool small = p2 < 0x1p-100f;
        const float2 vs = small ? cscale(v, 0x1p100f) : v;
        const float p2s = small ? cabs2(vs) : p2;
        const bool live = p2s > 0.0f;
        const float rinv = live ? __builtin_amdgcn_rsqf(p2s) : 0.0f;
        const float amp = p2s * rinv * (small ? 0x1p-100f : 1.0f) * inv_scale;
        const float d = amp - m;
        e_acc = fmaf(d, d, e_acc);
        i_acc += I;
        if constexpr (!kDelta<PREC>) mmax = fmaxf(mmax, m);
        const float s = m * rinv;
        float pr = live ? vs.x * s : m, pi = live ? vs.y * s : 0.0f;
        if constexpr (kDelta<PREC>) {
          // transform the correction psi' - psi instead of psi': the forward
          // transform of psi is Phi exactly, so Phi' - Phi = FFT(psi' - psi),
          // and the rounding of the forward products scales with |psi' - psi|
          pr -= v.x * inv_scale;
          pi -= v.y * inv_scale;
          mmax = fmaxf(mmax, fmaxf(fabsf(pr), fabsf(pi)));
        }
        a2r[i][q] = pr;
        a2i[i][q] = pi;
      }
    }
  }
  const float s3 = PREC == 2 ? pow2_below(wave_max(mmax)) : 1.0f;

  // ---- stage 3: V[a][c] = sum_r F[a][r] psi'[r][c], B straight from a2
  f16v a3r[MS], a3i[MS];
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    a3r[j] = f16v{};
    a3i[j] = f16v{};
  }
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      re[e] = a2r[k / 2][8 * (k % 2) + e];
      im[e] = a2i[k / 2][8 * (k % 2) + e];
    }
    const Op<PREC> B = make_data<PREC>(re, im, s3);
#pragma unroll
    for (int j = 0; j < MS; ++j) {
      if (j < mt) {
        const Op<PREC> A =
            load_tab<PREC>(tabF, G::FPL, (size_t)(ub + 32 * j + c32) * n + 16 * k + 8 * h);
        cmac<PREC>(a3r[j], a3i[j], A, B);
      }
    }
  }
  lds_barrier();  // every wave is done with its M1 region

  // ---- V to LDS as [a][c] (unscaled)
  {
    float* VR = lds;
    float* VI = lds + box * pv;
    const float u3 = 1.0f / s3;
    const int c = 32 * w + c32;
    float vm = 0.0f;
#pragma unroll
    for (int j = 0; j < MS; ++j) {
      if (j < mt) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int ar = 32 * j + 8 * (q / 4) + 4 * h + (q % 4);
          if (ar < box) {
            const float vr = a3r[j][q] * u3, vi = a3i[j][q] * u3;
            VR[ar * pv + c] = vr;
            VI[ar * pv + c] = vi;
            vm = fmaxf(vm, vr * vr + vi * vi);
          }
        }
      }
    }
    vm = wave_max(vm);
    if (lane == 0) red_v[w] = vm;
  }
  lds_barrier();
  float vmax2 = red_v[0];
#pragma unroll
  for (int v = 1; v < W; ++v) vmax2 = fmaxf(vmax2, red_v[v]);
  const float s4 = PREC == 2 ? pow2_below(__builtin_sqrtf(vmax2)) : 1.0f;

  // ---- stage 4: Phi'^T[b][a] = sum_c F[b][c] V[a][c], tiles (jb, ja) over waves
  const int T4 = mt * mt;
  f16v a4r[T4W], a4i[T4W];
#pragma unroll
  for (int s = 0; s < T4W; ++s) {
    a4r[s] = f16v{};
    a4i[s] = f16v{};
  }
  {
    const float* VR = lds;
    const float* VI = lds + box * pv;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
#pragma unroll
      for (int s = 0; s < T4W; ++s) {
        const int tt = w + s * W;
        if (tt < T4) {
          const int jb = tt / mt, ja = tt - (tt / mt) * mt;
          const Op<PREC> A =
              load_tab<PREC>(tabF, G::FPL, (size_t)(ub + 32 * jb + c32) * n + 16 * k + 8 * h);
          const int ar = min(32 * ja + c32, box - 1);
          const int o = ar * pv + 16 * k + 4 * h;  // K order of acc_perm
          float re[8], im[8];
          ld8(VR + o, VR + o + 8, re);
          ld8(VI + o, VI + o + 8, im);
          cmac<PREC>(a4r[s], a4i[s], A, make_data<PREC>(re, im, s4));
        }
      }
    }
  }
  lds_barrier();  // V consumed

  // ---- Phi' to LDS as [b][a]
  {
    float* QR = lds;
    float* QI = lds + box * pp;
    const float u4s = 1.0f / s4;
#pragma unroll
    for (int s = 0; s < T4W; ++s) {
      const int tt = w + s * W;
      if (tt < T4) {
        const int jb = tt / mt, ja = tt - (tt / mt) * mt;
        const int ar = 32 * ja + c32;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int br = 32 * jb + 8 * (q / 4) + 4 * h + (q % 4);
          if (br < box && ar < box) {
            QR[br * pp + ar] = a4r[s][q] * u4s;
            QI[br * pp + ar] = a4i[s][q] * u4s;
          }
        }
      }
    }
  }
  {
    const double e = wave_sum((double)e_acc), s = wave_sum((double)i_acc);
    if (lane == 0) {
      red_e[w] = e;
      red_i[w] = s;
    }
  }
  lds_barrier();

  // ---- update S and P on the support pixels
  {
    const float* QR = lds;
    const float* QI = lds + box * pp;
    const int mode = t.mode;
    const float smax = __uint_as_float(*t.smax);  // max |S_stored|^2
    const float inv_ps = pmax2 > 0.0f ? 1.0f / (pmax2 * sig) : 0.0f;
    const float inv_ss = smax > 0.0f ? 1.0f / (smax * sig) : 0.0f;
    float2* __restrict__ Dp = t.dP + (size_t)it.slot * n * n;
    for (int e0 = 0; e0 < box * box; e0 += kFill * NT) {
      float2 xb[kFill], pb[kFill];
      int ab[kFill], bb[kFill];
#pragma unroll
      for (int j = 0; j < kFill; ++j) {
        const int e = e0 + j * NT + tid;
        const int ar = (int)(((float)e + 0.5f) * rbox);
        const int a = ub + ar, b = ub + (e - ar * box);
        bool in = e < box * box && a < n && b < n;
        if (in) {
          const int2 ch = chord[b];
          in = a >= ch.x && a <= ch.y;
        }
        ab[j] = in ? a : -1;
        bb[j] = b;
        xb[j] = in ? Sw[(size_t)a * N + b] : make_float2(0.0f, 0.0f);
        pb[j] = in ? Pp[a * n + b] : make_float2(0.0f, 0.0f);
      }
#pragma unroll
      for (int j = 0; j < kFill; ++j) {
      if (ab[j] < 0) continue;
      const int a = ab[j], b = bb[j], ar = a - ub, br = b - ub;
      const size_t so = (size_t)a * N + b;
      const int po = a * n + b;
      const float2 xs = xb[j];
      const float2 pv = pb[j];
      const float2 phi = cscale(cmul(pv, xs), sig);
      const float2 d = kDelta<PREC> ? make_float2(QR[br * pp + ar], QI[br * pp + ar])
                                    : make_float2(QR[br * pp + ar] - phi.x, QI[br * pp + ar] - phi.y);
      // S_stored += conj(P) D / (max|P|^2 sigma)
      if (pmax2 > 0.0f) {
        const float2 u = cscale(cmulc(d, pv), inv_ps);
        Sw[so] = make_float2(xs.x + u.x, xs.y + u.y);
      }
      if (mode != 0) {
        const float2 dp = cscale(cmulc(d, xs), inv_ss);
        if (mode == 1)
          Pp[po] = make_float2(pv.x + dp.x, pv.y + dp.y);
        else
          Dp[po] = dp;
      }
      }
    }
  }
  if (tid == 0) {
    double e = 0.0, s = 0.0;
    for (int v = 0; v < W; ++v) {
      e += red_e[v];
      s += red_i[v];
    }
    t.e_part[(size_t)it.iter * t.e_stride + it.led] = e;
    t.i_part[(size_t)it.iter * t.e_stride + it.led] = s;
  }
}

// ===================================================== DFT matrix tables
// E[r][a] (rows r < n, columns a < n + 16) and F[a][p] (rows a < n + 32,
// columns p < n holding r = 16 (p/16) + acc_perm(p%16)); zero where a >= n.
// Angles are exact integer fractions of a turn, evaluated in FP64 and
// rounded once to FP32 before the split (precision 1: hi = bf16(x),
// lo = bf16(x - hi); precision 2: fp16(x)).
__global__ void dft_table_kernel(uint16_t* __restrict__ E, uint16_t* __restrict__ F, int n,
                                 int prec) {
  const int EP = n + 16, FR = n + 32;
  const size_t epl = (size_t)n * EP, fpl = (size_t)FR * n;
  const size_t total = epl + fpl;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    int a, r;
    double sgn;
    uint16_t* dst;
    size_t pl;
    if (i < epl) {
      r = (int)(i / EP);
      a = (int)(i % EP);
      sgn = 1.0;
      dst = E + i;
      pl = epl;
    } else {
      const size_t j = i - epl;
      a = (int)(j / n);
      const int p = (int)(j % n);
      r = 16 * (p / 16) + acc_perm(p % 16);
      sgn = -1.0;
      dst = F + j;
      pl = fpl;
    }
    float re = 0.0f, im = 0.0f;
    if (a < n) {
      long k = ((long)(a - n / 2) * r) % n;
      if (k < 0) k += n;
      double sv, cv;
      sincospi(2.0 * (double)k / (double)n, &sv, &cv);
      re = (float)cv;
      im = (float)(sgn * sv);
    }
    if (prec == 1) {
      const __bf16 rh = (__bf16)re, ih = (__bf16)im;
      const __bf16 rl = (__bf16)(re - (float)rh), il = (__bf16)(im - (float)ih);
      dst[0] = __builtin_bit_cast(uint16_t, rh);
      dst[pl] = __builtin_bit_cast(uint16_t, rl);
      dst[2 * pl] = __builtin_bit_cast(uint16_t, ih);
      dst[3 * pl] = __builtin_bit_cast(uint16_t, il);
    } else {
      dst[0] = __builtin_bit_cast(uint16_t, (_Float16)re);
      dst[pl] = __builtin_bit_cast(uint16_t, (_Float16)im);
    }
  }
}

namespace {

template <int n>
size_t mfma_lds_bytes(int box) {
  const size_t phi = 2 * (size_t)box * (box + 4);
  const size_t m1 = (size_t)Geo<n>::W * 2 * 32 * (box + 4);
  const size_t v = 2 * (size_t)box * (n + 4);
  const size_t q = 2 * (size_t)box * (box + 1);
  return sizeof(float) * std::max(std::max(phi, m1), std::max(v, q));
}

template <int n, int MS, int PREC>
hipError_t launch_mfma_nsp(const TileDev* tiles, const Item* items, int count, int box_max,
                           const uint16_t* E, const uint16_t* F, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    attr = true;
    (void)hipFuncSetAttribute((const void*)mfma_update_kernel<n, MS, PREC>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
  }
  const size_t lds = mfma_lds_bytes<n>(box_max);
  hipLaunchKernelGGL((mfma_update_kernel<n, MS, PREC>), dim3(xcd_grid(count)), dim3(Geo<n>::NT),
                     lds, st, tiles, items, E, F, count);
  return hipGetLastError();
}

template <int n, int MS>
hipError_t launch_mfma_ns(int prec, const TileDev* tiles, const Item* items, int count,
                          int box_max, const uint16_t* E, const uint16_t* F, hipStream_t st) {
  switch (prec) {
    case 1: return launch_mfma_nsp<n, MS, 1>(tiles, items, count, box_max, E, F, st);
    case 2: return launch_mfma_nsp<n, MS, 2>(tiles, items, count, box_max, E, F, st);
    default: return hipErrorInvalidValue;
  }
}

template <int n>
hipError_t launch_mfma_n(int prec, const TileDev* tiles, const Item* items, int count, int box_max,
                         const uint16_t* E, const uint16_t* F, hipStream_t st) {
  if (box_max < 16 || box_max > n || box_max % 16) return hipErrorInvalidValue;
  switch ((box_max + 31) / 32) {
    case 1: return launch_mfma_ns<n, 1>(prec, tiles, items, count, box_max, E, F, st);
    case 2: return launch_mfma_ns<n, 2>(prec, tiles, items, count, box_max, E, F, st);
    case 3:
      if constexpr (n >= 96) return launch_mfma_ns<n, 3>(prec, tiles, items, count, box_max, E, F, st);
      return hipErrorInvalidValue;
    case 4:
      if constexpr (n >= 128) return launch_mfma_ns<n, 4>(prec, tiles, items, count, box_max, E, F, st);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

std::mutex g_tab_mu;
std::map<std::tuple<int, int, int>, void*> g_tabs;  // (device, n, prec) -> E planes, F planes

}  // namespace

int mfma_box(int kx0, int nd) {
  const int ub = kx0 & ~7;
  return ((kx0 + nd - ub + 15) >> 4) << 4;
}

hipError_t dft_tables(int n, int prec, const uint16_t** E, const uint16_t** F) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const int planes = prec == 1 ? 4 : 2;
  const size_t epl = (size_t)n * (n + 16), fpl = (size_t)(n + 32) * n;
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto key = std::make_tuple(dev, n, prec);
  auto it = g_tabs.find(key);
  void* p = nullptr;
  if (it != g_tabs.end()) {
    p = it->second;
  } else {
    e = hipMalloc(&p, sizeof(uint16_t) * planes * (epl + fpl));
    if (e != hipSuccess) return e;
    uint16_t* Ep = (uint16_t*)p;
    uint16_t* Fp = Ep + planes * epl;
    hipLaunchKernelGGL(dft_table_kernel, dim3(64), dim3(256), 0, nullptr, Ep, Fp, n, prec);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      (void)hipFree(p);
      return e;
    }
    g_tabs[key] = p;  // kept for the life of the process
  }
  *E = (const uint16_t*)p;
  *F = (const uint16_t*)p + planes * epl;
  return hipSuccess;
}

hipError_t launch_update_mfma(int n, int prec, const TileDev* tiles, const Item* items, int count,
                              int box_max, const uint16_t* E, const uint16_t* F, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  switch (n) {
    case 64: return launch_mfma_n<64>(prec, tiles, items, count, box_max, E, F, st);
    case 96: return launch_mfma_n<96>(prec, tiles, items, count, box_max, E, F, st);
    case 128: return launch_mfma_n<128>(prec, tiles, items, count, box_max, E, F, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fpm

// gfx950 kernels for the FPM alternating-projection sweep.
//
// Data path of one (tile, LED) update, one workgroup of 4n threads:
//   phase A   gather X = sigma * S on the support columns, Phi = P X / n^2,
//             IFFT along ky      (thread = (support column, quarter))
//   LDS       transpose T[kx][y]
//   phase B   IFFT along kx      (thread = (row y, quarter))
//   modulus   psi' = sqrt(I) psi/|psi|, residual partials   (I prefetched)
//   phase B'  FFT along x
//   LDS       transpose U[kx][y] on the support columns only
//   phase A'  FFT along y        (thread = (support column, quarter))
//   update    S and P on the support pixels only
// A length-n line FFT is split n = R * 4: each thread runs an R-point FFT
// in registers; the 4 threads of a line combine with a radix-4 step done
// as two radix-2 stages over DPP quad permutes (no LDS traffic).  The
// centring shifts of the method are folded away: the inverse transform of
// a centred spectrum equals the shifted one up to a (-1)^(x+y) factor,
// which the modulus projection and the forward transform cancel exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "fpm_internal.h"
#include "xcd_order.h"

namespace fpm {

namespace {

constexpr int kQ = 4;  // lanes per line of the default layout (Q = 8 also exists)

// ------------------------------------------------- compile-time twiddles
constexpr double kPiD = 3.14159265358979323846;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int i = 1; i < 14; ++i) {
    term *= -x2 / (double)((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) {
    term *= -x2 / (double)((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
// cos / sin of 2 pi k / m, reduced to the first octant by exact integer
// symmetry so the series stays on |x| <= pi/4.
constexpr double cos2pi(long k, long m) {
  k %= m;
  if (k < 0) k += m;
  // angle in units of 2pi/m; use 8k compared with m for octants
  if (2 * k > m) return cos2pi(m - k, m);          // cos(2pi - a) = cos a
  if (4 * k > m) return -cos2pi(m - 2 * k, 2 * m);  // a > pi/2: cos a = -cos(pi - a)
  if (8 * k > m) return taylor_sin(2.0 * kPiD * (double)(m - 4 * k) / (4.0 * (double)m));
  return taylor_cos(2.0 * kPiD * (double)k / (double)m);
}
constexpr double sin2pi(long k, long m) {
  k %= m;
  if (k < 0) k += m;
  if (2 * k > m) return -sin2pi(m - k, m);         // sin(2pi - a) = -sin a
  if (4 * k > m) return sin2pi(m - 2 * k, 2 * m);   // sin(pi - a) = sin a
  if (8 * k > m) return taylor_cos(2.0 * kPiD * (double)(m - 4 * k) / (4.0 * (double)m));
  return taylor_sin(2.0 * kPiD * (double)k / (double)m);
}

template <int M>
struct TwTab {
  float c[M], s[M];
  constexpr TwTab() : c(), s() {
    for (int k = 0; k < M; ++k) {
      c[k] = (float)cos2pi(k, M);
      s[k] = (float)sin2pi(k, M);
    }
  }
};
template <int M>
__device__ constexpr TwTab<M> kTw{};

// ------------------------------------------------------- complex helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// This file is compiled without floating-point contraction: every fused
// multiply-add is written out, so that two kernels running the same steps on
// a line (whatever their layout) round identically.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// products with the fused multiply-add placed explicitly (no contraction
// left to the compiler)
__device__ __forceinline__ float2 cmul_fma(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cmulc_fma(float2 a, float2 b) {  // a * conj(b)
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}
__device__ __forceinline__ float cabs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }

// multiply by W_len^k (INV: exp(+2 pi i k/len), else exp(-2 pi i k/len));
// k and len are compile-time after unrolling.
template <int R, bool INV>
__device__ __forceinline__ float2 tw_mul(float2 v, int k, int len) {
  if (k == 0) return v;
  if (4 * k == len) return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
  const int idx = k * (R / len);
  const float c = kTw<R>.c[idx];
  const float s = INV ? kTw<R>.s[idx] : -kTw<R>.s[idx];
  return make_float2(fmaf(v.x, c, -(v.y * s)), fmaf(v.x, s, v.y * c));
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
constexpr int bitrev(int v, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
  return r;
}

template <int R, bool INV, int ZLO = 0, int ZHI = 0>
__device__ __forceinline__ void fft_reg_pow2(float2 (&a)[R]);

// R-point FFT on registers, natural order in and out.  R = 2^k, or 3 * 2^k
// (one radix-3 decimation-in-time step over three power-of-two sub-FFTs:
// X[k + M s] = sum_r W_R^{r k} Y_r[k] W_3^{r s}, Y_r the M-point FFT of
// x[3 m + r]).
// ZLO / ZHI (power-of-two R only): inputs a[k] with k < ZLO or k >= R - ZHI
// are known to be zero, and the first butterfly stage skips the arithmetic
// on them (u + 0 and u - 0 are u, 0 + v and 0 - v are v and -v: the values
// are those of the full stage up to the sign of an exact zero).
template <int R, bool INV, int ZLO = 0, int ZHI = 0>
__device__ __forceinline__ void fft_reg(float2 (&a)[R]) {
  if constexpr (R % 3 == 0) {
    constexpr int M = R / 3;
    float2 y0[M], y1[M], y2[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      y0[m] = a[3 * m];
      y1[m] = a[3 * m + 1];
      y2[m] = a[3 * m + 2];
    }
    fft_reg_pow2<M, INV>(y0);
    fft_reg_pow2<M, INV>(y1);
    fft_reg_pow2<M, INV>(y2);
    // W_3 = exp(-+2 pi i / 3): -1/2 -+ i sqrt(3)/2
    const float s3 = INV ? 0.86602540378443864676f : -0.86602540378443864676f;
#pragma unroll
    for (int kk = 0; kk < M; ++kk) {
      const float2 t0 = y0[kk];
      const float2 t1 = tw_mul<R, INV>(y1[kk], kk, R);
      const float2 t2 = tw_mul<R, INV>(y2[kk], 2 * kk, R);
      const float2 sum = cadd(t1, t2), dif = csub(t1, t2);
      const float2 mid = make_float2(fmaf(-0.5f, sum.x, t0.x), fmaf(-0.5f, sum.y, t0.y));
      const float2 rot = make_float2(-s3 * dif.y, s3 * dif.x);  // i * s3 * dif
      a[kk] = cadd(t0, sum);
      a[kk + M] = cadd(mid, rot);
      a[kk + 2 * M] = csub(mid, rot);
    }
  } else {
    fft_reg_pow2<R, INV, ZLO, ZHI>(a);
  }
}

// R-point FFT on registers, natural order in and out (R a power of two).
template <int R, bool INV, int ZLO, int ZHI>
__device__ __forceinline__ void fft_reg_pow2(float2 (&a)[R]) {
  constexpr int LB = ilog2(R);
  float2 b[R];
#pragma unroll
  for (int i = 0; i < R; ++i) b[i] = a[bitrev(i, LB)];
  constexpr int kFirst = ZLO + ZHI > 0 ? 2 : 1;
  if constexpr (ZLO + ZHI > 0) {
    // first stage (twiddle 1) with the known-zero inputs folded away
#pragma unroll
    for (int i = 0; i < R; i += 2) {
      const int iu = bitrev(i, LB), iv = bitrev(i + 1, LB);
      const bool zu = iu < ZLO || iu >= R - ZHI, zv = iv < ZLO || iv >= R - ZHI;
      const float2 u = b[i], v = b[i + 1];
      if (zu && zv) {
        b[i] = make_float2(0.0f, 0.0f);
        b[i + 1] = b[i];
      } else if (zv) {
        b[i + 1] = u;
      } else if (zu) {
        b[i] = v;
        b[i + 1] = make_float2(-v.x, -v.y);
      } else {
        b[i] = cadd(u, v);
        b[i + 1] = csub(u, v);
      }
    }
  }
#pragma unroll
  for (int half = kFirst; half < R; half *= 2) {
#pragma unroll
    for (int i = 0; i < R; i += 2 * half) {
#pragma unroll
      for (int k = 0; k < half; ++k) {
        const float2 u = b[i + k];
        const float2 v = tw_mul<R, INV>(b[i + k + half], k, 2 * half);
        b[i + k] = cadd(u, v);
        b[i + k + half] = csub(u, v);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = b[i];
}

// --------------------------------------------------- cross-lane radix-4
// DPP quad permutes: xor 1 = [1,0,3,2], xor 2 = [2,3,0,1].
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  // every lane of a quad reads a valid partner, so no "old" value is needed
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
constexpr int kXor1 = 0xB1;
constexpr int kXor2 = 0x4E;

// radix-2 stage with the partner lane (lane ^ M): lower lane a+b, upper a-b
template <int CTRL>
__device__ __forceinline__ float2 xstage(float2 v, float sgn) {
  const float px = dpp<CTRL>(v.x), py = dpp<CTRL>(v.y);
  return make_float2(fmaf(sgn, v.x, px), fmaf(sgn, v.y, py));
}
// lane 3 multiplies by W_4 (INV: +i, else -i)
template <bool INV>
__device__ __forceinline__ float2 w4_lane3(float2 v, bool is3) {
  const float2 r = INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
  return is3 ? r : v;
}

// 4-point DFT across the 4 lanes of a line.  Input natural (lane q holds
// x_q); output bit-reversed (lane q holds X_{brev2(q)}).
template <bool INV, int R>
__device__ __forceinline__ void xlane_nat2brev(float2 (&a)[R], int q) {
  const float s2 = (q & 2) ? -1.0f : 1.0f, s1 = (q & 1) ? -1.0f : 1.0f;
  const bool is3 = (q == 3);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    float2 v = xstage<kXor2>(a[i], s2);
    v = w4_lane3<INV>(v, is3);
    a[i] = xstage<kXor1>(v, s1);
  }
}
// Input bit-reversed (lane q holds x_{brev2(q)}); output natural.
template <bool INV, int R>
__device__ __forceinline__ void xlane_brev2nat(float2 (&a)[R], int q) {
  const float s2 = (q & 2) ? -1.0f : 1.0f, s1 = (q & 1) ? -1.0f : 1.0f;
  const bool is3 = (q == 3);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    float2 v = xstage<kXor1>(a[i], s1);
    v = w4_lane3<INV>(v, is3);
    a[i] = xstage<kXor2>(v, s2);
  }
}

__device__ __forceinline__ int brev2(int q) { return ((q & 1) << 1) | ((q >> 1) & 1); }

// twiddle W_n^e from the LDS table tw[e] = exp(+2 pi i e / n)
template <bool INV>
__device__ __forceinline__ float2 lds_tw(const float2* tw, int e) {
  const float2 w = tw[e];
  return INV ? w : make_float2(w.x, -w.y);
}

// Twiddle table views.  TS = 0: tw[e] = W^e for e in [0, n).  TS > 0:
// tw[e TS] = W^e for e in [0, n/2) only (a strided column, e.g. the padding
// column of a transpose buffer), and W^(e + n/2) = -W^e.  The table is
// correctly rounded and W^(n/2) = -1, so both views give the same bits.
template <bool INV, int n, int TS>
__device__ __forceinline__ float2 tw_at(const float2* tw, int e) {
  if constexpr (TS == 0) {
    return lds_tw<INV>(tw, e);
  } else {
    const bool hi = e >= n / 2;
    const float2 w = tw[(hi ? e - n / 2 : e) * TS];
    const float c = hi ? -w.x : w.x, sn = hi ? -w.y : w.y;
    return make_float2(c, INV ? sn : -sn);
  }
}

// --------------------------------------------- cross-lane radix-8 (Q = 8)
// The 8 lanes of a line are relabelled ql = q (q < 4), 11 - q (q >= 4), so
// that the partner at logical distance 4 is the DPP row_half_mirror partner
// (lane i <-> 7 - i), while logical distances 2 and 1 stay the quad
// permutes xor 2 and xor 1.
constexpr int kMirror8 = 0x141;
// Q = 16: physical lane p of a row of 16 is relabelled ql = p ^ g(p3, p2)
// with g = 0, 3, 4, 7 for (p3, p2) = 00, 01, 10, 11; then the DPP
// row_mirror partner (15 - p) is at logical distance 8, the row_half_mirror
// partner (p ^ 7) at distance 4, and the quad permutes xor 2 / xor 1 at
// distances 2 / 1.  For p < 8 this is the Q = 8 relabelling.
constexpr int kMirror16 = 0x140;
template <int Q>
__device__ __forceinline__ int lane_log(int q) {
  if constexpr (Q == 4) return q;
  if constexpr (Q == 8) return q < 4 ? q : 11 - q;
  return q ^ ((q & 8) ? ((q & 4) ? 7 : 4) : ((q & 4) ? 3 : 0));
}
template <int Q>
__device__ __forceinline__ int brevq(int ql) {
  if constexpr (Q == 4) return ((ql & 1) << 1) | ((ql >> 1) & 1);
  if constexpr (Q == 8) return ((ql & 1) << 2) | (ql & 2) | ((ql >> 2) & 1);
  return ((ql & 1) << 3) | ((ql & 2) << 1) | ((ql >> 1) & 2) | ((ql >> 3) & 1);
}
// W_8^j, j = 0..3 (INV: exp(+2 pi i j / 8), else exp(-2 pi i j / 8))
template <bool INV>
__device__ __forceinline__ float2 w8(int j) {
  constexpr float h = 0.707106781186547524401f;
  const float c = j == 0 ? 1.0f : (j == 1 ? h : (j == 2 ? 0.0f : -h));
  const float sn = j == 0 ? 0.0f : (j == 1 ? h : (j == 2 ? 1.0f : h));
  return make_float2(c, INV ? sn : -sn);
}
// 8-point DFT across the lanes of a line, decimation in frequency: input
// natural (logical lane ql holds x_ql), output bit-reversed (X_{brev3(ql)}).
template <bool INV, int R>
__device__ __forceinline__ void xlane8_nat2brev(float2 (&a)[R], int ql) {
  const float s4 = (ql & 4) ? -1.0f : 1.0f, s2 = (ql & 2) ? -1.0f : 1.0f,
              s1 = (ql & 1) ? -1.0f : 1.0f;
  const float2 t8 = w8<INV>((ql & 4) ? (ql & 3) : 0);
  const bool is3 = (ql & 3) == 3;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    float2 v = cmul(xstage<kMirror8>(a[i], s4), t8);
    v = w4_lane3<INV>(xstage<kXor2>(v, s2), is3);
    a[i] = xstage<kXor1>(v, s1);
  }
}
// decimation in time: input bit-reversed, output natural
template <bool INV, int R>
__device__ __forceinline__ void xlane8_brev2nat(float2 (&a)[R], int ql) {
  const float s4 = (ql & 4) ? -1.0f : 1.0f, s2 = (ql & 2) ? -1.0f : 1.0f,
              s1 = (ql & 1) ? -1.0f : 1.0f;
  const float2 t8 = w8<INV>((ql & 4) ? (ql & 3) : 0);
  const bool is3 = (ql & 3) == 3;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    float2 v = w4_lane3<INV>(xstage<kXor1>(a[i], s1), is3);
    v = cmul(xstage<kXor2>(v, s2), t8);
    a[i] = xstage<kMirror8>(v, s4);
  }
}

// 16-point DFT across the lanes of a line, decimation in frequency: input
// natural, output bit-reversed (X_{brev4(ql)}).  The W16 twiddle of the upper
// half comes from the line's LDS table: W16^j = W_n^(j n / 16).
template <int n, bool INV, int R, int TS>
__device__ __forceinline__ void xlane16_nat2brev(float2 (&a)[R], int ql, const float2* tw) {
  const float s8 = (ql & 8) ? -1.0f : 1.0f, s4 = (ql & 4) ? -1.0f : 1.0f,
              s2 = (ql & 2) ? -1.0f : 1.0f, s1 = (ql & 1) ? -1.0f : 1.0f;
  const float2 t16 = tw_at<INV, n, TS>(tw, (ql & 8) ? (ql & 7) * (n / 16) : 0);
  const float2 t8 = w8<INV>((ql & 4) ? (ql & 3) : 0);
  const bool is3 = (ql & 3) == 3;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    float2 v = cmul(xstage<kMirror16>(a[i], s8), t16);
    v = cmul(xstage<kMirror8>(v, s4), t8);
    v = w4_lane3<INV>(xstage<kXor2>(v, s2), is3);
    a[i] = xstage<kXor1>(v, s1);
  }
}
// decimation in time: input bit-reversed, output natural
template <int n, bool INV, int R, int TS>
__device__ __forceinline__ void xlane16_brev2nat(float2 (&a)[R], int ql, const float2* tw) {
  const float s8 = (ql & 8) ? -1.0f : 1.0f, s4 = (ql & 4) ? -1.0f : 1.0f,
              s2 = (ql & 2) ? -1.0f : 1.0f, s1 = (ql & 1) ? -1.0f : 1.0f;
  const float2 t16 = tw_at<INV, n, TS>(tw, (ql & 8) ? (ql & 7) * (n / 16) : 0);
  const float2 t8 = w8<INV>((ql & 4) ? (ql & 3) : 0);
  const bool is3 = (ql & 3) == 3;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    float2 v = w4_lane3<INV>(xstage<kXor1>(a[i], s1), is3);
    v = cmul(xstage<kXor2>(v, s2), t8);
    v = cmul(xstage<kMirror8>(v, s4), t16);
    a[i] = xstage<kMirror16>(v, s8);
  }
}

// ------------------------------------ fused cross-lane stages (Q = 8)
// A cross-lane radix-2 stage as xstage writes it costs two VALU operations
// per component (a DPP move, then a fused multiply-add).  v_fmac_f32 with a
// DPP source does both: v <- v + m * partner(v).  It cannot give the lower
// lane a + b and the upper lane a - b with one multiplier pattern (the op is
// the same in every lane), but it gives the upper lane b - a = -(a - b): the
// lane's value comes out negated.  Each lane's values therefore carry a
// known sign sigma (+-1, the same for all of the lane's values), and a stage
// with signs sigma_own, sigma_partner and the butterfly sign sgn of
// xstage uses m = sigma_own * sigma_partner * sgn and yields sigma_own * sgn.
// Negation commutes with rounding to nearest, so every value is bitwise the
// xstage value up to its sign.  For the radix-8 steps of line_dit / line_dif:
// input signs +1 give m = sgn at every stage and output signs
// par(ql) = (-1)^popcount(ql); input signs par(ql) give m = -sgn and output
// signs +1.  The callers fold par(ql) into a scalar they multiply by anyway.
#define FPM_DPP_XOR1 "quad_perm:[1,0,3,2]"
#define FPM_DPP_XOR2 "quad_perm:[2,3,0,1]"
#define FPM_DPP_MIRROR8 "row_half_mirror"
#define FPM_DPP_MIRROR16 "row_mirror"
// operand i += m * partner(operand i); M is the operand number of m
#define FPM_FMACD(i, M, C) \
  "v_fmac_f32_dpp %" #i ", %" #i ", %" #M " " C " row_mask:0xf bank_mask:0xf\n\t"
// 8 complex values (16 VGPRs) per block.  A DPP source read needs two wait
// states after a VALU write of that register; the s_nop covers any write the
// compiler places just before the block, and inside it each instruction
// reads a register that no earlier instruction of the block wrote.
#define FPM_FMACD_BLOCK8(C)                                                                   \
  "s_nop 1\n\t" FPM_FMACD(0, 16, C) FPM_FMACD(1, 16, C) FPM_FMACD(2, 16, C)                     \
      FPM_FMACD(3, 16, C) FPM_FMACD(4, 16, C) FPM_FMACD(5, 16, C) FPM_FMACD(6, 16, C)           \
          FPM_FMACD(7, 16, C) FPM_FMACD(8, 16, C) FPM_FMACD(9, 16, C) FPM_FMACD(10, 16, C)      \
              FPM_FMACD(11, 16, C) FPM_FMACD(12, 16, C) FPM_FMACD(13, 16, C)                    \
                  FPM_FMACD(14, 16, C) FPM_FMACD(15, 16, C)
#define FPM_FMACD_BLOCK4(C)                                                                   \
  "s_nop 1\n\t" FPM_FMACD(0, 8, C) FPM_FMACD(1, 8, C) FPM_FMACD(2, 8, C) FPM_FMACD(3, 8, C)    \
      FPM_FMACD(4, 8, C) FPM_FMACD(5, 8, C) FPM_FMACD(6, 8, C) FPM_FMACD(7, 8, C)

template <int CTRL>
__device__ __forceinline__ void fmacd8(float2* a, float m) {
  if constexpr (CTRL == kXor1)
    asm volatile(FPM_FMACD_BLOCK8(FPM_DPP_XOR1)
                 : "+v"(a[0].x), "+v"(a[0].y), "+v"(a[1].x), "+v"(a[1].y), "+v"(a[2].x),
                   "+v"(a[2].y), "+v"(a[3].x), "+v"(a[3].y), "+v"(a[4].x), "+v"(a[4].y),
                   "+v"(a[5].x), "+v"(a[5].y), "+v"(a[6].x), "+v"(a[6].y), "+v"(a[7].x),
                   "+v"(a[7].y)
                 : "v"(m));
  else if constexpr (CTRL == kXor2)
    asm volatile(FPM_FMACD_BLOCK8(FPM_DPP_XOR2)
                 : "+v"(a[0].x), "+v"(a[0].y), "+v"(a[1].x), "+v"(a[1].y), "+v"(a[2].x),
                   "+v"(a[2].y), "+v"(a[3].x), "+v"(a[3].y), "+v"(a[4].x), "+v"(a[4].y),
                   "+v"(a[5].x), "+v"(a[5].y), "+v"(a[6].x), "+v"(a[6].y), "+v"(a[7].x),
                   "+v"(a[7].y)
                 : "v"(m));
  else if constexpr (CTRL == kMirror8)
    asm volatile(FPM_FMACD_BLOCK8(FPM_DPP_MIRROR8)
                 : "+v"(a[0].x), "+v"(a[0].y), "+v"(a[1].x), "+v"(a[1].y), "+v"(a[2].x),
                   "+v"(a[2].y), "+v"(a[3].x), "+v"(a[3].y), "+v"(a[4].x), "+v"(a[4].y),
                   "+v"(a[5].x), "+v"(a[5].y), "+v"(a[6].x), "+v"(a[6].y), "+v"(a[7].x),
                   "+v"(a[7].y)
                 : "v"(m));
  else
    asm volatile(FPM_FMACD_BLOCK8(FPM_DPP_MIRROR16)
                 : "+v"(a[0].x), "+v"(a[0].y), "+v"(a[1].x), "+v"(a[1].y), "+v"(a[2].x),
                   "+v"(a[2].y), "+v"(a[3].x), "+v"(a[3].y), "+v"(a[4].x), "+v"(a[4].y),
                   "+v"(a[5].x), "+v"(a[5].y), "+v"(a[6].x), "+v"(a[6].y), "+v"(a[7].x),
                   "+v"(a[7].y)
                 : "v"(m));
}
template <int CTRL>
__device__ __forceinline__ void fmacd4(float2* a, float m) {
  if constexpr (CTRL == kXor1)
    asm volatile(FPM_FMACD_BLOCK4(FPM_DPP_XOR1)
                 : "+v"(a[0].x), "+v"(a[0].y), "+v"(a[1].x), "+v"(a[1].y), "+v"(a[2].x),
                   "+v"(a[2].y), "+v"(a[3].x), "+v"(a[3].y)
                 : "v"(m));
  else if constexpr (CTRL == kXor2)
    asm volatile(FPM_FMACD_BLOCK4(FPM_DPP_XOR2)
                 : "+v"(a[0].x), "+v"(a[0].y), "+v"(a[1].x), "+v"(a[1].y), "+v"(a[2].x),
                   "+v"(a[2].y), "+v"(a[3].x), "+v"(a[3].y)
                 : "v"(m));
  else if constexpr (CTRL == kMirror8)
    asm volatile(FPM_FMACD_BLOCK4(FPM_DPP_MIRROR8)
                 : "+v"(a[0].x), "+v"(a[0].y), "+v"(a[1].x), "+v"(a[1].y), "+v"(a[2].x),
                   "+v"(a[2].y), "+v"(a[3].x), "+v"(a[3].y)
                 : "v"(m));
  else
    asm volatile(FPM_FMACD_BLOCK4(FPM_DPP_MIRROR16)
                 : "+v"(a[0].x), "+v"(a[0].y), "+v"(a[1].x), "+v"(a[1].y), "+v"(a[2].x),
                   "+v"(a[2].y), "+v"(a[3].x), "+v"(a[3].y)
                 : "v"(m));
}
#undef FPM_FMACD_BLOCK4
#undef FPM_FMACD_BLOCK8
#undef FPM_FMACD
#undef FPM_DPP_MIRROR16
#undef FPM_DPP_MIRROR8
#undef FPM_DPP_XOR2
#undef FPM_DPP_XOR1

// a[i] <- a[i] + m * partner(a[i]) for all i, both components
template <int CTRL, int R>
__device__ __forceinline__ void xstage_fused(float2 (&a)[R], float m) {
  static_assert(R % 4 == 0, "blocks of 4 complex values");
#pragma unroll
  for (int i = 0; i + 8 <= R; i += 8) fmacd8<CTRL>(a + i, m);
  if constexpr (R % 8 != 0) fmacd4<CTRL>(a + (R / 8) * 8, m);
}

__device__ __forceinline__ float par8(int ql) {  // (-1)^popcount(ql), ql < 8
  return (__builtin_popcount(ql) & 1) ? -1.0f : 1.0f;
}

// xlane8_nat2brev / xlane8_brev2nat with fused stages, stage by stage over
// the lane's values.  flip = +1: input signs +1, output signs par8(ql);
// flip = -1: input signs par8(ql), output signs +1.
template <bool INV, int R>
__device__ __forceinline__ void xlane8_nat2brev_f(float2 (&a)[R], int ql, float flip) {
  const float s4 = (ql & 4) ? -flip : flip, s2 = (ql & 2) ? -flip : flip,
              s1 = (ql & 1) ? -flip : flip;
  const float2 t8 = w8<INV>((ql & 4) ? (ql & 3) : 0);
  const bool is3 = (ql & 3) == 3;
  xstage_fused<kMirror8>(a, s4);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = cmul(a[i], t8);
  xstage_fused<kXor2>(a, s2);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = w4_lane3<INV>(a[i], is3);
  xstage_fused<kXor1>(a, s1);
}
template <bool INV, int R>
__device__ __forceinline__ void xlane8_brev2nat_f(float2 (&a)[R], int ql, float flip) {
  const float s4 = (ql & 4) ? -flip : flip, s2 = (ql & 2) ? -flip : flip,
              s1 = (ql & 1) ? -flip : flip;
  const float2 t8 = w8<INV>((ql & 4) ? (ql & 3) : 0);
  const bool is3 = (ql & 3) == 3;
  xstage_fused<kXor1>(a, s1);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = w4_lane3<INV>(a[i], is3);
  xstage_fused<kXor2>(a, s2);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = cmul(a[i], t8);
  xstage_fused<kMirror8>(a, s4);
}

// Line FFT over Q lanes, decimation in time.  In: logical lane ql holds
// x[ql + Q p] in a[p].  Out: it holds X[R * brevq(ql) + k] in a[k].
template <int n, bool INV, int Q = kQ, int TS = 0>
__device__ __forceinline__ void line_dit(float2 (&a)[n / Q], int ql, const float2* tw) {
  constexpr int R = n / Q;
  fft_reg<R, INV>(a);
#pragma unroll
  for (int k = 1; k < R; ++k) a[k] = cmul(a[k], tw_at<INV, n, TS>(tw, ql * k));
  if constexpr (Q == 4)
    xlane_nat2brev<INV>(a, ql);
  else if constexpr (Q == 8)
    xlane8_nat2brev<INV>(a, ql);
  else
    xlane16_nat2brev<n, INV, R, TS>(a, ql, tw);
}
// Line FFT over Q lanes, decimation in frequency.  In: logical lane ql holds
// x[R * brevq(ql) + m] in a[m].  Out: it holds X[ql + Q k] in a[k].
template <int n, bool INV, int Q = kQ, int TS = 0>
__device__ __forceinline__ void line_dif(float2 (&a)[n / Q], int ql, const float2* tw) {
  constexpr int R = n / Q;
  if constexpr (Q == 4)
    xlane_brev2nat<INV>(a, ql);
  else if constexpr (Q == 8)
    xlane8_brev2nat<INV>(a, ql);
  else
    xlane16_brev2nat<n, INV, R, TS>(a, ql, tw);
#pragma unroll
  for (int m = 1; m < R; ++m) a[m] = cmul(a[m], tw_at<INV, n, TS>(tw, ql * m));
  fft_reg<R, INV>(a);
}

// Q = 16 counterparts (n = 256 kernel): four fused stages; the sign rule is
// the same with par16(ql) = (-1)^popcount(ql) over four bits.
__device__ __forceinline__ float par16(int ql) {
  return (__builtin_popcount(ql) & 1) ? -1.0f : 1.0f;
}
template <int n, bool INV, int R, int TS>
__device__ __forceinline__ void xlane16_nat2brev_f(float2 (&a)[R], int ql, const float2* tw,
                                                   float flip) {
  const float s8 = (ql & 8) ? -flip : flip, s4 = (ql & 4) ? -flip : flip,
              s2 = (ql & 2) ? -flip : flip, s1 = (ql & 1) ? -flip : flip;
  const float2 t16 = tw_at<INV, n, TS>(tw, (ql & 8) ? (ql & 7) * (n / 16) : 0);
  const float2 t8 = w8<INV>((ql & 4) ? (ql & 3) : 0);
  const bool is3 = (ql & 3) == 3;
  xstage_fused<kMirror16>(a, s8);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = cmul(a[i], t16);
  xstage_fused<kMirror8>(a, s4);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = cmul(a[i], t8);
  xstage_fused<kXor2>(a, s2);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = w4_lane3<INV>(a[i], is3);
  xstage_fused<kXor1>(a, s1);
}
template <int n, bool INV, int R, int TS>
__device__ __forceinline__ void xlane16_brev2nat_f(float2 (&a)[R], int ql, const float2* tw,
                                                   float flip) {
  const float s8 = (ql & 8) ? -flip : flip, s4 = (ql & 4) ? -flip : flip,
              s2 = (ql & 2) ? -flip : flip, s1 = (ql & 1) ? -flip : flip;
  const float2 t16 = tw_at<INV, n, TS>(tw, (ql & 8) ? (ql & 7) * (n / 16) : 0);
  const float2 t8 = w8<INV>((ql & 4) ? (ql & 3) : 0);
  const bool is3 = (ql & 3) == 3;
  xstage_fused<kXor1>(a, s1);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = w4_lane3<INV>(a[i], is3);
  xstage_fused<kXor2>(a, s2);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = cmul(a[i], t8);
  xstage_fused<kMirror8>(a, s4);
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = cmul(a[i], t16);
  xstage_fused<kMirror16>(a, s8);
}

// line_dit / line_dif for Q = 8 with the fused cross-lane step (flip as
// for xlane8_nat2brev_f; the register FFT and twiddles are linear, so the
// lane signs pass through them unchanged).
template <int n, bool INV, int TS = 0, int Z = 0, int Q = 8>
__device__ __forceinline__ void line_dit_f(float2 (&a)[n / Q], int ql, const float2* tw,
                                           float flip) {
  constexpr int R = n / Q;
  fft_reg<R, INV, Z, Z>(a);
#pragma unroll
  for (int k = 1; k < R; ++k) a[k] = cmul(a[k], tw_at<INV, n, TS>(tw, ql * k));
  if constexpr (Q == 8)
    xlane8_nat2brev_f<INV>(a, ql, flip);
  else
    xlane16_nat2brev_f<n, INV, R, TS>(a, ql, tw, flip);
}
template <int n, bool INV, int TS = 0, int Q = 8>
__device__ __forceinline__ void line_dif_f(float2 (&a)[n / Q], int ql, const float2* tw,
                                           float flip) {
  constexpr int R = n / Q;
  if constexpr (Q == 8)
    xlane8_brev2nat_f<INV>(a, ql, flip);
  else
    xlane16_brev2nat_f<n, INV, R, TS>(a, ql, tw, flip);
#pragma unroll
  for (int m = 1; m < R; ++m) a[m] = cmul(a[m], tw_at<INV, n, TS>(tw, ql * m));
  fft_reg<R, INV>(a);
}

// The same two transforms with the line's twiddles W^(ql k), k < R, held in
// registers (twl[k] in the inverse orientation exp(+2 pi i ql k / n), the
// forward one taken as its conjugate): a thread keeps its lane ql for the
// whole kernel, so it reads its R - 1 twiddles once instead of once per
// line.  The values, and so the results, are bitwise those of the LDS forms.
template <int n, bool INV, int Z = 0, int Q = 8>
__device__ __forceinline__ void line_dit_fr(float2 (&a)[n / Q], int ql, const float2 (&twl)[n / Q],
                                            const float2* tw, float flip) {
  constexpr int R = n / Q;
  fft_reg<R, INV, Z, Z>(a);
#pragma unroll
  for (int k = 1; k < R; ++k) a[k] = cmul(a[k], INV ? twl[k] : make_float2(twl[k].x, -twl[k].y));
  if constexpr (Q == 8)
    xlane8_nat2brev_f<INV>(a, ql, flip);
  else
    xlane16_nat2brev_f<n, INV, R, 0>(a, ql, tw, flip);
}
template <int n, bool INV, int Q = 8>
__device__ __forceinline__ void line_dif_fr(float2 (&a)[n / Q], int ql, const float2 (&twl)[n / Q],
                                            const float2* tw, float flip) {
  constexpr int R = n / Q;
  if constexpr (Q == 8)
    xlane8_brev2nat_f<INV>(a, ql, flip);
  else
    xlane16_brev2nat_f<n, INV, R, 0>(a, ql, tw, flip);
#pragma unroll
  for (int m = 1; m < R; ++m) a[m] = cmul(a[m], INV ? twl[m] : make_float2(twl[m].x, -twl[m].y));
  fft_reg<R, INV>(a);
}

// P + acc / count with one fused multiply-add per component (the group
// mean, written the same way wherever it is applied)
__device__ __forceinline__ float2 pupil_mean_step(float2 p, float2 acc, int count) {
  const float inv = 1.0f / (float)count;
  return make_float2(fmaf(acc.x, inv, p.x), fmaf(acc.y, inv, p.y));
}

// A copy of v the compiler cannot see through: each phase then reads its own
// twiddles from LDS instead of keeping one set live in registers across the
// whole kernel.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Barrier that orders LDS only, so global loads in flight (the intensity
// prefetch) are not drained at every phase boundary.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Raw buffer access: an offset at or beyond the record count reads 0 and
// drops a store, which turns the support-disc predicates into a select on
// the offset instead of a branch per element.
typedef float v2f __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kOob = 0x7FFFFFF0;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, kRsrcWord3);
}
__device__ __forceinline__ float2 bload2(__amdgpu_buffer_rsrc_t r, int off) {
  const v2f v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, int off, float2 x) {
  v2f v;
  v.x = x.x;
  v.y = x.y;
  __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
}

// complex elements per row of the LDS transpose buffer; the padding only
// moves rows across LDS banks (the autotuner picks it per tile size)
template <int n, int PAD = 16>
constexpr int pitch() {
  return n + PAD;
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

// ------------------------------------------------ phase A: gather + IFFT
// Thread (c, q) with c < nd: support column kx = kx0 + c, rows ky = q + 4p.
// Sw / Pw: buffer views of the LED's spectrum window and of the pupil.
// Returns the partial max |P|^2 of this thread's support pixels.
// Z: rows q + Q p with p < Z or p >= R - Z lie outside every chord of the
// launch (the support's row range starts at or after Q Z and ends at or
// before n - Q Z), so those values are zero without a load.
template <int n, int Q = kQ, int Z = 0>
__device__ __forceinline__ float gather_phi(__amdgpu_buffer_rsrc_t Sw, __amdgpu_buffer_rsrc_t Pw,
                                            int N, int kx, int2 ch, int q, float scale,
                                            float2 (&a)[n / Q]) {
  constexpr int R = n / Q;
  float pm = 0.0f;
  const int s0 = (q * N + kx) * 8, p0 = (q * n + kx) * 8;
#pragma unroll
  for (int p = 0; p < R; ++p) {
    if (p < Z || p >= R - Z) {
      a[p] = make_float2(0.0f, 0.0f);
      continue;
    }
    const int ky = q + Q * p;
    const bool in = ky >= ch.x && ky <= ch.y;
    const float2 xs = bload2(Sw, in ? s0 + p * (Q * 8) * N : kOob);
    const float2 pv = bload2(Pw, in ? p0 + p * (Q * 8 * n) : kOob);
    pm = fmaxf(pm, cabs2(pv));
    a[p] = cscale(cmul(pv, xs), scale);
  }
  return pm;
}

// phase B input: logical lane q of row y takes kx = q + Q p from T[kx - kx0][y]
template <int n, int PAD = 16, int Q = kQ, int Z = 0>
__device__ __forceinline__ void load_rows(const float2* buf, int kx0, int nd, int y, int q,
                                          float2 (&a)[n / Q]) {
  constexpr int R = n / Q;
#pragma unroll
  for (int p = 0; p < R; ++p) {
    if (p < Z || p >= R - Z) {  // outside every support column (see gather_phi)
      a[p] = make_float2(0.0f, 0.0f);
      continue;
    }
    const int c = q + Q * p - kx0;
    a[p] = (c >= 0 && c < nd) ? buf[c * pitch<n, PAD>() + y] : make_float2(0.0f, 0.0f);
  }
}

// threads of the iteration-end kernel (one workgroup per tile)
constexpr int kIterEndThreads = 1024;

// max(I, 0) as one integer maximum: a float with its sign bit clear compares
// as a non-negative integer in the order of its value, every other one
// (negative values and -0) gives +0.  The result is fmaxf(I, 0) for every
// input but NaN, which the entry points reject before any kernel runs.
__device__ __forceinline__ float clamp0(float I) {
  return __int_as_float(max(__float_as_int(I), 0));
}

// Modulus projection of one row segment and its residual partials.
// a[k] holds psi at (row `line`, column xc + k) of the unshifted frame.
// zpar = 1: the lane's values carry the sign -1 (fused cross-lane steps);
// the projection is odd in psi, so only the zero-field value needs it.
template <int R>
__device__ __forceinline__ void modulus_row(float2 (&a)[R], const float (&ipre)[R], int line,
                                            int xc, float& e_acc, float& i_acc, int zpar = 0) {
  // Where no value of the wave's rows is zero or below 2^-100 in |psi|^2
  // (everywhere but the windows a sweep has not reached yet), the scaling
  // and zero-field selects below are the identity; that case takes the
  // same operations without them, one branch for the wave.
  float p2v[R];
  bool plain = true;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    p2v[k] = cabs2(a[k]);
    plain &= p2v[k] >= 0x1p-100f;
  }
  if (__all(plain)) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const float I = ipre[k];
      const float m = __builtin_amdgcn_sqrtf(clamp0(I));
      const float rinv = __builtin_amdgcn_rsqf(p2v[k]);
      const float d = p2v[k] * rinv - m;
      e_acc = fmaf(d, d, e_acc);
      i_acc += I;
      a[k] = cscale(a[k], m * rinv);
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const float I = ipre[k];
    const float m = __builtin_amdgcn_sqrtf(clamp0(I));
    // psi' = m psi / |psi| through the hardware reciprocal square root, which
    // flushes denormal inputs: a field whose |psi|^2 is below 2^-100 is
    // first scaled by 2^100 (exact), so every nonzero psi keeps its phase.
    // Where psi = 0 the method sets psi' = sqrt(I) in the centred frame; this
    // frame differs from it by (-1)^(x+y), so the zero-field value is
    // (-1)^(x+y) sqrt(I) here.
    const float m_zero = ((line + xc + k + zpar) & 1) ? -m : m;
    const float p2 = p2v[k];
    const bool small = p2 < 0x1p-100f;
    const float2 as = small ? cscale(a[k], 0x1p100f) : a[k];
    const float p2s = small ? cabs2(as) : p2;
    const bool live = p2s > 0.0f;
    const float rinv = live ? __builtin_amdgcn_rsqf(p2s) : 0.0f;
    const float amp = p2s * rinv * (small ? 0x1p-100f : 1.0f);
    const float d = amp - m;
    e_acc = fmaf(d, d, e_acc);
    i_acc += I;
    const float s = m * rinv;
    a[k] = live ? cscale(as, s) : make_float2(m_zero, 0.0f);
  }
}

// Spectrum (and pupil) update of one support column kx: a[k] = Phi'(ky =
// q + Q k, kx), q the logical lane.  S_stored += conj(P) D / (max|P|^2 sigma); the pupil step
// conj(sigma S_stored) D / (sigma^2 smax) = conj(S_stored) D / (sigma smax)
// goes to P (mode 1) or to the increment slot (mode 2).
// SEQ (one workgroup runs every member of a tile's LED group in slot
// order): the increments are summed in place in slot 0, and the last member
// applies P <- P + sum / count -- the same operations in the same order as
// pupil_reduce_kernel, so both forms give the same bits.
// The stored spectrum of a support column (the values update_column reads),
// loaded ahead of the column transform where registers allow.
template <int n, int Q = kQ, int Z = 0>
__device__ __forceinline__ void load_column(__amdgpu_buffer_rsrc_t Sw, int N, int kx, int2 ch,
                                            int q, float2 (&xs)[n / Q]) {
  constexpr int R = n / Q;
  const int s0 = (q * N + kx) * 8;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k < Z || k >= R - Z) continue;  // outside every chord (see gather_phi)
    const int ky = q + Q * k;
    const bool in = ky >= ch.x && ky <= ch.y;
    xs[k] = bload2(Sw, in ? s0 + k * (Q * 8) * N : kOob);
  }
}
template <int n, int Q = kQ, int Z = 0>
__device__ __forceinline__ void load_pupil_column(__amdgpu_buffer_rsrc_t Pw, int kx, int2 ch,
                                                  int q, float2 (&pv)[n / Q]) {
  constexpr int R = n / Q;
  const int p0 = (q * n + kx) * 8;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k < Z || k >= R - Z) continue;  // outside every chord (see gather_phi)
    const int ky = q + Q * k;
    const bool in = ky >= ch.x && ky <= ch.y;
    pv[k] = bload2(Pw, in ? p0 + k * (Q * 8 * n) : kOob);
  }
}

// The update of one support pixel from the transformed exit wave av (with
// the lane sign folded into sig_d, inv_ps and inv_ss), the stored spectrum
// xs and the pupil pv: the spectrum step and, with pupil recovery, the pupil
// step or its increment.  offS / offP are kOob outside the pixel's chord.
template <bool SEQ>
__device__ __forceinline__ void update_px(float2 av, float2 xs, float2 pv,
                                          __amdgpu_buffer_rsrc_t Sw, __amdgpu_buffer_rsrc_t Pw,
                                          __amdgpu_buffer_rsrc_t Dw, int offS, int offP,
                                          float sig_d, float inv_ps, float inv_ss, bool upd_s,
                                          int mode, int slot, int count) {
  // explicit fused multiply-adds: every caller rounds the update identically,
  // whatever the compiler contracts elsewhere
  const float2 px = cmul_fma(pv, xs);  // D = Phi' - sigma P X
  const float2 d = make_float2(fmaf(-px.x, sig_d, av.x), fmaf(-px.y, sig_d, av.y));
  const float2 ts = cmulc_fma(d, pv);
  bstore2(Sw, upd_s ? offS : kOob, make_float2(fmaf(ts.x, inv_ps, xs.x), fmaf(ts.y, inv_ps, xs.y)));
  if (mode != 0) {
    const float2 tp = cmulc_fma(d, xs);
    if (mode == 1) {
      bstore2(Pw, offP, make_float2(fmaf(tp.x, inv_ss, pv.x), fmaf(tp.y, inv_ss, pv.y)));
    } else {
      // the increment is rounded before any sum, as when it is stored for
      // the separate group-mean kernel
      const float2 dp = make_float2(__fmul_rn(tp.x, inv_ss), __fmul_rn(tp.y, inv_ss));
      if constexpr (SEQ) {
        const float2 acc = slot == 0 ? dp : cadd(bload2(Dw, offP), dp);
        if (slot == count - 1)
          bstore2(Pw, offP, pupil_mean_step(pv, acc, count));
        else
          bstore2(Dw, offP, acc);
      } else {
        bstore2(Dw, offP, dp);
      }
    }
  }
}

template <int n, int Q = kQ, bool SEQ = false, bool PRE = false, int Z = 0>
__device__ __forceinline__ void update_column(const float2 (&a)[n / Q],
                                              __amdgpu_buffer_rsrc_t Sw,
                                              __amdgpu_buffer_rsrc_t Pw,
                                              __amdgpu_buffer_rsrc_t Dw, int N, int kx, int2 ch,
                                              int q, float sigf, float pmax2, float smax,
                                              int mode, int slot = 0, int count = 1,
                                              const float2* xs_pre = nullptr,
                                              const float2* pv_pre = nullptr,
                                              float lane_sign = 1.0f) {
  constexpr int R = n / Q;
  // a[] may carry a lane sign (fused cross-lane steps): D, and with it both
  // steps, then come out with that sign, which the step scales cancel; the
  // products with +-1 are exact, so the bits are those of lane_sign = 1
  const float inv_ps = lane_sign * (pmax2 > 0.0f ? 1.0f / (pmax2 * sigf) : 0.0f);
  const float inv_ss = lane_sign * (smax > 0.0f ? 1.0f / (smax * sigf) : 0.0f);
  const float sig_d = lane_sign * sigf;
  const int s0 = (q * N + kx) * 8, p0 = (q * n + kx) * 8;
  const bool upd_s = pmax2 > 0.0f;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (k < Z || k >= R - Z) continue;  // outside every chord (see gather_phi)
    const int ky = q + Q * k;
    const bool in = ky >= ch.x && ky <= ch.y;
    const int offS = in ? s0 + k * (Q * 8) * N : kOob;
    const int offP = in ? p0 + k * (Q * 8 * n) : kOob;
    // stored spectrum (this WG's own support pixels), loaded here or ahead
    const float2 xs = PRE ? xs_pre[k] : bload2(Sw, offS);
    const float2 pv = PRE ? pv_pre[k] : bload2(Pw, offP);
    update_px<SEQ>(a[k], xs, pv, Sw, Pw, Dw, offS, offP, sig_d, inv_ps, inv_ss, upd_s, mode, slot,
                   count);
  }
}

}  // namespace

// ===================================================== the update kernel
// t.mode: 0 = spectrum only, 1 = pupil updated in place (one LED per tile in
// the launch), 2 = pupil increment written to dP[slot] (LED groups).
// Q lanes per line: 4 (R = n/4 points per lane) or 8 (R = n/8, twice the
// waves per update); PAD and Q are the autotuner's choices.
// SEQ: workgroup b runs items ranges[b].x .. + ranges[b].y - 1 one after
// another (the members of one tile's LED group, in slot order); otherwise
// workgroup b runs item b.
template <int n, int PAD, int Q, bool SEQ>
__global__ __launch_bounds__(n * Q) void update_kernel(const TileDev* __restrict__ tiles,
                                                       const Item* __restrict__ items,
                                                       const int2* __restrict__ ranges,
                                                       int count) {
  constexpr int R = n / Q;
  constexpr int NT = n * Q;
  constexpr int NW = NT / 64;
  extern __shared__ float2 sbuf[];  // [nd][pitch]
  __shared__ float2 tw[n];
  __shared__ float red_pmax[NW];
  __shared__ double red_e[NW], red_i[NW];

  // the body of one item; the group-sequential form loops over its range,
  // the other runs it once (a loop there, even of one trip, costs registers)
  auto run_item = [&](const int ii) {
  const Item it = items[ii];
  const TileDev t = tiles[it.tile];
  const int mode = t.mode;
  const int tid = threadIdx.x;
  const int q = lane_log<Q>(tid % Q), line = tid / Q;
  const int wave = tid >> 6;
  const int N = t.N;

  // buffer views: this LED's spectrum window, the pupil, its intensity image,
  // the pupil-increment slot
  const size_t woff = (size_t)it.wy0 * N + it.wx0;
  const __amdgpu_buffer_rsrc_t Sw = make_rsrc(t.S + woff, (unsigned)(((size_t)N * N - woff) * 8));
  const __amdgpu_buffer_rsrc_t Pw = make_rsrc(t.P, n * n * 8);
  const __amdgpu_buffer_rsrc_t Iw = make_rsrc(t.I + (size_t)it.led * n * n, n * n * 4);
  const __amdgpu_buffer_rsrc_t Dw = make_rsrc(t.dP + (SEQ ? 0 : (size_t)it.slot * n * n), n * n * 8);

  // twiddle table W_n^e = exp(+2 pi i e/n), correctly rounded at compile time
  for (int e = tid; e < n; e += NT) tw[e] = make_float2(kTw<n>.c[e], kTw<n>.s[e]);

  // prefetch this thread's intensities for the modulus step: row `line`,
  // columns [R*brevq(q), +R)
  const int xc = R * brevq<Q>(q);
  float ipre[R];
#pragma unroll
  for (int v = 0; v < R / 4; ++v) {
    const v4f f = __builtin_amdgcn_raw_buffer_load_b128(Iw, (line * n + xc + 4 * v) * 4, 0, 0);
    ipre[4 * v] = f.x;
    ipre[4 * v + 1] = f.y;
    ipre[4 * v + 2] = f.z;
    ipre[4 * v + 3] = f.w;
  }

  const float sigf = (float)*t.sigma;
  float2 a[R];
  float pm = 0.0f;
  const bool col_line = line < t.nd;
  const int kx = t.kx0 + (col_line ? line : 0);
  const int2 ch = col_line ? t.chord[kx] : make_int2(n, -1);
  lds_barrier();  // twiddles ready

  // ---- phase A: support columns, IFFT along ky
  if (col_line) {
    pm = gather_phi<n, Q>(Sw, Pw, N, kx, ch, q, sigf / (float)(n * n), a);
    line_dit<n, true, Q>(a, opaque(q), tw);
    float2* dst = sbuf + line * pitch<n, PAD>() + xc;
#pragma unroll
    for (int k = 0; k < R; ++k) dst[k] = a[k];
  }
  pm = wave_max(pm);
  if ((tid & 63) == 0) red_pmax[wave] = pm;
  lds_barrier();

  // ---- phase B: rows, IFFT along kx
  load_rows<n, PAD, Q>(sbuf, t.kx0, t.nd, line, q, a);
  lds_barrier();  // T fully consumed; the buffer is reused below
  line_dit<n, true, Q>(a, opaque(q), tw);

  // ---- modulus constraint + residual partials (row `line`, x = xc + k)
  float e_acc = 0.0f, i_acc = 0.0f;
  modulus_row<R>(a, ipre, line, xc, e_acc, i_acc);
  {
    double e = wave_sum((double)e_acc), s = wave_sum((double)i_acc);
    if ((tid & 63) == 0) {
      red_e[wave] = e;
      red_i[wave] = s;
    }
  }

  // ---- phase B': FFT along x (lane q holds x-chunk brevq(q))
  line_dif<n, false, Q>(a, opaque(q), tw);
  // a[k] = row-transform at kx = q + Q k; keep the support columns only
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int c = q + Q * k - t.kx0;
    if (c >= 0 && c < t.nd) sbuf[c * pitch<n, PAD>() + line] = a[k];
  }
  lds_barrier();

  // ---- phase A': support columns, FFT along y, then the update
  if (col_line) {
    const float2* srcp = sbuf + line * pitch<n, PAD>() + xc;
#pragma unroll
    for (int m = 0; m < R; ++m) a[m] = srcp[m];
    line_dif<n, false, Q>(a, opaque(q), tw);
    // a[k] = Phi'(ky = q + Q k, kx)
    float pmax2 = red_pmax[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) pmax2 = fmaxf(pmax2, red_pmax[w]);
    const float smax = __uint_as_float(*t.smax);  // max |S_stored|^2
    update_column<n, Q, SEQ>(a, Sw, Pw, Dw, N, kx, ch, q, sigf, pmax2, smax, mode, it.slot,
                             it.gsize);
  }

  if (tid == 0) {
    double e = 0.0, s = 0.0;
    for (int w = 0; w < NW; ++w) {
      e += red_e[w];
      s += red_i[w];
    }
    t.e_part[(size_t)it.iter * t.e_stride + it.led] = e;
    t.i_part[(size_t)it.iter * t.e_stride + it.led] = s;
  }
  };
  if constexpr (SEQ) {
    const int2 rg = ranges[blockIdx.x];
    for (int ii = rg.x; ii < rg.x + rg.y; ++ii) {
      run_item(ii);
      lds_barrier();  // LDS and reductions are reused by the next member
    }
  } else {
    const int ii = xcd_item((int)blockIdx.x, count);
    if (ii >= 0) run_item(ii);
  }
}

// Two-workgroups-per-CU form of the update: n Q / ROUNDS threads run the
// lines of each phase in ROUNDS rounds (lines l, l + n/ROUNDS, ...), so a
// workgroup holds half the waves and, with the twiddles in the padding column
// of the transpose buffer (rows max(nd, n/2)), under half of the CU's LDS:
// two updates share a CU and fill each other's barrier and memory waits.
// Each line is transformed exactly as in update_kernel, so both give the
// same bits.  A phase-B thread reads and writes only its own columns of its
// own row, so the row transforms work in place without a barrier.
// Z (Q = 8 only): the values q + Q k with k < Z or k >= R - Z of every line
// lie outside the support of every tile of the launch (the launcher derives
// Z from the widest support), so they are neither loaded nor stored, and
// the row and column IFFTs skip their first-stage arithmetic.
template <int n, int PAD, int Q, int ROUNDS, bool SEQ, int Z = 0>
__global__ __launch_bounds__(n * Q / ROUNDS, 2 * (n * Q / ROUNDS) / 256) void update_kernel_rounds(
    const TileDev* __restrict__ tiles, const Item* __restrict__ items,
    const int2* __restrict__ ranges, int count) {
  constexpr int R = n / Q;
  constexpr int NT = n * Q / ROUNDS;
  constexpr int LPR = NT / Q;  // lines per round
  constexpr int NW = NT / 64;
  constexpr int PT = pitch<n, PAD>();
  static_assert(PAD >= 1 && LPR * ROUNDS == n && NT % 64 == 0, "layout");
  static_assert(R % 4 == 0, "intensities are read four at a time");
  extern __shared__ float2 sbuf[];  // [max(nd, n/2)][PT]; column n: twiddles
  float2* const tw = sbuf + n;
  // Q = 8: position pos (< n) of a row sits at pos ^ (2 ((pos / 16) mod 8)),
  // a permutation within each aligned block of 16 that keeps pairs
  // together.  The lanes of a line read and write runs xc .. xc + R - 1
  // with xc = 16 brev(q): unswizzled, all eight of them start in the same
  // LDS bank; swizzled, the eight runs start in eight different banks.
  auto sw = [](int pos) { return Q == 8 ? pos ^ ((pos >> 3) & 14) : pos; };
  __shared__ float red_pmax[NW];
  // residual partials per (round, wave): the waves of update_kernel, in order
  __shared__ double red_e[ROUNDS * NW], red_i[ROUNDS * NW];

  auto run_item = [&](const int ii) {
  const Item it = items[ii];
  const TileDev t = tiles[it.tile];
  const int mode = t.mode;
  const int tid = threadIdx.x;
  const int q_item = lane_log<Q>(tid % Q), l0 = tid / Q;
  const int wave = tid >> 6;
  const int N = t.N;
  const int xc = R * brevq<Q>(q_item);
  const size_t woff = (size_t)it.wy0 * N + it.wx0;
  const __amdgpu_buffer_rsrc_t Sw = make_rsrc(t.S + woff, (unsigned)(((size_t)N * N - woff) * 8));
  const __amdgpu_buffer_rsrc_t Pw = make_rsrc(t.P, n * n * 8);
  const __amdgpu_buffer_rsrc_t Iw = make_rsrc(t.I + (size_t)it.led * n * n, n * n * 4);
  const __amdgpu_buffer_rsrc_t Dw = make_rsrc(t.dP + (SEQ ? 0 : (size_t)it.slot * n * n), n * n * 8);
  for (int e = tid; e < n / 2; e += NT) tw[e * PT] = make_float2(kTw<n>.c[e], kTw<n>.s[e]);
  const float sigf = (float)*t.sigma;
  float2 a[R];
  lds_barrier();  // twiddles ready
  // Q = 8 with R <= 16: the thread's line twiddles live in registers
  constexpr bool kTwReg = Q == 8 && R <= 16;
  float2 twl[R];
  if constexpr (kTwReg) {
    twl[0] = make_float2(1.0f, 0.0f);
#pragma unroll
    for (int k = 1; k < R; ++k) twl[k] = tw_at<true, n, PT>(tw, q_item * k);
  }

  // ---- phase A: support columns, IFFT along ky
  // Q = 8: sigma P S of every support column is first read row by row (a
  // wave takes two rows of LPR consecutive columns, whole row segments) into
  // the column's LDS row at its ky; after one barrier each column's lanes
  // take their values from there.  Read column by column, every load
  // instruction of a wave touched eight rows, 64 bytes of each.  Thread
  // (c_off, y_off) takes the rows y_off + Q p of its columns, the rows lane
  // q = y_off of a line holds; the input sign of row ky is par8(ky mod 8).
  float pm = 0.0f;
  const int c_off = tid % LPR, y_off = tid / LPR;  // y_off < Q
  if constexpr (Q == 8) {
    const float s0 = sigf / (float)(n * n);
#pragma unroll 1
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int c = LPR * rd + c_off;
      if (c < t.nd) {
        const int kx = t.kx0 + c;
        const int2 ch = t.chord[kx];
        float2 xs[R], pv[R];
#pragma unroll
        for (int p = Z; p < R - Z; ++p) {
          const int ky = y_off + Q * p;
          const bool in = ky >= ch.x && ky <= ch.y;
          xs[p] = bload2(Sw, in ? (ky * N + kx) * 8 : kOob);
          pv[p] = bload2(Pw, in ? (ky * n + kx) * 8 : kOob);
        }
        float2* col = sbuf + c * PT;
#pragma unroll
        for (int p = Z; p < R - Z; ++p) {
          const int ky = y_off + Q * p;
          pm = fmaxf(pm, cabs2(pv[p]));
          col[sw(ky)] = cscale(cmul(pv[p], xs[p]), par8(ky & 7) * s0);
        }
      }
    }
    lds_barrier();
  }
#pragma unroll 1
  for (int rd = 0; rd < ROUNDS; ++rd) {
    const int line = l0 + LPR * rd;
    if (line < t.nd) {
      const int q = R > 16 ? opaque(q_item) : q_item;
      if constexpr (Q == 8) {
        // input signs par8(q) (folded into the staged values), output signs +1
        const float2* col = sbuf + line * PT;
#pragma unroll
        for (int p = 0; p < R; ++p)
          a[p] = (p < Z || p >= R - Z) ? make_float2(0.0f, 0.0f) : col[sw(q + Q * p)];
        if constexpr (kTwReg)
          line_dit_fr<n, true, Z>(a, q, twl, tw, -1.0f);
        else
          line_dit_f<n, true, PT, Z>(a, q, tw, -1.0f);
      } else {
        const int kx = t.kx0 + line;
        pm = fmaxf(pm, gather_phi<n, Q>(Sw, Pw, N, kx, t.chord[kx], q, sigf / (float)(n * n), a));
        line_dit<n, true, Q, PT>(a, q, tw);
      }
      float2* dst = sbuf + line * PT;
#pragma unroll
      for (int k = 0; k < R; ++k) dst[sw(xc + k)] = a[k];
    }
  }
  pm = wave_max(pm);
  if ((tid & 63) == 0) red_pmax[wave] = pm;
  lds_barrier();

  // ---- phase B: rows, IFFT along kx, modulus, FFT along x, in place
#pragma unroll 1
  for (int rd = 0; rd < ROUNDS; ++rd) {
    const int line = l0 + LPR * rd;
    const int q = R > 16 ? opaque(q_item) : q_item;
    // the row's intensities are requested first, so that their latency
    // overlaps the row transform; with 32 points per lane that costs more
    // registers than the latency it hides, and they are requested after it
    float iv[R];
    auto load_iv = [&](int row) {
#pragma unroll
      for (int v = 0; v < R / 4; ++v) {
        const v4f f = __builtin_amdgcn_raw_buffer_load_b128(Iw, (row * n + xc + 4 * v) * 4, 0, 0);
        iv[4 * v] = f.x;
        iv[4 * v + 1] = f.y;
        iv[4 * v + 2] = f.z;
        iv[4 * v + 3] = f.w;
      }
    };
    if constexpr (R <= 16) load_iv(line);
#pragma unroll
    for (int p = 0; p < R; ++p) {  // load_rows, through the swizzle
      if (p < Z || p >= R - Z) {
        a[p] = make_float2(0.0f, 0.0f);
        continue;
      }
      const int c = q + Q * p - t.kx0;
      a[p] = (c >= 0 && c < t.nd) ? sbuf[c * PT + sw(line)] : make_float2(0.0f, 0.0f);
    }
    // Q = 8: the row IFFT leaves lane signs par8(q), which the modulus keeps
    // and the row FFT removes
    if constexpr (kTwReg)
      line_dit_fr<n, true, Z>(a, q, twl, tw, 1.0f);
    else if constexpr (Q == 8)
      line_dit_f<n, true, PT, Z>(a, q, tw, 1.0f);
    else
      line_dit<n, true, Q, PT>(a, q, tw);
    if constexpr (R > 16) load_iv(opaque(line));
    float e_acc = 0.0f, i_acc = 0.0f;
    modulus_row<R>(a, iv, line, xc, e_acc, i_acc, Q == 8 ? (__builtin_popcount(q) & 1) : 0);
    {
      const double e = wave_sum((double)e_acc), s2 = wave_sum((double)i_acc);
      if ((tid & 63) == 0) {
        red_e[rd * NW + wave] = e;
        red_i[rd * NW + wave] = s2;
      }
    }
    if constexpr (kTwReg)
      line_dif_fr<n, false>(a, q, twl, tw, -1.0f);
    else if constexpr (Q == 8)
      line_dif_f<n, false, PT>(a, q, tw, -1.0f);
    else
      line_dif<n, false, Q, PT>(a, q, tw);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (k < Z || k >= R - Z) continue;  // no support column there
      const int c = q + Q * k - t.kx0;
      if (c >= 0 && c < t.nd) sbuf[c * PT + sw(line)] = a[k];
    }
  }
  lds_barrier();

  // ---- phase A': support columns, FFT along y, then the update
  float pmax2 = red_pmax[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) pmax2 = fmaxf(pmax2, red_pmax[w]);
  const float smax = __uint_as_float(*t.smax);  // max |S_stored|^2
  if constexpr (Q == 8) {
    // the column FFTs' outputs go back to each column's LDS row at their ky
    // (a line's lanes read all of the row before any of them writes it: one
    // wave); after one barrier the update runs row by row over whole row
    // segments, as the gather does, with the lane sign par8(ky mod 8)
#pragma unroll 1
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int line = l0 + LPR * rd;
      if (line < t.nd) {
        const int q = q_item;
        float2* col = sbuf + line * PT;
#pragma unroll
        for (int m = 0; m < R; ++m) a[m] = col[sw(xc + m)];
        if constexpr (kTwReg)
          line_dif_fr<n, false>(a, q, twl, tw, 1.0f);  // output signs par8(q)
        else
          line_dif_f<n, false, PT>(a, q, tw, 1.0f);
#pragma unroll
        for (int k = Z; k < R - Z; ++k) col[sw(q + Q * k)] = a[k];
      }
    }
    lds_barrier();
    const float ips = pmax2 > 0.0f ? 1.0f / (pmax2 * sigf) : 0.0f;
    const float iss = smax > 0.0f ? 1.0f / (smax * sigf) : 0.0f;
#pragma unroll 1
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int c = LPR * rd + c_off;
      if (c < t.nd) {
        const int kx = t.kx0 + c;
        const int2 ch = t.chord[kx];
        float2 xs[R], pv[R];
        int offS[R], offP[R];
#pragma unroll
        for (int p = Z; p < R - Z; ++p) {
          const int ky = y_off + Q * p;
          const bool in = ky >= ch.x && ky <= ch.y;
          offS[p] = in ? (ky * N + kx) * 8 : kOob;
          offP[p] = in ? (ky * n + kx) * 8 : kOob;
          xs[p] = bload2(Sw, offS[p]);
          pv[p] = bload2(Pw, offP[p]);
        }
        const float2* col = sbuf + c * PT;
#pragma unroll
        for (int p = Z; p < R - Z; ++p) {
          const int ky = y_off + Q * p;
          const float ls = par8(ky & 7);
          update_px<SEQ>(col[sw(ky)], xs[p], pv[p], Sw, Pw, Dw, offS[p], offP[p], ls * sigf, ls * ips,
                         ls * iss, pmax2 > 0.0f, mode, it.slot, it.gsize);
        }
      }
    }
  } else {
#pragma unroll 1
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int line = l0 + LPR * rd;
      if (line < t.nd) {
        const int q = R > 16 ? opaque(q_item) : q_item;
        const int kx = t.kx0 + line;
        const int2 ch = t.chord[kx];
        // the column's stored spectrum is requested before its transform where
        // registers allow (R <= 16); longer lane segments load it in the update
        constexpr bool kPre = R <= 16;
        float2 xs[kPre ? R : 1], pv[kPre ? R : 1];
        if constexpr (kPre) {
          load_column<n, Q, Z>(Sw, N, kx, ch, q, xs);
          load_pupil_column<n, Q, Z>(Pw, kx, ch, q, pv);
        }
        const float2* srcp = sbuf + line * PT;
#pragma unroll
        for (int m = 0; m < R; ++m) a[m] = srcp[sw(xc + m)];
        line_dif<n, false, Q, PT>(a, q, tw);
        update_column<n, Q, SEQ, kPre>(a, Sw, Pw, Dw, N, kx, ch, q, sigf, pmax2, smax, mode,
                                       it.slot, it.gsize, xs, pv);
      }
    }
  }
  if (tid == 0) {
    double e = 0.0, s2 = 0.0;
    for (int w = 0; w < ROUNDS * NW; ++w) {
      e += red_e[w];
      s2 += red_i[w];
    }
    t.e_part[(size_t)it.iter * t.e_stride + it.led] = e;
    t.i_part[(size_t)it.iter * t.e_stride + it.led] = s2;
  }
  };
  if constexpr (SEQ) {
    const int2 rg = ranges[blockIdx.x];
    for (int ii = rg.x; ii < rg.x + rg.y; ++ii) {
      run_item(ii);
      lds_barrier();  // LDS and reductions are reused by the next member
    }
  } else {
    const int ii = xcd_item((int)blockIdx.x, count);
    if (ii >= 0) run_item(ii);
  }
}

// ================================================ forward model per LED
// I_j = |IFFT_n(P * W_j(S))|^2 (the (-1)^(x+y) of the centring shift drops
// out of the modulus).  sigma = 1, S is the object's scaled spectrum.
template <int n>
__global__ __launch_bounds__(n * kQ) void forward_kernel(const TileDev* __restrict__ tiles,
                                                         const Item* __restrict__ items,
                                                         float* __restrict__ out,
                                                         const int64_t* __restrict__ out_off) {
  constexpr int R = n / kQ;
  constexpr int NT = n * kQ;
  extern __shared__ float2 sbuf[];
  __shared__ float2 tw[n];
  const Item it = items[blockIdx.x];
  const TileDev t = tiles[it.tile];
  const int tid = threadIdx.x;
  const int q = tid & 3, line = tid >> 2;
  for (int e = tid; e < n; e += NT) tw[e] = make_float2(kTw<n>.c[e], kTw<n>.s[e]);
  lds_barrier();
  float2 a[R];
  if (line < t.nd) {
    const size_t woff = (size_t)it.wy0 * t.N + it.wx0;
    const __amdgpu_buffer_rsrc_t Sw =
        make_rsrc(t.S + woff, (unsigned)(((size_t)t.N * t.N - woff) * 8));
    const __amdgpu_buffer_rsrc_t Pw = make_rsrc(t.P, n * n * 8);
    const int kx = t.kx0 + line;
    gather_phi<n>(Sw, Pw, t.N, kx, t.chord[kx], q, 1.0f / (float)(n * n), a);
    line_dit<n, true>(a, q, tw);
    float2* dst = sbuf + line * pitch<n>() + R * brevq<kQ>(q);
#pragma unroll
    for (int k = 0; k < R; ++k) dst[k] = a[k];
  }
  lds_barrier();
  load_rows<n>(sbuf, t.kx0, t.nd, line, q, a);
  line_dit<n, true>(a, q, tw);
  float4* dst = reinterpret_cast<float4*>(out + out_off[it.tile] + (size_t)it.led * n * n +
                                          (size_t)line * n + R * brevq<kQ>(q));
#pragma unroll
  for (int v = 0; v < R / 4; ++v)
    dst[v] = make_float4(cabs2(a[4 * v]), cabs2(a[4 * v + 1]), cabs2(a[4 * v + 2]),
                         cabs2(a[4 * v + 3]));
}

// ============================== sides whose transposes exceed LDS (n = 256)
// Persistent form of the update: 512 threads run the lines of each phase in
// Q n/512 rounds (Q = 16 lanes per line and R = n/16 points per lane by
// default, which needs no register spills; Q = 8, R = n/8 also exists), and
// each workgroup loops over items blockIdx.x, blockIdx.x + gridDim.x, ...
// The two transposes ([nd][n] complex values, 321 KB at n = 256 and NA 0.1)
// do not fit in LDS; they go through this workgroup's own slot of global
// scratch, or with HALF, rows 0 .. n/2 - 1 through LDS (up to kBigLdsCols
// support columns, 157 KB: the workgroup then has the CU's LDS to itself,
// which its registers already impose) and only rows n/2 .. n - 1 through the
// slot.  Phase B writes the support columns of its rows back in place: a
// thread reads and writes only its own columns (one residue mod Q) of its
// own row, so no other thread's input is overwritten.
constexpr int kBigThreads = 512;
constexpr int kBigLdsCols = 157;

// Transpose layout (slot and LDS half): blocks of four consecutive rows of
// one support column, (row / 4, column, row % 4), `cols` columns per block
// row.  A wave of the row phase then reads and writes 16 columns x 4 rows =
// 512 contiguous bytes per instruction, and a column lane 4 rows = 32
// contiguous bytes, instead of 8-byte pieces n * 8 bytes apart.
template <int cols>
__device__ __forceinline__ int big_block(int c, int r) {
  return ((r >> 2) * cols + c) * 4 + (r & 3);
}

// FUSED (Q = 16): the fused cross-lane steps and the support pruning Z of
// update_kernel_rounds, with the same lane-sign bookkeeping (par16).
template <int n, int Q, bool FUSED = false, int Z = 0, bool HALF = false>
__global__ __launch_bounds__(kBigThreads) void update_kernel_big(const TileDev* __restrict__ tiles,
                                                                 const Item* __restrict__ items,
                                                                 int count,
                                                                 float2* __restrict__ scratch) {
  constexpr int R = n / Q;
  constexpr int NT = kBigThreads;
  constexpr int LPR = NT / Q;        // lines per round
  constexpr int ROUNDS = n / LPR;
  constexpr int NW = NT / 64;
  __shared__ float2 tw[n];
  __shared__ float red_pmax[NW];
  __shared__ double red_e[NW], red_i[NW];
  // rows 0 .. n/2 - 1 of the transposes (HALF); one element otherwise
  __shared__ float2 lh[HALF ? kBigLdsCols * (n / 2) : 1];
  const int tid0 = threadIdx.x;
  for (int e = tid0; e < n; e += NT) tw[e] = make_float2(kTw<n>.c[e], kTw<n>.s[e]);
  float2* __restrict__ sb = scratch + (size_t)blockIdx.x * n * n;
  __syncthreads();

  // items in XCD-aware order: the workgroups on XCD x (b mod kXcds = x; the
  // grid is a multiple of kXcds) run block x of the items, so a tile's
  // members share its pupil in that XCD's L2
  const int per = (count + kXcds - 1) / kXcds, wg_per_xcd = (int)gridDim.x / kXcds;
  const int xcd = (int)blockIdx.x % kXcds;
  for (int m = (int)blockIdx.x / kXcds; m < per && xcd * per + m < count; m += wg_per_xcd) {
    const int ii = xcd * per + m;
    // lane indices are re-derived per item through an opaque copy, so the
    // compiler does not hoist every address they feed out of the item loop
    // (that kept hundreds of values live across the whole kernel)
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const int q_item = lane_log<Q>(tid % Q), l0 = tid / Q;
    const int wave = tid >> 6;
    const int xc = R * brevq<Q>(q_item);
    const Item it = items[ii];
    const TileDev t = tiles[it.tile];
    const int N = t.N;
    const size_t woff = (size_t)it.wy0 * N + it.wx0;
    const __amdgpu_buffer_rsrc_t Sw = make_rsrc(t.S + woff, (unsigned)(((size_t)N * N - woff) * 8));
    const __amdgpu_buffer_rsrc_t Pw = make_rsrc(t.P, n * n * 8);
    const __amdgpu_buffer_rsrc_t Iw = make_rsrc(t.I + (size_t)it.led * n * n, n * n * 4);
    const __amdgpu_buffer_rsrc_t Dw = make_rsrc(t.dP + (size_t)it.slot * n * n, n * n * 8);
    const float sigf = (float)*t.sigma;
    float2 a[R];

    // ---- phase A: support columns, IFFT along ky, to the scratch slot
    // HALF form: sigma P S of rows 0 .. n/2 - 1 of every support column is
    // first read row by row (a wave takes two rows of LPR consecutive
    // columns: whole row segments instead of 32-byte pieces of sixteen rows)
    // into the LDS half at the column's ky; thread (c_off, y_off) takes the
    // rows y_off + Q p, those lane q = y_off of a line holds, and the input
    // sign of row ky is par16(ky mod 16).  Rows n/2 .. n - 1 are read by the
    // column's lanes, one round ahead, so that their latency overlaps the
    // previous column's transform (the LDS half already limits the CU to
    // this workgroup, so the registers that takes cost no occupancy).
    float pm = 0.0f;
    constexpr int RH = R / 2;  // values q + Q p with p < RH lie in rows 0 .. n/2 - 1
    const int c_off = tid0 % LPR, y_off = tid0 / LPR;  // y_off < Q
    if constexpr (HALF) {
      const float s0 = sigf / (float)(n * n);
#pragma unroll 1
      for (int rd = 0; rd < ROUNDS; ++rd) {
        const int c = LPR * rd + c_off;
        if (c < t.nd) {
          const int kx = t.kx0 + c;
          const int2 ch = t.chord[kx];
          float2 xs[RH], pv[RH];
#pragma unroll
          for (int p = Z; p < RH; ++p) {
            const int ky = y_off + Q * p;
            const bool in = ky >= ch.x && ky <= ch.y;
            xs[p] = bload2(Sw, in ? (ky * N + kx) * 8 : kOob);
            pv[p] = bload2(Pw, in ? (ky * n + kx) * 8 : kOob);
          }
#pragma unroll
          for (int p = Z; p < RH; ++p) {
            const int ky = y_off + Q * p;
            pm = fmaxf(pm, cabs2(pv[p]));
            lh[big_block<kBigLdsCols>(c, ky)] = cscale(cmul(pv[p], xs[p]), par16(ky & 15) * s0);
          }
        }
      }
      __syncthreads();
    }
    float2 gs[HALF ? R : 1], gp[HALF ? R : 1];
    auto gather_load = [&](int line, int q) {
      const int kx = t.kx0 + line;
      const int2 ch = t.chord[kx];
      const int s0 = (q * N + kx) * 8, p0 = (q * n + kx) * 8;
#pragma unroll
      for (int p = RH; p < R - Z; ++p) {
        const int ky = q + Q * p;
        const bool in = ky >= ch.x && ky <= ch.y;
        gs[p] = bload2(Sw, in ? s0 + p * (Q * 8) * N : kOob);
        gp[p] = bload2(Pw, in ? p0 + p * (Q * 8 * n) : kOob);
      }
    };
    if constexpr (HALF) {
      if (l0 < t.nd) gather_load(l0, q_item);
    }
#pragma unroll 1
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int line = l0 + LPR * rd;
      int q = q_item;  // opaque per round: keeps twiddle reads inside the round
      asm volatile("" : "+v"(q));
      if (line < t.nd) {
        const int kx = t.kx0 + line;
        if constexpr (HALF) {
          // sigma P S on the column: the staged values, and gather_phi's
          // arithmetic on the requested ones (each lane reads its line's LDS
          // values before any lane of the line, in the same wave, writes
          // the line's transform over them)
          const float scale = par16(q) * (sigf / (float)(n * n));
#pragma unroll
          for (int p = 0; p < R; ++p) {
            if (p < Z || p >= R - Z) {
              a[p] = make_float2(0.0f, 0.0f);
            } else if (p < RH) {
              a[p] = lh[big_block<kBigLdsCols>(line, q + Q * p)];
            } else {
              pm = fmaxf(pm, cabs2(gp[p]));
              a[p] = cscale(cmul(gp[p], gs[p]), scale);
            }
          }
          if (rd + 1 < ROUNDS && line + LPR < t.nd) gather_load(line + LPR, q);
          line_dit_f<n, true, 0, Z, Q>(a, q, tw, -1.0f);
        } else if constexpr (FUSED) {
          pm = fmaxf(pm, gather_phi<n, Q, Z>(Sw, Pw, N, kx, t.chord[kx], q,
                                             par16(q) * (sigf / (float)(n * n)), a));
          line_dit_f<n, true, 0, Z, Q>(a, q, tw, -1.0f);
        } else {
          pm = fmaxf(pm, gather_phi<n, Q>(Sw, Pw, N, kx, t.chord[kx], q, sigf / (float)(n * n), a));
          line_dit<n, true, Q>(a, q, tw);
        }
        // rows xc .. xc + R - 1 of support column `line`, four rows at a time
        // (all in the LDS half or all in the slot: R divides n/2)
        if (HALF && xc < n / 2) {
          float4* dst = reinterpret_cast<float4*>(lh);
#pragma unroll
          for (int j = 0; j < R / 4; ++j) {
            const int b = big_block<kBigLdsCols>(line, xc + 4 * j) / 2;
            dst[b] = make_float4(a[4 * j].x, a[4 * j].y, a[4 * j + 1].x, a[4 * j + 1].y);
            dst[b + 1] =
                make_float4(a[4 * j + 2].x, a[4 * j + 2].y, a[4 * j + 3].x, a[4 * j + 3].y);
          }
        } else {
          float4* dst = reinterpret_cast<float4*>(sb);
#pragma unroll
          for (int j = 0; j < R / 4; ++j) {
            const size_t b = (size_t)big_block<n>(line, xc + 4 * j) / 2;
            dst[b] = make_float4(a[4 * j].x, a[4 * j].y, a[4 * j + 1].x, a[4 * j + 1].y);
            dst[b + 1] =
                make_float4(a[4 * j + 2].x, a[4 * j + 2].y, a[4 * j + 3].x, a[4 * j + 3].y);
          }
        }
      }
    }
    pm = wave_max(pm);
    if ((tid & 63) == 0) red_pmax[wave] = pm;
    __syncthreads();

    // ---- phase B: rows, IFFT along kx, modulus, FFT along x
    // (HALF form: a row held in the global slot is requested one round
    // ahead; rows are disjoint between rounds, so the request never reads a
    // value the current round still writes)
    float e_acc = 0.0f, i_acc = 0.0f;
    float2 nx[HALF ? R : 1];
    auto slot_row = [&](int row, int q, float2(&dst)[HALF ? R : 1]) {
#pragma unroll
      for (int p = 0; p < R; ++p) {
        if (p < Z || p >= R - Z) continue;  // outside every support column
        const int c = q + Q * p - t.kx0;
        dst[p] = (c >= 0 && c < t.nd) ? sb[big_block<n>(c, row)] : make_float2(0.0f, 0.0f);
      }
    };
    if constexpr (HALF) {
      if (l0 >= n / 2) slot_row(l0, q_item, nx);
    }
#pragma unroll 1
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int line = l0 + LPR * rd;
      int q = q_item;  // opaque per round: keeps twiddle reads inside the round
      asm volatile("" : "+v"(q));
      const bool in_lds = HALF && line < n / 2;  // uniform over the round
#pragma unroll
      for (int p = 0; p < R; ++p) {
        if (p < Z || p >= R - Z) {  // outside every support column
          a[p] = make_float2(0.0f, 0.0f);
          continue;
        }
        const int c = q + Q * p - t.kx0;
        const bool live = c >= 0 && c < t.nd;
        if (in_lds)
          a[p] = live ? lh[big_block<kBigLdsCols>(c, line)] : make_float2(0.0f, 0.0f);
        else if constexpr (HALF)
          a[p] = nx[p];
        else
          a[p] = live ? sb[big_block<n>(c, line)] : make_float2(0.0f, 0.0f);
      }
      if constexpr (HALF) {
        const int next = line + LPR;
        if (rd + 1 < ROUNDS && next >= n / 2) slot_row(next, q, nx);
      }
      if constexpr (FUSED)
        line_dit_f<n, true, 0, Z, Q>(a, q, tw, 1.0f);  // lane signs par16(q)
      else
        line_dit<n, true, Q>(a, q, tw);
      float iv[R];
#pragma unroll
      for (int v = 0; v < R / 4; ++v) {
        const v4f f = __builtin_amdgcn_raw_buffer_load_b128(Iw, (line * n + xc + 4 * v) * 4, 0, 0);
        iv[4 * v] = f.x;
        iv[4 * v + 1] = f.y;
        iv[4 * v + 2] = f.z;
        iv[4 * v + 3] = f.w;
      }
      if constexpr (FUSED) {
        modulus_row<R>(a, iv, line, xc, e_acc, i_acc, __builtin_popcount(q) & 1);
        line_dif_f<n, false, 0, Q>(a, q, tw, -1.0f);  // lane signs removed
      } else {
        modulus_row<R>(a, iv, line, xc, e_acc, i_acc);
        line_dif<n, false, Q>(a, q, tw);
      }
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if (k < Z || k >= R - Z) continue;  // no support column there
        const int c = q + Q * k - t.kx0;
        if (c >= 0 && c < t.nd) {
          if (in_lds)
            lh[big_block<kBigLdsCols>(c, line)] = a[k];
          else
            sb[big_block<n>(c, line)] = a[k];
        }
      }
    }
    {
      const double e = wave_sum((double)e_acc), s = wave_sum((double)i_acc);
      if ((tid & 63) == 0) {
        red_e[wave] = e;
        red_i[wave] = s;
      }
    }
    __syncthreads();

    // ---- phase A': support columns, FFT along y, update
    float pmax2 = red_pmax[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) pmax2 = fmaxf(pmax2, red_pmax[w]);
    const float smax = __uint_as_float(*t.smax);
    const float ips = pmax2 > 0.0f ? 1.0f / (pmax2 * sigf) : 0.0f;
    const float iss = smax > 0.0f ? 1.0f / (smax * sigf) : 0.0f;
#pragma unroll 1
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int line = l0 + LPR * rd;
      int q = q_item;  // opaque per round: keeps twiddle reads inside the round
      asm volatile("" : "+v"(q));
      if (line < t.nd) {
#pragma unroll
        for (int j = 0; j < R / 4; ++j) {
          float4 f0, f1;
          if (HALF && xc < n / 2) {
            const float4* src = reinterpret_cast<const float4*>(lh);
            const int b = big_block<kBigLdsCols>(line, xc + 4 * j) / 2;
            f0 = src[b];
            f1 = src[b + 1];
          } else {
            const float4* src = reinterpret_cast<const float4*>(sb);
            const size_t b = (size_t)big_block<n>(line, xc + 4 * j) / 2;
            f0 = src[b];
            f1 = src[b + 1];
          }
          a[4 * j] = make_float2(f0.x, f0.y);
          a[4 * j + 1] = make_float2(f0.z, f0.w);
          a[4 * j + 2] = make_float2(f1.x, f1.y);
          a[4 * j + 3] = make_float2(f1.z, f1.w);
        }
        const int kx = t.kx0 + line;
        if constexpr (HALF) {
          // rows n/2 .. n - 1 updated here, column by column; rows 0 .. n/2 - 1
          // go back to the LDS half for the row-segment update below
          line_dif_f<n, false, 0, Q>(a, q, tw, 1.0f);  // lane signs par16(q)
#pragma unroll
          for (int k = Z; k < RH; ++k) lh[big_block<kBigLdsCols>(line, q + Q * k)] = a[k];
          const int2 ch = t.chord[kx];
          const float ls = par16(q);
#pragma unroll
          for (int k = RH; k < R - Z; ++k) {
            const int ky = q + Q * k;
            const bool in = ky >= ch.x && ky <= ch.y;
            const int offS = in ? (ky * N + kx) * 8 : kOob;
            const int offP = in ? (ky * n + kx) * 8 : kOob;
            update_px<false>(a[k], bload2(Sw, offS), bload2(Pw, offP), Sw, Pw, Dw, offS, offP,
                             ls * sigf, ls * ips, ls * iss, pmax2 > 0.0f, t.mode, 0, 1);
          }
        } else if constexpr (FUSED) {
          line_dif_f<n, false, 0, Q>(a, q, tw, 1.0f);  // lane signs par16(q)
          update_column<n, Q, false, false, Z>(a, Sw, Pw, Dw, N, kx, t.chord[kx], q, sigf, pmax2,
                                               smax, t.mode, 0, 1, nullptr, nullptr, par16(q));
        } else {
          line_dif<n, false, Q>(a, q, tw);
          update_column<n, Q>(a, Sw, Pw, Dw, N, kx, t.chord[kx], q, sigf, pmax2, smax, t.mode);
        }
      }
    }
    if constexpr (HALF) {
      // the update of rows 0 .. n/2 - 1 by whole row segments, the pixels each
      // thread staged in phase A (lane sign par16(ky mod 16) of each value)
      __syncthreads();
#pragma unroll 1
      for (int rd = 0; rd < ROUNDS; ++rd) {
        const int c = LPR * rd + c_off;
        if (c < t.nd) {
          const int kx = t.kx0 + c;
          const int2 ch = t.chord[kx];
          float2 xs[RH], pv[RH];
          int offS[RH], offP[RH];
#pragma unroll
          for (int p = Z; p < RH; ++p) {
            const int ky = y_off + Q * p;
            const bool in = ky >= ch.x && ky <= ch.y;
            offS[p] = in ? (ky * N + kx) * 8 : kOob;
            offP[p] = in ? (ky * n + kx) * 8 : kOob;
            xs[p] = bload2(Sw, offS[p]);
            pv[p] = bload2(Pw, offP[p]);
          }
#pragma unroll
          for (int p = Z; p < RH; ++p) {
            const int ky = y_off + Q * p;
            const float ls = par16(ky & 15);
            update_px<false>(lh[big_block<kBigLdsCols>(c, ky)], xs[p], pv[p], Sw, Pw, Dw, offS[p],
                             offP[p], ls * sigf, ls * ips, ls * iss, pmax2 > 0.0f, t.mode, 0, 1);
          }
        }
      }
    }
    if (tid == 0) {
      double e = 0.0, s = 0.0;
      for (int w = 0; w < NW; ++w) {
        e += red_e[w];
        s += red_i[w];
      }
      t.e_part[(size_t)it.iter * t.e_stride + it.led] = e;
      t.i_part[(size_t)it.iter * t.e_stride + it.led] = s;
    }
    __syncthreads();  // the slot and the reduction arrays are reused by the next item
  }
}

// forward model for the same sides: phases A and B, |psi|^2 out
template <int n, int Q = 8>
__global__ __launch_bounds__(kBigThreads) void forward_kernel_big(const TileDev* __restrict__ tiles,
                                                                  const Item* __restrict__ items,
                                                                  int count, float* __restrict__ out,
                                                                  const int64_t* __restrict__ out_off,
                                                                  float2* __restrict__ scratch) {
  constexpr int R = n / Q;
  constexpr int NT = kBigThreads;
  constexpr int LPR = NT / Q;
  constexpr int ROUNDS = n / LPR;
  __shared__ float2 tw[n];
  const int tid0 = threadIdx.x;
  for (int e = tid0; e < n; e += NT) tw[e] = make_float2(kTw<n>.c[e], kTw<n>.s[e]);
  float2* __restrict__ sb = scratch + (size_t)blockIdx.x * n * n;
  __syncthreads();
  for (int ii = blockIdx.x; ii < count; ii += gridDim.x) {
    int tid = tid0;  // opaque per item, as in update_kernel_big
    asm volatile("" : "+v"(tid));
    const int q = lane_log<Q>(tid % Q), l0 = tid / Q;
    const int xc = R * brevq<Q>(q);
    const Item it = items[ii];
    const TileDev t = tiles[it.tile];
    const size_t woff = (size_t)it.wy0 * t.N + it.wx0;
    const __amdgpu_buffer_rsrc_t Sw =
        make_rsrc(t.S + woff, (unsigned)(((size_t)t.N * t.N - woff) * 8));
    const __amdgpu_buffer_rsrc_t Pw = make_rsrc(t.P, n * n * 8);
    float2 a[R];
#pragma unroll 1
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int line = l0 + LPR * rd;
      if (line < t.nd) {
        const int kx = t.kx0 + line;
        gather_phi<n, Q>(Sw, Pw, t.N, kx, t.chord[kx], q, 1.0f / (float)(n * n), a);
        line_dit<n, true, Q>(a, q, tw);
        float4* dst = reinterpret_cast<float4*>(sb + (size_t)line * n + xc);
#pragma unroll
        for (int k = 0; k < R / 2; ++k)
          dst[k] = make_float4(a[2 * k].x, a[2 * k].y, a[2 * k + 1].x, a[2 * k + 1].y);
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int line = l0 + LPR * rd;
      load_rows<n, 0, Q>(sb, t.kx0, t.nd, line, q, a);
      line_dit<n, true, Q>(a, q, tw);
      float4* dst = reinterpret_cast<float4*>(out + out_off[it.tile] + (size_t)it.led * n * n +
                                              (size_t)line * n + xc);
#pragma unroll
      for (int v = 0; v < R / 4; ++v)
        dst[v] = make_float4(cabs2(a[4 * v]), cabs2(a[4 * v + 1]), cabs2(a[4 * v + 2]),
                             cabs2(a[4 * v + 3]));
    }
    __syncthreads();
  }
}

// ============================================== pupil mean of a group
// P <- P + (1/count) sum_m dP[m] on D0, members summed in slot order.
// Block (r, tile): support row ky = kx0 + r (D0 is symmetric under
// transposition, so the column chords are also the row chords); threads run
// along the row, so every access is contiguous.
__global__ __launch_bounds__(64) void pupil_reduce_kernel(const TileDev* __restrict__ tiles,
                                                           const StepTile* __restrict__ steps) {
  const StepTile s = steps[blockIdx.y];
  const TileDev t = tiles[s.tile];
  if ((int)blockIdx.x >= t.nd) return;
  const int n = t.n, nn = n * n;
  const int ky = t.kx0 + blockIdx.x;
  const int2 ch = t.chord[ky];
  for (int kx = ch.x + (int)threadIdx.x; kx <= ch.y; kx += 64) {
    const int px = ky * n + kx;
    float2 acc = t.dP[px];
    int m = 1;
    // four increments requested at a time, summed in slot order
    for (; m + 4 <= s.count; m += 4) {
      const float2 d0 = t.dP[(size_t)m * nn + px], d1 = t.dP[(size_t)(m + 1) * nn + px];
      const float2 d2 = t.dP[(size_t)(m + 2) * nn + px], d3 = t.dP[(size_t)(m + 3) * nn + px];
      acc = cadd(cadd(cadd(cadd(acc, d0), d1), d2), d3);
    }
    for (; m < s.count; ++m) acc = cadd(acc, t.dP[(size_t)m * nn + px]);
    t.P[px] = pupil_mean_step(t.P[px], acc, s.count);
  }
}

// ============================================ end of an iteration (FP64)
// residual = sum_j e_j / sum_j I_j (LEDs in grid order); with pupil
// recovery: s = sqrt(|D0| / sum_D0 |P|^2), P <- s P, sigma <- sigma / s.
// Also clears the running spectrum maximum for the next iteration.
__global__ __launch_bounds__(kIterEndThreads) void iter_end_kernel(const TileDev* __restrict__ tiles,
                                                                   const int* __restrict__ ids,
                                                                   int iter) {
  const TileDev t = tiles[ids[blockIdx.x]];
  const int pupil_update = t.mode != 0;
  const int tid = threadIdx.x;
  __shared__ double r0[kIterEndThreads], r1[256];
  __shared__ double s_scale;
  // residual: the first 256 threads sum the per-LED partials
  if (tid < 256) {
    double e = 0.0, s = 0.0;
    const size_t e0 = (size_t)iter * t.e_stride;
    for (int j = tid; j < t.L; j += 256) {
      e += t.e_part[e0 + j];
      s += t.i_part[e0 + j];
    }
    r0[tid] = e;
    r1[tid] = s;
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      r0[tid] += r0[tid + o];
      r1[tid] += r1[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) t.residual[iter] = r1[0] > 0.0 ? r0[0] / r1[0] : 0.0;
  __syncthreads();
  if (pupil_update) {
    // thread (kx, y0) takes column kx, rows y0, y0 + per, ... (one chord
    // lookup per thread)
    const int n = t.n, per = kIterEndThreads / n;
    const int kx = tid % n, y0 = tid / n;
    double E = 0.0;
    if (y0 < per) {
      const int2 ch = t.chord[kx];
      for (int ky = y0; ky < n; ky += per) {
        if (ky >= ch.x && ky <= ch.y) {
          const float2 p = t.P[ky * n + kx];
          E += (double)p.x * (double)p.x + (double)p.y * (double)p.y;
        }
      }
    }
    r0[tid] = E;
    __syncthreads();
    for (int o = kIterEndThreads / 2; o > 0; o >>= 1) {
      if (tid < o) r0[tid] += r0[tid + o];
      __syncthreads();
    }
    if (tid == 0) {
      const double sc = r0[0] > 0.0 ? sqrt((double)t.nd0 / r0[0]) : 1.0;
      s_scale = sc;
      *t.sigma = *t.sigma / sc;
    }
    __syncthreads();
    const float sc = (float)s_scale;
    if (y0 < per)
      for (int ky = y0; ky < n; ky += per) t.P[ky * n + kx] = cscale(t.P[ky * n + kx], sc);
  }
  if (tid == 0) *t.smax = 0u;
}

// max |S_stored|^2 over the whole spectrum (order-free: max of non-negative
// floats via their bit patterns)
__global__ __launch_bounds__(256) void smax_kernel(const TileDev* __restrict__ tiles,
                                                   const int* __restrict__ ids) {
  const TileDev t = tiles[ids[blockIdx.y]];
  // two complex values per 16-byte load (S is 256-byte aligned)
  const size_t NN2 = (size_t)t.N * t.N / 2;
  const float4* S4 = reinterpret_cast<const float4*>(t.S);
  float m = 0.0f;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < NN2; i += (size_t)gridDim.x * 256) {
    const float4 v = S4[i];
    m = fmaxf(m, fmaxf(fmaf(v.x, v.x, v.y * v.y), fmaf(v.z, v.z, v.w * v.w)));
  }
  if ((t.N & 1) && blockIdx.x == 0 && threadIdx.x == 0)  // odd N: the last value
    m = fmaxf(m, cabs2(t.S[(size_t)t.N * t.N - 1]));
  m = wave_max(m);
  __shared__ float wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float v = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
    atomicMax(t.smax, __float_as_uint(v));
  }
}

// initial state: S = 0 except the centred window <- (-1)^(x+y) sqrt(I_j0) (its
// 2-D FFT follows as line FFTs), P = P_init, sigma = 1, smax = 0
__global__ __launch_bounds__(256) void init_state_kernel(const TileDev* __restrict__ tiles,
                                                         const int* __restrict__ ids) {
  const TileDev t = tiles[ids[blockIdx.y]];
  const size_t NN = (size_t)t.N * t.N;
  const int n = t.n;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < NN; i += (size_t)gridDim.x * 256) {
    const int r = (int)(i / t.N), c = (int)(i % t.N);
    const int u = r - t.wy0_j0, v = c - t.wx0_j0;
    float2 val = make_float2(0.0f, 0.0f);
    if (u >= 0 && u < n && v >= 0 && v < n) {
      const float I = t.I[(size_t)t.j0 * n * n + (size_t)u * n + v];
      const float m = sqrtf(fmaxf(I, 0.0f));
      val = make_float2(((u + v) & 1) ? -m : m, 0.0f);
    }
    t.S[i] = val;
  }
  if (blockIdx.x == 0) {
    for (int px = threadIdx.x; px < n * n; px += 256) t.P[px] = t.P0[px];
    if (threadIdx.x == 0) {
      *t.sigma = 1.0;
      *t.smax = 0u;
    }
  }
}

// ======================================================= line FFTs
// One workgroup per line: load into LDS, Stockham passes of radix 4/2/3/5,
// store with an optional scale and (-1)^(line+elem) modulation.
namespace {
__device__ __forceinline__ void dft3(float2& a0, float2& a1, float2& a2, bool inv) {
  const float s = inv ? 0.86602540378443864676f : -0.86602540378443864676f;
  const float2 t1 = cadd(a1, a2), t2 = csub(a1, a2);
  const float2 m1 = make_float2(fmaf(-0.5f, t1.x, a0.x), fmaf(-0.5f, t1.y, a0.y));
  const float2 m2 = make_float2(-s * t2.y, s * t2.x);
  a0 = cadd(a0, t1);
  a1 = cadd(m1, m2);
  a2 = csub(m1, m2);
}
__device__ __forceinline__ void dft5(float2 (&v)[5], bool inv) {
  float2 o[5];
  for (int k = 0; k < 5; ++k) {
    float2 acc = v[0];
    for (int j = 1; j < 5; ++j) {
      const int e = (j * k) % 5;
      const float c = kTw<5>.c[e], s = inv ? kTw<5>.s[e] : -kTw<5>.s[e];
      acc = cadd(acc, make_float2(fmaf(v[j].x, c, -(v[j].y * s)), fmaf(v[j].x, s, v[j].y * c)));
    }
    o[k] = acc;
  }
  for (int k = 0; k < 5; ++k) v[k] = o[k];
}
}  // namespace

// C lines of one job per workgroup (256 / C threads per line): the lines'
// elements are loaded and stored with the line index fastest where lines are
// closer in memory than elements (column passes: runs of C adjacent values
// per row instead of one value per row), element index fastest otherwise.
__global__ __launch_bounds__(256) void line_fft_kernel(const LineJob* __restrict__ jobs, int len,
                                                       int inverse, int C) {
  const LineJob job = jobs[blockIdx.y];
  const int line0 = blockIdx.x * C;
  if (line0 >= job.nlines) return;  // the whole workgroup
  extern __shared__ float2 lbuf[];
  float2* x = lbuf;
  float2* y = lbuf + C * len;
  float2* w = lbuf + 2 * C * len;  // w[e] = W_len^e, in FP64 and rounded once
  const float sgn = inverse ? 1.0f : -1.0f;
  const bool line_fast = job.line_stride < job.elem_stride;
  for (int i = threadIdx.x; i < len; i += 256) {
    double s, c;
    sincospi((double)sgn * 2.0 * (double)i / (double)len, &s, &c);
    w[i] = make_float2((float)c, (float)s);
  }
  for (int idx = threadIdx.x; idx < C * len; idx += 256) {
    const int c = line_fast ? idx % C : idx / len, i = line_fast ? idx / C : idx % len;
    if (line0 + c < job.nlines)
      x[c * len + i] = job.base[(size_t)(line0 + c) * job.line_stride + (size_t)i * job.elem_stride];
  }
  __syncthreads();
  const int tpl = 256 / C, lc = threadIdx.x / tpl, lt = threadIdx.x % tpl;
  int ns = 1;
  int rem = len;
  while (rem > 1) {
    int r = (rem % 4 == 0) ? 4 : (rem % 2 == 0) ? 2 : (rem % 3 == 0) ? 3 : 5;
    const int m = len / r;
    const int wstep = len / (ns * r);  // W_{ns r}^{k q} = W_len^{k q wstep}
    const float2* xl = x + lc * len;
    float2* yl = y + lc * len;
    for (int j = lt; j < m; j += tpl) {
      const int k = j % ns;
      float2 v[5];
      for (int q = 0; q < r; ++q) {
        float2 e = xl[j + q * m];
        if (q > 0 && k > 0) e = cmul(e, w[k * q * wstep]);
        v[q] = e;
      }
      if (r == 2) {
        const float2 t0 = v[0];
        v[0] = cadd(t0, v[1]);
        v[1] = csub(t0, v[1]);
      } else if (r == 4) {
        const float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        const float2 b0 = cadd(v[1], v[3]), b1d = csub(v[1], v[3]);
        const float2 b1 = inverse ? make_float2(-b1d.y, b1d.x) : make_float2(b1d.y, -b1d.x);
        v[0] = cadd(a0, b0);
        v[2] = csub(a0, b0);
        v[1] = cadd(a1, b1);
        v[3] = csub(a1, b1);
      } else if (r == 3) {
        dft3(v[0], v[1], v[2], inverse);
      } else {
        dft5(v, inverse);
      }
      const int d = (j / ns) * ns * r + k;
      for (int q = 0; q < r; ++q) yl[d + q * ns] = v[q];
    }
    __syncthreads();
    float2* tmp = x;
    x = y;
    y = tmp;
    ns *= r;
    rem /= r;
  }
  for (int idx = threadIdx.x; idx < C * len; idx += 256) {
    const int c = line_fast ? idx % C : idx / len, i = line_fast ? idx / C : idx % len;
    const int line = line0 + c;
    if (line < job.nlines) {
      float2 v = cscale(x[c * len + i], job.scale);
      if (job.modulate && ((line + i) & 1)) v = make_float2(-v.x, -v.y);
      job.base[(size_t)line * job.line_stride + (size_t)i * job.elem_stride] = v;
    }
  }
}

// dst[off[t] + i] = sigma * S * up^2 / N^2   (object finalise, before the
// inverse line FFTs)
__global__ __launch_bounds__(256) void scale_spectrum_kernel(const TileDev* __restrict__ tiles,
                                                             float2* __restrict__ dst,
                                                             const int64_t* __restrict__ off) {
  const TileDev t = tiles[blockIdx.y];
  float2* out = dst + off[blockIdx.y];
  const size_t NN = (size_t)t.N * t.N;
  const float sc = (float)(*t.sigma * (double)t.up * (double)t.up / (double)NN);
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < NN; i += (size_t)gridDim.x * 256)
    out[i] = cscale(t.S[i], sc);
}

// which = 1: pupil, 2: initial pupil (complex64 [n][n]); 3: residual (double)
__global__ __launch_bounds__(256) void gather_kernel(const TileDev* __restrict__ tiles,
                                                     void* __restrict__ dst,
                                                     const int64_t* __restrict__ off, int which) {
  const TileDev t = tiles[blockIdx.y];
  if (which == 3) {
    double* out = (double*)dst + off[blockIdx.y];
    for (int i = blockIdx.x * 256 + threadIdx.x; i < t.iters; i += gridDim.x * 256)
      out[i] = t.residual[i];
    return;
  }
  float2* out = (float2*)dst + off[blockIdx.y];
  const float2* src = which == 1 ? t.P : t.P0;
  const int nn = t.n * t.n;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nn; i += gridDim.x * 256) out[i] = src[i];
}

// S = (-1)^(x+y) * object / up^2 into the tile's spectrum buffer
__global__ __launch_bounds__(256) void obj_mod_kernel(const TileDev* __restrict__ tiles,
                                                      const float2* __restrict__ src,
                                                      const int64_t* __restrict__ src_off) {
  const TileDev t = tiles[blockIdx.y];
  const int N = t.N;
  const size_t NN = (size_t)N * N;
  const float2* s = src + src_off[blockIdx.y];
  const float sc = 1.0f / (float)(t.up * t.up);
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < NN; i += (size_t)gridDim.x * 256) {
    const int r = (int)(i / N), c = (int)(i % N);
    t.S[i] = cscale(s[i], ((r + c) & 1) ? -sc : sc);
  }
}

// one LED's images of every tile into the stacks: block t copies tile t's
// n^2 floats from src + src_off[t] to stack + i_off[t] + led n^2
__global__ __launch_bounds__(256) void online_scatter_kernel(const TileDev* __restrict__ table,
                                                             const float* __restrict__ src,
                                                             const int64_t* __restrict__ src_off,
                                                             float* __restrict__ stack,
                                                             const int64_t* __restrict__ i_off,
                                                             int led) {
  const int t = blockIdx.x;
  const int nn = table[t].n * table[t].n;
  const float* s = src + src_off[t];
  float* d = stack + i_off[t] + (size_t)led * nn;
  for (int i = threadIdx.x; i < nn; i += 256) d[i] = s[i];
}

__global__ void set_j0_kernel(TileDev* __restrict__ table, int count, int j0) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) table[t].j0 = j0;
}

__global__ void set_intensity_kernel(TileDev* __restrict__ table, int count,
                                     const float* __restrict__ base,
                                     const int64_t* __restrict__ i_off) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) table[t].I = base + i_off[t];
}

// ============================================ device-mode status checks
// Status word of a device-mode call: bit 0 a negative or non-finite
// intensity, bit 1 a residual that is not finite.  Cleared by a kernel (no
// memset node), set with atomic OR, read by the host later.
__global__ void status_clear_kernel(int* __restrict__ status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *status = 0;
}
__global__ __launch_bounds__(256) void validate_intensity_kernel(const float* __restrict__ I,
                                                                 int64_t count,
                                                                 int* __restrict__ status) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * 256 * 4;
  for (int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4; i < count; i += stride) {
    if (i + 4 <= count) {
      const float4 v = *reinterpret_cast<const float4*>(I + i);
      // v >= 0 is false for NaN; v <= FLT_MAX is false for +Inf
      bad |= !(v.x >= 0.0f && v.x <= 3.402823466e38f) || !(v.y >= 0.0f && v.y <= 3.402823466e38f) ||
             !(v.z >= 0.0f && v.z <= 3.402823466e38f) || !(v.w >= 0.0f && v.w <= 3.402823466e38f);
    } else {
      for (int64_t k = i; k < count; ++k) bad |= !(I[k] >= 0.0f && I[k] <= 3.402823466e38f);
    }
  }
  if (__builtin_amdgcn_ballot_w64(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(status, 1);
}
// one thread per tile: every residual of its history
__global__ void check_residuals_kernel(const TileDev* __restrict__ tiles, int count,
                                       int* __restrict__ status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const TileDev d = tiles[t];
  bool bad = false;
  for (int k = 0; k < d.iters; ++k) {
    const double r = d.residual[k];
    bad |= !(r == r) || r > 1.79e308 || r < -1.79e308;
  }
  if (bad) atomicOr(status, 2);
}
// dst <- src (bytes, 16-byte aligned both) unless the status word is set
__global__ __launch_bounds__(256) void copy_if_ok_kernel(void* __restrict__ dst,
                                                         const void* __restrict__ src,
                                                         int64_t bytes,
                                                         const int* __restrict__ status) {
  if (*status != 0) return;
  const int64_t n16 = bytes / 16;
  const float4* s4 = reinterpret_cast<const float4*>(src);
  float4* d4 = reinterpret_cast<float4*>(dst);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * 256)
    d4[i] = s4[i];
  const unsigned char* sb = reinterpret_cast<const unsigned char*>(src);
  unsigned char* db = reinterpret_cast<unsigned char*>(dst);
  if (blockIdx.x == 0)
    for (int64_t i = n16 * 16 + threadIdx.x; i < bytes; i += 256) db[i] = sb[i];
}

// ========================================================== launchers
namespace {
template <int n, int PAD = 16>
size_t update_lds(int nd_max) {
  return (size_t)nd_max * pitch<n, PAD>() * sizeof(float2);
}
template <int n, int PAD, int Q>
hipError_t launch_update_np(const TileDev* tiles, const Item* items, int count, int nd_max,
                            const int2* ranges, int nranges, hipStream_t st) {
  const size_t lds = update_lds<n, PAD>(nd_max);
  if (ranges) {
    hipLaunchKernelGGL((update_kernel<n, PAD, Q, true>), dim3(nranges), dim3(n * Q), lds, st,
                       tiles, items, ranges, nranges);
  } else {
    hipLaunchKernelGGL((update_kernel<n, PAD, Q, false>), dim3(xcd_grid(count)), dim3(n * Q), lds,
                       st, tiles, items, nullptr, count);
  }
  return hipGetLastError();
}
template <int n, int PAD, int Q, int ROUNDS, int Z>
hipError_t launch_update_rounds_z(const TileDev* tiles, const Item* items, int count, size_t lds,
                                  const int2* ranges, int nranges, hipStream_t st) {
  if (ranges) {
    hipLaunchKernelGGL((update_kernel_rounds<n, PAD, Q, ROUNDS, true, Z>), dim3(nranges),
                       dim3(n * Q / ROUNDS), lds, st, tiles, items, ranges, nranges);
  } else {
    hipLaunchKernelGGL((update_kernel_rounds<n, PAD, Q, ROUNDS, false, Z>), dim3(xcd_grid(count)),
                       dim3(n * Q / ROUNDS), lds, st, tiles, items, nullptr, count);
  }
  return hipGetLastError();
}
// Values a lane may skip at each end of a line (kernel template Z): the
// support D0 is the disc centred at n/2, so every tile of the launch has its
// support columns and rows within n/2 - R .. n/2 + R, R = nd_max / 2 (at
// least half the widest support), and Z Q <= n/2 - R - 1 keeps both ends clear.
template <int n, int Q>
constexpr int prune_limit() {
  return Q == 8 ? (n / Q >= 16 ? 3 : (n / Q >= 12 ? 2 : 1)) : 0;
}
inline int prune_count(int n, int Q, int nd_max) {
  const int lim = n / 2 - nd_max / 2 - 1;
  return lim > 0 ? lim / Q : 0;
}
template <int n, int PAD, int Q, int ROUNDS>
hipError_t launch_update_rounds(const TileDev* tiles, const Item* items, int count, int nd_max,
                                const int2* ranges, int nranges, hipStream_t st) {
  // rows: the support columns, and at least n/2 for the twiddle column
  const size_t lds = update_lds<n, PAD>(nd_max > n / 2 ? nd_max : n / 2);
  constexpr int zl = prune_limit<n, Q>();
  const int z = Q == 8 ? std::min(zl, prune_count(n, Q, nd_max)) : 0;
  if constexpr (zl >= 3)
    if (z >= 3)
      return launch_update_rounds_z<n, PAD, Q, ROUNDS, 3>(tiles, items, count, lds, ranges,
                                                         nranges, st);
  if constexpr (zl >= 2)
    if (z >= 2)
      return launch_update_rounds_z<n, PAD, Q, ROUNDS, 2>(tiles, items, count, lds, ranges,
                                                         nranges, st);
  if constexpr (zl >= 1)
    if (z >= 1)
      return launch_update_rounds_z<n, PAD, Q, ROUNDS, 1>(tiles, items, count, lds, ranges,
                                                         nranges, st);
  return launch_update_rounds_z<n, PAD, Q, ROUNDS, 0>(tiles, items, count, lds, ranges, nranges,
                                                     st);
}
template <int n>
hipError_t launch_update_n(const TileDev* tiles, const Item* items, int count, int nd_max,
                           int variant, const int2* ranges, int nranges, hipStream_t st) {
  switch (variant) {
    case 0: return launch_update_np<n, 16, 4>(tiles, items, count, nd_max, ranges, nranges, st);
    case 1: return launch_update_np<n, 1, 4>(tiles, items, count, nd_max, ranges, nranges, st);
    case 2: return launch_update_np<n, 8, 4>(tiles, items, count, nd_max, ranges, nranges, st);
    case 3: return launch_update_np<n, 32, 4>(tiles, items, count, nd_max, ranges, nranges, st);
    case 4: return launch_update_np<n, 1, 8>(tiles, items, count, nd_max, ranges, nranges, st);
    case 5: return launch_update_np<n, 16, 8>(tiles, items, count, nd_max, ranges, nranges, st);
    case 6:
      return launch_update_rounds<n, 1, 8, 2>(tiles, items, count, nd_max, ranges, nranges, st);
    case 7:
      return launch_update_rounds<n, 1, 8, 4>(tiles, items, count, nd_max, ranges, nranges, st);
    case 8:
      return launch_update_rounds<n, 1, 4, 2>(tiles, items, count, nd_max, ranges, nranges, st);
    default: return hipErrorInvalidValue;
  }
}
template <int n>
hipError_t launch_forward_n(const TileDev* tiles, const Item* items, int count, float* out,
                            const int64_t* off, int nd_max, hipStream_t st) {
  const size_t lds = update_lds<n>(nd_max);
  hipLaunchKernelGGL(forward_kernel<n>, dim3(count), dim3(n * kQ), lds, st, tiles, items, out,
                     off);
  return hipGetLastError();
}
// the LDS limit of every round-form instantiation Z = 0 .. ZMAX
template <int n, int Q, int ROUNDS, int ZMAX>
void set_rounds_attr(int big) {
  (void)hipFuncSetAttribute((const void*)update_kernel_rounds<n, 1, Q, ROUNDS, false, ZMAX>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel_rounds<n, 1, Q, ROUNDS, true, ZMAX>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  if constexpr (ZMAX > 0) set_rounds_attr<n, Q, ROUNDS, ZMAX - 1>(big);
}
template <int n>
void set_lds_limit_n(int big) {
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 16, 4, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 16, 4, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 1, 4, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 1, 4, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 8, 4, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 8, 4, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 32, 4, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 32, 4, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 1, 8, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 1, 8, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 16, 8, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  (void)hipFuncSetAttribute((const void*)update_kernel<n, 16, 8, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
  set_rounds_attr<n, 8, 2, prune_limit<n, 8>()>(big);
  set_rounds_attr<n, 8, 4, prune_limit<n, 8>()>(big);
  set_rounds_attr<n, 4, 2, 0>(big);
  (void)hipFuncSetAttribute((const void*)forward_kernel<n>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, big);
}
bool g_attr_done = false;
void set_lds_limits() {
  if (g_attr_done) return;
  g_attr_done = true;
  const int big = 160 * 1024 - 4096;
  set_lds_limit_n<64>(big);
  set_lds_limit_n<96>(big);
  set_lds_limit_n<128>(big);
  (void)hipGetLastError();
}
}  // namespace

hipError_t launch_update(int n, const TileDev* tiles, const Item* items, int count, int nd_max,
                         int variant, float2* big_scratch, hipStream_t st, const int2* ranges,
                         int nranges) {
  if (count <= 0) return hipSuccess;
  set_lds_limits();
  if (n == 256) {
    if (!big_scratch) return hipErrorInvalidValue;
    // 16 lanes per line (R = 16: no spills); variant 1: 8 lanes (R = 32)
    const int grid = xcd_grid(count) < kBigSlots ? xcd_grid(count) : kBigSlots;
    static_assert(kBigSlots % kXcds == 0, "whole XCD blocks of slots");
    // variant 1: 8 lanes per line (R = 32); 2: 16 lanes, unfused cross-lane
    // steps; otherwise 16 lanes with the fused steps and support pruning
    // (the same bits as variant 2 up to the sign of exact zeros)
    if (variant == 1) {
      hipLaunchKernelGGL((update_kernel_big<256, 8>), dim3(grid), dim3(kBigThreads), 0, st, tiles,
                         items, count, big_scratch);
    } else if (variant == 2) {
      hipLaunchKernelGGL((update_kernel_big<256, 16>), dim3(grid), dim3(kBigThreads), 0, st, tiles,
                         items, count, big_scratch);
    } else {
      const int z = std::min(3, prune_count(256, 16, nd_max));
      if (z >= 3 && nd_max <= kBigLdsCols)
        hipLaunchKernelGGL((update_kernel_big<256, 16, true, 3, true>), dim3(grid),
                           dim3(kBigThreads), 0, st, tiles, items, count, big_scratch);
      else if (z >= 3)
        hipLaunchKernelGGL((update_kernel_big<256, 16, true, 3>), dim3(grid), dim3(kBigThreads), 0,
                           st, tiles, items, count, big_scratch);
      else if (z == 2)
        hipLaunchKernelGGL((update_kernel_big<256, 16, true, 2>), dim3(grid), dim3(kBigThreads), 0,
                           st, tiles, items, count, big_scratch);
      else if (z == 1)
        hipLaunchKernelGGL((update_kernel_big<256, 16, true, 1>), dim3(grid), dim3(kBigThreads), 0,
                           st, tiles, items, count, big_scratch);
      else
        hipLaunchKernelGGL((update_kernel_big<256, 16, true, 0>), dim3(grid), dim3(kBigThreads), 0,
                           st, tiles, items, count, big_scratch);
    }
    return hipGetLastError();
  }
  switch (n) {
    case 64: return launch_update_n<64>(tiles, items, count, nd_max, variant, ranges, nranges, st);
    case 96: return launch_update_n<96>(tiles, items, count, nd_max, variant, ranges, nranges, st);
    case 128:
      return launch_update_n<128>(tiles, items, count, nd_max, variant, ranges, nranges, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_forward_leds(int n, const TileDev* tiles, const Item* items, int count,
                               float* out, const int64_t* out_off, int nd_max,
                               float2* big_scratch, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  set_lds_limits();
  if (n == 256) {
    if (!big_scratch) return hipErrorInvalidValue;
    const int grid = count < kBigSlots ? count : kBigSlots;
    hipLaunchKernelGGL(forward_kernel_big<256>, dim3(grid), dim3(kBigThreads), 0, st, tiles, items,
                       count, out, out_off, big_scratch);
    return hipGetLastError();
  }
  switch (n) {
    case 64: return launch_forward_n<64>(tiles, items, count, out, out_off, nd_max, st);
    case 96: return launch_forward_n<96>(tiles, items, count, out, out_off, nd_max, st);
    case 128: return launch_forward_n<128>(tiles, items, count, out, out_off, nd_max, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pupil_reduce(const TileDev* tiles, const StepTile* steps, int count, int rows,
                               hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(pupil_reduce_kernel, dim3(rows, count), dim3(64), 0, st, tiles, steps);
  return hipGetLastError();
}

hipError_t launch_iter_end(const TileDev* tiles, const int* ids, int count, int iter,
                           hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(iter_end_kernel, dim3(count), dim3(kIterEndThreads), 0, st, tiles, ids, iter);
  return hipGetLastError();
}

hipError_t launch_smax(const TileDev* tiles, const int* ids, int count, int NN_max,
                       hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int chunks = (NN_max / 2 + 256 * 16 - 1) / (256 * 16);
  hipLaunchKernelGGL(smax_kernel, dim3(chunks, count), dim3(256), 0, st, tiles, ids);
  return hipGetLastError();
}

hipError_t launch_init_state(const TileDev* tiles, const int* ids, int count, int /*n*/,
                             int N_max, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int chunks = ((size_t)N_max * N_max + 256 * 16 - 1) / (256 * 16);
  hipLaunchKernelGGL(init_state_kernel, dim3(chunks, count), dim3(256), 0, st, tiles, ids);
  return hipGetLastError();
}

hipError_t launch_line_fft(const LineJob* jobs, int njobs, int len, int max_lines, int inverse,
                           hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  // lines per workgroup: the largest power of two (at most 8) with C len <= 2048
  int C = 1;
  while (C < 8 && 2 * C * len <= 2048) C *= 2;
  const size_t lds = (size_t)(2 * C + 1) * len * sizeof(float2);
  hipLaunchKernelGGL(line_fft_kernel, dim3((max_lines + C - 1) / C, njobs), dim3(256), lds, st,
                     jobs, len, inverse, C);
  return hipGetLastError();
}

hipError_t launch_scale_spectrum(const TileDev* tiles, int count, float2* dst, const int64_t* off,
                                 int N_max, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int chunks = (int)(((size_t)N_max * N_max + 256 * 16 - 1) / (256 * 16));
  hipLaunchKernelGGL(scale_spectrum_kernel, dim3(chunks, count), dim3(256), 0, st, tiles, dst, off);
  return hipGetLastError();
}

hipError_t launch_gather(const TileDev* tiles, int count, void* dst, const int64_t* off, int which,
                         int n_max, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int chunks = which == 3 ? 1 : (n_max * n_max + 255) / 256;
  hipLaunchKernelGGL(gather_kernel, dim3(chunks, count), dim3(256), 0, st, tiles, dst, off, which);
  return hipGetLastError();
}

hipError_t launch_object_to_spectrum(const TileDev* tiles, int count, const float2* src_base,
                                     const int64_t* src_off, int N_max, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int chunks = (int)(((size_t)N_max * N_max + 256 * 16 - 1) / (256 * 16));
  hipLaunchKernelGGL(obj_mod_kernel, dim3(chunks, count), dim3(256), 0, st, tiles, src_base, src_off);
  return hipGetLastError();
}

hipError_t launch_online_scatter(const TileDev* table, int count, const float* src,
                                 const int64_t* src_off, float* stack, const int64_t* i_off,
                                 int led, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(online_scatter_kernel, dim3(count), dim3(256), 0, st, table, src, src_off,
                     stack, i_off, led);
  return hipGetLastError();
}

hipError_t launch_set_j0(TileDev* table, int count, int j0, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(set_j0_kernel, dim3((count + 255) / 256), dim3(256), 0, st, table, count, j0);
  return hipGetLastError();
}

hipError_t launch_set_intensity(TileDev* table, int count, const float* base, const int64_t* i_off,
                                hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(set_intensity_kernel, dim3((count + 255) / 256), dim3(256), 0, st, table, count,
                     base, i_off);
  return hipGetLastError();
}

hipError_t launch_status_clear(int* status, hipStream_t st) {
  hipLaunchKernelGGL(status_clear_kernel, dim3(1), dim3(64), 0, st, status);
  return hipGetLastError();
}
hipError_t launch_validate_intensity(const float* I, int64_t count, int* status, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + 1023) / 1024, 2048);
  hipLaunchKernelGGL(validate_intensity_kernel, dim3((unsigned)blocks), dim3(256), 0, st, I, count,
                     status);
  return hipGetLastError();
}
hipError_t launch_check_residuals(const TileDev* tiles, int count, int* status, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_residuals_kernel, dim3((count + 255) / 256), dim3(256), 0, st, tiles,
                     count, status);
  return hipGetLastError();
}
hipError_t launch_copy_if_ok(void* dst, const void* src, int64_t bytes, const int* status,
                             hipStream_t st) {
  if (bytes <= 0) return hipSuccess;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((bytes / 16 + 255) / 256, 4096));
  hipLaunchKernelGGL(copy_if_ok_kernel, dim3((unsigned)blocks), dim3(256), 0, st, dst, src, bytes,
                     status);
  return hipGetLastError();
}

}  // namespace fpm

// Device-side building blocks for gfx950: MFMA wrappers, activation
// difference streams, level sets, cut-cell clipping and problem data.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "nbm_internal.hpp"

namespace nbm {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// Streaming (non-temporal) accesses for data that crosses HBM exactly once
// between two kernels: the weight-gradient operands, written by the forward/
// backward pass and read once by the contraction, and the per-work-group
// weight-gradient partial rows, read once by the reduction.  They bypass the cache
// retention the rest of the working set (weights, tables, centres) relies on.
__device__ __forceinline__ void st_stream(bf4* p, bf4 v) {
  __builtin_nontemporal_store(__builtin_bit_cast(u2, v), (u2*)p);
}
__device__ __forceinline__ void st_stream(float* p, f4 v) { __builtin_nontemporal_store(v, (f4*)p); }
__device__ __forceinline__ void st_stream(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ bf4 ld_stream(const bf4* p) {
  return __builtin_bit_cast(bf4, __builtin_nontemporal_load((const u2*)p));
}
__device__ __forceinline__ f4 ld_stream(const float* p) { return __builtin_nontemporal_load((const f4*)p); }
__device__ __forceinline__ u4 ld_stream(const u4* p) { return __builtin_nontemporal_load(p); }

// v_mfma_f32_16x16x4f32: lane l supplies A[l%16][k], B[k][l%16] with k = l/16;
// result lane l holds C[4*(l/16)+r][l%16], r = 0..3.
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// v_mfma_f32_16x16x32_bf16: lane l supplies 8 consecutive K values of row
// (A) / column (B) l%16 for K group l/16; result layout as above.
__device__ __forceinline__ f4 mfma32(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Wave priority around matrix-core clusters.  Two work-groups share each
// SIMD and run the same sequence; with equal priority they enter their MFMA
// and VALU phases in step.  The wave issuing its MFMA block at raised
// priority keeps the matrix core, the other falls into its VALU phase, and
// the two units overlap instead of alternating.
__device__ __forceinline__ void mfma_phase_begin() { __builtin_amdgcn_s_setprio(1); }
__device__ __forceinline__ void mfma_phase_end() { __builtin_amdgcn_s_setprio(0); }

// Sum over the 16 lanes of a DPP row (lanes 16k .. 16k+15) by row rotations
// (row_ror 8, 4, 2, 1): one VALU add per step, no LDS traffic; lane 16k holds
// the row sum in a fixed order.
template <int CTRL>
__device__ __forceinline__ float row_rotate(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_sum(float v) {
  v += row_rotate<0x128>(v);   // row_ror:8
  v += row_rotate<0x124>(v);   // row_ror:4
  v += row_rotate<0x122>(v);   // row_ror:2
  v += row_rotate<0x121>(v);   // row_ror:1
  return v;
}

template <int PREC> struct Op;
template <> struct Op<0> { typedef float T; static constexpr int bytes = 4; };
template <> struct Op<1> { typedef __bf16 T; static constexpr int bytes = 2; };

__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(__bf16 x) { return (float)x; }
template <class T> __device__ __forceinline__ T from_f(float x);
template <> __device__ __forceinline__ float from_f<float>(float x) { return x; }
template <> __device__ __forceinline__ __bf16 from_f<__bf16>(float x) { return (__bf16)x; }

// ---------------------------------------------------------------------------
// Activation difference streams.
// A point and its 2d stencil neighbours are propagated as a base stream
// a = s(z) and, per axis, D = s(z+p) - s(z) and E = s(z+p) - 2 s(z) + s(z-m),
// where p and e are the pre-activation differences and m = p - e.  This is an
// exact rewriting of evaluating the network at x and x +- h e_i; the forms
// below avoid the cancellation of forming those differences from point values
// (sum-to-product identities for sin, addition theorems for tanh).
//
// The difference arguments are O(h), so their sin / cos / tanh are evaluated
// by truncated Taylor series where the argument is small (truncation error
// below FP32 rounding) and by the general library function otherwise.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// sin x = x (1 - x^2/3! + x^4/5! - x^6/7! + x^8/9!), |x| <= pi/4: next term
// x^11/11! < 2e-9
__device__ __forceinline__ float sin_taylor(float x) {
  float y = x * x;
  float p = 1.0f / 362880.0f;
  p = fmaf(p, y, -1.0f / 5040.0f);
  p = fmaf(p, y, 1.0f / 120.0f);
  p = fmaf(p, y, -1.0f / 6.0f);
  p = fmaf(p, y, 1.0f);
  return x * p;
}
// cos x = 1 - x^2/2! + ... - x^10/10!, |x| <= pi/4: next term < 2e-10
__device__ __forceinline__ float cos_taylor(float x) {
  float y = x * x;
  float p = -1.0f / 3628800.0f;
  p = fmaf(p, y, 1.0f / 40320.0f);
  p = fmaf(p, y, -1.0f / 720.0f);
  p = fmaf(p, y, 1.0f / 24.0f);
  p = fmaf(p, y, -0.5f);
  return fmaf(p, y, 1.0f);
}
// tanh x = x - x^3/3 + 2x^5/15 - 17x^7/315 + 62x^9/2835 - 1382x^11/155925
//          + 21844x^13/6081075, |x| <= 0.4: next term < 2e-9 relative
__device__ __forceinline__ float tanh_taylor(float x) {
  float y = x * x;
  float p = 21844.0f / 6081075.0f;
  p = fmaf(p, y, -1382.0f / 155925.0f);
  p = fmaf(p, y, 62.0f / 2835.0f);
  p = fmaf(p, y, -17.0f / 315.0f);
  p = fmaf(p, y, 2.0f / 15.0f);
  p = fmaf(p, y, -1.0f / 3.0f);
  p = fmaf(p, y, 1.0f);
  return x * p;
}

constexpr float kSmallTrig = 0.78539816f;   // pi / 4
constexpr float kSmallTanh = 0.4f;

__device__ __forceinline__ void sincos_small(float x, float* s, float* c) {
  if (fabsf(x) <= kSmallTrig) {
    *s = sin_taylor(x);
    *c = cos_taylor(x);
  } else {
    sincosf(x, s, c);
  }
}
__device__ __forceinline__ float sin_small(float x) {
  return fabsf(x) <= kSmallTrig ? sin_taylor(x) : sinf(x);
}
__device__ __forceinline__ float tanh_small(float x) {
  return fabsf(x) <= kSmallTanh ? tanh_taylor(x) : tanhf(x);
}

// base sin / cos of a pre-activation z: the hardware sine/cosine unit on z/(2 pi);
// pre-activations are O(1-10), where its absolute error (~1e-7) is below what
// every stream formula needs
__device__ __forceinline__ void sincos_base(float z, float* s, float* c) {
  *s = __sinf(z);
  *c = __cosf(z);
}

struct TanhBase { float t, q; };   // t = tanh z, q = 1 - t^2

// t = (1 - e) / (1 + e), q = 4 e / (1 + e)^2 with e = exp(-2|z|): branch free;
// t carries an absolute (not relative) error of a few ulp of 1 near z = 0,
// which is the accuracy every stream formula below needs
__device__ __forceinline__ TanhBase tanh_base(float z) {
  float ez = __expf(-2.0f * fabsf(z));
  float r = rcp(1.0f + ez);
  float t = (1.0f - ez) * r;
  t = z < 0.0f ? -t : t;
  float q = 4.0f * ez * r * r;
  return {t, q};
}

template <int ACT>
__device__ __forceinline__ float act_base(float z) {
  if (ACT == 0) return tanh_base(z).t;
  return __sinf(z);
}

// Short series for the second-difference argument e = O(h^2):
// sin e = e (1 - e^2/6 + e^4/120), cos e = 1 - e^2/2 + e^4/24,
// tanh e = e (1 - e^2/3 + 2 e^4/15); |e| <= 1/32: next terms < 1e-11 relative.
constexpr float kTinyArg = 0.03125f;
__device__ __forceinline__ float sin_short(float e) {
  float y = e * e;
  return e * fmaf(fmaf(y, 1.0f / 120.0f, -1.0f / 6.0f), y, 1.0f);
}
__device__ __forceinline__ float cos_short(float e) {
  float y = e * e;
  return fmaf(fmaf(y, 1.0f / 24.0f, -0.5f), y, 1.0f);
}
__device__ __forceinline__ float tanh_short(float e) {
  float y = e * e;
  return e * fmaf(fmaf(y, 2.0f / 15.0f, -1.0f / 3.0f), y, 1.0f);
}

// Argument tiers for the difference arguments.  The tiny tier (taken when
// the whole wavefront has |p| <= 1/64 (tanh) or |p| <= 1/32 (sin) and
// |e| <= 1/64) is the Taylor form below; TIER 1: the longer series above;
// TIER 0: library functions for large arguments.
constexpr float kTinyP = 0.015625f;   // 1/64

// Per-axis trigonometric factors of the sin streams.  Series tiers: Taylor
// series for p/2, short series for e/2, and the half-angle m/2 = p/2 - e/2
// by the addition theorem.
struct SinAxis { float sp, cp, sm, cm, se, ce; };

template <int TIER>
__device__ __forceinline__ SinAxis sin_axis(float p, float e) {
  SinAxis r;
  float hp = 0.5f * p, he = 0.5f * e;
  if (TIER == 1) {
    r.sp = sin_taylor(hp);
    r.cp = cos_taylor(hp);
    r.se = sin_short(he);
    r.ce = cos_short(he);
    r.sm = r.sp * r.ce - r.cp * r.se;   // sin(p/2 - e/2)
    r.cm = r.cp * r.ce + r.sp * r.se;   // cos(p/2 - e/2)
  } else {
    float hm = 0.5f * (p - e);
    sincos_small(hp, &r.sp, &r.cp);
    sincos_small(hm, &r.sm, &r.cm);
    sincos_small(he, &r.se, &r.ce);
  }
  return r;
}

// Per-axis tanh factors: T_p, T_m, T_e, T_s with m = p - e, s = p + m.
struct TanhAxis { float Tp, Tm, Te, Ts; };

template <int TIER>
__device__ __forceinline__ TanhAxis tanh_axis(float p, float e) {
  TanhAxis r;
  float m = p - e;
  if (TIER == 1) {
    r.Tp = tanh_taylor(p);
    r.Tm = tanh_taylor(m);
    r.Ts = tanh_taylor(p + m);
    r.Te = tanh_short(e);
  } else {
    r.Tp = tanh_small(p);
    r.Tm = tanh_small(m);
    r.Te = tanh_small(e);
    r.Ts = tanh_small(p + m);
  }
  return r;
}

template <int ACT, int D>
__device__ __forceinline__ bool tiny_args(const float* p, const float* e) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    if (ACT == 1) ok = ok && fabsf(p[i]) <= 2.0f * kTinyP && fabsf(e[i]) <= kTinyP;
    else ok = ok && fabsf(p[i]) <= kTinyP && fabsf(e[i]) <= kTinyP;
  }
  return ok;
}

template <int ACT, int D>
__device__ __forceinline__ bool fast_args(const float* p, const float* e) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    if (ACT == 1) ok = ok && fabsf(p[i]) <= 2.0f * kSmallTrig && fabsf(e[i]) <= kTinyArg;
    else ok = ok && fabsf(p[i]) <= 0.5f * kSmallTanh && fabsf(e[i]) <= kTinyArg;
  }
  return ok;
}

template <int ACT, int D, int TIER>
__device__ __forceinline__ void act_fwd_impl(float z, const float* p, const float* e, float& a,
                                             float* Dv, float* Ev) {
  if (ACT == 1) {
    float S, C;
    sincos_base(z, &S, &C);
    a = S;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      SinAxis f = sin_axis<TIER>(p[i], e[i]);
      float cs2 = f.cp * f.cm - f.sp * f.sm;  // cos((p+m)/2)
      Dv[i] = 2.0f * f.sp * (C * f.cp - S * f.sp);
      Ev[i] = -2.0f * S * (f.sp * f.sp + f.sm * f.sm) + 2.0f * C * cs2 * f.se;
    }
  } else {
    TanhBase tb = tanh_base(z);
    float t = tb.t, q = tb.q;
    a = t;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      TanhAxis f = tanh_axis<TIER>(p[i], e[i]);
      // 1/(1 + t T_p) and 1/(1 - t T_m) from one reciprocal of their product
      float dP = 1.0f + t * f.Tp, dM = 1.0f - t * f.Tm;
      float R = rcp(dP * dM);
      float rP = dM * R, rM = dP * R;
      float qP = q * rP;
      Dv[i] = f.Tp * qP;
      Ev[i] = qP * (f.Te * (1.0f - f.Tp * f.Tm) - t * f.Tm * f.Ts * (1.0f + f.Tp * f.Tm) * rM);
    }
  }
}

template <int ACT, int D, int TIER>
__device__ __forceinline__ void act_bwd_impl(float z, const float* p, const float* e, float ab,
                                             const float* Db, const float* Eb, float& zb, float* pb,
                                             float* eb) {
  if (ACT == 1) {
    float S, C;
    sincos_base(z, &S, &C);
    zb = ab * C;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      SinAxis f = sin_axis<TIER>(p[i], e[i]);
      float sp = f.sp, cp = f.cp, sm = f.sm, cm = f.cm, se = f.se, ce = f.ce;
      float cs2 = cp * cm - sp * sm;        // cos(s/2), s = p + m
      float ss2 = sp * cm + cp * sm;        // sin(s/2)
      float sq = sp * sp + sm * sm;
      float dDdz = -2.0f * sp * (S * cp + C * sp);             // cos(z+p) - cos z
      float dDdp = C * (1.0f - 2.0f * sp * sp) - S * (2.0f * sp * cp);   // cos(z+p)
      float dEdz = -2.0f * C * sq - 2.0f * S * cs2 * se;
      float dEdp = -2.0f * (S * ce + C * se) * ss2;              // -2 sin(z+e/2) sin(s/2)
      float dEde = C * (1.0f - 2.0f * sm * sm) + S * (2.0f * sm * cm);   // cos(z-m)
      zb += Db[i] * dDdz + Eb[i] * dEdz;
      pb[i] = Db[i] * dDdp + Eb[i] * dEdp;
      eb[i] = Eb[i] * dEde;
    }
  } else {
    TanhBase tb = tanh_base(z);
    float t = tb.t, q = tb.q;
    zb = ab * q;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      TanhAxis f = tanh_axis<TIER>(p[i], e[i]);
      float Tp = f.Tp, Tm = f.Tm;
      float dP = 1.0f + t * Tp, dM = 1.0f - t * Tm;
      float R = rcp(dP * dM);
      float rP = dM * R, rM = dP * R;
      float qP = q * rP, qM = q * rM;
      float Dd = Tp * qP;
      float Bd = Tm * qM;
      float Ed = qP * (f.Te * (1.0f - Tp * Tm) - t * Tm * f.Ts * (1.0f + Tp * Tm) * rM);
      float dDdz = -Dd * (2.0f * t + Dd);
      float dDdp = qP * (1.0f - Tp * Tp) * rP;
      float dEdz = -2.0f * t * Ed - Dd * Dd - Bd * Bd;
      float dEdp = -(Dd + Bd) * (2.0f * t + Ed);
      float dEde = qM * (1.0f - Tm * Tm) * rM;
      zb += Db[i] * dDdz + Eb[i] * dEdz;
      pb[i] = Db[i] * dDdp + Eb[i] * dEdp;
      eb[i] = Eb[i] * dEde;
    }
  }
}

// First layer: the differences p = h W1[n] are constants of the network and
// e = 0 (so m = p), hence the per-axis factors (tanh: T_p, T_{2p}; sin:
// sin(p/2), cos(p/2)) are computed once per network and each centre only
// needs its base evaluation.  The stream formulas below are those above with
// e = 0 substituted.
struct L1Axes { float u[3], v[3]; };

template <int ACT, int D>
__device__ inline L1Axes l1_axes(const float* p) {
  L1Axes r;
  for (int i = 0; i < 3; ++i) { r.u[i] = 0.f; r.v[i] = 0.f; }
  for (int i = 0; i < D; ++i) {
    if (ACT == 1) {
      sincos_small(0.5f * p[i], &r.u[i], &r.v[i]);
    } else {
      r.u[i] = tanh_small(p[i]);
      r.v[i] = tanh_small(2.0f * p[i]);
    }
  }
  return r;
}

template <int ACT, int D>
__device__ __forceinline__ void act_fwd_l1(float z, const L1Axes& f, float& a, float* Dv, float* Ev) {
  if (ACT == 1) {
    float S, C;
    sincos_base(z, &S, &C);
    a = S;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const float sp = f.u[i], cp = f.v[i];
      Dv[i] = 2.0f * sp * (C * cp - S * sp);
      Ev[i] = -4.0f * S * sp * sp;
    }
  } else {
    TanhBase tb = tanh_base(z);
    const float t = tb.t, q = tb.q;
    a = t;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const float Tp = f.u[i], Ts = f.v[i];
      const float dP = 1.0f + t * Tp, dM = 1.0f - t * Tp;
      const float R = rcp(dP * dM);
      const float qP = q * dM * R, rM = dP * R;
      Dv[i] = Tp * qP;
      Ev[i] = -qP * t * Tp * Ts * (1.0f + Tp * Tp) * rM;
    }
  }
}

template <int ACT, int D>
__device__ __forceinline__ void act_bwd_l1(float z, const L1Axes& f, float ab, const float* Db,
                                           const float* Eb, float& zb, float* pb) {
  if (ACT == 1) {
    float S, C;
    sincos_base(z, &S, &C);
    zb = ab * C;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const float sp = f.u[i], cp = f.v[i];
      const float dDdz = -2.0f * sp * (S * cp + C * sp);
      const float dDdp = C * (1.0f - 2.0f * sp * sp) - S * (2.0f * sp * cp);
      const float dEdz = -4.0f * C * sp * sp;
      const float dEdp = -4.0f * S * sp * cp;
      zb += Db[i] * dDdz + Eb[i] * dEdz;
      pb[i] = Db[i] * dDdp + Eb[i] * dEdp;
    }
  } else {
    TanhBase tb = tanh_base(z);
    const float t = tb.t, q = tb.q;
    zb = ab * q;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const float Tp = f.u[i], Ts = f.v[i];
      const float dP = 1.0f + t * Tp, dM = 1.0f - t * Tp;
      const float R = rcp(dP * dM);
      const float rP = dM * R, rM = dP * R;
      const float qP = q * rP, qM = q * rM;
      const float Dd = Tp * qP;
      const float Bd = Tp * qM;
      const float Ed = -qP * t * Tp * Ts * (1.0f + Tp * Tp) * rM;
      const float dDdz = -Dd * (2.0f * t + Dd);
      const float dDdp = qP * (1.0f - Tp * Tp) * rP;
      const float dEdz = -2.0f * t * Ed - Dd * Dd - Bd * Bd;
      const float dEdp = -(Dd + Bd) * (2.0f * t + Ed);
      zb += Db[i] * dDdz + Eb[i] * dEdz;
      pb[i] = Db[i] * dDdp + Eb[i] * dEdp;
    }
  }
}

// Tiny tier: the streams from the Taylor series of the activation about the
// centre's pre-activation z,
//   a(z + x) = a(z) + sum_{k>=1} c_k x^k,   c_k = a^(k)(z) / k!,
// truncated after k = 7.  On the tier's arguments (|x| <= |p| + |e|, at most
// 1/32 for tanh and 3/64 for sin) the first omitted term is below 3e-14 and
// that of the derivative series below 1e-11 (|c_k| <= 0.39 for tanh and
// 1/k! for sin, k >= 2).  With f(x) = sum_{k>=2} c_k x^k and m = p - e:
//   D = a(z+p) - a(z)            = c_1 p + f(p),
//   E = a(z+p) - 2 a(z) + a(z-m) = c_1 e + f(p) + f(-m),
// the first-order part of E taking e itself (c_1 (p - m) would cancel); the
// higher terms are far below E's rounding level whatever cancels in them.
// The coefficients are formed once per z and shared by the d axes.
//   tanh (t = tanh z, q = 1 - t^2, u = t^2; from a' = 1 - a^2):
//     c_1 = q, c_2 = -tq, c_3 = q (u - 1/3), c_4 = tq (2/3 - u),
//     c_5 = q (u^2 - u + 2/15), c_6 = tq (-u^2 + 4u/3 - 17/45),
//     c_7 = q (u^3 - 5u^2/3 + 11u/15 - 17/315);
//   sin (S = sin z, C = cos z): c_k = S or C with the sign of the k-th
//     derivative, over k!.
//
// Micro tier (opt-in per call site, for the 128-wide kernels): when every
// lane also has |p|, |p - e| <= 1/256, f runs to k = 4 and the derivative
// series to k = 5; the first omitted terms are below 1.2e-13 and 4e-13
// (|c_5| <= 0.134, 6|c_6| <= 0.44), i.e. at most ~1e-7 of the residual once
// E is divided by h^2.
constexpr float kMicroX = 0.00390625f;   // 1/256
// Operands rounded to BF16 for the next product (micro tier 2): the same
// forms up to |p|, |p - e| <= 1/32, where the omitted terms (<= 4.1e-9 and
// 1.4e-8) stay two orders of magnitude below the BF16 rounding of values of
// the size of E there (2^-9 x^2 ~ 1.9e-6 at x = 1/32).
constexpr float kMicroXBf16 = 0.03125f;  // 1/32
// Series orders of the micro tier: f to k = F, the derivative series to
// k = G.  Sine with BF16 operands stops one term earlier (f to k = 3, g to
// k = 4): at |x| <= 1/32 the omitted terms are at most 2 x^4/24 and
// 2 x^4/24 again (|c_4| <= 1/24, 5|c_5| <= 1/24), 7.9e-8, one to two orders
// of magnitude below the BF16 rounding of the terms they sit next to
// (2^-9 x^2 ~ 1.9e-6 for f, 2^-9 x^2/2 for g).  For tanh |c_4| reaches 0.17
// and 5|c_5| 0.67, too close to that rounding, so tanh keeps the longer
// series.
template <int ACT, int MICRO>
struct MicroOrder {
  static constexpr int F = (MICRO == 2 && ACT == 1) ? 3 : 4;
  static constexpr int G = F + 1;
};
struct Taylor { float a, c[8]; };   // c[1..K]

template <int ACT, int K = 7>
__device__ __forceinline__ Taylor taylor_at(float z) {
  Taylor T;
  T.c[0] = 0.f;
  if (ACT == 1) {
    float S, C;
    sincos_base(z, &S, &C);
    T.a = S;
    T.c[1] = C;
    T.c[2] = S * (-1.0f / 2.0f);
    T.c[3] = C * (-1.0f / 6.0f);
    T.c[4] = S * (1.0f / 24.0f);
    T.c[5] = C * (1.0f / 120.0f);
    if (K >= 7) {
      T.c[6] = S * (-1.0f / 720.0f);
      T.c[7] = C * (-1.0f / 5040.0f);
    }
  } else {
    const TanhBase tb = tanh_base(z);
    const float t = tb.t, q = tb.q, u = t * t, tq = t * q;
    T.a = t;
    T.c[1] = q;
    T.c[2] = -tq;
    T.c[3] = q * (u - 1.0f / 3.0f);
    T.c[4] = tq * (2.0f / 3.0f - u);
    T.c[5] = q * fmaf(u, u - 1.0f, 2.0f / 15.0f);
    if (K >= 7) {
      T.c[6] = tq * fmaf(u, 4.0f / 3.0f - u, -17.0f / 45.0f);
      T.c[7] = q * fmaf(u, fmaf(u, u - 5.0f / 3.0f, 11.0f / 15.0f), -17.0f / 315.0f);
    }
  }
  return T;
}

// f(x) = sum_{k=2..KF} c_k x^k
template <int KF = 7>
__device__ __forceinline__ float taylor_f(const Taylor& T, float x) {
  float r = T.c[KF];
#pragma unroll
  for (int k = KF - 1; k >= 2; --k) r = fmaf(x, r, T.c[k]);
  return (x * x) * r;
}
// g(x) = sum_{k=3..KG} k c_k x^(k-1), from d[k] = k c_k: a'(z + x) = c_1 + d_2 x + g(x)
template <int KG = 7>
__device__ __forceinline__ float taylor_g(const float* d, float x) {
  float r = d[KG];
#pragma unroll
  for (int k = KG - 1; k >= 3; --k) r = fmaf(x, r, d[k]);
  return (x * x) * r;
}

template <int D, int KF = 7>
__device__ __forceinline__ void taylor_fwd(const Taylor& T, const float* p, const float* e, float* Dv,
                                           float* Ev) {
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const float m = p[i] - e[i];
    const float fp = taylor_f<KF>(T, p[i]), fm = taylor_f<KF>(T, -m);
    Dv[i] = fmaf(T.c[1], p[i], fp);
    Ev[i] = fmaf(T.c[1], e[i], fp + fm);
  }
}

// the derivatives of D and E by z, p and e are values of a' = c_1 + d_2 x + g(x):
//   dD/dz = a'(z+p) - a'(z) = d_2 p + g(p),        dD/dp = a'(z+p),
//   dE/dz = a'(z+p) - 2a'(z) + a'(z-m) = d_2 e + g(p) + g(-m),
//   dE/dp = a'(z+p) - a'(z-m) = d_2 (p + m) + g(p) - g(-m),   dE/de = a'(z-m)
template <int D, int KG = 7>
__device__ __forceinline__ void taylor_bwd(const Taylor& T, const float* p, const float* e, float ab,
                                           const float* Db, const float* Eb, float& zb, float* pb,
                                           float* eb) {
  float d[8];
#pragma unroll
  for (int k = 2; k <= KG; ++k) d[k] = (float)k * T.c[k];
  zb = ab * T.c[1];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const float m = p[i] - e[i];
    const float gp = taylor_g<KG>(d, p[i]), gm = taylor_g<KG>(d, -m);
    const float dDdz = fmaf(d[2], p[i], gp);
    const float dDdp = T.c[1] + dDdz;
    const float dEdz = fmaf(d[2], e[i], gp + gm);
    const float dEdp = fmaf(d[2], p[i] + m, gp - gm);
    const float dEde = T.c[1] + fmaf(-d[2], m, gm);
    zb = fmaf(Db[i], dDdz, fmaf(Eb[i], dEdz, zb));
    pb[i] = fmaf(Db[i], dDdp, Eb[i] * dEdp);
    eb[i] = Eb[i] * dEde;
  }
}

// Backward of the micro tier with BF16 operands, factored through
// A = a'(z+p) - c_1 = d_2 p + g(p) and B = a'(z-m) - c_1 = -d_2 m + g(-m):
//   dD/dz = A, dD/dp = c_1 + A, dE/dz = A + B, dE/dp = A - B, dE/de = c_1 + B,
// so with U = A (D^ + E^) and V = E^ B the adjoints are
//   z^ += U + V,  p^ = c_1 D^ + U - V,  e^ = c_1 E^ + V.
// A + B ~ d_2 e + d_3 (p^2 + m^2) is formed by cancellation here: its FP32
// rounding is at most 2^-24 |A| ~ 2^-24 |p|, relative 2^-24 |p| / |A + B|
// (2^-16 for e ~ h p at h = 1/256), far below the 2^-9 rounding of the BF16
// operands these adjoints feed.  The FP32 paths keep taylor_bwd's
// cancellation-free forms.
template <int D, int KG>
__device__ __forceinline__ void taylor_bwd_bf16(const Taylor& T, const float* p, const float* e, float ab,
                                                const float* Db, const float* Eb, float& zb, float* pb,
                                                float* eb) {
  float d[8];
#pragma unroll
  for (int k = 2; k <= KG; ++k) d[k] = (float)k * T.c[k];
  zb = ab * T.c[1];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const float m = p[i] - e[i];
    const float A = fmaf(d[2], p[i], taylor_g<KG>(d, p[i]));
    const float B = fmaf(-d[2], m, taylor_g<KG>(d, -m));
    const float U = A * (Db[i] + Eb[i]), V = Eb[i] * B;
    zb += U + V;
    pb[i] = fmaf(T.c[1], Db[i], U - V);
    eb[i] = fmaf(T.c[1], Eb[i], V);
  }
}

// Longer series and library paths kept out of line (each lane picks its
// tier there): taken only when some lane of the wavefront has a difference
// argument beyond the tiny tier, so the common path stays register-lean.
// Scalars in, a small struct out: everything travels in registers.
struct ActFwdOut { float a, D[3], E[3]; };
struct ActBwdOut { float zb, pb[3], eb[3]; };

template <int ACT, int D>
__device__ __attribute__((noinline)) ActFwdOut act_fwd_general(float z, float p0, float p1, float p2,
                                                               float e0, float e1, float e2) {
  const float p[3] = {p0, p1, p2}, e[3] = {e0, e1, e2};
  ActFwdOut r;
  if (fast_args<ACT, D>(p, e)) act_fwd_impl<ACT, D, 1>(z, p, e, r.a, r.D, r.E);
  else act_fwd_impl<ACT, D, 0>(z, p, e, r.a, r.D, r.E);
  return r;
}
template <int ACT, int D>
__device__ __attribute__((noinline)) ActBwdOut act_bwd_general(float z, float p0, float p1, float p2,
                                                               float e0, float e1, float e2, float ab,
                                                               float D0, float D1, float D2, float E0,
                                                               float E1, float E2) {
  const float p[3] = {p0, p1, p2}, e[3] = {e0, e1, e2};
  const float Db[3] = {D0, D1, D2}, Eb[3] = {E0, E1, E2};
  ActBwdOut r;
  if (fast_args<ACT, D>(p, e)) act_bwd_impl<ACT, D, 1>(z, p, e, ab, Db, Eb, r.zb, r.pb, r.eb);
  else act_bwd_impl<ACT, D, 0>(z, p, e, ab, Db, Eb, r.zb, r.pb, r.eb);
  return r;
}

// forward: base a, and per-axis D, E from (z, p, e).  One wave-uniform
// branch takes the inline tiny-argument tier when every lane qualifies.
// MICRO: 0 = no micro tier, 1 = up to kMicroX, 2 = up to kMicroXBf16 (BF16
// operand paths only)
template <int D, int MICRO>
__device__ __forceinline__ bool micro_args(const float* p, const float* e) {
  constexpr float X = MICRO == 2 ? kMicroXBf16 : kMicroX;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < D; ++i) ok = ok && fabsf(p[i]) <= X && fabsf(p[i] - e[i]) <= X;
  return ok;
}

// The micro tier's forms without their check, for callers that have
// established micro_args for every lane (and keep that decision for the
// backward of the same arguments).
template <int ACT, int D, int MICRO>
__device__ __forceinline__ void act_fwd_micro(float z, const float* p, const float* e, float& a,
                                              float* Dv, float* Ev) {
  const Taylor T = taylor_at<ACT, MicroOrder<ACT, MICRO>::G>(z);
  a = T.a;
  taylor_fwd<D, MicroOrder<ACT, MICRO>::F>(T, p, e, Dv, Ev);
}
template <int ACT, int D, int MICRO>
__device__ __forceinline__ void act_bwd_micro(float z, const float* p, const float* e, float ab,
                                              const float* Db, const float* Eb, float& zb, float* pb,
                                              float* eb) {
  constexpr int KG = MicroOrder<ACT, MICRO>::G;
  if constexpr (MICRO == 2) taylor_bwd_bf16<D, KG>(taylor_at<ACT, KG>(z), p, e, ab, Db, Eb, zb, pb, eb);
  else taylor_bwd<D, KG>(taylor_at<ACT, KG>(z), p, e, ab, Db, Eb, zb, pb, eb);
}
template <int ACT, int D, int MICRO>
__device__ __forceinline__ void act_fb_micro(float z, const float* p, const float* e, float ab,
                                             const float* Db, const float* Eb, float& a, float* Dv,
                                             float* Ev, float& zb, float* pb, float* eb) {
  const Taylor T = taylor_at<ACT, MicroOrder<ACT, MICRO>::G>(z);
  a = T.a;
  taylor_fwd<D, MicroOrder<ACT, MICRO>::F>(T, p, e, Dv, Ev);
  if constexpr (MICRO == 2) taylor_bwd_bf16<D, MicroOrder<ACT, MICRO>::G>(T, p, e, ab, Db, Eb, zb, pb, eb);
  else taylor_bwd<D, MicroOrder<ACT, MICRO>::G>(T, p, e, ab, Db, Eb, zb, pb, eb);
}

// the largest micro argument of one element, max_i max(|p_i|, |p_i - e_i|):
// micro_args holds iff it is <= the bound (a running maximum checks many
// elements with one comparison)
template <int D>
__device__ __forceinline__ float micro_extent(const float* p, const float* e) {
  float r = 0.f;
#pragma unroll
  for (int i = 0; i < D; ++i) r = fmaxf(r, fmaxf(fabsf(p[i]), fabsf(p[i] - e[i])));
  return r;
}
template <int MICRO>
constexpr float micro_bound() { return MICRO == 2 ? kMicroXBf16 : kMicroX; }

template <int ACT, int D, int MICRO = 0>
__device__ __forceinline__ void act_fwd(float z, const float* p, const float* e, float& a,
                                        float* Dv, float* Ev) {
  if (MICRO > 0 && __all(micro_args<D, MICRO>(p, e))) {
    act_fwd_micro<ACT, D, MICRO>(z, p, e, a, Dv, Ev);
  } else if (__all(tiny_args<ACT, D>(p, e))) {
    const Taylor T = taylor_at<ACT>(z);
    a = T.a;
    taylor_fwd<D>(T, p, e, Dv, Ev);
  } else {
    const ActFwdOut r = act_fwd_general<ACT, D>(z, p[0], D > 1 ? p[1] : 0.f, D > 2 ? p[2] : 0.f, e[0],
                                                D > 1 ? e[1] : 0.f, D > 2 ? e[2] : 0.f);
    a = r.a;
    for (int i = 0; i < D; ++i) { Dv[i] = r.D[i]; Ev[i] = r.E[i]; }
  }
}

// backward: given stream adjoints (ab, Db, Eb) return (zb, pb, eb)
template <int ACT, int D, int MICRO = 0>
__device__ __forceinline__ void act_bwd(float z, const float* p, const float* e, float ab,
                                        const float* Db, const float* Eb, float& zb, float* pb,
                                        float* eb) {
  if (MICRO > 0 && __all(micro_args<D, MICRO>(p, e))) {
    act_bwd_micro<ACT, D, MICRO>(z, p, e, ab, Db, Eb, zb, pb, eb);
  } else if (__all(tiny_args<ACT, D>(p, e))) {
    taylor_bwd<D>(taylor_at<ACT>(z), p, e, ab, Db, Eb, zb, pb, eb);
  } else {
    const ActBwdOut r = act_bwd_general<ACT, D>(
        z, p[0], D > 1 ? p[1] : 0.f, D > 2 ? p[2] : 0.f, e[0], D > 1 ? e[1] : 0.f, D > 2 ? e[2] : 0.f,
        ab, Db[0], D > 1 ? Db[1] : 0.f, D > 2 ? Db[2] : 0.f, Eb[0], D > 1 ? Eb[1] : 0.f,
        D > 2 ? Eb[2] : 0.f);
    zb = r.zb;
    for (int i = 0; i < D; ++i) { pb[i] = r.pb[i]; eb[i] = r.eb[i]; }
  }
}

// Forward and backward streams of one (z, p, e) together: the per-axis
// factors are formed once and shared (used where the adjoints are at hand
// when the activations are evaluated, or where the backward pass recomputes
// the activations it needs).
struct ActFBOut { float a, D[3], E[3], zb, pb[3], eb[3]; };

template <int ACT, int D>
__device__ __attribute__((noinline)) ActFBOut act_fb_general(float z, float p0, float p1, float p2,
                                                             float e0, float e1, float e2, float ab,
                                                             float D0, float D1, float D2, float E0,
                                                             float E1, float E2) {
  const float p[3] = {p0, p1, p2}, e[3] = {e0, e1, e2};
  const float Db[3] = {D0, D1, D2}, Eb[3] = {E0, E1, E2};
  ActFBOut r;
  if (fast_args<ACT, D>(p, e)) {
    act_fwd_impl<ACT, D, 1>(z, p, e, r.a, r.D, r.E);
    act_bwd_impl<ACT, D, 1>(z, p, e, ab, Db, Eb, r.zb, r.pb, r.eb);
  } else {
    act_fwd_impl<ACT, D, 0>(z, p, e, r.a, r.D, r.E);
    act_bwd_impl<ACT, D, 0>(z, p, e, ab, Db, Eb, r.zb, r.pb, r.eb);
  }
  return r;
}

template <int ACT, int D, int MICRO = 0>
__device__ __forceinline__ void act_fb(float z, const float* p, const float* e, float ab,
                                       const float* Db, const float* Eb, float& a, float* Dv,
                                       float* Ev, float& zb, float* pb, float* eb) {
  if (MICRO > 0 && __all(micro_args<D, MICRO>(p, e))) {
    act_fb_micro<ACT, D, MICRO>(z, p, e, ab, Db, Eb, a, Dv, Ev, zb, pb, eb);
  } else if (__all(tiny_args<ACT, D>(p, e))) {
    const Taylor T = taylor_at<ACT>(z);
    a = T.a;
    taylor_fwd<D>(T, p, e, Dv, Ev);
    taylor_bwd<D>(T, p, e, ab, Db, Eb, zb, pb, eb);
  } else {
    const ActFBOut r = act_fb_general<ACT, D>(
        z, p[0], D > 1 ? p[1] : 0.f, D > 2 ? p[2] : 0.f, e[0], D > 1 ? e[1] : 0.f, D > 2 ? e[2] : 0.f,
        ab, Db[0], D > 1 ? Db[1] : 0.f, D > 2 ? Db[2] : 0.f, Eb[0], D > 1 ? Eb[1] : 0.f,
        D > 2 ? Eb[2] : 0.f);
    a = r.a;
    zb = r.zb;
    for (int i = 0; i < D; ++i) { Dv[i] = r.D[i]; Ev[i] = r.E[i]; pb[i] = r.pb[i]; eb[i] = r.eb[i]; }
  }
}

// first layer, forward and backward together (e = 0, constant axis factors)
template <int ACT, int D>
__device__ __forceinline__ void act_fb_l1(float z, const L1Axes& f, float ab, const float* Db,
                                          const float* Eb, float& a, float* Dv, float* Ev, float& zb,
                                          float* pb) {
  act_fwd_l1<ACT, D>(z, f, a, Dv, Ev);
  act_bwd_l1<ACT, D>(z, f, ab, Db, Eb, zb, pb);
}

// The first-layer forms above, out of line: taken only by wavefronts with a
// first-layer argument beyond the micro bound, so the common path keeps its
// registers.
template <int ACT, int D>
__device__ __attribute__((noinline)) ActFwdOut act_fwd_l1_general(float z, L1Axes f) {
  ActFwdOut r;
  act_fwd_l1<ACT, D>(z, f, r.a, r.D, r.E);
  return r;
}
struct ActFBL1Out { float a, D[3], E[3], zb, pb[3]; };
template <int ACT, int D>
__device__ __attribute__((noinline)) ActFBL1Out act_fb_l1_general(float z, L1Axes f, float ab, float D0,
                                                                   float D1, float D2, float E0, float E1,
                                                                   float E2) {
  const float Db[3] = {D0, D1, D2}, Eb[3] = {E0, E1, E2};
  ActFBL1Out r;
  act_fb_l1<ACT, D>(z, f, ab, Db, Eb, r.a, r.D, r.E, r.zb, r.pb);
  return r;
}

// First layer with micro arguments (every |p| <= 1/256 in the wavefront):
// e = 0 and m = p, so the Taylor forms (values to k = 4, derivatives to
// k = 5, first omitted terms as in the micro tier) reduce to
//   D = c1 p + c2 p^2 + c3 p^3 + c4 p^4,      E = 2 (c2 p^2 + c4 p^4),
//   dD/dz = d2 p + d3 p^2 + d4 p^3 + d5 p^4,  dD/dp = c1 + dD/dz,
//   dE/dz = 2 (d3 p^2 + d5 p^4),              dE/dp = 2 (d2 p + d4 p^3),
// with d_k = k c_k.  The per-network axis factors are then u = p, v = p^2.
template <int D>
__device__ __forceinline__ bool l1_micro(const float* p) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < D; ++i) ok = ok && fabsf(p[i]) <= kMicroX;
  return ok;
}
template <int D>
__device__ inline L1Axes l1_axes_micro(const float* p) {
  L1Axes r;
  for (int i = 0; i < 3; ++i) { r.u[i] = 0.f; r.v[i] = 0.f; }
  for (int i = 0; i < D; ++i) { r.u[i] = p[i]; r.v[i] = p[i] * p[i]; }
  return r;
}

template <int ACT, int D>
__device__ __forceinline__ void act_fwd_l1_micro(float z, const L1Axes& f, float& a, float* Dv, float* Ev) {
  const Taylor T = taylor_at<ACT, 5>(z);
  a = T.a;
  const float e2 = 2.0f * T.c[2], e4 = 2.0f * T.c[4];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const float p = f.u[i], p2 = f.v[i];
    Dv[i] = p * fmaf(p, fmaf(p, fmaf(p, T.c[4], T.c[3]), T.c[2]), T.c[1]);
    Ev[i] = p2 * fmaf(p2, e4, e2);
  }
}

template <int ACT, int D>
__device__ __forceinline__ void act_fb_l1_micro(float z, const L1Axes& f, float ab, const float* Db,
                                                const float* Eb, float& a, float* Dv, float* Ev,
                                                float& zb, float* pb) {
  const Taylor T = taylor_at<ACT, 5>(z);
  a = T.a;
  const float e2 = 2.0f * T.c[2], e4 = 2.0f * T.c[4];
  const float d2 = 2.0f * T.c[2], d3 = 3.0f * T.c[3], d4 = 4.0f * T.c[4], d5 = 5.0f * T.c[5];
  const float g2 = 2.0f * d2, g3 = 2.0f * d3, g4 = 2.0f * d4, g5 = 2.0f * d5;
  zb = ab * T.c[1];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const float p = f.u[i], p2 = f.v[i];
    Dv[i] = p * fmaf(p, fmaf(p, fmaf(p, T.c[4], T.c[3]), T.c[2]), T.c[1]);
    Ev[i] = p2 * fmaf(p2, e4, e2);
    const float dDdz = p * fmaf(p, fmaf(p, fmaf(p, d5, d4), d3), d2);
    const float dDdp = T.c[1] + dDdz;
    const float dEdz = p2 * fmaf(p2, g5, g3);
    const float dEdp = p * fmaf(p2, g4, g2);
    zb = fmaf(Db[i], dDdz, fmaf(Eb[i], dEdz, zb));
    pb[i] = fmaf(Db[i], dDdp, Eb[i] * dEdp);
  }
}

// first-layer dispatch: the micro forms inline, the others out of line
template <int ACT, int D>
__device__ __forceinline__ void act_fwd_l1_any(bool micro, float z, const L1Axes& f, float& a, float* Dv,
                                               float* Ev) {
  if (micro) {
    act_fwd_l1_micro<ACT, D>(z, f, a, Dv, Ev);
  } else {
    const ActFwdOut r = act_fwd_l1_general<ACT, D>(z, f);
    a = r.a;
    for (int i = 0; i < D; ++i) { Dv[i] = r.D[i]; Ev[i] = r.E[i]; }
  }
}
template <int ACT, int D>
__device__ __forceinline__ void act_fb_l1_any(bool micro, float z, const L1Axes& f, float ab,
                                              const float* Db, const float* Eb, float& a, float* Dv,
                                              float* Ev, float& zb, float* pb) {
  if (micro) {
    act_fb_l1_micro<ACT, D>(z, f, ab, Db, Eb, a, Dv, Ev, zb, pb);
  } else {
    const ActFBL1Out r = act_fb_l1_general<ACT, D>(z, f, ab, Db[0], D > 1 ? Db[1] : 0.f, D > 2 ? Db[2] : 0.f,
                                                   Eb[0], D > 1 ? Eb[1] : 0.f, D > 2 ? Eb[2] : 0.f);
    a = r.a;
    zb = r.zb;
    for (int i = 0; i < D; ++i) { Dv[i] = r.D[i]; Ev[i] = r.E[i]; pb[i] = r.pb[i]; }
  }
}

// ---------------------------------------------------------------------------
// Level sets (FP64).  Omega^- = {phi < 0}; phi = 0 belongs to Omega^+.
// ---------------------------------------------------------------------------
// level set stored on a coarse mesh of phi_n intervals per axis over
// [-1, 1]^D: multilinear interpolation of the nodal values (the last cell
// serves points on the upper faces)
template <int D>
__device__ inline double phi_mesh(const Problem& P, const double* x) {
  const int n = P.phi_n;
  int j[3] = {0, 0, 0};
  double f[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < D; ++a) {
    const double t = (x[a] + 1.0) * (0.5 * n);
    int ja = (int)floor(t);
    ja = ja < 0 ? 0 : (ja > n - 1 ? n - 1 : ja);
    j[a] = ja;
    f[a] = t - (double)ja;
  }
  const int64_t s1 = n + 1, s2 = s1 * s1;
  double acc = 0.0;
  for (int c = 0; c < (1 << D); ++c) {
    double w = 1.0;
    int64_t q = 0;
    for (int a = 0; a < D; ++a) {
      const int bit = (c >> a) & 1;
      w *= bit ? f[a] : 1.0 - f[a];
      q += (int64_t)(j[a] + bit) * (a == 0 ? 1 : (a == 1 ? s1 : s2));
    }
    acc += w * P.phitab[q];
  }
  return acc;
}

template <int D>
__device__ inline double phi_at(const Problem& P, const double* x) {
  if (P.iface == 3) return phi_mesh<D>(P, x);
  if (P.iface == 2) {
    double s = -P.pc;
    for (int i = 0; i < D; ++i) s += P.pn[i] * x[i];
    return s;
  }
  double r2 = 0.0;
  for (int i = 0; i < D; ++i) r2 += x[i] * x[i];
  double r = sqrt(r2);
  if (P.iface == 0) return r - P.R;
  // star, written as a rational function of the coordinates:
  // sin(5 theta) sin(4 psi) = 4 z (z^2 - rho^2) Im((x + i y)^5) / (rho^4 r^4)
  if (r2 == 0.0) return -P.R;
  double X = x[0], Y = x[1], Z = (D > 2) ? x[2] : 0.0;
  double rho2 = X * X + Y * Y;
  if (rho2 == 0.0) return r - P.R;
  double x2 = X * X, y2 = Y * Y;
  double im5 = Y * (5.0 * x2 * x2 - 10.0 * x2 * y2 + y2 * y2);
  double ang = 4.0 * Z * (Z * Z - rho2) * im5 / (rho2 * rho2 * r2 * r2);
  return r - P.R - P.amp * ang;
}

template <int D>
__device__ inline bool is_minus(const Problem& P, const double* x) {
  if (P.iface == 0) {
    double r2 = 0.0;
    for (int i = 0; i < D; ++i) r2 += x[i] * x[i];
    return r2 < P.R * P.R;
  }
  return phi_at<D>(P, x) < 0.0;
}

template <int D>
__device__ inline void grad_phi(const Problem& P, const double* x, double* g) {
  if (P.iface == 2) {
    for (int i = 0; i < D; ++i) g[i] = P.pn[i];
    return;
  }
  if (P.iface == 0) {
    double r2 = 0.0;
    for (int i = 0; i < D; ++i) r2 += x[i] * x[i];
    double r = sqrt(r2);
    for (int i = 0; i < D; ++i) g[i] = r > 0.0 ? x[i] / r : 0.0;
    return;
  }
  const double st = 1e-6;
  for (int i = 0; i < D; ++i) {
    double xp[3], xm[3];
    for (int j = 0; j < D; ++j) { xp[j] = x[j]; xm[j] = x[j]; }
    xp[i] += st;
    xm[i] -= st;
    g[i] = (phi_at<D>(P, xp) - phi_at<D>(P, xm)) / (2.0 * st);
  }
}

// one Newton step onto Gamma: pi, signed distance, unit normal at pi
template <int D>
__device__ inline void project(const Problem& P, const double* y, double* pi, double& dist,
                               double* nrm) {
  double ph = phi_at<D>(P, y);
  double g[3];
  grad_phi<D>(P, y, g);
  double g2 = 0.0;
  for (int i = 0; i < D; ++i) g2 += g[i] * g[i];
  if (g2 <= 0.0) g2 = 1.0;
  for (int i = 0; i < D; ++i) pi[i] = y[i] - ph / g2 * g[i];
  dist = ph / sqrt(g2);
  double gn[3];
  grad_phi<D>(P, pi, gn);
  double nn = 0.0;
  for (int i = 0; i < D; ++i) nn += gn[i] * gn[i];
  nn = sqrt(nn);
  for (int i = 0; i < D; ++i) nrm[i] = nn > 0.0 ? gn[i] / nn : 0.0;
}

// ---------------------------------------------------------------------------
// Problem data (paper Sec. 2 and 4.1).  T = float for uncut cells, double
// for cut cells.
// ---------------------------------------------------------------------------
template <class T, int D>
__device__ inline T u_side(const Problem& P, int s, const T* x) {
  if (P.kind == 0) return s == 0 ? exp(x[0] + x[1]) : sin(T(M_PI) * x[0]) * cos(T(M_PI) * x[1]);
  if (P.kind == 1) return s == 0 ? exp(x[2]) : cos(x[0]) * sin(x[1]);
  if (P.kind == 3) {
    const double* c = s == 0 ? P.lin_a : P.lin_b;
    T v = T(c[3]);
    for (int i = 0; i < D; ++i) v += T(c[i]) * x[i];
    return v;
  }
  return T(0);
}

template <class T, int D>
__device__ inline void grad_u_side(const Problem& P, int s, const T* x, T* g) {
  for (int i = 0; i < D; ++i) g[i] = T(0);
  if (P.kind == 0) {
    if (s == 0) {
      T e = exp(x[0] + x[1]);
      g[0] = e;
      g[1] = e;
    } else {
      g[0] = T(M_PI) * cos(T(M_PI) * x[0]) * cos(T(M_PI) * x[1]);
      g[1] = -T(M_PI) * sin(T(M_PI) * x[0]) * sin(T(M_PI) * x[1]);
    }
  } else if (P.kind == 1) {
    if (s == 0) {
      g[2] = exp(x[2]);
    } else {
      g[0] = -sin(x[0]) * sin(x[1]);
      g[1] = cos(x[0]) * cos(x[1]);
    }
  } else if (P.kind == 3) {
    const double* c = s == 0 ? P.lin_a : P.lin_b;
    for (int i = 0; i < D; ++i) g[i] = T(c[i]);
  }
}

// Fourier forcing f(x) = sum_k a_k cos(pi k.x) + b_k sin(pi k.x), built from
// per-axis phase factors exp(i pi k_a x_a), k_a in [-8, 8].
template <class T, int D>
__device__ inline T fourier_f(const Problem& P, const T* x) {
  T cr[D][9], ci[D][9];
  for (int a = 0; a < D; ++a)
    for (int k = 0; k <= 8; ++k) {
      T sv, cv;
      if (sizeof(T) == 4) {
        float s_, c_;
        sincospif((float)(k * (float)x[a]), &s_, &c_);
        sv = T(s_); cv = T(c_);
      } else {
        double s_, c_;
        sincospi((double)k * (double)x[a], &s_, &c_);
        sv = T(s_); cv = T(c_);
      }
      cr[a][k] = cv;
      ci[a][k] = sv;
    }
  T acc = T(0);
  for (int m = 0; m < P.n_modes; ++m) {
    T re = T(1), im = T(0), ka, aa, bb;
    int kk[3];
    if (sizeof(T) == 4) {
      const float* md = P.modes32 + 8 * m;
      kk[0] = (int)md[0]; kk[1] = (int)md[1]; kk[2] = (int)md[2];
      aa = T(md[3]); bb = T(md[4]);
    } else {
      const double* md = P.modes64 + 5 * m;
      kk[0] = (int)md[0]; kk[1] = (int)md[1]; kk[2] = (int)md[2];
      aa = T(md[3]); bb = T(md[4]);
    }
    (void)ka;
    for (int a = 0; a < D; ++a) {
      int k = kk[a];
      T fr = cr[a][k < 0 ? -k : k];
      T fi = k < 0 ? -ci[a][-k] : ci[a][k];
      T nr = re * fr - im * fi;
      T ni = re * fi + im * fr;
      re = nr;
      im = ni;
    }
    acc += aa * re + bb * im;
  }
  return acc;
}

// diffusion coefficient mu^s(x): constant, or the Sec. 4.1 functions
// mu^- = y^2 ln(x + 2) + 4, mu^+ = e^-z
template <class T, int D>
__device__ inline T mu_at(const Problem& P, int s, const T* x) {
  if (P.mu_kind == 0) return T(P.mu[s]);
  return s == 0 ? x[1] * x[1] * log(x[0] + T(2)) + T(4) : exp(-x[2]);
}
template <class T, int D>
__device__ inline void grad_mu(const Problem& P, int s, const T* x, T* g) {
  for (int i = 0; i < D; ++i) g[i] = T(0);
  if (P.mu_kind == 0) return;
  if (s == 0) {
    g[0] = x[1] * x[1] / (x[0] + T(2));
    g[1] = T(2) * x[1] * log(x[0] + T(2));
  } else {
    g[2] = -exp(-x[2]);
  }
}

// Laplacian of the manufactured u^s
template <class T, int D>
__device__ inline T lap_u_side(const Problem& P, int s, const T* x) {
  if (P.kind == 0)
    return s == 0 ? T(2) * exp(x[0] + x[1]) : T(-2.0 * M_PI * M_PI) * sin(T(M_PI) * x[0]) * cos(T(M_PI) * x[1]);
  if (P.kind == 1) return s == 0 ? exp(x[2]) : T(-2) * cos(x[0]) * sin(x[1]);
  return T(0);
}

// f^s = k^s u^s - div(mu^s grad u^s) = k^s u^s - mu^s Laplacian(u^s)
// - grad mu^s . grad u^s for the manufactured problems; the Fourier series
template <class T, int D>
__device__ inline T f_side(const Problem& P, int s, const T* x) {
  if (P.kind == 2) return fourier_f<T, D>(P, x);
  T f = -mu_at<T, D>(P, s, x) * lap_u_side<T, D>(P, s, x);
  if (P.mu_kind != 0) {
    T gm[3], gu[3];
    grad_mu<T, D>(P, s, x, gm);
    grad_u_side<T, D>(P, s, x, gu);
    for (int i = 0; i < D; ++i) f -= gm[i] * gu[i];
  }
  if (P.kc[s] != 0.0) f += T(P.kc[s]) * u_side<T, D>(P, s, x);
  return f;
}

template <int D>
__device__ inline double alpha_at(const Problem& P, const double* y) {
  if (P.kind == 2) return P.alpha_c;
  return u_side<double, D>(P, 1, y) - u_side<double, D>(P, 0, y);
}

template <int D>
__device__ inline double beta_at(const Problem& P, const double* y, const double* n) {
  if (P.kind == 2) return P.beta_c;
  double gp[3], gm[3];
  grad_u_side<double, D>(P, 1, y, gp);
  grad_u_side<double, D>(P, 0, y, gm);
  double a = 0.0, b = 0.0;
  for (int i = 0; i < D; ++i) { a += gp[i] * n[i]; b += gm[i] * n[i]; }
  return mu_at<double, D>(P, 1, y) * a - mu_at<double, D>(P, 0, y) * b;
}

template <int D>
__device__ inline float g_dirichlet(const Problem& P, const float* x) {
  if (P.kind == 2) return 0.0f;
  double xd[3];
  for (int i = 0; i < D; ++i) xd[i] = x[i];
  bool m = is_minus<D>(P, xd);
  return u_side<float, D>(P, m ? 0 : 1, x);
}

}  // namespace nbm

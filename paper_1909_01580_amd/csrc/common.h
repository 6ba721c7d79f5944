// Shared device helpers of the HGKS kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The per-lane arithmetic (reconstruction, flux) is also instantiated on the
// host by the operation-counting tool, hence host-and-device functions.
#define HGKS_FN __host__ __device__ __forceinline__

namespace hgks {

// A double constant in a scalar register pair.  FP64 vector instructions
// take no 64-bit literal, so a constant whose low word is not zero is
// otherwise rebuilt by two vector moves at every use; from a scalar pair it
// is a plain operand (one scalar operand per instruction: the addend or the
// multiplier of an FMA), built by scalar moves that issue beside the vector
// work.
HGKS_FN double sreg(double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm volatile("" : "=s"(r) : "0"(c));
  return r;
#else
  return c;
#endif
}
template <typename T> HGKS_FN T kconst(double c) { return T(c); }
template <> HGKS_FN double kconst<double>(double c) { return sreg(c); }

// exp(x) in double: Cody and Waite's reduction x = k ln2 + r, k = rint(x /
// ln2), |r| <= ln2 / 2, with ln2 split as hi + lo (hi has 21 significant
// bits, so k hi is exact for every k that does not overflow), then the
// Taylor polynomial of e^r to degree 13 (the first omitted term is below
// 7e-18 relative) by Horner's rule, scaled by 2^k.  Arguments below -1000
// are raised to -1000 (the result is 0 either way); NaN passes through.
constexpr double exp_taylor_coef(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f /= k;
  return f;
}
HGKS_FN double exp_cw(double x) {
  x = x < -1000.0 ? -1000.0 : x;
  const double k = rint(x * kconst<double>(1.4426950408889634));  // 1/ln2
  double r = fma(-k, 0.693146705627441406250, x);                 // ln2 hi
  r = fma(-k, kconst<double>(4.7493250390316727e-07), r);          // ln2 lo
  double p = kconst<double>(exp_taylor_coef(13));
#pragma unroll
  for (int n = 12; n >= 0; --n) p = fma(p, r, kconst<double>(exp_taylor_coef(n)));
  return ldexp(p, (int)k);
}

template <typename T> HGKS_FN T d_exp(T x);
template <> HGKS_FN double d_exp<double>(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return exp_cw(x);
#else
  return exp(x);
#endif
}
template <> HGKS_FN float d_exp<float>(float x) { return expf(x); }
// erf(x) = (2/sqrt(pi)) sum_n (-1)^n x^(2n+1) / (n! (2n+1)), its Maclaurin
// series, summed by Horner's rule in x^2 over the first N terms.  For
// |x| <= 1 the first omitted term is below 5e-18 with N = 18 (double) and
// 1.2e-9 with N = 11 (float).
constexpr double erf_series_coef(int n) {
  double f = 1.12837916709551257389615890312154517;  // 2/sqrt(pi)
  for (int k = 1; k <= n; ++k) f = -f / k;
  return f / (2 * n + 1);
}

template <int N, typename T>
HGKS_FN T erf_series(T x) {
  const T t = x * x;
  T s = T(erf_series_coef(N - 1));
#pragma unroll
  for (int n = N - 2; n >= 0; --n) s = s * t + kconst<T>(erf_series_coef(n));
  return s * x;
}

// erfc: 1 - erf by the series where |x| <= 1 (every smooth-flow interface
// state has |sqrt(lambda) U| well below 1); the library erfc elsewhere.
template <typename T> HGKS_FN T d_erfc(T x);
template <> HGKS_FN double d_erfc<double>(double x) {
  if (fabs(x) <= 1.0) return 1.0 - erf_series<18>(x);
  return erfc(x);
}
template <> HGKS_FN float d_erfc<float>(float x) {
  if (fabsf(x) <= 1.0f) return 1.0f - erf_series<11>(x);
  return erfcf(x);
}
template <typename T> HGKS_FN T d_sqrt(T x);
template <> HGKS_FN double d_sqrt<double>(double x) { return sqrt(x); }
template <> HGKS_FN float d_sqrt<float>(float x) { return sqrtf(x); }
// |x|.  For double and float the sign bit is cleared (an abs modifier on
// the instruction that uses it, or one bitwise and), where the comparison
// form costs a compare, a negation and two selects per double.
template <typename T> HGKS_FN T d_abs(T x) { return x < T(0) ? -x : x; }
template <> HGKS_FN double d_abs<double>(double x) { return __builtin_fabs(x); }
template <> HGKS_FN float d_abs<float>(float x) { return __builtin_fabsf(x); }

// The larger of a and b (one max instruction for double and float; the
// same value as the comparison form unless an argument is not a number).
template <typename T> HGKS_FN T d_max(T a, T b) { return a > b ? a : b; }
template <> HGKS_FN double d_max<double>(double a, double b) { return __builtin_fmax(a, b); }
template <> HGKS_FN float d_max<float>(float a, float b) { return __builtin_fmaxf(a, b); }

// Reciprocal of a nonzero finite x: the hardware estimate refined by
// Newton-Raphson steps r <- r + r (1 - x r) (two in double, one in float),
// at a fraction of the cost of a correctly rounded division.  On gfx950 the
// FP64 estimate is within 2^-24.4 of 1/x; one step leaves up to 11 ulp, two
// steps gave the correctly rounded 1/x on 4 million sampled inputs.
template <typename T> HGKS_FN T d_rcp(T x);
template <> HGKS_FN double d_rcp<double>(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
#else
  return 1.0 / x;
#endif
}
template <> HGKS_FN float d_rcp<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
#else
  return 1.0f / x;
#endif
}

// x plus x of lane l ^ MASK (MASK = 1 or 2) within each group of four
// lanes: a quad-permute DPP move per 32-bit half, which the vector unit
// does in the instruction itself (no LDS-unit round trip as for a general
// lane shuffle).
template <int MASK>
__device__ __forceinline__ float quad_xor_add(float x) {
  constexpr int ctrl = MASK == 1 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] / [2,3,0,1]
  return x + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), ctrl, 0xF, 0xF, false));
}

template <int MASK>
__device__ __forceinline__ double quad_xor_add(double x) {
  constexpr int ctrl = MASK == 1 ? 0xB1 : 0x4E;
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), ctrl, 0xF, 0xF, false);
  return x + __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Workgroups are dispatched round-robin over the eight XCDs (block b runs
// on XCD b % 8).  Remapping gives every XCD one contiguous range of logical
// blocks, so that neighbouring tiles share an L2.  The grid must hold
// 8 * ceil(nb / 8) blocks; logical ids >= nb do nothing.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb_padded) {
  const unsigned per = nb_padded >> 3;
  return (b & 7u) * per + (b >> 3);
}

}  // namespace hgks

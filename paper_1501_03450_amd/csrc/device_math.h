// Device math for the tracking kernels.
//
// FP64 transcendentals are multi-instruction sequences on CDNA, so the hot
// path evaluates the few functions it needs as truncated Taylor series on
// the small arguments the method produces, and falls back to the library
// function on the rare lane whose argument leaves the range where the
// truncation error stays below 2^-56 of the leading term.  Coefficients are
// reciprocal factorials and binomial ratios generated at compile time.
#pragma once

#include <hip/hip_runtime.h>

namespace st {

constexpr double inv_fact(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= (double)i;
  return 1.0 / f;
}

// Taylor coefficient of x^(2n+1) in asin(x): C(2n, n) / (4^n (2n + 1)).
constexpr double asin_coef(int n) {
  double c = 1.0;                      // C(2n, n) / 4^n, built as a product
  for (int i = 1; i <= n; ++i) c *= (double)(2 * i - 1) / (double)(2 * i);
  return c / (double)(2 * n + 1);
}

template <int K> struct IF { static constexpr double v = inv_fact(K); };
template <int K> struct AC { static constexpr double v = asin_coef(K); };

// cos(x) and sin(x)/x as series in t = x², NT terms each (u = -t), or
// cosh(x) and sinh(x)/x with u = +t.
template <int NT, int N = NT - 1>
struct Series {
  __device__ __forceinline__ static void eval(double u, double& c, double& s) {
    Series<NT, N - 1>::eval(u, c, s);
    c = fma(c, u, IF<2 * (NT - 1 - N)>::v);
    s = fma(s, u, IF<2 * (NT - 1 - N) + 1>::v);
  }
};
template <int NT>
struct Series<NT, 0> {
  __device__ __forceinline__ static void eval(double u, double& c, double& s) {
    c = IF<2 * (NT - 1)>::v;
    s = IF<2 * (NT - 1) + 1>::v;
  }
};

template <int NT>
__device__ __forceinline__ void cos_sinc_series(double t, double& c, double& s) {
  Series<NT>::eval(-t, c, s);
}
template <int NT>
__device__ __forceinline__ void cosh_sinhc_series(double t, double& c, double& s) {
  Series<NT>::eval(t, c, s);
}

// asin(x) for |x| <= kAsinPolyMax: 5 Taylor terms (through x^9); the first
// omitted term, C(10, 5)/(4^5 11) x^11, stays below 1.4e-17 |x| there.
constexpr double kAsinPolyMax = 0.03;
template <int N = 4>
struct AsinSeries {
  __device__ __forceinline__ static double eval(double t) {
    return fma(AsinSeries<N - 1>::eval(t), t, AC<4 - N>::v);
  }
};
template <>
struct AsinSeries<0> {
  __device__ __forceinline__ static double eval(double) { return AC<4>::v; }
};

// Beyond the series range the argument is reduced by halving, which keeps
// every lane on the same inline code (no calls, so no registers are spilled
// around them): with t = x², evaluate the series at t/4^k and apply the
// double-angle identities k times,
//   cos 2x = cos² x - t sinc² x,   sinc 2x = sinc x · cos x,
//   cosh 2x = cosh² x + t sinhc² x, sinhc 2x = sinhc x · cosh x.
// Non-finite or negative t gives NaN.
template <int NT, bool HYP>
__device__ __forceinline__ void halving_series(double t, double tmax, double& c, double& s) {
  int k = 0;
  while (t > tmax && k < 64) { t *= 0.25; ++k; }
  if (!(t <= tmax)) { c = s = __builtin_nan(""); return; }
  Series<NT>::eval(HYP ? t : -t, c, s);
  for (int i = 0; i < k; ++i) {
    const double c2 = HYP ? fma(t * s, s, c * c) : fma(-t * s, s, c * c);
    s = s * c;
    c = c2;
    t *= 4.0;
  }
}

// asin x = 2 asin(x / (sqrt 2 · sqrt(1 + sqrt(1 - x²)))) halves the argument.
__device__ __forceinline__ double asin_small(double x) {
  double scale = 1.0;
  int k = 0;
  while (!(fabs(x) <= kAsinPolyMax) && k < 8) {
    x = x * rsqrt(2.0 * (1.0 + sqrt(1.0 - x * x)));
    scale *= 2.0;
    ++k;
  }
  return scale * (x * AsinSeries<>::eval(x * x));
}

// 1/x and 1/sqrt(x): hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double hx = 0.5 * x;
  double e = fma(-hx * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-hx * y, y, 0.5);
  return fma(y, e, y);
}

// 1/sqrt(n2) for the squared norm of a quaternion that is a unit one up to
// the extrapolation's small change: with e = n2 - 1 (exact for n2 near 1),
// the binomial series 1 - e/2 + 3e²/8 - 5e³/16, whose first omitted term
// 35e⁴/128 stays below 3e-17 for |e| <= 1e-4; a larger |e| takes rsqrt_nr.
__device__ __forceinline__ double rsqrt_near_one(double n2) {
  const double e = n2 - 1.0;
  if (fabs(e) <= 1e-4) return fma(fma(fma(-0.3125, e, 0.375), e, -0.5), e, 1.0);
  return rsqrt_nr(n2);
}

// 1/sqrt(x) where it only scales a precession vector: one Newton step from
// the hardware estimate (measured within 2^-24.4 of 1/sqrt(x) on gfx950)
// leaves a relative error below 5e-15, i.e. below 1e-15 rad in the rotation
// of one slice edge (angles stay under 0.2 rad).  Orbit maps use rsqrt_nr.
__device__ __forceinline__ double rsqrt_omega(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-0.5 * x * y, y, 0.5);
  return fma(y, e, y);
}

// Quaternion terms of a rotation by θ = |ω|, ω = f Ω: with y = (θ/2)²,
// cos(θ/2) and sin(θ/2)/(θ/2).  NT series terms cover y <= ymax.
template <int NT>
__device__ __forceinline__ void rot_half_series(double y, double ymax, double& c, double& s) {
  if (y <= ymax) {
    cos_sinc_series<NT>(y, c, s);
  } else {
    halving_series<NT, false>(y, ymax, c, s);
  }
}

// The same with the vector factor sin(θ/2)/θ.
template <int NT>
__device__ __forceinline__ void rot_half_angle(double y, double ymax, double& c, double& sfac) {
  double s;
  rot_half_series<NT>(y, ymax, c, s);
  sfac = 0.5 * s;
}

}  // namespace st

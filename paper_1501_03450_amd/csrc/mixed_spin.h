// Single-precision spin arithmetic for the mixed-precision mode.
//
// The orbit and Ω stay in double precision.  The rotation of one slice edge
// is built in single precision in deviation form q = (1 - d, v) with
// d = 1 - cos(θ/2) = 2 sin²(θ/4) evaluated by its own series (no
// cancellation against 1), v = sin(θ/2)/θ · ω.  The running product of a
// Romberg level is a compensated pair (hi, lo) of single-precision
// quaternions: each update Q <- q ⊗ Q = Q + Δ with Δ = -d Q + (0, v) ⊗ Q is
// added with an error-free sum (Fast2Sum for the scalar part, 2Sum for the
// vector part), so the product keeps about twice the single-precision
// significand.  The tableau, the normalisation and the composition of
// element quaternions are done in double precision by the caller.
#pragma once

#include "device_math.h"
#include "fp64_maps.h"

namespace st {

struct QuatF {
  float w, x, y, z;
};

struct QuatC {          // compensated quaternion hi + lo
  QuatF hi, lo;
};

__device__ __forceinline__ QuatC qc_ident() { return {{1.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}}; }

// Rotation by θ = |ω| in deviation form: y = (θ/2)² (single), d = 1 - cos(θ/2),
// and s = sin(θ/2)/θ.  Five series terms hold single precision for y <= 1;
// beyond, the double-precision series is used for the lane.
__device__ __forceinline__ void rot_deviation_f32(double y, float& d, float& s) {
  if (y <= 1.0) {
    const float t = (float)y;
    // d = Σ_{n>=1} (-1)^(n+1) t^n/(2n)!,  s = ½ Σ_{n>=0} (-t)^n/(2n+1)!
    float dd = fmaf(t, -(float)IF<10>::v, (float)IF<8>::v);
    dd = fmaf(t, dd, -(float)IF<6>::v);
    dd = fmaf(t, dd, (float)IF<4>::v);
    dd = fmaf(t, dd, -(float)IF<2>::v);
    d = -t * dd;
    float ss = fmaf(t, (float)IF<9>::v, -(float)IF<7>::v);
    ss = fmaf(t, ss, (float)IF<5>::v);
    ss = fmaf(t, ss, -(float)IF<3>::v);
    ss = fmaf(t, ss, 1.0f);
    s = 0.5f * ss;
  } else {
    double c, sf;
    halving_series<8, false>(y, 0.36, c, sf);
    d = (float)(1.0 - c);
    s = (float)(0.5 * sf);
  }
}

// (1 - d, v)² = (1 - (2d - d² + |v|²), 2 (1 - d) v): twice the angle.
__device__ __forceinline__ void dev_square(float& d, float& vx, float& vy, float& vz) {
  const float v2 = fmaf(vx, vx, fmaf(vy, vy, vz * vz));
  const float two_omd = 2.0f * (1.0f - d);
  d = fmaf(-d, d, fmaf(2.0f, d, v2));
  vx *= two_omd;
  vy *= two_omd;
  vz *= two_omd;
}

// Fast2Sum of the running hi with an increment, error carried into lo: exact
// only when |hi| >= |inc|, which holds for the scalar part (it starts at 1
// and the increments are small rotations).
__device__ __forceinline__ void comp_add_fast(float& hi, float& lo, float inc) {
  const float s = hi + inc;
  const float e = inc - (s - hi);
  hi = s;
  lo += e;
}

// 2Sum (Knuth): the rounding error of hi + inc for any magnitudes, for the
// vector part, which starts at 0 and is smaller than the first increments.
__device__ __forceinline__ void comp_add(float& hi, float& lo, float inc) {
  const float s = hi + inc;
  const float b = s - hi;
  const float e = (hi - (s - b)) + (inc - b);
  hi = s;
  lo += e;
}

// Q <- (1 - d, v) ⊗ Q, compensated.
__device__ __forceinline__ void qc_update(QuatC& Q, float d, float vx, float vy, float vz) {
  const QuatF& h = Q.hi;
  // (0, v) ⊗ h = (-v·h_v, h_w v + v × h_v), then -d h
  float dw = -fmaf(vx, h.x, fmaf(vy, h.y, vz * h.z));
  float dx = fmaf(h.w, vx, fmaf(vy, h.z, -vz * h.y));
  float dy = fmaf(h.w, vy, fmaf(vz, h.x, -vx * h.z));
  float dz = fmaf(h.w, vz, fmaf(vx, h.y, -vy * h.x));
  dw = fmaf(-d, h.w, dw);
  dx = fmaf(-d, h.x, dx);
  dy = fmaf(-d, h.y, dy);
  dz = fmaf(-d, h.z, dz);
  comp_add_fast(Q.hi.w, Q.lo.w, dw);
  comp_add(Q.hi.x, Q.lo.x, dx);
  comp_add(Q.hi.y, Q.lo.y, dy);
  comp_add(Q.hi.z, Q.lo.z, dz);
}

__device__ __forceinline__ Quat qc_to_double(const QuatC& Q) {
  return {(double)Q.hi.w + (double)Q.lo.w, (double)Q.hi.x + (double)Q.lo.x,
          (double)Q.hi.y + (double)Q.lo.y, (double)Q.hi.z + (double)Q.lo.z};
}

}  // namespace st

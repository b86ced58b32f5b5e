// Orbit maps, the T-BMT precession vector and quaternion algebra in double
// precision, one lane per particle.
//
// The maps are the exact flows of §3 evaluated in forms that avoid
// cancellation.  Pt is constant in every element of this model (no RF), so
// every quantity that depends only on Pt is computed once per particle.
#pragma once

#include "device_math.h"
#include "lattice_table.h"

namespace st {

struct Quat {
  double w, x, y, z;
};

__device__ __forceinline__ Quat qident() { return {1.0, 0.0, 0.0, 0.0}; }

// Hamilton product a ⊗ b (i j = k).
__device__ __forceinline__ Quat qmul(const Quat& a, const Quat& b) {
  Quat r;
  r.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
  r.x = a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y;
  r.y = a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x;
  r.z = a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w;
  return r;
}

// q ⊗ q for a rotation quaternion: the rotation about the same axis by
// twice the angle, (w² - |v|², 2 w v).
__device__ __forceinline__ Quat qsquare(const Quat& q) {
  const double tw = 2.0 * q.w;
  return {fma(q.w, q.w, -fma(q.x, q.x, fma(q.y, q.y, q.z * q.z))), tw * q.x, tw * q.y, tw * q.z};
}

// One Romberg step on quaternions: (c A - B) / (c - 1).
__device__ __forceinline__ Quat qextrapolate(const Quat& A, const Quat& B, double c) {
  const double inv = 1.0 / (c - 1.0);
  return {fma(c, A.w, -B.w) * inv, fma(c, A.x, -B.x) * inv, fma(c, A.y, -B.y) * inv,
          fma(c, A.z, -B.z) * inv};
}

// S <- q S q*: t = 2 v × S, S += w t + v × t.
__device__ __forceinline__ void qrotate(const Quat& q, double& sx, double& sy, double& sz) {
  double tx = 2.0 * (q.y * sz - q.z * sy);
  double ty = 2.0 * (q.z * sx - q.x * sz);
  double tz = 2.0 * (q.x * sy - q.y * sx);
  sx += q.w * tx + (q.y * tz - q.z * ty);
  sy += q.w * ty + (q.z * tx - q.x * tz);
  sz += q.w * tz + (q.x * ty - q.y * tx);
}

// Quantities of one particle that depend on Pt only (eq. pt, eq. ps,
// eq. quadSclP): P² = 1 + 2Pt/β0 + Pt², γ = γ0 (1 + β0 Pt), and the T-BMT
// factors a1 = 1 + Gγ, a2 = G(γ - 1).  The factors used at every slice edge
// stay in registers; the rarer ones cost one instruction each where they are
// used.
struct Particle {
  double Pt;
  double c3;       // P² - 1 = 2Pt/β0 + Pt², kept exactly (P² itself rounds it)
  double invP;
  double dib;      // 1/β - 1/β0
  double invP2_, invbeta_, a1_, a2_;
  // beam constants (kernel arguments, uniform)
  double ib0, beta0, ig2;

  __device__ __forceinline__ double P2() const { return 1.0 + c3; }
  __device__ __forceinline__ double P() const { return (1.0 + c3) * invP; }
  __device__ __forceinline__ double invP2() const { return invP2_; }
  __device__ __forceinline__ double c1() const { return c3 * ig2; }           // P² - (1 + β0 Pt)²
  __device__ __forceinline__ double c2() const { return fma(beta0, Pt, 1.0); }  // 1 + β0 Pt
  __device__ __forceinline__ double ib() const { return ib0 + Pt; }           // 1/β0 + Pt
  __device__ __forceinline__ double invbeta() const { return invbeta_; }      // (1/β0 + Pt)/P
  __device__ __forceinline__ double a1() const { return a1_; }                // 1 + Gγ
  __device__ __forceinline__ double a2() const { return a2_; }                // G(γ - 1)
};

__device__ __forceinline__ Particle make_particle(double Pt, const TrackArgs& a) {
  Particle p;
  p.Pt = Pt;
  p.ib0 = a.inv_beta0;
  p.beta0 = a.beta0;
  p.ig2 = a.inv_gamma0_sq;
  const double Gg0b0 = a.G * a.gamma0 * a.beta0;
  p.a1_ = fma(Gg0b0, Pt, fma(a.G, a.gamma0, 1.0));
  p.a2_ = fma(Gg0b0, Pt, a.G * (a.gamma0 - 1.0));
  p.c3 = Pt * fma(2.0, a.inv_beta0, Pt);
  p.invP = rsqrt_nr(p.P2());
  p.invP2_ = p.invP * p.invP;
  p.invbeta_ = (a.inv_beta0 + Pt) * p.invP;
  p.dib = -p.c1() * a.inv_beta0 * p.invP * rcp_nr(p.c2() + p.P());
  return p;
}

// With u = (Px² + Py²)/P², P/Ps = (1 - u)^(-1/2); g = P/Ps - 1 - u/2 is the
// binomial series Σ_{k≥2} C(2k, k) (u/4)^k.  For u ≤ 2^-12 its terms through
// u^4 leave less than 3e-19 (the first omitted one is 63/256 u^5); callers
// take a closed form beyond.  Transverse momenta of the tracked bunches keep
// u near 1e-8.
constexpr double kSeriesMaxU = 1.0 / 4096.0;
__device__ __forceinline__ double series_g(double u) {
  constexpr double c2 = 3.0 / 8.0, c3 = 5.0 / 16.0, c4 = 35.0 / 128.0;
  return (u * u) * fma(u, fma(u, c4, c3), c2);
}

// Exact drift of length L (flow of -Ps + Pt/β0).  With e = P/Ps - 1 =
// u/2 + g (series above), X and Y advance by L P(x,y) (1 + e)/P, and the
// flight-time change L/β0 - L(1/β0 + Pt)/Ps is -L (1/β - 1/β0) - L e/β,
// free of cancellation.  A lane with u > 2^-12 evaluates it as
// L (c1 - Px² - Py²) / (β0 Ps (Ps + 1 + β0 Pt)).
__device__ __forceinline__ void drift(double L, double& X, double Px, double& Y, double Py,
                                      double& T, const Particle& p, double inv_beta0) {
  const double pp = fma(Px, Px, Py * Py);
  const double u = pp * p.invP2();
  if (u <= kSeriesMaxU) {
    const double e = fma(u, 0.5, series_g(u));
    const double r = fma(p.invP, e, p.invP);       // 1/Ps
    X = fma(L * Px, r, X);
    Y = fma(L * Py, r, Y);
    T = fma(-L, fma(p.invbeta(), e, p.dib), T);
  } else {
    const double ps2 = p.P2() - pp;
    const double r = rsqrt_nr(ps2);
    const double ps = ps2 * r;
    X = fma(L * Px, r, X);
    Y = fma(L * Py, r, Y);
    T = fma(L * (p.c1() - pp) * r * inv_beta0, rcp_nr(ps + p.c2()), T);
  }
}

// Precession vector of eq. t-bmt.so for a field b = (bx, by, 0) without
// curvature (quadrupoles, thin multipoles):
// Ω = -(1/Ps) [a1 b - a2 (ũ·b)/P² ũ], ũ = (Px, Py, Ps).  r = 1/Ps.
__device__ __forceinline__ void omega_straight(double bx, double by, double Px, double Py,
                                               double r, const Particle& p,
                                               double& ox, double& oy, double& oz) {
  const double a1 = p.a1();
  double k = p.a2() * fma(Px, bx, Py * by) * p.invP2();
  ox = -r * fma(a1, bx, -k * Px);
  oy = -r * fma(a1, by, -k * Py);
  oz = k;
}

// Precession vector in a sector bend, b = (0, ηh, 0), with the frame term h ŷ.
__device__ __forceinline__ void omega_dipole(double h, double eta_h, double X, double Px, double Py,
                                             double r, const Particle& p,
                                             double& ox, double& oy, double& oz) {
  double w = fma(h, X, 1.0) * eta_h;
  double g = w * r;
  double a2py = p.a2() * Py * p.invP2();
  ox = g * a2py * Px;
  oy = fma(-g, fma(-a2py, Py, p.a1()), h);
  oz = w * a2py;
}

__device__ __forceinline__ void omega_bend(const BendParams& e, double X, double Px, double Py,
                                           double r, const Particle& p,
                                           double& ox, double& oy, double& oz) {
  omega_dipole(e.h, e.eta_h, X, Px, Py, r, p, ox, oy, oz);
}

// Drift of the curved frame over half a drift-kick slice (§3.6 eq. teapotD),
// a straight line seen from the rotating frame.  With u = Px/Ps, a = h ds/2
// and D = 1 - u tan a, the printed forms are evaluated without their
// cancellations:
//   X(s)  = [X sec a + (sec a - 1)/h + u tan(a)/h] / D
//   path  = (1/h + X) tan(a) / D
//   ΔT    = (ds/2)/β0 - (1/β0 + Pt) path/Ps           (the Pt/β0 term of
//           eq. generalH adds (ds/2)/β0)
//         = (1/β0) { [(ds/2 - tan(a)/h) - tan(a)(u ds/2 + X)] / D
//                    + path (Ps² - (1 + β0 Pt)²) / (Ps (Ps + 1 + β0 Pt)) }.
__device__ __forceinline__ void teapot_drift(const TeapotParams& t, double& X, double& Px, double& Y,
                                             double Py, double& T, const Particle& p) {
  const double pp = fma(Px, Px, Py * Py);
  const double ps2 = p.P2() - pp;
  const double r = rsqrt_nr(ps2);
  const double ps = ps2 * r;
  const double u = Px * r;
  const double inv_den = rcp_nr(fma(-u, t.tn, 1.0));
  const double path = fma(X, t.tn, t.tn_h) * inv_den;
  const double short_path = fma(-t.tn, fma(t.half, u, X), t.d0) * inv_den;   // ds/2 - path
  const double slow = path * (p.c1() - pp) * r * rcp_nr(ps + p.c2());
  T = fma(short_path + slow, p.ib0, T);
  X = fma(X, t.sec, fma(u, t.tn_h, t.omc_h)) * inv_den;
  Px = fma(Px, t.c, ps * t.sn);
  Y = fma(Py * r, path, Y);
}

// Dipole kick of a TEAPOT bend over a length len: Px -= ηh (1 + hX) len.
__device__ __forceinline__ void teapot_kick(const TeapotParams& t, double len, double X, double& Px) {
  Px = fma(-t.eta_h * len, fma(t.h, X, 1.0), Px);
}

// Solenoid body (§3.7 eq. solenoid).  The kinetic transverse momentum
// k = (Px + ηY, Py - ηX) keeps its length along the exact flow, so Ps,
// κ = η/Ps, cos(κ ds), sin(κ ds) and the flight-time step are constants of
// the particle in the element.
struct SolState {
  double ps, r;     // Ps and 1/Ps (eq. Hsolenoid)
  double c, sn;     // cos and sin of κ ds
  double dT;        // T step per slice: ds/β0 - (1/β0 + Pt) ds/Ps, cancellation-free
};

template <int NT>
__device__ __forceinline__ SolState sol_state(const SolenoidParams& sp, double X, double Px,
                                              double Y, double Py, const Particle& p, double ymax,
                                              double inv_beta0) {
  SolState st;
  const double kx = fma(sp.eta, Y, Px), ky = fma(-sp.eta, X, Py);
  const double kk = fma(kx, kx, ky * ky);
  const double ps2 = p.P2() - kk;
  st.r = rsqrt_nr(ps2);
  st.ps = ps2 * st.r;
  const double phi = sp.eta * st.r * sp.ds;
  double sfac;
  rot_half_angle<NT>(phi * phi, ymax, st.c, sfac);   // cos φ and sin(φ)/(2φ)
  st.sn = 2.0 * phi * sfac;
  st.dT = sp.ds * (p.c1() - kk) * st.r * inv_beta0 * rcp_nr(st.ps + p.c2());
  return st;
}

__device__ __forceinline__ void solenoid_slice(const SolenoidParams& sp, const SolState& st,
                                               double& X, double& Px, double& Y, double& Py,
                                               double& T) {
  // R2: rotation of (X, Y) and (Px, Py) by κ ds; R1: focusing rotations
  const double X2 = fma(st.c, X, st.sn * Y), Y2 = fma(-st.sn, X, st.c * Y);
  const double Px2 = fma(st.c, Px, st.sn * Py), Py2 = fma(-st.sn, Px, st.c * Py);
  const double sie = st.sn * sp.inv_eta, es = sp.eta * st.sn;
  X = fma(st.c, X2, sie * Px2);
  Px = fma(-es, X2, st.c * Px2);
  Y = fma(st.c, Y2, sie * Py2);
  Py = fma(-es, Y2, st.c * Py2);
  T += st.dT;
}

// Precession vector in the solenoid body: b = (0, 0, ks), û from the kinetic
// momentum (eq. mgVSol).
__device__ __forceinline__ void omega_solenoid(const SolenoidParams& sp, const SolState& st,
                                               double X, double Px, double Y, double Py,
                                               const Particle& p, double& ox, double& oy,
                                               double& oz) {
  const double kx = fma(sp.eta, Y, Px), ky = fma(-sp.eta, X, Py);
  const double g = p.a2() * p.invP2();
  ox = g * sp.ks * kx;
  oy = g * sp.ks * ky;
  oz = -sp.ks * st.r * fma(-g * st.ps, st.ps, p.a1());   // -(ks/Ps)(a1 - a2 Ps²/P²)
}

// Thin-pancake fringe spin kick (§4.4 eq. solFringe), sign +1 at the
// entrance and -1 at the exit, with the kinetic momentum at half the vector
// potential.  Returns ω.
__device__ __forceinline__ void solenoid_fringe(const SolenoidParams& sp, double sign, double X,
                                                double Px, double Y, double Py, const Particle& p,
                                                double& wx, double& wy, double& wz) {
  const double kx = fma(sp.eta_q, Y, Px), ky = fma(-sp.eta_q, X, Py);
  const double ps2 = p.P2() - fma(kx, kx, ky * ky);
  const double r = rsqrt_nr(ps2);
  const double ps = ps2 * r;
  const double f = sign * sp.eta * r;
  const double d = p.a2() * fma(X, Px, Y * Py) * p.invP2();
  wx = f * fma(p.a1(), X, -d * kx);
  wy = f * fma(p.a1(), Y, -d * ky);
  wz = -f * d * ps;
}

// Rectangular bend (§3.2).  Frame rotation by a face angle (the flow of
// eq. Hprot; T decreases for X > 0, which reaches the rotated face later).
__device__ __forceinline__ void rbend_rotate(const RbendFace& rb, double& X, double& Px, double& Y,
                                             double Py, double& T, const Particle& p) {
  const double ps2 = p.P2() - fma(Px, Px, Py * Py);
  const double r = rsqrt_nr(ps2);
  const double ps = ps2 * r;
  const double inv_den = rcp_nr(fma(-Px * r, rb.tn, 1.0));
  const double xt = X * rb.tn * inv_den;
  Y = fma(Py * r, xt, Y);
  T = fma(-p.ib() * r, xt, T);
  X = X * rb.sec * inv_den;
  Px = fma(Px, rb.c, ps * (rb.tn * rb.c));
}

// Thin dipole fringe without gap correction (eq. dipolefringe), sign +1 at
// the entrance and -1 at the exit.
__device__ __forceinline__ void rbend_fringe(const RbendParams& rb, double sign, double& X,
                                             double Px, double& Y, double& Py, double& T,
                                             const Particle& p) {
  const double ps2 = p.P2() - fma(Px, Px, Py * Py);
  const double r = rsqrt_nr(ps2);
  const double xp = Px * r, yp = Py * r;
  const double iq = rcp_nr(fma(yp, yp, 1.0));
  const double sf = sign * rb.fb;
  const double a = sf * xp * yp * iq * 2.0 * Y;
  const double Yf = 2.0 * Y * rcp_nr(1.0 + sqrt(1.0 + a));
  const double Yf2 = Yf * Yf;
  const double xy = xp * yp * iq;
  X = fma(0.5 * sf * r * (fma(xp, xp, 1.0) * iq - 2.0 * xy * xy), Yf2, X);
  Py = fma(-sf * xp * iq, Yf, Py);
  T = fma(-sf * p.ib() * xp * 0.5 * r * r * fma(-yp, yp, 1.0) * iq * iq, Yf2, T);
  Y = Yf;
}

// Body over a length s (eq. rbend), Pα² = P² - Py²:  Px(s) = Px - s fb,
// X += ρb [W(s) - W] = s (Px + Px(s)) / (W + W(s)), and the bending
// angle D = asin(Px/Pα) - asin(Px(s)/Pα) = asin((Px W(s) - Px(s) W)/Pα²);
// no reference flight time here (the element adds L_arc/β0).
__device__ __forceinline__ void rbend_body(const RbendParams& rb, double s, double& X, double& Px,
                                           double& Y, double Py, double& T, const Particle& p) {
  const double Pa2 = p.P2() - Py * Py;
  const double Px1 = fma(-s, rb.fb, Px);
  const double w02 = fma(-Px, Px, Pa2), w12 = fma(-Px1, Px1, Pa2);
  const double r0 = rsqrt_nr(w02), r1 = rsqrt_nr(w12);
  const double W0 = w02 * r0, W1 = w12 * r1;
  X = fma(s * (Px + Px1), rcp_nr(W0 + W1), X);
  const double D = asin_small(fma(Px, W1, -Px1 * W0) * rcp_nr(Pa2));
  Y = fma(Py * rb.rhob, D, Y);
  T = fma(-p.ib() * rb.rhob, D, T);
  Px = Px1;
}

__device__ __forceinline__ void teapot_slice(const TeapotParams& t, double& X, double& Px, double& Y,
                                             double Py, double& T, const Particle& p) {
  teapot_drift(t, X, Px, Y, Py, T, p);
  teapot_kick(t, t.ds, X, Px);
  teapot_drift(t, X, Px, Y, Py, T, p);
}

// Constants of one particle for the steps of a sector bend: the flight-time
// change of a step is c0 - ibh D, with c0 = (1 - 1/η) s/β0 - Pt s/η and
// ibh = (1/β0 + Pt)/(η h).
struct BendLane {
  double c0, ibh;
};

__device__ __forceinline__ BendLane bend_lane(const BendParams& e, const BendStep& k,
                                              const Particle& p) {
  return {fma(-p.Pt, k.s_eta, k.tconst), p.ib() * e.inv_eta_h};
}

// One step of the exact sector bend over the slice length (§3.1 eq. sbend),
// from the state (X, Px) with Ps = W0 to the next slice edge.  Pα² = P² - Py²
// is passed in; W1 = sqrt(Pα² - Px(s)²) is returned through W0/r0 (it is Ps
// at the new edge) and wme = W - η is carried from edge to edge.  X(s) is
// evaluated as
//   X cos(hs) + [(W1 - W0) + (W0 - η)(1 - cos hs) + Px sin(hs)] / (η h),
// with W1 - W0 = (Px - Px(s))(Px + Px(s))/(W0 + W1), and
// asin(Px/Pα) - asin(Px(s)/Pα) = asin((Px W1 - Px(s) W0)/Pα²): both
// algebraically identical to the printed forms and free of cancellation.
// YT = false leaves Y and T alone: they enter neither the next step nor Ω,
// and the angle differences of the steps telescope, so a caller that steps
// through a whole bend applies bend_yt once with the entrance and exit
// values instead.
template <bool YT = true>
__device__ __forceinline__ void bend_step(const BendParams& e, const BendStep& k,
                                          const BendLane& bl, double& X, double& Px, double Py,
                                          double& Y, double& T, double& W0, double& r0,
                                          double& wme, double Pa2, double invPa2) {
  double A = fma(-e.eta_h, X, wme);
  double px1 = fma(Px, k.cs, A * k.sn);
  double ps2n = fma(-px1, px1, Pa2);
  double r1 = rsqrt_nr(ps2n);
  double W1 = ps2n * r1;
  double dW = (Px - px1) * (Px + px1) * rcp_nr(W0 + W1);
  double X1 = fma(X, k.cs, fma(wme, k.omc, fma(Px, k.sn, dW)) * e.inv_eta_h);
  if constexpr (YT) {
    double D = asin_small(fma(Px, W1, -px1 * W0) * invPa2);
    Y = fma(Py, fma(D, e.inv_eta_h, k.s_eta), Y);
    T += fma(-bl.ibh, D, bl.c0);
  }
  wme += dW;
  X = X1;
  Px = px1;
  W0 = W1;
  r0 = r1;
}

// Y and T over a stretch of the bend of length k (BendStep) from the
// horizontal momenta and Ps at its ends: the same angle difference and
// updates as one step, bl being bend_lane(e, k, p).
__device__ __forceinline__ void bend_yt(const BendParams& e, const BendStep& k, const BendLane& bl,
                                        double Px0, double W0, double Px1, double W1, double Py,
                                        double& Y, double& T, double invPa2) {
  const double D = asin_small(fma(Px0, W1, -Px1 * W0) * invPa2);
  Y = fma(Py, fma(D, e.inv_eta_h, k.s_eta), Y);
  T += fma(-bl.ibh, D, bl.c0);
}

// Matrix-kick quadrupole constants of one particle (§3.3 eq. quadL over
// s = ds/2): κ² = |k1|/P; cos, sin(κs)/κ, κP sin(κs) and their hyperbolic
// twins, all functions of (κs)² = |k1| s²/P.  The flight-time brace of
// eq. quadL is a quadratic form in (X, Px, Y, Py) at the entrance of the
// step; its six coefficients, with the factor -1/β = -(1/β0 + Pt)/P
// folded in, are constants of the particle in the element.
struct MKConst {
  double cf, sfP, kf;    // focusing plane:   cos κs, sin κs /(κ P), κ P sin κs
  double cd, sdP, kd;    // defocusing plane: cosh κs, sinh κs /(κ P), κ P sinh κs
  double tpx, tpy;       // ΔT = Px (tpx Px + txp X) + Py (tpy Py + typ Y)
  double txx, tyy;       //      + txx X² + tyy Y²
  double txp, typ;
};

__device__ __forceinline__ MKConst mk_const(const QuadParams& e, const Particle& p) {
  MKConst m;
  double t = e.kabs_hds2 * p.invP;       // (κ s)²
  double kabs = fabs(e.k1);
  double C, Sc, Ch, Sh;
  if (t <= 0.04) {
    cos_sinc_series<7>(t, C, Sc);
    cosh_sinhc_series<7>(t, Ch, Sh);
  } else {
    halving_series<7, false>(t, 0.04, C, Sc);
    halving_series<7, true>(t, 0.04, Ch, Sh);
  }
  const double hs = e.hds;
  const double sf = hs * Sc, sd = hs * Sh;
  m.cf = C;  m.sfP = sf * p.invP;  m.kf = kabs * sf;
  m.cd = Ch; m.sdP = sd * p.invP;  m.kd = kabs * sd;
  const double kap2 = kabs * p.invP;
  // brace = A1 (px² + py² + κ²X² - κ²Y²) + A2 (px² - κ²X²) + A3 (py² + κ²Y²)
  //         - A4 X px + A5 Y py,  px = Px/P, py = Py/P,
  // A1 = s/4, A2 = sf cf/4, A3 = sd cd/4, A4 = κ² sf²/2, A5 = κ² sd²/2
  const double A1 = 0.25 * hs, A2 = 0.25 * sf * C, A3 = 0.25 * sd * Ch;
  const double nib = -p.invbeta();       // -1/β
  const double nibP = nib * p.invP;
  m.tpx = nibP * p.invP * (A1 + A2);
  m.tpy = nibP * p.invP * (A1 + A3);
  m.txx = nib * kap2 * (A1 - A2);
  m.tyy = nib * kap2 * (A3 - A1);
  m.txp = -nibP * (0.5 * kap2 * sf * sf);
  m.typ = nibP * (0.5 * kap2 * sd * sd);
  return m;
}

// Linear part of the matrix-kick quadrupole over ds/2 in (focusing,
// defocusing) coordinates.
__device__ __forceinline__ void mk_linear(const MKConst& m, double& xf, double& pxf, double& yd,
                                          double& pyd, double& T, const Particle&) {
  const double x0 = xf, y0 = yd, p0 = pxf, q0 = pyd;
  const double dT = fma(p0, fma(m.tpx, p0, m.txp * x0),
                        fma(q0, fma(m.tpy, q0, m.typ * y0), fma(m.txx * x0, x0, m.tyy * y0 * y0)));
  xf = fma(x0, m.cf, p0 * m.sfP);
  pxf = fma(p0, m.cf, -x0 * m.kf);
  yd = fma(y0, m.cd, q0 * m.sdP);
  pyd = fma(q0, m.cd, y0 * m.kd);
  T += dT;
}

// Nonlinear "kick of positions" over ds (§3.3 eq. quadNL).  With
// u = (Px² + Py²)/P², 1/Ps - 1/P = (u/2 + g)/P and the flight-time term is
// -ds/β g - ds (1/β - 1/β0), g = P/Ps - 1 - u/2 (series_g); a lane
// with larger angles takes the closed form g = u²(2 + ρ)/(2ρ(1 + ρ)²),
// ρ = Ps/P.
__device__ __forceinline__ void mk_nonlinear(double ds, double& X, double Px, double& Y,
                                             double Py, double& T, const Particle& p) {
  const double pp = fma(Px, Px, Py * Py);
  const double u = pp * p.invP2();
  double g, d;
  if (u <= kSeriesMaxU) {
    g = series_g(u);
    d = fma(u, 0.5, g) * p.invP;         // 1/Ps - 1/P
  } else {
    const double ps2 = p.P2() - pp;
    const double r = rsqrt_nr(ps2);
    d = r - p.invP;
    const double rho = ps2 * r * p.invP;
    const double opr = 1.0 + rho;
    g = u * u * (2.0 + rho) * (p.P() * r) * 0.5 * rcp_nr(opr * opr);
  }
  X = fma(ds * Px, d, X);
  Y = fma(ds * Py, d, Y);
  T = T - ds * fma(p.invbeta(), g, p.dib);
}

}  // namespace st

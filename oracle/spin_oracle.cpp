// TEST INFRASTRUCTURE — not part of the product path.
//
// A plain, slow CPU implementation of the spin–orbit tracking method of
// D. T. Abell, D. Meiser, V. H. Ranjbar and D. P. Barber, "Accurate and
// efficient spin integration for particle accelerators" (2015).  It exists to
// check the GPU library; only the tests, the smoke check and the CPU-baseline
// leg of the benchmark load it.  It shares no code with the GPU library.
//
// Every map is the paper's own formula, written in its order and notation,
// one particle at a time.  The scalar type is a template parameter:
//   long double  x87 extended precision: the parity reference.  The printed
//                sector-bend X(s) and the drift flight time lose up to
//                log10(1/(h·|X|)) digits to cancellation; 64-bit mantissas
//                keep that loss below 1e-16 of the coordinate.
//   double       the CPU baseline that is timed next to the GPU.
//   Dual         forward-mode derivatives: the one-turn Jacobian.
//   Counted      a double that counts its operations: the flop model.
//
// Coordinates (§2.1, eq. psvars): z = (X, Px, Y, Py, T, Pt); Px, Py scaled by
// p0 = m γ0 β0 c, T = -c Δt, Pt = (E - E0)/(p0 c).
// Spin (§2.2): dS/ds = Ω × S with Ω from eq. t-bmt.so.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace oracle {

// ---------------------------------------------------------------------------
// Scalar types
// ---------------------------------------------------------------------------

// Forward-mode dual number with ND derivative components.
template <class B, int ND>
struct Dual {
  B v;
  B d[ND];
  Dual() : v(0) { for (int i = 0; i < ND; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < ND; ++i) d[i] = 0; }
  Dual(long double x) : v(x) { for (int i = 0; i < ND; ++i) d[i] = 0; }
  Dual(int x) : v(x) { for (int i = 0; i < ND; ++i) d[i] = 0; }
};
template <class B, int ND> Dual<B, ND> operator+(const Dual<B, ND>& a, const Dual<B, ND>& b) {
  Dual<B, ND> r; r.v = a.v + b.v; for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <class B, int ND> Dual<B, ND> operator-(const Dual<B, ND>& a, const Dual<B, ND>& b) {
  Dual<B, ND> r; r.v = a.v - b.v; for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <class B, int ND> Dual<B, ND> operator-(const Dual<B, ND>& a) {
  Dual<B, ND> r; r.v = -a.v; for (int i = 0; i < ND; ++i) r.d[i] = -a.d[i]; return r; }
template <class B, int ND> Dual<B, ND> operator*(const Dual<B, ND>& a, const Dual<B, ND>& b) {
  Dual<B, ND> r; r.v = a.v * b.v; for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <class B, int ND> Dual<B, ND> operator/(const Dual<B, ND>& a, const Dual<B, ND>& b) {
  Dual<B, ND> r; r.v = a.v / b.v;
  for (int i = 0; i < ND; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v; return r; }
template <class B, int ND> Dual<B, ND>& operator+=(Dual<B, ND>& a, const Dual<B, ND>& b) { a = a + b; return a; }
template <class B, int ND> Dual<B, ND>& operator-=(Dual<B, ND>& a, const Dual<B, ND>& b) { a = a - b; return a; }
template <class B, int ND> Dual<B, ND>& operator*=(Dual<B, ND>& a, const Dual<B, ND>& b) { a = a * b; return a; }
template <class B, int ND> bool operator==(const Dual<B, ND>& a, const Dual<B, ND>& b) { return a.v == b.v; }
template <class B, int ND> bool operator<(const Dual<B, ND>& a, const Dual<B, ND>& b) { return a.v < b.v; }
template <class B, int ND> bool operator>(const Dual<B, ND>& a, const Dual<B, ND>& b) { return a.v > b.v; }
template <class B, int ND> bool operator<=(const Dual<B, ND>& a, const Dual<B, ND>& b) { return a.v <= b.v; }
template <class B, int ND> Dual<B, ND> chain(const Dual<B, ND>& a, B f, B df) {
  Dual<B, ND> r; r.v = f; for (int i = 0; i < ND; ++i) r.d[i] = df * a.d[i]; return r; }
template <class B, int ND> Dual<B, ND> sqrt(const Dual<B, ND>& a) {
  B s = std::sqrt(a.v); return chain(a, s, B(0.5) / s); }
template <class B, int ND> Dual<B, ND> sin(const Dual<B, ND>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <class B, int ND> Dual<B, ND> cos(const Dual<B, ND>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <class B, int ND> Dual<B, ND> sinh(const Dual<B, ND>& a) { return chain(a, std::sinh(a.v), std::cosh(a.v)); }
template <class B, int ND> Dual<B, ND> cosh(const Dual<B, ND>& a) { return chain(a, std::cosh(a.v), std::sinh(a.v)); }
template <class B, int ND> Dual<B, ND> asin(const Dual<B, ND>& a) {
  return chain(a, std::asin(a.v), B(1) / std::sqrt(B(1) - a.v * a.v)); }
template <class B, int ND> bool finite_(const Dual<B, ND>& a) { return std::isfinite(a.v); }
template <class B, int ND> B value_(const Dual<B, ND>& a) { return a.v; }

// A double that counts the floating-point operations applied to it.
struct Counts { long long add, mul, div, sqrt, sincos, asin, hyp; };
inline Counts g_counts;
struct Counted {
  double v;
  Counted() : v(0) {}
  Counted(double x) : v(x) {}
  Counted(long double x) : v(double(x)) {}
  Counted(int x) : v(x) {}
};
inline Counted operator+(Counted a, Counted b) { ++g_counts.add; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { ++g_counts.add; return Counted(a.v - b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline Counted operator*(Counted a, Counted b) { ++g_counts.mul; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { ++g_counts.div; return Counted(a.v / b.v); }
inline Counted& operator+=(Counted& a, Counted b) { a = a + b; return a; }
inline Counted& operator-=(Counted& a, Counted b) { a = a - b; return a; }
inline Counted& operator*=(Counted& a, Counted b) { a = a * b; return a; }
inline bool operator==(Counted a, Counted b) { return a.v == b.v; }
inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
inline Counted sqrt(Counted a) { ++g_counts.sqrt; return Counted(std::sqrt(a.v)); }
inline Counted sin(Counted a) { ++g_counts.sincos; return Counted(std::sin(a.v)); }
inline Counted cos(Counted a) { ++g_counts.sincos; return Counted(std::cos(a.v)); }
inline Counted sinh(Counted a) { ++g_counts.hyp; return Counted(std::sinh(a.v)); }
inline Counted cosh(Counted a) { ++g_counts.hyp; return Counted(std::cosh(a.v)); }
inline Counted asin(Counted a) { ++g_counts.asin; return Counted(std::asin(a.v)); }
inline bool finite_(Counted a) { return std::isfinite(a.v); }
inline double value_(Counted a) { return a.v; }

inline bool finite_(double a) { return std::isfinite(a); }
inline bool finite_(long double a) { return std::isfinite(a); }
inline double value_(double a) { return a; }
inline long double value_(long double a) { return a; }

// ---------------------------------------------------------------------------
// Lattice and beam
// ---------------------------------------------------------------------------

enum Kind : int32_t { MARKER = 0, DRIFT = 1, SBEND = 2, QUAD = 3, THIN = 4, SNAKE = 5, SOLENOID = 6,
                      RBEND = 7 };
enum Method : int32_t { EXACT = 0, DKD = 1, MK = 2, TEAPOT = 3, DKD4 = 4, MK4 = 5 };
// DKD4 and MK4: quadrupole slices composed of three second-order slices into
// a fourth-order symmetric integrator (Yoshida's triple jump).
// Where the spin is integrated inside a thick element:
//   EDGES     Ω at the N + 1 slice edges, trapezoid products and Romberg (§4.3)
//   KICK      drift-kick slices only: the rotation by Δs Ω sits between the two
//             half kicks of each slice (the DKS placement of §5.2)
//   MIDPOINT  piece-wise constant rotation by Δs Ω at the middle of each slice,
//             between two half slices (§4.1 eq. pwcSpin; DKDS in §5.2)
enum SpinPlace : int32_t { EDGES = 0, KICK = 1, MIDPOINT = 2 };

struct Elem {             // the oracle's own element record
  int32_t kind, method, nsl, rows, spin;
  int32_t fringe;         // sector bend or quadrupole: 1 adds the fringe spin kicks
  double L, angle, eta, k1, k1l, k2l, phi, mu;
  double ks;              // solenoid field b0/(Bρ)0 [1/m]
  double asym;            // rectangular bend: the faces turned by asym from the
                          // symmetric placement, φ^entr = θ/2 + asym and
                          // φ^exit = asym - θ/2 (§3.2)
};

enum { X = 0, PX = 1, Y = 2, PY = 3, TT = 4, PT = 5 };

// Reference-particle constants and the per-particle quantities that depend
// only on Pt, which no element in this model changes.
template <class T>
struct Ref {
  T G, gamma0, beta0;
  Ref(double G_, double gamma0_) : G(G_), gamma0(gamma0_) {
    using std::sqrt;
    beta0 = sqrt(T(1) - T(1) / (gamma0 * gamma0));
  }
};

// ---------------------------------------------------------------------------
// Quaternions: Hamilton convention (i j = k), q = (w, x, y, z).
// ---------------------------------------------------------------------------

template <class T> struct Quat { T w, x, y, z; };

template <class T> Quat<T> qident() { return {T(1), T(0), T(0), T(0)}; }

template <class T> Quat<T> qmul(const Quat<T>& a, const Quat<T>& b) {
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

template <class T> Quat<T> qconj(const Quat<T>& a) { return {a.w, -a.x, -a.y, -a.z}; }

// Rotation by the angle |ω| about ω/|ω| (active, right-handed): the
// quaternion (cos(θ/2), sin(θ/2) ω/θ) with θ = |ω|  (§4.1, quaternions).
template <class T> Quat<T> qrot(T wx, T wy, T wz) {
  using std::cos; using std::sin; using std::sqrt;
  T th = sqrt(wx * wx + wy * wy + wz * wz);
  // At zero angle the quaternion is the identity, and its first derivative
  // is (0, ½ dω): sin(θ/2)/θ tends to ½ while cos(θ/2) is flat.  Written
  // with ω itself so that forward-mode derivatives keep that term.
  if (th == T(0)) return {T(1), T(0.5) * wx, T(0.5) * wy, T(0.5) * wz};
  T c = cos(th / T(2));
  T f = sin(th / T(2)) / th;
  return {c, f * wx, f * wy, f * wz};
}

template <class T> Quat<T> qnormalise(const Quat<T>& q) {
  using std::sqrt;
  T n = sqrt(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
  return {q.w / n, q.x / n, q.y / n, q.z / n};
}

// S' = q S q*.
template <class T> void qrotate(const Quat<T>& q, T s[3]) {
  Quat<T> v{T(0), s[0], s[1], s[2]};
  Quat<T> r = qmul(qmul(q, v), qconj(q));
  s[0] = r.x; s[1] = r.y; s[2] = r.z;
}

// ---------------------------------------------------------------------------
// Orbit maps (§3)
// ---------------------------------------------------------------------------

// Ps of eq. ps.
template <class T> T ps_of(const T z[6], const Ref<T>& r) {
  using std::sqrt;
  T Pt = z[PT];
  return sqrt(T(1) + T(2) / r.beta0 * Pt + Pt * Pt - z[PX] * z[PX] - z[PY] * z[PY]);
}

// Exact drift: the flow of H_drift = -Ps + Pt/β0 (§3.4 eq. HmultD; the h → 0
// limit of the TEAPOT drift, §3.6).  Momenta are constant, so
// X' = Px/Ps, Y' = Py/Ps, T' = -(1/β0 + Pt)/Ps + 1/β0.
template <class T> void drift(T z[6], T L, const Ref<T>& r) {
  T ps = ps_of(z, r);
  z[X] = z[X] + L * z[PX] / ps;
  z[Y] = z[Y] + L * z[PY] / ps;
  z[TT] = z[TT] + L / r.beta0 - L * (T(1) / r.beta0 + z[PT]) / ps;
}

// Multipole kick: the flow of the vector-potential term alone (§3.4, eq. Amult
// with m = 2 and m = 3, normal components) over an integrated strength:
// Px -= k1l X + (k2l/2)(X² - Y²),  Py += k1l Y + k2l X Y.
template <class T> void kick(T z[6], T k1l, T k2l) {
  T x = z[X], y = z[Y];
  z[PX] = z[PX] - (k1l * x + k2l / T(2) * (x * x - y * y));
  z[PY] = z[PY] + (k1l * y + k2l * x * y);
}

// Exact sector bend over a length s from the current state (§3.1 eq. sbend,
// with Pα of eq. planarP and η of eq. eta).  Px'(s) is dPx/ds.
template <class T> void sbend_step(T z[6], T s, T h, T eta, const Ref<T>& r) {
  using std::asin; using std::cos; using std::sin; using std::sqrt;
  T Pt = z[PT], Py = z[PY];
  T Pa = sqrt(T(1) + T(2) / r.beta0 * Pt + Pt * Pt - Py * Py);
  T Xi = z[X], Pxi = z[PX];
  T c = cos(h * s), sn = sin(h * s);
  T A = sqrt(Pa * Pa - Pxi * Pxi) - eta * (T(1) + h * Xi);
  T Px = Pxi * c + A * sn;
  T dPx = h * (-Pxi * sn + A * c);                     // dPx/ds at s
  T Xs = (T(1) / h) * ((T(1) / eta) * (sqrt(Pa * Pa - Px * Px) - dPx / h) - T(1));
  T D = asin(Pxi / Pa) - asin(Px / Pa);
  z[X] = Xs;
  z[PX] = Px;
  z[Y] = z[Y] + (T(1) / eta) * Py * s + (T(1) / (eta * h)) * Py * D;
  z[TT] = z[TT] - (T(1) / eta) * Pt * s - (T(1) / (eta * h)) * (T(1) / r.beta0 + Pt) * D
          + (T(1) - T(1) / eta) * s / r.beta0;
}

// TEAPOT drift in a sector bend over a length s (§3.6 eq. teapotD): the flow
// of H_D = -(1 + hX) Ps, a straight line seen from the rotating frame.  The
// Pt/β0 term of eq. generalH (the reference particle's flight time) is
// added to T here, as in the straight drift.
template <class T> void teapot_drift(T z[6], T s, T h, const Ref<T>& r) {
  using std::cos; using std::sin;
  T ps = ps_of(z, r);
  T Xi = z[X], Pxi = z[PX];
  T c = cos(h * s), sn = sin(h * s);
  T tn = sn / c;
  T R = T(1) / h + Xi;
  T den = T(1) - (Pxi / ps) * tn;
  T path = R * tn / den;
  z[X] = R * (T(1) / c) / den - T(1) / h;
  z[PX] = Pxi * c + ps * sn;
  z[Y] = z[Y] + (z[PY] / ps) * path;
  z[TT] = z[TT] - (T(1) / r.beta0 + z[PT]) / ps * path + s / r.beta0;
}

// Kick of the sector-bend dipole over a length s (§3.6 eq. teapotHK): with
// the field b_y = η h on the reference arc the vector-potential term is
// H_K = η h (X + h X²/2), so Px -= η h (1 + hX) s.
template <class T> void bend_kick(T z[6], T s, T h, T eta) {
  z[PX] = z[PX] - eta * h * (T(1) + h * z[X]) * s;
}

// Solenoid body over a length s (§3.7 eq. solenoid): with η = b0/(2 (Bρ)0),
// Ps from eq. Hsolenoid (kinetic transverse momenta Px + ηY, Py - ηX) and
// κ = η/Ps, the commuting rotations R1 (eq. rotPS) and R2 (eq. rotXY) act on
// (X, Px, Y, Py) and T moves by eq. solT.
template <class T> T sol_ps(const T z[6], T eta, const Ref<T>& r) {
  using std::sqrt;
  T Pt = z[PT];
  T kx = z[PX] + eta * z[Y], ky = z[PY] - eta * z[X];
  return sqrt(T(1) + T(2) / r.beta0 * Pt + Pt * Pt - kx * kx - ky * ky);
}

template <class T> void solenoid_body(T z[6], T s, T eta, const Ref<T>& r) {
  using std::cos; using std::sin;
  T ps = sol_ps(z, eta, r);
  T kap = eta / ps;
  T c = cos(kap * s), sn = sin(kap * s);
  // R2: rotation of (X, Y) and of (Px, Py) by the angle κs
  T X2 = c * z[X] + sn * z[Y], Y2 = -sn * z[X] + c * z[Y];
  T Px2 = c * z[PX] + sn * z[PY], Py2 = -sn * z[PX] + c * z[PY];
  // R1: the focusing rotations in (X, Px) and (Y, Py)
  z[X] = c * X2 + sn / eta * Px2;
  z[PX] = -eta * sn * X2 + c * Px2;
  z[Y] = c * Y2 + sn / eta * Py2;
  z[PY] = -eta * sn * Y2 + c * Py2;
  z[TT] = z[TT] - (T(1) / r.beta0 + z[PT]) * s / ps + s / r.beta0;
}

// Precession vector in the solenoid body (eq. t-bmt.so with b = (0, 0, ks)
// and û from the kinetic momentum of eq. mgVSol).
template <class T> void omega_solenoid(const T z[6], T ks, const Ref<T>& r, T out[3]) {
  using std::sqrt;
  T eta = ks / T(2);
  T Pt = z[PT];
  T P = sqrt(T(1) + T(2) / r.beta0 * Pt + Pt * Pt);
  T ps = sol_ps(z, eta, r);
  T u[3] = {(z[PX] + eta * z[Y]) / P, (z[PY] - eta * z[X]) / P, ps / P};
  T gamma = r.gamma0 * (T(1) + r.beta0 * Pt);
  T a1 = T(1) + r.G * gamma, a2 = r.G * (gamma - T(1));
  T b[3] = {T(0), T(0), ks};
  T ub = u[2] * ks;
  for (int i = 0; i < 3; ++i) out[i] = -(T(1) / ps) * (a1 * b[i] - a2 * ub * u[i]);
}

// Thin-pancake fringe of a solenoid (§4.4 eq. solFringe): the orbit is
// unchanged; the spin turns by ω = ±(b0/2)/((Bρ)0 Ps) [(1 + Gγ)(X, Y, 0)
// - G(γ - 1)(X Px + Y Py)/P² mγV], with mγV and Ps taken at half the vector
// potential; + at the entrance, - at the exit.
template <class T> Quat<T> solenoid_fringe(const T z[6], T ks, T sign, const Ref<T>& r) {
  using std::sqrt;
  T eta_h = ks / T(4);                       // half of b0/(2 (Bρ)0)
  T Pt = z[PT];
  T P2 = T(1) + T(2) / r.beta0 * Pt + Pt * Pt;
  T kx = z[PX] + eta_h * z[Y], ky = z[PY] - eta_h * z[X];
  T ps = sqrt(P2 - kx * kx - ky * ky);
  T gamma = r.gamma0 * (T(1) + r.beta0 * Pt);
  T a1 = T(1) + r.G * gamma, a2 = r.G * (gamma - T(1));
  T f = sign * (ks / T(2)) / ps;
  T d = (z[X] * z[PX] + z[Y] * z[PY]) / P2;
  return qrot(f * (a1 * z[X] - a2 * d * kx), f * (a1 * z[Y] - a2 * d * ky), f * (-a2 * d * ps));
}

// ---- Rectangular bend (§3.2): in the magnet's Cartesian frame the design
// orbit enters at the angle φ^entr to the magnet's axis and leaves at φ^exit,
// turning by θ = φ^entr - φ^exit on a circle of radius ρ with
// L = ρ (sin φ^entr - sin φ^exit); the field is b1/(Bρ)0 = η/ρ.  The
// symmetric magnet has φ^exit = -φ^entr = -θ/2.

// Dynamic rotation of the frame by φ: the flow of eq. Hprot, H = -X Ps,
// over the angle φ (eq. prot).  T follows that flow, dT/dφ = -X (1/β0 +
// Pt)/Ps, so a particle outside the reference (X > 0) reaches the rotated
// face later; the printed T(φ) carries the opposite sign, at odds with the
// printed Hamiltonian whose X, Px and Y flows it matches.
template <class T> void prot(T z[6], T phi, const Ref<T>& r) {
  using std::cos; using std::sin;
  T ps = ps_of(z, r);
  T c = cos(phi), sn = sin(phi), tn = sn / c;
  T Xi = z[X], Pxi = z[PX];
  T den = T(1) - (Pxi / ps) * tn;
  z[X] = Xi * (T(1) / c) / den;
  z[PX] = Pxi * c + ps * sn;
  z[Y] = z[Y] + (z[PY] / ps) * Xi * tn / den;
  z[TT] = z[TT] - (T(1) / r.beta0 + z[PT]) / ps * Xi * tn / den;
}

// Thin dipole fringe without gap correction (eq. dipolefringe); sign +1 at
// the entrance, -1 at the exit; fb = b1/(Bρ)0.
template <class T> void dipole_fringe(T z[6], T fb, T sign, const Ref<T>& r) {
  using std::sqrt;
  T ps = ps_of(z, r);
  T xp = z[PX] / ps, yp = z[PY] / ps;
  T q = T(1) + yp * yp;
  T sf = sign * fb;
  T Yf = T(2) * z[Y] / (T(1) + sqrt(T(1) + sf * (xp * yp / q) * T(2) * z[Y]));
  z[X] = z[X] + sf / (T(2) * ps) * ((T(1) + xp * xp) / q - T(2) * (xp * yp) * (xp * yp) / (q * q)) * Yf * Yf;
  z[PY] = z[PY] - sf * xp / q * Yf;
  z[TT] = z[TT] - sf * (T(1) / r.beta0 + z[PT]) * xp / (T(2) * ps * ps) * (T(1) - yp * yp) / (q * q) * Yf * Yf;
  z[Y] = Yf;
}

// Body of the rectangular bend over a length s (eq. rbend; Pα of eq.
// planarP).  The printed T has no reference flight time; the element adds the
// design arc's L_arc/β0 at its end (eq. Toffset).
template <class T> void rbend_body(T z[6], T s, T fb, const Ref<T>& r) {
  using std::asin; using std::sqrt;
  T Pt = z[PT], Py = z[PY];
  T Pa = sqrt(T(1) + T(2) / r.beta0 * Pt + Pt * Pt - Py * Py);
  T rhob = T(1) / fb;
  T Pxi = z[PX];
  T Px = Pxi - s * fb;
  T D = asin(Pxi / Pa) - asin(Px / Pa);
  z[X] = z[X] + rhob * (sqrt(Pa * Pa - Px * Px) - sqrt(Pa * Pa - Pxi * Pxi));
  z[PX] = Px;
  z[Y] = z[Y] + Py * rhob * D;
  z[TT] = z[TT] - (T(1) / r.beta0 + Pt) * rhob * D;
}

// Spin kick across a rectangular-bend fringe (§4.5 eq. skfringe with m = 1
// and eq. skfringeRB).  The longitudinal fringe field integrates to b1 Y;
// the printed x̂ term lacks that Y (as printed it is not dimensionless), and
// splitting b1 Y ẑ into parts along and across the velocity (of slope Px)
// gives ω = ±(b1/(Bρ)0) [-(1 + G) Y ẑ + G(γ - 1) Px Y x̂].
template <class T> Quat<T> rbend_fringe_spin(const T z[6], T fb, T sign, const Ref<T>& r) {
  T gamma = r.gamma0 * (T(1) + r.beta0 * z[PT]);
  T f = sign * fb * z[Y];
  return qrot(f * r.G * (gamma - T(1)) * z[PX], T(0), -f * (T(1) + r.G));
}

// Spin kick across the thin fringe of a normal 2m-pole crossed about
// normally (§4.5 eq. skfringe): a rotation about ẑ by
//   -sign (b_m/(Bρ)0) (1 + G) r^m sin(m φ)/m,   r^m sin(m φ) = Im (X + iY)^m,
// sign +1 at the entrance and -1 at the exit.  A sector bend is the m = 1
// case with b1/(Bρ)0 = η h, a quadrupole the m = 2 case with b2/(Bρ)0 = k1.
template <class T> Quat<T> multipole_fringe_spin(const Elem& e, const T z[6], T sign,
                                                 const Ref<T>& r) {
  int m = e.kind == SBEND ? 1 : 2;
  T bm = e.kind == SBEND ? T(e.eta) * T(e.angle) / T(e.L) : T(e.k1);
  T re = T(1), im = T(0);                       // (X + iY)^m
  for (int k = 0; k < m; ++k) {
    T nre = re * z[X] - im * z[Y];
    im = re * z[Y] + im * z[X];
    re = nre;
  }
  return qrot(T(0), T(0), -sign * bm * (T(1) + r.G) * im / T(m));
}

// Matrix-kick quadrupole, linear part over a length s (§3.3 eq. quadL).  The
// printed solution is for a focusing gradient; a defocusing one (k1 < 0) is
// the same map with the roles of (X, Px) and (Y, Py) exchanged.
template <class T> void quad_linear(T z[6], T s, T k1, const Ref<T>& r) {
  using std::cos; using std::cosh; using std::sin; using std::sinh; using std::sqrt;
  T Pt = z[PT];
  T P = sqrt(T(1) + T(2) / r.beta0 * Pt + Pt * Pt);       // eq. quadSclP
  bool focusing_x = !(k1 < T(0));
  T kabs = focusing_x ? k1 : -k1;
  T kap = sqrt(kabs / P);                                 // eq. kappa2
  int ix = focusing_x ? X : Y, ipx = focusing_x ? PX : PY;
  int iy = focusing_x ? Y : X, ipy = focusing_x ? PY : PX;
  T Xi = z[ix], Pxi = z[ipx], Yi = z[iy], Pyi = z[ipy];
  T ks = kap * s;
  T cs = cos(ks), sn = sin(ks), ch = cosh(ks), sh = sinh(ks);
  z[ix] = Xi * cs + s * (Pxi / P) * (sn / ks);
  z[ipx] = Pxi * cs - kap * P * Xi * sn;
  z[iy] = Yi * ch + s * (Pyi / P) * (sh / ks);
  z[ipy] = Pyi * ch + kap * P * Yi * sh;
  T px = Pxi / P, py = Pyi / P;
  T sin2 = sin(T(2) * ks), sinh2 = sinh(T(2) * ks);
  T brace = s / T(4) * (px * px + py * py + kap * kap * (Xi * Xi - Yi * Yi))
          + s / T(4) * (px * px - kap * Xi * kap * Xi) * (sin2 / (T(2) * ks))
          + s / T(4) * (py * py + kap * Yi * kap * Yi) * (sinh2 / (T(2) * ks))
          - ks / T(2) * (Xi * px * (sn * sn / ks) - Yi * py * (sh * sh / ks));
  z[TT] = z[TT] - (T(1) / P) * (T(1) / r.beta0 + Pt) * brace;
}

// Matrix-kick quadrupole, nonlinear "kick of positions" over s (§3.3 eq. quadNL).
template <class T> void quad_nonlinear(T z[6], T s, const Ref<T>& r) {
  using std::sqrt;
  T Pt = z[PT];
  T P = sqrt(T(1) + T(2) / r.beta0 * Pt + Pt * Pt);
  T ps = ps_of(z, r);
  T Pxi = z[PX], Pyi = z[PY];
  z[X] = z[X] + s * Pxi * (T(1) / ps - T(1) / P);
  z[Y] = z[Y] + s * Pyi * (T(1) / ps - T(1) / P);
  z[TT] = z[TT] - s * (T(1) / r.beta0 + Pt) * (T(1) / ps - (T(1) / P) * (Pxi * Pxi + Pyi * Pyi) / (T(2) * P * P))
          + s / r.beta0;
}

// ---------------------------------------------------------------------------
// Spin precession vector (§2.2 eq. t-bmt.so)
// ---------------------------------------------------------------------------

// Ω = -(1 + hX)/Ps [ (1 + Gγ) b - G(γ - 1)(u·b) u ] + h ŷ, with b = B/(Bρ)0,
// u = (Px, Py, Ps)/|(Px, Py, Ps)| and γ the particle's own Lorentz factor
// γ = γ0 (1 + β0 Pt) (from eq. pt).
template <class T> void omega(const T z[6], T h, const T b[3], const Ref<T>& r, T out[3]) {
  using std::sqrt;
  T ps = ps_of(z, r);
  T Pt = z[PT];
  T P = sqrt(T(1) + T(2) / r.beta0 * Pt + Pt * Pt);
  T u[3] = {z[PX] / P, z[PY] / P, ps / P};
  T gamma = r.gamma0 * (T(1) + r.beta0 * Pt);
  T a1 = T(1) + r.G * gamma, a2 = r.G * (gamma - T(1));
  T ub = u[0] * b[0] + u[1] * b[1] + u[2] * b[2];
  T f = -(T(1) + h * z[X]) / ps;
  for (int i = 0; i < 3; ++i) out[i] = f * (a1 * b[i] - a2 * ub * u[i]);
  out[1] = out[1] + h;
}

// Field b = B/(Bρ)0 at the particle for the thick elements.
template <class T> void field(const Elem& e, const T z[6], T b[3]) {
  if (e.kind == SBEND) {
    T h = T(e.angle) / T(e.L);
    b[0] = T(0); b[1] = T(e.eta) * h; b[2] = T(0);
  } else {  // QUAD: b = k1 (Y, X, 0)
    b[0] = T(e.k1) * z[Y]; b[1] = T(e.k1) * z[X]; b[2] = T(0);
  }
}

// ---------------------------------------------------------------------------
// Romberg quadrature for spin (§4.3)
// ---------------------------------------------------------------------------

// 2-adic valuation of n > 0.
inline int v2(int n) { int k = 0; while ((n & 1) == 0) { n >>= 1; ++k; } return k; }

// Given Ω at the N + 1 slice edges of an element (uniform slices of length
// ds) and R requested tableau rows, return the normalised Romberg limit.
// The coarse approximations keep every 2^m-th edge with weight 2^m ds and
// halve the weights of the first and last edges (eq. Qhs); later factors
// multiply on the left.  The tableau follows eq. romberg.
template <class T>
Quat<T> romberg_spin(const std::vector<T>& om, int N, T ds, int R) {
  int Re = std::min(R, 1 + v2(N));
  int K = Re - 1;
  std::vector<std::vector<Quat<T>>> tab(Re, std::vector<Quat<T>>(Re));
  for (int k = 0; k <= K; ++k) {
    int stride = 1 << (K - k);
    Quat<T> Qk = qident<T>();
    for (int j = 0; j <= N; j += stride) {
      T w = (j == 0 || j == N) ? T(0.5) : T(1);
      T step = w * T(stride) * ds;
      Quat<T> q = qrot(step * om[3 * j], step * om[3 * j + 1], step * om[3 * j + 2]);
      Qk = qmul(q, Qk);
    }
    tab[0][k] = Qk;
  }
  T four = T(1);
  for (int j = 1; j <= K; ++j) {
    four = four * T(4);
    for (int k = j; k <= K; ++k) {
      const Quat<T>& a = tab[j - 1][k];
      const Quat<T>& b = tab[j - 1][k - 1];
      T den = four - T(1);
      tab[j][k] = {(four * a.w - b.w) / den, (four * a.x - b.x) / den,
                   (four * a.y - b.y) / den, (four * a.z - b.z) / den};
    }
  }
  return qnormalise(tab[K][K]);
}

// ---------------------------------------------------------------------------
// One element: orbit map and spin quaternion
// ---------------------------------------------------------------------------

// The drift and kick halves of a drift-kick slice (TEAPOT bend or DKD quad).
template <class T>
void dk_drift(const Elem& e, T z[6], T s, const Ref<T>& r) {
  if (e.kind == SBEND) teapot_drift(z, s, T(e.angle) / T(e.L), r);
  else                 drift(z, s, r);
}

template <class T>
void dk_kick(const Elem& e, T z[6], T s) {
  if (e.kind == SBEND) bend_kick(z, s, T(e.angle) / T(e.L), T(e.eta));
  else                 kick(z, T(e.k1) * s, T(0));
}

// Entrance and exit angles of the design orbit in a rectangular bend.
template <class T> T rbend_phi_entr(const Elem& e) { return T(e.angle) / T(2) + T(e.asym); }
template <class T> T rbend_phi_exit(const Elem& e) { return T(e.asym) - T(e.angle) / T(2); }

template <class T> T rbend_fb(const Elem& e) {
  using std::sin;
  return T(e.eta) * (sin(rbend_phi_entr<T>(e)) - sin(rbend_phi_exit<T>(e))) / T(e.L);
}

// One second-order quadrupole slice: drift-kick-drift (§3.4 applied to
// m = 2) or matrix-kick-matrix (§3.3 eq. quadConcat).
template <class T>
void quad_slice2(const Elem& e, T z[6], T ds, const Ref<T>& r) {
  if (e.method == DKD || e.method == DKD4) {
    drift(z, ds / T(2), r);
    kick(z, T(e.k1) * ds, T(0));
    drift(z, ds / T(2), r);
  } else {
    quad_linear(z, ds / T(2), T(e.k1), r);
    quad_nonlinear(z, ds, r);
    quad_linear(z, ds / T(2), T(e.k1), r);
  }
}

template <class T>
void slice(const Elem& e, T z[6], T ds, const Ref<T>& r) {
  if (e.kind == RBEND) {
    rbend_body(z, ds, rbend_fb<T>(e), r);
  } else if (e.kind == SOLENOID) {
    solenoid_body(z, ds, T(e.ks) / T(2), r);
  } else if (e.kind == SBEND && e.method == TEAPOT) {   // drift-kick-drift (§3.6)
    dk_drift(e, z, ds / T(2), r);
    dk_kick(e, z, ds);
    dk_drift(e, z, ds / T(2), r);
  } else if (e.kind == SBEND) {
    sbend_step(z, ds, T(e.angle) / T(e.L), T(e.eta), r);
  } else if (e.method == DKD4 || e.method == MK4) {
    // The symmetric second-order slice S2 has an error odd in ds starting at
    // ds^3; S2(x1 ds) S2(x0 ds) S2(x1 ds) with 2 x1 + x0 = 1 and
    // 2 x1^3 + x0^3 = 0 cancels it, leaving fourth order (the higher-order
    // compositions §3.3 refers to).
    using std::cbrt;
    T c2 = T(cbrt(2.0L));
    T x1 = T(1) / (T(2) - c2), x0 = -c2 / (T(2) - c2);
    quad_slice2(e, z, x1 * ds, r);
    quad_slice2(e, z, x0 * ds, r);
    quad_slice2(e, z, x1 * ds, r);
  } else {
    quad_slice2(e, z, ds, r);
  }
}

template <class T>
Quat<T> element(const Elem& e, T z[6], const Ref<T>& r) {
  switch (e.kind) {
    case DRIFT:
      drift(z, T(e.L), r);
      return qident<T>();
    case RBEND: {
      // frame rotation by φ^entr into the magnet, fringe, body, the design
      // orbit's horizontal offset (eq. Xoffset), fringe, rotation by
      // -φ^exit out; the rotations turn the spin components with the frame
      // about ŷ
      using std::sin; using std::cos;
      T phe = rbend_phi_entr<T>(e), phx = rbend_phi_exit<T>(e);
      T fb = rbend_fb<T>(e);
      prot(z, phe, r);
      dipole_fringe(z, fb, T(1), r);
      Quat<T> qin = rbend_fringe_spin(z, fb, T(1), r);
      int N = e.nsl;
      T ds = T(e.L) / T(N);
      T b[3] = {T(0), fb, T(0)};
      Quat<T> Qb;
      if (e.spin == MIDPOINT) {
        Qb = qident<T>();
        for (int j = 0; j < N; ++j) {
          slice(e, z, ds / T(2), r);
          T w[3];
          omega(z, T(0), b, r, w);
          Qb = qmul(qrot(ds * w[0], ds * w[1], ds * w[2]), Qb);
          slice(e, z, ds / T(2), r);
        }
        Qb = qnormalise(Qb);
      } else {
        std::vector<T> om(3 * (N + 1));
        omega(z, T(0), b, r, &om[0]);
        for (int j = 1; j <= N; ++j) {
          slice(e, z, ds, r);
          omega(z, T(0), b, r, &om[3 * j]);
        }
        Qb = romberg_spin(om, N, ds, e.rows);
      }
      // the design orbit leaves the body displaced by X^offset from where it
      // entered (zero for the symmetric magnet): refer X to it again
      T sdiff = sin(phe) - sin(phx);
      z[X] = z[X] - (-T(e.L) * (cos(phe) - cos(phx)) / sdiff);
      Quat<T> qout = rbend_fringe_spin(z, fb, T(-1), r);
      dipole_fringe(z, fb, T(-1), r);
      prot(z, -phx, r);
      // T as a deviation from the design particle's flight time over the arc
      // (eq. Toffset)
      T larc = T(e.L) * (phe - phx) / sdiff;
      z[TT] = z[TT] + larc / r.beta0;
      return qmul(qrot(T(0), -phx, T(0)), qmul(qout, qmul(Qb, qmul(qin, qrot(T(0), phe, T(0))))));
    }
    case SOLENOID: {
      // entrance fringe, body (edge Ω with Romberg, or midpoint PWC), exit fringe
      Quat<T> qin = solenoid_fringe(z, T(e.ks), T(1), r);
      int N = e.nsl;
      T ds = T(e.L) / T(N);
      Quat<T> Qb;
      if (e.spin == MIDPOINT) {
        Qb = qident<T>();
        for (int j = 0; j < N; ++j) {
          slice(e, z, ds / T(2), r);
          T w[3];
          omega_solenoid(z, T(e.ks), r, w);
          Qb = qmul(qrot(ds * w[0], ds * w[1], ds * w[2]), Qb);
          slice(e, z, ds / T(2), r);
        }
        Qb = qnormalise(Qb);
      } else {
        std::vector<T> om(3 * (N + 1));
        omega_solenoid(z, T(e.ks), r, &om[0]);
        for (int j = 1; j <= N; ++j) {
          slice(e, z, ds, r);
          omega_solenoid(z, T(e.ks), r, &om[3 * j]);
        }
        Qb = romberg_spin(om, N, ds, e.rows);
      }
      Quat<T> qout = solenoid_fringe(z, T(e.ks), T(-1), r);
      return qmul(qout, qmul(Qb, qin));
    }
    case SBEND:
    case QUAD: {
      if (e.fringe) {   // fringe spin kicks around the body (§4.5)
        Quat<T> qin = multipole_fringe_spin(e, z, T(1), r);
        Elem body = e;
        body.fringe = 0;
        Quat<T> Qb = element(body, z, r);
        Quat<T> qout = multipole_fringe_spin(e, z, T(-1), r);
        return qmul(qout, qmul(Qb, qin));
      }
      int N = e.nsl;
      T ds = T(e.L) / T(N);
      T h = e.kind == SBEND ? T(e.angle) / T(e.L) : T(0);
      T b[3];
      if (e.spin != EDGES) {
        // piece-wise constant rotations ω = Δs Ω (eq. pwcSpin), one per slice,
        // Ω taken at the slice's middle state; later slices on the left
        Quat<T> Q = qident<T>();
        for (int j = 0; j < N; ++j) {
          if (e.spin == KICK) {
            dk_drift(e, z, ds / T(2), r);
            dk_kick(e, z, ds / T(2));
          } else {
            slice(e, z, ds / T(2), r);
          }
          T w[3];
          field(e, z, b);
          omega(z, h, b, r, w);
          Q = qmul(qrot(ds * w[0], ds * w[1], ds * w[2]), Q);
          if (e.spin == KICK) {
            dk_kick(e, z, ds / T(2));
            dk_drift(e, z, ds / T(2), r);
          } else {
            slice(e, z, ds / T(2), r);
          }
        }
        return qnormalise(Q);
      }
      std::vector<T> om(3 * (N + 1));
      field(e, z, b);
      omega(z, h, b, r, &om[0]);
      for (int j = 1; j <= N; ++j) {
        slice(e, z, ds, r);
        field(e, z, b);
        omega(z, h, b, r, &om[3 * j]);
      }
      return romberg_spin(om, N, ds, e.rows);
    }
    case THIN: {
      // Half kick, spin rotation by the integrated Ω at the mid state, half kick.
      kick(z, T(e.k1l) / T(2), T(e.k2l) / T(2));
      T x = z[X], y = z[Y];
      T b[3] = {T(e.k1l) * y + T(e.k2l) * x * y,
                T(e.k1l) * x + T(e.k2l) / T(2) * (x * x - y * y), T(0)};
      T w[3];
      omega(z, T(0), b, r, w);
      Quat<T> q = qrot(w[0], w[1], w[2]);
      kick(z, T(e.k1l) / T(2), T(e.k2l) / T(2));
      return q;
    }
    case SNAKE: {
      using std::cos; using std::sin;
      T hphi = T(e.phi) / T(2);
      T sh = sin(hphi);
      return {cos(hphi), sh * sin(T(e.mu)), T(0), sh * cos(T(e.mu))};
    }
    default:
      return qident<T>();
  }
}

// ---------------------------------------------------------------------------
// Particle and bunch tracking
// ---------------------------------------------------------------------------

template <class T>
bool in_bounds(const T z[6], double aperture) {
  for (int i = 0; i < 6; ++i) if (!finite_(z[i])) return false;
  auto ax = std::fabs((long double)value_(z[X]));
  auto ay = std::fabs((long double)value_(z[Y]));
  return ax <= aperture && ay <= aperture;
}

// Track one particle for `turns` turns.  Returns -1 while alive, else the
// index of the element where it was lost; the state is then frozen at that
// element's entrance.  sums (if given) receives (Sx, Sy, Sz, 1) after each
// reported turn.  qturn receives the one-turn quaternion of the last turn
// (the product of the element quaternions, later elements on the left).
template <class T>
int track_particle(const Elem* el, int ne, const Ref<T>& r, double aperture, T z[6], T s[3],
                   int turns, int report_every, long double* sums, Quat<T>* qturn) {
  Quat<T> qt = qident<T>();
  for (int t = 1; t <= turns; ++t) {
    qt = qident<T>();
    for (int e = 0; e < ne; ++e) {
      T z0[6];
      for (int i = 0; i < 6; ++i) z0[i] = z[i];
      Quat<T> q = element(el[e], z, r);
      if (!in_bounds(z, aperture)) {
        for (int i = 0; i < 6; ++i) z[i] = z0[i];
        if (qturn) *qturn = qt;
        return e;
      }
      qrotate(q, s);
      qt = qmul(q, qt);
    }
    if (sums && report_every > 0 && t % report_every == 0) {
      long double* o = sums + 4 * (t / report_every - 1);
      o[0] += (long double)value_(s[0]);
      o[1] += (long double)value_(s[1]);
      o[2] += (long double)value_(s[2]);
      o[3] += 1.0L;
    }
  }
  if (qturn) *qturn = qt;
  return -1;
}

template <class T>
int track_bunch(const Elem* el, int ne, double G, double gamma0, double aperture, int n,
                double* z, double* s, int32_t* alive, int turns, int report_every,
                double* pol, double* qout, int threads) {
  Ref<T> r(G, gamma0);
  int n_rep = report_every > 0 ? turns / report_every : 0;
  if (threads < 1) threads = 1;
  if (threads > n) threads = std::max(1, n);
  std::vector<std::vector<long double>> part(threads, std::vector<long double>(4 * std::max(n_rep, 1), 0.0L));
  auto work = [&](int tid) {
    int lo = (int)((long long)n * tid / threads), hi = (int)((long long)n * (tid + 1) / threads);
    for (int j = lo; j < hi; ++j) {
      if (alive[j] != 1) continue;
      T zz[6], ss[3];
      for (int i = 0; i < 6; ++i) zz[i] = T(z[(size_t)i * n + j]);
      for (int i = 0; i < 3; ++i) ss[i] = T(s[(size_t)i * n + j]);
      Quat<T> q = qident<T>();
      int lost = track_particle(el, ne, r, aperture, zz, ss, turns, report_every,
                                n_rep ? part[tid].data() : nullptr, &q);
      for (int i = 0; i < 6; ++i) z[(size_t)i * n + j] = (double)value_(zz[i]);
      for (int i = 0; i < 3; ++i) s[(size_t)i * n + j] = (double)value_(ss[i]);
      if (lost >= 0) alive[j] = -(1 + lost);
      if (qout) {
        qout[(size_t)0 * n + j] = (double)value_(q.w);
        qout[(size_t)1 * n + j] = (double)value_(q.x);
        qout[(size_t)2 * n + j] = (double)value_(q.y);
        qout[(size_t)3 * n + j] = (double)value_(q.z);
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  if (pol && n_rep > 0) {
    for (int k = 0; k < n_rep; ++k) {
      long double acc[4] = {0, 0, 0, 0};
      for (int t = 0; t < threads; ++t)
        for (int i = 0; i < 4; ++i) acc[i] += part[t][4 * k + i];
      for (int i = 0; i < 3; ++i) pol[4 * k + i] = acc[3] > 0 ? (double)(acc[i] / acc[3]) : 0.0;
      pol[4 * k + 3] = (double)acc[3];
    }
  }
  return 0;
}

}  // namespace oracle

using namespace oracle;

extern "C" {

// Track n particles (SoA z[6][n], s[3][n], alive[n]) for `turns` turns, in
// extended (ld = 1) or double (ld = 0) precision.  Updates z, s, alive in
// place; pol receives (Px, Py, Pz, N_alive) per report; qout (4×n SoA) the
// last turn's quaternion.  Returns 0.
int oracle_track(const Elem* el, int ne, double G, double gamma0, double aperture, int n,
                 double* z, double* s, int32_t* alive, int turns, int report_every,
                 double* pol, double* qout, int threads, int ld) {
  if (ld) return track_bunch<long double>(el, ne, G, gamma0, aperture, n, z, s, alive, turns,
                                          report_every, pol, qout, threads);
  return track_bunch<double>(el, ne, G, gamma0, aperture, n, z, s, alive, turns, report_every,
                             pol, qout, threads);
}

// One-particle tracking with forward-mode derivatives w.r.t. the initial
// 6-D orbit: J (6×6, row i = d z_i / d z0_j) and dQ (4×6) of the last turn's
// quaternion; zout (6), sout (3), qout (4) the values.  Returns the loss
// element index or -1.
int oracle_jacobian(const Elem* el, int ne, double G, double gamma0, double aperture,
                    const double* z0, const double* s0, int turns, double* J, double* dQ,
                    double* zout, double* sout, double* qout) {
  using D = Dual<long double, 6>;
  Ref<D> r(G, gamma0);
  D z[6], s[3];
  for (int i = 0; i < 6; ++i) { z[i] = D((long double)z0[i]); z[i].d[i] = 1.0L; }
  for (int i = 0; i < 3; ++i) s[i] = D((long double)s0[i]);
  Quat<D> q = qident<D>();
  int lost = track_particle(el, ne, r, aperture, z, s, turns, 0, nullptr, &q);
  for (int i = 0; i < 6; ++i) {
    zout[i] = (double)z[i].v;
    for (int j = 0; j < 6; ++j) J[6 * i + j] = (double)z[i].d[j];
  }
  for (int i = 0; i < 3; ++i) sout[i] = (double)s[i].v;
  const D* qc[4] = {&q.w, &q.x, &q.y, &q.z};
  for (int i = 0; i < 4; ++i) {
    qout[i] = (double)qc[i]->v;
    for (int j = 0; j < 6; ++j) dQ[6 * i + j] = (double)qc[i]->d[j];
  }
  return lost;
}

// Count the floating-point operations of tracking one particle for `turns`
// turns.  counts = {add/sub, mul, div, sqrt, sin/cos, asin, sinh/cosh}.
int oracle_count_ops(const Elem* el, int ne, double G, double gamma0, double aperture,
                     const double* z0, int turns, long long* counts) {
  Ref<Counted> r(G, gamma0);
  g_counts = Counts{0, 0, 0, 0, 0, 0, 0};
  Counted z[6], s[3] = {Counted(0.0), Counted(1.0), Counted(0.0)};
  for (int i = 0; i < 6; ++i) z[i] = Counted(z0[i]);
  g_counts = Counts{0, 0, 0, 0, 0, 0, 0};
  int lost = track_particle(el, ne, r, aperture, z, s, turns, 0, nullptr, (Quat<Counted>*)nullptr);
  counts[0] = g_counts.add; counts[1] = g_counts.mul; counts[2] = g_counts.div;
  counts[3] = g_counts.sqrt; counts[4] = g_counts.sincos; counts[5] = g_counts.asin;
  counts[6] = g_counts.hyp;
  return lost;
}

// The Romberg machinery alone: Ω given at N + 1 edges (row-major (N+1)×3),
// slice length ds, R rows; q_out receives the normalised limit (w, x, y, z).
int oracle_romberg(const double* om, int N, double ds, int R, double* q_out, int ld) {
  if (ld) {
    std::vector<long double> v(om, om + 3 * (N + 1));
    Quat<long double> q = romberg_spin<long double>(v, N, (long double)ds, R);
    q_out[0] = (double)q.w; q_out[1] = (double)q.x; q_out[2] = (double)q.y; q_out[3] = (double)q.z;
  } else {
    std::vector<double> v(om, om + 3 * (N + 1));
    Quat<double> q = romberg_spin<double>(v, N, ds, R);
    q_out[0] = q.w; q_out[1] = q.x; q_out[2] = q.y; q_out[3] = q.z;
  }
  return 0;
}

// Ω of eq. t-bmt.so at one state for a given curvature h and field b.
int oracle_omega(const double* z, double h, const double* b, double G, double gamma0, double* out) {
  Ref<long double> r(G, gamma0);
  long double zz[6], bb[3], o[3];
  for (int i = 0; i < 6; ++i) zz[i] = z[i];
  for (int i = 0; i < 3; ++i) bb[i] = b[i];
  omega(zz, (long double)h, bb, r, o);
  for (int i = 0; i < 3; ++i) out[i] = (double)o[i];
  return 0;
}

// The dynamic rotation of a rectangular-bend face alone (eq. prot), for the
// pins: z (6) rotated by phi in extended precision.
int oracle_rotate(const double* z_in, double phi, double G, double gamma0, double* z_out) {
  Ref<long double> r(G, gamma0);
  long double z[6];
  for (int i = 0; i < 6; ++i) z[i] = z_in[i];
  prot(z, (long double)phi, r);
  for (int i = 0; i < 6; ++i) z_out[i] = (double)z[i];
  return 0;
}

int oracle_elem_size(void) { return (int)sizeof(Elem); }

}  // extern "C"

// Persistent tracking kernel: one lane per particle, all turns and all
// elements of the ring in one launch, state in registers.
//
// Per element (wave-uniform walk of the lattice index sequence):
//   drift            exact flow, no spin
//   sector bend      exact steps of ds between slice edges (§3.1)
//   quadrupole       DKD or MK slices (§3.4, §3.3)
//   thin multipole   half kick, rotation by the integrated Ω, half kick
//   snake            fixed rotation
// Thick elements with spin evaluate Ω at the N + 1 slice edges (§4.3) and
// fold each edge into the running product of every Romberg level that keeps
// it, so no Ω record ever leaves the registers.  The tableau and the
// normalisation follow at the element exit, and the element quaternion is
// composed into the turn quaternion, which rotates the spin once per turn.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fp64_maps.h"
#include "mixed_spin.h"
#include "track_kernels.h"

namespace st {

namespace {

constexpr int kBlock = 256;

typedef const DevElem __attribute__((address_space(4))) ConstElem;
typedef const uint32_t __attribute__((address_space(4))) ConstSeq;

// Member-wise copy of one element record out of the constant address space
// (uniform address: scalar loads).
__device__ __forceinline__ DevElem load_elem(const ConstElem* p) {
  DevElem d;
  d.kind = p->kind;
  d.orbit = p->orbit;
  d.nsl = p->nsl;
  d.K = p->K;
  d.flags = p->flags;
  d.place = p->place;
  d.hw_end = p->hw_end;
  d.hw_in = p->hw_in;
  d.hw2_end = p->hw2_end;
  d.hw2_in = p->hw2_in;
#pragma unroll
  for (int i = 0; i < kElemWords; ++i) d.v[i] = p->v[i];
  return d;
}

// Waves per SIMD the register allocation aims at: two, for every variant.
// The plain double kernel fits in 236 VGPRs with no scratch at two waves; at
// three waves (168 VGPRs) it ran at the same speed, but spilled 70 VGPRs at
// the element entrances, and with 2^20 lanes those spill slots (228 B each)
// were written back to memory, about 500 GB per 100-turn launch.
#ifndef ST_WAVES_PER_EU
#define ST_WAVES_PER_EU 2
#endif
#ifndef ST_WAVES_PER_EU_WIDE
#define ST_WAVES_PER_EU_WIDE 2
#endif
#ifndef ST_WAVES_PER_EU_ORBIT
#define ST_WAVES_PER_EU_ORBIT 3
#endif

// Romberg spin integration through one thick element, fused with its orbit
// slices (KIND: 0 sector bend, 1 MK quadrupole focusing in x, 3 MK
// quadrupole focusing in y, 2 DKD quadrupole, 4 drift-kick (TEAPOT) sector
// bend).  In the MIXED kernel,
// elements flagged F_SPIN32 use single-precision edge quaternions and
// compensated single-precision level products.  Returns the normalised
// element quaternion.
// One second-order quadrupole step over the length of q: matrix-kick-matrix
// (KIND 1 focusing in x, 3 focusing in y) or drift-kick-drift (KIND 2).
template <int KIND>
__device__ __forceinline__ void quad_step2(const QuadParams& q, const MKConst& mc, double& X,
                                           double& Px, double& Y, double& Py, double& T,
                                           const Particle& p, const TrackArgs& a) {
  if (KIND == 1) {
    mk_linear(mc, X, Px, Y, Py, T, p);
    mk_nonlinear(q.ds, X, Px, Y, Py, T, p);
    mk_linear(mc, X, Px, Y, Py, T, p);
  } else if (KIND == 3) {
    mk_linear(mc, Y, Py, X, Px, T, p);
    mk_nonlinear(q.ds, X, Px, Y, Py, T, p);
    mk_linear(mc, Y, Py, X, Px, T, p);
  } else {
    drift(q.hds, X, Px, Y, Py, T, p, a.inv_beta0);
    Px = fma(-q.k1ds, X, Px);
    Py = fma(q.k1ds, Y, Py);
    drift(q.hds, X, Px, Y, Py, T, p, a.inv_beta0);
  }
}

// Fourth-order quadrupole slice (orbit methods DKD4, MK4): the second-order
// step over x1 ds, x0 ds and x1 ds (2 x1 + x0 = 1, 2 x1^3 + x0^3 = 0).  m1 and
// m0 are the MK constants of the two step lengths.
template <int KIND>
__device__ __forceinline__ void quad_slice4(const Quad4Params& q4, const MKConst& m1,
                                            const MKConst& m0, double& X, double& Px, double& Y,
                                            double& Py, double& T, const Particle& p,
                                            const TrackArgs& a) {
  quad_step2<KIND>(q4.s1, m1, X, Px, Y, Py, T, p, a);
  quad_step2<KIND>(q4.s0, m0, X, Px, Y, Py, T, p, a);
  quad_step2<KIND>(q4.s1, m1, X, Px, Y, Py, T, p, a);
}

// Matrix-kick constants of the last quadrupole a lane crossed, kept in the
// block's LDS (one column per lane).  They depend only on the particle's P
// and on the element's |k1| and slice length, so quadrupoles that share
// those (in a FODO ring the focusing and defocusing ones usually do) reuse
// them instead of re-evaluating the series.  The key is element data, the
// same for every lane of a wave.
constexpr int kMKWords = sizeof(MKConst) / sizeof(double);
struct MKCache {
  double (*slot)[kBlock];
  int tid;
  double k1abs, hds;       // key of the stored constants (NaN: none yet)
};

__device__ __forceinline__ MKConst mk_cached(const QuadParams& q, const Particle& p,
                                             MKCache* c) {
  MKConst m;
  double* w = reinterpret_cast<double*>(&m);
  const double ka = fabs(q.k1);
  if (c && ka == c->k1abs && q.hds == c->hds) {
#pragma unroll
    for (int i = 0; i < kMKWords; ++i) w[i] = c->slot[i][c->tid];
    return m;
  }
  m = mk_const(q, p);
  if (c) {
#pragma unroll
    for (int i = 0; i < kMKWords; ++i) c->slot[i][c->tid] = w[i];
    c->k1abs = ka;
    c->hds = q.hds;
  }
  return m;
}

// Y4: quadrupoles with the fourth-order slice (extended kernels only).
// PEEL: the entrance edge is folded outside the slice loop, where the level
// products are set instead of multiplied into the identity (the extended
// kernels keep one copy of the edge code, which holds their registers down).
// NS > 0: the element has NS slices and KS + 1 effective Romberg rows, known
// at compile time, so the edge loop unrolls completely and the choice of the
// levels each edge feeds is made by the compiler (no loop-carried copies, no
// branches); NS == 0 reads both from the element.
template <int NT, int KIND, bool MIXED, bool Y4 = false, bool PEEL = true, int NS = 0, int KS = 0>
__device__ __forceinline__ Quat thick_element(const DevElem& el, double& X, double& Px, double& Y,
                                              double& Py, double& T, const Particle& p,
                                              const TrackArgs& a, MKCache* mkc = nullptr) {
  static_assert(kMaxRows == 4, "the level products below are written out for four rows");
  static_assert(NS == 0 || (KS >= 0 && KS < kMaxRows && NS % (1 << KS) == 0),
                "NS slices must be divisible by 2^KS");
  const int N = NS > 0 ? NS : el.nsl;
  const int K = NS > 0 ? KS : el.K;
  const double ds = KIND == 0 ? el.b.ds : (KIND == 4 ? el.tp.ds : el.q.ds);
  // MIXED: this element's edges are built and multiplied in single
  // precision (the caller picks this instantiation for flagged elements)
  constexpr bool spin32 = MIXED;
  // running products of the Romberg levels: level m keeps every 2^m-th edge
  Quat Q0 = qident(), Q1 = qident(), Q2 = qident(), Q3 = qident();
  QuatC C0 = qc_ident(), C1 = qc_ident(), C2 = qc_ident(), C3 = qc_ident();

  // bend invariants of this particle: Py and Pt do not change in a bend
  double Pa2 = p.P2() - Py * Py;
  MKConst mc, mc0;
  if constexpr (Y4) {
    if (KIND == 1 || KIND == 3) { mc = mk_const(el.q4.s1, p); mc0 = mk_const(el.q4.s0, p); }
  } else {
    if (KIND == 1 || KIND == 3) mc = mk_cached(el.q, p, mkc);
  }

  // Ps and 1/Ps at the entrance edge (outside bends 1/Ps only enters Ω)
  double ps2 = fma(-Px, Px, Pa2);
  double r = KIND == 0 ? rsqrt_nr(ps2) : rsqrt_omega(ps2);
  double W = ps2 * r;
  double invPa2 = 0.0, wme = 0.0;
  // entrance Px and Ps of a bend: Y and T follow once from the two ends
  const double Px_in = Px, W_in = W;
  if (KIND == 0) {
    invPa2 = rcp_nr(Pa2);
    // W - η = (W² - η²)/(W + η) with W² - η² = (1 - η²) + (P² - 1) - Py² - Px²
    wme = (el.b.one_m_eta2 + ((p.c3 - Py * Py) - Px * Px)) * rcp_nr(W + el.b.eta);
  }

  // Fold the rotation of edge j into the running products of the levels
  // that keep it.  The entrance edge starts every level (FIRST: the
  // products are set, not multiplied into the identity).
  auto fold = [&](int j, auto first_tag) {
    constexpr bool FIRST = decltype(first_tag)::value;
    double ox, oy, oz;
    if (KIND == 0)      omega_bend(el.b, X, Px, Py, r, p, ox, oy, oz);
    else if (KIND == 4) omega_dipole(el.tp.h, el.tp.eta_h, X, Px, Py, r, p, ox, oy, oz);
    else                omega_straight(el.q.k1 * Y, el.q.k1 * X, Px, Py, r, p, ox, oy, oz);
    const double om2 = fma(ox, ox, fma(oy, oy, oz * oz));
    // Level m keeps this edge when 2^m divides j, with step w 2^m ds: the
    // rotation about Ω by 2^m times the finest angle, i.e. the finest
    // quaternion squared m times.
    const bool end_edge = j == 0 || j == N;
    if constexpr (spin32) {
      const double f = (end_edge ? 0.5 : 1.0) * ds;
      float d, sf;
      rot_deviation_f32(0.25 * f * f * om2, d, sf);
      float vx = sf * (float)(f * ox), vy = sf * (float)(f * oy), vz = sf * (float)(f * oz);
      qc_update(C0, d, vx, vy, vz);
      if (K >= 1 && (j & 1) == 0) {
        dev_square(d, vx, vy, vz);
        qc_update(C1, d, vx, vy, vz);
        if (K >= 2 && (j & 3) == 0) {
          dev_square(d, vx, vy, vz);
          qc_update(C2, d, vx, vy, vz);
          if (K >= 3 && (j & 7) == 0) {
            dev_square(d, vx, vy, vz);
            qc_update(C3, d, vx, vy, vz);
          }
        }
      }
    } else {
      // half angle θ/2 = hw |Ω|: q = (cos θ/2, sin(θ/2)/(θ/2) hw Ω)
      double c, sc;
      rot_half_series<NT>((end_edge ? el.hw2_end : el.hw2_in) * om2, a.ymax, c, sc);
      const double g = sc * (end_edge ? el.hw_end : el.hw_in);
      Quat qb = {c, g * ox, g * oy, g * oz};
      Q0 = FIRST ? qb : qmul(qb, Q0);
      if (K >= 1 && (j & 1) == 0) {
        qb = qsquare(qb);
        Q1 = FIRST ? qb : qmul(qb, Q1);
        if (K >= 2 && (j & 3) == 0) {
          qb = qsquare(qb);
          Q2 = FIRST ? qb : qmul(qb, Q2);
          if (K >= 3 && (j & 7) == 0) {
            qb = qsquare(qb);
            Q3 = FIRST ? qb : qmul(qb, Q3);
          }
        }
      }
    }
  };

  int j0 = 0;
  if constexpr (PEEL) {
    fold(0, std::true_type{});
    j0 = 1;
  }
#pragma unroll
  for (int j = j0; j <= N; ++j) {
    if (j > 0) {
      if (KIND == 0) {
        bend_step<false>(el.b, el.b.slice, BendLane{0.0, 0.0}, X, Px, Py, Y, T, W, r, wme, Pa2,
                         invPa2);
      } else {
        if (KIND == 4) {
          teapot_slice(el.tp, X, Px, Y, Py, T, p);
        } else if (Y4) {
          quad_slice4<KIND>(el.q4, mc, mc0, X, Px, Y, Py, T, p, a);
        } else {
          quad_step2<KIND>(el.q, mc, X, Px, Y, Py, T, p, a);
        }
        ps2 = p.P2() - fma(Px, Px, Py * Py);
        r = rsqrt_omega(ps2);
      }
    }
    fold(j, std::false_type{});
  }
  if (KIND == 0)
    bend_yt(el.b, el.b.whole, bend_lane(el.b, el.b.whole, p), Px_in, W_in, Px, W, Py, Y, T, invPa2);
  if constexpr (spin32) {
    Q0 = qc_to_double(C0);
    if (K >= 1) Q1 = qc_to_double(C1);
    if (K >= 2) Q2 = qc_to_double(C2);
    if (K >= 3) Q3 = qc_to_double(C3);
  }

  // Romberg tableau (§4.3 eq. romberg) with levels indexed by stride 2^m:
  // V_j[m] = (4^j V_{j-1}[m] - V_{j-1}[m+1]) / (4^j - 1), limit V_K[0].
  if (K >= 1) {
    Q0 = qextrapolate(Q0, Q1, 4.0);
    if (K >= 2) {
      Q1 = qextrapolate(Q1, Q2, 4.0);
      if (K >= 3) Q2 = qextrapolate(Q2, Q3, 4.0);
      Q0 = qextrapolate(Q0, Q1, 16.0);
      if (K >= 3) {
        Q1 = qextrapolate(Q1, Q2, 16.0);
        Q0 = qextrapolate(Q0, Q1, 64.0);
      }
    }
  }
  const double inv = rsqrt_near_one(fma(Q0.w, Q0.w, fma(Q0.x, Q0.x, fma(Q0.y, Q0.y, Q0.z * Q0.z))));
  return {Q0.w * inv, Q0.x * inv, Q0.y * inv, Q0.z * inv};
}

// Orbit only through a thick element (surrogate tracking, no spin): the
// sector bend is an exact flow and is crossed in one step; quadrupoles keep
// their slices, and matrix-kick ones take their constants from the lane's
// cache when one is passed.
template <int KIND, bool Y4 = false>
__device__ __forceinline__ void thick_orbit(const DevElem& el, double& X, double& Px, double& Y,
                                            double& Py, double& T, const Particle& p,
                                            const TrackArgs& a, MKCache* mkc = nullptr) {
  if (KIND == 0) {
    const double Pa2 = p.P2() - Py * Py;
    const double ps2 = fma(-Px, Px, Pa2);
    double r = rsqrt_nr(ps2);
    double W = ps2 * r;
    double wme = (el.b.one_m_eta2 + ((p.c3 - Py * Py) - Px * Px)) * rcp_nr(W + el.b.eta);
    bend_step(el.b, el.b.whole, bend_lane(el.b, el.b.whole, p), X, Px, Py, Y, T, W, r, wme, Pa2,
              rcp_nr(Pa2));
    return;
  }
  if constexpr (Y4) {
    MKConst m1, m0;
    if (KIND == 1 || KIND == 3) { m1 = mk_const(el.q4.s1, p); m0 = mk_const(el.q4.s0, p); }
    for (int j = 0; j < el.nsl; ++j) quad_slice4<KIND>(el.q4, m1, m0, X, Px, Y, Py, T, p, a);
    return;
  }
  MKConst mc;
  if (KIND == 1 || KIND == 3) mc = mk_cached(el.q, p, mkc);
  for (int j = 0; j < el.nsl; ++j) {
    if (KIND == 4) teapot_slice(el.tp, X, Px, Y, Py, T, p);
    else           quad_step2<KIND>(el.q, mc, X, Px, Y, Py, T, p, a);
  }
}

// Piece-wise constant spin through a thick element (§4.1 eq. pwcSpin): one
// rotation by ds·Ω per slice, later slices on the left, Ω taken between the
// two half kicks of a drift-kick slice (PLACE == P_KICK; KIND 2 or 4) or at
// the middle of the slice (P_MIDPOINT: the element carries 2N orbit half
// slices and the rotation follows every odd one).
template <int NT, int KIND, int PLACE, bool Y4 = false>
__device__ __forceinline__ Quat pwc_element(const DevElem& el, double& X, double& Px, double& Y,
                                            double& Py, double& T, const Particle& p,
                                            const TrackArgs& a) {
  const double ds_orb = KIND == 0 ? el.b.ds : (KIND == 4 ? el.tp.ds : el.q.ds);
  const double w = PLACE == P_MIDPOINT ? 2.0 * ds_orb : ds_orb;   // spin step
  Quat Q = qident();
  MKConst mc, mc0;
  if constexpr (Y4) {
    if (KIND == 1 || KIND == 3) { mc = mk_const(el.q4.s1, p); mc0 = mk_const(el.q4.s0, p); }
  } else {
    if (KIND == 1 || KIND == 3) mc = mk_const(el.q, p);
  }
  double Pa2 = 0.0, invPa2 = 0.0, W = 0.0, r = 0.0, wme = 0.0;
  BendLane bl{0.0, 0.0};
  if (KIND == 0) {
    bl = bend_lane(el.b, el.b.slice, p);
    Pa2 = p.P2() - Py * Py;
    invPa2 = rcp_nr(Pa2);
    const double ps2 = fma(-Px, Px, Pa2);
    r = rsqrt_nr(ps2);
    W = ps2 * r;
    wme = (el.b.one_m_eta2 + ((p.c3 - Py * Py) - Px * Px)) * rcp_nr(W + el.b.eta);
  }
  for (int j = 1; j <= el.nsl; ++j) {
    if (PLACE == P_KICK) {
      if (KIND == 4) {
        teapot_drift(el.tp, X, Px, Y, Py, T, p);
        teapot_kick(el.tp, 0.5 * el.tp.ds, X, Px);
      } else {
        drift(el.q.hds, X, Px, Y, Py, T, p, a.inv_beta0);
        Px = fma(-0.5 * el.q.k1ds, X, Px);
        Py = fma(0.5 * el.q.k1ds, Y, Py);
      }
    } else if (KIND == 0) {
      bend_step(el.b, el.b.slice, bl, X, Px, Py, Y, T, W, r, wme, Pa2, invPa2);
    } else if (KIND == 4) {
      teapot_slice(el.tp, X, Px, Y, Py, T, p);
    } else if (Y4) {
      quad_slice4<KIND>(el.q4, mc, mc0, X, Px, Y, Py, T, p, a);
    } else {
      quad_step2<KIND>(el.q, mc, X, Px, Y, Py, T, p, a);
    }
    if (PLACE == P_KICK || (j & 1)) {
      if (KIND != 0) r = rsqrt_nr(p.P2() - fma(Px, Px, Py * Py));
      double ox, oy, oz;
      if (KIND == 0)      omega_bend(el.b, X, Px, Py, r, p, ox, oy, oz);
      else if (KIND == 4) omega_dipole(el.tp.h, el.tp.eta_h, X, Px, Py, r, p, ox, oy, oz);
      else                omega_straight(el.q.k1 * Y, el.q.k1 * X, Px, Py, r, p, ox, oy, oz);
      double c, sfac;
      rot_half_angle<NT>(0.25 * w * w * fma(ox, ox, fma(oy, oy, oz * oz)), a.ymax, c, sfac);
      const double g = sfac * w;
      Q = qmul(Quat{c, g * ox, g * oy, g * oz}, Q);
    }
    if (PLACE == P_KICK) {
      if (KIND == 4) {
        teapot_kick(el.tp, 0.5 * el.tp.ds, X, Px);
        teapot_drift(el.tp, X, Px, Y, Py, T, p);
      } else {
        Px = fma(-0.5 * el.q.k1ds, X, Px);
        Py = fma(0.5 * el.q.k1ds, Y, Py);
        drift(el.q.hds, X, Px, Y, Py, T, p, a.inv_beta0);
      }
    }
  }
  const double inv = rsqrt_near_one(fma(Q.w, Q.w, fma(Q.x, Q.x, fma(Q.y, Q.y, Q.z * Q.z))));
  return {Q.w * inv, Q.x * inv, Q.y * inv, Q.z * inv};
}

// Solenoid (§3.7, §4.4): entrance fringe kick, body slices with the spin at
// the slice edges (Romberg) or at the slice middles (PLACE == P_MIDPOINT: 2N
// orbit half slices), exit fringe kick; later rotations on the left.
template <int NT, int PLACE>
__device__ __forceinline__ Quat solenoid_element(const DevElem& el, double& X, double& Px,
                                                 double& Y, double& Py, double& T,
                                                 const Particle& p, const TrackArgs& a) {
  const SolenoidParams& sp = el.sol;
  auto rot = [&](double wx, double wy, double wz) {
    double c, sfac;
    rot_half_angle<NT>(0.25 * fma(wx, wx, fma(wy, wy, wz * wz)), a.ymax, c, sfac);
    return Quat{c, sfac * wx, sfac * wy, sfac * wz};
  };
  double wx, wy, wz;
  solenoid_fringe(sp, 1.0, X, Px, Y, Py, p, wx, wy, wz);
  const Quat qin = rot(wx, wy, wz);
  const SolState st = sol_state<NT>(sp, X, Px, Y, Py, p, a.ymax, a.inv_beta0);
  Quat Q;
  if (PLACE == P_MIDPOINT) {
    Q = qident();
    const double w = 2.0 * sp.ds;
    for (int j = 1; j <= el.nsl; ++j) {
      solenoid_slice(sp, st, X, Px, Y, Py, T);
      if (j & 1) {
        double ox, oy, oz;
        omega_solenoid(sp, st, X, Px, Y, Py, p, ox, oy, oz);
        Q = qmul(rot(w * ox, w * oy, w * oz), Q);
      }
    }
  } else {
    // Romberg levels over the slice edges, as for the other thick elements
    const int N = el.nsl, K = el.K;
    const double ds = sp.ds;
    Quat Q0 = qident(), Q1 = qident(), Q2 = qident(), Q3 = qident();
    for (int j = 0; j <= N; ++j) {
      if (j > 0) solenoid_slice(sp, st, X, Px, Y, Py, T);
      double ox, oy, oz;
      omega_solenoid(sp, st, X, Px, Y, Py, p, ox, oy, oz);
      const double f = ((j == 0 || j == N) ? 0.5 : 1.0) * ds;
      Quat qb = rot(f * ox, f * oy, f * oz);
      Q0 = qmul(qb, Q0);
      if (K >= 1 && (j & 1) == 0) {
        qb = qsquare(qb);
        Q1 = qmul(qb, Q1);
        if (K >= 2 && (j & 3) == 0) {
          qb = qsquare(qb);
          Q2 = qmul(qb, Q2);
          if (K >= 3 && (j & 7) == 0) {
            qb = qsquare(qb);
            Q3 = qmul(qb, Q3);
          }
        }
      }
    }
    if (K >= 1) {
      Q0 = qextrapolate(Q0, Q1, 4.0);
      if (K >= 2) {
        Q1 = qextrapolate(Q1, Q2, 4.0);
        if (K >= 3) Q2 = qextrapolate(Q2, Q3, 4.0);
        Q0 = qextrapolate(Q0, Q1, 16.0);
        if (K >= 3) {
          Q1 = qextrapolate(Q1, Q2, 16.0);
          Q0 = qextrapolate(Q0, Q1, 64.0);
        }
      }
    }
    Q = Q0;
  }
  const double inv = rsqrt_near_one(fma(Q.w, Q.w, fma(Q.x, Q.x, fma(Q.y, Q.y, Q.z * Q.z))));
  Q = {Q.w * inv, Q.x * inv, Q.y * inv, Q.z * inv};
  solenoid_fringe(sp, -1.0, X, Px, Y, Py, p, wx, wy, wz);
  return qmul(rot(wx, wy, wz), qmul(Q, qin));
}

// Rectangular bend (§3.2, §4.5): frame rotation by φ^entr into the magnet
// (the spin components turn with the frame about ŷ), entrance fringe and its
// spin kick, body slices with Romberg over the edges or midpoint rotations,
// X referred to the design orbit's exit point (eq. Xoffset), exit fringe and
// kick, frame rotation by -φ^exit out; T referred to the design arc (eq.
// Toffset).
template <int NT, int PLACE>
__device__ __forceinline__ Quat rbend_element(const DevElem& el, double& X, double& Px, double& Y,
                                              double& Py, double& T, const Particle& p,
                                              const TrackArgs& a) {
  const RbendParams& rb = el.rb;
  auto rot = [&](double wx, double wy, double wz) {
    double c, sfac;
    rot_half_angle<NT>(0.25 * fma(wx, wx, fma(wy, wy, wz * wz)), a.ymax, c, sfac);
    return Quat{c, sfac * wx, sfac * wy, sfac * wz};
  };
  // fringe kick ±fb Y [G(γ - 1) Px x̂ - (1 + G) ẑ]
  auto fringe_spin = [&](double sign) {
    const double f = sign * rb.fb * Y;
    return rot(f * p.a2() * Px, 0.0, -f * (1.0 + a.G));
  };
  rbend_rotate(rb.in, X, Px, Y, Py, T, p);
  rbend_fringe(rb, 1.0, X, Px, Y, Py, T, p);
  const Quat qin = fringe_spin(1.0);
  Quat Q;
  auto omega_at = [&](double& ox, double& oy, double& oz) {
    const double r = rsqrt_nr(p.P2() - fma(Px, Px, Py * Py));
    omega_dipole(0.0, rb.fb, X, Px, Py, r, p, ox, oy, oz);
  };
  if (PLACE == P_MIDPOINT) {
    Q = qident();
    const double w = 2.0 * rb.ds;
    for (int j = 1; j <= el.nsl; ++j) {
      rbend_body(rb, rb.ds, X, Px, Y, Py, T, p);
      if (j & 1) {
        double ox, oy, oz;
        omega_at(ox, oy, oz);
        Q = qmul(rot(w * ox, w * oy, w * oz), Q);
      }
    }
  } else {
    const int N = el.nsl, K = el.K;
    Quat Q0 = qident(), Q1 = qident(), Q2 = qident(), Q3 = qident();
    for (int j = 0; j <= N; ++j) {
      if (j > 0) rbend_body(rb, rb.ds, X, Px, Y, Py, T, p);
      double ox, oy, oz;
      omega_at(ox, oy, oz);
      const double f = ((j == 0 || j == N) ? 0.5 : 1.0) * rb.ds;
      Quat qb = rot(f * ox, f * oy, f * oz);
      Q0 = qmul(qb, Q0);
      if (K >= 1 && (j & 1) == 0) {
        qb = qsquare(qb);
        Q1 = qmul(qb, Q1);
        if (K >= 2 && (j & 3) == 0) {
          qb = qsquare(qb);
          Q2 = qmul(qb, Q2);
          if (K >= 3 && (j & 7) == 0) {
            qb = qsquare(qb);
            Q3 = qmul(qb, Q3);
          }
        }
      }
    }
    if (K >= 1) {
      Q0 = qextrapolate(Q0, Q1, 4.0);
      if (K >= 2) {
        Q1 = qextrapolate(Q1, Q2, 4.0);
        if (K >= 3) Q2 = qextrapolate(Q2, Q3, 4.0);
        Q0 = qextrapolate(Q0, Q1, 16.0);
        if (K >= 3) {
          Q1 = qextrapolate(Q1, Q2, 16.0);
          Q0 = qextrapolate(Q0, Q1, 64.0);
        }
      }
    }
    Q = Q0;
  }
  const double inv = rsqrt_near_one(fma(Q.w, Q.w, fma(Q.x, Q.x, fma(Q.y, Q.y, Q.z * Q.z))));
  Q = {Q.w * inv, Q.x * inv, Q.y * inv, Q.z * inv};
  X -= rb.xoff;
  const Quat qout = fringe_spin(-1.0);
  rbend_fringe(rb, -1.0, X, Px, Y, Py, T, p);
  rbend_rotate(rb.out, X, Px, Y, Py, T, p);
  T += rb.larc_ib0;
  const Quat qfi = {rb.in.qw, 0.0, rb.in.qy, 0.0}, qfo = {rb.out.qw, 0.0, rb.out.qy, 0.0};
  return qmul(qfo, qmul(qout, qmul(Q, qmul(qin, qfi))));
}

// Spin kick across the thin fringe of a normal 2m-pole face crossed about
// normally (§4.5 eq. skfringe): a rotation about ẑ by
// -sign (1 + G) (b_m/(Bρ)0) Im[(X + iY)^m]/m, sign +1 at the entrance.
// Sector bends (KIND 0, 4) are m = 1 with b1/(Bρ)0 = ηh; quadrupoles m = 2
// with b2/(Bρ)0 = k1.
template <int NT, int KIND>
__device__ __forceinline__ Quat fringe_kick(const DevElem& el, double X, double Y, double sign,
                                            const TrackArgs& a) {
  const double im = (KIND == 0) ? el.b.eta_h * Y : (KIND == 4) ? el.tp.eta_h * Y : el.q.k1 * X * Y;
  const double w = -sign * (1.0 + a.G) * im;
  double c, sfac;
  rot_half_angle<NT>(0.25 * w * w, a.ymax, c, sfac);
  return Quat{c, 0.0, 0.0, sfac * w};
}

// Spin and orbit of a thick element with the extended methods: TEAPOT bends,
// the piece-wise constant placements and the fringe spin kicks.
template <int NT, int KIND, bool Y4>
__device__ __forceinline__ Quat thick_body_ext(const DevElem& el, double& X, double& Px, double& Y,
                                            double& Py, double& T, const Particle& p,
                                            const TrackArgs& a) {
  if (el.place == P_KICK) {   // one kick per slice: not with the composed slices
    if constexpr (!Y4 && (KIND == 2 || KIND == 4))
      return pwc_element<NT, KIND, P_KICK>(el, X, Px, Y, Py, T, p, a);
    return qident();   // rejected on the host
  }
  if (el.place == P_MIDPOINT)
    return pwc_element<NT, KIND, P_MIDPOINT, Y4>(el, X, Px, Y, Py, T, p, a);
  return thick_element<NT, KIND, false, Y4, false>(el, X, Px, Y, Py, T, p, a);
}

// The body between the fringe spin kicks of its faces (elements flagged
// F_FRINGE): q_exit · Q_body · q_entrance.
template <int NT, int KIND, bool Y4>
__device__ __forceinline__ Quat thick_ext_y(const DevElem& el, double& X, double& Px, double& Y,
                                         double& Py, double& T, const Particle& p,
                                         const TrackArgs& a) {
  if (!(el.flags & F_FRINGE)) return thick_body_ext<NT, KIND, Y4>(el, X, Px, Y, Py, T, p, a);
  const Quat qin = fringe_kick<NT, KIND>(el, X, Y, 1.0, a);
  const Quat Q = thick_body_ext<NT, KIND, Y4>(el, X, Px, Y, Py, T, p, a);
  return qmul(fringe_kick<NT, KIND>(el, X, Y, -1.0, a), qmul(Q, qin));
}

template <int NT, int KIND>
__device__ __forceinline__ Quat thick_ext(const DevElem& el, double& X, double& Px, double& Y,
                                       double& Py, double& T, const Particle& p,
                                       const TrackArgs& a) {
  if constexpr (KIND == 1 || KIND == 2 || KIND == 3) {
    if (el.orbit == M_DKD4 || el.orbit == M_MK4)
      return thick_ext_y<NT, KIND, true>(el, X, Px, Y, Py, T, p, a);
  }
  return thick_ext_y<NT, KIND, false>(el, X, Px, Y, Py, T, p, a);
}

template <int NT>
__device__ __forceinline__ Quat thin_element(const DevElem& e, double X, double& Px, double Y,
                                             double& Py, const Particle& p, const TrackArgs& a) {
  const double hk1 = 0.5 * e.t.k1l, hk2 = 0.5 * e.t.k2l;
  Px -= fma(hk1, X, 0.5 * hk2 * (X * X - Y * Y));
  Py += fma(hk1, Y, hk2 * X * Y);
  double ps2 = p.P2() - fma(Px, Px, Py * Py);
  double r = rsqrt_omega(ps2);
  double bx = fma(e.t.k2l * X, Y, e.t.k1l * Y);
  double by = fma(e.t.k1l, X, 0.5 * e.t.k2l * (X * X - Y * Y));
  double ox, oy, oz;
  omega_straight(bx, by, Px, Py, r, p, ox, oy, oz);
  const double y = 0.25 * fma(ox, ox, fma(oy, oy, oz * oz));
  Px -= fma(hk1, X, 0.5 * hk2 * (X * X - Y * Y));
  Py += fma(hk1, Y, hk2 * X * Y);
  double c, sfac;
  rot_half_angle<NT>(y, a.ymax, c, sfac);
  return {c, sfac * ox, sfac * oy, sfac * oz};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// SURR: surrogate tracking; lanes with fallback[j] == 0 leave the spin to the
// network (the caller rotates it), and waves without a fallback lane skip the
// spin arithmetic altogether.
// Sector bends and DKD/MK quadrupoles of the standard rings, with unrolled
// bodies for their slice counts and Romberg depths: sector bends with 8
// slices and 3 or 4 rows, MK quadrupoles with 4 slices and 3 rows, DKD
// quadrupoles with 8 slices and 3 rows; other elements take the loop.
// S32: the element's spin edges in single precision (mixed mode).
template <int NT, bool S32>
__device__ __forceinline__ Quat standard_thick(const DevElem& e, double& X, double& Px, double& Y,
                                               double& Py, double& T, const Particle& p,
                                               const TrackArgs& a, MKCache* mkc) {
  if (e.kind == K_SBEND) {
    if (e.nsl == 8 && e.K == 3) return thick_element<NT, 0, S32, false, true, 8, 3>(e, X, Px, Y, Py, T, p, a);
    if (e.nsl == 8 && e.K == 2) return thick_element<NT, 0, S32, false, true, 8, 2>(e, X, Px, Y, Py, T, p, a);
    return thick_element<NT, 0, S32>(e, X, Px, Y, Py, T, p, a);
  }
  if (e.orbit != M_MK) {
    if (e.nsl == 8 && e.K == 2) return thick_element<NT, 2, S32, false, true, 8, 2>(e, X, Px, Y, Py, T, p, a);
    return thick_element<NT, 2, S32>(e, X, Px, Y, Py, T, p, a);
  }
  if (e.nsl == 4 && e.K == 2) {
    if (e.q.k1 >= 0.0) return thick_element<NT, 1, S32, false, true, 4, 2>(e, X, Px, Y, Py, T, p, a, mkc);
    return thick_element<NT, 3, S32, false, true, 4, 2>(e, X, Px, Y, Py, T, p, a, mkc);
  }
  if (e.q.k1 >= 0.0) return thick_element<NT, 1, S32>(e, X, Px, Y, Py, T, p, a, mkc);
  return thick_element<NT, 3, S32>(e, X, Px, Y, Py, T, p, a, mkc);
}

// EXT: the kernel also knows the drift-kick sector bend and the piece-wise
// constant spin placements (kept out of the other instantiations so that
// their register allocation is not shaped by code they never run).
// ORBIT: the network turns of the particles on the network, the first
// a.feat_n lanes of the lane order: the orbit only, with the network's inputs
// written at the start of each turn. With ORBIT false, SURR launches leave
// those lanes to the ORBIT launch and take the particles that fall back.
template <int NT, bool MIXED, bool SURR, bool EXT, bool ORBIT>
__device__ __forceinline__ void track_body(const TrackArgs a) {
  __shared__ double red[kBlock / 64][4];
  // Cold per-lane data in LDS: the spin (touched once per turn) and the
  // orbit at the current element's entrance (read back only on a loss).
  __shared__ double cold[8][kBlock];
  __shared__ double mk_slot[EXT ? 1 : kMKWords][kBlock];
  const int tid = threadIdx.x;
  const int64_t g = (int64_t)blockIdx.x * kBlock + tid;
  const bool valid = ORBIT ? g < a.feat_n : (g < a.n && !(SURR && g < a.feat_n));
  const int64_t j = (valid && a.perm) ? (int64_t)a.perm[g] : g;
  int32_t status = valid ? a.alive[j] : 0;
  bool live = status == 1;
  const int64_t n = a.n;

  double X = 0, Px = 0, Y = 0, Py = 0, T = 0, Pt = 0;
  cold[0][tid] = 0.0; cold[1][tid] = 0.0; cold[2][tid] = 0.0;
  if (valid) {
    X = a.z[j]; Px = a.z[n + j]; Y = a.z[2 * n + j]; Py = a.z[3 * n + j];
    T = a.z[4 * n + j]; Pt = a.z[5 * n + j];
    cold[0][tid] = a.spin[j]; cold[1][tid] = a.spin[n + j]; cold[2][tid] = a.spin[2 * n + j];
  }
  // Without reports the kernel has no barrier, so a wave with no live lane
  // (a replay of a few particles) may leave at once.
  if (a.report_every == 0 && !__any(live)) {
    if (ORBIT && a.turns_done && g < a.feat_n) a.turns_done[g] = 0;
    return;
  }
  const Particle p = make_particle(Pt, a);
  MKCache mkc{mk_slot, tid, __builtin_nan(""), __builtin_nan("")};
  Quat qturn = qident();
  const bool spin_lane = !ORBIT && (!SURR || (valid && a.fallback[j] != 0));
  // The lattice is read-only for the whole launch: reading it through the
  // constant address space lets the uniform loads go through the scalar cache.
  const ConstElem* tab = (const ConstElem*)(a.tab);
  const ConstSeq* seq = (const ConstSeq*)(a.seq);

  int turns_done = 0;
  for (int t = 1; t <= a.turns; ++t) {
    const bool was_live = live;
    if (was_live) qturn = qident();
    if (ORBIT && a.feat && live) {
      // the network's inputs at the start of this turn
      float* f = a.feat + ((int64_t)(t - 1) * a.feat_n + g) * a.feat_n_in;
      f[0] = (float)((X - a.feat_center[0]) * a.feat_inv_scale[0]);
      f[1] = (float)((Px - a.feat_center[1]) * a.feat_inv_scale[1]);
      f[2] = (float)((Y - a.feat_center[2]) * a.feat_inv_scale[2]);
      f[3] = (float)((Py - a.feat_center[3]) * a.feat_inv_scale[3]);
      f[4] = (float)((T - a.feat_center[4]) * a.feat_inv_scale[4]);
      f[5] = (float)((Pt - a.feat_center[5]) * a.feat_inv_scale[5]);
      if (a.feat_n_in == 7) f[6] = (float)a.feat_extra;
    }
    for (int ie = 0; ie < a.n_elems; ++ie) {
      const DevElem e = load_elem(tab + seq[ie]);
      if (!live) continue;
      if (e.kind == K_DRIFT) {           // no spin; the entrance state is cheap to keep
        const double X0 = X, Y0 = Y, T0 = T;
        drift(e.d.L, X, Px, Y, Py, T, p, a.inv_beta0);
        if (!(fabs(X) <= a.aperture && fabs(Y) <= a.aperture && isfinite(T))) {
          X = X0; Y = Y0; T = T0;
          live = false;
          status = -(1 + ie);
        }
        continue;
      }
      cold[3][tid] = X; cold[4][tid] = Px; cold[5][tid] = Y; cold[6][tid] = Py; cold[7][tid] = T;
      Quat q;
      bool spin = true;
      if (SURR && !__any(spin_lane)) {   // no lane of this wave needs the spin
        spin = false;
        if (e.kind == K_SBEND) {
          if (EXT && e.orbit == M_TEAPOT) thick_orbit<4>(e, X, Px, Y, Py, T, p, a);
          else                            thick_orbit<0>(e, X, Px, Y, Py, T, p, a);
        } else if (EXT && e.kind == K_QUAD && (e.orbit == M_DKD4 || e.orbit == M_MK4)) {
          if (e.orbit == M_DKD4)  thick_orbit<2, true>(e, X, Px, Y, Py, T, p, a);
          else if (e.q.k1 >= 0.0) thick_orbit<1, true>(e, X, Px, Y, Py, T, p, a);
          else                    thick_orbit<3, true>(e, X, Px, Y, Py, T, p, a);
        } else if (e.kind == K_QUAD) {
          MKCache* const c = EXT ? nullptr : &mkc;   // (the extended kernels keep no cache)
          if (e.orbit != M_MK)    thick_orbit<2>(e, X, Px, Y, Py, T, p, a);
          else if (e.q.k1 >= 0.0) thick_orbit<1>(e, X, Px, Y, Py, T, p, a, c);
          else                    thick_orbit<3>(e, X, Px, Y, Py, T, p, a, c);
        } else if (EXT && e.kind == K_RBEND) {
          rbend_rotate(e.rb.in, X, Px, Y, Py, T, p);
          rbend_fringe(e.rb, 1.0, X, Px, Y, Py, T, p);
          rbend_body(e.rb, e.rb.L, X, Px, Y, Py, T, p);
          X -= e.rb.xoff;
          rbend_fringe(e.rb, -1.0, X, Px, Y, Py, T, p);
          rbend_rotate(e.rb.out, X, Px, Y, Py, T, p);
          T += e.rb.larc_ib0;
        } else if (EXT && e.kind == K_SOLENOID) {
          const SolState st = sol_state<NT>(e.sol, X, Px, Y, Py, p, a.ymax, a.inv_beta0);
          for (int jj = 0; jj < e.nsl; ++jj) solenoid_slice(e.sol, st, X, Px, Y, Py, T);
        } else if (e.kind == K_THIN) {
          const double hk1 = 0.5 * e.t.k1l, hk2 = 0.5 * e.t.k2l;
          for (int h = 0; h < 2; ++h) {
            Px -= fma(hk1, X, 0.5 * hk2 * (X * X - Y * Y));
            Py += fma(hk1, Y, hk2 * X * Y);
          }
        }
      } else if (EXT && e.kind == K_RBEND) {
        if (e.place == P_MIDPOINT) q = rbend_element<NT, P_MIDPOINT>(e, X, Px, Y, Py, T, p, a);
        else                       q = rbend_element<NT, P_EDGES>(e, X, Px, Y, Py, T, p, a);
      } else if (EXT && e.kind == K_SOLENOID) {
        if (e.place == P_MIDPOINT) q = solenoid_element<NT, P_MIDPOINT>(e, X, Px, Y, Py, T, p, a);
        else                       q = solenoid_element<NT, P_EDGES>(e, X, Px, Y, Py, T, p, a);
      } else if (EXT && (e.kind == K_SBEND || e.kind == K_QUAD)) {
        if (e.kind == K_SBEND) {
          if (e.orbit == M_TEAPOT) q = thick_ext<NT, 4>(e, X, Px, Y, Py, T, p, a);
          else                     q = thick_ext<NT, 0>(e, X, Px, Y, Py, T, p, a);
        } else {
          if (e.orbit == M_DKD || e.orbit == M_DKD4) q = thick_ext<NT, 2>(e, X, Px, Y, Py, T, p, a);
          else if (e.q.k1 >= 0.0) q = thick_ext<NT, 1>(e, X, Px, Y, Py, T, p, a);
          else                    q = thick_ext<NT, 3>(e, X, Px, Y, Py, T, p, a);
        }
      } else switch (e.kind) {
        case K_SBEND:
        case K_QUAD:
          // the mixed kernel carries both instantiations; an element runs one
          if (MIXED && (e.flags & F_SPIN32))
            q = standard_thick<NT, MIXED>(e, X, Px, Y, Py, T, p, a, &mkc);
          else
            q = standard_thick<NT, false>(e, X, Px, Y, Py, T, p, a, &mkc);
          break;
        case K_THIN:
          q = thin_element<NT>(e, X, Px, Y, Py, p, a);
          break;
        case K_SNAKE:
          q = {e.s.qw, e.s.qx, e.s.qy, e.s.qz};
          break;
        default:
          spin = false;
          break;
      }
      const bool ok = fabs(X) <= a.aperture && fabs(Y) <= a.aperture && isfinite(Px) &&
                      isfinite(Py) && isfinite(T);
      if (!ok) {
        X = cold[3][tid]; Px = cold[4][tid]; Y = cold[5][tid]; Py = cold[6][tid]; T = cold[7][tid];
        live = false;
        status = -(1 + ie);
        continue;
      }
      if (spin) qturn = qmul(q, qturn);
    }
    if (was_live && live) ++turns_done;
    // A particle lost during this turn still receives the rotation of the
    // elements it completed before the loss.
    double sx = cold[0][tid], sy = cold[1][tid], sz = cold[2][tid];
    if (was_live && spin_lane) {
      qrotate(qturn, sx, sy, sz);
      cold[0][tid] = sx; cold[1][tid] = sy; cold[2][tid] = sz;
    }
    if (a.report_every > 0 && t % a.report_every == 0) {
      double v0 = live ? sx : 0.0, v1 = live ? sy : 0.0, v2 = live ? sz : 0.0;
      double v3 = live ? 1.0 : 0.0;
      v0 = wave_sum(v0); v1 = wave_sum(v1); v2 = wave_sum(v2); v3 = wave_sum(v3);
      const int lane = tid & 63, wv = tid >> 6;
      if (lane == 0) { red[wv][0] = v0; red[wv][1] = v1; red[wv][2] = v2; red[wv][3] = v3; }
      __syncthreads();
      if (tid < 4) {
        double s = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) s += red[k][tid];
        const int rep = t / a.report_every - 1;
        a.partials[((int64_t)rep * a.n_blocks + blockIdx.x) * 4 + tid] = s;
      }
      __syncthreads();
    }
  }

  if (ORBIT && a.turns_done && g < a.feat_n) a.turns_done[g] = turns_done;
  if (valid && a.alive[j] == 1) {
    a.z[j] = X; a.z[n + j] = Px; a.z[2 * n + j] = Y; a.z[3 * n + j] = Py; a.z[4 * n + j] = T;
    if (!ORBIT) {
      a.spin[j] = cold[0][tid]; a.spin[n + j] = cold[1][tid]; a.spin[2 * n + j] = cold[2][tid];
    }
    a.alive[j] = status;
    if (a.qout) {
      a.qout[j] = qturn.w; a.qout[n + j] = qturn.x; a.qout[2 * n + j] = qturn.y;
      a.qout[3 * n + j] = qturn.z;
    }
  }
}

template <int NT, bool MIXED, bool SURR, bool EXT>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((MIXED || SURR || EXT) ? ST_WAVES_PER_EU_WIDE : ST_WAVES_PER_EU)))
track_kernel(const TrackArgs a) {
  track_body<NT, MIXED, SURR, EXT, false>(a);
}

// Without the spin arithmetic the orbit push needs about 140 registers, so
// three waves share a SIMD (the LDS of three workgroups fits a CU).
template <int NT, bool EXT>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(ST_WAVES_PER_EU_ORBIT)))
orbit_kernel(const TrackArgs a) {
  track_body<NT, false, true, EXT, true>(a);
}

// Deterministic second pass of the polarization reduction: one block per
// report sums the per-block partials in a fixed order.
__global__ void __launch_bounds__(256) reduce_polarization_kernel(const double* partials,
                                                                  int n_blocks, double* out) {
  __shared__ double acc[256][4];
  const int rep = blockIdx.x;
  double s[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < n_blocks; b += 256)
    for (int c = 0; c < 4; ++c) s[c] += partials[((int64_t)rep * n_blocks + b) * 4 + c];
  for (int c = 0; c < 4; ++c) acc[threadIdx.x][c] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 4; ++c) acc[threadIdx.x][c] += acc[threadIdx.x + w][c];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nal = acc[0][3];
    const double inv = nal > 0 ? 1.0 / nal : 0.0;
    out[rep * 4 + 0] = acc[0][0] * inv;
    out[rep * 4 + 1] = acc[0][1] * inv;
    out[rep * 4 + 2] = acc[0][2] * inv;
    out[rep * 4 + 3] = nal;
  }
}

}  // namespace

int track_block_size() { return kBlock; }

template <bool MIXED, bool SURR, bool EXT>
hipError_t launch_nt(const TrackArgs& a, int nt, hipStream_t stream) {
  const dim3 grid((unsigned)a.n_blocks), block(kBlock);
  switch (nt) {
    case 5:  hipLaunchKernelGGL((track_kernel<5, MIXED, SURR, EXT>), grid, block, 0, stream, a); break;
    case 6:  hipLaunchKernelGGL((track_kernel<6, MIXED, SURR, EXT>), grid, block, 0, stream, a); break;
    case 8:  hipLaunchKernelGGL((track_kernel<8, MIXED, SURR, EXT>), grid, block, 0, stream, a); break;
    case 12: hipLaunchKernelGGL((track_kernel<12, MIXED, SURR, EXT>), grid, block, 0, stream, a); break;
    default: hipLaunchKernelGGL((track_kernel<16, MIXED, SURR, EXT>), grid, block, 0, stream, a); break;
  }
  return hipGetLastError();
}

template <bool EXT>
hipError_t launch_orbit(const TrackArgs& a, int nt, hipStream_t stream) {
  const dim3 grid((unsigned)((a.feat_n + kBlock - 1) / kBlock)), block(kBlock);
  switch (nt) {
    case 5:  hipLaunchKernelGGL((orbit_kernel<5, EXT>), grid, block, 0, stream, a); break;
    case 6:  hipLaunchKernelGGL((orbit_kernel<6, EXT>), grid, block, 0, stream, a); break;
    case 8:  hipLaunchKernelGGL((orbit_kernel<8, EXT>), grid, block, 0, stream, a); break;
    case 12: hipLaunchKernelGGL((orbit_kernel<12, EXT>), grid, block, 0, stream, a); break;
    default: hipLaunchKernelGGL((orbit_kernel<16, EXT>), grid, block, 0, stream, a); break;
  }
  return hipGetLastError();
}

// Surrogate turns: the particles on the network (the first a.feat_n lanes of
// the lane order) on the orbit-only kernel, then the ones that fall back on
// the full kernel, whose workgroups below a.feat_n leave at once.
template <bool EXT>
hipError_t launch_surrogate(const TrackArgs& a, int nt, hipStream_t stream) {
  if (a.feat_n > 0) {
    const hipError_t e = launch_orbit<EXT>(a, nt, stream);
    if (e != hipSuccess) return e;
  }
  if (a.feat_n >= a.n) return hipSuccess;
  return launch_nt<false, true, EXT>(a, nt, stream);
}

hipError_t launch_track(const TrackArgs& a, int nt, bool mixed, bool ext, hipStream_t stream) {
  // the extended methods run in double precision only
  if (ext) return a.fallback ? launch_surrogate<true>(a, nt, stream)
                             : launch_nt<false, false, true>(a, nt, stream);
  if (a.fallback) return launch_surrogate<false>(a, nt, stream);
  return mixed ? launch_nt<true, false, false>(a, nt, stream)
               : launch_nt<false, false, false>(a, nt, stream);
}

hipError_t launch_reduce_polarization(const double* partials, int n_blocks, int n_reports,
                                      double* out, hipStream_t stream) {
  if (n_reports <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_polarization_kernel, dim3(n_reports), dim3(256), 0, stream, partials,
                     n_blocks, out);
  return hipGetLastError();
}

}  // namespace st

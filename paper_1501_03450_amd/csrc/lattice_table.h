// Device-side lattice representation shared by the host setup code and the
// tracking kernels.
//
// A ring of ~1.7k elements repeats a handful of distinct magnets, so the
// lattice is stored as a small table of unique elements with every per-element
// constant precomputed on the host (trigonometry of the bend angle per slice,
// reciprocals, snake quaternions), plus a 32-bit index sequence.  The kernels
// walk the sequence with wave-uniform loads, so the table is read through the
// scalar cache and every branch on the element kind is uniform.
#pragma once

#include <stdint.h>

namespace st {

enum : int32_t { K_MARKER = 0, K_DRIFT = 1, K_SBEND = 2, K_QUAD = 3, K_THIN = 4, K_SNAKE = 5,
                 K_SOLENOID = 6, K_RBEND = 7 };
enum : int32_t { M_EXACT = 0, M_DKD = 1, M_MK = 2, M_TEAPOT = 3, M_DKD4 = 4, M_MK4 = 5 };
// spin placement in thick elements: Romberg over the slice edges, or one
// piece-wise constant rotation per slice between the half kicks or at the
// slice's middle
enum : int32_t { P_EDGES = 0, P_KICK = 1, P_MIDPOINT = 2 };

constexpr int kMaxRows = 4;   // Romberg tableau rows supported by the kernels

// Per-kind parameters, precomputed on the host.
struct BendStep {          // constants of one exact step of length s
  double cs, sn, omc;      // cos(h s), sin(h s), 1 - cos(h s)
  double s_eta;            // s / η
  double tconst;           // (1 - 1/η) s / β0
};
struct BendParams {        // sector bend (§3.1)
  double ds;               // slice length L/N
  double h, eta, eta_h, inv_eta_h;
  double one_m_eta2;       // 1 - η²
  BendStep slice;          // s = ds
  BendStep whole;          // s = L (orbit-only passes)
};
struct QuadParams {        // quadrupole (§3.3, §3.4)
  double ds, hds;          // slice length and half of it
  double k1, k1ds;         // gradient, DKD kick k1·ds
  double kabs_hds2;        // |k1| (ds/2)²: (κ ds/2)² times P
};
struct Quad4Params {       // fourth-order quadrupole slice (M_DKD4, M_MK4)
  QuadParams q;            // the whole slice (Ω weights, k1)
  QuadParams s1, s0;       // the composed steps of lengths x1 ds and x0 ds
};
struct TeapotParams {       // drift-kick sector bend (§3.6)
  double ds;                // orbit slice length (kick length)
  double h, eta_h;          // curvature and dipole field ηh
  double half, half_ib0;    // drift half ds/2 and (ds/2)/β0
  double c, sn, tn, sec;    // cos, sin, tan, 1/cos of h ds/2
  double tn_h, omc_h;       // tan(h ds/2)/h and (1/cos(h ds/2) - 1)/h
  double d0;                // ds/2 - tan(h ds/2)/h
};
struct SolenoidParams {     // solenoid (§3.7, §4.4)
  double ds;                // orbit slice length
  double ks;                // b0/(Bρ)0
  double eta, inv_eta;      // ks/2 and its inverse
  double eta_q;             // ks/4: half the vector potential at a fringe
};
struct RbendFace {          // frame rotation by φ at a rectangular-bend face
  double c, tn, sec;        // cos φ, tan φ, 1/cos φ
  double qw, qy;            // the spin's frame rotation (cos φ/2, sin φ/2 ŷ)
};
struct RbendParams {        // rectangular bend (§3.2, §4.5)
  double ds;                // orbit slice length along the magnet
  double L;                 // straight length (one-step orbit)
  double fb, rhob;          // b1/(Bρ)0 and its inverse
  double xoff;              // the design orbit's exit X in the magnet (eq. Xoffset)
  double larc_ib0;          // design arc length / β0 (eq. Toffset)
  RbendFace in, out;        // rotations by φ^entr and by -φ^exit
};
struct DriftParams { double L; };
struct ThinParams { double k1l, k2l; };             // thin multipole (§3.5)
struct SnakeParams { double qw, qx, qy, qz; };      // fixed rotation quaternion

constexpr int kElemWords = sizeof(BendParams) / sizeof(double);   // largest member
static_assert(sizeof(TeapotParams) <= sizeof(BendParams), "element union size");
static_assert(sizeof(SolenoidParams) <= sizeof(BendParams), "element union size");
static_assert(sizeof(RbendParams) <= sizeof(BendParams), "element union size");
static_assert(sizeof(Quad4Params) <= sizeof(BendParams), "element union size");

// element flags: single-precision spin arithmetic; thin-fringe spin kicks at
// both faces (sector bends and quadrupoles, extended kernels only)
enum : int32_t { F_SPIN32 = 1, F_FRINGE = 2 };

struct DevElem {
  int32_t kind, orbit, nsl, K;   // K = R_e - 1: Romberg levels minus one
  int32_t flags, place;          // place: P_EDGES, P_KICK or P_MIDPOINT (nsl = 2N orbit
                                 // half slices for P_MIDPOINT)
  // Romberg edge rotations of sliced elements: half the step w ds of an end
  // edge (w = 1/2) and of an interior edge (w = 1), and their squares
  double hw_end, hw_in, hw2_end, hw2_in;
  union {
    BendParams b;
    TeapotParams tp;
    SolenoidParams sol;
    RbendParams rb;
    QuadParams q;
    Quad4Params q4;
    DriftParams d;
    ThinParams t;
    SnakeParams s;
    double v[kElemWords];
  };
};

struct TrackArgs {
  double* z;          // 6 × n SoA
  double* spin;       // 3 × n SoA
  int32_t* alive;     // n
  double* qout;       // 4 × n SoA or null
  int64_t n;
  const DevElem* tab;
  const uint32_t* seq;
  int32_t n_elems;
  int32_t turns;
  int32_t report_every;
  int32_t n_blocks;
  double* partials;   // [n_reports][n_blocks][4]
  double beta0, inv_beta0, gamma0, inv_gamma0_sq, G, aperture;
  double ymax;        // largest (θ/2)² the quaternion polynomial covers
  // surrogate tracking: lanes with fallback[j] == 0 skip the spin arithmetic
  const int32_t* fallback;
  // optional lane order: lane g works on particle perm[g] (a permutation of
  // 0..n-1), so that particles taking the same path share waves
  const int32_t* perm;
  // surrogate tracking over several turns (null otherwise): the particles on
  // the network are lanes g < feat_n (the lane order puts them first); such a
  // lane writes its network inputs at the start of every turn,
  // feat[(turn * feat_n + g) * feat_n_in + i] = (z_i - center_i) *
  // inv_scale_i (i < 6) and extra (i = 6), and the number of turns it
  // completes alive, turns_done[g]; these lanes run on an orbit-only kernel,
  // the lanes from feat_n on (the particles that fall back) on the full one
  float* feat;
  int32_t* turns_done;
  int64_t feat_n;
  int32_t feat_n_in;
  double feat_center[6], feat_inv_scale[6], feat_extra;
};

}  // namespace st

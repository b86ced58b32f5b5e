// C ABI of the tracking library: context, validation, lattice compression
// and kernel launches.  See include/spintrack.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "lattice_table.h"
#include "spintrack.h"
#include "track_kernels.h"

// The network's device and input width, for argument checks.
int st_mlp_device_of(const st_mlp* m);
int st_mlp_inputs_of(const st_mlp* m);

struct st_ctx {
  int device = 0;
  std::string err;
  double* scratch = nullptr;   // this device's copy of the file-scope scratch array
  // lattice
  bool have_lattice = false;
  st_beam beam{};
  double beta0 = 0.0;
  int n_elems = 0;
  int n_unique = 0;
  int nt = 16;             // quaternion series terms
  bool ext = false;        // lattice needs the extended kernel (TEAPOT, PWC placements,
                           // solenoids, rectangular bends, fringe spin kicks)
  double ymax = 0.0;
  st::DevElem* d_tab = nullptr;
  uint32_t* d_seq = nullptr;
  // particles
  int64_t n = 0;
  double* z = nullptr;
  double* spin = nullptr;
  int32_t* alive = nullptr;
  double* qout = nullptr;
  bool have_particles = false;
  // polarization
  double* d_partials = nullptr;
  size_t partials_cap = 0;     // doubles
  double* d_pol = nullptr;
  size_t pol_cap = 0;          // doubles
  int64_t n_reports = 0;
  // surrogate tracking scratch
  float* d_feat = nullptr;     // [turns of a batch][n][8] network inputs
  float* d_qnn = nullptr;      // [turns of a batch][n][4] network quaternions
  int32_t* d_done = nullptr;   // turns completed in a multi-turn launch
  int64_t feat_cap = 0;        // samples (turn, particle) d_feat and d_qnn hold
  double* d_q64 = nullptr;     // 4 × n
  double* d_ck = nullptr;      // checkpoint of the last audit: z (6 × n) then spin (3 × n)
  int32_t* d_ck_alive = nullptr;
  int32_t* d_ralive = nullptr; // live set of a replay
  int32_t* d_failed = nullptr; // particles that failed the last audit
  int32_t* d_perm = nullptr;   // lane order of the surrogate turns
  int32_t* d_rperm = nullptr;  // lane order of a replay
  int32_t* d_pcount = nullptr; // partition counts and offsets, 3 per 256 particles
  int32_t* d_poff = nullptr;
  int64_t surr_cap = 0;
};

// Polarization partials of st_track_noalloc: a fixed array in device memory,
// one copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in for
// the device symbol); it uses the device address that hipGetSymbolAddress
// returns, taken once per device by st_create.
constexpr size_t kScratchDoubles = ST_NOALLOC_SCRATCH_BYTES / sizeof(double);

// Device memory for the network inputs and quaternions of the turns that one
// surrogate launch covers (48 bytes per particle and turn).
constexpr size_t kSurrogateBatchBytes = (size_t)512 << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (resolved once).
hipError_t scratch_address(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

namespace {

struct DeviceGuard {
  int old = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    if (old != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
  }
};

st_status fail(st_ctx* c, st_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

st_status hip_fail(st_ctx* c, hipError_t e, const char* what) {
  return fail(c, ST_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool finite_all(const st_element& e) {
  const double v[] = {e.L,         e.angle,    e.eta, e.k1, e.k1l, e.k2l,
                      e.snake_phi, e.snake_mu, e.ks,  e.asym};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

int v2(int n) {
  int k = 0;
  while ((n & 1) == 0) { n >>= 1; ++k; }
  return k;
}

// Largest (θ/2)² for which NT terms of the cos series stay below 2^-56.
double series_ymax(int nt) {
  return std::exp((-56.0 * std::log(2.0) + std::lgamma(2.0 * nt + 1.0)) / nt);
}

std::string validate(const st_element& e, int64_t i) {
  const std::string at = "element " + std::to_string(i) + ": ";
  if (!finite_all(e)) return at + "non-finite parameter";
  if (e.kind < ST_MARKER || e.kind > ST_RBEND) return at + "unknown kind " + std::to_string(e.kind);
  if (e.orbit < ST_ORB_EXACT || e.orbit > ST_ORB_MK4) return at + "unknown orbit method";
  if ((e.orbit == ST_ORB_DKD4 || e.orbit == ST_ORB_MK4) && e.kind != ST_QUAD)
    return at + "fourth-order slices apply to quadrupoles";
  if (e.spin_place < ST_SPIN_EDGES || e.spin_place > ST_SPIN_MIDPOINT)
    return at + "unknown spin placement";
  if (e.fringe != 0 && e.fringe != 1) return at + "fringe must be 0 or 1";
  if (e.fringe != 0 && e.kind != ST_SBEND && e.kind != ST_QUAD)
    return at + "fringe spin kicks apply to sector bends and quadrupoles";
  if (e.L < 0.0) return at + "negative length";
  const bool sliced = e.kind == ST_SBEND || e.kind == ST_QUAD || e.kind == ST_SOLENOID ||
                      e.kind == ST_RBEND;
  if (sliced && e.n_slices < 1) return at + "n_slices must be >= 1";
  switch (e.kind) {
    case ST_DRIFT:
      if (e.orbit != ST_ORB_EXACT) return at + "drifts use the exact method";
      break;
    case ST_SBEND:
      if (e.orbit != ST_ORB_EXACT && e.orbit != ST_ORB_TEAPOT)
        return at + "sector bends use the exact or the TEAPOT method";
      if (!(e.L > 0.0)) return at + "sector bend needs L > 0";
      if (e.angle == 0.0) return at + "sector bend needs a non-zero angle";
      if (e.orbit == ST_ORB_EXACT && !(e.eta > 0.0)) return at + "exact sector bend needs eta > 0";
      if (std::fabs(0.5 * e.angle / e.n_slices) >= 1.0)
        return at + "slice angle too large for the TEAPOT drift";
      break;
    case ST_QUAD:
      if (e.orbit != ST_ORB_DKD && e.orbit != ST_ORB_MK && e.orbit != ST_ORB_DKD4 &&
          e.orbit != ST_ORB_MK4)
        return at + "quadrupoles use DKD, MK, DKD4 or MK4";
      if (!(e.L > 0.0)) return at + "quadrupole needs L > 0";
      break;
    case ST_RBEND:
      if (e.orbit != ST_ORB_EXACT) return at + "rectangular bends use the exact body map";
      if (!(e.L > 0.0)) return at + "rectangular bend needs L > 0";
      if (e.angle == 0.0) return at + "rectangular bend needs angle != 0";
      if (!(std::fabs(0.5 * e.angle + e.asym) < 1.5) || !(std::fabs(e.asym - 0.5 * e.angle) < 1.5))
        return at + "rectangular bend needs |phi_entr| and |phi_exit| < 1.5";
      if (e.eta == 0.0) return at + "rectangular bend needs eta != 0";
      if (e.spin_place == ST_SPIN_KICK) return at + "the kick spin placement needs drift-kick slices";
      break;
    case ST_SOLENOID:
      if (e.orbit != ST_ORB_EXACT) return at + "solenoids use the exact body map";
      if (!(e.L > 0.0)) return at + "solenoid needs L > 0";
      if (e.ks == 0.0) return at + "solenoid needs ks != 0";
      if (e.spin_place == ST_SPIN_KICK) return at + "the kick spin placement needs drift-kick slices";
      break;
    default:
      break;
  }
  if (e.kind != ST_SOLENOID && e.ks != 0.0) return at + "ks applies to solenoids only";
  if (e.kind != ST_RBEND && e.asym != 0.0) return at + "asym applies to rectangular bends only";
  if (sliced) {
    if (e.romberg_rows < 1 || e.romberg_rows > st::kMaxRows)
      return at + "romberg_rows must be in 1.." + std::to_string(st::kMaxRows);
    if (e.spin_place != ST_SPIN_EDGES && e.romberg_rows != 1)
      return at + "piece-wise constant spin placements take romberg_rows = 1";
    if (e.spin_place == ST_SPIN_KICK && e.orbit != ST_ORB_DKD && e.orbit != ST_ORB_TEAPOT)
      return at + "the kick spin placement needs drift-kick slices";
    if (e.spin_place == ST_SPIN_MIDPOINT && e.n_slices > (1 << 29))
      return at + "too many slices";
  } else if (e.spin_place != ST_SPIN_EDGES || e.orbit == ST_ORB_TEAPOT) {
    return at + "spin placements and TEAPOT slices apply to thick elements only";
  }
  return std::string();
}

// Finest-slice rotation angle of an element for a particle at amplitude r_ref
// (the element's spin-step size: used to choose the series length and, in the
// mixed mode, the precision of the spin arithmetic).
double design_angle(const st_element& e, const st_beam& b, double r_ref);

// Single precision keeps the spin error per element near ε32·Σ|q ⊗ Q - Q|,
// which grows with the slice rotation; above this angle the element stays in
// double precision in ST_MIXED.
constexpr double kSpin32MaxAngle = 0.02;

st::DevElem derive(const st_element& e, const st_beam& beam, double beta0) {
  st::DevElem d;
  std::memset(&d, 0, sizeof(d));
  d.kind = e.kind;
  d.orbit = e.orbit;
  d.place = e.spin_place;
  d.nsl = 1;
  d.K = 0;
  // Only the sliced elements: a thin element costs one rotation, and its
  // quaternion would need a double-precision renormalisation anyway.
  const bool thick = e.kind == ST_SBEND || e.kind == ST_QUAD;   // (solenoids: double only)
  if (thick && (beam.precision == ST_MIXED_ALL ||
                (beam.precision == ST_MIXED && design_angle(e, beam, 0.005) <= kSpin32MaxAngle)))
    d.flags |= st::F_SPIN32;
  if (e.fringe) d.flags |= st::F_FRINGE;
  // orbit slices: the midpoint placement runs 2N half slices
  const int n_orb = e.spin_place == ST_SPIN_MIDPOINT ? 2 * e.n_slices : e.n_slices;
  if (e.kind == ST_SBEND || e.kind == ST_QUAD || e.kind == ST_SOLENOID || e.kind == ST_RBEND) {
    d.nsl = n_orb;
    const int re = std::min(e.romberg_rows, 1 + v2(e.n_slices));
    d.K = re - 1;
    const double ds = e.L / n_orb;
    d.hw_end = 0.25 * ds;
    d.hw_in = 0.5 * ds;
    d.hw2_end = d.hw_end * d.hw_end;
    d.hw2_in = d.hw_in * d.hw_in;
  }
  if (e.kind == ST_SBEND && e.orbit == ST_ORB_TEAPOT) {
    st::TeapotParams& t = d.tp;
    t.ds = e.L / n_orb;
    t.h = e.angle / e.L;
    t.eta_h = e.eta * t.h;
    t.half = 0.5 * t.ds;
    t.half_ib0 = t.half / beta0;
    const double a = t.h * t.half;
    t.c = std::cos(a);
    t.sn = std::sin(a);
    t.tn = t.sn / t.c;
    t.sec = 1.0 / t.c;
    // the small differences in extended precision: tan(a) - a and 1 - cos(a)
    const long double al = (long double)t.h * (long double)t.half;
    const long double tl = std::tan(al);
    t.tn_h = (double)(tl / (long double)t.h);
    t.d0 = (double)(-(tl - al) / (long double)t.h);
    const long double s2 = std::sin(0.5L * al);
    t.omc_h = (double)(2.0L * s2 * s2 / (std::cos(al) * (long double)t.h));   // (sec - 1)/h
  } else if (e.kind == ST_SBEND) {
    st::BendParams& b = d.b;
    b.ds = e.L / n_orb;
    b.h = e.angle / e.L;
    b.eta = e.eta;
    b.eta_h = e.eta * b.h;
    b.inv_eta_h = 1.0 / (e.eta * b.h);
    b.one_m_eta2 = (1.0 - e.eta) * (1.0 + e.eta);
    auto step = [&](double s) {
      st::BendStep k;
      k.cs = std::cos(b.h * s);
      k.sn = std::sin(b.h * s);
      const double s2 = std::sin(0.5 * b.h * s);
      k.omc = 2.0 * s2 * s2;
      k.s_eta = s / e.eta;
      k.tconst = (1.0 - 1.0 / e.eta) * s / beta0;
      return k;
    };
    b.slice = step(b.ds);
    b.whole = step(e.L);
  } else if (e.kind == ST_QUAD) {
    auto fill = [&](st::QuadParams& q, double ds) {
      q.ds = ds;
      q.hds = 0.5 * ds;
      q.k1 = e.k1;
      q.k1ds = e.k1 * ds;
      q.kabs_hds2 = std::fabs(e.k1) * q.hds * q.hds;
    };
    fill(d.q, e.L / n_orb);
    if (e.orbit == ST_ORB_DKD4 || e.orbit == ST_ORB_MK4) {
      // triple jump: 2 x1 + x0 = 1, 2 x1^3 + x0^3 = 0
      const long double c2 = std::cbrt(2.0L);
      const long double x1 = 1.0L / (2.0L - c2), x0 = -c2 / (2.0L - c2);
      const long double ds = (long double)e.L / n_orb;
      fill(d.q4.s1, (double)(x1 * ds));
      fill(d.q4.s0, (double)(x0 * ds));
    }
  } else if (e.kind == ST_RBEND) {
    // faces at φ^entr = θ/2 + asym and φ^exit = asym - θ/2; with
    // sin φ^entr - sin φ^exit = 2 cos(asym) sin(θ/2) and cos φ^entr -
    // cos φ^exit = -2 sin(asym) sin(θ/2), eq. Xoffset is L tan(asym), free
    // of the cancellation in the difference of cosines
    st::RbendParams& rb = d.rb;
    const double half = 0.5 * e.angle;
    const double sdiff = 2.0 * std::cos(e.asym) * std::sin(half);   // sin φ^entr - sin φ^exit
    rb.ds = e.L / n_orb;
    rb.L = e.L;
    rb.fb = e.eta * sdiff / e.L;
    rb.rhob = 1.0 / rb.fb;
    rb.xoff = e.L * std::tan(e.asym);
    rb.larc_ib0 = e.angle * e.L / sdiff / beta0;
    auto face = [](st::RbendFace& f, double phi) {
      f.c = std::cos(phi);
      f.tn = std::sin(phi) / f.c;
      f.sec = 1.0 / f.c;
      f.qw = std::cos(0.5 * phi);
      f.qy = std::sin(0.5 * phi);
    };
    face(rb.in, half + e.asym);
    face(rb.out, half - e.asym);                                      // -φ^exit
  } else if (e.kind == ST_SOLENOID) {
    st::SolenoidParams& sp = d.sol;
    sp.ds = e.L / n_orb;
    sp.ks = e.ks;
    sp.eta = 0.5 * e.ks;
    sp.inv_eta = 2.0 / e.ks;
    sp.eta_q = 0.25 * e.ks;
  } else if (e.kind == ST_DRIFT) {
    d.d.L = e.L;
  } else if (e.kind == ST_THIN) {
    d.t.k1l = e.k1l;
    d.t.k2l = e.k2l;
  } else if (e.kind == ST_SNAKE) {
    const double hp = 0.5 * e.snake_phi;
    d.s.qw = std::cos(hp);
    d.s.qx = std::sin(hp) * std::sin(e.snake_mu);
    d.s.qy = 0.0;
    d.s.qz = std::sin(hp) * std::cos(e.snake_mu);
  }
  return d;
}

// Largest rotation angle a particle at amplitude r_ref meets in one series
// evaluation of this element: the finest Romberg level, w ds |Ω| with w = 1
// at interior edges (coarser levels are obtained by squaring).
double design_angle(const st_element& e, const st_beam& b, double r_ref) {
  const double a1 = 1.0 + b.G * b.gamma0;
  if (e.kind == ST_SBEND || e.kind == ST_QUAD) {
    const double ds = e.L / e.n_slices;
    const double f = (e.n_slices > 1 || e.spin_place != ST_SPIN_EDGES) ? ds : 0.5 * ds;
    double om;
    if (e.kind == ST_SBEND) {
      const double h = e.angle / e.L;
      om = std::fabs(a1 * e.eta * h - h);
    } else {
      om = a1 * std::fabs(e.k1) * r_ref;
    }
    return f * om;
  }
  if (e.kind == ST_THIN) return a1 * (std::fabs(e.k1l) * r_ref + 0.5 * std::fabs(e.k2l) * r_ref * r_ref);
  if (e.kind == ST_RBEND) {
    const double ds = e.L / e.n_slices;
    const double f = (e.n_slices > 1 || e.spin_place != ST_SPIN_EDGES) ? ds : 0.5 * ds;
    return a1 * std::fabs(e.eta * 2.0 * std::cos(e.asym) * std::sin(0.5 * e.angle) / e.L) * f;
  }
  if (e.kind == ST_SOLENOID) {
    const double ds = e.L / e.n_slices;
    const double f = (e.n_slices > 1 || e.spin_place != ST_SPIN_EDGES) ? ds : 0.5 * ds;
    return a1 * std::fabs(e.ks) * f;
  }
  return 0.0;
}

st::TrackArgs track_args(const st_ctx* c) {
  st::TrackArgs a{};
  a.z = c->z;
  a.spin = c->spin;
  a.alive = c->alive;
  a.n = c->n;
  a.tab = c->d_tab;
  a.seq = c->d_seq;
  a.n_elems = c->n_elems;
  a.n_blocks = (int32_t)((c->n + st::track_block_size() - 1) / st::track_block_size());
  a.beta0 = c->beta0;
  a.inv_beta0 = 1.0 / c->beta0;
  a.gamma0 = c->beam.gamma0;
  a.inv_gamma0_sq = 1.0 / (c->beam.gamma0 * c->beam.gamma0);
  a.G = c->beam.G;
  a.aperture = c->beam.aperture;
  a.ymax = c->ymax;
  return a;
}

// Grow the polarization buffers for n_rep reports of nb blocks each.
st_status ensure_polarization(st_ctx* c, int64_t n_rep, int64_t nb) {
  hipError_t e;
  if (n_rep <= 0) return ST_OK;
  const size_t need = (size_t)n_rep * (size_t)nb * 4;
  if (need > c->partials_cap) {
    if (c->d_partials) { (void)hipFree(c->d_partials); c->d_partials = nullptr; c->partials_cap = 0; }
    if ((e = hipMalloc(&c->d_partials, need * sizeof(double))) != hipSuccess)
      return fail(c, ST_ENOMEM, std::string("polarization partials: ") + hipGetErrorString(e));
    c->partials_cap = need;
  }
  if ((size_t)n_rep * 4 > c->pol_cap) {
    if (c->d_pol) { (void)hipFree(c->d_pol); c->d_pol = nullptr; c->pol_cap = 0; }
    if ((e = hipMalloc(&c->d_pol, (size_t)n_rep * 4 * sizeof(double))) != hipSuccess)
      return fail(c, ST_ENOMEM, std::string("polarization history: ") + hipGetErrorString(e));
    c->pol_cap = (size_t)n_rep * 4;
  }
  return ST_OK;
}

// Queue one tracking launch and, with reports, the second pass of the
// polarization reduction: partials holds reports x blocks x 4 doubles (every
// slot is written by the tracking kernel before the reduction reads it), pol
// receives 4 doubles per report.
st_status launch_tracking(st_ctx* c, int64_t turns, double* partials, double* pol,
                          hipStream_t s) {
  const int64_t nb = (c->n + st::track_block_size() - 1) / st::track_block_size();
  const int rep_every = c->beam.report_every;
  const int64_t n_rep = rep_every > 0 ? turns / rep_every : 0;
  st::TrackArgs a = track_args(c);
  a.qout = c->qout;
  a.turns = (int32_t)turns;
  a.report_every = rep_every;
  a.partials = partials;
  hipError_t e;
  if ((e = st::launch_track(a, c->nt, c->beam.precision != ST_FP64, c->ext, s)) != hipSuccess)
    return hip_fail(c, e, "launch track");
  if (n_rep > 0 &&
      (e = st::launch_reduce_polarization(partials, (int)nb, (int)n_rep, pol, s)) != hipSuccess)
    return hip_fail(c, e, "launch polarization reduction");
  return ST_OK;
}

}  // namespace

extern "C" {

st_status st_create(st_ctx** out, int device) {
  if (!out) return ST_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return ST_EINVAL;
  if (device >= kMaxDevices) return ST_EINVAL;
  st_ctx* c = new (std::nothrow) st_ctx();
  if (!c) return ST_ENOMEM;
  c->device = device;
  {
    DeviceGuard g(device);
    if (scratch_address(device, &c->scratch) != hipSuccess) {
      delete c;
      return ST_EDEVICE;
    }
  }
  *out = c;
  return ST_OK;
}

st_status st_destroy(st_ctx* c) {
  if (!c) return ST_OK;
  {
    DeviceGuard g(c->device);
    if (c->d_tab) (void)hipFree(c->d_tab);
    if (c->d_seq) (void)hipFree(c->d_seq);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_pol) (void)hipFree(c->d_pol);
    for (void* p : {(void*)c->d_feat, (void*)c->d_qnn, (void*)c->d_q64, (void*)c->d_ck,
                    (void*)c->d_ck_alive, (void*)c->d_ralive, (void*)c->d_failed, (void*)c->d_perm,
                    (void*)c->d_rperm, (void*)c->d_pcount, (void*)c->d_poff, (void*)c->d_done})
      if (p) (void)hipFree(p);
  }
  delete c;
  return ST_OK;
}

const char* st_last_error(const st_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

st_status st_load_lattice(st_ctx* c, const st_element* els, int64_t n, const st_beam* b) {
  if (!c) return ST_EINVAL;
  if (!b) return fail(c, ST_EINVAL, "beam is NULL");
  if (n < 0 || n > std::numeric_limits<int32_t>::max()) return fail(c, ST_EINVAL, "bad element count");
  if (n > 0 && !els) return fail(c, ST_EINVAL, "elements are NULL");
  if (!std::isfinite(b->G) || !std::isfinite(b->gamma0) || !(b->gamma0 > 1.0))
    return fail(c, ST_EINVAL, "gamma0 must be finite and > 1, G finite");
  if (!(b->aperture > 0.0)) return fail(c, ST_EINVAL, "aperture must be > 0");
  if (b->precision != ST_FP64 && b->precision != ST_MIXED && b->precision != ST_MIXED_ALL)
    return fail(c, ST_EINVAL, "unknown precision");
  if (b->report_every < 0) return fail(c, ST_EINVAL, "report_every must be >= 0");
  for (int64_t i = 0; i < n; ++i) {
    std::string m = validate(els[i], i);
    if (!m.empty()) return fail(c, ST_EINVAL, m);
  }
  const double beta0 = std::sqrt(1.0 - 1.0 / (b->gamma0 * b->gamma0));

  // compress: unique elements (equal bytes: st_element has no padding) and
  // the index sequence
  static_assert(sizeof(st_element) == 6 * sizeof(int32_t) + 10 * sizeof(double),
                "st_element must have no padding bytes");
  std::vector<st_element> uniq;
  std::unordered_map<std::string, uint32_t> index;
  std::vector<uint32_t> seq((size_t)n);
  double theta = 0.0;
  bool ext = false;
  for (int64_t i = 0; i < n; ++i) {
    ext = ext || els[i].orbit == ST_ORB_TEAPOT || els[i].orbit == ST_ORB_DKD4 ||
          els[i].orbit == ST_ORB_MK4 || els[i].spin_place != ST_SPIN_EDGES ||
          els[i].kind == ST_SOLENOID || els[i].kind == ST_RBEND || els[i].fringe != 0;
    const std::string key(reinterpret_cast<const char*>(&els[i]), sizeof(st_element));
    auto it = index.find(key);
    uint32_t k;
    if (it != index.end()) {
      k = it->second;
    } else {
      if (uniq.size() >= 65535) return fail(c, ST_EINVAL, "more than 65535 distinct elements");
      k = (uint32_t)uniq.size();
      uniq.push_back(els[i]);
      index.emplace(key, k);
    }
    seq[(size_t)i] = k;
    theta = std::max(theta, design_angle(els[i], *b, 0.02));
  }
  std::vector<st::DevElem> tab(std::max<size_t>(uniq.size(), 1));
  for (size_t u = 0; u < uniq.size(); ++u) tab[u] = derive(uniq[u], *b, beta0);

  DeviceGuard g(c->device);
  if (c->d_tab) { (void)hipFree(c->d_tab); c->d_tab = nullptr; }
  if (c->d_seq) { (void)hipFree(c->d_seq); c->d_seq = nullptr; }
  c->have_lattice = false;
  hipError_t e;
  if ((e = hipMalloc(&c->d_tab, tab.size() * sizeof(st::DevElem))) != hipSuccess)
    return fail(c, ST_ENOMEM, std::string("lattice table: ") + hipGetErrorString(e));
  if ((e = hipMalloc(&c->d_seq, std::max<size_t>(seq.size(), 1) * sizeof(uint32_t))) != hipSuccess)
    return fail(c, ST_ENOMEM, std::string("lattice sequence: ") + hipGetErrorString(e));
  if ((e = hipMemcpy(c->d_tab, tab.data(), tab.size() * sizeof(st::DevElem), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(c, e, "upload lattice table");
  if (n > 0 && (e = hipMemcpy(c->d_seq, seq.data(), seq.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(c, e, "upload lattice sequence");

  // series terms: cover the design angles with 10% margin; lanes beyond use sincos
  const double y = 1.21 * 0.25 * theta * theta;
  c->nt = 16;
  for (int nt : {5, 6, 8, 12, 16})
    if (series_ymax(nt) >= y) { c->nt = nt; break; }
  c->ymax = series_ymax(c->nt);
  c->beam = *b;
  c->beta0 = beta0;
  c->ext = ext;
  c->n_elems = (int)n;
  c->n_unique = (int)uniq.size();
  c->have_lattice = true;
  c->err.clear();
  return ST_OK;
}

st_status st_bind_particles(st_ctx* c, int64_t n, double* z, double* spin, int32_t* alive) {
  if (!c) return ST_EINVAL;
  if (n < 0) return fail(c, ST_EINVAL, "negative particle count");
  if (n > (int64_t)std::numeric_limits<int32_t>::max() * 256)
    return fail(c, ST_EINVAL, "too many particles");
  if (n > 0 && (!z || !spin || !alive)) return fail(c, ST_EINVAL, "particle pointers are NULL");
  c->n = n;
  c->z = z;
  c->spin = spin;
  c->alive = alive;
  c->qout = nullptr;
  c->have_particles = true;
  c->err.clear();
  return ST_OK;
}

st_status st_bind_quaternions(st_ctx* c, double* q) {
  if (!c) return ST_EINVAL;
  if (!c->have_particles) return fail(c, ST_ESTATE, "bind particles first");
  c->qout = q;
  return ST_OK;
}

st_status st_track(st_ctx* c, int64_t turns, void* stream) {
  if (!c) return ST_EINVAL;
  if (!c->have_lattice) return fail(c, ST_ESTATE, "no lattice loaded");
  if (!c->have_particles) return fail(c, ST_ESTATE, "no particles bound");
  if (turns < 0 || turns > std::numeric_limits<int32_t>::max())
    return fail(c, ST_EINVAL, "turns must be in 0..2^31-1");
  c->n_reports = 0;
  if (turns == 0 || c->n == 0) return ST_OK;
  DeviceGuard g(c->device);
  const int64_t nb = (c->n + st::track_block_size() - 1) / st::track_block_size();
  const int rep_every = c->beam.report_every;
  const int64_t n_rep = rep_every > 0 ? turns / rep_every : 0;
  st_status pst = ensure_polarization(c, n_rep, nb);
  if (pst != ST_OK) return pst;
  pst = launch_tracking(c, turns, c->d_partials, c->d_pol, (hipStream_t)stream);
  if (pst != ST_OK) return pst;
  c->n_reports = n_rep;
  c->err.clear();
  return ST_OK;
}

st_status st_track_noalloc(st_ctx* c, int64_t turns, double* d_pol, int64_t capacity,
                           int64_t* n_reports, void* stream) {
  if (!c) return ST_EINVAL;
  if (n_reports) *n_reports = 0;
  if (!c->have_lattice) return fail(c, ST_ESTATE, "no lattice loaded");
  if (!c->have_particles) return fail(c, ST_ESTATE, "no particles bound");
  if (turns < 0 || turns > std::numeric_limits<int32_t>::max())
    return fail(c, ST_EINVAL, "turns must be in 0..2^31-1");
  const int64_t nb = (c->n + st::track_block_size() - 1) / st::track_block_size();
  const int rep_every = c->beam.report_every;
  const int64_t n_rep = (rep_every > 0 && c->n > 0) ? turns / rep_every : 0;
  if (n_rep > 0 && (uint64_t)n_rep * (uint64_t)nb * 4 > kScratchDoubles)
    return fail(c, ST_EINVAL,
                "polarization scratch of " + std::to_string(n_rep) + " reports x " +
                    std::to_string(nb) + " blocks x 4 doubles exceeds the " +
                    std::to_string(kScratchDoubles) +
                    " doubles of the fixed scratch array (fewer reports per call, or st_track)");
  if (n_rep > 0 && (!d_pol || capacity < n_rep))
    return fail(c, ST_EINVAL, "d_pol must hold the " + std::to_string(n_rep) +
                                  " reports of this call (4 doubles each)");
  c->n_reports = 0;             // st_polarization does not see this call's history
  if (turns == 0 || c->n == 0) return ST_OK;
  DeviceGuard g(c->device);
  const st_status pst = launch_tracking(c, turns, c->scratch, d_pol, (hipStream_t)stream);
  if (pst != ST_OK) return pst;
  if (n_reports) *n_reports = n_rep;
  c->err.clear();
  return ST_OK;
}

st_status st_polarization(st_ctx* c, double* d_out, int64_t capacity, int64_t* n_reports,
                          void* stream) {
  if (!c) return ST_EINVAL;
  if (capacity < 0) return fail(c, ST_EINVAL, "negative capacity");
  if (n_reports) *n_reports = c->n_reports;
  if (!d_out || capacity == 0 || c->n_reports == 0) return ST_OK;
  DeviceGuard g(c->device);
  const int64_t k = std::min(capacity, c->n_reports);
  hipError_t e = hipMemcpyAsync(d_out, c->d_pol, (size_t)k * 4 * sizeof(double),
                                hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "copy polarization");
  return ST_OK;
}

st_status st_read_particles(st_ctx* c, double* h_z, double* h_spin, int32_t* h_alive, void* stream) {
  if (!c) return ST_EINVAL;
  if (!c->have_particles) return fail(c, ST_ESTATE, "no particles bound");
  if (c->n == 0) return ST_OK;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (h_z && (e = hipMemcpyAsync(h_z, c->z, (size_t)c->n * 6 * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(c, e, "read z");
  if (h_spin && (e = hipMemcpyAsync(h_spin, c->spin, (size_t)c->n * 3 * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(c, e, "read spin");
  if (h_alive && (e = hipMemcpyAsync(h_alive, c->alive, (size_t)c->n * sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(c, e, "read alive");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "synchronise");
  return ST_OK;
}

}  // extern "C"

extern "C" st_status st_track_surrogate(st_ctx* c, st_mlp* m, int64_t turns, int32_t audit_every,
                                        double threshold, const double* center,
                                        const double* inv_scale, double extra,
                                        int32_t* d_fallback, void* stream) {
  if (!c) return ST_EINVAL;
  if (!m) return fail(c, ST_EINVAL, "network is NULL");
  if (!c->have_lattice) return fail(c, ST_ESTATE, "no lattice loaded");
  if (!c->have_particles) return fail(c, ST_ESTATE, "no particles bound");
  if (turns < 0 || turns > std::numeric_limits<int32_t>::max())
    return fail(c, ST_EINVAL, "turns must be in 0..2^31-1");
  if (audit_every < 1) return fail(c, ST_EINVAL, "audit_every must be >= 1");
  if (c->n > std::numeric_limits<int32_t>::max())
    return fail(c, ST_EINVAL, "surrogate tracking takes at most 2^31-1 particles");
  if (!(threshold >= 0.0) || !std::isfinite(threshold)) return fail(c, ST_EINVAL, "bad threshold");
  if (!center || !inv_scale) return fail(c, ST_EINVAL, "feature scaling is NULL");
  if (c->n > 0 && !d_fallback) return fail(c, ST_EINVAL, "fallback array is NULL");
  if (st_mlp_device_of(m) != c->device) return fail(c, ST_EINVAL, "network on another device");
  if (c->beam.report_every > 0 && c->beam.report_every % audit_every != 0)
    return fail(c, ST_EINVAL, "report_every must be a multiple of audit_every");
  c->n_reports = 0;
  if (c->n == 0) return ST_OK;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  const int64_t n = c->n;
  if (n > c->surr_cap) {
    for (void* p : {(void*)c->d_q64, (void*)c->d_ck, (void*)c->d_ck_alive, (void*)c->d_ralive,
                    (void*)c->d_failed, (void*)c->d_perm, (void*)c->d_rperm, (void*)c->d_pcount,
                    (void*)c->d_poff, (void*)c->d_done})
      if (p) (void)hipFree(p);
    c->d_q64 = nullptr; c->d_ck = nullptr; c->d_ck_alive = nullptr; c->d_ralive = nullptr;
    c->d_failed = nullptr; c->d_perm = nullptr; c->d_rperm = nullptr; c->d_pcount = nullptr;
    c->d_poff = nullptr; c->d_done = nullptr; c->surr_cap = 0;
    const size_t nparts = (size_t)((n + 255) / 256) * 3;
    if ((e = hipMalloc(&c->d_q64, (size_t)n * 4 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&c->d_ck, (size_t)n * 9 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&c->d_ck_alive, (size_t)n * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&c->d_ralive, (size_t)n * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&c->d_failed, (size_t)n * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&c->d_perm, (size_t)n * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&c->d_rperm, (size_t)n * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&c->d_pcount, nparts * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&c->d_poff, nparts * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&c->d_done, (size_t)n * sizeof(int32_t))) != hipSuccess)
      return fail(c, ST_ENOMEM, std::string("surrogate scratch: ") + hipGetErrorString(e));
    c->surr_cap = n;
  }
  // Turns between audits run as one launch of the orbit push; the network
  // inputs and quaternions of all of them are held at once, up to
  // kSurrogateBatchBytes (48 bytes per particle and turn).
  const int64_t k_max = std::max<int64_t>(
      1, std::min<int64_t>((int64_t)audit_every, (int64_t)(kSurrogateBatchBytes / (48 * (size_t)n))));
  if (k_max * n > c->feat_cap) {
    if (c->d_feat) (void)hipFree(c->d_feat);
    if (c->d_qnn) (void)hipFree(c->d_qnn);
    c->d_feat = nullptr; c->d_qnn = nullptr; c->feat_cap = 0;
    if ((e = hipMalloc(&c->d_feat, (size_t)(k_max * n) * 8 * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&c->d_qnn, (size_t)(k_max * n) * 4 * sizeof(float))) != hipSuccess)
      return fail(c, ST_ENOMEM, std::string("surrogate batch buffers: ") + hipGetErrorString(e));
    c->feat_cap = k_max * n;
  }
  if (turns == 0) return ST_OK;      // the scratch is reserved for later calls
  const int bs = st::track_block_size();
  const int64_t nb = (n + bs - 1) / bs;
  const int rep_every = c->beam.report_every;
  const int64_t n_rep = rep_every > 0 ? turns / rep_every : 0;
  st_status pst = ensure_polarization(c, n_rep, nb);
  if (pst != ST_OK) return pst;
  // Checkpoint of the state at the start and after every audit: a particle
  // that fails an audit is rolled back to it and replayed in double precision.
  auto checkpoint = [&]() -> hipError_t {
    hipError_t r = hipMemcpyAsync(c->d_ck, c->z, (size_t)n * 6 * sizeof(double),
                                  hipMemcpyDeviceToDevice, s);
    if (r == hipSuccess)
      r = hipMemcpyAsync(c->d_ck + 6 * n, c->spin, (size_t)n * 3 * sizeof(double),
                         hipMemcpyDeviceToDevice, s);
    if (r == hipSuccess)
      r = hipMemcpyAsync(c->d_ck_alive, c->alive, (size_t)n * sizeof(int32_t),
                         hipMemcpyDeviceToDevice, s);
    return r;
  };
  if ((e = checkpoint()) != hipSuccess) return hip_fail(c, e, "checkpoint");
  // lane order: particles on the network first, then the fallback ones, so
  // that waves take one path or the other
  auto order = [&]() -> hipError_t {
    return st::launch_partition(0, nullptr, c->alive, d_fallback, n, c->d_pcount, c->d_poff,
                                c->d_perm, s);
  };
  if ((e = order()) != hipSuccess) return hip_fail(c, e, "lane order");
  // particles of the first key of a lane order (the exclusive offset of the
  // second key in the first block): those on the network, or in a replay's
  // order those that failed the audit
  int32_t n_first = 0;
  auto count_first = [&]() -> hipError_t {
    hipError_t r = hipMemcpyAsync(&n_first, c->d_poff + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (r == hipSuccess) r = hipStreamSynchronize(s);
    return r;
  };
  // audits: after the first turn, so that particles the network cannot
  // follow are found before a long replay, then every audit_every-th turn,
  // and after the last turn of the call, so that no network turn goes
  // unchecked
  auto is_audit = [&](int64_t t) { return t % audit_every == 0 || t == 1 || t == turns; };
  int64_t last_audit = 0;
  for (int64_t t = 1; t <= turns;) {
    if (!is_audit(t)) {
      // the network turns up to the next audit (at most k_max of them): one
      // launch pushes the orbits and writes every turn's network inputs, one
      // inference covers them all, and each particle is then rotated by its
      // turns' quaternions in order (the spin does not act on the orbit)
      int64_t k = 1;
      while (k < k_max && !is_audit(t + k)) ++k;
      if ((e = count_first()) != hipSuccess) return hip_fail(c, e, "network count");
      const int32_t n_net = n_first;
      st::TrackArgs a = track_args(c);
      a.turns = (int)k;
      a.report_every = 0;
      a.partials = nullptr;
      a.fallback = d_fallback;
      a.perm = c->d_perm;
      a.feat = n_net > 0 ? c->d_feat : nullptr;
      a.turns_done = n_net > 0 ? c->d_done : nullptr;
      a.feat_n = n_net;
      a.feat_n_in = st_mlp_inputs_of(m);
      for (int i = 0; i < 6; ++i) { a.feat_center[i] = center[i]; a.feat_inv_scale[i] = inv_scale[i]; }
      a.feat_extra = extra;
      if ((e = st::launch_track(a, c->nt, false, c->ext, s)) != hipSuccess)
        return hip_fail(c, e, "surrogate turns");
      if (n_net > 0) {
        const st_status ms = st_mlp_infer(m, c->d_feat, c->d_qnn, k * n_net, stream);
        if (ms != ST_OK) return fail(c, ms, std::string("network: ") + st_mlp_last_error(m));
        if ((e = st::launch_surrogate_spin_turns(c->spin, c->d_perm, c->d_done, c->d_qnn, n_net, n,
                                                 s)) != hipSuccess)
          return hip_fail(c, e, "surrogate spin");
      }
      t += k;
      continue;
    }
    st_status ms = st_mlp_features(m, c->z, n, center, inv_scale, extra, c->d_feat, stream);
    if (ms == ST_OK) ms = st_mlp_infer(m, c->d_feat, c->d_qnn, n, stream);
    if (ms != ST_OK) return fail(c, ms, std::string("network: ") + st_mlp_last_error(m));
    st::TrackArgs a = track_args(c);
    a.turns = 1;
    a.qout = c->d_q64;
    if ((e = st::launch_track(a, c->nt, false, c->ext, s)) != hipSuccess) return hip_fail(c, e, "audit turn");
    if ((e = st::launch_audit(c->alive, d_fallback, c->d_failed, c->d_qnn, c->d_q64, n, threshold,
                              (int32_t)t, s)) != hipSuccess)
      return hip_fail(c, e, "audit");
    // Roll the particles that failed back to the last checkpoint and replay
    // the turns since then in double precision; the orbit is the same as on
    // the surrogate path, so only their spins change.
    if ((e = st::launch_replay_prepare(c->d_failed, c->z, c->spin, c->d_ck, c->d_ck + 6 * n,
                                       c->d_ck_alive, c->d_ralive, n, s)) != hipSuccess)
      return hip_fail(c, e, "rollback");
    if ((e = st::launch_partition(1, c->d_failed, c->alive, d_fallback, n, c->d_pcount,
                                  c->d_poff, c->d_rperm, s)) != hipSuccess)
      return hip_fail(c, e, "replay order");
    // the replay launch covers only the blocks of the failed particles'
    // lanes (the lanes past them in the last block are not live in the replay)
    if ((e = count_first()) != hipSuccess) return hip_fail(c, e, "replay count");
    if (n_first > 0) {
      st::TrackArgs r = track_args(c);
      r.alive = c->d_ralive;
      r.perm = c->d_rperm;
      r.n_blocks = (int32_t)((n_first + st::track_block_size() - 1) / st::track_block_size());
      r.turns = (int)(t - last_audit);
      r.report_every = 0;
      r.partials = nullptr;
      if ((e = st::launch_track(r, c->nt, false, c->ext, s)) != hipSuccess) return hip_fail(c, e, "replay");
    }
    if ((e = st::launch_replay_finish(c->d_failed, c->d_ralive, c->alive, n, s)) != hipSuccess)
      return hip_fail(c, e, "replay status");
    if ((e = checkpoint()) != hipSuccess) return hip_fail(c, e, "checkpoint");
    if ((e = order()) != hipSuccess) return hip_fail(c, e, "lane order");
    last_audit = t;
    if (n_rep > 0 && t % rep_every == 0) {
      const int64_t rep = t / rep_every - 1;
      if ((e = st::launch_polarization_partials(c->spin, c->alive, n, c->d_partials + rep * nb * 4,
                                                s)) != hipSuccess)
        return hip_fail(c, e, "polarization");
    }
    ++t;
  }
  if (n_rep > 0 && (e = st::launch_reduce_polarization(c->d_partials, (int)nb, (int)n_rep, c->d_pol,
                                                       s)) != hipSuccess)
    return hip_fail(c, e, "polarization reduction");
  c->n_reports = n_rep;
  c->err.clear();
  return ST_OK;
}

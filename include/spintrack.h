/* spintrack.h — C ABI of the MI355X spin–orbit tracking library.
 *
 * The library pushes particles through a ring lattice with the method of
 * Abell, Meiser, Ranjbar & Barber, "Accurate and efficient spin integration
 * for particle accelerators" (2015): symplectic orbit maps per element (exact
 * drift and sector bend, drift-kick and matrix-kick quadrupoles, thin
 * multipoles) fused with Thomas-BMT spin integration, where Ω at each slice
 * edge becomes a rotation quaternion, Romberg extrapolation over slice
 * refinements accelerates convergence, and quaternions compose element by
 * element.
 *
 * Conventions shared by every entry point
 *   - Every call returns st_status.  Invalid arguments are rejected with
 *     ST_EINVAL before any device work; st_last_error() then describes why.
 *   - Particle arrays live in caller-owned DEVICE memory as structure of
 *     arrays: z is 6 rows of n doubles (X, Px, Y, Py, T, Pt), spin is 3 rows
 *     of n doubles (Sx, Sy, Sz), alive is n int32.  The library never frees
 *     them; a binding stays valid until the next st_bind_particles or
 *     st_destroy.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is queued
 *     asynchronously on it unless stated otherwise.
 *   - A context is not thread-safe; distinct contexts may be used from
 *     distinct threads and streams.
 *   - Lost particles are not errors: alive[j] = -(1 + e) records that
 *     particle j left the aperture, or met a negative square-root radicand
 *     or a non-finite value, in element e; its state is frozen at that
 *     element's entrance.  Particles with alive[j] != 1 on entry are skipped.
 *
 * Coordinates and units (§2.1 eq. psvars and eq. pt): X, Y in metres; Px, Py
 * momenta scaled by p0 = m γ0 β0 c; T = -c Δt in metres; Pt = (E - E0)/(p0 c).
 * Spin (§2.2): unit 3-vector in the local (x, y, s) frame, dS/ds = Ω × S with
 * Ω from eq. t-bmt.so.
 */
#ifndef SPINTRACK_H
#define SPINTRACK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct st_ctx st_ctx;

typedef enum {
  ST_OK = 0,
  ST_EINVAL = -1,   /* invalid argument; nothing was queued                    */
  ST_ENOMEM = -2,   /* a device allocation failed                              */
  ST_EDEVICE = -3,  /* a HIP runtime call failed                               */
  ST_ESTATE = -4    /* call out of order (e.g. st_track before a lattice)      */
} st_status;

typedef enum {
  ST_MARKER = 0,    /* does nothing                                            */
  ST_DRIFT = 1,     /* field-free length L (§3.4 eq. HmultD)                   */
  ST_SBEND = 2,     /* sector bend: L, angle, eta (§3.1 eq. sbend)             */
  ST_QUAD = 3,      /* normal quadrupole: L, k1 (§3.3 / §3.4)                  */
  ST_THIN = 4,      /* thin normal multipole: k1l, k2l (§3.5)                  */
  ST_SNAKE = 5      /* thin spin rotator: snake_phi about (sin mu, 0, cos mu)  */
} st_kind;

typedef enum {
  ST_ORB_EXACT = 0, /* exact flow: drifts and sector bends                     */
  ST_ORB_DKD = 1,   /* drift-kick-drift slices (quadrupoles)                   */
  ST_ORB_MK = 2     /* matrix-kick-matrix slices (§3.3 eq. quadConcat)         */
} st_orbit;

typedef enum {
  ST_FP64 = 0,      /* every step in double precision                          */
  ST_MIXED = 1      /* orbit and final Romberg step in double; per-slice
                       quaternions, level products and the Romberg tableau in
                       single precision with compensated sums                  */
} st_precision;

/* One lattice element.  SI units; strengths normalised to (Bρ)0.
 *   L            length [m] (0 for thin elements and snakes)
 *   angle        sector-bend geometric angle [rad]; curvature h = angle/L
 *   eta          sector-bend powering b1/(h (Bρ)0) (§3.1 eq. eta); 1 = design
 *   k1           quadrupole gradient b2/(Bρ)0 [m^-2]
 *   k1l, k2l     thin multipole integrated strengths [m^-1], [m^-2]: the kick
 *                is Px -= k1l X + k2l (X²-Y²)/2, Py += k1l Y + k2l X Y
 *   snake_phi    snake rotation angle [rad]; axis (sin mu, 0, cos mu) in (x, y, s)
 *   n_slices     orbit slices N of a thick element with spin (sbend, quad)
 *   romberg_rows requested tableau rows R ≥ 1 (§4.3 eq. romberg); the rows
 *                used are R_e = min(R, 1 + ν2(N)), ν2 the power of 2 in N
 */
typedef struct {
  int32_t kind, orbit, n_slices, romberg_rows;
  double L, angle, eta, k1, k1l, k2l, snake_phi, snake_mu;
} st_element;

/* Beam and run parameters.
 *   G            gyromagnetic anomaly (g-2)/2
 *   gamma0       Lorentz factor of the reference particle
 *   aperture     a particle with |X| or |Y| above this [m] after an element is lost
 *   precision    st_precision
 *   report_every polarization is recorded after every report_every-th turn of
 *                a st_track call (0 = never)
 */
typedef struct {
  double G, gamma0, aperture;
  int32_t precision, report_every;
} st_beam;

/* Create a context on HIP device `device`.  *out receives the handle. */
st_status st_create(st_ctx** out, int device);

/* Release the context and everything the library allocated for it.
 * Caller-owned particle memory is not touched.  NULL is accepted. */
st_status st_destroy(st_ctx* ctx);

/* Copy n elements (host memory) and the beam into the context.  Validation:
 * known kind and orbit method; finite parameters; L ≥ 0; sbends need L > 0,
 * angle ≠ 0 and eta > 0 with the exact method; quadrupoles need L > 0 and the
 * DKD or MK method; thick elements with spin need n_slices ≥ 1 and
 * romberg_rows in 1..4; gamma0 > 1; aperture > 0; report_every ≥ 0.
 * Synchronous; replaces any earlier lattice. */
st_status st_load_lattice(st_ctx* ctx, const st_element* host_elems, int64_t n,
                          const st_beam* beam);

/* Bind n particles held in caller-owned device memory (layout above).
 * n may be 0.  Pointers must be non-NULL when n > 0. */
st_status st_bind_particles(st_ctx* ctx, int64_t n, double* d_z, double* d_spin,
                            int32_t* d_alive);

/* Optionally bind a device array q (4 rows of n doubles: w, x, y, z) that
 * st_track fills with each particle's one-turn spin quaternion of the last
 * turn it tracked (the product of the element quaternions, later elements on
 * the left).  NULL unbinds.  Must follow st_bind_particles. */
st_status st_bind_quaternions(st_ctx* ctx, double* d_q);

/* Track the bound particles for `turns` turns (≥ 0), asynchronously on
 * `stream`.  Updates z, spin, alive (and q if bound) in place and records
 * the polarization history of this call.  Each call starts at the lattice
 * start, so track(a + b) equals track(a) followed by track(b). */
st_status st_track(st_ctx* ctx, int64_t turns, void* stream);

/* Polarization history of the last st_track: for each report k, four doubles
 * (Px, Py, Pz, N_alive) with P = Σ_alive S_j / N_alive (0 if none alive).
 * Writes min(capacity, n_reports) reports to caller-owned DEVICE memory
 * d_out, queued on `stream`; *n_reports (host) receives the number of
 * reports recorded.  d_out may be NULL to query the count. */
st_status st_polarization(st_ctx* ctx, double* d_out, int64_t capacity,
                          int64_t* n_reports, void* stream);

/* Copy the bound particles to HOST memory (any pointer may be NULL to skip
 * that array).  Synchronises `stream` before returning. */
st_status st_read_particles(st_ctx* ctx, double* h_z, double* h_spin, int32_t* h_alive,
                            void* stream);

/* Human-readable description of the last error on this context (owned by
 * the context; valid until the next call).  Never NULL. */
const char* st_last_error(const st_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SPINTRACK_H */

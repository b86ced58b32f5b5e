/* spintrack.h — C ABI of the MI355X spin–orbit tracking library.
 *
 * The library pushes particles through a ring lattice with the method of
 * Abell, Meiser, Ranjbar & Barber, "Accurate and efficient spin integration
 * for particle accelerators" (2015): symplectic orbit maps per element (exact
 * drift and sector bend, drift-kick and matrix-kick quadrupoles, thin
 * multipoles) fused with Thomas-BMT spin integration, where Ω at each slice
 * edge becomes a rotation quaternion, Romberg extrapolation over slice
 * refinements accelerates convergence, and quaternions compose element by
 * element.  The paper's comparison methods are there too: drift-kick (TEAPOT)
 * sector bends, piece-wise constant spin placements, solenoids, rectangular
 * bends, fringe spin kicks, and fourth-order quadrupole slices.
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
  ST_SNAKE = 5,     /* thin spin rotator: snake_phi about (sin mu, 0, cos mu)  */
  ST_SOLENOID = 6,  /* solenoid: L, ks = b0/(Bρ)0, exact body map (§3.7 eq.
                       solenoid) between thin-pancake fringes whose spin kicks
                       follow §4.4 eq. solFringe; spin_place EDGES or MIDPOINT */
  ST_RBEND = 7      /* rectangular bend: straight length L, design bend
                       `angle`, faces at φ^entr = angle/2 + asym and
                       φ^exit = asym - angle/2 to the design orbit, powering
                       eta != 0; frame rotations by φ^entr and -φ^exit (eq.
                       prot), thin dipole fringes (eq. dipolefringe), exact
                       body (§3.2 eq. rbend), the design orbit's horizontal
                       offset (eq. Xoffset) and flight time (eq. Toffset),
                       fringe spin kicks (§4.5); spin_place EDGES or MIDPOINT */
} st_kind;

typedef enum {
  ST_ORB_EXACT = 0, /* exact flow: drifts and sector bends                     */
  ST_ORB_DKD = 1,   /* drift-kick-drift slices (quadrupoles)                   */
  ST_ORB_MK = 2,    /* matrix-kick-matrix slices (§3.3 eq. quadConcat)         */
  ST_ORB_TEAPOT = 3, /* sector bend in drift-kick-drift slices: the drift of the
                       curved frame (§3.6 eq. teapotD) and the dipole kick
                       Px -= eta h (1 + hX) ds (from eq. teapotHK)             */
  ST_ORB_DKD4 = 4,  /* quadrupoles: each slice is three DKD slices of lengths
                       x1 ds, x0 ds, x1 ds, x1 = 1/(2 - 2^(1/3)), x0 = 1 - 2 x1
                       (a fourth-order symmetric composition; §3.3 after eq.
                       quadConcat); spin_place EDGES or MIDPOINT             */
  ST_ORB_MK4 = 5    /* quadrupoles: the same composition of MK slices          */
} st_orbit;

typedef enum {
  ST_SPIN_EDGES = 0,   /* Ω at the N + 1 slice edges, trapezoid level products
                          and the Romberg tableau (§4.3)                       */
  ST_SPIN_KICK = 1,    /* drift-kick slices only: one rotation by ds·Ω per
                          slice between its two half kicks (§5.2, "DKS")      */
  ST_SPIN_MIDPOINT = 2 /* one rotation by ds·Ω per slice, Ω at the slice's
                          middle between two half slices (§4.1 eq. pwcSpin;
                          "DKDS" for drift-kick slices)                        */
} st_spin_place;

typedef enum {
  ST_FP64 = 0,      /* every step in double precision                          */
  ST_MIXED = 1,     /* orbit, Ω, tableau, normalisation and element composition
                       in double; the edge quaternions and Romberg level
                       products in single precision with compensated sums, in
                       the elements whose finest-slice design rotation is at
                       most 0.02 rad (at 5 mm amplitude); double elsewhere     */
  ST_MIXED_ALL = 2  /* as ST_MIXED, single precision in every element          */
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
 *                used are R_e = min(R, 1 + ν2(N)), ν2 the power of 2 in N;
 *                must be 1 unless spin_place is ST_SPIN_EDGES
 *   spin_place   where the spin is integrated in a thick element
 *                (st_spin_place); ST_SPIN_KICK needs DKD quadrupole or
 *                TEAPOT bend slices
 *   fringe       sector bends and quadrupoles: 1 adds the spin kicks of thin
 *                magnet fringes at both faces (§4.5 eq. skfringe): rotations
 *                about the longitudinal axis by -(1 + G) b1 Y / (Bρ)0 (bend,
 *                b1/(Bρ)0 = eta·h) or -(1 + G) k1 X Y (quadrupole) at the
 *                entrance and the opposite expression at the exit; the orbit
 *                is unchanged.  0 for every other kind
 *   ks           solenoid longitudinal field b0/(Bρ)0 [m^-1] (0 otherwise)
 *   asym         rectangular bends: the turn of both faces away from the
 *                symmetric placement [rad]; the design orbit meets the
 *                entrance face at φ^entr = angle/2 + asym and the exit face at
 *                φ^exit = asym - angle/2 to the magnet's axis (§3.2), so the
 *                field is b1/(Bρ)0 = eta (sin φ^entr - sin φ^exit)/L.  0 is
 *                the symmetric magnet, and 0 for every other kind
 */
typedef struct {
  int32_t kind, orbit, n_slices, romberg_rows, spin_place, fringe;
  double L, angle, eta, k1, k1l, k2l, snake_phi, snake_mu, ks, asym;
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

/* Create a context on HIP device `device`.  *out receives the handle.
 * Passage: §6 — the bunch is moved to the GPU's global memory and tracked
 * there; a context is that device plus the lattice tables and scratch the
 * tracking needs. */
st_status st_create(st_ctx** out, int device);

/* Release the context and everything the library allocated for it.
 * Caller-owned particle memory is not touched.  NULL is accepted.
 * Passage: not in the paper (resource management). */
st_status st_destroy(st_ctx* ctx);

/* Copy n elements (host memory) and the beam into the context.
 * Passage: the element maps of §3 (§3.1 eq. sbend, §3.2 eq. rbend, §3.3
 * eq. quadL/quadNL/quadConcat, §3.4 eq. HmultD, §3.5, §3.6 eq. teapotD, §3.7
 * eq. solenoid), the spin placements of §4.1 and §4.3, the fringe kicks of
 * §4.4 and §4.5; units of §2.1.  Validation:
 * known kind, orbit method and spin placement; finite parameters; L ≥ 0;
 * sbends need L > 0, angle ≠ 0, the exact or TEAPOT method and, with the
 * exact method, eta > 0; quadrupoles need L > 0 and the DKD, MK, DKD4 or MK4
 * method; solenoids need L > 0 and ks ≠ 0; rectangular bends need L > 0,
 * angle ≠ 0, |φ^entr| < 1.5, |φ^exit| < 1.5 and eta ≠ 0 (asym ≠ 0 only
 * for them); thick elements need n_slices ≥ 1 and
 * romberg_rows in 1..4 (1 with a piece-wise constant placement); the kick
 * placement needs DKD or TEAPOT slices; fringe is 0 or 1 and only on sbends
 * and quadrupoles; gamma0 > 1; aperture > 0; report_every ≥ 0.
 * Synchronous; replaces any earlier lattice. */
st_status st_load_lattice(st_ctx* ctx, const st_element* host_elems, int64_t n,
                          const st_beam* beam);

/* Bind n particles held in caller-owned device memory (layout above).
 * n may be 0.  Pointers must be non-NULL when n > 0.
 * Passage: §6 — one GPU thread per particle, whose 6-D orbit (§2.1 eq.
 * psvars) and 3-D spin (§2.2) stay in global memory for the whole run. */
st_status st_bind_particles(st_ctx* ctx, int64_t n, double* d_z, double* d_spin,
                            int32_t* d_alive);

/* Passage: §6 (the quaternions that accumulate spin rotations belong to the
 * resident state) and §4.1 (the element rotations compose as quaternions).
 * Optionally bind a device array q (4 rows of n doubles: w, x, y, z) that
 * st_track fills with each particle's one-turn spin quaternion of the last
 * turn it tracked (the product of the element quaternions, later elements on
 * the left).  NULL unbinds.  Must follow st_bind_particles. */
st_status st_bind_quaternions(st_ctx* ctx, double* d_q);

/* Passage: §6 (the push of every particle through each element: orbit by
 * the element's integrator, Ω recorded at every slice edge, the quaternion
 * updated by piece-wise constant spin integration plus Romberg steps, then
 * the spin), with the orbit maps of §3, Ω of §2.2 eq. t-bmt.so, the slice
 * rotations of §4.1 and the tableau of §4.3 eq. romberg.
 * Track the bound particles for `turns` turns (≥ 0), asynchronously on
 * `stream`.  Updates z, spin, alive (and q if bound) in place and records
 * the polarization history of this call.  Each call starts at the lattice
 * start, so track(a + b) equals track(a) followed by track(b). */
st_status st_track(st_ctx* ctx, int64_t turns, void* stream);

/* Size of the fixed device scratch array behind st_track_noalloc. */
#define ST_NOALLOC_SCRATCH_BYTES (16u << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * st_track with every piece of device memory it needs already in place: it
 * runs the same kernels (results bit-identical to st_track's) and calls no
 * hipMalloc, hipFree or allocating library routine.  The per-block
 * polarization partials live in a fixed array of ST_NOALLOC_SCRATCH_BYTES in
 * device memory, one copy per GPU, whose address st_create takes; each GPU
 * holds it until the process ends.  The caller passes the outputs: d_pol
 * (caller-owned DEVICE memory, `capacity` reports of 4 doubles: Px, Py, Pz,
 * N_alive, as in st_polarization) receives this call's polarization history,
 * and *n_reports (host, may be NULL) the number of reports written.  The
 * lattice must be loaded and the particles bound beforehand (those calls do
 * allocate).
 * Limits: reports x blocks x 4 doubles must fit the scratch array, with
 * reports = turns / report_every and blocks = ceil(n / 256), i.e.
 * reports x ceil(n / 256) <= 524288 (e.g. 128 reports of 2^20 particles);
 * larger requests fail with ST_EINVAL before any device work, as does
 * capacity < reports.  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents (every slot a call reads it writes first):
 * calls that overlap in time on one GPU, from any context or stream, race
 * and must be serialised by the caller.  st_polarization reports no history
 * after this call. */
st_status st_track_noalloc(st_ctx* ctx, int64_t turns, double* d_pol, int64_t capacity,
                           int64_t* n_reports, void* stream);

/* Passage: not a formula of the paper.  §6 copies particle data back to the
 * host for analysis such as the invariant spin field (§1); this call gives
 * the plain bunch-mean spin of that analysis on the device instead.
 * Polarization history of the last st_track: for each report k, four doubles
 * (Px, Py, Pz, N_alive) with P = Σ_alive S_j / N_alive (0 if none alive).
 * Writes min(capacity, n_reports) reports to caller-owned DEVICE memory
 * d_out, queued on `stream`; *n_reports (host) receives the number of
 * reports recorded.  d_out may be NULL to query the count. */
st_status st_polarization(st_ctx* ctx, double* d_out, int64_t capacity,
                          int64_t* n_reports, void* stream);

/* Copy the bound particles to HOST memory (any pointer may be NULL to skip
 * that array).  Synchronises `stream` before returning.
 * Passage: §6 — particle data is copied back to the host for analysis. */
st_status st_read_particles(st_ctx* ctx, double* h_z, double* h_spin, int32_t* h_alive,
                            void* stream);

/* Human-readable description of the last error on this context (owned by
 * the context; valid until the next call).  Never NULL.
 * Passage: not in the paper (error reporting). */
const char* st_last_error(const st_ctx* ctx);

/* ------------------------------------------------------------------------
 * Spin surrogate (not part of the paper's method): an MLP
 * n_in -> 256 -> 256 -> 256 -> 4 with SiLU activations and normalised output
 * q = y/|y| that maps a particle's turn-start coordinates to its one-turn spin
 * quaternion.  The two 256×256 layers run in bf16 on the matrix cores with
 * fp32 accumulation; the first and last layers in fp32.  Training minimises
 * the mean of |q - t|² over a batch with Adam (β1 0.9, β2 0.999, ε 1e-8) on
 * fp32 master weights.  The flat parameter layout is W1 [256][n_in], b1 [256],
 * W2 [256][256], b2, W3 [256][256], b3, W4 [4][256], b4 [4] (W row-major
 * [out][in]).  Device arrays are row-major per sample: inputs x [n][n_in],
 * quaternions [n][4] (w, x, y, z).
 * ------------------------------------------------------------------------ */
typedef struct st_mlp st_mlp;

/* Passage: not in the paper (learned spin surrogate).
 * Create a network on HIP device `device` with n_in inputs (1..8) and hidden
 * width 256 (the only width supported).  Weights are uniform in
 * ±1/sqrt(fan_in) from a counter-based generator keyed by `seed`; biases 0. */
st_status st_mlp_create(st_mlp** out, int device, int32_t n_in, int32_t width, uint64_t seed);

/* Release the network.  NULL is accepted.
 * Passage: not in the paper (learned spin surrogate). */
st_status st_mlp_destroy(st_mlp* m);

/* Last error on this network (owned by it; never NULL).
 * Passage: not in the paper (learned spin surrogate). */
const char* st_mlp_last_error(const st_mlp* m);

/* Passage: not in the paper (learned spin surrogate).
 * Copy the fp32 master parameters to h_get and/or replace them from h_set
 * (host memory, *n_params floats; either pointer may be NULL).  *n_params
 * (host, may be NULL) receives the count.  Synchronous. */
st_status st_mlp_params(st_mlp* m, float* h_get, const float* h_set, int64_t* n_params);

/* Passage: not in the paper (learned spin surrogate).
 * Output frame of the network: with the last layer's output y, the
 * prediction is q = u/|u| for u = ref + scale ⊙ y (ref, scale: host, 4
 * doubles each, finite, scale > 0; stored as floats).  A reference
 * quaternion close to the targets and a scale of their spread around it let
 * the network learn only the deviation, so that its bf16 rounding error is
 * scaled down with it.  Default ref = 0, scale = 1.  Applies to training,
 * gradients, inference and surrogate tracking alike. */
st_status st_mlp_set_frame(st_mlp* m, const double* ref, const double* scale);

/* Passage: not in the paper (learned spin surrogate).
 * Linear part of the output frame: u = ref + lin x + scale ⊙ y, with x the
 * network's inputs and lin host row-major [4][n_in] doubles (finite; stored as
 * floats); NULL clears it (the default).  Applies wherever st_mlp_set_frame's
 * frame does.  ST_EINVAL for a non-finite value. */
st_status st_mlp_set_linear_frame(st_mlp* m, const double* lin);

/* Result of st_mlp_fit_frame (host struct; lin rows hold n_in used columns,
 * the rest zero). */
typedef struct {
  double ref[4];         /* intercept of each component */
  double lin[4][8];      /* slope per input */
  double scale[4];       /* max(resid_rms, floor) */
  double resid_rms[4];   /* RMS of the targets about ref + lin x */
  double resid_max[4];   /* largest residual magnitude */
} st_frame_fit;

/* Passage: not in the paper (learned spin surrogate).
 * Double-precision least-squares fit of the targets d_t [n][4] on the inputs
 * d_x [n][n_in] (device floats) plus a constant: the affine map ref + lin x
 * that minimises the summed squared residual of every component, from the
 * normal equations summed on the device in double (fixed order) and solved
 * on the host by Cholesky, with a ridge of 1e-12 of the mean diagonal on the
 * input columns.  Then it sets the network's whole frame: ref and lin as
 * fitted, scale = max(RMS residual, floor) per component, so that the network
 * learns only what the affine map leaves.  *out (host, may be NULL) receives
 * the fit.  Synchronous on `stream` (returns after the fit); allocates and
 * frees about 0.5 MB of device memory.  ST_EINVAL for NULL inputs, n <
 * n_in + 1, floor <= 0, or inputs whose normal equations are not positive
 * definite; ST_ENOMEM, ST_EDEVICE on device failures. */
st_status st_mlp_fit_frame(st_mlp* m, const float* d_x, const float* d_t, int64_t n, double floor,
                           st_frame_fit* out, void* stream);

/* Passage: not in the paper (learned spin surrogate).
 * One Adam step (learning rate lr > 0) on `batch` samples: inputs d_x, unit
 * quaternion targets d_t (device).  d_loss (device, 1 float, may be NULL)
 * receives the batch's mean loss before the step.  Queued on `stream`. */
st_status st_mlp_train_step(st_mlp* m, const float* d_x, const float* d_t, int64_t batch,
                            float lr, float* d_loss, void* stream);

/* Passage: not in the paper (learned spin surrogate).
 * Gradient of the batch's mean loss into d_grad (device, n_params floats)
 * without updating the weights; d_loss as in st_mlp_train_step. */
st_status st_mlp_gradient(st_mlp* m, const float* d_x, const float* d_t, int64_t batch,
                          float* d_grad, float* d_loss, void* stream);

/* Inference: d_q [n][4] (device) from d_x [n][n_in] (device).
 * Passage: not in the paper (learned spin surrogate). */
st_status st_mlp_infer(st_mlp* m, const float* d_x, float* d_q, int64_t n, void* stream);

/* Passage: not in the paper (learned spin surrogate).
 * Network inputs from particle coordinates (d_z: device 6×n SoA doubles):
 * x[j][i] = (z[i][j] - center[i]) * inv_scale[i] for i < 6 and, when
 * n_in == 7, x[j][6] = extra.  center, inv_scale: host, 6 doubles. */
st_status st_mlp_features(st_mlp* m, const double* d_z, int64_t n, const double* center,
                          const double* inv_scale, double extra, float* d_x, void* stream);

/* Passage: not in the paper (learned spin surrogate); the targets are the
 * one-turn quaternions of §4.1 composed by st_track.
 * Training targets from tracked one-turn quaternions (d_q: device 4×n SoA
 * doubles, as filled by st_track with st_bind_quaternions): t[j] = ±q_j
 * with the sign that makes t·ref >= 0 (ref: host, 4 doubles), as floats. */
st_status st_mlp_targets(st_mlp* m, const double* d_q, int64_t n, const double* ref, float* d_t,
                         void* stream);

/* Passage: not in the paper (learned spin surrogate with audits); its
 * audit and fallback turns are the method of st_track.
 * Track the bound particles for `turns` turns with the surrogate for spin.
 * Each turn a particle with d_fallback[j] == 0 gets the orbit push and a spin
 * rotation by the network's quaternion for its turn-start coordinates
 * (inputs as in st_mlp_features); a particle with d_fallback[j] != 0 gets the
 * full double-precision turn.  On the first turn of the call, on every
 * audit_every-th turn (>= 1) and on the call's last turn, every particle gets
 * the full double-precision turn and its network quaternion is compared with
 * the tracked one (the early audit finds the particles the network cannot
 * follow before they cost a long replay; the closing one leaves no network
 * turn unchecked).  When the largest component difference (after aligning
 * the sign) exceeds `threshold`, the particle falls back: d_fallback[j] is
 * set to the turn number (1-based, counted within this call), its state is
 * rolled back to the previous audit (or the start) and the turns since then
 * are replayed in double precision, so its spin carries no network error.
 * Only particles with d_fallback[j] == 0 are audited, so a non-zero value
 * left by an earlier call or set by the caller is never rolled back again:
 * such a particle runs every turn in double precision.  It stays on the
 * double-precision path afterwards.  The orbit is the double-precision orbit
 * throughout, and the spin does not act on it, so the turns between two
 * audits run as one launch of the orbit push that records every turn's
 * network inputs, one inference over all of them, and one pass that rotates
 * each particle by its turns' quaternions in turn order (the result is that
 * of applying them turn by turn).  d_fallback: device int32 [n], initialised
 * by the caller (0 = start on the network).  Polarization is recorded as in
 * st_track; the beam's report_every must then be a multiple of audit_every,
 * so that every report follows an audit.  Requires a lattice, particles and
 * a network created on the same device.  At most 2^31-1 particles; library
 * scratch: about 130 bytes per particle plus 48 bytes per particle and turn
 * of one launch, at most 512 MiB for the latter (longer stretches between
 * audits are split into several launches).  turns = 0 only reserves that
 * scratch for the bound particles and this audit_every, so that later calls
 * allocate nothing but the polarization history.  The particles on the
 * network and those on the fallback path are processed in separate waves. */
st_status st_track_surrogate(st_ctx* ctx, st_mlp* m, int64_t turns, int32_t audit_every,
                             double threshold, const double* center, const double* inv_scale,
                             double extra, int32_t* d_fallback, void* stream);

/* Measured peaks of the device: the denominators of the roofline fractions
 * (not a step of the method).
 *   fp64_fma_tflops   FP64 vector FMA rate, eight independent v_fma_f64 chains
 *                     per lane, 16 workgroups of 256 lanes per compute unit
 *   fp32_fma_tflops   the same with v_fma_f32, one operation per instruction
 *                     (the library is built without packed FP32 instructions)
 *   bf16_mfma_tflops  dense bf16 matrix rate, four independent chains of
 *                     v_mfma_f32_16x16x32_bf16 per wave
 *   copy_gbps         HBM bandwidth of a 16-byte copy of 1 GiB into 1 GiB,
 *                     read plus written bytes
 * Each is timed with HIP events over 10 launches after a warm-up launch. */
typedef struct {
  double fp64_fma_tflops, bf16_mfma_tflops, copy_gbps, fp32_fma_tflops;
} st_peaks;

/* Passage: not in the paper (measurement).
 * Run the four microbenchmarks on HIP device `device` and fill *out.
 * Synchronous; allocates and frees 2 GiB of device memory.  ST_EINVAL for a
 * NULL out or an unknown device, ST_EDEVICE if an allocation, launch or timing
 * call fails (out is then incomplete). */
st_status st_measure_peaks(int device, st_peaks* out);

#ifdef __cplusplus
}
#endif

#endif /* SPINTRACK_H */

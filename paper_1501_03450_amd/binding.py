"""ctypes binding of libspintrack.so: the C ABI of include/spintrack.h.

Argument marshalling only.  Functions keep the C names; each raises
SpinTrackError when the library returns a non-zero status.  Device memory
and streams come from PyTorch (tensor.data_ptr(), stream.cuda_stream).
The library must have been built (paper_1501_03450_amd/build.py); importing
this module fails loudly if it is missing.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# SPINTRACK_LIB selects another build of the same library (e.g. a different
# occupancy target); the default is the in-tree build.
LIB_PATH = os.environ.get("SPINTRACK_LIB", os.path.join(_HERE, "libspintrack.so"))

ST_OK, ST_EINVAL, ST_ENOMEM, ST_EDEVICE, ST_ESTATE = 0, -1, -2, -3, -4
ST_MARKER, ST_DRIFT, ST_SBEND, ST_QUAD, ST_THIN, ST_SNAKE, ST_SOLENOID, ST_RBEND = range(8)
ST_ORB_EXACT, ST_ORB_DKD, ST_ORB_MK, ST_ORB_TEAPOT, ST_ORB_DKD4, ST_ORB_MK4 = range(6)
ST_SPIN_EDGES, ST_SPIN_KICK, ST_SPIN_MIDPOINT = range(3)
ST_FP64, ST_MIXED, ST_MIXED_ALL = 0, 1, 2

KIND_CODES = {"marker": ST_MARKER, "drift": ST_DRIFT, "sbend": ST_SBEND, "quad": ST_QUAD,
              "thin": ST_THIN, "snake": ST_SNAKE, "solenoid": ST_SOLENOID, "rbend": ST_RBEND}
ORBIT_CODES = {"exact": ST_ORB_EXACT, "dkd": ST_ORB_DKD, "mk": ST_ORB_MK, "teapot": ST_ORB_TEAPOT,
               "dkd4": ST_ORB_DKD4, "mk4": ST_ORB_MK4}
SPIN_CODES = {"edges": ST_SPIN_EDGES, "kick": ST_SPIN_KICK, "midpoint": ST_SPIN_MIDPOINT}
PRECISION_CODES = {"fp64": ST_FP64, "mixed": ST_MIXED, "mixed_all": ST_MIXED_ALL}

EXPORTS = ("st_create", "st_destroy", "st_load_lattice", "st_bind_particles",
           "st_bind_quaternions", "st_track", "st_track_noalloc", "st_polarization", "st_read_particles",
           "st_last_error", "st_mlp_create", "st_mlp_destroy", "st_mlp_last_error",
           "st_mlp_params", "st_mlp_set_frame", "st_mlp_set_linear_frame", "st_mlp_fit_frame",
           "st_mlp_train_step", "st_mlp_gradient", "st_mlp_infer",
           "st_mlp_features", "st_mlp_targets", "st_track_surrogate", "st_measure_peaks")


class st_element(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("orbit", ctypes.c_int32),
                ("n_slices", ctypes.c_int32), ("romberg_rows", ctypes.c_int32),
                ("spin_place", ctypes.c_int32), ("fringe", ctypes.c_int32),
                ("L", ctypes.c_double), ("angle", ctypes.c_double), ("eta", ctypes.c_double),
                ("k1", ctypes.c_double), ("k1l", ctypes.c_double), ("k2l", ctypes.c_double),
                ("snake_phi", ctypes.c_double), ("snake_mu", ctypes.c_double),
                ("ks", ctypes.c_double), ("asym", ctypes.c_double)]


class st_peaks(ctypes.Structure):
    _fields_ = [("fp64_fma_tflops", ctypes.c_double), ("bf16_mfma_tflops", ctypes.c_double),
                ("copy_gbps", ctypes.c_double), ("fp32_fma_tflops", ctypes.c_double)]


class st_frame_fit(ctypes.Structure):
    _fields_ = [("ref", ctypes.c_double * 4), ("lin", (ctypes.c_double * 8) * 4),
                ("scale", ctypes.c_double * 4), ("resid_rms", ctypes.c_double * 4),
                ("resid_max", ctypes.c_double * 4)]


class st_beam(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("gamma0", ctypes.c_double), ("aperture", ctypes.c_double),
                ("precision", ctypes.c_int32), ("report_every", ctypes.c_int32)]


class SpinTrackError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"spintrack status {status}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1501_03450_amd/build.py "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.st_create.argtypes = [P(vp), i32]
    lib.st_destroy.argtypes = [vp]
    lib.st_load_lattice.argtypes = [vp, P(st_element), i64, P(st_beam)]
    lib.st_bind_particles.argtypes = [vp, i64, vp, vp, vp]
    lib.st_bind_quaternions.argtypes = [vp, vp]
    lib.st_track.argtypes = [vp, i64, vp]
    lib.st_track_noalloc.argtypes = [vp, i64, vp, i64, P(i64), vp]
    lib.st_polarization.argtypes = [vp, vp, i64, P(i64), vp]
    lib.st_read_particles.argtypes = [vp, vp, vp, vp, vp]
    lib.st_last_error.argtypes = [vp]
    lib.st_last_error.restype = ctypes.c_char_p
    f64, f32, u64 = ctypes.c_double, ctypes.c_float, ctypes.c_uint64
    lib.st_mlp_create.argtypes = [P(vp), i32, ctypes.c_int32, ctypes.c_int32, u64]
    lib.st_mlp_destroy.argtypes = [vp]
    lib.st_mlp_last_error.argtypes = [vp]
    lib.st_mlp_last_error.restype = ctypes.c_char_p
    lib.st_mlp_params.argtypes = [vp, vp, vp, P(i64)]
    lib.st_mlp_set_frame.argtypes = [vp, P(f64), P(f64)]
    lib.st_mlp_set_linear_frame.argtypes = [vp, P(f64)]
    lib.st_mlp_fit_frame.argtypes = [vp, vp, vp, i64, f64, P(st_frame_fit), vp]
    lib.st_mlp_train_step.argtypes = [vp, vp, vp, i64, f32, vp, vp]
    lib.st_mlp_gradient.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    lib.st_mlp_infer.argtypes = [vp, vp, vp, i64, vp]
    lib.st_mlp_features.argtypes = [vp, vp, i64, P(f64), P(f64), f64, vp, vp]
    lib.st_mlp_targets.argtypes = [vp, vp, i64, P(f64), vp, vp]
    lib.st_track_surrogate.argtypes = [vp, vp, i64, ctypes.c_int32, f64, P(f64), P(f64), f64, vp, vp]
    lib.st_measure_peaks.argtypes = [i32, P(st_peaks)]
    for name in EXPORTS:
        if name not in ("st_last_error", "st_mlp_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


LIB = _load()


def _check(ctx, status):
    if status != ST_OK:
        msg = LIB.st_last_error(ctx).decode() if ctx else "invalid argument"
        raise SpinTrackError(status, msg)


def st_last_error(ctx) -> str:
    return LIB.st_last_error(ctx).decode()


def st_create(device: int = 0):
    h = ctypes.c_void_p()
    st = LIB.st_create(ctypes.byref(h), int(device))
    if st != ST_OK:
        raise SpinTrackError(st, f"cannot create a context on device {device}")
    return h


def st_measure_peaks(device: int = 0) -> dict:
    """FP64 and unpacked FP32 FMA and bf16 MFMA rates [TFLOP/s] and HBM copy
    bandwidth [GB/s] measured on `device`."""
    p = st_peaks()
    st = LIB.st_measure_peaks(int(device), ctypes.byref(p))
    if st != ST_OK:
        raise SpinTrackError(st, f"peak microbenchmarks failed on device {device}")
    return {"fp64_fma_tflops": p.fp64_fma_tflops, "bf16_mfma_tflops": p.bf16_mfma_tflops,
            "copy_gbps": p.copy_gbps, "fp32_fma_tflops": p.fp32_fma_tflops}


def st_destroy(ctx) -> None:
    LIB.st_destroy(ctx)


def element_array(elements):
    """Marshal element records (objects with the st_element field names,
    string kind/method) into a ctypes array."""
    arr = (st_element * max(len(elements), 1))()
    for i, e in enumerate(elements):
        a = arr[i]
        a.kind = KIND_CODES[e.kind] if isinstance(e.kind, str) else int(e.kind)
        method = getattr(e, "method", getattr(e, "orbit", "exact"))
        a.orbit = ORBIT_CODES[method] if isinstance(method, str) else int(method)
        a.n_slices = int(e.n_slices)
        a.romberg_rows = int(getattr(e, "rows", getattr(e, "romberg_rows", 1)))
        place = getattr(e, "spin", getattr(e, "spin_place", "edges"))
        a.spin_place = SPIN_CODES[place] if isinstance(place, str) else int(place)
        a.L, a.angle, a.eta = float(e.L), float(e.angle), float(e.eta)
        a.k1, a.k1l, a.k2l = float(e.k1), float(e.k1l), float(e.k2l)
        a.snake_phi, a.snake_mu = float(e.snake_phi), float(e.snake_mu)
        a.ks = float(getattr(e, "ks", 0.0))
        a.fringe = int(getattr(e, "fringe", 0))
        a.asym = float(getattr(e, "asym", 0.0))
    return arr


def st_load_lattice(ctx, elements, G, gamma0, aperture, precision="fp64", report_every=0):
    arr = element_array(elements)
    b = st_beam(G=float(G), gamma0=float(gamma0), aperture=float(aperture),
                precision=PRECISION_CODES[precision] if isinstance(precision, str) else int(precision),
                report_every=int(report_every))
    _check(ctx, LIB.st_load_lattice(ctx, arr, len(elements), ctypes.byref(b)))


def st_load_lattice_raw(ctx, arr, n, beam):
    """Pass an already marshalled st_element array and st_beam (validation tests)."""
    return LIB.st_load_lattice(ctx, arr, int(n), ctypes.byref(beam) if beam is not None else None)


def st_bind_particles(ctx, n, z_ptr, spin_ptr, alive_ptr):
    _check(ctx, LIB.st_bind_particles(ctx, int(n), z_ptr, spin_ptr, alive_ptr))


def st_bind_quaternions(ctx, q_ptr):
    _check(ctx, LIB.st_bind_quaternions(ctx, q_ptr))


def st_track(ctx, turns, stream=None):
    _check(ctx, LIB.st_track(ctx, int(turns), stream))


def st_track_noalloc(ctx, turns, d_pol_ptr, capacity, stream=None) -> int:
    """Track with no device allocation; returns the number of reports written."""
    n = ctypes.c_int64(0)
    _check(ctx, LIB.st_track_noalloc(ctx, int(turns), d_pol_ptr, int(capacity), ctypes.byref(n),
                                     stream))
    return int(n.value)


def st_polarization(ctx, d_out_ptr=None, capacity=0, stream=None) -> int:
    n = ctypes.c_int64(0)
    _check(ctx, LIB.st_polarization(ctx, d_out_ptr, int(capacity), ctypes.byref(n), stream))
    return int(n.value)


def st_read_particles(ctx, h_z_ptr, h_spin_ptr, h_alive_ptr, stream=None):
    _check(ctx, LIB.st_read_particles(ctx, h_z_ptr, h_spin_ptr, h_alive_ptr, stream))


# ---------------------------------------------------------------- surrogate --

def _check_mlp(m, status):
    if status != ST_OK:
        msg = LIB.st_mlp_last_error(m).decode() if m else "invalid argument"
        raise SpinTrackError(status, msg)


def _d6(v):
    return (ctypes.c_double * 6)(*[float(x) for x in v])


def st_mlp_create(device=0, n_in=6, width=256, seed=0):
    h = ctypes.c_void_p()
    st = LIB.st_mlp_create(ctypes.byref(h), int(device), int(n_in), int(width), int(seed))
    if st != ST_OK:
        raise SpinTrackError(st, f"cannot create a network (n_in={n_in}, width={width})")
    return h


def st_mlp_destroy(m):
    LIB.st_mlp_destroy(m)


def st_mlp_params(m, h_get_ptr=None, h_set_ptr=None) -> int:
    n = ctypes.c_int64(0)
    _check_mlp(m, LIB.st_mlp_params(m, h_get_ptr, h_set_ptr, ctypes.byref(n)))
    return int(n.value)


def st_mlp_set_frame(m, ref, scale):
    r = (ctypes.c_double * 4)(*[float(x) for x in ref])
    c = (ctypes.c_double * 4)(*[float(x) for x in scale])
    _check_mlp(m, LIB.st_mlp_set_frame(m, r, c))


def st_mlp_set_linear_frame(m, lin=None):
    """lin: [4][n_in] values (None clears the linear part)."""
    if lin is None:
        _check_mlp(m, LIB.st_mlp_set_linear_frame(m, None))
        return
    flat = [float(v) for row in lin for v in row]
    _check_mlp(m, LIB.st_mlp_set_linear_frame(m, (ctypes.c_double * len(flat))(*flat)))


def st_mlp_fit_frame(m, x_ptr, t_ptr, n, floor, stream=None) -> dict:
    """The fitted frame as a dict of lists (lin rows with 8 columns)."""
    f = st_frame_fit()
    _check_mlp(m, LIB.st_mlp_fit_frame(m, x_ptr, t_ptr, int(n), float(floor), ctypes.byref(f),
                                       stream))
    return {"ref": list(f.ref), "lin": [list(r) for r in f.lin], "scale": list(f.scale),
            "resid_rms": list(f.resid_rms), "resid_max": list(f.resid_max)}


def st_mlp_train_step(m, x_ptr, t_ptr, batch, lr, loss_ptr=None, stream=None):
    _check_mlp(m, LIB.st_mlp_train_step(m, x_ptr, t_ptr, int(batch), float(lr), loss_ptr, stream))


def st_mlp_gradient(m, x_ptr, t_ptr, batch, grad_ptr, loss_ptr=None, stream=None):
    _check_mlp(m, LIB.st_mlp_gradient(m, x_ptr, t_ptr, int(batch), grad_ptr, loss_ptr, stream))


def st_mlp_infer(m, x_ptr, q_ptr, n, stream=None):
    _check_mlp(m, LIB.st_mlp_infer(m, x_ptr, q_ptr, int(n), stream))


def st_mlp_features(m, z_ptr, n, center, inv_scale, extra, x_ptr, stream=None):
    _check_mlp(m, LIB.st_mlp_features(m, z_ptr, int(n), _d6(center), _d6(inv_scale), float(extra),
                                      x_ptr, stream))


def st_mlp_targets(m, q_ptr, n, ref, t_ptr, stream=None):
    r = (ctypes.c_double * 4)(*[float(x) for x in ref])
    _check_mlp(m, LIB.st_mlp_targets(m, q_ptr, int(n), r, t_ptr, stream))


def st_track_surrogate(ctx, m, turns, audit_every, threshold, center, inv_scale, extra,
                       fallback_ptr, stream=None):
    _check(ctx, LIB.st_track_surrogate(ctx, m, int(turns), int(audit_every), float(threshold),
                                       _d6(center), _d6(inv_scale), float(extra), fallback_ptr,
                                       stream))

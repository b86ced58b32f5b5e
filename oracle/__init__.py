"""CPU oracle for the spin–orbit tracker — TEST INFRASTRUCTURE ONLY.

A plain, slow, single-particle-at-a-time implementation of the method of
Abell, Meiser, Ranjbar & Barber (2015), written from the paper in C++ and
called through ctypes.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does,
and this package never imports the GPU library.

Functions
  track(...)          whole-bunch tracking (extended or double precision)
  jacobian(...)       one-particle one-turn Jacobian by forward-mode duals
  count_ops(...)      operation counts of tracking one particle
  romberg(...)        the Romberg quadrature for spin on given edge values of Ω
  omega(...)          Ω of the T-BMT equation in s at one state
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spin_oracle.cpp")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lock = threading.Lock()
_lib = None

KIND_CODES = {"marker": 0, "drift": 1, "sbend": 2, "quad": 3, "thin": 4, "snake": 5,
              "solenoid": 6, "rbend": 7}
METHOD_CODES = {"exact": 0, "dkd": 1, "mk": 2, "teapot": 3, "dkd4": 4, "mk4": 5}
SPIN_CODES = {"edges": 0, "kick": 1, "midpoint": 2}


class _Elem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("method", ctypes.c_int32),
                ("nsl", ctypes.c_int32), ("rows", ctypes.c_int32),
                ("spin", ctypes.c_int32), ("fringe", ctypes.c_int32),
                ("L", ctypes.c_double), ("angle", ctypes.c_double), ("eta", ctypes.c_double),
                ("k1", ctypes.c_double), ("k1l", ctypes.c_double), ("k2l", ctypes.c_double),
                ("phi", ctypes.c_double), ("mu", ctypes.c_double), ("ks", ctypes.c_double),
                ("asym", ctypes.c_double)]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no FP contraction).  Returns the path."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-ffp-contract=off", "-std=c++17", "-shared", "-fPIC", "-pthread",
               _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER
            dp, ip = P(ctypes.c_double), P(ctypes.c_int32)
            lib.oracle_track.argtypes = [P(_Elem), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, dp, dp, ip, ctypes.c_int,
                                         ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int]
            lib.oracle_jacobian.argtypes = [P(_Elem), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, dp, dp, ctypes.c_int, dp, dp, dp, dp, dp]
            lib.oracle_count_ops.argtypes = [P(_Elem), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, dp, ctypes.c_int, P(ctypes.c_longlong)]
            lib.oracle_romberg.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, ctypes.c_int]
            lib.oracle_omega.argtypes = [dp, ctypes.c_double, dp, ctypes.c_double, ctypes.c_double, dp]
            lib.oracle_rotate.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
            assert lib.oracle_elem_size() == ctypes.sizeof(_Elem)
            _lib = lib
    return _lib


def _elems(elements):
    arr = (_Elem * len(elements))()
    for i, e in enumerate(elements):
        a = arr[i]
        a.kind = KIND_CODES[e.kind]
        a.method = METHOD_CODES[e.method]
        a.nsl, a.rows = int(e.n_slices), int(e.rows)
        a.spin = SPIN_CODES[getattr(e, "spin", "edges")]
        a.L, a.angle, a.eta = e.L, e.angle, e.eta
        a.k1, a.k1l, a.k2l = e.k1, e.k1l, e.k2l
        a.phi, a.mu = e.snake_phi, e.snake_mu
        a.ks = getattr(e, "ks", 0.0)
        a.fringe = int(bool(getattr(e, "fringe", False)))
        a.asym = float(getattr(e, "asym", 0.0))
        if a.asym != 0.0 and e.kind != "rbend":
            raise ValueError("asym applies to rectangular bends")
        if a.fringe and e.kind not in ("sbend", "quad"):
            raise ValueError("fringe spin kicks apply to sector bends and quadrupoles")
        if e.kind == "sbend" and e.method not in ("exact", "teapot"):
            raise ValueError("sector bends use the exact map or teapot drift-kick slices")
        if e.kind == "quad" and e.method not in ("dkd", "mk", "dkd4", "mk4"):
            raise ValueError("quadrupoles use dkd, mk, dkd4 or mk4 slices")
        if e.kind != "quad" and e.method in ("dkd4", "mk4"):
            raise ValueError("fourth-order compositions apply to quadrupoles")
        if e.kind == "rbend":
            if e.method != "exact" or e.n_slices < 1 or e.rows < 1 or e.L <= 0 or e.angle == 0:
                raise ValueError("rectangular bends: exact body, L > 0, angle != 0, n_slices, rows >= 1")
            if a.spin == SPIN_CODES["kick"]:
                raise ValueError("the kick spin placement needs drift-kick slices")
            if a.spin != SPIN_CODES["edges"] and e.rows != 1:
                raise ValueError("piece-wise constant spin placements take rows = 1")
            if not (abs(e.angle / 2 + a.asym) < 1.5 and abs(a.asym - e.angle / 2) < 1.5):
                raise ValueError("rectangular bends need |phi_entr|, |phi_exit| < 1.5")
        if e.kind == "solenoid":
            if e.method != "exact" or e.n_slices < 1 or e.rows < 1 or e.L <= 0 or e.ks == 0:
                raise ValueError("solenoids: exact body, L > 0, ks != 0, n_slices, rows >= 1")
            if a.spin == SPIN_CODES["kick"]:
                raise ValueError("the kick spin placement needs drift-kick slices")
            if a.spin != SPIN_CODES["edges"] and e.rows != 1:
                raise ValueError("piece-wise constant spin placements take rows = 1")
        if e.kind in ("sbend", "quad"):
            if a.spin == SPIN_CODES["kick"] and e.method not in ("dkd", "teapot"):
                raise ValueError("the kick spin placement needs drift-kick slices")
            if a.spin != SPIN_CODES["edges"] and e.rows != 1:
                raise ValueError("piece-wise constant spin placements take rows = 1")
        if e.kind in ("sbend", "quad") and (e.n_slices < 1 or e.rows < 1 or e.L <= 0):
            raise ValueError("thick elements need L > 0, n_slices >= 1, rows >= 1")
    return arr


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def track(elements, beam, z, spin, alive=None, turns=1, report_every=0, extended=True,
          threads=None, want_quaternion=False):
    """Track copies of (z[6][n], spin[3][n], alive[n]).

    Returns dict(z, spin, alive, pol[n_reports][4] or None, q[4][n] or None).
    `extended` selects x87 long double (the parity reference) or double.
    """
    lib = _load()
    z = np.array(z, dtype=np.float64, order="C", copy=True)
    spin = np.array(spin, dtype=np.float64, order="C", copy=True)
    n = z.shape[1]
    alive = np.ones(n, np.int32) if alive is None else np.array(alive, dtype=np.int32, copy=True)
    n_rep = turns // report_every if report_every > 0 else 0
    pol = np.zeros((max(n_rep, 1), 4))
    q = np.zeros((4, n)) if want_quaternion else None
    if threads is None:
        threads = os.cpu_count() or 1
    els = _elems(elements)
    lib.oracle_track(els, len(elements), beam.G, beam.gamma0, beam.aperture, n, _dp(z), _dp(spin),
                     alive.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(turns),
                     int(report_every), _dp(pol), _dp(q) if q is not None else None,
                     int(threads), 1 if extended else 0)
    return {"z": z, "spin": spin, "alive": alive, "pol": pol[:n_rep] if n_rep else None, "q": q}


def rotate(z, phi, beam):
    """The frame rotation of a rectangular-bend face (eq. prot) on one state."""
    lib = _load()
    zi = np.ascontiguousarray(z, dtype=np.float64)
    zo = np.zeros(6)
    lib.oracle_rotate(_dp(zi), float(phi), beam.G, beam.gamma0, _dp(zo))
    return zo


def jacobian(elements, beam, z0, s0=(0.0, 1.0, 0.0), turns=1):
    """Forward-mode derivatives of one particle's tracking (extended precision).

    Returns dict(J[6][6], dQ[4][6], z[6], spin[3], q[4], lost)."""
    lib = _load()
    z0 = np.ascontiguousarray(z0, dtype=np.float64)
    s0 = np.ascontiguousarray(s0, dtype=np.float64)
    J, dQ = np.zeros(36), np.zeros(24)
    zo, so, qo = np.zeros(6), np.zeros(3), np.zeros(4)
    lost = lib.oracle_jacobian(_elems(elements), len(elements), beam.G, beam.gamma0, beam.aperture,
                               _dp(z0), _dp(s0), int(turns), _dp(J), _dp(dQ), _dp(zo), _dp(so), _dp(qo))
    return {"J": J.reshape(6, 6), "dQ": dQ.reshape(4, 6), "z": zo, "spin": so, "q": qo, "lost": lost}


OP_NAMES = ("add", "mul", "div", "sqrt", "sincos", "asin", "sinhcosh")


def count_ops(elements, beam, z0, turns=1):
    """Operation counts of tracking one particle for `turns` turns."""
    lib = _load()
    z0 = np.ascontiguousarray(z0, dtype=np.float64)
    c = (ctypes.c_longlong * 7)()
    lib.oracle_count_ops(_elems(elements), len(elements), beam.G, beam.gamma0, beam.aperture,
                         _dp(z0), int(turns), c)
    return dict(zip(OP_NAMES, [int(v) for v in c]))


def romberg(omega_edges, ds, rows, extended=True):
    """Normalised Romberg-limit quaternion from Ω at N + 1 slice edges."""
    lib = _load()
    om = np.ascontiguousarray(omega_edges, dtype=np.float64)
    assert om.ndim == 2 and om.shape[1] == 3
    q = np.zeros(4)
    lib.oracle_romberg(_dp(om), om.shape[0] - 1, float(ds), int(rows), _dp(q), 1 if extended else 0)
    return q


def omega(z, h, b, beam):
    """Ω of the T-BMT equation in s (eq. t-bmt.so) at state z, curvature h, field b."""
    lib = _load()
    z = np.ascontiguousarray(z, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    out = np.zeros(3)
    lib.oracle_omega(_dp(z), float(h), _dp(b), beam.G, beam.gamma0, _dp(out))
    return out

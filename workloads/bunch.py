"""Seeded Gaussian bunches in the canonical coordinates (X, Px, Y, Py, T, Pt).

The bunch recipe: X, Y with σ = 1 mm; Px, Py with σ = 0.1 mrad (Px, Py are
momenta scaled by the reference momentum, so they are taken as the angles);
T with σ = 1 cm; a relative momentum deviation δ with σ = 1e-3, converted to
the scaled energy deviation Pt through the definition of Pt in §2.1 (eq. pt):
Pt = E/(p0 c) - 1/β0 with E/(p0 c) = sqrt((1+δ)^2 + 1/(β0 γ0)^2).  No
truncation.  Spins start vertical, (0, 1, 0).

Random numbers come from numpy's Philox counter-based generator keyed by the
seed, so a (seed, n) pair always gives the same bunch on any machine.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

PROTON_G = 1.792847
SEED_BASE = 1501034500


@dataclasses.dataclass(frozen=True)
class Beam:
    G: float = PROTON_G
    gamma0: float = 25.0
    # Loss aperture on |X| and |Y| (m).  On the RHIC-scale ring the bunch
    # stays inside it for 1000 turns; on the small ring, whose dispersion
    # reaches ~18 m, the δ tails of the unmatched bunch swing out to ~0.1 m
    # and a sixth of the 1024-particle bunch is lost within 256 turns.
    aperture: float = 0.05

    @property
    def beta0(self) -> float:
        return math.sqrt(1.0 - 1.0 / (self.gamma0 * self.gamma0))


SIGMAS = {"X": 1e-3, "Px": 1e-4, "Y": 1e-3, "Py": 1e-4, "T": 1e-2, "delta": 1e-3}


def _coords(g: np.ndarray, scale: float, beam: Beam) -> np.ndarray:
    """Coordinates from standard normals g[6][n] (rows X, Px, Y, Py, T, δ)."""
    z = np.empty(g.shape, dtype=np.float64)
    z[0] = SIGMAS["X"] * scale * g[0]
    z[1] = SIGMAS["Px"] * scale * g[1]
    z[2] = SIGMAS["Y"] * scale * g[2]
    z[3] = SIGMAS["Py"] * scale * g[3]
    z[4] = SIGMAS["T"] * scale * g[4]
    delta = SIGMAS["delta"] * scale * g[5]
    b0g0 = beam.beta0 * beam.gamma0
    z[5] = np.sqrt((1.0 + delta) ** 2 + 1.0 / (b0g0 * b0g0)) - 1.0 / beam.beta0
    return z


def _draw(n: int, seed: int, scale: float, beam: Beam):
    rng = np.random.Generator(np.random.Philox(key=seed))
    return _coords(rng.standard_normal((6, n)), scale, beam)


def gaussian_bunch(n: int, seed: int, beam: Beam = Beam(), scale: float = 1.0):
    """Return (z[6][n], spin[3][n], alive[n]) as contiguous SoA numpy arrays."""
    z = _draw(n, seed, scale, beam)
    spin = np.zeros((3, n), dtype=np.float64)
    spin[1] = 1.0
    alive = np.ones(n, dtype=np.int32)
    return np.ascontiguousarray(z), spin, alive


def widened_bunch(n: int, seed: int, beam: Beam = Beam(), factor: float = 3.0):
    """The same recipe with every σ multiplied by `factor` (surrogate training inputs)."""
    return gaussian_bunch(n, seed, beam, scale=factor)


def energy_scan_gammas(n_energies: int = 256, G: float = PROTON_G,
                       ggamma_lo: float = 45.0, ggamma_hi: float = 50.0) -> np.ndarray:
    """Reference γ0 values with Gγ0 uniform (bin centres) in [lo, hi]."""
    i = np.arange(n_energies, dtype=np.float64)
    ggamma = ggamma_lo + (ggamma_hi - ggamma_lo) * (i + 0.5) / n_energies
    return ggamma / G


def energy_scan_bunches(gammas, n_per: int, seed: int, G: float = PROTON_G, scale: float = 1.0):
    """One bunch per reference energy from a single seeded draw: bunch i uses
    the normals of columns [i·n_per, (i+1)·n_per) of one (6, len·n_per) draw,
    converted to Pt with its own β0.  Returns a list of (beam, z, spin, alive)."""
    gammas = np.asarray(gammas, dtype=np.float64)
    rng = np.random.Generator(np.random.Philox(key=seed))
    g_all = rng.standard_normal((6, len(gammas) * n_per))
    out = []
    for i, g0 in enumerate(gammas):
        beam = Beam(G=G, gamma0=float(g0))
        z = _coords(g_all[:, i * n_per:(i + 1) * n_per], scale, beam)
        spin = np.zeros((3, n_per))
        spin[1] = 1.0
        out.append((beam, np.ascontiguousarray(z), spin, np.ones(n_per, dtype=np.int32)))
    return out


def random_spins(n: int, seed: int, opening_angle: float) -> np.ndarray:
    """Unit spins uniform on the cap of half-angle `opening_angle` about +y.

    Uniform on a spherical cap: cos of the polar angle uniform in
    [cos α, 1], azimuth uniform (the area element of the sphere is
    d(cos θ) dφ).
    """
    rng = np.random.Generator(np.random.Philox(key=seed))
    u = rng.random(n)
    phi = 2.0 * math.pi * rng.random(n)
    cz = 1.0 - u * (1.0 - math.cos(opening_angle))
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    spin = np.empty((3, n))
    spin[1] = cz
    spin[0] = sz * np.cos(phi)
    spin[2] = sz * np.sin(phi)
    return spin

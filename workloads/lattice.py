"""Ring lattices used as tracking workloads.

Each element is a plain record.  Units are SI; magnet strengths are already
normalised to the reference rigidity (Bρ)0, so a quadrupole carries
k1 = b2/(Bρ)0 in m^-2 and a thin sextupole carries its integrated strength
K2L = (∂²By/∂x²)·ℓ/(Bρ)0 in m^-2 (MAD sign convention).

Element kinds
  drift   straight field-free region of length L
  sbend   sector bend of length L and geometric bend angle `angle`
          (curvature h = angle/L); eta = b1/(h (Bρ)0) is the powering ratio
  quad    normal quadrupole of length L, gradient k1
  thin    thin normal multipole: integrated quadrupole k1l and sextupole k2l
  snake   thin spin rotator: rotation angle snake_phi about the horizontal
          axis (sin mu, 0, cos mu) in (x, y, s); transparent to the orbit
  solenoid  longitudinal field ks = b0/(Bρ)0 over L with thin-pancake fringes
  rbend   rectangular bend of straight length L bending the design orbit by
          `angle`; the design orbit meets the entrance face at angle/2 + asym
          and the exit face at asym - angle/2 (asym = 0: symmetric); eta is
          the powering ratio
  marker  does nothing

Orbit integration methods
  exact   exact flow (drift, sector bend, solenoid)
  dkd     drift-kick-drift slices (quadrupoles)
  mk      matrix-kick-matrix slices (quadrupoles)
  teapot  drift-kick-drift slices of a sector bend in its curved frame
  dkd4, mk4  quadrupole slices of three dkd or mk steps of lengths
          x1 ds, x0 ds, x1 ds (x1 = 1/(2 - 2^(1/3)), x0 = 1 - 2 x1): fourth order

Spin placement in thick elements (`spin`)
  edges     Ω at the slice edges, Romberg tableau over R rows (default)
  kick      drift-kick slices: one rotation per slice between its half kicks
  midpoint  one rotation per slice with Ω at the slice's middle

`fringe` (sector bends and quadrupoles) adds the spin kicks of thin magnet
fringes at both faces; the orbit is unchanged.

`n_slices` is the number of orbit slices N; `rows` is the number R of
Romberg tableau rows requested for the element's spin (R = 1 means the plain
trapezoid product with no extrapolation).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

KINDS = ("marker", "drift", "sbend", "quad", "thin", "snake", "solenoid", "rbend")
METHODS = ("exact", "dkd", "mk", "teapot", "dkd4", "mk4")
SPIN_PLACES = ("edges", "kick", "midpoint")


@dataclasses.dataclass(frozen=True)
class Element:
    kind: str
    L: float = 0.0
    angle: float = 0.0
    eta: float = 1.0
    k1: float = 0.0
    k1l: float = 0.0
    k2l: float = 0.0
    snake_phi: float = 0.0
    snake_mu: float = 0.0
    method: str = "exact"
    n_slices: int = 1
    rows: int = 1
    name: str = ""
    spin: str = "edges"
    ks: float = 0.0
    fringe: bool = False
    asym: float = 0.0          # rectangular bend: φ^entr = angle/2 + asym, φ^exit = asym - angle/2

    def __post_init__(self):
        if self.kind not in KINDS:
            raise ValueError(f"unknown element kind {self.kind!r}")
        if self.method not in METHODS:
            raise ValueError(f"unknown integration method {self.method!r}")
        if self.spin not in SPIN_PLACES:
            raise ValueError(f"unknown spin placement {self.spin!r}")
        if self.fringe and self.kind not in ("sbend", "quad"):
            raise ValueError("fringe spin kicks apply to sector bends and quadrupoles")
        if self.asym != 0.0 and self.kind != "rbend":
            raise ValueError("asym applies to rectangular bends")


def drift(L: float, name: str = "D") -> Element:
    return Element("drift", L=L, name=name)


def sbend(L: float, angle: float, n: int, rows: int, eta: float = 1.0, name: str = "SB",
          method: str = "exact", spin: str = "edges", fringe: bool = False) -> Element:
    """Sector bend; fringe=True adds the thin-fringe spin kicks of its faces."""
    return Element("sbend", L=L, angle=angle, eta=eta, n_slices=n, rows=rows, name=name,
                   method=method, spin=spin, fringe=fringe)


def quad(L: float, k1: float, method: str, n: int, rows: int, name: str = "Q",
         spin: str = "edges", fringe: bool = False) -> Element:
    """Quadrupole; fringe=True adds the thin-fringe spin kicks of its faces."""
    return Element("quad", L=L, k1=k1, method=method, n_slices=n, rows=rows, name=name, spin=spin,
                   fringe=fringe)


def solenoid(L: float, ks: float, n: int, rows: int, name: str = "SOL",
             spin: str = "edges") -> Element:
    """Solenoid of length L and longitudinal field ks = b0/(Bρ)0 [1/m], with
    thin-pancake fringes; n body slices and R Romberg rows for the spin."""
    return Element("solenoid", L=L, ks=ks, n_slices=n, rows=rows, name=name, spin=spin)


def rbend(L: float, angle: float, n: int, rows: int, eta: float = 1.0, name: str = "RB",
          spin: str = "edges", asym: float = 0.0) -> Element:
    return Element("rbend", L=L, angle=angle, eta=eta, n_slices=n, rows=rows, name=name, spin=spin,
                   asym=asym)


def thin(k1l: float = 0.0, k2l: float = 0.0, name: str = "M") -> Element:
    return Element("thin", k1l=k1l, k2l=k2l, name=name)


def snake(phi: float, mu: float, name: str = "SNAKE") -> Element:
    return Element("snake", snake_phi=phi, snake_mu=mu, name=name)


def small_ring(quad_slices: int = 8, bend_slices: int = 8, rows: int = 3,
               quad_method: str = "dkd", with_snake: bool = True) -> List[Element]:
    """16-cell FODO ring of 480 m with one thin full snake (the small test ring).

    Cell: QF(1 m, k1=+0.05) D2 SB(10 m, 2π/32) D2 QD(1 m, k1=-0.05) D2 SB D2.
    The snake rotates spin by π about the longitudinal axis (mu = 0) and sits
    at the end of the ring.
    """
    th = 2.0 * math.pi / 32.0
    cell = [
        quad(1.0, +0.05, quad_method, quad_slices, rows, "QF"),
        drift(2.0, "D2"),
        sbend(10.0, th, bend_slices, rows, name="SB"),
        drift(2.0, "D2"),
        quad(1.0, -0.05, quad_method, quad_slices, rows, "QD"),
        drift(2.0, "D2"),
        sbend(10.0, th, bend_slices, rows, name="SB"),
        drift(2.0, "D2"),
    ]
    ring = cell * 16
    if with_snake:
        ring = ring + [snake(math.pi, 0.0, "SNAKE")]
    return ring


# Geometry of the RHIC-scale ring: 6 arcs of 11 FODO cells (4 sector bends
# each, 264 bends summing to 2π) and 6 straights of 27 FODO cells whose drift
# length closes the circumference at 3800 m.
RHIC_CIRCUMFERENCE = 3800.0
ARC_CELLS_PER_ARC = 11
STRAIGHT_CELLS = 27
N_ARCS = 6


# The ring's thin sextupoles have gradient k2 = ±0.5 m^-3 over a nominal
# length of 0.1 m, i.e. integrated K2L = ±0.05 m^-2.  (With K2L = ±0.5 about a
# quarter of the Gaussian bunch is lost within 200 turns, and no arc drift
# lengths or straight-cell count tried keeps 99 %; with ±0.05 none of 512
# particles is lost in 1000 turns at the 0.05 m aperture.)
RHIC_SEXT_K2L = 0.05


def rhic_like_ring(quad_slices: int = 4, bend_slices: int = 8, rows: int = 4,
                   sext_k2l: float = RHIC_SEXT_K2L, with_snakes: bool = True,
                   straight_cells: int = STRAIGHT_CELLS) -> List[Element]:
    """RHIC-scale synthetic ring: 1706 elements, 3800 m, two snakes at ±45°.

    Arc cell (16 elements, 42.8 m):
      QF(1.1, +0.08, MK) d0.3 SF(thin +K2L) d0.3 SB(9.45, 2π/264) d0.5 SB d0.3
      QD(1.1, -0.08, MK) d0.3 SD(thin -K2L) d0.3 SB d0.5 SB d0.3
    Straight cell: QF d_a QD d_a.  Snakes (angle π, axes +45° and -45°) sit at
    the start of straights 1 and 4, so exactly π of bending separates them.
    """
    th = 2.0 * math.pi / (4 * ARC_CELLS_PER_ARC * N_ARCS)
    QF = quad(1.1, +0.08, "mk", quad_slices, rows, "QF")
    QD = quad(1.1, -0.08, "mk", quad_slices, rows, "QD")
    SB = sbend(9.45, th, bend_slices, rows, name="SB")
    d03, d05 = drift(0.3, "d0.3"), drift(0.5, "d0.5")
    SF, SD = thin(k2l=+sext_k2l, name="SF"), thin(k2l=-sext_k2l, name="SD")
    arc_cell = [QF, d03, SF, d03, SB, d05, SB, d03, QD, d03, SD, d03, SB, d05, SB, d03]
    arc_len = sum(e.L for e in arc_cell) * ARC_CELLS_PER_ARC
    straight_len = (RHIC_CIRCUMFERENCE - N_ARCS * arc_len) / N_ARCS
    a = (straight_len / straight_cells - 2 * 1.1) / 2.0
    da = drift(a, "da")
    straight = [QF, da, QD, da] * straight_cells
    ring: List[Element] = []
    for k in range(N_ARCS):
        ring += arc_cell * ARC_CELLS_PER_ARC
        if with_snakes and k == 0:
            ring.append(snake(math.pi, +math.pi / 4, "SNAKE+45"))
        if with_snakes and k == 3:
            ring.append(snake(math.pi, -math.pi / 4, "SNAKE-45"))
        ring += straight
    return ring


def uniform_bend_ring(n_bends: int = 16, L: float = 5.0, n_slices: int = 8, rows: int = 3) -> List[Element]:
    """A ring made only of identical sector bends (total angle 2π)."""
    return [sbend(L, 2.0 * math.pi / n_bends, n_slices, rows) for _ in range(n_bends)]


def lattice_summary(elements: Sequence[Element]) -> dict:
    counts = {}
    for e in elements:
        counts[e.kind] = counts.get(e.kind, 0) + 1
    def path_length(e):
        # a rectangular bend's straight length L spans the design arc of
        # radius L/(2 cos(asym) sin(angle/2))
        if e.kind == "rbend":
            return e.L * e.angle / (2.0 * math.cos(e.asym) * math.sin(e.angle / 2.0))
        return e.L
    return {
        "n_elements": len(elements),
        "circumference_m": float(sum(path_length(e) for e in elements)),
        "total_bend_angle": float(sum(e.angle for e in elements)),
        "counts": counts,
    }


ELEMENT_DTYPE = np.dtype([
    ("kind", "U8"), ("method", "U8"), ("spin", "U8"), ("n_slices", "i4"), ("rows", "i4"),
    ("fringe", "i4"), ("L", "f8"), ("angle", "f8"), ("eta", "f8"), ("k1", "f8"), ("k1l", "f8"),
    ("k2l", "f8"), ("snake_phi", "f8"), ("snake_mu", "f8"), ("ks", "f8"), ("asym", "f8"),
])


def element_table(elements: Sequence[Element]) -> np.ndarray:
    """Elements as a numpy structured array (names for kind and method)."""
    out = np.zeros(len(elements), dtype=ELEMENT_DTYPE)
    for i, e in enumerate(elements):
        out[i] = (e.kind, e.method, e.spin, e.n_slices, e.rows, int(e.fringe), e.L, e.angle,
                  e.eta, e.k1, e.k1l, e.k2l, e.snake_phi, e.snake_mu, e.ks, e.asym)
    return out

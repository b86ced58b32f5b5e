"""Pins of the two oracle outputs that are neither orbit nor spin: the
polarization reduction, and the operation counter whose totals are the
numerator of the benchmark's roofline.

The polarization is P = Σ S_j / N_alive over the particles still alive after
a reported turn, at the lattice start (the quantity the paper's invariant-spin
-field and polarization studies average, §1).  The pin recomputes it with
numpy from the oracle's own per-turn states, on a bunch that loses particles
in several different turns, so a division by the bunch size, a lost particle
still counted, or a report taken at the wrong turn all fail.

The operation counts are pinned by hand counts of the printed formulas (§3.1
eq. sbend, §3.3 eq. quadL and eq. quadNL, §3.4 eq. HmultD at zero
multipoles, §2.2 eq. t-bmt.so, §4.1 and §4.3), and the benchmark's constants
are pinned to the counter on the ring it times.
"""

import os
import sys

import numpy as np
import pytest

import oracle
from workloads import Beam, gaussian_bunch, rhic_like_ring, small_ring
from workloads.bunch import random_spins
from workloads.lattice import drift, quad, sbend, thin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def lossy_ring(k2l):
    """The small ring with one pair of strong thin sextupoles: particles of a
    widened bunch leave a narrow aperture over several turns."""
    ring = small_ring(quad_slices=2, bend_slices=2, rows=2)
    return ring[:8] + [thin(k2l=k2l)] + ring[8:40] + [thin(k2l=-k2l)] + ring[40:]


def per_turn_reference(ring, beam, z, s, a, turns):
    """Track one turn at a time (double precision, so that the state passed
    from call to call is exactly the state inside one long call) and average
    the spins of the particles still alive with numpy."""
    ref = []
    for _ in range(turns):
        r = oracle.track(ring, beam, z, s, a, turns=1, extended=False)
        z, s, a = r["z"], r["spin"], r["alive"]
        live = a == 1
        n_alive = int(live.sum())
        mean = s[:, live].sum(axis=1) / n_alive if n_alive else np.zeros(3)
        ref.append((mean, n_alive, a.copy()))
    return ref


@pytest.mark.parametrize("k2l,aperture,every", [(2.0, 0.05, 1), (2.0, 0.05, 3), (10.0, 0.02, 2)])
def test_polarization_is_the_mean_spin_of_the_particles_alive_after_the_turn(k2l, aperture, every):
    beam = Beam(aperture=aperture)
    ring = lossy_ring(k2l)
    n, turns = 400, 12
    z, _, a = gaussian_bunch(n, 7, beam, scale=3.0)
    s = random_spins(n, 8, 1.0)
    a[::37] = -5                  # a few particles arrive already lost
    ref = per_turn_reference(ring, beam, z, s, a, turns)
    out = oracle.track(ring, beam, z, s, a, turns=turns, report_every=every, extended=False)
    pol = out["pol"]
    assert pol.shape == (turns // every, 4)
    counts = [ref[t][1] for t in range(turns)]
    # the losses really happen in several turns, and some particles survive
    # or (last case) none do
    assert len(set(counts)) >= 4
    for k in range(turns // every):
        mean, n_alive, _ = ref[(k + 1) * every - 1]
        assert pol[k, 3] == n_alive
        np.testing.assert_allclose(pol[k, :3], mean, rtol=1e-13, atol=1e-15)
    # the long call ends in the per-turn calls' final state, loss flags included
    np.testing.assert_array_equal(out["alive"], ref[-1][2])
    if counts[-1] == 0:
        np.testing.assert_array_equal(pol[-1], 0.0)


def test_polarization_of_an_unpolarised_cap_is_its_mean_direction():
    # Spins uniform on a cap of half-angle α about +y average to
    # (1 + cos α)/2 ŷ; with a ring of identity spin transport (a drift) the
    # report is that mean, up to the sampling noise of n spins.
    beam = Beam()
    n, alpha = 40000, 1.2
    z, _, a = gaussian_bunch(n, 11, beam)
    s = random_spins(n, 12, alpha)
    out = oracle.track([drift(1.0)], beam, z, s, a, turns=1, report_every=1, extended=False)
    pol = out["pol"][0]
    assert pol[3] == n
    expect = np.array([0.0, (1 + np.cos(alpha)) / 2, 0.0])
    np.testing.assert_allclose(pol[:3], expect, atol=5e-3)


# ----------------------------------------------------------- op counter ----

Z0 = np.array([1e-3, -2e-4, 5e-4, 1e-4, 1e-3, 2e-4])   # generic: every rotation non-zero


def test_counts_of_one_drift():
    """Hand count of one drift element in a one-element ring, one turn.

    Ps = sqrt(1 + (2/β0) Pt + Pt² - Px² - Py²)          div 1, mul 4, add 4, sqrt 1
    X += L Px / Ps ; Y += L Py / Ps                      div 2, mul 2, add 2
    T += L/β0 - L (1/β0 + Pt)/Ps                         div 3, mul 1, add 3
    per element, whatever the kind: S ← q S q* (two Hamilton products) and
    the turn quaternion q ⊗ Q (one), 16 mul + 12 add each  mul 48, add 36
    total: add 45, mul 55, div 6, sqrt 1.
    """
    c = oracle.count_ops([drift(2.0)], Beam(), Z0)
    assert c == {"add": 45, "mul": 55, "div": 6, "sqrt": 1, "sincos": 0, "asin": 0, "sinhcosh": 0}


OMEGA = dict(add=16, mul=26, div=6, sqrt=2)
"""Ω of eq. t-bmt.so at one state:
Ps (div 1, mul 4, add 4, sqrt 1); P (div 1, mul 2, add 2, sqrt 1);
û = (Px, Py, Ps)/P (div 3); γ = γ0(1 + β0 Pt) (mul 2, add 1);
a1 = 1 + Gγ, a2 = G(γ - 1) (mul 2, add 2); û·b (mul 3, add 2);
f = -(1 + hX)/Ps (mul 1, add 1, div 1); three components
f (a1 b_i - a2 (û·b) u_i) (mul 12, add 3); + h on the y component (add 1)."""

EDGE_QUATERNION = dict(add=14, mul=27, div=3, sqrt=1, sincos=2)
"""One trapezoid factor of §4.3 at a slice edge: step = w · stride · ds
(mul 2), ω = step Ω (mul 3), q(ω) = (cos θ/2, sin(θ/2) ω/θ) with
θ = |ω| (mul 3, add 2, sqrt 1; θ/2 and sin(θ/2)/θ: div 3; cos, sin: 2;
mul 3), and the level product q ⊗ Q (mul 16, add 12)."""


def add_counts(*parts, **extra):
    tot = {}
    for p in parts + (extra,):
        for k, v in p.items():
            tot[k] = tot.get(k, 0) + v
    return tot


def full(c):
    return {k: c.get(k, 0) for k in oracle.OP_NAMES}


def test_counts_of_one_exact_sector_bend_step():
    """Hand count of a sector bend with one slice and one tableau row (§3.1
    eq. sbend, the spin from §4.1 at the two edges).

    ds = L/N, h = θ/L                                     div 2
    field b = (0, ηh, 0), twice (with h = θ/L again)      div 2, mul 2
    Ω at both edges                                       2 × OMEGA
    the step, called with h = θ/L                         div 1, plus
      Pα = sqrt(1 + (2/β0)Pt + Pt² - Py²)                 div 1, mul 3, add 3, sqrt 1
      cos(hs), sin(hs)                                    mul 2, sincos 2
      A = sqrt(Pα² - Px²) - η(1 + hX)                     mul 4, add 3, sqrt 1
      Px(s) = Px cos + A sin                              mul 2, add 1
      Px'(s) = h(-Px sin + A cos)                         mul 3, add 1
      X(s) = (1/h)((1/η)(sqrt(Pα² - Px(s)²) - Px'/h) - 1) div 3, mul 4, add 3, sqrt 1
      D = asin(Px/Pα) - asin(Px(s)/Pα)                    div 2, asin 2, add 1
      Y += (1/η) Py s + (1/(ηh)) Py D                     div 2, mul 5, add 2
      T += -(1/η) Pt s - (1/(ηh))(1/β0 + Pt) D
           + (1 - 1/η) s/β0                               div 5, mul 6, add 5
    tableau of one row: two edge factors                  2 × EDGE_QUATERNION
    normalisation Q/|Q|                                   mul 4, add 3, sqrt 1, div 4
    per-element spin rotation and turn product            mul 48, add 36
    """
    step = dict(div=1 + 1 + 3 + 2 + 2 + 5, mul=3 + 2 + 4 + 2 + 3 + 4 + 5 + 6,
                add=3 + 3 + 1 + 1 + 3 + 1 + 2 + 5, sqrt=3, sincos=2, asin=2)
    expect = add_counts(OMEGA, OMEGA, step, EDGE_QUATERNION, EDGE_QUATERNION,
                        div=2 + 2 + 4, mul=2 + 4 + 48, add=3 + 36, sqrt=1)
    c = oracle.count_ops([sbend(10.0, 0.2, 1, 1)], Beam(), Z0)
    assert c == full(expect)
    assert c == {"add": 118, "mul": 189, "div": 40, "sqrt": 10, "sincos": 6, "asin": 2,
                 "sinhcosh": 0}


@pytest.mark.parametrize("k1", [0.05, -0.05])
def test_counts_of_one_matrix_kick_quadrupole_slice(k1):
    """Hand count of a quadrupole with one MK slice and one tableau row (§3.3
    eq. quadConcat: linear map over ds/2, eq. quadNL over ds, linear map over
    ds/2).  The defocusing case swaps the planes and costs the same.

    ds = L/N                                              div 1
    field b = k1 (Y, X, 0), twice                         mul 4
    Ω at both edges                                       2 × OMEGA
    ds/2, twice                                           div 2
    eq. quadL, twice, each:
      P = sqrt(1 + (2/β0)Pt + Pt²)                        div 1, mul 2, add 2, sqrt 1
      κ = sqrt(|k1|/P), κs                                div 1, sqrt 1, mul 1
      cos, sin, cosh, sinh of κs                          sincos 2, sinhcosh 2
      X, Px, Y, Py                                        div 4, mul 14, add 4
      px = Px/P, py = Py/P                                div 2
      sin 2κs, sinh 2κs                                   mul 2, sincos 1, sinhcosh 1
      the four terms of the T brace                       div 8, mul 28, add 9
      T -= (1/P)(1/β0 + Pt) brace                         div 2, mul 2, add 2
    eq. quadNL:
      P and Ps                                            div 2, mul 6, add 6, sqrt 2
      X, Y += s P(x,y) (1/Ps - 1/P)                       div 4, mul 4, add 4
      T                                                   div 5, mul 7, add 5
    two edge factors, normalisation, per-element rotation as for the bend
    """
    lin = dict(div=1 + 1 + 4 + 2 + 8 + 2, mul=2 + 1 + 14 + 2 + 28 + 2, add=2 + 4 + 9 + 2,
               sqrt=2, sincos=3, sinhcosh=3)
    nl = dict(div=2 + 4 + 5, mul=6 + 4 + 7, add=6 + 4 + 5, sqrt=2)
    expect = add_counts(OMEGA, OMEGA, lin, lin, nl, EDGE_QUATERNION, EDGE_QUATERNION,
                        div=1 + 2 + 4, mul=4 + 4 + 48, add=3 + 36, sqrt=1)
    c = oracle.count_ops([quad(1.0, k1, "mk", 1, 1)], Beam(), Z0)
    assert c == full(expect)
    assert c == {"add": 148, "mul": 277, "div": 72, "sqrt": 13, "sincos": 10, "asin": 0,
                 "sinhcosh": 6}


def test_counts_add_up_over_a_lattice_and_over_turns():
    one = [oracle.count_ops([e], Beam(), Z0) for e in (drift(2.0), sbend(10.0, 0.2, 1, 1))]
    both = oracle.count_ops([drift(2.0), sbend(10.0, 0.2, 1, 1)], Beam(), Z0)
    assert both == {k: one[0][k] + one[1][k] for k in oracle.OP_NAMES}
    two = oracle.count_ops([drift(2.0)], Beam(), Z0, turns=2)
    assert two == {k: 2 * one[0][k] for k in oracle.OP_NAMES}


def test_benchmark_constants_are_the_counter_on_the_timed_ring():
    # bench.py's roofline numerator: flops counted as add/sub = 1 and mul = 1
    # (the oracle contracts no FMA), divisions, square roots and elementary
    # functions reported apart; and the all-operations count kept next to it
    sys.path.insert(0, ROOT)
    import bench
    c = oracle.count_ops(rhic_like_ring(), Beam(), Z0)
    assert bench.FLOPS_PER_PARTICLE_TURN == c["add"] + c["mul"]
    assert bench.OPS_PER_PARTICLE_TURN == sum(c.values())
    assert bench.OTHER_OPS_PER_PARTICLE_TURN == {k: c[k] for k in
                                                 ("div", "sqrt", "sincos", "asin", "sinhcosh")}
    # the count does not depend on the particle, only on the lattice
    c2 = oracle.count_ops(rhic_like_ring(), Beam(), Z0 * -0.7)
    assert c2 == c

"""Pins of the oracle's drift-kick sector bend (§3.6, the TEAPOT split) and
of the piece-wise constant spin placements (§4.1 eq. pwcSpin; the DKS and
DKDS placements of §5.2): brute-force integration of the curved drift
Hamiltonian, the flow's group property, convergence orders against the exact
sector bend and a brute-force spin integration, and the one-turn comparison
of drift-kick against bend-kick/matrix-kick orbits that the paper prints."""

import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import bruteforce as bf
import oracle
from workloads import Beam, small_ring
from workloads.lattice import drift, quad, sbend, snake

BEAM = Beam()
WIDE = Beam(aperture=10.0)        # the curved drift moves a particle far from the arc
Z0 = np.array([1e-3, 1e-4, 2e-3, -2e-4, 0.01, 1e-3])
S0 = np.array([0.1952, 0.9759, 0.0976]) / np.linalg.norm([0.1952, 0.9759, 0.0976])
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_elements.json")))
L, ANG = 10.0, 2 * math.pi / 32
H = ANG / L


def run(elems, z, s=S0, beam=BEAM):
    r = oracle.track(elems, beam, np.asarray(z, float)[:, None], np.asarray(s, float)[:, None],
                     want_quaternion=True)
    assert r["alive"][0] == 1
    return r["z"][:, 0], r["spin"][:, 0]


def curved_drift(length, h=H):
    # a sector "bend" with no field (η = 0) is the drift of the curved frame:
    # its drift-kick slice has no kick
    return sbend(length, h * length, 1, 1, eta=0.0, method="teapot")


def test_curved_drift_is_the_flow_of_its_hamiltonian():
    f = bf._rhs_thick("drift", {"h": H}, WIDE)
    sol = solve_ivp(f, (0.0, L), np.concatenate([Z0, S0]), method="DOP853", rtol=1e-13, atol=1e-16)
    z, _ = run([curved_drift(L)], Z0, beam=WIDE)
    np.testing.assert_allclose(z, sol.y[:6, -1], rtol=0, atol=2e-14)
    assert abs(z[0]) > 0.5                  # a straight line leaves the arc quadratically


def test_curved_drift_group_property():
    a, _ = run([curved_drift(0.7), curved_drift(1.6)], Z0, beam=WIDE)
    b, _ = run([curved_drift(2.3)], Z0, beam=WIDE)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-16)


def test_curved_drift_becomes_the_straight_drift_as_the_curvature_vanishes():
    # the difference from the straight drift is first order in h
    b, _ = run([drift(2.0)], Z0)
    d = [np.abs(run([curved_drift(2.0, h=h)], Z0)[0] - b).max() for h in (1e-3, 1e-4, 1e-5)]
    ratios = np.array(d[:-1]) / np.array(d[1:])
    assert np.all(np.abs(ratios - 10.0) < 0.1), (d, ratios)


def test_drift_kick_bend_converges_at_second_order_to_the_exact_bend():
    zx, _ = run([sbend(L, ANG, 1, 1)], Z0)
    errs = [np.abs(run([sbend(L, ANG, N, 1, method="teapot")], Z0)[0] - zx).max()
            for N in (8, 16, 32)]
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.1), ratios


def test_drift_kick_bend_keeps_the_design_orbit_only_approximately():
    # the design particle leaves the arc in each drift and is pulled back by
    # the kick: the orbit error is second order in the slice length
    z = np.zeros(6)
    d = [np.abs(run([sbend(L, ANG, N, 1, method="teapot")], z)[0]).max() for N in (8, 16)]
    assert d[0] > 1e-6 and 3.8 < d[0] / d[1] < 4.2


@pytest.mark.parametrize("elem", [
    lambda N: sbend(L, ANG, N, 1, method="teapot", spin="kick"),
    lambda N: sbend(L, ANG, N, 1, method="teapot", spin="midpoint"),
    lambda N: sbend(L, ANG, N, 1, spin="midpoint"),
    lambda N: quad(1.1, 0.08, "dkd", N, 1, spin="kick"),
    lambda N: quad(1.1, 0.08, "mk", N, 1, spin="midpoint"),
    lambda N: quad(1.1, -0.08, "mk", N, 1, spin="midpoint"),
], ids=["teapot-kick", "teapot-midpoint", "exact-midpoint", "dkd-kick", "mk-midpoint",
        "mk-defocusing-midpoint"])
def test_piecewise_constant_spin_converges_at_second_order_to_brute_force(elem):
    _, sb = bf.track_element(elem(1), BEAM, Z0, S0)
    errs = [np.abs(run([elem(N)], Z0)[1] - sb).max() for N in (8, 16, 32)]
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.3), (errs, ratios)


def test_midpoint_spin_with_an_exact_orbit_is_the_pwc_product_of_mid_slice_rotations():
    # exact bend, midpoint placement, two slices: the quaternion is
    # q(Δs Ω(z(3Δs/2))) q(Δs Ω(z(Δs/2))) with the mid states from the exact map
    ds = L / 2
    zm1, _ = run([sbend(ds / 2, ANG / 4, 1, 1)], Z0)
    zm2, _ = run([sbend(3 * ds / 2, 3 * ANG / 4, 1, 1)], Z0)
    b = np.array([0.0, H, 0.0])

    def qrot(w):
        th = np.linalg.norm(w)
        return np.concatenate([[math.cos(th / 2)], math.sin(th / 2) / th * w])

    def qmul(a, c):
        return np.array([a[0] * c[0] - a[1:] @ c[1:],
                         *(a[0] * c[1:] + c[0] * a[1:] + np.cross(a[1:], c[1:]))])
    q1 = qrot(ds * np.array(bf._omega(zm1[0], zm1[1], zm1[3], zm1[5], H, b, BEAM)))
    q2 = qrot(ds * np.array(bf._omega(zm2[0], zm2[1], zm2[3], zm2[5], H, b, BEAM)))
    q = qmul(q2, q1)
    r = oracle.track([sbend(L, ANG, 2, 1, spin="midpoint")], BEAM, Z0[:, None], S0[:, None],
                     want_quaternion=True)
    np.testing.assert_allclose(r["q"][:, 0], q, rtol=0, atol=1e-14)


def _ring(style, N):
    th = 2 * math.pi / 32
    if style == "dk":
        qf = quad(1.0, 0.05, "dkd", N, 1, "QF", spin="kick")
        qd = quad(1.0, -0.05, "dkd", N, 1, "QD", spin="kick")
        sb = sbend(10.0, th, N, 1, method="teapot", spin="kick")
    else:
        qf = quad(1.0, 0.05, "mk", N, 1, "QF", spin="midpoint")
        qd = quad(1.0, -0.05, "mk", N, 1, "QD", spin="midpoint")
        sb = sbend(10.0, th, N, 1, spin="midpoint")
    cell = [qf, drift(2.0), sb, drift(2.0), qd, drift(2.0), sb, drift(2.0)]
    return cell * 16 + [snake(math.pi, 0.0)]


def test_one_turn_spin_bend_kick_orbits_beat_drift_kick_by_the_printed_decades():
    z0 = np.array([2e-3, -1e-4, 1e-3, 1e-4, 0.0, 5e-4])
    _, sb = bf.track_line(small_ring(), BEAM, z0, S0)
    decades = []
    for N in (4, 8, 16):
        e_dk = np.abs(run(_ring("dk", N), z0)[1] - sb).max()
        e_bk = np.abs(run(_ring("bkmk", N), z0)[1] - sb).max()
        decades.append(math.log10(e_dk / e_bk))
    printed = GOLDEN["one_turn_spin_dk_vs_bkmk"]["decades"]
    assert np.all(np.abs(np.array(decades) - printed) < 0.5), decades


def test_invalid_spin_placements_are_rejected():
    with pytest.raises(ValueError):
        oracle.track([sbend(L, ANG, 4, 1, spin="kick")], BEAM, Z0[:, None], S0[:, None])
    with pytest.raises(ValueError):
        oracle.track([quad(1.0, 0.05, "mk", 4, 2, spin="midpoint")], BEAM, Z0[:, None], S0[:, None])

"""Pins of the oracle's multipole fringe spin kicks (§4.5 eq. skfringe) on
sector bends (m = 1) and quadrupoles (m = 2): brute-force Lorentz tracking
through short linear fringes built from a vector potential (so that the
longitudinal fringe field is there), the order of what the lowest-order
kick leaves out, and the planes where the longitudinal fringe field
vanishes."""

import numpy as np
import pytest

import bruteforce as bf
import oracle
from workloads import Beam
from workloads.lattice import drift, quad, sbend

BEAM = Beam()
S0 = np.array([0.1952, 0.9759, 0.0976]) / np.linalg.norm([0.1952, 0.9759, 0.0976])


def run(elems, z, s=S0):
    r = oracle.track(elems, BEAM, np.asarray(z, float)[:, None], np.asarray(s, float)[:, None],
                     want_quaternion=True)
    assert r["alive"][0] == 1
    return r["z"][:, 0], r["spin"][:, 0], r["q"][:, 0]


def residuals(make, z0, eps):
    """Spin error against the brute force of the hard-edge magnet (between
    drifts of eps/2) with and without the fringe kicks."""
    _, sb = bf.track_fringed(make(True), eps, BEAM, z0, S0)
    _, s_on, _ = run([drift(eps / 2), make(True), drift(eps / 2)], z0)
    _, s_off, _ = run([drift(eps / 2), make(False), drift(eps / 2)], z0)
    return np.abs(s_on - sb).max(), np.abs(s_off - sb).max()


def test_quadrupole_fringe_kicks_against_brute_force():
    # The kick (1 + G) k1 X Y is second order; what the lowest-order form
    # leaves out is third order, so halving every amplitude shrinks the
    # spin error without kicks 4x and with kicks about 8x.
    make = lambda fr: quad(1.0, 0.5, "mk", 32, 4, fringe=fr)
    base = np.array([5e-3, -3e-3, 5e-3, 2e-3, 0.0, 1e-3])
    on, off = [], []
    for scale in (1.0, 0.5, 0.25):
        z0 = base * np.array([scale] * 4 + [1.0, 1.0])
        a, b = residuals(make, z0, 1e-3)
        on.append(a)
        off.append(b)
    on, off = np.array(on), np.array(off)
    assert off[0] > 1e-5
    assert np.all(on < 0.03 * off), (on, off)
    assert np.all(np.abs(off[:-1] / off[1:] - 4.0) < 0.1), off
    assert np.all(on[:-1] / on[1:] > 6.5), on


def test_sector_bend_fringe_kicks_against_brute_force():
    # m = 1: the kick (1 + G) η h Y is first order; the residual (the part of
    # the longitudinal field across the velocity, of order Px Y, and the
    # kinetic swing inside a short fringe) is of higher order.
    make = lambda fr: sbend(3.0, 0.12, 32, 4, fringe=fr)
    base = np.array([1e-3, -6e-4, 1e-3, 4e-4, 0.0, 2e-4])
    on, off = [], []
    for scale in (1.0, 0.5, 0.25):
        z0 = base * np.array([scale] * 4 + [1.0, 1.0])
        a, b = residuals(make, z0, 4e-3)
        on.append(a)
        off.append(b)
    on, off = np.array(on), np.array(off)
    assert off[0] > 1e-4
    assert np.all(on < 0.01 * off), (on, off)
    assert np.all(np.abs(off[:-1] / off[1:] - 2.0) < 0.05), off
    assert np.all(on[:-1] / on[1:] > 2.8), on


@pytest.mark.parametrize("z0", [
    [0.0, 0.0, 2e-3, 3e-4, 0.01, 1e-3],      # X = 0 plane: no quadrupole B_s
    [2e-3, 3e-4, 0.0, 0.0, 0.01, 1e-3],      # midplane: no B_s at all
])
def test_quadrupole_kicks_vanish_where_the_fringe_field_does(z0):
    for method in ("mk", "dkd"):
        _, s1, q1 = run([quad(1.0, 0.5, method, 8, 3, fringe=True)], z0)
        _, s0, q0 = run([quad(1.0, 0.5, method, 8, 3)], z0)
        np.testing.assert_array_equal(q1, q0)
        np.testing.assert_array_equal(s1, s0)


@pytest.mark.parametrize("method", ["exact", "teapot"])
def test_sector_bend_kicks_vanish_in_the_midplane(method):
    z0 = [2e-3, 3e-4, 0.0, 0.0, 0.01, 1e-3]
    _, _, q1 = run([sbend(3.0, 0.12, 8, 3, method=method, fringe=True)], z0)
    _, _, q0 = run([sbend(3.0, 0.12, 8, 3, method=method)], z0)
    np.testing.assert_array_equal(q1, q0)


def test_kicks_leave_the_orbit_alone_and_wrap_every_spin_placement():
    # the orbit is that of the hard-edge magnet; the element quaternion is
    # q_exit · Q_body · q_entrance for Romberg and piece-wise constant bodies
    z0 = np.array([2e-3, 3e-4, -1.5e-3, 2e-4, 0.01, 1e-3])
    for mk in (lambda fr, sp: quad(1.0, 0.5, "dkd", 8, 1 if sp != "edges" else 3, spin=sp,
                                   fringe=fr),
               lambda fr, sp: sbend(3.0, 0.12, 8, 1 if sp != "edges" else 3, spin=sp,
                                    method="teapot", fringe=fr)):
        for sp in ("edges", "kick", "midpoint"):
            z1, _, q1 = run([mk(True, sp)], z0)
            z0b, _, q0 = run([mk(False, sp)], z0)
            np.testing.assert_array_equal(z1, z0b)
            assert np.abs(q1 - q0).max() > 1e-8
            assert abs(np.linalg.norm(q1) - 1.0) < 1e-15


def test_fringe_flag_is_rejected_off_bends_and_quadrupoles():
    from workloads.lattice import Element
    with pytest.raises(ValueError):
        Element("drift", L=1.0, fringe=True)
    with pytest.raises(ValueError):
        Element("rbend", L=1.0, angle=0.1, n_slices=4, rows=1, fringe=True)

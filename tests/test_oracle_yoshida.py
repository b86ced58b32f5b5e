"""Pins of the oracle's fourth-order quadrupole slices (dkd4, mk4): three
second-order slices of lengths x1 ds, x0 ds, x1 ds composed symmetrically
(the higher-order compositions §3.3 mentions).  Pinned by the order of
convergence to brute-force Lorentz tracking, the field-free limit (a drift),
time reversal, symplecticity, and the spin order that the better orbit lets
the Romberg tableau reach."""

import numpy as np
import pytest

import bruteforce as bf
import oracle
from workloads import Beam
from workloads.lattice import drift, quad

BEAM = Beam()
S0 = np.array([0.1952, 0.9759, 0.0976]) / np.linalg.norm([0.1952, 0.9759, 0.0976])
Z_SMALL = np.array([5e-3, -3e-3, 5e-3, 2e-3, 0.01, 1e-3])
Z_LARGE = np.array([2e-2, 1e-2, -2e-2, 1e-2, 0.01, 1e-3])


def run(elems, z, s=S0):
    r = oracle.track(elems, BEAM, np.asarray(z, float)[:, None], np.asarray(s, float)[:, None])
    assert r["alive"][0] == 1
    return r["z"][:, 0], r["spin"][:, 0]


def errors(method, rows, z0, Ns=(2, 4, 8, 16)):
    zb, sb = bf.track_element(quad(1.0, 0.5, "mk", 1, 1), BEAM, z0, S0)
    eo, es = [], []
    for N in Ns:
        z, s = run([quad(1.0, 0.5, method, N, rows)], z0)
        eo.append(np.abs(z - zb).max())
        es.append(np.abs(s - sb).max())
    return np.array(eo), np.array(es)


def slopes(e):
    return np.log2(e[:-1] / e[1:])


@pytest.mark.parametrize("method,z0", [("dkd4", Z_SMALL), ("mk4", Z_LARGE)])
def test_orbit_converges_at_fourth_order_to_brute_force(method, z0):
    eo, _ = errors(method, 1, z0)
    assert np.all(np.abs(slopes(eo) - 4.0) < 0.1), (eo, slopes(eo))
    # and the second-order slice it is built from converges at second order
    e2, _ = errors(method[:-1], 1, z0)
    assert np.all(np.abs(slopes(e2) - 2.0) < 0.1), (e2, slopes(e2))
    assert eo[-1] < 0.01 * e2[-1]


def test_field_free_composition_is_a_drift():
    # the three lengths add up to ds (2 x1 + x0 = 1), and drifts compose exactly
    z0 = Z_LARGE
    zd, sd = run([drift(1.3)], z0)
    for method in ("dkd4", "mk4"):
        for N in (1, 3):
            z, s = run([quad(1.3, 0.0 if method == "dkd4" else 1e-300, method, N, 1)], z0)
            np.testing.assert_allclose(z, zd, rtol=0, atol=2e-16)


@pytest.mark.parametrize("method", ["dkd4", "mk4"])
def test_fourth_order_slice_is_time_reversible(method):
    # symmetric composition of reversible flows: M(R M(z)) = R z
    R = np.array([1, -1, 1, -1, -1, 1.0])
    e = quad(1.1, 0.08, method, 4, 1)
    z1, _ = run([e], Z_SMALL)
    z2, _ = run([e], R * z1)
    np.testing.assert_allclose(R * z2, Z_SMALL, rtol=0, atol=2e-16)


@pytest.mark.parametrize("method", ["dkd4", "mk4"])
def test_fourth_order_slice_is_symplectic(method):
    J = oracle.jacobian([quad(1.1, 0.5, method, 3, 1)], BEAM, Z_LARGE)["J"]
    S = np.kron(np.eye(3), np.array([[0.0, 1.0], [-1.0, 0.0]]))
    assert np.abs(J.T @ S @ J - S).max() < 1e-14


def test_spin_order_follows_the_orbit_order():
    # Romberg over the slice edges cannot beat the orbit error at the edges:
    # with two tableau rows (fourth order in the spin) the second-order dkd
    # orbit holds the spin at second order, the fourth-order orbit lets it
    # reach fourth order; with three rows mk4 reaches sixth order where mk
    # stalls at second.
    _, s2 = errors("dkd", 2, Z_SMALL)
    _, s4 = errors("dkd4", 2, Z_SMALL)
    assert np.all(np.abs(slopes(s2) - 2.0) < 0.15), s2
    assert np.all(np.abs(slopes(s4) - 4.0) < 0.1), s4
    _, m2 = errors("mk", 3, Z_LARGE)
    _, m4 = errors("mk4", 3, Z_LARGE)
    assert slopes(m2)[-1] < 2.5, m2
    assert np.all(np.abs(slopes(m4)[1:] - 6.0) < 0.2), m4


def test_fourth_order_methods_are_rejected_where_they_do_not_apply():
    from workloads.lattice import Element
    with pytest.raises(ValueError):
        oracle.track([Element("sbend", L=1.0, angle=0.1, n_slices=4, rows=1, method="dkd4")], BEAM,
                     Z_SMALL[:, None].copy(), S0[:, None].copy())
    with pytest.raises(ValueError):
        oracle.track([quad(1.0, 0.05, "dkd4", 4, 1, spin="kick")], BEAM,
                     Z_SMALL[:, None].copy(), S0[:, None].copy())

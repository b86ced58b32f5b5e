"""Pins of the oracle's orbit maps (§3) against mathematics that needs no
implementation: group properties, conserved quantities, closed-form loci,
textbook matrices, time reversal, symplecticity and a brute-force ODE
integration of the general Hamiltonian."""

import math

import numpy as np
import pytest

import bruteforce as bf
import oracle
from workloads import Beam, rhic_like_ring, small_ring
from workloads.lattice import drift, quad, sbend, snake, thin

BEAM = Beam()
Z0 = np.array([1e-3, 1e-4, 2e-3, -2e-4, 0.01, 1e-3])
S0 = np.array([0.0, 1.0, 0.0])


def run(elems, z, s=S0, beam=BEAM, **kw):
    r = oracle.track(elems, beam, np.asarray(z, float)[:, None], np.asarray(s, float)[:, None],
                     want_quaternion=True, **kw)
    return r["z"][:, 0], r["spin"][:, 0], r["q"][:, 0], r["alive"][0]


def ps(z, beam=BEAM):
    b0 = beam.beta0
    return math.sqrt(1 + 2 * z[5] / b0 + z[5] ** 2 - z[1] ** 2 - z[3] ** 2)


# ---------------------------------------------------------------- drift ----

def test_drift_group_property():
    a, _, _, _ = run([drift(0.7), drift(1.6)], Z0)
    b, _, _, _ = run([drift(2.3)], Z0)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-16)


def test_drift_is_a_straight_line_at_the_particle_speed():
    L = 2.0
    z1, _, _, _ = run([drift(L)], Z0)
    P = math.sqrt(1 + 2 * Z0[5] / BEAM.beta0 + Z0[5] ** 2)
    v = np.array([Z0[1], Z0[3], ps(Z0)]) / P           # unit velocity
    path = L / v[2]                                     # straight path to s = L
    np.testing.assert_allclose(z1[0] - Z0[0], path * v[0], rtol=1e-15, atol=1e-19)
    np.testing.assert_allclose(z1[2] - Z0[2], path * v[1], rtol=1e-15, atol=1e-19)
    # -c Δt relative to the reference: c t_ref = L/β0, c t = path/β,
    # β = p/E = P/(1/β0 + Pt) in scaled units (eq. pt)
    beta = P / (1 / BEAM.beta0 + Z0[5])
    np.testing.assert_allclose(z1[4] - Z0[4], L / BEAM.beta0 - path / beta, rtol=1e-12, atol=1e-17)
    np.testing.assert_array_equal(z1[[1, 3, 5]], Z0[[1, 3, 5]])


# ----------------------------------------------------------- sector bend ----

SB = dict(L=10.0, angle=2 * math.pi / 32)


def test_sbend_preserves_origin_when_correctly_powered():
    z1, _, _, _ = run([sbend(SB["L"], SB["angle"], 8, 3)], np.zeros(6))
    np.testing.assert_allclose(z1, 0.0, atol=1e-18)


@pytest.mark.parametrize("eta", [1.0, 1.01])
def test_sbend_is_an_exact_flow(eta):
    # one step of L, eight steps of L/8 and two bends of L/2 agree
    one, _, _, _ = run([sbend(SB["L"], SB["angle"], 1, 1, eta=eta)], Z0)
    eight, _, _, _ = run([sbend(SB["L"], SB["angle"], 8, 1, eta=eta)], Z0)
    halves, _, _, _ = run([sbend(SB["L"] / 2, SB["angle"] / 2, 1, 1, eta=eta)] * 2, Z0)
    np.testing.assert_allclose(one, eight, rtol=0, atol=2e-17)
    np.testing.assert_allclose(one, halves, rtol=0, atol=2e-17)


@pytest.mark.parametrize("eta", [1.0, 1.01])
def test_sbend_conserves_P_alpha_Py_Pt_and_the_hamiltonian(eta):
    h = SB["angle"] / SB["L"]
    z1, _, _, _ = run([sbend(SB["L"], SB["angle"], 4, 1, eta=eta)], Z0)
    b0 = BEAM.beta0

    def H(z):  # eq. generalH with the sector-bend potential (§3.1 eq. sbendA)
        return -(1 + h * z[0]) * ps(z) + eta / 2 * (1 + h * z[0]) ** 2 + z[5] / b0

    assert z1[3] == Z0[3] and z1[5] == Z0[5]
    assert abs(H(z1) - H(Z0)) < 1e-15


def test_sbend_px_sym_locus():
    # eq. dpx0: entering with Px = Px_sym(X) the particle leaves with the same Px
    import mpmath as mp
    mp.mp.dps = 40
    h, L = mp.mpf(SB["angle"]) / SB["L"], mp.mpf(SB["L"])
    b0 = mp.sqrt(1 - 1 / mp.mpf(BEAM.gamma0) ** 2)
    for X, Py, Pt in [(3e-3, 1e-4, 1e-3), (-2e-2, -2e-4, -2e-4), (5e-2, 0.0, 2e-4)]:
        c, s = mp.cos(h * L / 2), mp.sin(h * L / 2)
        pxs = float(c * (mp.sqrt(1 + 2 * Pt / b0 + Pt ** 2 - Py ** 2 - (1 + h * X) ** 2 * c * c)
                         - (1 + h * X) * s))
        z = np.array([X, pxs, 0.0, Py, 0.0, Pt])
        z1, _, _, _ = run([sbend(SB["L"], SB["angle"], 1, 1)], z)
        assert abs(z1[1] - pxs) < 4e-18


@pytest.mark.parametrize("eta", [1.0, 1.01])
def test_sbend_matches_brute_force(eta):
    e = sbend(SB["L"], SB["angle"], 8, 3, eta=eta)
    zb, _ = bf.track_element(e, BEAM, Z0, S0)
    z1, _, _, _ = run([e], Z0)
    np.testing.assert_allclose(z1, zb, rtol=0, atol=5e-15)


# ------------------------------------------------------------ quadrupoles ----

def _element_jacobian(e, z):
    r = oracle.jacobian([e], BEAM, z)
    return r["J"]


@pytest.mark.parametrize("k1", [0.05, -0.08])
@pytest.mark.parametrize("Pt", [0.0, 2e-3])
def test_mk_quad_linear_part_is_the_textbook_thick_quad(k1, Pt):
    L = 1.1
    J = _element_jacobian(quad(L, k1, "mk", 4, 1), np.array([0, 0, 0, 0, 0, Pt]))
    P = math.sqrt(1 + 2 * Pt / BEAM.beta0 + Pt * Pt)
    k = math.sqrt(abs(k1) / P)
    foc = np.array([[math.cos(k * L), math.sin(k * L) / (k * P)],
                    [-k * P * math.sin(k * L), math.cos(k * L)]])
    defo = np.array([[math.cosh(k * L), math.sinh(k * L) / (k * P)],
                     [k * P * math.sinh(k * L), math.cosh(k * L)]])
    Mx, My = (foc, defo) if k1 > 0 else (defo, foc)
    np.testing.assert_allclose(J[0:2, 0:2], Mx, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(J[2:4, 2:4], My, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(J[0:2, 2:4], 0.0, atol=1e-18)


def test_mk_nonlinear_part_is_fourth_order():
    # The map minus its linearisation is O(amplitude^3) (H_NL ~ p^4, §3.3).
    e = quad(1.1, 0.08, "mk", 1, 1)
    J = _element_jacobian(e, np.zeros(6))
    u = np.array([1.0, 0.3, -0.7, 0.5, 0.0, 0.0])
    wide = Beam(aperture=0.25)          # the largest amplitude leaves X > 0.05 m
    res = []
    for a in [4e-2, 2e-2, 1e-2]:
        z1, _, _, alive = run([e], a * u, beam=wide)
        assert alive == 1
        res.append(np.abs(z1[:4] - J[:4, :4] @ (a * u[:4])).max())
    ratios = np.array(res[:-1]) / np.array(res[1:])
    assert np.all(np.abs(ratios - 8.0) < 0.2), ratios


@pytest.mark.parametrize("method", ["mk", "dkd"])
def test_quad_slice_is_time_reversible(method):
    # A symmetric composition of reversible flows is reversible: with
    # R = diag(1, -1, 1, -1, -1, 1), M(R M(z)) = R z.
    R = np.array([1, -1, 1, -1, -1, 1.0])
    e = quad(1.1, 0.08, method, 4, 1)
    z1, _, _, _ = run([e], Z0 * 5)
    z2, _, _, _ = run([e], R * z1)
    np.testing.assert_allclose(R * z2, Z0 * 5, rtol=0, atol=1e-16)


@pytest.mark.parametrize("method", ["mk", "dkd"])
def test_quad_converges_at_second_order_to_brute_force(method):
    zb, _ = bf.track_element(quad(1.1, 0.08, method, 1, 1), BEAM, Z0, S0)
    errs = []
    for N in [4, 8, 16]:
        z1, _, _, _ = run([quad(1.1, 0.08, method, N, 1)], Z0)
        errs.append(np.abs(z1 - zb).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.3), (errs, ratios)


def test_dkd_quad_linear_part_converges_to_textbook():
    L, k1 = 1.0, 0.05
    k = math.sqrt(k1)
    foc = np.array([[math.cos(k * L), math.sin(k * L) / k], [-k * math.sin(k * L), math.cos(k * L)]])
    e8 = np.abs(_element_jacobian(quad(L, k1, "dkd", 8, 1), np.zeros(6))[:2, :2] - foc).max()
    e16 = np.abs(_element_jacobian(quad(L, k1, "dkd", 16, 1), np.zeros(6))[:2, :2] - foc).max()
    assert 3.8 < e8 / e16 < 4.2


# ------------------------------------------------------------- thin lens ----

@pytest.mark.parametrize("k1l,k2l", [(0.0, 0.5), (0.01, -0.05)])
def test_thin_multipole_kick(k1l, k2l):
    # eq. Amult: V = Re[(b_m/(m Bρ))(X+iY)^m]; kick = -grad V integrated
    z1, _, _, _ = run([thin(k1l=k1l, k2l=k2l)], Z0)
    zb, _ = bf.track_element(thin(k1l=k1l, k2l=k2l), BEAM, Z0, S0)
    np.testing.assert_allclose(z1, zb, rtol=0, atol=1e-18)
    x, y = Z0[0], Z0[2]
    w = complex(x, y)
    V = lambda ww: (k1l / 2 * ww ** 2 + k2l / 6 * ww ** 3).real
    d = 1e-7
    gx = (V(w + d) - V(w - d)) / (2 * d)
    gy = (V(w + 1j * d) - V(w - 1j * d)) / (2 * d)
    assert abs((z1[1] - Z0[1]) + gx) < 1e-15 and abs((z1[3] - Z0[3]) + gy) < 1e-15


def test_snake_is_transparent_to_the_orbit():
    z1, _, _, _ = run([snake(math.pi, 0.3)], Z0)
    np.testing.assert_array_equal(z1, Z0)


# ---------------------------------------------------------- one-turn maps ----

def _symplectic_error(J):
    S = np.kron(np.eye(3), np.array([[0.0, 1.0], [-1.0, 0.0]]))
    return np.abs(J.T @ S @ J - S).max() / max(1.0, np.abs(J).max() ** 2)


@pytest.mark.parametrize("ring", ["small", "rhic"])
def test_one_turn_map_is_symplectic(ring):
    elems = small_ring() if ring == "small" else rhic_like_ring()
    r = oracle.jacobian(elems, BEAM, Z0)
    assert r["lost"] == -1
    assert _symplectic_error(r["J"]) < 1e-12


def test_one_turn_small_ring_matches_brute_force():
    # Bends and drifts are exact; DKD quads converge at second order.
    elems_ref = small_ring()
    zs = [np.array([2e-3, -1e-4, 1e-3, 1e-4, 0.0, 5e-4]),
          np.array([-1e-3, 5e-5, -2e-3, 0.0, 0.0, -1e-3])]
    for z0 in zs:
        zb, _ = bf.track_line(elems_ref, BEAM, z0, S0)
        errs = []
        for N in [8, 16]:
            z1, _, _, _ = run(small_ring(quad_slices=N), z0)
            errs.append(np.abs(z1 - zb)[:4].max())
        assert 3.5 < errs[0] / errs[1] < 4.5, errs


# ----------------------------------------------------------------- losses ----

def test_loss_is_flagged_at_the_element_and_frozen_at_its_entrance():
    beam = Beam(aperture=0.01)
    elems = [drift(1.0), quad(1.0, -0.5, "mk", 4, 1), drift(5.0), drift(1.0)]
    z0 = np.array([4e-3, 1e-3, 0, 0, 0, 0])
    zin, _, _, _ = run(elems[:2], z0, beam=beam)                   # entrance of element 2
    z1, s1, _, alive = run(elems, z0, beam=beam, turns=3)
    assert alive == -(1 + 2)
    np.testing.assert_array_equal(z1, zin)


def test_non_finite_radicand_is_a_loss():
    z0 = np.array([0, 0.9999, 0, 0.5, 0, 0])                         # Px² + Py² > P²
    _, _, _, alive = run([drift(1.0)], z0)
    assert alive == -1

"""Pins of the oracle's spin integration (§2.2, §4) against textbook special
cases of the T-BMT equation, closed forms, the Romberg error orders, a
brute-force ODE integration, and the behaviours the paper prints for its
single-element examples (§5.2)."""

import json
import math
import os

import numpy as np
import pytest

import bruteforce as bf
import oracle
from workloads import Beam, rhic_like_ring, small_ring, uniform_bend_ring
from workloads.bunch import random_spins
from workloads.lattice import quad, sbend, thin

BEAM = Beam()
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_elements.json")))


def run(elems, z, s, beam=BEAM, **kw):
    r = oracle.track(elems, beam, np.asarray(z, float)[:, None], np.asarray(s, float)[:, None],
                     want_quaternion=True, **kw)
    return r["z"][:, 0], r["spin"][:, 0], r["q"][:, 0], r["alive"][0]


def rotate(q, S):
    w, v = q[0], np.asarray(q[1:])
    t = 2 * np.cross(v, S)
    return S + w * t + np.cross(v, t)


def particle_gamma(Pt, beam=BEAM):
    return beam.gamma0 * (1 + beam.beta0 * Pt)


# ------------------------------------------------------ Ω special cases ----

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_omega_splits_into_textbook_longitudinal_and_transverse_rates(seed):
    # In the lab frame the T-BMT precession about the part of B along the
    # velocity goes with (1 + G) and about the transverse part with (1 + Gγ).
    # In s the rate carries ds/dt = v_s/(1 + hX) -> the factor (1 + hX)/Ps.
    rng = np.random.default_rng(seed)
    z = np.array([1e-2, 3e-3, -2e-2, 2e-3, 0.0, 2e-3]) * rng.uniform(-1, 1, 6)
    b = rng.normal(size=3)
    h = 0.0
    om = oracle.omega(z, h, b, BEAM)
    b0 = BEAM.beta0
    Pt = z[5]
    P = math.sqrt(1 + 2 * Pt / b0 + Pt * Pt)
    Ps = math.sqrt(P * P - z[1] ** 2 - z[3] ** 2)
    u = np.array([z[1], z[3], Ps]) / P
    g = particle_gamma(Pt)
    b_par = (u @ b) * u
    b_perp = b - b_par
    expect = -(1 + h * z[0]) / Ps * ((1 + BEAM.G) * b_par + (1 + BEAM.G * g) * b_perp)
    np.testing.assert_allclose(om, expect, rtol=1e-14, atol=1e-16)


def test_omega_on_the_design_orbit_of_a_dipole():
    h = 0.02
    om = oracle.omega(np.zeros(6), h, np.array([0.0, h, 0.0]), BEAM)
    np.testing.assert_allclose(om, [0.0, -BEAM.G * BEAM.gamma0 * h, 0.0], rtol=1e-15, atol=1e-20)


def test_omega_midplane_is_vertical_and_quad_axis_is_zero():
    z = np.array([3e-3, 2e-4, 0.0, 0.0, 0.1, 1e-3])
    om = oracle.omega(z, 0.0, np.array([0.0, 0.05 * z[0], 0.0]), BEAM)       # quad, Y = 0
    assert om[0] == 0.0 and om[2] == 0.0 and om[1] != 0.0
    om = oracle.omega(np.array([0, 1e-4, 0, -1e-4, 0, 1e-3]), 0.0, np.zeros(3), BEAM)
    np.testing.assert_array_equal(om, 0.0)


# ------------------------------------------------------------ spin tune ----

def test_spin_tune_in_a_ring_of_bends_is_G_gamma():
    ring = uniform_bend_ring(16, 5.0, 8, 3)
    _, _, q, _ = run(ring, np.zeros(6), [0.0, 1.0, 0.0])
    a = math.pi * BEAM.G * BEAM.gamma0
    np.testing.assert_allclose(q, [math.cos(a), 0.0, -math.sin(a), 0.0], atol=2e-14)


def test_spin_precesses_with_the_momentum_G_gamma_times_faster():
    # Relative to the curvilinear frame a longitudinal spin turns by Gγθ in
    # the sense the momentum turns (towards -x for h > 0).
    th = 0.05
    _, s1, _, _ = run([sbend(2.0, th, 8, 3)], np.zeros(6), [0.0, 0.0, 1.0])
    a = BEAM.G * BEAM.gamma0 * th
    np.testing.assert_allclose(s1, [-math.sin(a), 0.0, math.cos(a)], atol=1e-14)


@pytest.mark.parametrize("X,Px,Pt", [(3e-3, 2e-4, 0.0), (-1e-2, -5e-4, 1e-3), (2e-2, 1e-3, -2e-3)])
def test_midplane_bend_spin_angle_closed_form(X, Px, Pt):
    # With Y = Py = 0 all Ω are vertical; integrating Ω_y along the exact
    # orbit gives  -Gγ h L - (1 + Gγ)[asin(Px_in/Pα) - asin(Px_out/Pα)].
    L, th = 10.0, 2 * math.pi / 32
    h = th / L
    z0 = np.array([X, Px, 0.0, 0.0, 0.0, Pt])
    z1, _, q, _ = run([sbend(L, th, 64, 4)], z0, [0.0, 1.0, 0.0])
    b0 = BEAM.beta0
    Pa = math.sqrt(1 + 2 * Pt / b0 + Pt * Pt)
    g = particle_gamma(Pt)
    D = math.asin(Px / Pa) - math.asin(z1[1] / Pa)
    phi = -BEAM.G * g * h * L - (1 + BEAM.G * g) * D
    assert abs(q[1]) < 1e-15 and abs(q[3]) < 1e-15
    got = 2 * math.atan2(q[2], q[0])
    assert abs(math.remainder(got - phi, 2 * math.pi)) < 1e-12


# ----------------------------------------------------------- snake rings ----

def test_small_ring_design_orbit_quaternion_and_flip():
    a = math.pi * BEAM.G * BEAM.gamma0
    _, s1, q, _ = run(small_ring(), np.zeros(6), [0.0, 1.0, 0.0], turns=3)
    np.testing.assert_allclose(q, [0.0, math.sin(a), 0.0, math.cos(a)], atol=2e-14)
    np.testing.assert_allclose(s1, [0.0, -1.0, 0.0], atol=1e-13)       # odd turns flip S_y


def test_two_snakes_at_plus_minus_45_degrees_give_spin_tune_one_half():
    expect = GOLDEN["rhic_snakes"]["spin_tune"]
    _, s1, q, _ = run(rhic_like_ring(), np.zeros(6), [0.0, 1.0, 0.0], turns=2)
    tune = 2 * math.acos(min(1.0, abs(q[0]))) / (2 * math.pi)
    assert abs(tune - expect) < 1e-14
    np.testing.assert_allclose(np.abs(q), [0.0, 0.0, 1.0, 0.0], atol=1e-14)   # ±j: about ŷ
    np.testing.assert_allclose(s1, [0.0, 1.0, 0.0], atol=1e-13)


# ------------------------------------------------------------- Romberg ----

def _rotating_field_errors(R, Ns, L=1.0, eps=0.7, b=2.3, c=1.1):
    S0 = np.array([0.1952, 0.9759, 0.0976])
    S0 = S0 / np.linalg.norm(S0)
    # Ω(s) = (ε cos bs, ε sin bs, c): in the frame rotating with b about ẑ the
    # field is constant, so S(s) = R_z(bs) exp(s[(ε, 0, c - b)]×) S0.
    w = np.array([eps, 0.0, c - b])
    th, n = np.linalg.norm(w) * L, w / np.linalg.norm(w)
    S = S0 * math.cos(th) + np.cross(n, S0) * math.sin(th) + n * (n @ S0) * (1 - math.cos(th))
    cz, sz = math.cos(b * L), math.sin(b * L)
    exact = np.array([cz * S[0] - sz * S[1], sz * S[0] + cz * S[1], S[2]])
    errs = []
    for N in Ns:
        s = np.linspace(0.0, L, N + 1)
        om = np.stack([eps * np.cos(b * s), eps * np.sin(b * s), c * np.ones_like(s)], 1)
        q = oracle.romberg(om, L / N, R)
        errs.append(np.abs(rotate(q, S0) - exact).max())
    return np.array(errs)


@pytest.mark.parametrize("R,order", [(1, 2), (2, 4), (3, 6), (4, 8)])
def test_romberg_error_order_is_2R(R, order):
    Ns = [8, 16, 32, 64] if R < 4 else [8, 16, 32]
    errs = _rotating_field_errors(R, Ns)
    slopes = np.log2(errs[:-1] / errs[1:])
    assert np.all(np.abs(slopes - order) < 0.15), slopes


def test_romberg_rows_limited_by_the_power_of_two_in_N():
    # N = 12 = 4·3 and N = 20 = 4·5 support three rows; N = 6 supports two.
    e12 = _rotating_field_errors(4, [12, 20])
    e12_3 = _rotating_field_errors(3, [12, 20])
    np.testing.assert_allclose(e12, e12_3, rtol=0, atol=1e-17)
    e6 = _rotating_field_errors(4, [6])
    e6_2 = _rotating_field_errors(2, [6])
    np.testing.assert_allclose(e6, e6_2, rtol=0, atol=1e-17)


def test_element_quaternions_are_normalised_and_spin_norm_is_kept():
    for e in [sbend(10.0, 2 * math.pi / 32, 8, 3), quad(1.1, 0.08, "mk", 4, 4), thin(k2l=0.5)]:
        _, _, q, _ = run([e], np.array([1e-3, 1e-4, 2e-3, -2e-4, 0.0, 1e-3]), [0.0, 1.0, 0.0])
        assert abs(np.linalg.norm(q) - 1.0) < 1e-15
    r = oracle.track(small_ring(), BEAM, np.array([[1e-3, 2e-3], [1e-4, 0], [2e-3, -1e-3],
                                                   [-1e-4, 1e-4], [0, 0], [1e-3, -1e-3]]),
                     random_spins(2, 7, math.pi), turns=256)
    assert np.abs(np.linalg.norm(r["spin"], axis=0) - 1).max() < 1e-13


# -------------------------------------------------------- brute force ----

Z0 = np.array([1e-3, 1e-4, 2e-3, -2e-4, 0.0, 1e-3])
SPIN = np.array([0.1952, 0.9759, 0.0976]) / np.linalg.norm([0.1952, 0.9759, 0.0976])


@pytest.mark.parametrize("kind", ["sbend", "mk"])
def test_spin_converges_to_brute_force_with_romberg_orders(kind):
    def elem(N, R):
        return sbend(10.0, 2 * math.pi / 32, N, R) if kind == "sbend" else quad(1.1, 0.08, "mk", N, R)
    _, sb = bf.track_element(elem(1, 1), BEAM, Z0, SPIN)
    e1 = [np.abs(run([elem(N, 1)], Z0, SPIN)[1] - sb).max() for N in [8, 16, 32]]
    e2 = [np.abs(run([elem(N, 2)], Z0, SPIN)[1] - sb).max() for N in [4, 8, 16]]
    s1 = np.log2(np.array(e1[:-1]) / np.array(e1[1:]))
    s2 = np.log2(np.array(e2[:-1]) / np.array(e2[1:]))
    assert np.all(np.abs(s1 - 2) < 0.1), s1
    assert np.all(s2 > 3.6), s2
    assert np.abs(run([elem(16, 4)], Z0, SPIN)[1] - sb).max() < 1e-11


def test_thin_multipole_spin_is_a_symmetric_approximation_of_the_kick_flow():
    # The half-kick / rotation / half-kick step is second order: its local
    # error against the exact kick flow is third order in the lens strength.
    z = np.array([2e-2, 1e-3, -1e-2, 2e-3, 0.0, 1e-3])
    errs = []
    for f in [1.0, 0.5, 0.25]:
        e = thin(k1l=0.02 * f, k2l=-0.5 * f)
        _, sb = bf.track_element(e, BEAM, z, SPIN)
        errs.append(np.abs(run([e], z, SPIN)[1] - sb).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 8.0) < 0.5), ratios
    assert errs[0] < 1e-10


def test_one_turn_spin_of_the_small_ring_converges_to_brute_force():
    z0 = np.array([2e-3, -1e-4, 1e-3, 1e-4, 0.0, 5e-4])
    _, sb = bf.track_line(small_ring(), BEAM, z0, SPIN)
    errs = [np.abs(run(small_ring(quad_slices=N, bend_slices=N), z0, SPIN)[1] - sb).max()
            for N in [8, 16]]
    assert 3.0 < errs[0] / errs[1] < 5.0, errs           # limited by the DKD orbit, 2nd order
    assert errs[1] < 1e-4


# ---------------------------------------------- the paper's element examples ----

def _paper_setup():
    p = GOLDEN["proton"]
    gamma0 = p["total_energy_GeV"] / p["mass_GeV"]
    beam = Beam(G=p["G"], gamma0=gamma0)
    mom = math.sqrt(p["total_energy_GeV"] ** 2 - p["mass_GeV"] ** 2)
    brho = mom / 0.299792458
    fp = GOLDEN["footnote_particle"]
    b0 = beam.beta0
    Pt = math.sqrt((1 + fp["delta"]) ** 2 + 1 / (b0 * gamma0) ** 2) - 1 / b0
    z0 = np.array([fp["X"], fp["Px"], fp["Y"], fp["Py"], fp["T"], Pt])
    s0 = np.array(fp["spin"]) / np.linalg.norm(fp["spin"])
    return beam, brho, z0, s0


def test_paper_arc_dipole_pwc_slope_minus_two_and_one_romberg_step_slope_minus_four():
    beam, brho, z0, s0 = _paper_setup()
    d = GOLDEN["rhic_arc_dipole"]
    ang = math.radians(d["angle_deg"])
    assert abs(ang / d["L"] * brho - d["field_T_approx"]) < 0.02 * d["field_T_approx"]
    _, sb = bf.track_element(sbend(d["L"], ang, 1, 1), beam, z0, s0)
    pwc = [np.abs(run([sbend(d["L"], ang, N, 1)], z0, s0, beam=beam)[1] - sb).max() for N in [8, 16, 32, 64]]
    k1 = [np.abs(run([sbend(d["L"], ang, N, 2)], z0, s0, beam=beam)[1] - sb).max() for N in [8, 32]]
    slope_pwc = np.polyfit(np.log2([8, 16, 32, 64]), np.log2(pwc), 1)[0]
    slope_k1 = (np.log2(k1[1]) - np.log2(k1[0])) / 2
    assert abs(slope_pwc - GOLDEN["printed_behaviour"]["pwc_slope"]) < 0.05
    assert abs(slope_k1 - GOLDEN["printed_behaviour"]["dipole_k1_slope_between_8_and_64_slices"]) < 0.7


def test_paper_ir_quad_four_slices_two_romberg_steps_gain_four_decades():
    beam, brho, z0, s0 = _paper_setup()
    qd = GOLDEN["rhic_ir_quad"]
    k1 = qd["b2_T_per_m"] / brho
    _, sb = bf.track_element(quad(qd["L"], k1, "mk", 1, 1), beam, z0, s0)
    pwc4 = np.abs(run([quad(qd["L"], k1, "mk", 4, 1)], z0, s0, beam=beam)[1] - sb).max()
    rom4 = np.abs(run([quad(qd["L"], k1, "mk", 4, 3)], z0, s0, beam=beam)[1] - sb).max()
    decades = math.log10(pwc4 / rom4)
    assert abs(decades - GOLDEN["printed_behaviour"]["quad_4_slices_2_romberg_error_reduction_decades"]) < 0.5
    # ... to the level of some four hundred PWC slices
    pwc256 = np.abs(run([quad(qd["L"], k1, "mk", 256, 1)], z0, s0, beam=beam)[1] - sb).max()
    pwc512 = np.abs(run([quad(qd["L"], k1, "mk", 512, 1)], z0, s0, beam=beam)[1] - sb).max()
    assert pwc512 < rom4 < pwc256


def test_quaternion_derivatives_at_the_design_orbit_match_differences_of_tracked_values():
    # Forward-mode dQ of the one-turn quaternion at the design orbit, where the
    # quadrupoles rotate the spin by exactly zero, against central differences
    # of tracked quaternions (values only, extended precision).
    from workloads.lattice import drift as _drift
    ring = small_ring()
    jac = oracle.jacobian(ring, BEAM, np.zeros(6))
    h = 1e-9
    fd = np.zeros((4, 6))
    for i in range(6):
        z = np.zeros((6, 2))
        z[i, 0], z[i, 1] = h, -h
        s = np.zeros((3, 2))
        s[1] = 1.0
        q = oracle.track(ring, BEAM, z, s, turns=1, want_quaternion=True)["q"]
        fd[:, i] = (q[:, 0] - q[:, 1]) / (2 * h)
    assert np.abs(fd).max() > 1.0                      # the quadrupoles' share is not small
    assert np.abs(jac["dQ"] - fd).max() <= 1e-6 * np.abs(fd).max()
    # a ring of drifts and quadrupoles alone: Ω = 0 on the design orbit, so
    # every spin derivative there comes from the zero-angle quaternions
    straight = [quad(1.0, 0.05, "mk", 4, 3), _drift(2.0), quad(1.0, -0.05, "mk", 4, 3), _drift(2.0)]
    j2 = oracle.jacobian(straight, BEAM, np.zeros(6))
    fd2 = np.zeros((4, 6))
    for i in range(6):
        z = np.zeros((6, 2))
        z[i, 0], z[i, 1] = h, -h
        s = np.zeros((3, 2))
        s[1] = 1.0
        q = oracle.track(straight, BEAM, z, s, turns=1, want_quaternion=True)["q"]
        fd2[:, i] = (q[:, 0] - q[:, 1]) / (2 * h)
    assert np.abs(fd2).max() > 1e-2
    assert np.abs(j2["dQ"] - fd2).max() <= 1e-6 * np.abs(fd2).max()

"""Pins of the oracle's solenoid (§3.7 eq. solenoid, eq. mgVSol; the
thin-pancake fringe spin kick of §4.4 eq. solFringe): brute-force
integration of the solenoid Hamiltonian with the Lorentz-force spin
equation, through a body alone and through finite linear-ramp fringes whose
length goes to zero; the textbook spin rotation on the axis; the exact
flow's group property; the Romberg orders of the body spin."""

import math

import numpy as np
import pytest

import bruteforce as bf
import oracle
from workloads import Beam
from workloads.lattice import solenoid

BEAM = Beam()
Z0 = np.array([2e-3, 3e-4, -1e-3, 2e-4, 0.01, 1e-3])
S0 = np.array([0.1952, 0.9759, 0.0976]) / np.linalg.norm([0.1952, 0.9759, 0.0976])
# 2.1 m at 1.3 T for the γ0 = 25 protons: ks = b0/(Bρ)0
BRHO = BEAM.beta0 * BEAM.gamma0 * 0.938272 / 0.299792458
KS = 1.3 / BRHO
L = 2.1


def run(elems, z=Z0, s=S0):
    r = oracle.track(elems, BEAM, np.asarray(z, float)[:, None], np.asarray(s, float)[:, None],
                     want_quaternion=True)
    assert r["alive"][0] == 1
    return r["z"][:, 0], r["spin"][:, 0], r["q"][:, 0]


def test_body_map_is_the_flow_of_the_solenoid_hamiltonian():
    # the fringes leave the orbit unchanged, so the element's orbit is the body flow
    zb, _ = bf.track_solenoid(L, KS, 0.0, BEAM, Z0, S0)
    z, _, _ = run([solenoid(L, KS, 4, 1)])
    np.testing.assert_allclose(z, zb, rtol=0, atol=3e-15)


def test_thin_fringe_model_is_the_limit_of_short_linear_fringes():
    z, s, _ = run([solenoid(L, KS, 16, 4)])
    dz, ds = [], []
    for eps in (4e-3, 2e-3, 1e-3):
        zb, sb = bf.track_solenoid(L, KS, eps, BEAM, Z0, S0)
        dz.append(np.abs(zb - z).max())
        ds.append(np.abs(sb - s).max())
    # both differences vanish linearly with the fringe length
    assert np.all(np.abs(np.array(dz[:-1]) / np.array(dz[1:]) - 2.0) < 0.1), dz
    assert np.all(np.abs(np.array(ds[:-1]) / np.array(ds[1:]) - 2.0) < 0.1), ds
    assert ds[-1] < 1e-6


def test_fringe_kick_is_what_the_short_fringes_do_to_the_spin():
    # the fringes' radial field turns an off-axis spin by far more than the
    # remaining error of the thin model
    _, s_full, _ = run([solenoid(L, KS, 16, 4)])
    _, s_fringes = bf.track_solenoid(L, KS, 1e-3, BEAM, Z0, S0)
    _, s_body = bf.track_solenoid(L, KS, 0.0, BEAM, Z0, S0)
    effect = np.abs(s_fringes - s_body).max()
    assert effect > 1e-4
    assert np.abs(s_full - s_fringes).max() < 0.05 * effect


def test_on_axis_spin_turns_about_s_by_one_plus_G_times_the_field_integral():
    z = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    _, _, q = run([solenoid(L, KS, 1, 1)], z=z)
    P = 1.0
    angle = (1.0 + BEAM.G) * KS * L / P
    # rotation by -angle about +s (Ω = -(1 + G) ks ŝ / P for a particle on axis)
    np.testing.assert_allclose(q, [math.cos(angle / 2), 0.0, 0.0, -math.sin(angle / 2)],
                               rtol=0, atol=1e-15)


def test_two_halves_are_one_solenoid():
    # the exit kick of the first half and the entrance kick of the second are
    # opposite rotations at the same state
    a = run([solenoid(L / 2, KS, 8, 4), solenoid(L / 2, KS, 8, 4)])
    b = run([solenoid(L, KS, 16, 4)])
    np.testing.assert_allclose(a[0], b[0], rtol=0, atol=1e-16)
    np.testing.assert_allclose(a[1], b[1], rtol=0, atol=1e-14)


@pytest.mark.parametrize("R,order", [(1, 2), (2, 4), (3, 6)])
def test_body_spin_romberg_order_is_2R(R, order):
    # a strong field so that the slice error is far above round-off
    ks = 40 * KS
    ref = run([solenoid(L, ks, 256, 4)])[1]
    Ns = [4, 8, 16] if R < 3 else [8, 16, 32]
    errs = [np.abs(run([solenoid(L, ks, N, R)])[1] - ref).max() for N in Ns]
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - order) < 0.35), (errs, slopes)


def test_midpoint_body_spin_is_second_order():
    ks = 40 * KS
    ref = run([solenoid(L, ks, 256, 4)])[1]
    errs = [np.abs(run([solenoid(L, ks, N, 1, spin="midpoint")])[1] - ref).max() for N in (4, 8, 16)]
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.3), (errs, ratios)


def test_paper_solenoid_at_200_GeV_four_slices_and_romberg_reach_round_off():
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_elements.json")))
    p, sol = g["proton"], g["solenoid"]
    gamma0 = p["total_energy_GeV"] / p["mass_GeV"]
    beam = Beam(G=p["G"], gamma0=gamma0)
    brho = math.sqrt(p["total_energy_GeV"] ** 2 - p["mass_GeV"] ** 2) / 0.299792458
    ks = sol["field_T"] / brho
    fp = g["footnote_particle"]
    b0 = beam.beta0
    Pt = math.sqrt((1 + fp["delta"]) ** 2 + 1 / (b0 * gamma0) ** 2) - 1 / b0
    z0 = np.array([fp["X"], fp["Px"], fp["Y"], fp["Py"], fp["T"], Pt])
    s0 = np.array(fp["spin"]) / np.linalg.norm(fp["spin"])

    def spin(N, R):
        r = oracle.track([solenoid(sol["L"], ks, N, R)], beam, z0[:, None], s0[:, None])
        return r["spin"][:, 0]
    ref = spin(128, 4)
    # the on-axis rotation (1 + G) ks L is of the printed order (about 10 mrad)
    rot = (1 + p["G"]) * ks * sol["L"]
    assert 0.5 * sol["rotation_200GeV_rad_order"] < rot < 2 * sol["rotation_200GeV_rad_order"]
    # plain trapezoid products at four slices are far from round-off, one or
    # two Romberg steps reach it
    assert np.abs(spin(4, 1) - ref).max() > 1e-12
    assert np.abs(spin(4, 2) - ref).max() < 1e-15
    assert np.abs(spin(4, 3) - ref).max() < 1e-15

"""Pins of the oracle's rectangular bend (§3.2: body eq. rbend, thin dipole
fringe eq. dipolefringe, dynamic rotations eq. prot, the offsets eq. Xoffset
and eq. Toffset of a magnet whose faces are not symmetric about the design
orbit) and of its fringe spin kicks (§4.5 eq. skfringe, eq. skfringeRB): the
flow of the rotation Hamiltonian, brute-force Lorentz tracking through linear
fringes whose length goes to zero, the design orbit and its spin rotation
(that of a sector bend of the same angle), the textbook edge focusing of a
rectangular magnet, and the Romberg orders of the body spin."""

import math

import numpy as np
import pytest

import bruteforce as bf
import oracle
from workloads import Beam
from workloads.lattice import rbend, sbend

BEAM = Beam()
Z0 = np.array([2e-3, 3e-4, -1.5e-3, 2e-4, 0.01, 1e-3])
S0 = np.array([0.1952, 0.9759, 0.0976]) / np.linalg.norm([0.1952, 0.9759, 0.0976])
L, ANG = 3.0, 0.12


def run(elems, z=Z0, s=S0, beam=BEAM):
    r = oracle.track(elems, beam, np.asarray(z, float)[:, None], np.asarray(s, float)[:, None],
                     want_quaternion=True)
    assert r["alive"][0] == 1
    return r["z"][:, 0], r["spin"][:, 0], r["q"][:, 0]


def faces(asym):
    """Entrance and exit angles of the design orbit, and the radius of its
    circle in the magnet: L = ρ (sin φ^entr - sin φ^exit)."""
    phe, phx = ANG / 2 + asym, asym - ANG / 2
    return phe, phx, L / (math.sin(phe) - math.sin(phx))


@pytest.mark.parametrize("asym", [0.0, 0.03, -0.05])
def test_design_particle_keeps_its_orbit_and_turns_like_in_a_sector_bend(asym):
    # With faces turned from the symmetric placement the design orbit still
    # enters and leaves on the reference (the horizontal offset of eq.
    # Xoffset), its flight time is that of the arc (eq. Toffset), and its spin
    # turns as in a sector bend of the same angle along the same arc.
    z0 = np.zeros(6)
    z, _, q = run([rbend(L, ANG, 64, 4, asym=asym)], z=z0)
    np.testing.assert_allclose(z, 0.0, atol=2e-15)
    _, _, rho = faces(asym)
    _, _, qs = run([sbend(rho * ANG, ANG, 8, 4)], z=z0)
    np.testing.assert_allclose(q, qs, rtol=0, atol=1e-14)


@pytest.mark.parametrize("asym", [0.0, 0.03, -0.05])
def test_linear_optics_is_the_sector_bend_with_edge_focusing(asym):
    # hard-edge rectangular magnet = sector bend between edges at the angles
    # of the orbit to the faces, e1 = φ^entr and e2 = -φ^exit (θ/2 each in the
    # symmetric magnet): Px += X tan(e)/ρ, Py -= Y tan(e)/ρ (transverse 4×4
    # block at Pt = 0)
    phe, phx, rho = faces(asym)
    Jr = oracle.jacobian([rbend(L, ANG, 8, 1, asym=asym)], BEAM, np.zeros(6))["J"]
    Js = oracle.jacobian([sbend(rho * ANG, ANG, 8, 1)], BEAM, np.zeros(6))["J"]

    def edge(e):
        E = np.eye(6)
        E[1, 0] = math.tan(e) / rho
        E[3, 2] = -math.tan(e) / rho
        return E
    M = edge(-phx) @ Js @ edge(phe)
    idx = np.ix_([0, 1, 2, 3], [0, 1, 2, 3])
    np.testing.assert_allclose(Jr[idx], M[idx], rtol=0, atol=1e-12)


def test_frame_rotation_is_the_flow_of_its_hamiltonian():
    for phi in (0.06, -0.3):
        np.testing.assert_allclose(oracle.rotate(Z0, phi, BEAM), bf.track_prot(phi, BEAM, Z0),
                                   rtol=0, atol=2e-15)
    # group property of the flow
    np.testing.assert_allclose(oracle.rotate(oracle.rotate(Z0, 0.04, BEAM), 0.03, BEAM),
                               oracle.rotate(Z0, 0.07, BEAM), rtol=0, atol=1e-16)


@pytest.mark.parametrize("asym", [0.0, 0.03])
def test_thin_fringe_orbit_is_the_limit_of_short_linear_fringes(asym):
    # X, Y and T converge linearly in the fringe length; the momenta agree to
    # the higher orders that the thin map and the lowest-order vector
    # potential of the brute force treat differently
    z, _, _ = run([rbend(L, ANG, 16, 4, asym=asym)])
    d = []
    for eps in (4e-3, 2e-3, 1e-3):
        zb, _ = bf.track_rbend(L, ANG, 1.0, eps, BEAM, Z0, S0, asym=asym)
        d.append(np.abs(zb - z))
    d = np.array(d)
    for c in (0, 2, 4):
        r = d[:-1, c] / d[1:, c]
        assert np.all(np.abs(r - 2.0) < 0.15), (c, d[:, c])
    phe, _, rho = faces(asym)
    kick_py = math.tan(phe) / rho * abs(Z0[2])          # the entrance edge focusing kick
    assert d[-1, 3] < 2e-3 * kick_py and d[-1, 1] < 1e-12


def test_fringe_spin_kick_is_right_to_first_order_in_the_entry_slope():
    # The printed kick is the lowest order of the thin-fringe limit; what it
    # leaves out is second order in the slope Px ≈ θ/2 at the face (and first
    # order in Y), so the residual against the brute force falls 4x when the
    # bend angle halves while the kick itself only halves.
    res, kick = [], []
    for ang in (0.12, 0.06):
        _, s, _ = run([rbend(L, ang, 16, 4)])
        _, sb = bf.track_rbend(L, ang, 1.0, 1e-4, BEAM, Z0, S0)
        res.append(np.abs(s - sb).max())
        gamma = BEAM.gamma0 * (1 + BEAM.beta0 * Z0[5])
        kick.append(2 * math.sin(ang / 2) / L * abs(Z0[2]) * BEAM.G * (gamma - 1) * math.sin(ang / 2))
    assert 3.3 < res[0] / res[1] < 4.7, res
    assert res[0] < 0.1 * kick[0], (res, kick)


@pytest.mark.parametrize("R,order", [(1, 2), (2, 4)])
def test_body_spin_romberg_order(R, order):
    ref = run([rbend(L, ANG, 512, 4)])[1]
    errs = [np.abs(run([rbend(L, ANG, N, R)])[1] - ref).max() for N in (8, 16, 32)]
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - order) < 0.35), (errs, slopes)


def test_fringe_spin_kick_of_a_turned_face_stays_below_a_tenth_of_its_size():
    # with the faces turned by 0.03 the entry slope grows from sin(0.06) to
    # sin(0.09): the thin-fringe spin kick still matches the brute force to
    # well within the kick's own size
    asym = 0.03
    phe, _, rho = faces(asym)
    _, s, _ = run([rbend(L, ANG, 16, 4, asym=asym)])
    _, sb = bf.track_rbend(L, ANG, 1.0, 1e-4, BEAM, Z0, S0, asym=asym)
    gamma = BEAM.gamma0 * (1 + BEAM.beta0 * Z0[5])
    kick = abs(Z0[2]) / rho * BEAM.G * (gamma - 1) * math.sin(phe)
    assert np.abs(s - sb).max() < 0.1 * kick

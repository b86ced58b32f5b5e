"""Parity of the HIP FP64 path with the CPU oracle, element by element,
through the C ABI.

Tolerance (stated for the double-precision method): orbit
|Δz_i| <= 1e-12 · max(|z_i|, σ_i) with σ_i the bunch RMS of coordinate i,
spin components |ΔS_c| <= 1e-10.  The oracle runs in x87 extended precision.

The orbit bound binds after one turn.  Over t turns FP64 round-off is
amplified by the ring itself (a one-ulp change of the input grows to 4e-13
of the RMS in one turn of the RHIC-scale ring), so multi-turn runs are held
to 1e-12 · t and to a tenth of the divergence of a plain double-precision
evaluation of the printed maps (the oracle's double instantiation).
"""

import math

import numpy as np
import pytest

import oracle
from workloads import Beam, gaussian_bunch, rhic_like_ring, small_ring
from workloads.bunch import random_spins
from workloads.lattice import drift, quad, sbend, snake, thin

pytestmark = pytest.mark.gpu

BEAM = Beam()
ORBIT_TOL = 1e-12
SPIN_TOL = 1e-10


def gpu_run(elements, beam, z, s, alive=None, turns=1, report_every=0, want_q=False):
    import torch
    from paper_1501_03450_amd import SpinTracker
    tr = SpinTracker(elements, beam, report_every=report_every)
    tr.set_particles(z, s, alive)
    q = tr.enable_quaternions() if want_q else None
    tr.track(turns)
    torch.cuda.synchronize()
    zz, ss, aa = tr.read()
    pol = tr.polarization().cpu().numpy()
    qq = q.cpu().numpy() if q is not None else None
    tr.close()
    return {"z": zz, "spin": ss, "alive": aa, "pol": pol, "q": qq}


def orbit_rel_err(g, o):
    live = o["alive"] == 1
    if not live.any():
        return 0.0, None
    zo, zg = o["z"][:, live], g["z"][:, live]
    sig = np.sqrt(np.mean(zo ** 2, axis=1) - np.mean(zo, axis=1) ** 2) if zo.shape[1] > 1 else np.abs(zo[:, 0])
    scale = np.maximum(np.abs(zo), np.maximum(sig, 1e-300)[:, None])
    rel = np.abs(zg - zo) / scale
    return rel.max(), np.unravel_index(np.argmax(rel), rel.shape)


def assert_parity(g, o, label="", orbit_tol=ORBIT_TOL):
    np.testing.assert_array_equal(g["alive"], o["alive"], err_msg=label)
    err, worst = orbit_rel_err(g, o)
    assert err <= orbit_tol, f"{label} orbit rel err {err:.3e} at coord {worst}"
    ds = np.abs(g["spin"] - o["spin"]).max() if g["spin"].size else 0.0
    assert ds <= SPIN_TOL, f"{label} spin err {ds:.3e}"


def assert_multiturn_parity(g, o, elements, beam, z, s, a, turns, label):
    """1e-12 · turns, and no more than a tenth of plain-FP64 divergence."""
    od = oracle.track(elements, beam, z, s, a, turns=turns, extended=False)
    plain, _ = orbit_rel_err(od, o)
    err, worst = orbit_rel_err(g, o)
    print(f"{label}: GPU orbit rel err {err:.3e}, plain FP64 {plain:.3e}")
    assert_parity(g, o, label, orbit_tol=ORBIT_TOL * turns)
    assert err <= 0.1 * plain, f"{label}: {err:.3e} vs plain FP64 {plain:.3e}"


def both(elements, beam, z, s, alive=None, turns=1, report_every=0, want_q=False):
    g = gpu_run(elements, beam, z, s, alive, turns, report_every, want_q)
    o = oracle.track(elements, beam, z, s, alive, turns=turns, report_every=report_every,
                     want_quaternion=want_q)
    return g, o


# ------------------------------------------------------------ elements ----

ELEMENTS = {
    "drift": [drift(2.0)],
    "sbend_R3_N8": [sbend(10.0, 2 * math.pi / 32, 8, 3)],
    "sbend_R4_N8": [sbend(9.45, 2 * math.pi / 264, 8, 4)],
    "sbend_R1_N5": [sbend(10.0, 0.2, 5, 1)],
    "sbend_eta": [sbend(10.0, 2 * math.pi / 32, 12, 4, eta=1.003)],
    "quad_mk_f": [quad(1.1, 0.08, "mk", 4, 4)],
    "quad_mk_d": [quad(1.1, -0.08, "mk", 6, 2)],
    "quad_dkd_f": [quad(1.0, 0.05, "dkd", 8, 3)],
    "quad_dkd_d": [quad(1.0, -0.05, "dkd", 3, 1)],
    # beyond the series ranges: the halving fallbacks for the quaternion
    # half angle (|Ω| ds ≈ 13 rad), asin (η = 1.2, 0.3 rad per step) and the
    # MK phase (κ ds/2 ≈ 0.39)
    "sbend_strong_mispowered": [sbend(2.0, 0.6, 2, 2, eta=1.2)],
    "quad_mk_strong": [quad(1.1, 2.0, "mk", 2, 2)],
    "quad_mk_strong_d": [quad(1.1, -2.0, "mk", 2, 2)],
    "thin": [thin(k1l=0.01, k2l=-0.5)],
    "snake": [snake(math.pi, math.pi / 4)],
}


@pytest.mark.parametrize("name", sorted(ELEMENTS))
def test_single_element_parity(name):
    z, _, _ = gaussian_bunch(300, 11, BEAM, scale=3.0)
    s = random_spins(300, 12, math.pi)
    g, o = both(ELEMENTS[name], BEAM, z, s, want_q=True)
    assert_parity(g, o, name)
    assert np.abs(g["q"] - o["q"]).max() <= SPIN_TOL


# ---------------------------------------------------------------- rings ----

def test_small_ring_full_configuration():
    # 1024 protons, 16 FODO cells + snake, DKD quads N=8, bends N=8, R=3
    z, s, a = gaussian_bunch(1024, 1501034500, BEAM)
    g, o = both(small_ring(), BEAM, z, s, a, turns=1)
    assert_parity(g, o, "small ring 1 turn")
    g, o = both(small_ring(), BEAM, z, s, a, turns=256, report_every=32)
    assert_multiturn_parity(g, o, small_ring(), BEAM, z, s, a, 256, "small ring 256 turns")
    np.testing.assert_allclose(g["pol"], o["pol"], rtol=0, atol=SPIN_TOL)


@pytest.mark.parametrize("variant", ["mk_quads", "rows1", "rows4_n16"])
def test_small_ring_variants_ragged_bunch(variant):
    ring = {"mk_quads": small_ring(quad_method="mk"),
            "rows1": small_ring(rows=1),
            "rows4_n16": small_ring(quad_slices=16, bend_slices=16, rows=4)}[variant]
    z, s, a = gaussian_bunch(1000, 21, BEAM)
    g, o = both(ring, BEAM, z, s, a, turns=4)
    assert_multiturn_parity(g, o, ring, BEAM, z, s, a, 4, variant)


def test_rhic_ring_one_turn_ragged():
    z, s, a = gaussian_bunch(777, 1501034501, BEAM)
    g, o = both(rhic_like_ring(), BEAM, z, s, a, turns=1, want_q=True)
    assert_parity(g, o, "rhic 1 turn")
    assert np.abs(g["q"] - o["q"]).max() <= SPIN_TOL


def test_rhic_ring_ten_turns():
    z, s, a = gaussian_bunch(256, 1501034501, BEAM)
    g, o = both(rhic_like_ring(), BEAM, z, s, a, turns=10, report_every=5)
    assert_multiturn_parity(g, o, rhic_like_ring(), BEAM, z, s, a, 10, "rhic 10 turns")
    np.testing.assert_allclose(g["pol"], o["pol"], rtol=0, atol=SPIN_TOL)


def test_rhic_ring_thousand_turns_long_term():
    # The full 1000-turn run on a sample. Round-off compounds over turns: an
    # amplitude error grows about linearly and the amplitude-dependent tune
    # turns it into a phase error that grows about quadratically, so a
    # per-turn bound does not hold this far out. The comparator is the
    # oracle's own plain double evaluation of the same maps: the GPU (whose
    # maps use cancellation-free forms) must drift at most a tenth as far from
    # the extended-precision result, in orbit and in spin, and its
    # polarization reports must follow the oracle's to 1e-9.
    z, s, a = gaussian_bunch(48, 1501034501, BEAM)
    turns = 1000
    g, o = both(rhic_like_ring(), BEAM, z, s, a, turns=turns, report_every=100)
    od = oracle.track(rhic_like_ring(), BEAM, z, s, a, turns=turns, report_every=100,
                      extended=False)
    np.testing.assert_array_equal(g["alive"], o["alive"])
    err, _ = orbit_rel_err(g, o)
    plain, _ = orbit_rel_err(od, o)
    ds = np.abs(g["spin"] - o["spin"]).max()
    ds_plain = np.abs(od["spin"] - o["spin"]).max()
    dp = np.abs(g["pol"][:, :3] - o["pol"][:, :3]).max()
    print(f"1000 turns: orbit {err:.3e} (plain {plain:.3e}), spin {ds:.3e} (plain {ds_plain:.3e}), "
          f"polarization {dp:.3e}")
    assert err <= 0.1 * plain
    assert ds <= 0.1 * ds_plain
    assert dp <= 1e-9


def test_rhic_full_bunch_sampled_against_the_oracle():
    # 2^20 particles in the benchmark's launch configuration, one turn;
    # 192 sampled particles (including the first and last) are re-tracked by
    # the oracle one by one.
    n = 1 << 20
    z, s, a = gaussian_bunch(n, 1501034501, BEAM)
    g = gpu_run(rhic_like_ring(), BEAM, z, s, a, turns=1, report_every=1)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 190, replace=False)]))
    o = oracle.track(rhic_like_ring(), BEAM, z[:, idx], s[:, idx], a[idx], turns=1)
    sub = {"z": g["z"][:, idx], "spin": g["spin"][:, idx], "alive": g["alive"][idx]}
    assert_parity(sub, o, "rhic 2^20 sampled")
    # properties at full size: unit spins, polarization = mean spin of the alive
    assert np.abs(np.linalg.norm(g["spin"], axis=0) - 1).max() < 1e-13
    live = g["alive"] == 1
    np.testing.assert_allclose(g["pol"][0, :3], g["spin"][:, live].mean(axis=1), rtol=0, atol=1e-13)
    assert g["pol"][0, 3] == live.sum()


# ---------------------------------------------------------- edge cases ----

def test_empty_and_single_particle():
    g = gpu_run(small_ring(), BEAM, np.zeros((6, 0)), np.zeros((3, 0)), turns=3)
    assert g["z"].shape == (6, 0)
    z, s, a = gaussian_bunch(1, 3, BEAM)
    g, o = both(small_ring(), BEAM, z, s, a, turns=3)
    assert_parity(g, o, "n=1")


def test_empty_and_drift_only_lattices():
    # no elements: every turn is the identity and the polarization is the
    # mean spin; drifts alone move the orbit and leave the spin exactly as it
    # was (no field, Ω = 0)
    z, s, a = gaussian_bunch(100, 5, BEAM)
    g, o = both([], BEAM, z, s, a, turns=3, report_every=1)
    np.testing.assert_array_equal(g["z"], z)
    np.testing.assert_array_equal(g["spin"], s)
    np.testing.assert_allclose(g["pol"], o["pol"], rtol=0, atol=SPIN_TOL)
    g, o = both([drift(2.0), drift(3.5)], BEAM, z, s, a, turns=3)
    assert_parity(g, o, "drifts")
    np.testing.assert_array_equal(g["spin"], s)


def test_distinct_element_limit():
    # the element table holds up to 65535 distinct records; a ring of that
    # many distinct drifts loads, one more is rejected before device work
    from paper_1501_03450_amd import binding as B
    beam = B.st_beam(G=1.79, gamma0=25.0, aperture=0.1, precision=0, report_every=0)
    ctx = B.st_create(0)
    elems = [drift(1.0 + 1e-6 * i) for i in range(65536)]
    assert B.st_load_lattice_raw(ctx, B.element_array(elems[:65535]), 65535, beam) == B.ST_OK
    assert B.st_load_lattice_raw(ctx, B.element_array(elems), 65536, beam) == B.ST_EINVAL
    assert "65535" in B.st_last_error(ctx)
    # repeats of the same records do not count against the limit
    arr = B.element_array(elems[:1000] * 70)
    assert B.st_load_lattice_raw(ctx, arr, 70000, beam) == B.ST_OK
    B.st_destroy(ctx)


def test_losses_flag_the_same_element_and_freeze_the_state():
    z, s, a = gaussian_bunch(300, 31, BEAM)
    beam = Beam(aperture=0.02)
    z[0, :20] = 0.0199          # start near the aperture
    z[1, :20] = 2e-3            # and head out
    z[1, 20] = 2.0              # |Px| > P: negative radicand in the first drift
    z[0, 21] = np.nan           # non-finite input
    a[22] = 0                   # dead on input: untouched
    a[23] = -7
    g, o = both(small_ring(), beam, z, s, a, turns=2)
    assert (g["alive"][:22] < 0).all()
    assert g["alive"][22] == 0 and g["alive"][23] == -7
    np.testing.assert_array_equal(g["z"][:, 22:24], z[:, 22:24])
    ok = np.isfinite(o["z"]).all(axis=0)
    assert_parity({k: v[..., ok] for k, v in g.items() if k in ("z", "spin", "alive")},
                  {k: v[..., ok] for k, v in o.items() if k in ("z", "spin", "alive")}, "losses")


def test_checkpoint_resume_is_bitwise():
    import torch
    from paper_1501_03450_amd import SpinTracker
    z, s, a = gaussian_bunch(500, 41, BEAM)
    one = gpu_run(rhic_like_ring(), BEAM, z, s, a, turns=3)
    tr = SpinTracker(rhic_like_ring(), BEAM)
    tr.set_particles(z, s, a)
    tr.track(1)
    z1, s1, a1 = tr.read()
    tr.close()
    tr = SpinTracker(rhic_like_ring(), BEAM)
    tr.set_particles(z1, s1, a1)
    tr.track(2)
    torch.cuda.synchronize()
    z2, s2, a2 = tr.read()
    tr.close()
    np.testing.assert_array_equal(z2, one["z"])
    np.testing.assert_array_equal(s2, one["spin"])
    np.testing.assert_array_equal(a2, one["alive"])


def test_invalid_lattices_are_rejected_before_device_work():
    from paper_1501_03450_amd import binding as B
    ctx = B.st_create(0)
    good = B.element_array([sbend(10.0, 0.2, 8, 3)])
    beam = B.st_beam(G=1.79, gamma0=25.0, aperture=0.1, precision=0, report_every=0)
    assert B.st_load_lattice_raw(ctx, good, 1, beam) == B.ST_OK
    bad_cases = []
    for field, value in [("kind", 9), ("orbit", 7), ("L", -1.0), ("n_slices", 0),
                         ("romberg_rows", 0), ("romberg_rows", 5), ("angle", 0.0),
                         ("eta", 0.0), ("L", float("nan")), ("orbit", B.ST_ORB_MK)]:
        arr = B.element_array([sbend(10.0, 0.2, 8, 3)])
        setattr(arr[0], field, value)
        bad_cases.append(arr)
    q = B.element_array([quad(1.0, 0.1, "mk", 4, 2)])
    q[0].orbit = B.ST_ORB_EXACT
    bad_cases.append(q)
    for arr in bad_cases:
        assert B.st_load_lattice_raw(ctx, arr, 1, beam) == B.ST_EINVAL
        assert B.st_last_error(ctx)
    for n_slices in (0, -2):
        arr = B.element_array([sbend(10.0, 0.2, 8, 3)])
        arr[0].n_slices = n_slices
        assert B.st_load_lattice_raw(ctx, arr, 1, beam) == B.ST_EINVAL
        assert "n_slices" in B.st_last_error(ctx)
    for bf, bv in [("gamma0", 1.0), ("aperture", 0.0), ("precision", 3), ("report_every", -1)]:
        b2 = B.st_beam(G=1.79, gamma0=25.0, aperture=0.1, precision=0, report_every=0)
        setattr(b2, bf, bv)
        assert B.st_load_lattice_raw(ctx, good, 1, b2) == B.ST_EINVAL
    assert B.LIB.st_track(ctx, -1, None) != B.ST_OK
    B.st_destroy(ctx)

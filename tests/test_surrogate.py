"""The spin surrogate: network kernels against the CPU float64 reference
network (same bf16-rounded weights and inputs), Adam against the textbook
update, training on tracked one-turn quaternions, and surrogate tracking
with audits and fallback through the C ABI.

There is no paper pin for the surrogate (it is not part of the method); the
plain double-precision tracker is what its spin error is measured against."""

import numpy as np
import pytest

from oracle import mlp_ref as M
from workloads import Beam, gaussian_bunch, rhic_like_ring, small_ring

pytestmark = pytest.mark.gpu

BEAM = Beam()
SIG = np.array([1e-3, 1e-4, 1e-3, 1e-4, 1e-2, 1e-3 * BEAM.beta0])


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _params(m):
    from paper_1501_03450_amd import binding as B
    n = B.st_mlp_params(m)
    out = np.zeros(n, dtype=np.float32)
    B.st_mlp_params(m, out.ctypes.data)
    return out


def _cpu_params(theta, n_in):
    """Master weights as the GPU uses them: W2, W3 rounded to bf16."""
    p = M.unflatten(theta.astype(np.float64), n_in)
    p[2] = M.bf16_round(p[2])
    p[4] = M.bf16_round(p[4])
    return p


def _data(n, n_in, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, n_in)).astype(np.float32)
    t = rng.normal(size=(n, 4))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    return x, t.astype(np.float32)


def _coherent_data(n, n_in, seed):
    """Inputs with a non-zero mean and targets clustered about one direction,
    so that the mean-loss gradient is a coherent sum rather than a cancelling
    one (which would magnify the kernels' bf16 rounding)."""
    rng = np.random.default_rng(seed)
    x = (1.0 + 0.3 * rng.normal(size=(n, n_in))).astype(np.float32)
    t = np.array([1.0, 2.0, 3.0, 4.0]) + 0.2 * rng.normal(size=(n, 4))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    return x, t.astype(np.float32)


def _rel_fro(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("n_in", [6, 7])
def test_forward_matches_the_cpu_reference(n_in):
    import torch
    from paper_1501_03450_amd import binding as B
    m = B.st_mlp_create(0, n_in, 256, seed=11)
    # Output bias of unit size: at random initialisation the last layer's
    # output is small (|y| ~ 0.03) and q = y/|y| would magnify the bf16
    # rounding of the hidden activations; a trained network has |y| ~ 1.
    theta = _params(m)
    theta[M.n_params(n_in) - 4:] = (0.5, -0.5, 0.5, 0.5)
    B.st_mlp_params(m, None, theta.ctypes.data)
    x, _ = _data(1000, n_in, 1)
    dx = _dev(x, np.float32)
    dq = torch.zeros((1000, 4), dtype=torch.float32, device="cuda")
    B.st_mlp_infer(m, dx.data_ptr(), dq.data_ptr(), 1000)
    torch.cuda.synchronize()
    # same rounding points as the kernels: bf16 W2, W3 and hidden activations,
    # everything else float32 with float32 accumulation
    q_cpu, _ = M.forward(_cpu_params(_params(m), n_in), x.astype(np.float64),
                         round_act=M.bf16_round)
    err = np.abs(dq.cpu().numpy() - q_cpu).max()
    print(f"n_in {n_in}: forward max abs err {err:.3e}")
    assert err < 1e-3
    B.st_mlp_destroy(m)


FRAME = ((0.05, -0.1, 0.98, 0.1), (0.02, 0.05, 0.01, 0.03))
# a linear frame part [4][6] of the size the fitted frames have (a few 1e-2 per
# input unit)
LIN = np.array([[0.010, -0.020, 0.000, 0.030, 0.0, 0.005],
                [-0.030, 0.010, 0.020, 0.000, 0.0, -0.010],
                [0.000, 0.005, -0.010, 0.020, 0.0, 0.010],
                [0.020, 0.000, 0.010, -0.030, 0.0, 0.020]])


@pytest.mark.parametrize("frame", [None, FRAME, FRAME + (LIN,)],
                         ids=["no_frame", "frame", "affine_frame"])
def test_gradient_matches_the_cpu_reference_tensor_by_tensor(frame):
    import torch
    from paper_1501_03450_amd import binding as B
    n_in = 6
    m = B.st_mlp_create(0, n_in, 256, seed=12)
    ref, scale = frame[:2] if frame else (None, None)
    lin = frame[2] if frame and len(frame) > 2 else None
    if frame:
        B.st_mlp_set_frame(m, ref, scale)
    if lin is not None:
        B.st_mlp_set_linear_frame(m, lin)
    x, t = _data(1000, n_in, 2)            # 1000: several tiles and a ragged tail
    dx, dt = _dev(x, np.float32), _dev(t, np.float32)
    n = B.st_mlp_params(m)
    g = torch.zeros(n, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    B.st_mlp_gradient(m, dx.data_ptr(), dt.data_ptr(), 1000, g.data_ptr(), loss.data_ptr())
    torch.cuda.synchronize()
    p = _cpu_params(_params(m), n_in)
    g_cpu = M.backward(p, x.astype(np.float64), t.astype(np.float64), ref, scale,
                       round_act=M.bf16_round, round_dz=M.bf16_round,
                       round_ds=M.bf16_round, lin=lin)
    g_gpu = M.unflatten(g.cpu().numpy(), n_in)
    for k, (a, b) in enumerate(zip(g_gpu, g_cpu)):
        assert _rel_fro(a, b) <= 1e-2, (k, _rel_fro(a, b))
    l_cpu = M.loss(p, x.astype(np.float64), t.astype(np.float64), ref, scale,
                   round_act=M.bf16_round, lin=lin)
    assert abs(loss.item() - l_cpu) <= 1e-3 * max(1.0, l_cpu)
    B.st_mlp_destroy(m)


@pytest.mark.parametrize("targets", ["coherent", "random"])
def test_gradient_of_a_large_ragged_batch_matches_the_cpu_reference(targets):
    # 70001 samples: 1094 tiles of 64, so the per-tile partials are reduced
    # in two passes.  Coherent targets give a gradient that is a coherent
    # sum; random unit targets about a fixed output frame give a cancelling
    # one (the true gradient shrinks as 1/sqrt(B)), the regime near
    # convergence.  The reference rounds where the kernels do.
    import torch
    from paper_1501_03450_amd import binding as B
    n_in, n = 6, 70001
    m = B.st_mlp_create(0, n_in, 256, seed=14)
    B.st_mlp_set_frame(m, *FRAME)
    x, t = (_coherent_data if targets == "coherent" else _data)(n, n_in, 4)
    dx, dt = _dev(x, np.float32), _dev(t, np.float32)   # keep both alive during the call
    g = torch.zeros(B.st_mlp_params(m), dtype=torch.float32, device="cuda")
    B.st_mlp_gradient(m, dx.data_ptr(), dt.data_ptr(), n, g.data_ptr())
    torch.cuda.synchronize()
    p = _cpu_params(_params(m), n_in)
    g_cpu = M.backward(p, x.astype(np.float64), t.astype(np.float64), *FRAME,
                       round_act=M.bf16_round, round_dz=M.bf16_round,
                       round_ds=M.bf16_round)
    errs = [_rel_fro(a, b) for a, b in zip(M.unflatten(g.cpu().numpy(), n_in), g_cpu)]
    print(f"{targets}: per-tensor relative errors", [f"{e:.1e}" for e in errs])
    assert max(errs) <= 1e-2, errs
    B.st_mlp_destroy(m)


def test_fitted_frame_is_the_least_squares_fit():
    # 100003 samples (a ragged last block range): targets an affine map of the
    # inputs plus noise; the library's double-precision normal equations
    # against numpy's least-squares solver on the same float inputs
    import torch
    from paper_1501_03450_amd import binding as B
    n_in, n = 7, 100003
    m = B.st_mlp_create(0, n_in, 256, seed=16)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(n, n_in)).astype(np.float32)
    x[:, 6] = rng.uniform(-1, 1, size=n)
    c0 = np.array([0.1, -0.2, 0.95, 0.2])
    A = rng.normal(scale=0.05, size=(4, n_in))
    t = (c0 + x.astype(np.float64) @ A.T + rng.normal(scale=1e-3, size=(n, 4))).astype(np.float32)
    dx, dt = _dev(x, np.float32), _dev(t, np.float32)
    f = B.st_mlp_fit_frame(m, dx.data_ptr(), dt.data_ptr(), n, 1e-5)
    r = M.fit_frame(x, t, 1e-5)
    lin = np.array([row[:n_in] for row in f["lin"]])
    assert np.abs(np.array(f["ref"]) - r["ref"]).max() <= 1e-12
    assert np.abs(lin - r["lin"]).max() <= 1e-12
    np.testing.assert_allclose(f["resid_rms"], r["resid_rms"], rtol=1e-9)
    np.testing.assert_allclose(f["resid_max"], r["resid_max"], rtol=1e-9)
    np.testing.assert_allclose(f["scale"], r["scale"], rtol=1e-9)
    assert all(v == 0.0 for row in f["lin"] for v in row[n_in:])
    # the network's frame is set from the fit: with a zero last layer the
    # prediction is the normalised affine map
    theta = _params(m)
    theta[M.n_params(n_in) - 4 - 4 * 256:] = 0.0
    B.st_mlp_params(m, None, theta.ctypes.data)
    q = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    B.st_mlp_infer(m, dx.data_ptr(), q.data_ptr(), n)
    torch.cuda.synchronize()
    u = r["ref"] + x.astype(np.float64) @ r["lin"].T
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    assert np.abs(q.cpu().numpy() - u).max() <= 1e-6
    B.st_mlp_destroy(m)


def test_fitted_frame_of_a_narrow_bunch_is_the_oracle_spin_jacobian():
    # Targets tracked by the GPU for one turn of the RHIC-scale ring from a
    # bunch a thousandth of the base size: the fitted slopes, per unit of
    # each coordinate, are the one-turn quaternion's derivatives at the
    # design orbit, which the oracle computes in forward mode.
    import oracle
    from paper_1501_03450_amd import binding as B
    from paper_1501_03450_amd import surrogate as S
    ring = rhic_like_ring()
    ref = S.design_quaternion(ring, BEAM)
    inv = 1.0 / SIG
    sur = S.new_surrogate(6, 1, np.zeros(6), inv, ref)
    z, _, _ = gaussian_bunch(65536, 1501034517, BEAM, scale=1e-3)
    x, t = S.label_bunch(sur, ring, BEAM, z)
    f = S.fit_frame(sur, x, t)
    dq_fit = sur.lin * inv[None, :]
    jac = oracle.jacobian(ring, BEAM, np.zeros(6))
    sgn = 1.0 if float(np.dot(jac["q"], ref)) >= 0 else -1.0
    dq = sgn * jac["dQ"]
    err = np.abs(dq_fit - dq).max() / np.abs(dq).max()
    print(f"fitted slopes vs oracle dQ: relative {err:.2e}; intercept - design "
          f"{np.abs(np.array(f['ref']) - ref).max():.2e}")
    assert err <= 1e-3
    assert np.abs(np.array(f["ref"]) - ref).max() <= 1e-6
    sur.close()


def test_gradient_of_a_batch_is_the_weighted_mean_of_its_parts():
    # 300000 samples (4688 tiles: three reduction passes) against the two
    # halves computed separately: the mean-loss gradient is linear in the
    # per-sample terms
    import torch
    from paper_1501_03450_amd import binding as B
    n_in, n, h = 6, 300000, 131072
    m = B.st_mlp_create(0, n_in, 256, seed=15)
    x, t = _coherent_data(n, n_in, 5)
    dx, dt = _dev(x, np.float32), _dev(t, np.float32)
    npar = B.st_mlp_params(m)
    g = [torch.zeros(npar, dtype=torch.float32, device="cuda") for _ in range(3)]
    B.st_mlp_gradient(m, dx.data_ptr(), dt.data_ptr(), n, g[0].data_ptr())
    B.st_mlp_gradient(m, dx[:h].data_ptr(), dt[:h].data_ptr(), h, g[1].data_ptr())
    B.st_mlp_gradient(m, dx[h:].data_ptr(), dt[h:].data_ptr(), n - h, g[2].data_ptr())
    torch.cuda.synchronize()
    whole = g[0].cpu().numpy().astype(np.float64)
    parts = (h * g[1].cpu().numpy().astype(np.float64) +
             (n - h) * g[2].cpu().numpy().astype(np.float64)) / n
    errs = [_rel_fro(a, b) for a, b in zip(M.unflatten(whole, n_in), M.unflatten(parts, n_in))]
    print("per-tensor relative differences", [f"{e:.1e}" for e in errs])
    assert max(errs) <= 1e-4, errs
    B.st_mlp_destroy(m)


@pytest.mark.parametrize("batch", [512, 70001])
def test_adam_step_is_the_textbook_update(batch):
    # 70001 samples are 1094 tiles: the train step leaves the last pass of
    # the per-tile partial sums to the Adam kernel, the gradient call does it
    # in the reduction kernel
    import torch
    from paper_1501_03450_amd import binding as B
    n_in = 6
    m = B.st_mlp_create(0, n_in, 256, seed=13)
    x, t = _data(batch, n_in, 3)
    dx, dt = _dev(x, np.float32), _dev(t, np.float32)
    n = B.st_mlp_params(m)
    p0 = _params(m).astype(np.float64)
    g = torch.zeros(n, dtype=torch.float32, device="cuda")
    loss_g = torch.zeros(1, dtype=torch.float32, device="cuda")
    loss_t = torch.zeros(1, dtype=torch.float32, device="cuda")
    B.st_mlp_gradient(m, dx.data_ptr(), dt.data_ptr(), batch, g.data_ptr(), loss_g.data_ptr())
    B.st_mlp_train_step(m, dx.data_ptr(), dt.data_ptr(), batch, 1e-3, loss_t.data_ptr())
    torch.cuda.synchronize()
    p1 = _params(m).astype(np.float64)
    ref = M.adam_step(p0.copy(), np.zeros(n), np.zeros(n), g.cpu().numpy().astype(np.float64), 1, 1e-3)
    np.testing.assert_allclose(p1, ref, rtol=0, atol=1e-6)
    assert abs(loss_t.item() - loss_g.item()) <= 1e-6 * loss_g.item()
    B.st_mlp_destroy(m)


def _tracked_quaternions(ring, n, seed, widen=1.0):
    import torch
    from paper_1501_03450_amd import SpinTracker
    z, s, a = gaussian_bunch(n, seed, BEAM, scale=widen)
    tr = SpinTracker(ring, BEAM)
    tr.set_particles(z, s, a)
    q = tr.enable_quaternions()
    tr.track(1)
    torch.cuda.synchronize()
    zt = torch.as_tensor(z).cuda().contiguous()
    return tr, zt, q


def test_training_on_tracked_one_turn_quaternions_reduces_the_loss():
    import torch
    from paper_1501_03450_amd import binding as B
    n = 1 << 14
    tr, z0, q = _tracked_quaternions(rhic_like_ring(), n, 101)
    m = B.st_mlp_create(0, 6, 256, seed=5)
    x = torch.zeros((n, 6), dtype=torch.float32, device="cuda")
    t = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    B.st_mlp_features(m, z0.data_ptr(), n, np.zeros(6), 1.0 / SIG, 0.0, x.data_ptr())
    B.st_mlp_targets(m, q.data_ptr(), n, (0.0, 0.0, 1.0, 0.0), t.data_ptr())
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    for step in range(400):
        lo = (step * 4096) % n
        B.st_mlp_train_step(m, x[lo:lo + 4096].data_ptr(), t[lo:lo + 4096].data_ptr(), 4096,
                            1e-3, loss.data_ptr())
        losses.append(loss.item())
    print(f"loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.05 * losses[0]
    # the network's spin prediction is closer to the tracker than "no rotation
    # information" (the mean quaternion of the bunch)
    dq = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    B.st_mlp_infer(m, x.data_ptr(), dq.data_ptr(), n)
    tt = t.cpu().numpy()
    err_net = np.abs(dq.cpu().numpy() - tt).max(axis=1)
    mean = tt.mean(0) / np.linalg.norm(tt.mean(0))
    err_mean = np.abs(tt - mean).max(axis=1)
    assert np.median(err_net) < 0.3 * np.median(err_mean)
    B.st_mlp_destroy(m)
    tr.close()


def _surrogate_run(ring, z, s, a, turns, audit_every, threshold, seed=7):
    import torch
    from paper_1501_03450_amd import SpinTracker
    from paper_1501_03450_amd import binding as B
    m = B.st_mlp_create(0, 6, 256, seed=seed)
    tr = SpinTracker(ring, BEAM)
    tr.set_particles(z, s, a)
    fb = torch.zeros(z.shape[1], dtype=torch.int32, device="cuda")
    B.st_track_surrogate(tr.ctx, m, turns, audit_every, threshold, np.zeros(6), 1.0 / SIG, 0.0,
                         fb.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = tr.read()
    tr.close()
    B.st_mlp_destroy(m)
    return out, fb.cpu().numpy()


def test_particles_that_start_on_the_fallback_path_are_tracked_in_double_precision():
    # every third particle starts on the fallback path (d_fallback != 0) and no
    # audit flags the others: the lanes are reordered so that the two groups
    # share no wave, and every particle must still get its own state back
    import torch
    from paper_1501_03450_amd import SpinTracker
    from paper_1501_03450_amd import binding as B
    ring = rhic_like_ring()
    z, s, a = gaussian_bunch(1000, 206, BEAM)
    turns = 3
    m = B.st_mlp_create(0, 6, 256, seed=3)
    tr = SpinTracker(ring, BEAM)
    tr.set_particles(z, s, a)
    fb0 = np.zeros(1000, dtype=np.int32)
    fb0[::3] = -1
    fb = torch.as_tensor(fb0).cuda()
    B.st_track_surrogate(tr.ctx, m, turns, 1000, 1e9, np.zeros(6), 1.0 / SIG, 0.0, fb.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    zs, ss, as_ = tr.read()
    tr.close()
    B.st_mlp_destroy(m)
    z64, s64, a64 = _fp64_run(ring, z, s, a, turns)
    np.testing.assert_array_equal(fb.cpu().numpy(), fb0)
    np.testing.assert_array_equal(as_, a64)
    sig = z64.std(axis=1)
    rel = np.abs(zs - z64) / np.maximum(np.abs(z64), sig[:, None])
    assert rel.max() < 1e-12 * turns * 10
    assert np.abs(ss[:, ::3] - s64[:, ::3]).max() <= 1e-12
    # the others carry the untrained network's rotations
    assert np.abs(ss[:, 1::3] - s64[:, 1::3]).max() > 1e-3


def _fp64_run(ring, z, s, a, turns):
    import torch
    from paper_1501_03450_amd import SpinTracker
    tr = SpinTracker(ring, BEAM)
    tr.set_particles(z, s, a)
    tr.track(turns)
    torch.cuda.synchronize()
    out = tr.read()
    tr.close()
    return out


def test_auditing_every_turn_is_exactly_the_double_precision_tracker():
    z, s, a = gaussian_bunch(700, 201, BEAM)
    (zs, ss, as_), fb = _surrogate_run(small_ring(), z, s, a, 4, 1, 1e9)
    z64, s64, a64 = _fp64_run(small_ring(), z, s, a, 4)
    np.testing.assert_array_equal(zs, z64)
    np.testing.assert_array_equal(ss, s64)
    assert (fb == 0).all()


def test_threshold_zero_sends_every_particle_to_the_fallback_at_the_first_audit():
    # the first audit comes after the first turn
    z, s, a = gaussian_bunch(700, 202, BEAM)
    (zs, ss, as_), fb = _surrogate_run(rhic_like_ring(), z, s, a, 5, 3, 0.0)
    assert (fb[as_ == 1] == 1).all()


def test_a_particle_that_fails_its_audit_is_replayed_in_double_precision():
    # threshold 0 over one turn: every particle that completes the turn fails
    # the audit after it, is rolled back to the start and replayed in one
    # double-precision launch, so the result is the plain tracker's bit for
    # bit; particles lost in the δ tails during the turn are not audited
    z, s, a = gaussian_bunch(700, 204, BEAM)
    (zs, ss, as_), fb = _surrogate_run(small_ring(), z, s, a, 1, 4, 0.0)
    z64, s64, a64 = _fp64_run(small_ring(), z, s, a, 1)
    assert (a64 == 1).sum() > 500
    assert (fb[a64 == 1] == 1).all() and (fb[a64 != 1] == 0).all()
    np.testing.assert_array_equal(zs, z64)
    np.testing.assert_array_equal(ss, s64)
    np.testing.assert_array_equal(as_, a64)


def test_after_a_rollback_the_spin_stays_the_double_precision_spin():
    # threshold 0, audits at turns 1, 3 and 6 of 7: rollback and replay at
    # turn 1, double-precision turns on the fallback path afterwards
    z, s, a = gaussian_bunch(700, 205, BEAM)
    (zs, ss, as_), fb = _surrogate_run(rhic_like_ring(), z, s, a, 7, 3, 0.0)
    z64, s64, a64 = _fp64_run(rhic_like_ring(), z, s, a, 7)
    np.testing.assert_array_equal(as_, a64)
    sig = z64.std(axis=1)
    rel = np.abs(zs - z64) / np.maximum(np.abs(z64), sig[:, None])
    assert rel.max() <= 1e-12 * 7
    assert np.abs(ss - s64).max() <= 1e-12


def test_orbit_only_lanes_on_an_extended_lattice():
    # fourth-order quadrupoles with fringe kicks, TEAPOT bends: the orbit of
    # lanes that leave the spin to the network follows the double-precision
    # orbit
    import dataclasses
    ring = [dataclasses.replace(e, method="mk4", fringe=True) if e.kind == "quad" else
            dataclasses.replace(e, method="teapot", rows=1) if e.kind == "sbend" else e
            for e in rhic_like_ring()]
    z, s, a = gaussian_bunch(700, 207, BEAM)
    turns = 2
    (zs, ss, as_), fb = _surrogate_run(ring, z, s, a, turns, 1000, 1e9)
    z64, _, _ = _fp64_run(ring, z, s, a, turns)
    assert (fb == 0).all()
    # the same maps inlined in another kernel path: the compiler may contract
    # a few products into fused multiply-adds differently (an ulp or so)
    sig = z64.std(axis=1)
    rel = np.abs(zs - z64) / np.maximum(np.abs(z64), sig[:, None])
    assert rel.max() < 1e-12 * turns


def test_without_fallback_the_orbit_is_the_double_precision_orbit():
    z, s, a = gaussian_bunch(700, 203, BEAM)
    turns = 3
    (zs, ss, as_), fb = _surrogate_run(rhic_like_ring(), z, s, a, turns, 1000, 1e9)
    z64, _, _ = _fp64_run(rhic_like_ring(), z, s, a, turns)
    assert (fb == 0).all()
    sig = z64.std(axis=1)
    rel = np.abs(zs - z64) / np.maximum(np.abs(z64), sig[:, None])
    assert rel.max() < 1e-12 * turns * 10      # bends crossed in one exact step
    np.testing.assert_allclose(np.linalg.norm(ss, axis=0), 1.0, atol=1e-6)


def test_what_a_trained_network_gains_over_tracking_without_it():
    # Surrogate tracking hands the spin of every particle that passes its
    # audit to the network, so those particles skip the double-precision spin
    # arithmetic.  A network trained on tracked one-turn quaternions keeps most
    # of the bunch on that path at a 1e-2 audit threshold, with the
    # polarization still following the plain tracker; the same network
    # untrained keeps almost none.
    import torch
    from paper_1501_03450_amd import SpinTracker
    from paper_1501_03450_amd import surrogate as S
    ring = rhic_like_ring()
    widen = 3.0
    ref = S.design_quaternion(ring, BEAM)
    c, inv = S.feature_map(BEAM, widen)
    z, _, _ = gaussian_bunch(1 << 17, 301, BEAM, scale=widen)

    def network(trained):
        sur = S.new_surrogate(6, 3, c, inv, ref)
        x, t = S.label_bunch(sur, ring, BEAM, z)
        S.set_scale(sur, S.frame_from_targets(t[:65536].cpu().numpy(), ref))
        if trained:
            S.train(sur, x, t, 80, 16384, 3e-3)
        return sur

    zb, sb, ab = gaussian_bunch(1 << 14, 302, BEAM)
    turns, audit, thr = 100, 50, 1e-2
    ref_run = SpinTracker(ring, BEAM, report_every=turns)
    ref_run.set_particles(zb, sb, ab)
    ref_run.track(turns)
    p64 = ref_run.polarization().cpu().numpy()[-1, :3]
    ref_run.close()
    frac, perr = {}, {}
    for trained in (True, False):
        sur = network(trained)
        tr = SpinTracker(ring, BEAM, report_every=turns)
        tr.set_particles(zb, sb, ab)
        fb = torch.zeros(zb.shape[1], dtype=torch.int32, device="cuda")
        S.track(sur, tr, turns, audit, thr, fb)
        torch.cuda.synchronize()
        frac[trained] = float((fb.cpu().numpy() != 0).mean())
        perr[trained] = float(np.abs(tr.polarization().cpu().numpy()[-1, :3] - p64).max())
        tr.close()
        sur.close()
    print(f"fallback fraction: trained {frac[True]:.3f}, untrained {frac[False]:.3f}; "
          f"polarization error trained {perr[True]:.2e}")
    assert frac[True] < 0.5
    assert frac[False] > 0.95
    assert perr[True] < 1e-2


def _qrot(q, s):
    """S' = q S q* for unit quaternions q [4][n] (w, x, y, z) and vectors s [3][n]."""
    w, v = q[0], q[1:]
    t = 2.0 * np.cross(v.T, s.T).T
    return s + w * t + np.cross(v.T, t.T).T


def test_network_turns_rotate_by_the_networks_quaternions_along_the_double_precision_orbit():
    # Twelve turns with audits after turns 1, 6 and 12 and no fallback: the
    # turns in between run as multi-turn launches (four and five turns).  The
    # spin must be the one obtained turn by turn: the double-precision
    # one-turn rotation on the audit turns and the network's quaternion of
    # the turn-start coordinates on the others, for the turns a particle
    # completes.  Every fifth particle starts on the fallback path and gets
    # the double-precision rotation every turn.  A line of matrix-kick
    # quadrupoles and drifts with a snake, where the orbit-only push is the
    # double-precision orbit bit for bit (bends would be crossed in one step
    # there), and a 1 cm aperture that loses 7 % of the bunch over the twelve
    # turns.
    import math
    import torch
    from paper_1501_03450_amd import SpinTracker
    from paper_1501_03450_amd import binding as B
    from paper_1501_03450_amd import surrogate as S
    from workloads.lattice import drift, quad, snake
    beam = Beam(aperture=0.01)
    ring = [quad(1.0, 0.05, "mk", 4, 3), drift(2.0), quad(1.0, -0.05, "mk", 4, 3),
            drift(2.0)] * 16 + [snake(math.pi, 0.0)]
    z, s, a = gaussian_bunch(1500, 208, beam)
    turns, every = 12, 6
    m = B.st_mlp_create(0, 6, 256, seed=21)
    ref = S.design_quaternion(ring, beam)
    B.st_mlp_set_frame(m, ref, (0.05, 0.05, 0.05, 0.05))
    inv = 1.0 / SIG
    tr = SpinTracker(ring, beam)
    tr.set_particles(z, s, a)
    fb0 = np.zeros(1500, dtype=np.int32)
    fb0[::5] = -1
    fb = torch.as_tensor(fb0).cuda()
    B.st_track_surrogate(tr.ctx, m, turns, every, 1e9, np.zeros(6), inv, 0.0, fb.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    zs, ss, as_ = tr.read()
    tr.close()
    np.testing.assert_array_equal(fb.cpu().numpy(), fb0)

    # turn by turn
    ft = SpinTracker(ring, beam)
    ft.set_particles(z, s, a)
    q64 = ft.enable_quaternions()
    x = torch.empty((1500, 6), dtype=torch.float32, device="cuda")
    qn = torch.empty((1500, 4), dtype=torch.float32, device="cuda")
    spin = s.copy()
    for t in range(1, turns + 1):
        B.st_mlp_features(m, ft.z.data_ptr(), 1500, np.zeros(6), inv, 0.0, x.data_ptr())
        B.st_mlp_infer(m, x.data_ptr(), qn.data_ptr(), 1500)
        before = ft.alive.cpu().numpy() == 1
        ft.track(1)
        torch.cuda.synchronize()
        after = ft.alive.cpu().numpy() == 1
        full = before if (t % every == 0 or t == 1 or t == turns) else before & (fb0 != 0)
        net = before & after & ~full
        q = q64.cpu().numpy()
        spin[:, full] = _qrot(q[:, full], spin[:, full])
        q = qn.cpu().numpy().astype(np.float64).T
        q = q / np.linalg.norm(q, axis=0)
        spin[:, net] = _qrot(q[:, net], spin[:, net])
    zf, _, af = ft.read()
    ft.close()
    B.st_mlp_destroy(m)
    np.testing.assert_array_equal(as_, af)
    np.testing.assert_array_equal(zs, zf)
    lost = (af != 1).sum()
    assert 50 < lost < 200
    assert np.abs(ss - spin).max() <= 1e-12


def _tracker_pair(ring, beam, z, s, a, fb0, turns, audit_every, threshold):
    """(surrogate run, plain double-precision run) of the same bunch."""
    import torch
    from paper_1501_03450_amd import SpinTracker
    from paper_1501_03450_amd import binding as B
    m = B.st_mlp_create(0, 6, 256, seed=5)
    tr = SpinTracker(ring, beam)
    tr.set_particles(z, s, a)
    fb = torch.as_tensor(fb0).cuda()
    B.st_track_surrogate(tr.ctx, m, turns, audit_every, threshold, np.zeros(6), 1.0 / SIG, 0.0,
                         fb.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = tr.read()
    tr.close()
    B.st_mlp_destroy(m)
    ft = SpinTracker(ring, beam)
    ft.set_particles(z, s, a)
    ft.track(turns)
    torch.cuda.synchronize()
    ref = ft.read()
    ft.close()
    return out, ref, fb.cpu().numpy()


def test_fallback_particles_get_the_double_precision_turn_bit_for_bit():
    # Every particle starts on the fallback path; three turns, audits after
    # turns 1 and 3 and a network turn between them, where the fallback lanes
    # run the full double-precision turn inside the surrogate launch.  Orbit,
    # spin and status must be the plain tracker's bit for bit.  A 2 cm
    # aperture loses about a fifth of the bunch in drifts, bends and
    # quadrupoles, so the partial turns of lost particles are covered too.
    n = 1200
    beam = Beam(aperture=0.02)
    z, s, a = gaussian_bunch(n, 209, beam)
    fb0 = np.full(n, -1, dtype=np.int32)
    (zs, ss, as_), (z64, s64, a64), fb = _tracker_pair(rhic_like_ring(), beam, z, s, a, fb0, 3,
                                                       1000, 1e9)
    np.testing.assert_array_equal(fb, fb0)
    assert 0.1 * n < (a64 != 1).sum() < 0.4 * n
    np.testing.assert_array_equal(as_, a64)
    np.testing.assert_array_equal(zs, z64)
    np.testing.assert_array_equal(ss, s64)


def test_replays_on_a_ring_with_bends_are_the_double_precision_turns_bit_for_bit():
    # Threshold 0 with an audit every second turn: every particle fails the
    # audit after turn 1 and is replayed (a launch over the failed lanes
    # only), the survivors run turns 2 to 5 on the fallback path; on the
    # RHIC-scale ring (sector bends, matrix-kick quadrupoles, thin
    # sextupoles, snakes) the result must be the plain tracker's bit for bit.
    beam = Beam(aperture=0.02)
    z, s, a = gaussian_bunch(600, 210, beam)
    fb0 = np.zeros(600, dtype=np.int32)
    (zs, ss, as_), (z64, s64, a64), fb = _tracker_pair(rhic_like_ring(), beam, z, s, a, fb0, 5, 2,
                                                       0.0)
    assert (fb[a64 == 1] == 1).all()
    np.testing.assert_array_equal(as_, a64)
    np.testing.assert_array_equal(zs, z64)
    np.testing.assert_array_equal(ss, s64)

"""Pins of the CPU reference network used to check the GPU surrogate kernels:
central finite differences of the loss for every parameter tensor, the
normalised output, the textbook Adam update and the bf16 rounding rule."""

import numpy as np
import pytest

from oracle import mlp_ref as M


def _setup(n_in=7, batch=8, seed=0):
    rng = np.random.default_rng(seed)
    params = []
    for s in M.shapes(n_in):
        fan_in = s[1] if len(s) == 2 else 256
        params.append(rng.normal(0, 1.0 / np.sqrt(fan_in), size=s))
    x = rng.normal(size=(batch, n_in))
    t = rng.normal(size=(batch, 4))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    return params, x, t


def test_output_is_a_unit_quaternion():
    params, x, _ = _setup()
    q, _ = M.forward(params, x)
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-15)


@pytest.mark.parametrize("frame", [None, ((0.1, -0.3, 0.9, 0.2), (0.05, 0.02, 0.1, 0.03))])
def test_backward_matches_central_differences_for_every_tensor(frame):
    params, x, t = _setup()
    ref, scale = frame if frame else (None, None)
    grads = M.backward(params, x, t, ref=ref, scale=scale)
    rng = np.random.default_rng(1)
    h = 1e-6
    for k, (p, g) in enumerate(zip(params, grads)):
        flat = p.ravel()
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = M.loss(params, x, t, ref, scale)
            flat[idx] = old - h
            lm = M.loss(params, x, t, ref, scale)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            gk = g.ravel()[idx]
            assert abs(fd - gk) <= 1e-6 * max(1e-3, abs(fd)), (k, idx, fd, gk)


def test_output_frame_with_zero_weights_returns_the_reference_direction():
    params, x, _ = _setup()
    params = [np.zeros_like(p) for p in params]
    ref = np.array([0.0, 0.6, 0.0, -0.8])
    q, _ = M.forward(params, x, ref=ref, scale=(0.01, 0.01, 0.01, 0.01))
    np.testing.assert_allclose(q, np.broadcast_to(ref, q.shape), atol=1e-15)


def test_adam_first_step_is_lr_times_sign():
    # With m0 = v0 = 0 the bias-corrected first step is -lr·g/(|g| + eps).
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 2.0])
    m, v = np.zeros(3), np.zeros(3)
    out = M.adam_step(theta.copy(), m, v, g, 1, lr=0.01)
    np.testing.assert_allclose(out, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_rounding_is_round_to_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, -3.14159265])
    r = M.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                                      # exactly half way to 1 + 2^-7: ties to even
    assert r[2] == 1.0 + 2 ** -7                            # above half way: rounds up
    assert r[3] == 1.0                                      # below half way: rounds down
    assert abs(r[4] + 3.140625) < 1e-12


def test_rounded_backward_is_the_gradient_of_the_rounded_forward_in_the_last_layer():
    # With the activations rounded (bf16, as the kernels hold them), the
    # rounded network is still differentiable in W4 and b4 (the rounded h3
    # does not depend on them): those two gradients must match central
    # differences of the rounded loss.  Rounding dz changes only the tensors
    # before the last layer, and by about the bf16 step.
    params, x, t = _setup(batch=16)
    frame = ((0.1, -0.3, 0.9, 0.2), (0.05, 0.02, 0.1, 0.03))
    gr = M.backward(params, x, t, *frame, round_act=M.bf16_round, round_dz=M.bf16_round)
    h = 1e-6
    for k in (6, 7):
        flat = params[k].ravel()
        for idx in range(0, flat.size, max(1, flat.size // 12)):
            old = flat[idx]
            flat[idx] = old + h
            lp = M.loss(params, x, t, *frame, round_act=M.bf16_round)
            flat[idx] = old - h
            lm = M.loss(params, x, t, *frame, round_act=M.bf16_round)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gr[k].ravel()[idx]) <= 1e-6 * max(1e-3, abs(fd)), (k, idx)
    g = M.backward(params, x, t, *frame)
    for k in range(8):
        rel = np.linalg.norm(gr[k] - g[k]) / np.linalg.norm(g[k])
        assert rel < 2e-2, (k, rel)
    assert not np.array_equal(gr[0], g[0])          # the rounding does reach dz1


def test_identity_rounding_gives_the_plain_gradient():
    params, x, t = _setup()
    same = M.backward(params, x, t, round_act=lambda v: v, round_dz=lambda v: v)
    plain = M.backward(params, x, t)
    for a, b in zip(same, plain):
        np.testing.assert_array_equal(a, b)


# ------------------------------------------------------ affine output frame --

def test_fit_frame_recovers_an_exact_affine_map():
    # targets exactly affine in the inputs: the fit returns that map, with no
    # residual, and the scale falls to the floor
    rng = np.random.default_rng(21)
    x = rng.normal(size=(500, 6))
    c0 = np.array([0.3, -0.1, 0.9, 0.2])
    A = rng.normal(size=(4, 6))
    f = M.fit_frame(x, c0 + x @ A.T, floor=1e-7)
    assert np.abs(f["ref"] - c0).max() < 1e-13
    assert np.abs(f["lin"] - A).max() < 1e-13
    assert f["resid_rms"].max() < 1e-13 and f["resid_max"].max() < 1e-13
    np.testing.assert_array_equal(f["scale"], np.full(4, 1e-7))


def test_fit_frame_residual_is_orthogonal_to_the_inputs_and_minimal():
    # least squares: the residual of every component is orthogonal to the
    # constant and to each input, and any perturbation of the fit raises
    # the summed squared residual
    rng = np.random.default_rng(22)
    x = rng.normal(size=(2000, 7))
    t = np.sin(x[:, :4]) + 0.1 * x[:, 4:5] ** 2
    f = M.fit_frame(x, t, floor=1e-9)
    r = t - f["ref"] - x @ f["lin"].T
    A = np.concatenate([np.ones((2000, 1)), x], axis=1)
    assert np.abs(A.T @ r).max() < 1e-9 * np.abs(A).sum(axis=0).max()
    np.testing.assert_allclose(f["resid_rms"], np.sqrt((r * r).mean(axis=0)), rtol=1e-12)
    base = (r * r).sum()
    for k in range(20):
        d = rng.normal(scale=1e-3, size=(4, 7))
        r2 = t - f["ref"] - x @ (f["lin"] + d).T
        assert (r2 * r2).sum() > base


def test_forward_with_a_linear_frame_adds_it_before_normalising():
    # with a zero last layer the prediction is the normalised affine map
    rng = np.random.default_rng(23)
    n_in = 6
    p = [rng.normal(scale=0.1, size=s) for s in M.shapes(n_in)]
    p[6][:] = 0.0
    p[7][:] = 0.0
    x = rng.normal(size=(10, n_in))
    ref = np.array([0.1, 0.2, 0.9, -0.3])
    lin = rng.normal(scale=0.05, size=(4, n_in))
    q, _ = M.forward(p, x, ref=ref, scale=np.ones(4), lin=lin)
    u = ref + x @ lin.T
    np.testing.assert_allclose(q, u / np.linalg.norm(u, axis=1, keepdims=True), rtol=1e-14)

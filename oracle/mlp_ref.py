"""CPU reference for the spin surrogate network — TEST INFRASTRUCTURE ONLY.

A plain float64 numpy implementation of the surrogate the GPU library trains
and evaluates: an MLP n_in → 256 → 256 → 256 → 4 with SiLU activations whose
output y is normalised, q = y/|y|, and trained on the mean squared error
L = (1/B) Σ_b |q_b - t_b|² with Adam.  The GPU kernels compute in bf16 with
float32 accumulation; the tests feed this reference the same bf16-rounded
weights and inputs and compare gradients tensor by tensor.

Parameter layout (shared with the library's flat parameter vector):
W1 [256][n_in], b1 [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256],
W4 [4][256], b4 [4]; each W row-major [out][in].
"""

from __future__ import annotations

import numpy as np

WIDTH = 256
N_OUT = 4


def shapes(n_in: int, width: int = WIDTH):
    return [(width, n_in), (width,), (width, width), (width,), (width, width), (width,),
            (N_OUT, width), (N_OUT,)]


def n_params(n_in: int, width: int = WIDTH) -> int:
    return sum(int(np.prod(s)) for s in shapes(n_in, width))


def unflatten(theta, n_in, width=WIDTH):
    out, o = [], 0
    for s in shapes(n_in, width):
        k = int(np.prod(s))
        out.append(np.asarray(theta[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def flatten(params):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, round_act=None, ref=None, scale=None, lin=None):
    """q = u/|u| with u = ref + lin x + scale ⊙ y for a batch x [B][n_in] (the
    output frame; ref = 0, lin = 0, scale = 1 by default).  round_act, when given, is applied
    to each hidden activation before it enters the next layer (the GPU
    kernels hold them in bf16)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = params
    r = round_act if round_act is not None else (lambda v: v)
    z1 = x @ W1.T + b1
    h1 = r(silu(z1))
    z2 = h1 @ W2.T + b2
    h2 = r(silu(z2))
    z3 = h2 @ W3.T + b3
    h3 = r(silu(z3))
    y = h3 @ W4.T + b4
    u = _frame(y, ref, scale)
    if lin is not None:
        u = u + x @ np.asarray(lin, dtype=np.float64).T
    q = u / np.linalg.norm(u, axis=1, keepdims=True)
    return q, (x, z1, h1, z2, h2, z3, h3, u)


def _frame(y, ref, scale):
    ref = np.zeros(N_OUT) if ref is None else np.asarray(ref, dtype=np.float64)
    scale = np.ones(N_OUT) if scale is None else np.asarray(scale, dtype=np.float64)
    return ref + scale * y


def loss(params, x, t, ref=None, scale=None, round_act=None, lin=None):
    q, _ = forward(params, x, round_act=round_act, ref=ref, scale=scale, lin=lin)
    return float(np.mean(np.sum((q - t) ** 2, axis=1)))


def backward(params, x, t, ref=None, scale=None, round_act=None, round_dz=None, lin=None,
             round_ds=None):
    """Gradients of L with respect to every parameter (same order).

    With round_act, round_dz and round_ds (all None: plain float64) the
    gradient follows the GPU kernels' rounding points: the hidden activations
    rounded as in forward(); the back-propagated dz of each hidden layer
    rounded before it enters the next product (dz3 after its bias gradient is
    summed, dz2 and dz1 before theirs); the SiLU derivatives of layers 2 and 3
    rounded as the forward pass hands them to the backward pass (bf16)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = params
    rd = round_dz if round_dz is not None else (lambda v: v)
    rs = round_ds if round_ds is not None else (lambda v: v)
    q, (x, z1, h1, z2, h2, z3, h3, u) = forward(params, x, round_act=round_act, ref=ref,
                                                scale=scale, lin=lin)
    B = x.shape[0]
    dq = 2.0 * (q - t) / B
    nu = np.linalg.norm(u, axis=1, keepdims=True)
    du = (dq - q * np.sum(q * dq, axis=1, keepdims=True)) / nu
    dy = du * (np.ones(N_OUT) if scale is None else np.asarray(scale, dtype=np.float64))
    gW4 = dy.T @ h3
    gb4 = dy.sum(0)
    dz3 = (dy @ W4) * rs(dsilu(z3))
    gb3 = dz3.sum(0)
    dz3 = rd(dz3)
    gW3 = dz3.T @ h2
    dz2 = rd((dz3 @ W3) * rs(dsilu(z2)))
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = rd((dz2 @ W2) * dsilu(z1))
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    return [gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4]


def fit_frame(x, t, floor):
    """Affine frame by least squares: the intercept ref [4] and slopes lin
    [4][n_in] minimising sum |t - ref - lin x|^2 per component over the
    samples, the RMS and largest residual per component, and scale =
    max(RMS, floor).  numpy's least-squares solver in float64."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    A = np.concatenate([np.ones((x.shape[0], 1)), x], axis=1)
    c, *_ = np.linalg.lstsq(A, t, rcond=None)
    r = t - A @ c
    rms = np.sqrt(np.mean(r * r, axis=0))
    return {"ref": c[0], "lin": c[1:].T, "resid_rms": rms, "resid_max": np.abs(r).max(axis=0),
            "scale": np.maximum(rms, floor)}


def adam_step(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of flat float64 arrays, in place."""
    m *= beta1
    m += (1.0 - beta1) * g
    v *= beta2
    v += (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta -= lr * mhat / (np.sqrt(vhat) + eps)
    return theta


def bf16_round(a):
    """Round float64 values to bfloat16 (round to nearest even), as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)

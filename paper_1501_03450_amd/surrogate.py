"""Training and use of the spin surrogate: a network that predicts a
particle's one-turn spin quaternion from its turn-start coordinates.

Host-side orchestration of the C ABI only.  Labels come from the
double-precision tracker (one turn per sample with the element quaternions
composed into a one-turn quaternion), the network trains with the library's
fused forward/backward/Adam kernels, and surrogate tracking audits it against
the tracker every few turns with a per-particle fallback.  This module moves
device pointers, chooses learning-rate schedules and keeps the bookkeeping.

The surrogate is not part of the paper's method: its spin error is measured
against the double-precision tracker, never assumed.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import binding as B
from .tracker import SpinTracker

# σ of the base bunch in (X, Px, Y, Py, T, δ); Pt ≈ β0 δ for the feature scale.
BASE_SIGMAS = np.array([1e-3, 1e-4, 1e-3, 1e-4, 1e-2, 1e-3])

# Operations of one sample (multiply-add = 2), width 256 and n_in inputs:
# forward 2(n_in·256 + 2·256² + 4·256), backward twice the hidden-layer
# products plus the small layers.
def flops_per_sample(n_in: int, train: bool) -> int:
    w = 256
    fwd = 2 * (n_in * w + 2 * w * w + 4 * w)
    if not train:
        return fwd
    bwd = 2 * (4 * w) + 2 * (2 * w * w) + 2 * (2 * w * w) + 2 * (4 * w) + 2 * (n_in * w)
    return fwd + bwd


def mfma_flops_per_sample(train: bool) -> int:
    """The part of flops_per_sample on the matrix cores (the 256×256 layers)."""
    return 2 * 2 * 256 * 256 * (3 if train else 1)


@dataclasses.dataclass
class Surrogate:
    """A trained network and the maps around it."""
    net: object                    # st_mlp handle
    n_in: int
    center: np.ndarray             # feature map: (z - center) * inv_scale
    inv_scale: np.ndarray
    ref: np.ndarray                # output frame: q = (ref + lin x + scale ⊙ y)/|…|
    scale: np.ndarray
    gamma_center: float = 0.0      # energy input (n_in == 7): (γ0 - centre)/half-width
    gamma_half_width: float = 1.0
    losses: list = dataclasses.field(default_factory=list)
    lin: np.ndarray = None         # [4][n_in]; None: no linear part

    def extra(self, gamma0: float) -> float:
        if self.n_in < 7:
            return 0.0
        return (gamma0 - self.gamma_center) / self.gamma_half_width

    def close(self):
        if self.net is not None:
            B.st_mlp_destroy(self.net)
            self.net = None


def feature_map(beam, widen: float):
    """Centre 0 and unit scale at the widened bunch's σ."""
    sig = BASE_SIGMAS.copy()
    sig[5] *= beam.beta0
    return np.zeros(6), 1.0 / (widen * sig)


def design_quaternion(ring, beam, device: int = 0) -> np.ndarray:
    """One-turn quaternion of the on-axis particle, from the tracker."""
    import torch
    tr = SpinTracker(ring, beam, device=device)
    z = np.zeros((6, 1))
    s = np.zeros((3, 1))
    s[1] = 1.0
    tr.set_particles(z, s)
    q = tr.enable_quaternions()
    tr.track(1)
    torch.cuda.synchronize()
    out = q[:, 0].cpu().numpy().copy()
    tr.close()
    return out


def label_bunch(sur: Surrogate, ring, beam, z, stream=None, device: int = 0):
    """Inputs and targets of one bunch: features of the turn-start
    coordinates, targets the tracked one-turn quaternions (sign aligned with
    the frame's reference).  Particles lost during the turn are dropped."""
    import torch
    dev = torch.device("cuda", device)
    n = z.shape[1]
    z0 = torch.as_tensor(np.ascontiguousarray(z)).to(dev)
    s = np.zeros((3, n))
    s[1] = 1.0
    tr = SpinTracker(ring, beam, device=device)
    tr.set_particles(z, s)
    q = tr.enable_quaternions()
    st = stream.cuda_stream if stream is not None else None
    tr.track(1, stream=stream)
    x = torch.empty((n, sur.n_in), dtype=torch.float32, device=dev)
    t = torch.empty((n, 4), dtype=torch.float32, device=dev)
    B.st_mlp_features(sur.net, z0.data_ptr(), n, sur.center, sur.inv_scale,
                      sur.extra(beam.gamma0), x.data_ptr(), st)
    B.st_mlp_targets(sur.net, q.data_ptr(), n, sur.ref, t.data_ptr(), st)
    if stream is not None:
        stream.synchronize()
    else:
        torch.cuda.synchronize(dev)
    keep = tr.alive == 1
    tr.close()
    if bool(keep.all()):
        return x, t
    return x[keep].contiguous(), t[keep].contiguous()


def frame_from_targets(t_host: np.ndarray, ref: np.ndarray, floor: float = 1e-5):
    """Output scale: RMS spread of the targets about ref, per component."""
    dev = t_host.astype(np.float64) - ref[None, :]
    return np.maximum(np.sqrt((dev * dev).mean(axis=0)), floor)


def fit_frame(sur: Surrogate, x, t, floor: float = 1e-5, stream=None) -> dict:
    """Affine output frame fitted by the library in double precision (least
    squares of the targets on the inputs): the network then learns only the
    residual of ref + lin x, scaled by its RMS."""
    f = B.st_mlp_fit_frame(sur.net, x.data_ptr(), t.data_ptr(), x.shape[0], floor,
                           stream.cuda_stream if stream is not None else None)
    sur.ref = np.array(f["ref"])
    sur.scale = np.array(f["scale"])
    sur.lin = np.array([row[:sur.n_in] for row in f["lin"]])
    return f


def train(sur: Surrogate, x, t, epochs: int, batch: int, lr: float, lr_final: float = None,
          stream=None, log=None):
    """Adam over contiguous batches of (x, t), cosine learning-rate decay from
    lr to lr_final; records the mean batch loss of each epoch."""
    import torch
    n = x.shape[0]
    steps = max(1, n // batch)
    total = steps * epochs
    lr_final = lr * 1e-2 if lr_final is None else lr_final
    loss = torch.zeros(steps, dtype=torch.float32, device=x.device)
    st = stream.cuda_stream if stream is not None else None
    k = 0
    for ep in range(epochs):
        for i in range(steps):
            c = 0.5 * (1.0 + math.cos(math.pi * k / max(1, total - 1)))
            rate = lr_final + (lr - lr_final) * c
            lo = i * batch
            B.st_mlp_train_step(sur.net, x[lo].data_ptr(), t[lo].data_ptr(), batch, rate,
                                loss[i].data_ptr(), st)
            k += 1
        mean = float(loss.mean().item())
        sur.losses.append(mean)
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss {mean:.3e}")
    return sur.losses


def component_errors(sur: Surrogate, x, t, stream=None) -> np.ndarray:
    """Largest component difference |q_net - t| per sample (host array)."""
    import torch
    n = x.shape[0]
    q = torch.empty((n, 4), dtype=torch.float32, device=x.device)
    B.st_mlp_infer(sur.net, x.data_ptr(), q.data_ptr(), n,
                   stream.cuda_stream if stream is not None else None)
    if stream is not None:
        stream.synchronize()
    qh = q.cpu().numpy().astype(np.float64)
    th = t.cpu().numpy().astype(np.float64)
    return np.abs(qh - th).max(axis=1)


def new_surrogate(n_in: int, seed: int, center, inv_scale, ref, device: int = 0,
                  gamma_center: float = 0.0, gamma_half_width: float = 1.0) -> Surrogate:
    """A fresh network with the output frame at ref and unit scale (set the
    scale with set_scale once the targets are known)."""
    net = B.st_mlp_create(device, n_in, 256, seed=seed)
    ref = np.asarray(ref, float)
    sur = Surrogate(net, n_in, np.asarray(center, float), np.asarray(inv_scale, float), ref,
                    np.ones(4), gamma_center, gamma_half_width)
    B.st_mlp_set_frame(net, ref, sur.scale)
    return sur


def set_scale(sur: Surrogate, scale) -> None:
    sur.scale = np.asarray(scale, float)
    B.st_mlp_set_frame(sur.net, sur.ref, sur.scale)


def track(sur: Surrogate, tracker: SpinTracker, turns: int, audit_every: int, threshold: float,
          fallback, stream=None) -> None:
    """Surrogate tracking of the tracker's bound bunch (fallback: device int32
    tensor [n], zero for particles that start on the network)."""
    B.st_track_surrogate(tracker.ctx, sur.net, turns, audit_every, threshold, sur.center,
                         sur.inv_scale, sur.extra(tracker.beam.gamma0), fallback.data_ptr(),
                         stream.cuda_stream if stream is not None else None)


# ---------------------------------------------------------------------------
# Energy scans: one bunch per reference energy, networks per energy band
# ---------------------------------------------------------------------------

def band_slices(n_energies: int, n_bands: int):
    """Contiguous bands of energies (index ranges)."""
    edges = np.linspace(0, n_energies, n_bands + 1).round().astype(int)
    return [range(edges[b], edges[b + 1]) for b in range(n_bands)]


def train_band(ring, beams, n_per_energy: int, seed: int, epochs: int, batch: int, lr: float,
               widen: float = 3.0, net_seed: int = 1, device: int = 0, log=None,
               linear_frame: bool = False) -> Surrogate:
    """A 7-input network for a band of reference energies: inputs are the six
    coordinates and the energy offset within the band; labels are tracked one
    turn at each energy of the band (widened bunch).  The output frame is the
    design quaternion with the targets' RMS spread, or the fitted affine map
    (linear_frame; it does worse here: the one-turn quaternion is far from
    affine along the energy input)."""
    import torch
    from workloads import gaussian_bunch
    g = np.array([b.gamma0 for b in beams])
    centre = 0.5 * (g.min() + g.max())
    half = max(0.5 * (g.max() - g.min()), 1e-12)
    mid = beams[int(np.argmin(np.abs(g - centre)))]
    ref = design_quaternion(ring, mid, device=device)
    c, inv = feature_map(mid, widen)
    sur = new_surrogate(7, net_seed, c, inv, ref, device=device, gamma_center=centre,
                        gamma_half_width=half)
    xs, ts = [], []
    for k, beam in enumerate(beams):
        z, _, _ = gaussian_bunch(n_per_energy, seed + k, beam, scale=widen)
        x, t = label_bunch(sur, ring, beam, z, device=device)
        xs.append(x)
        ts.append(t)
    # interleave the energies so that every batch sees the whole band
    n = min(x.shape[0] for x in xs)
    x = torch.stack([v[:n] for v in xs], dim=1).reshape(-1, 7).contiguous()
    t = torch.stack([v[:n] for v in ts], dim=1).reshape(-1, 4).contiguous()
    if linear_frame:
        fit_frame(sur, x, t)
    else:
        set_scale(sur, frame_from_targets(t[:65536].cpu().numpy(), ref))
    train(sur, x, t, epochs, min(batch, x.shape[0]), lr, log=log)
    return sur


_STREAMS: dict = {}


def _stream_pool(dev, k: int):
    """The first k of a pool of streams kept for the process: HIP gives
    streams hardware queues round robin in creation order, so reusing them
    keeps the scans' streams on distinct queues."""
    import torch
    pool = _STREAMS.setdefault(dev.index, [])
    while len(pool) < k:
        pool.append(torch.cuda.Stream(device=dev))
    return pool[:k]


def energy_scan(ring, bunches, turns: int, nets=None, audit_every: int = 50,
                threshold: float = 1e-6, n_streams: int = 4, device: int = 0, log=None):
    """Track one bunch per reference energy, spread over n_streams streams.

    bunches: list of (beam, z, spin, alive); nets: None for the plain
    double-precision tracker, else one Surrogate per bunch (shared objects
    allowed).  Returns wall-clock seconds of the tracking (from the first
    launch to the last completion, inputs resident), and per bunch the final
    polarization (Px, Py, Pz, N_alive), the survival and the fallback
    fraction."""
    import time
    import torch
    dev = torch.device("cuda", device)
    streams = _stream_pool(dev, n_streams)
    trackers, falls = [], []
    for (beam, z, s, a) in bunches:
        tr = SpinTracker(ring, beam, device=device, report_every=turns)
        tr.set_particles(z, s, a)
        trackers.append(tr)
        falls.append(torch.zeros(z.shape[1], dtype=torch.int32, device=dev) if nets else None)
    if nets is not None:
        # reserve the surrogate scratch outside the timed region
        for i, tr in enumerate(trackers):
            track(nets[i], tr, 0, audit_every, threshold, falls[i])
    torch.cuda.synchronize(dev)

    # One host thread per stream: surrogate tracking queues a few launches per
    # turn, and a full queue blocks only the thread that feeds it.
    errors = []

    done = [torch.cuda.Event() for _ in trackers]

    def feed(k):
        try:
            for i in range(k, len(trackers), n_streams):
                st = streams[k]
                if nets is None:
                    trackers[i].track(turns, stream=st)
                else:
                    track(nets[i], trackers[i], turns, audit_every, threshold, falls[i], stream=st)
                done[i].record(st)
        except Exception as e:          # reported after the join
            errors.append(e)

    import threading
    t0 = time.perf_counter()
    threads = [threading.Thread(target=feed, args=(k,)) for k in range(n_streams)]
    for th in threads:
        th.start()
    # progress while the threads feed and the streams drain
    last = time.perf_counter()
    while any(th.is_alive() for th in threads) or not all(ev.query() for ev in done):
        time.sleep(0.05)
        if log and time.perf_counter() - last > 20.0:
            last = time.perf_counter()
            log(f"{sum(ev.query() for ev in done)}/{len(trackers)} bunches done after "
                f"{last - t0:.1f} s")
    for th in threads:
        th.join()
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    if errors:
        raise errors[0]
    if log:
        log(f"tracked {len(trackers)} bunches x {turns} turns in {wall:.2f} s")
    pol, surv, fb = [], [], []
    for i, tr in enumerate(trackers):
        p = tr.polarization().cpu().numpy()
        pol.append(p[-1] if len(p) else np.full(4, np.nan))
        alive = tr.alive
        surv.append(float((alive == 1).float().mean().item()))
        if falls[i] is not None:
            fb.append(float((falls[i] != 0).float().mean().item()))
        tr.close()
    n_pt = sum(b[1].shape[1] for b in bunches) * turns
    return {"seconds": wall, "particle_turns": n_pt, "rate": n_pt / wall,
            "polarization": np.array(pol), "survival": np.array(surv),
            "fallback_fraction": np.array(fb) if fb else None}

#!/usr/bin/env python3
"""Throughput of the spin–orbit tracking hot path on one MI355X.

Workload: the RHIC-scale synthetic ring (1706 elements: 264 exact sector
bends with 8 slices and 4 Romberg rows, 456 matrix-kick quadrupoles with 4
slices, 132 thin sextupoles, 852 drifts, two ±45° snakes), 2^20 protons at
γ0 = 25 from the seeded 6-D Gaussian, spins vertical.  One step is one
st_track call of --turns-per-step turns over the whole bunch (orbit maps,
Ω at every slice edge, quaternion builds, Romberg level products and
tableau, element composition, spin rotation, loss checks and polarization
reduction), with the bunch resident in HBM.  The default 10 × 100 turns is
the full 1000-turn run.

Prints one JSON line (see the keys below).  `roofline.achieved` is the
algorithmic flop count of one particle-turn (the CPU oracle's counted adds
and multiplies for this ring; divisions, square roots and elementary
functions are listed apart under `ops_weighted`) times the particle-turns of
one launch, divided by the launch's average duration measured with HIP
events on the launch stream.  `cpu_baseline` times the CPU oracle on a bounded sample of
the same workload on the host cores (rank 0, N = 1 only).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

# The surrogate scans run many small bunches at once, each on its own stream;
# HIP maps streams onto at most GPU_MAX_HW_QUEUES hardware queues (4 by
# default), round robin in creation order, so raise that to 32 before the
# runtime starts: the scans' streams (4 double-precision, then 16 per
# surrogate scan) then land on queues of their own instead of sharing.
try:
    _queues = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _queues = 4
if _queues < 32:
    os.environ["GPU_MAX_HW_QUEUES"] = "32"

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-turns/s on 1.7k-element ring: FP64 vs mixed/surrogate @ spin err ≤1e-6"
# The oracle's counting scalar on this ring, per particle-turn.  Flops count
# each add/sub and each multiply once (the oracle forms no fused
# multiply-adds; an FMA would count 2); divisions, square roots and the
# elementary functions are reported apart and are not flops.
FLOPS_PER_PARTICLE_TURN = 1_196_956          # add/sub 428160 + mul 768796
OTHER_OPS_PER_PARTICLE_TURN = {"div": 200_882, "sqrt": 38_136, "sincos": 34_592, "asin": 4_224,
                               "sinhcosh": 10_944}
# every counted operation, each once (the earlier, operation-weighted figure)
OPS_PER_PARTICLE_TURN = FLOPS_PER_PARTICLE_TURN + sum(OTHER_OPS_PER_PARTICLE_TURN.values())
FP64_VECTOR_PEAK_TFLOPS = 78.6


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "track_fp64_rhic_ring_traffic.md")
COPY_BYTES = 1 << 30


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRACK_SOURCES = ("track.hip", "track_kernels.h", "fp64_maps.h", "device_math.h",
                 "lattice_table.h", "mixed_spin.h")


def kernel_source_hash() -> str:
    """Hash of the tracking kernel's sources: a recorded traffic figure is
    only valid for the kernel it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for name in TRACK_SOURCES:
        with open(os.path.join(ROOT, "paper_1501_03450_amd", "csrc", name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(n, turns):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    record, or None when the record is for another kernel or workload."""
    if not os.path.exists(TRAFFIC_RECORD):
        return None
    for line in open(TRAFFIC_RECORD):
        if line.startswith("traffic-record:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec["source_sha"] == kernel_source_hash() and rec["particles"] == n \
                    and rec["turns_per_launch"] == turns:
                return rec["bytes_per_launch"]
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--turns-per-step", type=int, default=100)
    ap.add_argument("--particles", type=int, default=1 << 20)
    ap.add_argument("--precision", choices=("fp64", "mixed", "mixed_all"), default="fp64",
                    help="precision of the timed launches (the headline is fp64; the others "
                         "are for profiling the mixed-precision kernel on the same workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the FP64 FMA / bf16 MFMA / HBM copy microbenchmarks")
    ap.add_argument("--cpu-sample-particles", type=int, default=32768)
    ap.add_argument("--cpu-sample-turns", type=int, default=10)
    ap.add_argument("--mixed-particles", type=int, default=4 << 20)
    ap.add_argument("--mixed-turns", type=int, default=20)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--band-energies", type=int, default=16,
                    help="energies of the default surrogate leg (the first band of the scan)")
    ap.add_argument("--scan-particles", type=int, default=65536)
    ap.add_argument("--scan-turns", type=int, default=100)
    ap.add_argument("--audit-every", type=int, default=50)
    ap.add_argument("--threshold", type=float, default=1e-6)
    ap.add_argument("--scan-streams", type=int, default=4,
                    help="streams the double-precision energy scans spread their bunches over")
    ap.add_argument("--surrogate-streams", type=int, default=16,
                    help="streams the surrogate energy scans spread their bunches over")
    ap.add_argument("--scan-thresholds", type=str, default=None,
                    help="comma-separated audit thresholds of the surrogate scans "
                         "(default: --threshold, 1e-4 and 1e-2)")
    ap.add_argument("--band-train-per-energy", type=int, default=262144)
    ap.add_argument("--band-epochs", type=int, default=3000,
                    help="training epochs of each energy-band network (262144 samples per "
                         "energy); the surrogate leg's fallback at 1e-4 falls from 63 %% at 300 "
                         "epochs to 28 %% at 3000")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the surrogate training leg (2^24 widened samples labelled by "
                         "one double-precision turn, batch 65536)")
    ap.add_argument("--c3-samples", type=int, default=1 << 24)
    ap.add_argument("--c3-epochs", type=int, default=200)
    ap.add_argument("--c3-frame", choices=("affine", "design"), default="affine",
                    help="output frame of the C3 network: the fitted affine map of the inputs, "
                         "or the design quaternion with the targets' spread")
    ap.add_argument("--band-frame", choices=("affine", "design"), default="design",
                    help="output frame of the energy-band networks (as --c3-frame)")
    ap.add_argument("--no-c0", action="store_true",
                    help="skip the small-ring leg (1024 protons x 256 turns on the GPU and on "
                         "the CPU oracle in full)")
    ap.add_argument("--c4", action="store_true",
                    help="full energy scan: 256 energies x 65536 particles, 16 bands")
    ap.add_argument("--c4-energies", type=int, default=256)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--compare-integrators", action="store_true",
                    help="one-turn errors and throughput of drift-kick vs bend-kick/matrix-kick "
                         "orbits with PWC and Romberg spin on the small ring")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run one device copy of 1 GiB and one tracking launch "
                         "(for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE), print the source hash")
    return ap.parse_args()


def host_cpu():
    """Host CPU facts recorded with the CPU baseline: the logical CPUs the OS
    reports, the CPUs this process may run on, and the model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "model": model}


# One GPU's share of the host: a GPU machine grants this many CPUs per GPU,
# whatever the OS reports, so the oracle's thread pool stops there.
CPU_SHARE_PER_GPU = 16


def cpu_baseline(ring, beam, z, s, a, n_sample, turns, n_1core, turns_1core):
    """The double-precision oracle on the host cores: one thread per usable
    CPU (at most one GPU's share of the host) on n_sample particles, and one
    thread on a smaller sample."""
    import oracle
    host = host_cpu()
    threads = max(1, min(CPU_SHARE_PER_GPU, host["usable_cpus"]))
    t0 = time.perf_counter()
    oracle.track(ring, beam, z[:, :n_sample], s[:, :n_sample], a[:n_sample], turns=turns,
                 extended=False, threads=threads)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.track(ring, beam, z[:, :n_1core], s[:, :n_1core], a[:n_1core], turns=turns_1core,
                 extended=False, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": n_sample * turns / dt, "unit": "particle-turns/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_sample} particles x {turns} turns of the same ring and bunch, "
                      f"double-precision oracle, {threads} threads, {dt:.1f} s",
            "value_1core": n_1core * turns_1core / dt1,
            "sample_1core": f"{n_1core} particles x {turns_1core} turns, 1 thread, {dt1:.1f} s",
            "host": host}


def c0_leg(beam, stream, threads):
    """The small ring in full: 1024 protons x 256 turns on the GPU (one launch,
    HIP events) and on the double-precision oracle (all threads), with the
    largest GPU-oracle differences at the end."""
    import torch
    import oracle
    from paper_1501_03450_amd import SpinTracker
    from workloads import gaussian_bunch, small_ring
    from workloads.bunch import SEED_BASE
    ring = small_ring()
    n, turns = 1024, 256
    z, s, a = gaussian_bunch(n, SEED_BASE, beam)
    tr = SpinTracker(ring, beam, device=0, report_every=turns)
    with torch.cuda.stream(stream):
        tr.set_particles(z, s, a)
    tr.track(4, stream=stream)                      # warm-up
    with torch.cuda.stream(stream):
        tr.set_particles(z, s, a)
    ms = timed_tracking(tr, turns, 1, stream)[0]
    zg, sg, ag = tr.read(stream=stream)
    tr.close()
    t0 = time.perf_counter()
    o = oracle.track(ring, beam, z, s, a, turns=turns, extended=False, threads=threads)
    dt = time.perf_counter() - t0
    live = (ag == 1) & (o["alive"] == 1)
    sig = o["z"][:, live].std(axis=1)
    rel = np.abs(zg[:, live] - o["z"][:, live]) / np.maximum(np.abs(o["z"][:, live]), sig[:, None])
    return {"workload": f"small_ring (129 elements: DKD quadrupoles 8 slices, exact bends 8 "
                        f"slices, 3 Romberg rows, one snake), {n} protons x {turns} turns, fp64",
            "unit": "particle-turns/s",
            "gpu_value": n * turns / (ms / 1e3), "gpu_ms": ms,
            "oracle_value": n * turns / dt, "oracle_seconds": dt, "oracle_threads": threads,
            "survival": float((ag == 1).mean()),
            "alive_identical": bool((ag == o["alive"]).all()),
            "orbit_rel_diff_vs_double_oracle_max": float(rel.max()),
            "spin_diff_vs_double_oracle_max": float(np.abs(sg[:, live] - o["spin"][:, live]).max())}


def timed_tracking(tracker, turns, steps, stream):
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        tracker.track(turns, stream=stream)
        ev[k + 1].record(stream)
    ev[-1].synchronize()
    return [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]


def mixed_leg(ring, beam, n, turns, stream):
    """Mixed precision against FP64 on the same GPU, bunch and turns."""
    import torch
    from paper_1501_03450_amd import SpinTracker
    from workloads import gaussian_bunch
    from workloads.bunch import SEED_BASE
    z, s, a = gaussian_bunch(n, SEED_BASE + 2, beam)
    out = {"workload": f"rhic_like_ring, {n} protons, {turns} turns from the same start"}
    res = {}
    for prec in ("fp64", "mixed", "mixed_all"):
        tr = SpinTracker(ring, beam, device=0, precision=prec, report_every=turns)
        with torch.cuda.stream(stream):
            tr.set_particles(z, s, a)
        tr.track(1, stream=stream)                  # warm-up and one-turn state
        stream.synchronize()
        z1, s1, _ = tr.read(stream=stream)
        with torch.cuda.stream(stream):
            tr.set_particles(z, s, a)
        ms = timed_tracking(tr, turns, 1, stream)[0]
        zt, st_, at = tr.read(stream=stream)
        pol = tr.polarization(stream=stream).cpu().numpy()
        tr.close()
        res[prec] = dict(ms=ms, s1=s1, z1=z1, zt=zt, st=st_, pol=pol)
        log(f"[bench] mixed leg: {prec} {n} x {turns} turns in {ms:.1f} ms")
    f = res["fp64"]
    out["fp64_value"] = n * turns / (f["ms"] / 1e3)
    out["unit"] = "particle-turns/s"
    for prec, key in (("mixed", "single_where_small_rotation"), ("mixed_all", "single_everywhere")):
        m = res[prec]
        out[key] = {
            "value": n * turns / (m["ms"] / 1e3),
            "speedup_vs_fp64": f["ms"] / m["ms"],
            "spin_err_one_turn_max": float(np.abs(m["s1"] - f["s1"]).max()),
            "orbit_identical_to_fp64": bool(np.array_equal(m["z1"], f["z1"])),
            f"mean_spin_err_after_{turns}_turns": float(np.linalg.norm(m["st"] - f["st"], axis=0).mean()),
            "polarization_err": float(np.abs(m["pol"][-1, :3] - f["pol"][-1, :3]).max()),
        }
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBPS = 8000.0


def train_bytes_per_sample(n_in):
    """HBM bytes one training sample needs between the two step kernels: the
    fused forward-backward kernel reads x and the target, writes the bf16
    activations h1, h2 and the bf16 SiLU derivative of layer 2 (read back by
    its own backward half; the layer-3 derivative stays in registers) and
    writes the bf16 gradients at the pre-activations of layers 2 and 3; the
    weight-gradient kernel reads h1, h2 and those two gradients (the split
    partials of the weight gradients are per batch, not per sample, and not
    counted)."""
    x, t, row = 4 * n_in, 16, 2 * 256
    train = x + t + 2 * row + row + row + 2 * row
    weight_grad = 4 * row
    return train + weight_grad


def quantiles(e):
    q = np.quantile(e, [0.5, 0.9, 0.99])
    return {"median": float(q[0]), "p90": float(q[1]), "p99": float(q[2]), "max": float(e.max()),
            "frac_le_1e-6": float(np.mean(e <= 1e-6)), "frac_le_1e-4": float(np.mean(e <= 1e-4))}


def error_histogram(e):
    """Counts of the per-sample errors per decade, from below 1e-8 to above 1e-1."""
    edges = [0.0] + [10.0 ** k for k in range(-8, 0)] + [np.inf]
    counts, _ = np.histogram(e, bins=edges)
    labels = ["<1e-8"] + [f"1e{k}..1e{k + 1}" for k in range(-8, -1)] + [">=1e-1"]
    return dict(zip(labels, [int(c) for c in counts]))


def frame_errors(sur, x, t):
    """Largest component error per sample of the output frame alone (the
    affine map normalised, no network), in double precision on the host."""
    xh = x.cpu().numpy().astype(np.float64)
    th = t.cpu().numpy().astype(np.float64)
    lin = sur.lin if sur.lin is not None else np.zeros((4, sur.n_in))
    u = sur.ref[None, :] + xh @ lin.T
    q = u / np.linalg.norm(u, axis=1, keepdims=True)
    return np.abs(q - th).max(axis=1)


def c3_leg(ring, beam, n_samples, epochs, batch, lr, linear_frame=True):
    """Surrogate training: labels from one double-precision turn of a
    widened bunch, Adam on the library's kernels, held-out errors."""
    import torch
    from paper_1501_03450_amd import surrogate as S
    from workloads import gaussian_bunch
    from workloads.bunch import SEED_BASE
    widen = 3.0
    ref = S.design_quaternion(ring, beam)
    c, inv = S.feature_map(beam, widen)
    sur = S.new_surrogate(6, 1, c, inv, ref)
    z, _, _ = gaussian_bunch(n_samples, SEED_BASE + 3, beam, scale=widen)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, t = S.label_bunch(sur, ring, beam, z)
    t_label = time.perf_counter() - t0
    del z
    if linear_frame:
        frame = S.fit_frame(sur, x, t)
    else:
        S.set_scale(sur, S.frame_from_targets(t[:65536].cpu().numpy(), ref))
        frame = None
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.train(sur, x, t, epochs, batch, lr, log=lambda m: log(f"[bench] c3 {m}"))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    steps = epochs * (x.shape[0] // batch)
    sps = steps * batch / t_train
    tflops = sps * S.flops_per_sample(6, True) / 1e12
    # inference over the whole training set: one warm-up pass, then a timed one
    from paper_1501_03450_amd import binding as B
    q = torch.empty((x.shape[0], 4), dtype=torch.float32, device=x.device)
    B.st_mlp_infer(sur.net, x.data_ptr(), q.data_ptr(), x.shape[0], None)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    B.st_mlp_infer(sur.net, x.data_ptr(), q.data_ptr(), x.shape[0], None)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t2
    del q
    zv, _, _ = gaussian_bunch(65536, SEED_BASE + 33, beam)
    xv, tv = S.label_bunch(sur, ring, beam, zv)
    ev = S.component_errors(sur, xv, tv)
    out = {
        "workload": f"{n_samples} samples (bunch sigma x{widen:g}), one double-precision turn of "
                    f"rhic_like_ring each; MLP 6-256-256-256-4 SiLU, bf16 MFMA, batch {batch}, "
                    f"{epochs} epochs, Adam lr {lr:g} cosine to {lr * 1e-2:g}",
        "labels_per_s": n_samples / t_label,
        "train_samples_per_s": sps,
        "train_tflops": tflops,
        "train_mfma_frac_of_bf16_peak": tflops / MFMA_BF16_PEAK_TFLOPS,
        "train_step_us": t_train / steps * 1e6,
        "train_hbm_bytes_per_sample": train_bytes_per_sample(6),
        "train_hbm_frac_of_8tbs": sps * train_bytes_per_sample(6) / (HBM_PEAK_GBPS * 1e9),
        "train_seconds": t_train,
        "infer_samples_per_s": x.shape[0] / t_infer,
        "infer_tflops": x.shape[0] / t_infer * S.flops_per_sample(6, False) / 1e12,
        "final_loss": sur.losses[-1],
        "output_frame_scale": [float(v) for v in sur.scale],
        "err_train_sample": quantiles(S.component_errors(sur, x[:65536], t[:65536])),
        "err_heldout_base_bunch": quantiles(ev),
        "err_heldout_histogram": error_histogram(ev),
        "output_frame": "affine least-squares fit" if linear_frame else "design quaternion",
        "frame_only_err_heldout": quantiles(frame_errors(sur, xv, tv)),
    }
    if frame is not None:
        out["frame_fit_resid_rms"] = frame["resid_rms"]
        out["frame_fit_resid_max"] = frame["resid_max"]
    sur.close()
    return out


def scan_leg(ring, n_energies, n_per, turns, audit_every, threshold, train_per_energy, epochs,
             lr, n_bands, thresholds=None, n_streams=4, surrogate_streams=16, linear_frame=True):
    """Energy scan with surrogate + fallback against plain double precision on
    the same bunches, plus the fallback fraction at looser thresholds."""
    from paper_1501_03450_amd import surrogate as S
    from workloads import energy_scan_bunches, energy_scan_gammas
    from workloads.bunch import SEED_BASE
    gam_all = energy_scan_gammas(256)
    gam = gam_all[:n_energies]
    bunches = energy_scan_bunches(gam, n_per, SEED_BASE + 4)
    beams = [b[0] for b in bunches]
    t0 = time.perf_counter()
    nets, per = [], []
    for b, rng_ in enumerate(S.band_slices(n_energies, n_bands)):
        sur = S.train_band(ring, [beams[i] for i in rng_], train_per_energy,
                           SEED_BASE + 3 + 1000 * (b + 1), epochs, 65536, lr, net_seed=b + 1,
                           linear_frame=linear_frame)
        log(f"[bench] band {b + 1}/{n_bands}: final loss {sur.losses[-1]:.3e}")
        nets.append(sur)
        per += [sur] * len(rng_)
    t_train = time.perf_counter() - t0
    f = S.energy_scan(ring, bunches, turns, None, n_streams=n_streams,
                      log=lambda m: log(f"[bench] fp64 scan {m}"))
    res = {}
    for thr in sorted(thresholds if thresholds else {threshold, 1e-4, 1e-2}):
        r = S.energy_scan(ring, bunches, turns, per, audit_every, thr, n_streams=surrogate_streams,
                          log=lambda m: log(f"[bench] surrogate scan (threshold {thr:g}) {m}"))
        dp = np.abs(r["polarization"][:, :3] - f["polarization"][:, :3]).max()
        res[f"{thr:g}"] = {"value": r["rate"], "speedup_vs_fp64": r["rate"] / f["rate"],
                           "fallback_fraction_mean": float(r["fallback_fraction"].mean()),
                           "fallback_fraction_max": float(r["fallback_fraction"].max()),
                           "polarization_err_max": float(dp)}
    for sur in nets:
        sur.close()
    pol = f["polarization"]
    return {
        "workload": f"{n_energies} energies (G*gamma0 from {gam[0] * beams[0].G:.4f} to "
                    f"{gam[-1] * beams[0].G:.4f}) x {n_per} particles x {turns} turns on "
                    f"rhic_like_ring; {n_bands} band networks (7 inputs, "
                    f"{'affine' if linear_frame else 'design-quaternion'} output frame), audit after the first "
                    f"turn and every {audit_every}; bunches over {n_streams} streams (FP64) and "
                    f"{surrogate_streams} streams (surrogate)",
        "unit": "particle-turns/s",
        "fp64_value": f["rate"],
        "surrogate_by_threshold": res,
        "band_training_seconds": t_train,
        "polarization_fp64": {"Py_min": float(pol[:, 1].min()), "Py_max": float(pol[:, 1].max()),
                              "per_energy_Py": [round(float(v), 6) for v in pol[:, 1]]},
        "survival_min": float(f["survival"].min()),
    }


def integrator_leg(beam, n=4096, slices=(1, 2, 4, 8, 16, 32, 64)):
    """The paper's integrator comparison (§5.2) on the small ring: one-turn
    orbit and spin errors of drift-kick (TEAPOT bends and DKD quadrupoles,
    DKS and DKDS spin placements) against bend-kick/matrix-kick orbits
    (midpoint PWC spin, and Romberg over the slice edges) and with
    fourth-order matrix-kick quadrupoles, against a reference of exact bends
    and fourth-order matrix-kick quadrupoles with 256 slices and 3 Romberg
    rows; plus each method's throughput on the same ring."""
    import math as m
    import torch
    from paper_1501_03450_amd import SpinTracker
    from workloads import gaussian_bunch
    from workloads.bunch import SEED_BASE, random_spins
    from workloads.lattice import drift, quad, sbend, snake
    th = 2 * m.pi / 32

    def ring(style, N):
        if style in ("dk_kick", "dk_midpoint"):
            place = "kick" if style == "dk_kick" else "midpoint"
            qf = quad(1.0, 0.05, "dkd", N, 1, "QF", spin=place)
            qd = quad(1.0, -0.05, "dkd", N, 1, "QD", spin=place)
            sb = sbend(10.0, th, N, 1, method="teapot", spin=place)
        elif style == "bkmk_midpoint":
            qf = quad(1.0, 0.05, "mk", N, 1, "QF", spin="midpoint")
            qd = quad(1.0, -0.05, "mk", N, 1, "QD", spin="midpoint")
            sb = sbend(10.0, th, N, 1, spin="midpoint")
        else:                                   # bkmk_romberg{R}, bkmk4_romberg{R}
            R = int(style[-1])
            mq = "mk4" if style.startswith("bkmk4") else "mk"
            qf = quad(1.0, 0.05, mq, N, R, "QF")
            qd = quad(1.0, -0.05, mq, N, R, "QD")
            sb = sbend(10.0, th, N, R)
        cell = [qf, drift(2.0), sb, drift(2.0), qd, drift(2.0), sb, drift(2.0)]
        return cell * 16 + [snake(m.pi, 0.0)]

    z, _, a = gaussian_bunch(n, SEED_BASE, beam)
    s = random_spins(n, SEED_BASE + 7, m.pi)
    n_time = 1 << 18                       # enough workgroups to fill the chip
    zt, st_, at = gaussian_bunch(n_time, SEED_BASE, beam)

    def one_turn(elems, turns=1, timing=False):
        tr = SpinTracker(elems, beam)
        if timing:
            tr.set_particles(zt, st_, at)
        else:
            tr.set_particles(z, s, a)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        tr.track(turns)
        ev1.record()
        ev1.synchronize()
        out = tr.read()
        tr.close()
        return out, ev0.elapsed_time(ev1) / 1e3

    (zr, sr, ar), _ = one_turn(ring("bkmk4_romberg3", 256))
    live = ar == 1
    sig = zr[:, live].std(axis=1)
    table = {}
    for style in ("dk_kick", "dk_midpoint", "bkmk_midpoint", "bkmk_romberg2", "bkmk_romberg3",
                  "bkmk4_romberg2", "bkmk4_romberg3"):
        rows = []
        for N in slices:
            if "_romberg" in style and N < 2 ** (int(style[-1]) - 1):
                continue
            (zz, ss, aa), _ = one_turn(ring(style, N))
            ok = live & (aa == 1)
            if not ok.any():
                raise RuntimeError(f"integrator comparison: {style} N={N} lost every particle")
            orb = float((np.abs(zz[:, ok] - zr[:, ok]) / sig[:, None]).max())
            spin = float(np.abs(ss[:, ok] - sr[:, ok]).max())
            (_, _, _), secs = one_turn(ring(style, N), turns=5, timing=True)
            rows.append({"slices": N, "orbit_err_over_sigma": orb, "spin_err": spin,
                         "particle_turns_per_s": n_time * 5 / secs})
            log(f"[bench] integrators {style} N={N}: orbit {orb:.2e} spin {spin:.2e}")
        table[style] = rows
    return {"workload": f"small ring (129 elements), {n} protons, all spin directions; "
                        "reference: exact bends and fourth-order matrix-kick quadrupoles, "
                        "256 slices, 3 Romberg rows",
            "one_turn": table}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(particles are independent: each GPU would track its own share)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1501_03450_amd import SpinTracker
    from workloads import Beam, gaussian_bunch, lattice_summary, rhic_like_ring
    from workloads.bunch import SEED_BASE

    beam = Beam()
    ring = rhic_like_ring()
    summ = lattice_summary(ring)
    n, T = args.particles, args.turns_per_step
    log(f"[bench] building bunch n={n} ring={summ['n_elements']} elements")
    z, s, a = gaussian_bunch(n, SEED_BASE + 1, beam)

    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    tr = SpinTracker(ring, beam, device=0, precision=args.precision, report_every=T)
    with torch.cuda.stream(stream):
        tr.set_particles(z, s, a)
    torch.cuda.synchronize()

    if args.traffic_probe:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        with torch.cuda.stream(stream):
            dst.copy_(src)
        stream.synchronize()
        tr.track(T, stream=stream)
        stream.synchronize()
        print(json.dumps({"source_sha": kernel_source_hash(), "particles": n,
                          "turns_per_launch": T, "copy_bytes": COPY_BYTES}), flush=True)
        tr.close()
        return

    for w in range(args.warmup):
        tr.track(T, stream=stream)
        stream.synchronize()
        log(f"[bench] warmup step {w + 1}/{args.warmup} done")

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        tr.track(T, stream=stream)
        ev[k + 1].record(stream)
    for k in range(args.steps):
        ev[k + 1].synchronize()
        log(f"[bench] step {k + 1}/{args.steps}: {ev[k].elapsed_time(ev[k + 1]):.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    total_s = sum(step_ms) / 1e3
    rate = n * T * args.steps / total_s

    pol = tr.polarization(stream=stream).cpu().numpy()
    _, _, alive = tr.read(stream=stream)
    survival = float((alive == 1).mean())
    tr.close()

    launch_s = np.mean(step_ms) / 1e3
    achieved = FLOPS_PER_PARTICLE_TURN * n * T / launch_s / 1e12
    achieved_ops = OPS_PER_PARTICLE_TURN * n * T / launch_s / 1e12
    out = {
        "metric": METRIC,
        "value": rate,
        "unit": "particle-turns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 orbit, f32 spin",
        "data": "synthetic",
        "config": {
            "workload": f"rhic_like_ring_{args.precision}",
            "elements": summ["n_elements"],
            "circumference_m": round(summ["circumference_m"], 3),
            "particles": n,
            "turns_per_step": T,
            "precision": args.precision,
            "quad": "MK, 4 slices", "bend": "exact, 8 slices", "romberg_rows": 4,
            "survival": survival,
            "final_polarization": [float(v) for v in pol[-1, :3]] if len(pol) else None,
            "wall_s": round(wall, 3),
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": recorded_traffic(n, T),
        },
        # the same launches with every counted operation as one (divisions,
        # square roots and elementary functions included)
        "ops_weighted": {
            "flops_per_particle_turn": FLOPS_PER_PARTICLE_TURN,
            "other_ops_per_particle_turn": OTHER_OPS_PER_PARTICLE_TURN,
            "achieved_tops": achieved_ops,
            "frac": achieved_ops / FP64_VECTOR_PEAK_TFLOPS,
        },
    }
    # the rates reported next to the headline: element passes, and the HBM
    # rate of the recorded per-launch traffic over the measured launch time
    traffic = out["roofline"]["traffic"]
    out["rates"] = {
        "particle_element_passes_per_s": rate * summ["n_elements"],
        "hbm_GB_per_s": (traffic / (np.mean(step_ms) / 1e3) / 1e9) if traffic else None,
    }
    if not args.no_peaks:
        # measured denominators next to the published ones (outside the timed region)
        from paper_1501_03450_amd import binding as B
        pk = B.st_measure_peaks(0)
        pk["track_frac_of_measured_fp64"] = achieved / pk["fp64_fma_tflops"]
        out["peaks_measured"] = pk
        log(f"[bench] measured peaks: {pk}")
    thresholds = ({float(v) for v in args.scan_thresholds.split(",")}
                  if args.scan_thresholds else None)
    if not args.no_mixed:
        out["mixed"] = mixed_leg(ring, beam, args.mixed_particles, args.mixed_turns, stream)
    if not args.no_surrogate:
        out["surrogate"] = scan_leg(ring, args.band_energies, args.scan_particles, args.scan_turns,
                                    args.audit_every, args.threshold, args.band_train_per_energy,
                                    args.band_epochs, args.lr, 1, thresholds, args.scan_streams,
                                    args.surrogate_streams, args.band_frame == "affine")
    if not args.no_c0:
        out["c0_small_ring"] = c0_leg(beam, stream, max(1, min(CPU_SHARE_PER_GPU,
                                                               host_cpu()["usable_cpus"])))
    if not args.no_c3:
        out["c3_training"] = c3_leg(ring, beam, args.c3_samples, args.c3_epochs, 65536, args.lr,
                                    args.c3_frame == "affine")
    if args.c4:
        out["c4_scan"] = scan_leg(ring, args.c4_energies, args.scan_particles, args.scan_turns,
                                  args.audit_every, args.threshold, args.band_train_per_energy,
                                  args.band_epochs, args.lr, max(1, args.c4_energies // 16),
                                  thresholds, args.scan_streams, args.surrogate_streams,
                                  args.band_frame == "affine")
    if args.compare_integrators:
        out["integrators"] = integrator_leg(beam)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(ring, beam, z, s, a, args.cpu_sample_particles,
                                           args.cpu_sample_turns, 1024, 10)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

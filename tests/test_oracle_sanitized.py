"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++ -fsanitize=address,undefined, every finding fatal) runs each of its
entry points on a ring holding every element kind, orbit method and spin
placement, with losses, and gives the results of the regular build."""

import ctypes
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from workloads import Beam, gaussian_bunch, small_ring
from workloads.lattice import drift, quad, rbend, sbend, snake, solenoid, thin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BEAM = Beam()


def every_kind_ring():
    th = 2 * math.pi / 32
    ring = small_ring(quad_slices=4, bend_slices=4)[:-1]
    ring[0] = quad(1.0, 0.05, "mk4", 2, 2, "QF", fringe=True)
    ring[2] = sbend(10.0, th, 4, 1, method="teapot", spin="kick")
    ring[4] = quad(1.0, -0.05, "dkd", 4, 1, "QD", spin="midpoint")
    ring[6] = sbend(10.0, th, 4, 3, fringe=True)
    ring[10] = rbend(2 * (10.0 / th) * math.sin(th / 2), th, 4, 3, asym=0.01)
    ring[12] = quad(1.0, -0.05, "mk", 4, 3, "QD")
    ring[13] = solenoid(2.0, 0.2, 4, 3)
    ring[20] = quad(1.0, -0.05, "dkd4", 2, 1, "QD", spin="midpoint")
    ring[22] = sbend(10.0, th, 4, 1, spin="midpoint")
    ring += [thin(k1l=0.01, k2l=0.3), drift(0.0), snake(math.pi, 0.3)]
    return ring


@pytest.mark.slow
def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "oracle_sanitized"
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-pthread",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "spin_oracle.cpp"),
                    os.path.join(ROOT, "tests", "oracle_sanitize_driver.cpp"), "-o", str(exe)],
                   check=True)
    ring = every_kind_ring()
    n, turns, rep = 48, 3, 1
    z, s, a = gaussian_bunch(n, 1501034599, BEAM)
    z[1, :3] = 0.03            # lost within the first cell
    a[5] = 0                   # lost before the run
    els = oracle._elems(ring)
    blob = (np.array([len(ring), n, turns, rep], np.int32).tobytes()
            + np.array([BEAM.G, BEAM.gamma0, BEAM.aperture]).tobytes()
            + bytes(memoryview(els)) + z.tobytes() + s.tobytes() + a.tobytes())
    (tmp_path / "in.bin").write_bytes(blob)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=87")
    r = subprocess.run([str(exe), str(tmp_path / "in.bin"), str(tmp_path / "out.bin")],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]

    out = np.frombuffer((tmp_path / "out.bin").read_bytes(), dtype=np.uint8)
    pos = 0

    def take(dtype, count):
        nonlocal pos
        k = np.dtype(dtype).itemsize * count
        v = out[pos:pos + k].view(dtype)
        pos += k
        return v

    for extended in (True, False):
        ref = oracle.track(ring, BEAM, z, s, a, turns=turns, report_every=rep, extended=extended,
                           want_quaternion=True)
        zz, ss = take(np.float64, 6 * n).reshape(6, n), take(np.float64, 3 * n).reshape(3, n)
        aa = take(np.int32, n)
        pol = take(np.float64, 4 * turns).reshape(turns, 4)
        q = take(np.float64, 4 * n).reshape(4, n)
        assert (ref["alive"] != 1).sum() >= 4       # the loss paths ran
        np.testing.assert_array_equal(aa, ref["alive"])
        np.testing.assert_allclose(zz, ref["z"], rtol=1e-14, atol=1e-18)
        np.testing.assert_allclose(ss, ref["spin"], rtol=0, atol=1e-14)
        np.testing.assert_allclose(pol, ref["pol"], rtol=0, atol=1e-14)
        np.testing.assert_allclose(q, ref["q"], rtol=0, atol=1e-14)
    jac = oracle.jacobian(ring, BEAM, z[:, 0])
    np.testing.assert_allclose(take(np.float64, 36).reshape(6, 6), jac["J"], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(take(np.float64, 24).reshape(4, 6), jac["dQ"], rtol=1e-13, atol=1e-15)
    counts = take(np.int64, 7)
    assert list(counts) == [oracle.count_ops(ring, BEAM, z[:, 0])[k] for k in oracle.OP_NAMES]
    assert pos + 13 * 8 == out.size

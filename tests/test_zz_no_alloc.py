"""st_track_noalloc, the tracking entry point that allocates nothing (its
polarization partials sit in a fixed device array), against st_track through
the C ABI: the same kernels, so the same bits, on two calls in a row with a
smaller bunch the second time, and its size limits refused before any
device work."""

import ctypes

import numpy as np
import pytest

from workloads import Beam, gaussian_bunch, small_ring
from workloads.bunch import random_spins

pytestmark = pytest.mark.gpu


def _bunch(n, seed, beam):
    z, _, a = gaussian_bunch(n, seed, beam)
    s = random_spins(n, seed + 1, 0.5)
    return z, s, a


def _context(ring, beam, report_every):
    from paper_1501_03450_amd import binding as B
    ctx = B.st_create(0)
    B.st_load_lattice(ctx, ring, beam.G, beam.gamma0, beam.aperture, "fp64", report_every)
    return ctx


def _bind(ctx, z, s, a):
    import torch
    from paper_1501_03450_amd import binding as B
    dz = torch.as_tensor(z).cuda().contiguous()
    ds = torch.as_tensor(s).cuda().contiguous()
    da = torch.as_tensor(a).cuda().contiguous()
    B.st_bind_particles(ctx, z.shape[1], dz.data_ptr(), ds.data_ptr(), da.data_ptr())
    return dz, ds, da


def _track_with_st_track(ring, beam, z, s, a, turns, report_every):
    import torch
    from paper_1501_03450_amd import binding as B
    ctx = _context(ring, beam, report_every)
    dz, ds, da = _bind(ctx, z, s, a)
    B.st_track(ctx, turns, None)
    n_rep = B.st_polarization(ctx)
    pol = torch.zeros((max(n_rep, 1), 4), dtype=torch.float64, device="cuda")
    if n_rep:
        B.st_polarization(ctx, pol.data_ptr(), n_rep, None)
    torch.cuda.synchronize()
    out = (dz.cpu().numpy(), ds.cpu().numpy(), da.cpu().numpy(), pol[:n_rep].cpu().numpy())
    B.st_destroy(ctx)
    return out


def test_no_alloc_tracking_is_st_track_bit_for_bit_on_two_calls_in_a_row():
    import torch
    from paper_1501_03450_amd import binding as B
    beam = Beam(aperture=0.05)            # losses in the δ tails
    ring = small_ring()
    report_every = 2
    ctx = _context(ring, beam, report_every)
    pol = torch.full((8, 4), float("nan"), dtype=torch.float64, device="cuda")
    for n, turns, seed in ((3000, 6, 11), (700, 4, 12)):      # the second call is smaller
        z, s, a = _bunch(n, seed, beam)
        print(f"no-alloc case: n={n} turns={turns} seed={seed}", flush=True)
        dz, ds, da = _bind(ctx, z, s, a)
        n_rep = B.st_track_noalloc(ctx, turns, pol.data_ptr(), pol.shape[0], None)
        torch.cuda.synchronize()
        assert n_rep == turns // report_every
        assert B.st_polarization(ctx) == 0          # the history went to the caller
        rz, rs, ra, rpol = _track_with_st_track(ring, beam, z, s, a, turns, report_every)
        assert np.array_equal(dz.cpu().numpy(), rz)
        assert np.array_equal(ds.cpu().numpy(), rs)
        assert np.array_equal(da.cpu().numpy(), ra)
        assert np.array_equal(pol[:n_rep].cpu().numpy(), rpol)
        assert (ra != 1).any() or n == 700     # the first bunch loses particles
    B.st_destroy(ctx)


def test_no_alloc_tracking_refuses_what_does_not_fit_before_device_work():
    import torch
    from paper_1501_03450_amd import binding as B
    beam = Beam()
    ring = small_ring()
    ctx = _context(ring, beam, 1)
    n = 1 << 20                                # 4096 blocks of 256
    z, s, a = _bunch(n, 21, beam)
    dz, ds, da = _bind(ctx, z, s, a)
    pol = torch.zeros((256, 4), dtype=torch.float64, device="cuda")
    max_reports = (16 << 20) // 8 // 4 // 4096            # 128 reports fit
    z0 = dz.cpu().numpy()
    # one report more than the scratch array holds
    st = B.LIB.st_track_noalloc(ctx, max_reports + 1, ctypes.c_void_p(pol.data_ptr()), 256,
                                None, None)
    assert st == B.ST_EINVAL
    assert "scratch" in B.st_last_error(ctx)
    # an output buffer smaller than the reports of the call
    st = B.LIB.st_track_noalloc(ctx, 8, ctypes.c_void_p(pol.data_ptr()), 7, None, None)
    assert st == B.ST_EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(dz.cpu().numpy(), z0)          # nothing ran
    # exactly as many reports as fit: runs, and gives st_track's bits
    n_rep = B.st_track_noalloc(ctx, max_reports, pol.data_ptr(), 256, None)
    torch.cuda.synchronize()
    assert n_rep == max_reports
    rz, rs, ra, rpol = _track_with_st_track(ring, beam, z, s, a, max_reports, 1)
    assert np.array_equal(dz.cpu().numpy(), rz)
    assert np.array_equal(ds.cpu().numpy(), rs)
    assert np.array_equal(pol[:max_reports].cpu().numpy(), rpol)
    B.st_destroy(ctx)

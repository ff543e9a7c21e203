"""Full red-black sweeps on multigrid level 0 (3-D FP64: NP_SWEEP_FULL, the
default, on level grids whose full sweep starts at least 4096 wavefronts;
NP_SWEEP_FULL_ALL on every level) against the half sweeps in place
(NP_SWEEP_HALF).

A full sweep relaxes the red points and then the black ones in one pass from
the potential into a second buffer, with the arithmetic of the two half
sweeps per point, and takes the stop test's residual norm inside the sweeps
(black points in the last post-smoothing sweep, red points in the next
cycle's first pre-smoothing sweep, which is dropped when the level stops).
The two schedules compute the same numbers: potentials, forces, cycle counts
and residual histories are compared for equality, bit for bit.  Parity of the
default (full-sweep) path with the oracle is what the other GPU tests check.
"""
import numpy as np
import pytest
import torch

from paper_2001_02327_amd import workloads as W
from paper_2001_02327_amd.solver import NestedPoissonSolver

pytestmark = pytest.mark.gpu


def _solve(wl, profile=False, **kw):
    dev = torch.device("cuda")
    rho, po = W.make_inputs(wl.geom, wl.prob, device=dev)
    s = NestedPoissonSolver(wl.geom, **kw)
    if profile:
        s.set_profiling(True)
    st = s.solve(rho, po)
    st["profile"] = s.profile() if profile else None
    phi = [s.potential(l).cpu().numpy() for l in range(wl.geom.nlevels)]
    F = [tuple(a.cpu().numpy() for a in s.forces(l)) for l in range(wl.geom.nlevels)]
    hist = [s.history(l) for l in range(wl.geom.nlevels)]
    torch.cuda.synchronize()
    s.close()
    return phi, F, st, hist


def _ragged():
    # N^0 = 12 and 24 on the two levels: odd row lengths on multigrid level 0 of level 1
    g = W.Geometry(dim=3, n=[22, 10], off=[(0, 0, 0), (4, 3, 6)], lo0=(-0.5, -0.5, -0.5), dx0=1.0 / 22)
    return W.Workload("ragged3d_22_10", g, W.Plummer([(1.0, 0.08, (0.05, -0.02, 0.03))]))


def _minimal():
    g = W.Geometry(dim=3, n=[8, 4], off=[(0, 0, 0), (2, 2, 2)], lo0=(-0.5, -0.5, -0.5), dx0=1.0 / 8)
    return W.Workload("minimal3d_8_4", g, W.Plummer([(1.0, 0.2, (0.0, 0.0, 0.0))]))


CASES = [W.c2_plummer(16), W.c2_plummer(32), W.paper3d(16), W.c3_plummer_offset(32), W.c4_multi_plummer(7, N=32),
         _ragged(), _minimal(), W.box_plummer_3d(1)]


def _assert_same(a, b):
    phi_a, F_a, st_a, h_a = a
    phi_b, F_b, st_b, h_b = b
    assert st_a["cycles"] == st_b["cycles"]
    for l in range(len(phi_a)):
        assert np.array_equal(h_a[l], h_b[l]), ("history", l)
        assert np.array_equal(phi_a[l], phi_b[l]), ("phi", l, np.abs(phi_a[l] - phi_b[l]).max())
        for ax in range(len(F_a[l])):
            assert np.array_equal(F_a[l][ax], F_b[l][ax]), ("F", l, ax)


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w.name)
def test_full_equals_half_sweeps(wl):
    full = _solve(wl, sweep="full_all")
    half = _solve(wl, sweep="half")
    _assert_same(full, half)


@pytest.mark.parametrize("pre_post", [(1, 1), (3, 2), (1, 3)])
def test_full_equals_half_other_schedules(pre_post):
    wl = W.c2_plummer(32)
    n_pre, n_post = pre_post
    _assert_same(_solve(wl, sweep="full_all", n_pre=n_pre, n_post=n_post),
                 _solve(wl, sweep="half", n_pre=n_pre, n_post=n_post))


def test_full_equals_half_force_change_rule():
    wl = W.paper3d(32)
    _assert_same(_solve(wl, sweep="full_all", stop_rule="force_delta"), _solve(wl, sweep="half", stop_rule="force_delta"))


def test_full_equals_half_patch_tree_and_interp_buffer():
    """A tree solved one patch after another, and the comparison scheme (whose
    refined levels keep the half sweeps)."""
    wl = W.two_patch_3d(32)
    _assert_same(_solve(wl, sweep="full_all", batch=False), _solve(wl, sweep="half", batch=False))
    wl = W.c2_plummer(32)
    _assert_same(_solve(wl, sweep="full_all", buffer="interp"), _solve(wl, sweep="half", buffer="interp"))


def test_full_equals_half_at_size():
    """Five levels of 128^3 (130^3 points on multigrid level 0: several z-chunks
    and row groups per block, ragged last chunk)."""
    wl = W.c5_two_plummer(N=128)
    _assert_same(_solve(wl, sweep="full_all"), _solve(wl, sweep="half"))


def _sweep_launches(wl, **kw):
    """Launch counts of the full and the half sweeps in one default solve (no
    arrays copied back)."""
    rho, po = W.make_inputs(wl.geom, wl.prob, device=torch.device("cuda"))
    s = NestedPoissonSolver(wl.geom, **kw)
    s.set_profiling(True)
    st = s.solve(rho, po)
    prof = s.profile()
    torch.cuda.synchronize()
    s.close()
    assert max(st["final_rel_residual"]) <= 1e-10
    return prof["full"][0], prof["smooth"][0]


def test_default_takes_full_sweeps_on_large_levels_only():
    """The default sweep setting runs full sweeps on a 512^3 level (7128
    wavefronts per full sweep) and half sweeps on a 512 x 512 x 64 slab (1080),
    on 2 x 256^3 (952) and on 3 x 128^3; the iterates are those of the half
    sweeps either way (the tests above)."""
    full, half = _sweep_launches(W.c5_two_plummer(N=512, nlevels=1))
    assert full > 0 and half == 0
    for wl in (W.slab_two_plummer(512), W.c5_two_plummer(N=256, nlevels=2), W.c2_plummer(128)):
        full, half = _sweep_launches(wl)
        assert full == 0 and half > 0, wl.name

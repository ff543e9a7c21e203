"""Batched patches on the GPU: the patches of one refinement depth with the
same extents are solved together, one launch per operator over all of them
(Sec. 2.1 places every patch inside one coarser patch and the one-way scheme
makes siblings independent, so they can run side by side; Sec. 4 names the
patch-based setting).

Pins: the batched solve equals the one-after-another solve bit for bit
(potentials, forces, cycle counts and residual histories of every entry: the
same arithmetic runs on every patch, each stopping at its own count); at the
oracle's per-entry cycle counts it matches the oracle (1e-12 / 1e-11); with
its own stop rule it takes the oracle's counts within one cycle.
"""
import numpy as np
import pytest
import torch

from paper_2001_02327_amd import _lib
from paper_2001_02327_amd import workloads as W
from paper_2001_02327_amd.solver import NestedPoissonSolver

from test_gpu_parity import assert_parity, oracle_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need the MI355X"


def _run(wl, fixed=None, **kw):
    rho, po = W.make_inputs(wl.geom, wl.prob, device="cuda")
    s = NestedPoissonSolver(wl.geom, **kw)
    if fixed is not None:
        s.set_fixed_cycles(fixed)
    st = s.solve(rho, po)
    L = wl.geom.nlevels
    phi = [s.potential(l).cpu().numpy() for l in range(L)]
    F = [tuple(a.cpu().numpy() for a in s.forces(l)) for l in range(L)]
    hist = [s.history(l) for l in range(L)]
    s.close()
    return phi, F, st, hist


def _uneven_2d():
    # four same-size children around sources of different widths, so the
    # members of the batch stop after different cycle counts
    g = W.many_patches_geometry(2, 64, 2, 16, depth2=True)
    terms = []
    for i, l in enumerate(c for c in range(1, g.nlevels) if g.par(c) == 0):
        lo = g.lo(l)
        terms.append((1.0 + 0.5 * i, 0.03 + 0.03 * i, tuple(lo[a] + 0.5 * g.ext(l)[a] * g.dx(l) for a in range(2))))
    return W.Workload("uneven_2d", g, W.GaussianSum(terms))


CASES = [W.many_patches_3d(32, 2, 8, depth2=True), W.many_patches_2d(64, 2, 16, depth2=True), _uneven_2d(),
         W.two_patch_3d(32), W.many_patches_3d(64, 2, 16)]


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w.name)
def test_batched_equals_one_after_another(wl):
    print("batch: %s, %d entries" % (wl.name, wl.geom.nlevels), flush=True)
    a = _run(wl)
    b = _run(wl, batch=False)
    assert a[2]["cycles"] == b[2]["cycles"]
    for l in range(wl.geom.nlevels):
        assert np.array_equal(a[0][l], b[0][l]), l
        for ax in range(wl.geom.dim):
            assert np.array_equal(a[1][l][ax], b[1][l][ax]), (l, ax)
        assert a[3][l] == b[3][l], l


def test_batch_members_stop_at_their_own_counts():
    wl = _uneven_2d()
    _, _, st, _ = _run(wl)
    kids = [l for l in range(1, wl.geom.nlevels) if wl.geom.par(l) == 0]
    assert len(set(st["cycles"][l] for l in kids)) > 1, st["cycles"]


@pytest.mark.parametrize("wl", CASES[:3], ids=lambda w: w.name)
def test_batched_parity_with_oracle(wl):
    res, F_o = oracle_solve(wl)
    assert res["status"] == 0
    phi, F, st, _ = _run(wl, fixed=res["cycles"])
    assert st["cycles"] == res["cycles"]
    assert_parity(wl, phi, F, res, F_o)
    _, _, st2, _ = _run(wl)
    for l in range(wl.geom.nlevels):
        assert abs(st2["cycles"][l] - res["cycles"][l]) <= 1, (st2["cycles"], res["cycles"])
        assert st2["final_rel_residual"][l] <= 1e-10


@pytest.mark.parametrize("wl", [CASES[0], CASES[2]], ids=lambda w: w.name)
def test_batched_coarse_post(wl):
    """V(1,1) on multigrid level 0 with two post-smoothing sweeps below it
    (np_config.coarse_post) on batched patches: equal to the one-after-another
    solve bit for bit, and to the oracle with the same schedule at its own
    per-entry cycle counts."""
    kw = dict(n_pre=1, n_post=1, coarse_post=2)
    res, F_o = oracle_solve(wl, max_cycles=120, **kw)
    assert res["status"] == 0
    a = _run(wl, fixed=res["cycles"], max_cycles=120, **kw)
    b = _run(wl, fixed=res["cycles"], max_cycles=120, batch=False, **kw)
    assert a[2]["cycles"] == res["cycles"]
    assert_parity(wl, a[0], a[1], res, F_o)
    for l in range(wl.geom.nlevels):
        assert np.array_equal(a[0][l], b[0][l]), l
        assert a[3][l] == b[3][l], l


def test_batch_cap_and_error_codes():
    """A cap that stops every member early reports NP_ENOTCONV with valid
    results, as one patch at a time does."""
    wl = W.many_patches_3d(32, 2, 8)
    rho, po = W.make_inputs(wl.geom, wl.prob, device="cuda")
    for batch in (True, False):
        s = NestedPoissonSolver(wl.geom, max_cycles=3, batch=batch)
        st = s.solve(rho, po, allow_notconv=True)
        assert st["status"] == _lib.NP_ENOTCONV
        assert all(c == 3 for c in st["cycles"])
        s.close()

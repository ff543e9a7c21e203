"""The benchmark workload at its full size (two Plummer spheres, 5 levels of
512^3 cells, 514^3 points on multigrid level 0) in the launch configuration
that bench.py times, checked where the oracle can follow at that size:

* one V(2,1) cycle of level 0 from the zero start against the oracle's cycle on
  the same 514^3 problem, at every point (1e-12 of max|Phi|, the parity bar),
  and one cycle of the benchmark's schedule (V(1,1) on level 0, V(1,2) below);
* the converged solves of the plain FP64 path and of the FP16-storage defect
  correction with adaptive inner cycles (V(2,1), and V(1,1) on level 0 with
  V(1,2) below as the benchmark runs it): on every level the outer ghost layer
  equals the oracle's interpolation of the GPU's level l-1 (1e-14), the stop
  criterion recomputed by the oracle in FP64 over every active point holds
  (||f - lap Phi||_inf <= 1e-10 ||f||_inf, the right-hand side of levels l >= 1
  rebuilt by the oracle's interface fill), and the forces equal the oracle's
  stencil applied to the GPU's potential (1e-11 of max|F|).
"""
import math

import numpy as np
import pytest
import torch

from oracle import core
from paper_2001_02327_amd import workloads as W
from paper_2001_02327_amd.solver import NestedPoissonSolver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def problem():
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    wl = W.c5_two_plummer()
    rho, po = W.make_inputs(wl.geom, wl.prob)
    return wl, rho, po


@pytest.mark.parametrize("schedule", [dict(), dict(n_pre=1, n_post=1, coarse_post=2)], ids=["v21", "v11_v12"])
def test_one_cycle_of_level0_at_514(problem, schedule):
    """One FP64 V-cycle of level 0 from the zero start, the paper's V(2,1) and
    the benchmark's V(1,1) with V(1,2) below level 0."""
    wl, rho, po = problem
    g = wl.geom
    s = NestedPoissonSolver(g, **schedule)
    s.set_fixed_cycles([1] + [0] * (g.nlevels - 1))
    s.solve([r.cuda() for r in rho], po.cuda())
    got = s.potential(0).cpu().numpy()
    s.close()
    u = np.ascontiguousarray(po.numpy())
    u[1:-1, 1:-1, 1:-1] = 0.0
    f = np.zeros_like(u)
    f[1:-1, 1:-1, 1:-1] = 4 * math.pi * g.G * rho[0].numpy()
    core.vcycle_patch(3, g.dx0, u, f, **schedule)
    err = np.abs(got - u).max() / np.abs(u).max()
    print("one level-0 V-cycle at 514^3 (%s): max relative difference %.2e" % (schedule, err))
    assert err <= 1e-12


@pytest.mark.parametrize("settings", [dict(), dict(precision="fp16s_dc", inner_cycles="adaptive"),
                                      dict(precision="fp16s_dc", inner_cycles="adaptive", n_pre=1, n_post=1,
                                           coarse_post=2)],
                         ids=["fp64", "fp16s_dc_adaptive", "fp16s_dc_v11_v12"])
def test_converged_solve_at_514(problem, settings):
    wl, rho, po = problem
    g = wl.geom
    fourpiG = 4 * math.pi * g.G
    s = NestedPoissonSolver(g, **settings)
    st = s.solve([r.cuda() for r in rho], po.cuda())
    f_prev = phi_prev = None
    for l in range(g.nlevels):
        dx = g.dx(l)
        phi = s.potential(l).cpu().numpy()
        if l == 0:
            f = np.zeros_like(phi)
            f[1:-1, 1:-1, 1:-1] = fourpiG * rho[0].numpy()
            ring_ref = np.ascontiguousarray(po.numpy())
        else:
            ring_ref, f = core.interface_fill(3, phi_prev, f_prev, g.n[l], g.off[l], rho[l].numpy(), fourpiG)
        ring = np.ones(phi.shape, dtype=bool)
        ring[1:-1, 1:-1, 1:-1] = False
        ring_err = np.abs(phi[ring] - ring_ref[ring]).max() / np.abs(ring_ref[ring]).max()
        assert ring_err <= 1e-14, (l, ring_err)
        fmax = np.abs(f[1:-1, 1:-1, 1:-1]).max()
        rnorm = core.residual_norm(3, dx, phi, f)
        print("level %d: %d V-cycles, ||r|| / ||f|| = %.3e (library %.3e)" %
              (l, st["cycles"][l], rnorm / fmax, st["final_rel_residual"][l]))
        assert rnorm <= 1e-10 * fmax * (1 + 1e-4), (l, rnorm / fmax)
        F = [a.cpu().numpy() for a in s.forces(l)]
        Fo = core.forces(3, dx, phi)
        fscale = max(np.abs(a).max() for a in Fo)
        for ax in range(3):
            e = np.abs(F[ax] - Fo[ax]).max() / fscale
            assert e <= 1e-11, (l, ax, e)
        del F, Fo
        f_prev, phi_prev = f, phi
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp16s_dc"])
def test_single_patch_1020(precision):
    """The largest patch tested: one level of 1020^3 cells, 1022^3 points on
    multigrid level 0 and 2^30 points in its two colour arrays (8.6 GB per FP64
    array), where the level-0 restriction takes its generic form (the arrays
    pass 2^31 bytes).  The stop criterion, recomputed by the oracle in FP64
    over every active point, holds, and the forces equal the oracle's stencil
    on sampled blocks (corners, edges, interior)."""
    n = 1020
    g = W.Geometry(dim=3, n=[n], off=[(0, 0, 0)], lo0=(-1.0, -1.0, -1.0), dx0=2.0 / n)
    prob = W.Plummer([(1.0, 0.1, (0.013, -0.021, 0.007))])
    print("case: single patch 1020^3, %s" % precision, flush=True)
    dev = torch.device("cuda")
    settings = dict(precision=precision, inner_cycles="adaptive") if precision != "fp64" else {}
    s = NestedPoissonSolver(g, **settings)
    rho, po = W.make_inputs(g, prob, device=dev)
    st = s.solve(rho, po)
    del po
    assert st["final_rel_residual"][0] <= 1e-10
    phi = s.potential(0).cpu().numpy()
    f = np.zeros_like(phi)
    f[1:-1, 1:-1, 1:-1] = 4 * math.pi * g.G * rho[0].cpu().numpy()
    del rho
    fmax = np.abs(f).max()
    rnorm = core.residual_norm(3, g.dx0, phi, f)
    print("%d V-cycles, ||r|| / ||f|| = %.3e (library %.3e)" % (st["cycles"][0], rnorm / fmax,
                                                               st["final_rel_residual"][0]), flush=True)
    assert rnorm <= 1e-10 * fmax * (1 + 1e-4)
    del f
    F = s.forces(0)
    B = 16
    for k0, j0, i0 in [(0, 0, 0), (n - B, n - B, n - B), (0, n - B, 500), (501, 300, 700)]:
        sub = np.ascontiguousarray(phi[k0:k0 + B + 4, j0:j0 + B + 4, i0:i0 + B + 4])
        Fo = core.forces(3, g.dx0, sub)
        fscale = max(np.abs(a).max() for a in Fo)
        for ax in range(3):
            Fg = F[ax][k0:k0 + B, j0:j0 + B, i0:i0 + B].cpu().numpy()
            e = np.abs(Fg - Fo[ax]).max() / fscale
            assert e <= 1e-11, ((k0, j0, i0), ax, e)
    del F
    s.close()

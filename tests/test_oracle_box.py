"""Pins of the oracle on non-cubic patches (Sec. 2.1 gives the cell counts per
direction; Sec. 2.2 builds the multigrid hierarchy along each axis; Sec. 2.4
applies the boundary rule to the y and z boundaries in the same way).

Reading: every axis halves its mesh with the same doubling of h, so the cells
stay cubes, and the hierarchy ends on the first level where some axis has a
single active cell (item 4 of Sec. 2.2 met per axis).
"""
import numpy as np
import pytest

from oracle import core, dense, norms
from paper_2001_02327_amd import workloads as W


def _inputs(wl):
    rho, po = W.make_inputs(wl.geom, wl.prob)
    return [r.numpy() for r in rho], po.numpy()


# ------------------------------------------------------------------ hierarchy
def test_plan3_hand_worked():
    # 64 x 32 x 48 cells: N^0 = (66, 34, 50); halves rounded up per axis; the
    # y axis reaches one cell first, on level 5
    assert core.plan3(3, (66, 34, 50)) == [(66, 34, 50), (33, 17, 25), (17, 9, 13), (8, 4, 6), (4, 2, 3), (2, 1, 2)]
    # 2-D 40 x 24 patch: N^0 = (42, 26)
    assert core.plan3(2, (42, 26)) == [(42, 26), (21, 13), (11, 7), (5, 3), (3, 2), (1, 1)]
    assert core.plan3(2, (26, 10)) == [(26, 10), (13, 5), (7, 3), (3, 1)]


@pytest.mark.parametrize("dim", [2, 3])
def test_plan3_reduces_to_the_cube_and_to_each_axis(dim):
    rng = np.random.default_rng(dim)
    for _ in range(300):
        N0 = tuple(int(v) for v in rng.integers(3, 400, size=dim))
        p3 = core.plan3(dim, N0)
        axes = [core.plan(v) for v in N0]
        # every axis follows its own one-axis hierarchy ...
        for L, row in enumerate(p3):
            for a in range(dim):
                assert row[a] == axes[a][L]
        # ... and the hierarchy stops on the first level with a one-cell axis
        assert min(p3[-1]) == 1
        assert all(min(row) > 1 for row in p3[:-1])
        # a cube is the one-axis hierarchy
        c = N0[0]
        assert core.plan3(dim, (c,) * dim) == [(v,) * dim for v in core.plan(c)]


def test_ghost_fill_per_axis_rules():
    """On a box level the right ghost of each axis follows that axis's own
    rule: lines vanishing at x_MG = 0 and x_MG = 1 along one axis (constant
    along the others, the left rule flips them too) are reproduced exactly."""
    N0 = (66, 34, 50)
    p = core.plan3(3, N0)
    for L in (1, 2, 3):
        N = p[L]
        h = [2.0 ** L / N0[a] for a in range(3)]
        for a in range(3):
            one, c = core.ghost_rule(N0[a], L, N[a])
            x = (np.arange(N[a] + 2) - 0.5) * h[a]  # centres, ghost 0 at -h/2
            for g in (lambda t: t, lambda t: 1.0 - t):
                shape = [1, 1, 1]
                shape[2 - a] = N[a] + 2
                e = np.broadcast_to(g(x).reshape(shape), (N[2] + 2, N[1] + 2, N[0] + 2)).copy()
                inner = (slice(1, -1),) * 3
                want = e.copy()
                e_in = np.zeros_like(e)
                e_in[inner] = e[inner]
                core.ghost_fill(3, N0, L, e_in)
                # the ghost layer along axis a: left = -e_1 everywhere, right by the rule
                sl_l = [slice(1, -1)] * 3
                sl_l[2 - a] = 0
                sl_1 = [slice(1, -1)] * 3
                sl_1[2 - a] = 1
                np.testing.assert_array_equal(e_in[tuple(sl_l)], -e_in[tuple(sl_1)])
                sl_r = [slice(1, -1)] * 3
                sl_r[2 - a] = N[a] + 1
                if g(1.0) == 0.0:
                    # the line through zero at x_MG = 1 continues exactly (x_N = 1: odd
                    # reflection about 1; else the rule's coefficient)
                    np.testing.assert_allclose(e_in[tuple(sl_r)], want[tuple(sl_r)], rtol=0, atol=1e-14)
                if g(0.0) == 0.0:
                    np.testing.assert_allclose(e_in[tuple(sl_l)], want[tuple(sl_l)], rtol=0, atol=1e-14)


# ------------------------------------------------------------------ nested solves
def _box3d():
    g = W.box_geometry(3, (12, 8, 10), (8, 6, 4), (2, 1, 3), dx0=1.0 / 12)
    return W.Workload("box3d_small", g, W.Plummer([(1.0, 0.2, (0.45, 0.3, 0.4))]))


def _box2d():
    g = W.box_geometry(2, (16, 10), (10, 6), (3, 2), (6, 4), (1, 1), dx0=1.0 / 16)
    return W.Workload("box2d_small", g, W.GaussianSum([(1.0, 0.2, (0.55, 0.35))]))


@pytest.mark.parametrize("make", [_box3d, _box2d, lambda: W.box_gaussian_2d(1)], ids=["3d", "2d", "2d_stack"])
def test_box_multigrid_reaches_the_direct_solution(make):
    wl = make()
    rho, po = _inputs(wl)
    it = core.solve(wl.geom, rho, po, tol=1e-13, max_cycles=200)
    assert it["status"] == 0, it["status_name"]
    ex, _ = dense.solve(wl.geom, rho, po)
    for l in range(wl.geom.nlevels):
        err = np.abs(it["phi"][l] - ex[l]).max() / np.abs(ex[l]).max()
        assert err <= 1e-11, (l, err)


@pytest.mark.parametrize("dim", [2, 3])
def test_box_linear_potential_exact(dim):
    """Zero density, linear potential: interpolation and Laplacian are exact,
    so every box level reproduces the plane and F = -(a, b, c)."""
    if dim == 3:
        g = W.box_geometry(3, (16, 8, 12), (8, 6, 10), (4, 1, 1), (4, 4, 6), (2, 1, 1), dx0=1.0 / 16)
        prob = W.Linear([0.7, -1.3, 0.4], 2.0)
    else:
        g = W.box_geometry(2, (16, 8), (12, 6), (2, 1), (8, 4), (1, 1), dx0=1.0 / 16)
        prob = W.Linear([0.7, -1.3], 2.0)
    wl = W.Workload("linear_box", g, prob)
    rho, po = _inputs(wl)
    res = core.solve(g, rho, po, tol=1e-14, max_cycles=200)
    assert res["status"] == 0
    for l in range(g.nlevels):
        x = g.mesh_pad(l, 2)
        np.testing.assert_allclose(res["phi"][l], prob.phi(*x).numpy(), rtol=0, atol=1e-12)
        F = core.forces(dim, g.dx(l), res["phi"][l])
        for a in range(dim):
            np.testing.assert_allclose(F[a], -prob.g[a], rtol=0, atol=1e-10)
        if l > 0:
            assert res["cycles"][l] == 0


def test_box_axis_permutation():
    """Swapping the x and y axes of a 2-D box problem transposes the solution:
    a cell count or a rule taken from the wrong axis would break this."""
    g1 = W.box_geometry(2, (24, 12), (14, 8), (4, 2), dx0=1.0 / 24)
    g2 = W.box_geometry(2, (12, 24), (8, 14), (2, 4), dx0=1.0 / 24)
    c = (0.5, 0.27)
    w1 = W.Workload("a", g1, W.GaussianSum([(1.0, 0.15, c)]))
    w2 = W.Workload("b", g2, W.GaussianSum([(1.0, 0.15, (c[1], c[0]))]))
    r1 = core.solve(g1, *_inputs(w1), tol=1e-13, max_cycles=200)
    r2 = core.solve(g2, *_inputs(w2), tol=1e-13, max_cycles=200)
    assert r1["cycles"] == r2["cycles"]
    for l in range(2):
        np.testing.assert_allclose(r1["phi"][l], r2["phi"][l].T, rtol=0, atol=1e-12 * np.abs(r1["phi"][l]).max())
        F1 = core.forces(2, g1.dx(l), r1["phi"][l])
        F2 = core.forces(2, g2.dx(l), r2["phi"][l])
        np.testing.assert_allclose(F1[0], F2[1].T, rtol=0, atol=1e-10 * np.abs(F1[0]).max())


def test_box_second_order():
    """Second order of the composite force and potential errors on the 2-D box
    stack under grid doubling (Sec. 3)."""
    out = []
    for k in (1, 2, 4):
        wl = W.box_gaussian_2d(k)
        g, prob = wl.geom, wl.prob
        rho, po = _inputs(wl)
        res = core.solve(g, rho, po, tol=1e-11, max_cycles=100)
        assert res["status"] == 0
        ef, ep = [], []
        for l in range(g.nlevels):
            F = core.forces(2, g.dx(l), res["phi"][l])
            x = g.mesh_pad(l, 0)
            Fa = [a.numpy() for a in prob.force(*x)]
            ef.append(np.sqrt(sum((F[a] - Fa[a]) ** 2 for a in range(2))))
            ep.append(res["phi"][l][2:-2, 2:-2] - prob.phi(*x).numpy())
        out.append((norms.composite_norms(g, ef), norms.composite_norms(g, ep)))
    for (fa, pa), (fb, pb) in zip(out[:-1], out[1:]):
        for x, y in list(zip(fa, fb)) + list(zip(pa, pb)):
            assert norms.order(x, y) > 1.75, (fa, fb, pa, pb)


def test_unstable_ghost_gain_refused():
    """Where x_N falls just below 1 the right-ghost line is steep (N^0 = 194:
    c_7 = -63 on the second level from the top) and the lagged refresh makes
    the V-cycle diverge (contraction 2.8 per cycle measured in 2-D); such
    hierarchies are refused, cubes and boxes alike, while gains up to 6
    (c = 20.3 for N^0 = 198 in 2-D) are accepted and converge."""
    one, c = core.ghost_rule(194, 7, 2)
    assert not one and c == -63.0
    assert not core.plan_stable(2, (194, 194))
    assert not core.plan_stable(2, (322, 194))   # the box's y axis
    assert not core.plan_stable(3, (194, 194, 194))
    assert core.plan_stable(3, (194, 50, 66))      # z reaches one cell before L = 7
    assert core.plan_stable(2, (198, 198))
    assert core.plan_stable(3, (98, 98, 98))       # c = -31: gain 5.2 in 3-D
    assert not core.plan_stable(2, (98, 98))       # gain 7.75 in 2-D
    g = W.box_geometry(2, (192, 200), (8, 16), (2, 4), dx0=1.0 / 16)
    wl = W.Workload("unstable", g, W.GaussianSum([(1.0, 0.2, (0.5, 0.5))]))
    res = core.solve(g, *_inputs(wl))
    assert res["status_name"] == "invalid"

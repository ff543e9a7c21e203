"""Pins of the CPU oracle's operators against facts fixed by the paper and by
mathematics (no GPU).  Each test names the passage it pins."""
from fractions import Fraction

import numpy as np
import pytest

from conftest import read_table
from oracle import core, dense


# ------------------------------------------------------------ hierarchy (Sec. 2.2)
def test_hierarchy_worked_sizes():
    """Fig. 1d's N^0 = 10 and hand-worked rows of tests/golden/hierarchy.txt."""
    for row in read_table("hierarchy.txt"):
        N0 = int(row[0])
        want = [int(v) for v in row[2:]]
        assert core.plan(N0) == want


def test_hierarchy_brute_force_rational():
    """N^L = round(1/h^L), h^L = 2^L/N^0, ties up, evaluated in exact rationals."""
    for N0 in range(1, 1100):
        want = [N0]
        L = 0
        while want[-1] > 1:
            L += 1
            x = Fraction(N0, 2 ** L)
            want.append(int(x + Fraction(1, 2)))  # floor(x + 1/2) for x > 0
        assert core.plan(N0) == want, N0


def test_right_edge_lands_on_one_for_power_of_two_patches():
    """With N^0 = 2^k + 2 the level-2 right-most centre is exactly x_MG = 1
    (so the first branch of eqn:boundary_value is exercised)."""
    for k in range(3, 11):
        N0 = 2 ** k + 2
        NL = core.plan(N0)
        one, _ = core.ghost_rule(N0, 2, NL[2])
        assert one
        x = Fraction(2 * NL[2] - 1, 2) * Fraction(4, N0)
        assert x == 1


# ------------------------------------------------------------ ghost rule (Sec. 2.4)
def _mg_coords(N0, L, N):
    h = 2.0 ** L / N0
    return (np.arange(N + 2) - 0.5) * h, h  # centres of indices 0..N+1


@pytest.mark.parametrize("N0", [10, 66, 130, 258, 37, 1000])
def test_ghost_rule_reproduces_lines_vanishing_at_the_edges(N0):
    """The left rule is exact for e = a x (zero at x_MG = 0); the right rule for
    e = b (1 - x) (zero at x_MG = 1), on both branches."""
    NL = core.plan(N0)
    for L in range(1, len(NL)):
        N = NL[L]
        if N < 2:
            continue
        x, h = _mg_coords(N0, L, N)
        e = np.zeros((N + 2, N + 2))
        # along x only: rows of the 2-D array carry the 1-D profile
        e[1:N + 1, 1:N + 1] = 3.0 * (1.0 - x[None, 1:N + 1])
        core.ghost_fill(2, N0, L, e)
        np.testing.assert_allclose(e[1:N + 1, N + 1], 3.0 * (1.0 - x[N + 1]), rtol=1e-12, atol=1e-13)
        e[1:N + 1, 1:N + 1] = 2.0 * x[None, 1:N + 1]
        core.ghost_fill(2, N0, L, e)
        np.testing.assert_allclose(e[1:N + 1, 0], 2.0 * x[0], rtol=1e-12)


def test_ghost_gain_bounded_and_literal_rule_unstable():
    """The reading used has |gain| <= 1 on every level; the factor exactly as
    printed exceeds 1 (e.g. 8 at N^0 = 10, L = 1)."""
    for N0 in [10, 66, 130, 258, 514]:
        NL = core.plan(N0)
        for L in range(1, len(NL)):
            one, c = core.ghost_rule(N0, L, NL[L])
            if not one:
                assert abs(c) <= 1.0
    one, c = core.ghost_rule(10, 1, 5, literal=True)
    assert not one and c == pytest.approx(8.0)


def test_literal_ghost_rule_breaks_the_solve():
    """Negative test planted in the oracle: the printed factor makes the
    iteration diverge or stall, the reading converges."""
    from paper_2001_02327_amd import workloads as W
    wl = W.paper3d(16)
    rho, po = W.make_inputs(wl.geom, wl.prob)
    rho = [r.numpy() for r in rho]
    ok = core.solve(wl.geom, rho, po.numpy(), max_cycles=40)
    bad = core.solve(wl.geom, rho, po.numpy(), max_cycles=40, ghost_literal=True)
    assert ok["status"] == 0
    assert bad["status"] != 0


def test_ghost_fill_corners_compose_axis_rules():
    """Edges and corners get the 1-D rule of every axis they are ghosts on."""
    N0, L = 130, 3
    N = core.plan(N0)[L]
    _, c = core.ghost_rule(N0, L, N)
    rng = np.random.default_rng(1)
    e = np.zeros((N + 2,) * 3)
    e[1:-1, 1:-1, 1:-1] = rng.standard_normal((N,) * 3)
    core.ghost_fill(3, N0, L, e)
    assert e[0, 0, 0] == pytest.approx(-e[1, 1, 1])
    assert e[N + 1, N + 1, N + 1] == pytest.approx(c ** 3 * e[N, N, N])
    assert e[0, N + 1, 0] == pytest.approx(c * e[1, N, 1])
    assert e[5, 0, N + 1] == pytest.approx(-c * e[5, 1, N])


# ------------------------------------------------------------ smoother (Sec. 2.3)
def test_rb_sweep_worked_example():
    """tests/golden/rb_sweep_2d_2x2.txt, worked by hand."""
    u = np.ones((4, 4))
    u[1:3, 1:3] = 0.0
    f = np.zeros((4, 4))
    for row in read_table("rb_sweep_2d_2x2.txt"):
        core.rb_sweep(2, 2, 0, 1.0, u, f)
        want = [float(v) for v in row[1:]]
        got = [u[1, 1], u[1, 2], u[2, 1], u[2, 2]]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_quadratic_is_solved_exactly(dim):
    """eqn:Laplacian2D/3D is exact on quadratics, so a patch with Phi = |x|^2
    on its ghost layer and f = 2d converges to |x|^2 at every centre."""
    N0 = 10 if dim == 3 else 22
    h = 1.0 / N0
    x = (np.arange(N0 + 2) - 0.5) * h
    if dim == 3:
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        exact = X ** 2 + Y ** 2 + Z ** 2
    else:
        Y, X = np.meshgrid(x, x, indexing="ij")
        exact = X ** 2 + Y ** 2
    u = exact.copy()
    u[(slice(1, -1),) * dim] = 0.0
    f = np.full_like(u, 2.0 * dim)
    for _ in range(40):
        core.vcycle_patch(dim, h, u, f)
    np.testing.assert_allclose(u, exact, rtol=0, atol=1e-12)


# ------------------------------------------------------------ restriction / prolongation
def _bilinear_weights_appendix(tx, ty):
    """Appendix A, (A1): the bilinear interpolant through corners A(x1,y1), B(x2,y1),
    C(x2,y2), D(x1,y2), evaluated at x - x1 = tx dx, y - y1 = ty dx."""
    return dict(A=(1 - tx) * (1 - ty), B=tx * (1 - ty), C=tx * ty, D=(1 - tx) * ty)


def test_prolongation_weights_match_appendix_a():
    """A unit value at one coarse cell, prolonged, gives the (A1) weights at
    the quarter points: 9/16, 3/16, 3/16, 1/16 (eqn:prolongation2D)."""
    Nc, Nf = 4, 8
    for (ci, cj) in [(2, 2)]:
        ec = np.zeros((Nc + 2, Nc + 2))
        ec[cj, ci] = 1.0
        uf = np.zeros((Nf + 2, Nf + 2))
        core.prolong_add(2, ec, uf)
        # fine cell (3,3) is the left/bottom child of coarse (2,2); its other coarse
        # neighbours are (1,2),(2,1),(1,1); coarse (2,2) is nearest -> weight of corner at
        # distance (0.25, 0.25) in units of the coarse spacing.
        w = _bilinear_weights_appendix(0.75, 0.75)  # fine point 3/4 of the way from (1,1) to (2,2)
        assert uf[3, 3] == pytest.approx(w["C"])
        assert uf[3, 3] == pytest.approx(9 / 16)
        assert uf[3, 2] == pytest.approx(3 / 16)   # fine (i=2, j=3): right child of coarse 1
        assert uf[2, 2] == pytest.approx(1 / 16)
    # weights of every fine cell sum to one for a constant coarse field
    ec = np.ones((Nc + 2, Nc + 2))
    uf = np.zeros((Nf + 2, Nf + 2))
    core.prolong_add(2, ec, uf)
    np.testing.assert_allclose(uf[1:-1, 1:-1], 1.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_prolongation_exact_on_linear_functions(dim):
    """Appendix A: the (bi/tri)linear interpolant reproduces linear functions."""
    Nc, Nf = 6, 12
    hc, hf = 2.0, 1.0
    xc = (np.arange(Nc + 2) - 0.5) * hc
    xf = (np.arange(Nf + 2) - 0.5) * hf
    g = [0.3, -1.7, 2.2]
    if dim == 3:
        Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
        ec = 1.0 + g[0] * X + g[1] * Y + g[2] * Z
        Z, Y, X = np.meshgrid(xf, xf, xf, indexing="ij")
        want = 1.0 + g[0] * X + g[1] * Y + g[2] * Z
    else:
        Y, X = np.meshgrid(xc, xc, indexing="ij")
        ec = 1.0 + g[0] * X + g[1] * Y
        Y, X = np.meshgrid(xf, xf, indexing="ij")
        want = 1.0 + g[0] * X + g[1] * Y
    uf = np.zeros((Nf + 2,) * dim)
    core.prolong_add(dim, np.ascontiguousarray(ec), uf)
    inner = (slice(1, -1),) * dim
    np.testing.assert_allclose(uf[inner], want[inner], rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_restriction_mean_and_overhang(dim):
    """eqn:restriction2D/3D: the coarse value is the mean of the 2^d children;
    exact on linear functions; children beyond the active range count as zero."""
    Nf, Nc = 8, 4
    xf = (np.arange(Nf + 2) - 0.5)
    xc = (np.arange(Nc + 2) - 0.5) * 2
    if dim == 3:
        Z, Y, X = np.meshgrid(xf, xf, xf, indexing="ij")
        r = 2.0 + X - 3 * Y + 0.5 * Z
        Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
        want = 2.0 + X - 3 * Y + 0.5 * Z
    else:
        Y, X = np.meshgrid(xf, xf, indexing="ij")
        r = 2.0 + X - 3 * Y
        Y, X = np.meshgrid(xc, xc, indexing="ij")
        want = 2.0 + X - 3 * Y
    fc = core.restrict(dim, np.ascontiguousarray(r), Nc)
    inner = (slice(1, -1),) * dim
    np.testing.assert_allclose(fc[inner], want[inner], rtol=0, atol=1e-12)
    # overhang: 9 fine cells -> 5 coarse cells; the 5th covers fine 9 and 10 (ghost)
    Nf, Nc = 9, 5
    r = np.zeros((Nf + 2,) * dim)
    r[(slice(1, -1),) * dim] = 1.0
    r[(slice(Nf + 1, Nf + 2),) + (slice(None),) * (dim - 1)] = 100.0  # ghost values are ignored
    fc = core.restrict(dim, r, Nc)
    last = (Nc,) * dim
    assert fc[last] == pytest.approx(0.5 ** dim)
    assert fc[(1,) * dim] == pytest.approx(1.0)


# ------------------------------------------------------------ force stencil
@pytest.mark.parametrize("dim", [2, 3])
def test_force_stencil_exact_on_quartics(dim):
    """Eqn:force_evaluation is fourth-order: exact for polynomials of degree <= 4."""
    n, dx = 12, 0.1
    x = (np.arange(n + 4) - 2 + 0.5) * dx - 0.3
    if dim == 3:
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        phi = X ** 4 - 2 * Y ** 3 * X + Z ** 4 * 0.5 + X * Y * Z
        want = (-(4 * X ** 3 - 2 * Y ** 3 + Y * Z), -(-6 * Y ** 2 * X + X * Z), -(2 * Z ** 3 + X * Y))
    else:
        Y, X = np.meshgrid(x, x, indexing="ij")
        phi = X ** 4 - 2 * Y ** 3 * X + 3 * X * Y
        want = (-(4 * X ** 3 - 2 * Y ** 3 + 3 * Y), -(-6 * Y ** 2 * X + 3 * X))
    phi = np.ascontiguousarray(phi)
    got = core.forces(dim, dx, phi)
    got2 = dense.forces(dim, dx, phi)
    inner = (slice(2, n + 2),) * dim
    for a in range(dim):
        np.testing.assert_allclose(got[a], want[a][inner], rtol=0, atol=1e-11)
        np.testing.assert_allclose(got2[a], want[a][inner], rtol=0, atol=1e-11)

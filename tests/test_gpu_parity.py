"""Parity of the HIP path (through the C ABI) with the CPU oracle.

FP64 tolerance: the GPU and the oracle run the same schedule but sum in a
different order and the GPU contracts multiply-adds, so each operator differs
by a few ulps; the iteration is contractive, so after k cycles the potentials
differ by O(k * 1e-16) relative.  The bar is 1e-12 relative (max norm, scaled
by max |Phi|) for the potential and 1e-11 for the forces (the force stencil
divides differences by 12 dx, amplifying the potential's rounding by up to
~|Phi| / (|F| dx)).
"""
import math

import numpy as np
import pytest
import torch

from oracle import core
from paper_2001_02327_amd import _lib
from paper_2001_02327_amd import workloads as W
from paper_2001_02327_amd.solver import NestedPoissonSolver

pytestmark = pytest.mark.gpu

PHI_RTOL = 1e-12
F_RTOL = 1e-11


@pytest.fixture(autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need the MI355X"


def _inputs(wl, device):
    return W.make_inputs(wl.geom, wl.prob, device=device)


def gpu_solve(wl, fixed=None, allow_notconv=False, **kw):
    dev = torch.device("cuda")
    rho, po = _inputs(wl, dev)
    s = NestedPoissonSolver(wl.geom, **kw)
    if fixed is not None:
        s.set_fixed_cycles(fixed)
    st = s.solve(rho, po, allow_notconv=allow_notconv)
    phi = [s.potential(l).cpu().numpy() for l in range(wl.geom.nlevels)]
    F = [tuple(a.cpu().numpy() for a in s.forces(l)) for l in range(wl.geom.nlevels)]
    hist = [s.history(l) for l in range(wl.geom.nlevels)]
    torch.cuda.synchronize()
    s.close()
    return phi, F, st, hist


def oracle_solve(wl, fixed=None, **kw):
    rho, po = _inputs(wl, "cpu")
    res = core.solve(wl.geom, [r.numpy() for r in rho], po.numpy(), fixed_cycles=fixed, **kw)
    F = [core.forces(wl.geom.dim, wl.geom.dx(l), res["phi"][l]) for l in range(wl.geom.nlevels)]
    return res, F


def assert_parity(wl, phi_g, F_g, res, F_o, phi_rtol=PHI_RTOL, f_rtol=F_RTOL):
    for l in range(wl.geom.nlevels):
        a, b = phi_g[l], res["phi"][l]
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
        assert err <= phi_rtol, ("phi", l, err)
        fmax = max(np.abs(x).max() for x in F_o[l])
        for ax in range(wl.geom.dim):
            e = np.abs(F_g[l][ax] - F_o[l][ax]).max() / max(fmax, 1e-300)
            assert e <= f_rtol, ("F", l, ax, e)


def _ragged3d():
    # non-power-of-two patches: N^0 = 12 and 24 give hierarchies 12,6,3,2,1 and 24,12,6,3,2,1
    g = W.Geometry(dim=3, n=[22, 10], off=[(0, 0, 0), (4, 3, 6)], lo0=(-0.5, -0.5, -0.5), dx0=1.0 / 22)
    return W.Workload("ragged3d_22_10", g, W.Plummer([(1.0, 0.08, (0.05, -0.02, 0.03))]))


def _ragged2d():
    g = W.Geometry(dim=2, n=[30, 14, 6], off=[(0, 0, 0), (5, 9, 0), (3, 2, 0)], lo0=(-0.5, -0.5, 0.0),
                   dx0=1.0 / 30, G=1.0)
    return W.Workload("ragged2d_30_14_6", g, W.Gaussian(0.15, 1.0))


def _minimal():
    g = W.Geometry(dim=3, n=[8, 4], off=[(0, 0, 0), (2, 2, 2)], lo0=(-0.5, -0.5, -0.5), dx0=1.0 / 8)
    return W.Workload("minimal3d_8_4", g, W.Plummer([(1.0, 0.2, (0.0, 0.0, 0.0))]))


SMALL = [W.paper2d(16), W.c1_gaussian_2d(32), W.c1_gaussian_2d(64), W.paper3d(16), W.c2_plummer(16), W.c4_multi_plummer(5, N=16),
         W.c3_plummer_offset(16), _ragged3d(), _ragged2d(), _minimal(), W.paper2d(8), W.c2_plummer(32)]


@pytest.mark.parametrize("wl", SMALL, ids=lambda w: w.name)
def test_pinned_cycle_parity(wl):
    """Same cycle count per level as the oracle's own stop: potentials and forces agree."""
    res, F_o = oracle_solve(wl)
    assert res["status"] == 0
    phi_g, F_g, st, _ = gpu_solve(wl, fixed=res["cycles"])
    assert st["cycles"] == res["cycles"]
    assert_parity(wl, phi_g, F_g, res, F_o)


@pytest.mark.parametrize("wl", [W.paper2d(16), W.c2_plummer(16), _ragged3d()], ids=lambda w: w.name)
def test_stop_rule_matches_oracle(wl):
    """With the residual stop rule the GPU takes the oracle's cycle counts and
    stops below the tolerance."""
    res, F_o = oracle_solve(wl)
    phi_g, F_g, st, hist = gpu_solve(wl)
    for l in range(wl.geom.nlevels):
        assert abs(st["cycles"][l] - res["cycles"][l]) <= 1
        assert st["final_rel_residual"][l] <= 1e-10
        np.testing.assert_allclose(hist[l][: len(res["hist"][l])][:3], res["hist"][l][:3], rtol=1e-9)
    if st["cycles"] == res["cycles"]:
        assert_parity(wl, phi_g, F_g, res, F_o)


@pytest.mark.parametrize("wl", [W.paper2d(32), W.paper3d(16)], ids=lambda w: w.name)
def test_force_change_stop_rule(wl):
    """The paper's rule max|F^q - F^{q-1}| < 1e-10 (Sec. 3.1)."""
    res, F_o = oracle_solve(wl, stop_rule=1)
    phi_g, F_g, st, _ = gpu_solve(wl, stop_rule="force_delta")
    for l in range(wl.geom.nlevels):
        assert abs(st["cycles"][l] - res["cycles"][l]) <= 1
    if st["cycles"] == res["cycles"]:
        assert_parity(wl, phi_g, F_g, res, F_o)


@pytest.mark.parametrize("wl", [W.paper2d(1024), W.paper3d(128)], ids=lambda w: w.name)
def test_paper_problems_largest_sizes(wl):
    """The paper's 2-D problem at its largest N (4 levels of 1024^2, finest
    spacing 1/8192) and its 3-D problem at N = 128, under the paper's own
    force-change rule: full-array parity at the oracle's cycle counts, and the
    GPU's own stop within one cycle of the oracle's on every level."""
    res, F_o = oracle_solve(wl, stop_rule=1)
    assert res["status"] == 0
    phi_g, F_g, _, _ = gpu_solve(wl, fixed=res["cycles"])
    assert_parity(wl, phi_g, F_g, res, F_o)
    _, _, st, _ = gpu_solve(wl, stop_rule="force_delta")
    for l in range(wl.geom.nlevels):
        assert abs(st["cycles"][l] - res["cycles"][l]) <= 1, (st["cycles"], res["cycles"])


@pytest.mark.parametrize("wl", [W.paper2d(16), W.paper3d(8), _ragged3d()], ids=lambda w: w.name)
def test_cycle_by_cycle(wl):
    """After 0, 1, 2 and 3 cycles on level 0 (and the interface fill alone on
    finer levels) the iterates agree: every kernel of one V-cycle is checked."""
    L = wl.geom.nlevels
    for k in range(4):
        fixed = [k] + [min(k, 1)] * (L - 1)
        res, F_o = oracle_solve(wl, fixed=fixed)
        phi_g, F_g, st, _ = gpu_solve(wl, fixed=fixed)
        assert_parity(wl, phi_g, F_g, res, F_o)


@pytest.mark.parametrize("n_pre,n_post", [(1, 1), (3, 2), (0, 2), (2, 0)])
def test_other_smoothing_counts(n_pre, n_post):
    """Other smoothing counts; n_post = 0 takes the full (both-colour)
    prolongation into level 0, n_post > 0 the black-only one."""
    wl = W.c2_plummer(16)
    res, F_o = oracle_solve(wl, n_pre=n_pre, n_post=n_post, max_cycles=120)
    phi_g, F_g, st, _ = gpu_solve(wl, fixed=res["cycles"], n_pre=n_pre, n_post=n_post, max_cycles=120)
    assert_parity(wl, phi_g, F_g, res, F_o)


@pytest.mark.parametrize("wl", [W.c2_plummer(16), _ragged3d(), W.paper2d(16)], ids=lambda w: w.name)
def test_coarse_post_parity(wl):
    """V(1,1) on multigrid level 0 with two post-smoothing sweeps below it
    (np_config.coarse_post; the coarse tail takes the count too): the iterates
    after one and two cycles on level 0 and at the oracle's own stop equal the
    oracle's with the same schedule."""
    L = wl.geom.nlevels
    kw = dict(n_pre=1, n_post=1, coarse_post=2)
    for k in (1, 2):
        fixed = [k] + [min(k, 1)] * (L - 1)
        res, F_o = oracle_solve(wl, fixed=fixed, **kw)
        phi_g, F_g, st, _ = gpu_solve(wl, fixed=fixed, **kw)
        assert_parity(wl, phi_g, F_g, res, F_o)
    res, F_o = oracle_solve(wl, max_cycles=120, **kw)
    assert res["status"] == 0
    phi_g, F_g, st, _ = gpu_solve(wl, fixed=res["cycles"], max_cycles=120, **kw)
    assert_parity(wl, phi_g, F_g, res, F_o)


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_potential_zero_density(dim):
    """rho = 0, Phi linear: exact on every level (stop scale from the boundary residual)."""
    geom = W.centred_geometry(dim, 3, 16, 0.5, 1.0)
    wl = W.Workload("linear", geom, W.Linear([0.7, -1.3, 0.4][:dim], 2.0))
    phi_g, F_g, st, _ = gpu_solve(wl, tol=1e-13, max_cycles=80)
    for l in range(geom.nlevels):
        x = geom.mesh(l, -2, geom.n[l] + 4)
        np.testing.assert_allclose(phi_g[l], wl.prob.phi(*x).numpy(), rtol=0, atol=2e-11)
        for a in range(dim):
            np.testing.assert_allclose(F_g[l][a], -wl.prob.g[a], rtol=0, atol=1e-9)
        if l > 0:
            assert st["cycles"][l] == 0


def test_error_paths():
    wl = W.c2_plummer(16)
    dev = torch.device("cuda")
    rho, po = _inputs(wl, dev)
    s = NestedPoissonSolver(wl.geom)
    with pytest.raises(_lib.NestedPoissonError) as e:
        s.forces(0)
    assert e.value.code == _lib.NP_ESTATE
    bad = [r.clone() for r in rho]
    bad[1][3, 4, 5] = float("nan")
    with pytest.raises(_lib.NestedPoissonError) as e:
        s.solve(bad, po)
    assert e.value.code == _lib.NP_ENONFINITE
    s.close()
    s = NestedPoissonSolver(wl.geom, max_cycles=1)
    st = s.solve(rho, po, allow_notconv=True)
    assert st["status"] == _lib.NP_ENOTCONV and st["cycles"][0] == 1
    s.close()
    with pytest.raises(TypeError):
        NestedPoissonSolver(wl.geom).solve([r.float() for r in rho], po)


def test_determinism_and_reuse():
    """Two solves on one handle are bitwise identical (colours are independent,
    reductions are order-free maxima)."""
    wl = W.c4_multi_plummer(11, N=32)
    dev = torch.device("cuda")
    rho, po = _inputs(wl, dev)
    s = NestedPoissonSolver(wl.geom)
    s.solve(rho, po)
    a = [s.potential(l).clone() for l in range(3)]
    s.solve(rho, po)
    b = [s.potential(l).clone() for l in range(3)]
    s.close()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_plummer_128_full_parity():
    """Three levels of 128^3 (the 3-D Plummer workload, a = 0.05): full-array
    parity with the oracle at the oracle's cycle counts."""
    wl = W.c2_plummer(128)
    res, F_o = oracle_solve(wl)
    assert res["status"] == 0
    phi_g, F_g, st, _ = gpu_solve(wl, fixed=res["cycles"])
    assert_parity(wl, phi_g, F_g, res, F_o)


def _deepest(dim):
    # the largest number of levels a solve takes: 16 patches of 8^d, each half
    # its parent's width, around a Plummer core of the finest level's size
    g = W.centred_geometry(dim, 16, 8, 0.5, 1.0)
    if dim == 2:
        terms = [(1.0, 0.5 ** k, (0.0, 0.0)) for k in (2, 5, 8, 11, 14)]
        return W.Workload("deepest2d_16x8", g, W.GaussianSum(terms))
    return W.Workload("deepest3d_16x8", g, W.Plummer([(1.0, 0.5 ** 13, (0.0, 0.0, 0.0))]))


@pytest.mark.parametrize("dim", [2, 3])
def test_maximum_depth_parity(dim):
    """Sixteen nested levels (the library's limit, 2^15 between the coarsest
    and finest spacing): cycle counts of the stop rule within one of the
    oracle's, and at the oracle's counts potentials and forces to the FP64 bars."""
    wl = _deepest(dim)
    res, F_o = oracle_solve(wl)
    assert res["status"] == 0
    phi_g, F_g, st, _ = gpu_solve(wl, fixed=res["cycles"])
    assert_parity(wl, phi_g, F_g, res, F_o)
    _, _, st_s, _ = gpu_solve(wl)
    for l in range(16):
        assert abs(st_s["cycles"][l] - res["cycles"][l]) <= 1
        assert st_s["final_rel_residual"][l] <= 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_maximum_depth_interp_buffer(dim):
    """The comparison scheme of Sec. 4 over sixteen nested levels (each level
    l >= 1 relaxes only Omega^l = 8^d cells between interpolated buffer layers):
    potentials and forces to the FP64 bars at the oracle's cycle counts."""
    wl = _deepest(dim)
    res, F_o = oracle_solve(wl, buffer_interp=True)
    assert res["status"] == 0
    phi_g, F_g, st, _ = gpu_solve(wl, fixed=res["cycles"], buffer="interp")
    assert_parity(wl, phi_g, F_g, res, F_o)


# ------------------------------------------------ comparison scheme of Sec. 4
INTERP_BUFFER = [W.paper2d(16), W.paper3d(16), W.c2_plummer(16), W.c3_plummer_offset(16), _ragged3d(), _ragged2d(),
                 _minimal()]


@pytest.mark.parametrize("wl", INTERP_BUFFER, ids=lambda w: w.name)
def test_interp_buffer_parity(wl):
    """Both buffer layers of levels l >= 1 interpolated and only Omega^l
    relaxed (its own hierarchy from N^0 = n): same cycle counts as the oracle's
    stop, potentials and forces to the FP64 bars."""
    res, F_o = oracle_solve(wl, buffer_interp=True)
    assert res["status"] == 0
    phi_g, F_g, st, _ = gpu_solve(wl, fixed=res["cycles"], buffer="interp")
    assert_parity(wl, phi_g, F_g, res, F_o)
    phi_s, F_s, st_s, _ = gpu_solve(wl, buffer="interp")
    for l in range(wl.geom.nlevels):
        assert abs(st_s["cycles"][l] - res["cycles"][l]) <= 1
        assert st_s["final_rel_residual"][l] <= 1e-10
    if st_s["cycles"] == res["cycles"]:
        assert_parity(wl, phi_s, F_s, res, F_o)


@pytest.mark.parametrize("wl", [W.paper2d(16), _ragged3d()], ids=lambda w: w.name)
def test_interp_buffer_cycle_by_cycle(wl):
    """0, 1 and 2 cycles per level with the interpolated buffer: the copies into
    and out of the relaxed domain and every V-cycle kernel on it agree."""
    L = wl.geom.nlevels
    for k in range(3):
        fixed = [k] * L
        res, F_o = oracle_solve(wl, fixed=fixed, buffer_interp=True)
        phi_g, F_g, st, _ = gpu_solve(wl, fixed=fixed, buffer="interp")
        assert_parity(wl, phi_g, F_g, res, F_o)


def test_interp_buffer_reuse_and_level0():
    """Two solves on one handle are identical; level 0 equals the relaxed
    scheme's bit for bit (the buffer mode concerns levels l >= 1 only)."""
    wl = W.c4_multi_plummer(11, N=32)
    dev = torch.device("cuda")
    rho, po = _inputs(wl, dev)
    s = NestedPoissonSolver(wl.geom, buffer="interp")
    s.solve(rho, po)
    a = [s.potential(l).clone() for l in range(3)]
    s.solve(rho, po)
    b = [s.potential(l).clone() for l in range(3)]
    s.close()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    s = NestedPoissonSolver(wl.geom)
    s.solve(rho, po)
    assert torch.equal(s.potential(0), a[0])
    s.close()


# ------------------------------------------------ several patches per level
TREES = [W.two_patch_2d(32), W.two_patch_2d(32, "middle"), W.two_patch_3d(16), W.two_patch_3d(32, "middle")]


@pytest.mark.parametrize("wl", TREES, ids=lambda w: w.name)
def test_patch_tree_parity(wl):
    """A tree of patches (two on level 1, one on level 2): with the oracle's
    cycle counts and with the stop rule, potentials and forces of every patch
    agree with the oracle."""
    res, F_o = oracle_solve(wl)
    assert res["status"] == 0
    phi_g, F_g, st, _ = gpu_solve(wl, fixed=res["cycles"])
    assert_parity(wl, phi_g, F_g, res, F_o)
    phi_s, F_s, st_s, _ = gpu_solve(wl)
    for l in range(wl.geom.nlevels):
        assert abs(st_s["cycles"][l] - res["cycles"][l]) <= 1
        assert st_s["final_rel_residual"][l] <= 1e-10
    if st_s["cycles"] == res["cycles"]:
        assert_parity(wl, phi_s, F_s, res, F_o)


def test_patch_tree_paths_match_stacks():
    """Each root-to-leaf path of the tree, solved on the GPU as a stack of one
    patch per level, gives the tree's potentials bit for bit."""
    wl = W.two_patch_3d(32)
    g = wl.geom
    phi_t, _, st_t, _ = gpu_solve(wl)
    dev = torch.device("cuda")
    rho, po = _inputs(wl, dev)
    for path in ([0, 1, 3], [0, 2]):
        chain = W.Geometry(dim=3, n=[g.n[l] for l in path], off=[g.off[l] for l in path], lo0=g.lo0, dx0=g.dx0,
                           G=g.G)
        s = NestedPoissonSolver(chain)
        st = s.solve([rho[l] for l in path], po)
        for k, l in enumerate(path):
            assert torch.equal(s.potential(k).cpu(), torch.from_numpy(phi_t[l])), (path, l)
            assert st["cycles"][k] == st_t["cycles"][l]
        s.close()


def test_patch_tree_with_interp_buffer():
    """The two extensions together: a tree of patches solved with both buffer
    layers interpolated (each patch from its own parent) agrees with the oracle."""
    wl = W.two_patch_3d(16, "middle")
    res, F_o = oracle_solve(wl, buffer_interp=True)
    assert res["status"] == 0
    phi_g, F_g, st, _ = gpu_solve(wl, fixed=res["cycles"], buffer="interp")
    assert_parity(wl, phi_g, F_g, res, F_o)


def test_patch_tree_force_change_stop():
    """The paper's force-change stop rule on a tree, FP64 and FP16-storage
    defect correction: cycle counts within one of the oracle's, and the FP16
    path reaches the oracle's potential to the defect-correction bar."""
    wl = W.two_patch_2d(32)
    res, F_o = oracle_solve(wl, stop_rule=1)
    assert res["status"] == 0
    phi_g, F_g, st, _ = gpu_solve(wl, stop_rule="force_delta")
    for l in range(wl.geom.nlevels):
        assert abs(st["cycles"][l] - res["cycles"][l]) <= 1
    if st["cycles"] == res["cycles"]:
        assert_parity(wl, phi_g, F_g, res, F_o)
    phi_h, _, st_h, _ = gpu_solve(wl, stop_rule="force_delta", precision="fp16s_dc", inner_cycles="adaptive")
    for l in range(wl.geom.nlevels):
        err = np.abs(phi_h[l] - res["phi"][l]).max() / np.abs(res["phi"][l]).max()
        assert err <= 1e-8, (l, err)

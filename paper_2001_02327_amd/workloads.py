"""Seeded synthetic inputs: nested geometries and closed-form density/potential
pairs.  This module holds the problem definitions only (geometry, densities,
analytic potentials and forces); it contains none of the solver's arithmetic,
so both the HIP path and the CPU oracle can take their inputs from it.

Problems
  * Paper2D   -- the 2-D model of Sec. 3.1: sigma = 4 R0^2/(R^2+R0^2)^2,
                 Phi = ln(R^2/R0^2 + 1), G = 1/(4 pi), R0 = 0.3.
  * Paper3D   -- the 3-D model of Sec. 3.2: rho = rho0 (1 - r^2/r0^2)^2 inside
                 r0, piecewise closed-form Phi and f_r, G = 1.
  * Plummer   -- superposed Plummer spheres, rho = 3M/(4 pi a^3) (1+r^2/a^2)^(-5/2),
                 Phi = -G M / sqrt(r^2+a^2) (textbook pair).
  * Gaussian  -- manufactured Phi = exp(-r^2/s^2), rho = lap(Phi)/(4 pi G).

Geometries follow Sec. 2.1: level l has n_l cells per axis of size
dx0 / 2^l; its lower corner sits `off[l]` coarse cells above that of level
l-1.  Level-0 boundary data (outer buffer potential, inner-buffer density) are
taken from the closed form.

Arrays are torch float64 tensors indexed [k, j, i] (x fastest); they can be
built on any device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch


# ------------------------------------------------------------------ geometry
@dataclass
class Geometry:
    dim: int
    n: List                           # cells of Omega^l: an int (the same along every
                                      # axis) or a tuple per axis (x, y[, z])
    off: List[Tuple[int, int, int]]   # l >= 1: corner offset in coarse cells (off[0] unused)
    lo0: Tuple[float, float, float]   # physical lower corner of Omega^0
    dx0: float
    G: float = 1.0
    # l >= 1: the entry patch l is refined out of (an earlier one); None = the
    # stack of one patch per level (parent l - 1); a tree gives several
    # disjoint patches per level, off[l] counted in cells of the parent
    parent: Optional[List[int]] = None

    @property
    def nlevels(self) -> int:
        return len(self.n)

    def ext(self, l: int) -> Tuple[int, ...]:
        """Cells of Omega^l along x, y[, z]."""
        n = self.n[l]
        if isinstance(n, (tuple, list)):
            assert len(n) == self.dim
            return tuple(int(v) for v in n)
        return (int(n),) * self.dim

    @property
    def cubic(self) -> bool:
        return all(len(set(self.ext(l))) == 1 for l in range(self.nlevels))

    def shape(self, l: int, pad: int = 0) -> Tuple[int, ...]:
        """Array shape [k, j, i] of Omega^l with `pad` extra cells on every side."""
        return tuple(v + 2 * pad for v in reversed(self.ext(l)))

    def par(self, l: int) -> int:
        return self.parent[l] if self.parent is not None else l - 1

    def depth(self, l: int) -> int:
        k = 0
        while l > 0:
            l = self.par(l)
            k += 1
        return k

    def children(self, l: int) -> List[int]:
        return [m for m in range(1, self.nlevels) if self.par(m) == l]

    def dx(self, l: int) -> float:
        return self.dx0 / (1 << self.depth(l))

    def lo(self, l: int) -> Tuple[float, ...]:
        if l == 0:
            return tuple(self.lo0[: self.dim])
        p = self.par(l)
        base = self.lo(p)
        return tuple(base[a] + self.off[l][a] * self.dx(p) for a in range(self.dim))

    def centres(self, l: int, first: int, count, device="cpu"):
        """Per-axis cell-centre coordinates for Omega^l cell indices first..first+count-1
        (index -2 = outer buffer layer, -1 = inner buffer layer); `count` is an
        int or one count per axis."""
        lo = self.lo(l)
        dx = self.dx(l)
        cnt = tuple(count) if isinstance(count, (tuple, list)) else (count,) * self.dim
        out = []
        for a in range(self.dim):
            i = torch.arange(first, first + cnt[a], dtype=torch.float64, device=device)
            out.append(lo[a] + (i + 0.5) * dx)
        return out

    def mesh_pad(self, l: int, pad: int = 0, device="cpu"):
        """Coordinate arrays of Omega^l with `pad` cells on every side."""
        return self.mesh(l, -pad, tuple(v + 2 * pad for v in self.ext(l)), device)

    def mesh(self, l: int, first: int, count, device="cpu"):
        """Coordinate arrays (x, y[, z]) broadcast to [k, j, i] shape."""
        ax = self.centres(l, first, count, device)
        if self.dim == 3:
            z, y, x = torch.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
            return x, y, z
        y, x = torch.meshgrid(ax[1], ax[0], indexing="ij")
        return x, y

    def describe(self) -> dict:
        d = dict(dim=self.dim, n=[list(v) if isinstance(v, (tuple, list)) else v for v in self.n],
                 off=[list(o) for o in self.off], lo0=list(self.lo0[: self.dim]),
                 dx0=self.dx0, G=self.G)
        if self.parent is not None:
            d["parent"] = list(self.parent)
        return d


def centred_geometry(dim: int, nlevels: int, N: int, half_width0: float, G: float) -> Geometry:
    """Levels of N cells each, level l covering [-w/2^l, w/2^l]^d (each level
    half the extent of the previous, so the offset is N/4 coarse cells)."""
    if N % 4:
        raise ValueError("N must be a multiple of 4 for centred nesting")
    off = [(0, 0, 0)] + [(N // 4,) * 3 for _ in range(1, nlevels)]
    return Geometry(dim=dim, n=[N] * nlevels, off=off, lo0=(-half_width0,) * 3, dx0=2 * half_width0 / N, G=G)


# ------------------------------------------------------------------ problems
class Problem:
    """Closed-form density/potential/force triple."""
    G: float = 1.0

    def rho(self, *x):
        raise NotImplementedError

    def phi(self, *x):
        raise NotImplementedError

    def force(self, *x):
        """Analytic F = -grad(Phi), tuple of d arrays."""
        raise NotImplementedError


class Paper2D(Problem):
    """Sec. 3.1 model (G = 1/(4 pi), so 4 pi G rho = sigma)."""

    def __init__(self, R0: float = 0.3):
        self.R0 = R0
        self.G = 1.0 / (4.0 * math.pi)

    def rho(self, x, y):
        R2 = x * x + y * y
        return 4 * self.R0 ** 2 / (R2 + self.R0 ** 2) ** 2

    def phi(self, x, y):
        return torch.log((x * x + y * y) / self.R0 ** 2 + 1.0)

    def force(self, x, y):
        R2 = x * x + y * y
        g = 2.0 / (R2 + self.R0 ** 2)   # f_R / R
        return (-g * x, -g * y)

    def fR(self, x, y):
        """The paper's radial acceleration f_R = |grad Phi| (positive)."""
        R = torch.sqrt(x * x + y * y)
        return 2 * R / (R * R + self.R0 ** 2)


class Paper3D(Problem):
    """Sec. 3.2 model: n = 2 polytrope-like ball, G = 1."""

    def __init__(self, rho0: float = 1.0, r0: float = 0.25):
        self.rho0, self.r0 = rho0, r0
        self.G = 1.0
        self.M = 32 * math.pi * rho0 * r0 ** 3 / 105

    def rho(self, x, y, z):
        r2 = x * x + y * y + z * z
        inside = r2 <= self.r0 ** 2
        return torch.where(inside, self.rho0 * (1 - r2 / self.r0 ** 2) ** 2, torch.zeros_like(r2))

    def phi(self, x, y, z):
        r2 = x * x + y * y + z * z
        r = torch.sqrt(r2)
        p, r0 = self.rho0, self.r0
        inner = -2.0 / 3.0 * math.pi * p * r0 ** 2 + 4 * math.pi * p * (r2 / 6 - r2 * r2 / (10 * r0 ** 2) +
                                                                        r2 ** 3 / (42 * r0 ** 4))
        outer = -self.M / torch.where(r > 0, r, torch.ones_like(r))
        return torch.where(r <= r0, inner, outer)

    def fr(self, x, y, z):
        """Radial acceleration f_r = -dPhi/dr (negative: pointing inward)."""
        r = torch.sqrt(x * x + y * y + z * z)
        p, r0 = self.rho0, self.r0
        inner = -4 * math.pi * p * (r / 3 - 2.0 / 5.0 * r ** 3 / r0 ** 2 + 1.0 / 7.0 * r ** 5 / r0 ** 4)
        outer = -self.M / torch.where(r > 0, r * r, torch.ones_like(r))
        return torch.where(r <= r0, inner, outer)

    def force(self, x, y, z):
        r = torch.sqrt(x * x + y * y + z * z)
        fr = self.fr(x, y, z)
        safe = torch.where(r > 0, r, torch.ones_like(r))
        s = torch.where(r > 0, fr / safe, torch.zeros_like(r))
        return (s * x, s * y, s * z)


class Plummer(Problem):
    """Superposition of Plummer spheres [(M, a, (cx, cy, cz)), ...]."""

    def __init__(self, spheres: Sequence[Tuple[float, float, Sequence[float]]], G: float = 1.0):
        self.spheres = [(float(M), float(a), tuple(float(c) for c in cen)) for M, a, cen in spheres]
        self.G = G

    def rho(self, *x):
        out = torch.zeros_like(x[0])
        for M, a, c in self.spheres:
            r2 = sum((x[i] - c[i]) ** 2 for i in range(len(x)))
            out = out + 3 * M / (4 * math.pi * a ** 3) * (1 + r2 / a ** 2) ** (-2.5)
        return out

    def phi(self, *x):
        out = torch.zeros_like(x[0])
        for M, a, c in self.spheres:
            r2 = sum((x[i] - c[i]) ** 2 for i in range(len(x)))
            out = out - self.G * M / torch.sqrt(r2 + a * a)
        return out

    def force(self, *x):
        out = [torch.zeros_like(x[0]) for _ in x]
        for M, a, c in self.spheres:
            r2 = sum((x[i] - c[i]) ** 2 for i in range(len(x)))
            s = -self.G * M / (r2 + a * a) ** 1.5
            for i in range(len(x)):
                out[i] = out[i] + s * (x[i] - c[i])
        return tuple(out)


class Gaussian(Problem):
    """Manufactured Phi = exp(-r^2/s^2); 4 pi G rho = lap(Phi) = Phi (4 r^2/s^4 - 2d/s^2)."""

    def __init__(self, s: float = 0.1, G: float = 1.0):
        self.s, self.G = s, G

    def phi(self, *x):
        r2 = sum(xi * xi for xi in x)
        return torch.exp(-r2 / self.s ** 2)

    def rho(self, *x):
        d = len(x)
        r2 = sum(xi * xi for xi in x)
        lap = torch.exp(-r2 / self.s ** 2) * (4 * r2 / self.s ** 4 - 2 * d / self.s ** 2)
        return lap / (4 * math.pi * self.G)

    def force(self, *x):
        ph = self.phi(*x)
        return tuple(2 * xi / self.s ** 2 * ph for xi in x)


class GaussianSum(Problem):
    """Manufactured Phi = sum_k A_k exp(-|x - c_k|^2 / s_k^2) in 2-D or 3-D;
    4 pi G rho = lap(Phi) = sum_k A_k exp(.) (4 r_k^2 / s_k^4 - 2d / s_k^2)."""

    def __init__(self, terms: Sequence[Tuple[float, float, Sequence[float]]], G: float = 1.0):
        self.terms = [(float(A), float(s), tuple(float(c) for c in cen)) for A, s, cen in terms]
        self.G = G

    def _each(self, x):
        for A, s, c in self.terms:
            dx = [x[i] - c[i] for i in range(len(x))]
            r2 = sum(v * v for v in dx)
            yield A, s, dx, r2, A * torch.exp(-r2 / s ** 2)

    def phi(self, *x):
        out = torch.zeros_like(x[0])
        for _, _, _, _, g in self._each(x):
            out = out + g
        return out

    def rho(self, *x):
        d = len(x)
        out = torch.zeros_like(x[0])
        for _, s, _, r2, g in self._each(x):
            out = out + g * (4 * r2 / s ** 4 - 2 * d / s ** 2)
        return out / (4 * math.pi * self.G)

    def force(self, *x):
        out = [torch.zeros_like(x[0]) for _ in x]
        for _, s, dx, _, g in self._each(x):
            for i in range(len(x)):
                out[i] = out[i] + 2 * dx[i] / s ** 2 * g
        return tuple(out)


class Linear(Problem):
    """rho = 0, Phi = a.x + b: the interpolation and the Laplacian are exact on it."""

    def __init__(self, grad: Sequence[float], const: float = 0.0, G: float = 1.0):
        self.g = tuple(float(v) for v in grad)
        self.c = const
        self.G = G

    def rho(self, *x):
        return torch.zeros_like(x[0])

    def phi(self, *x):
        return self.c + sum(self.g[i] * x[i] for i in range(len(x)))

    def force(self, *x):
        return tuple(torch.full_like(x[0], -self.g[i]) for i in range(len(x)))


class Quadratic(Problem):
    """Phi = |x|^2 (+ const); lap Phi = 2d exactly, also for the discrete Laplacian."""

    def __init__(self, dim: int, G: float = 1.0, const: float = 0.0):
        self.d, self.G, self.c = dim, G, const

    def rho(self, *x):
        return torch.full_like(x[0], 2.0 * self.d / (4 * math.pi * self.G))

    def phi(self, *x):
        return self.c + sum(xi * xi for xi in x)

    def force(self, *x):
        return tuple(-2 * xi for xi in x)


# ------------------------------------------------------------------ inputs
def make_inputs(geom: Geometry, prob: Problem, device="cpu"):
    """Caller inputs of a nested solve.

    rho[0]   : n0_a + 2 per axis   Omega^0 plus its inner buffer layer
    rho[l>=1]: n_l,a per axis      Omega^l
    phi_outer: n0_a + 4 per axis   closed-form potential (only its outer layer is used)
    """
    rho = []
    for l in range(geom.nlevels):
        x = geom.mesh_pad(l, 1 if l == 0 else 0, device)
        rho.append(prob.rho(*x).contiguous())
    x = geom.mesh_pad(0, 2, device)
    phi_outer = prob.phi(*x).contiguous()
    return rho, phi_outer


# ------------------------------------------------------------------ configs
def sphere_draw(seed: int):
    """Seeded 1..8 Plummer spheres: centres U[-0.4,0.4]^3, M ~ lognormal(0, 0.5),
    a ~ U[0.02, 0.1]; draw order K, centres, masses, radii."""
    rng = np.random.default_rng(seed)
    K = int(rng.integers(1, 9))
    cen = rng.uniform(-0.4, 0.4, size=(K, 3))
    M = rng.lognormal(mean=0.0, sigma=0.5, size=K)
    a = rng.uniform(0.02, 0.1, size=K)
    return [(float(M[i]), float(a[i]), tuple(float(v) for v in cen[i])) for i in range(K)]


@dataclass
class Workload:
    name: str
    geom: Geometry
    prob: Problem
    note: str = ""
    extra: dict = field(default_factory=dict)


def c1_gaussian_2d(N: int = 64) -> Workload:
    """2-D Gaussian manufactured solution on [-1,1]^2, N^2 base cells, one
    nested level at twice the resolution over [-0.5,0.5]^2 (N^2 cells)."""
    g = Geometry(dim=2, n=[N, N], off=[(0, 0, 0), (N // 4, N // 4, 0)], lo0=(-1.0, -1.0, 0.0), dx0=2.0 / N, G=1.0)
    return Workload("gaussian2d_2lev_%d" % N, g, Gaussian(0.1, 1.0))


def c2_plummer(N: int = 128, nlevels: int = 3) -> Workload:
    """3-D Plummer M=1, a=0.05 at the origin; domain [-1,1]^3; levels of N^3
    cells at 2x refinement, level k covering [-2^-k, 2^-k]^3."""
    g = centred_geometry(3, nlevels, N, 1.0, 1.0)
    return Workload("plummer_%dlev_%d" % (nlevels, N), g, Plummer([(1.0, 0.05, (0, 0, 0))]))


def c3_plummer_offset(N: int = 256, nlevels: int = 4) -> Workload:
    """Plummer a=0.02 (M=1) offset to (0.1,-0.05,0.03); 4 levels of N^3."""
    g = centred_geometry(3, nlevels, N, 1.0, 1.0)
    return Workload("plummer_offset_%dlev_%d" % (nlevels, N), g, Plummer([(1.0, 0.02, (0.1, -0.05, 0.03))]))


def c4_multi_plummer(seed: int, N: int = 128, nlevels: int = 3) -> Workload:
    g = centred_geometry(3, nlevels, N, 1.0, 1.0)
    return Workload("multi_plummer_seed%d_%dlev_%d" % (seed, nlevels, N), g, Plummer(sphere_draw(seed)),
                    extra=dict(seed=seed))


def c5_two_plummer(N: int = 512, nlevels: int = 5) -> Workload:
    """Two Plummer spheres: M=1, a=0.03 at the origin and M=0.3, a=0.015 at
    (0.2, 0, 0); 5 levels of N^3 cells."""
    g = centred_geometry(3, nlevels, N, 1.0, 1.0)
    return Workload("two_plummer_%dlev_%d" % (nlevels, N), g,
                    Plummer([(1.0, 0.03, (0, 0, 0)), (0.3, 0.015, (0.2, 0.0, 0.0))]))


def paper2d(N: int, nlevels: int = 4) -> Workload:
    """Sec. 3.1 setup: Omega^0 = [-0.5,0.5]^2, levels 0..3, N cells per axis each."""
    p = Paper2D(0.3)
    g = centred_geometry(2, nlevels, N, 0.5, p.G)
    return Workload("paper2d_%d" % N, g, p)


def paper3d(N: int, nlevels: int = 3) -> Workload:
    """Sec. 3.2 setup: Omega^0 = [-0.5,0.5]^3, levels 0..2, N cells per axis each."""
    p = Paper3D(1.0, 0.25)
    g = centred_geometry(3, nlevels, N, 0.5, p.G)
    return Workload("paper3d_%d" % N, g, p)


def two_patch_geometry(dim: int, N: int, grandchild_order: str = "last") -> Geometry:
    """A tree of patches on [-1, 1]^d: the base level (N cells per axis), two
    disjoint children of N/2 cells (each covering N/4 parent cells, width 1/2)
    centred at x = -1/2 and x = +1/2, and one grandchild of N/2 cells centred
    inside the first child.  Entry order [base, A, B, AA] ("last") or
    [base, A, AA, B] ("middle")."""
    if N % 8:
        raise ValueError("N must be a multiple of 8")
    q = N // 8
    A = (q, 3 * q, 3 * q)
    B = (5 * q, 3 * q, 3 * q)
    AA = (q, q, q)
    if grandchild_order == "last":
        off, parent = [(0, 0, 0), A, B, AA], [-1, 0, 0, 1]
    else:
        off, parent = [(0, 0, 0), A, AA, B], [-1, 0, 1, 0]
    if dim == 2:
        off = [(o[0], o[1], 0) for o in off]
    return Geometry(dim=dim, n=[N, N // 2, N // 2, N // 2], off=off, lo0=(-1.0, -1.0, -1.0), dx0=2.0 / N,
                    parent=parent)


def two_patch_2d(N: int = 64, grandchild_order: str = "last") -> Workload:
    """Two manufactured Gaussian sources at (-1/2, 0) and (1/2, 0), each under
    its own refined patch (a tree: two patches on level 1, one on level 2)."""
    g = two_patch_geometry(2, N, grandchild_order)
    return Workload("two_patch_2d_%d_%s" % (N, grandchild_order), g,
                    GaussianSum([(1.0, 0.12, (-0.5, 0.0)), (0.6, 0.2, (0.5, 0.0))]))


def two_patch_3d(N: int = 64, grandchild_order: str = "last") -> Workload:
    """Two Plummer spheres (M = 1, a = 0.1 at (-1/2, 0, 0); M = 0.5, a = 0.06 at
    (1/2, 0, 0)), each under its own refined patch (tree as in two_patch_2d)."""
    g = two_patch_geometry(3, N, grandchild_order)
    return Workload("two_patch_3d_%d_%s" % (N, grandchild_order), g,
                    Plummer([(1.0, 0.1, (-0.5, 0.0, 0.0)), (0.5, 0.06, (0.5, 0.0, 0.0))]))


def box_geometry(dim: int, n0, n1, off1, n2=None, off2=None, dx0: float = 1.0 / 32) -> Geometry:
    """Non-cubic nested patches (Sec. 2.1 gives the cell counts per direction;
    the cells stay cubes): base level of n0 = (nx, ny[, nz]) cells with its
    lower corner at the origin, a patch of n1 cells whose corner sits off1
    base cells in, and optionally a patch of n2 cells inside that one."""
    n = [tuple(n0), tuple(n1)]
    off = [(0, 0, 0), tuple(off1) + (0,) * (3 - dim)]
    if n2 is not None:
        n.append(tuple(n2))
        off.append(tuple(off2) + (0,) * (3 - dim))
    return Geometry(dim=dim, n=n, off=off, lo0=(0.0, 0.0, 0.0), dx0=dx0, G=1.0)


def box_plummer_3d(scale: int = 1) -> Workload:
    """A 3-D stack of non-cubic patches around a Plummer sphere (M = 1,
    a = 0.12): base 64 x 32 x 46 cells of 1/32, a 46 x 22 x 30 patch from
    base cell (8, 4, 8), a 30 x 16 x 22 patch inside it from (6, 3, 4);
    `scale` multiplies every cell count (and divides the spacing).  The counts
    keep every right-ghost gain of their hierarchies small at scales 1-8."""
    k = scale
    g = box_geometry(3, (64 * k, 32 * k, 46 * k), (46 * k, 22 * k, 30 * k), (8 * k, 4 * k, 8 * k),
                     (30 * k, 16 * k, 22 * k), (6 * k, 3 * k, 4 * k), dx0=1.0 / (32 * k))
    c = g.lo(2)
    e = g.ext(2)
    centre = tuple(c[a] + 0.5 * e[a] * g.dx(2) for a in range(3))
    return Workload("box_plummer_3d_%d" % k, g, Plummer([(1.0, 0.12, centre)]))


def slab_two_plummer(N: int = 512, parts: int = 8) -> Workload:
    """One z-slab of the two-Plummer level of c5_two_plummer: N x N x N/parts
    cells of 2/N on [-1, 1]^2 x [-1/parts, 1/parts], the two spheres in its
    mid-plane, a single level.  This is one GPU's share when a level of N^3
    cells is split into `parts` slabs along z; the closed-form potential on
    the z faces stands in for the halo planes the neighbouring slabs would
    send."""
    nz = N // parts
    g = Geometry(dim=3, n=[(N, N, nz)], off=[(0, 0, 0)], lo0=(-1.0, -1.0, -nz / N), dx0=2.0 / N, G=1.0)
    return Workload("slab_two_plummer_%dx%dx%d" % (N, N, nz), g,
                    Plummer([(1.0, 0.03, (0, 0, 0)), (0.3, 0.015, (0.2, 0.0, 0.0))]))


def box_gaussian_2d(scale: int = 1) -> Workload:
    """A 2-D stack of non-cubic patches around a manufactured Gaussian
    (s = 0.15): base 64 x 32 cells of 1/32, a 42 x 26 patch from base cell
    (10, 2), a 26 x 16 patch inside it from (8, 5); `scale` as above."""
    k = scale
    g = box_geometry(2, (64 * k, 32 * k), (42 * k, 26 * k), (10 * k, 2 * k), (26 * k, 16 * k), (8 * k, 5 * k),
                     dx0=1.0 / (32 * k))
    c = g.lo(2)
    e = g.ext(2)
    centre = tuple(c[a] + 0.5 * e[a] * g.dx(2) for a in range(2))
    return Workload("box_gaussian_2d_%d" % k, g, GaussianSum([(1.0, 0.15, centre)]))


def many_patches_geometry(dim: int, N: int, k: int = 2, m: int = None, depth2: bool = False) -> Geometry:
    """A base of N cells per axis on [-1, 1]^d with k^d disjoint children of m
    cells each (default N/4, each covering m/2 base cells) centred in the k^d
    cells of a regular split of the base; with depth2, the children carry one
    grandchild of m cells at their centre each (a second depth of same-size
    patches), as many as the 16 entries of a solver hold."""
    m = m or N // 4
    if N % (2 * k) or m % 4:
        raise ValueError("N must be a multiple of 2k and m of 4")
    span = N // k                 # base cells per split cell
    half = m // 2                 # base cells a child covers
    if half + 2 > span:
        raise ValueError("children too large for the split")
    n = [N]
    off = [(0, 0, 0)]
    parent = [-1]
    idx = []
    for c in range(k ** dim):
        pos = [(c // k ** a) % k for a in range(dim)]
        o = tuple(p * span + (span - half) // 2 for p in pos) + (0,) * (3 - dim)
        n.append(m)
        off.append(o)
        parent.append(0)
        idx.append(len(n) - 1)
    if depth2:
        for c in idx[:16 - len(n)]:
            n.append(m)
            off.append((m // 4,) * dim + (0,) * (3 - dim))
            parent.append(c)
    return Geometry(dim=dim, n=n, off=off, lo0=(-1.0, -1.0, -1.0), dx0=2.0 / N, parent=parent)


def many_patches_3d(N: int = 256, k: int = 2, m: int = None, depth2: bool = False) -> Workload:
    """k^3 same-size patches refined out of a base of N^3 cells (default: eight
    64^3 children of a 256^3 base), each around a Plummer sphere at its centre
    (M = 1, a = 0.04; the spheres' closed forms superposed)."""
    g = many_patches_geometry(3, N, k, m, depth2)
    cen = []
    for l in range(1, g.nlevels):
        if g.par(l) != 0:
            continue
        lo = g.lo(l)
        cen.append(tuple(lo[a] + 0.5 * g.ext(l)[a] * g.dx(l) for a in range(3)))
    return Workload("many_patches_3d_%d_k%d%s" % (N, k, "_d2" if depth2 else ""), g,
                    Plummer([(1.0, 0.04, c) for c in cen]))


def many_patches_2d(N: int = 128, k: int = 2, m: int = None, depth2: bool = False) -> Workload:
    """The 2-D form: k^2 same-size patches around Gaussian sources (width 0.06)."""
    g = many_patches_geometry(2, N, k, m, depth2)
    terms = []
    for l in range(1, g.nlevels):
        if g.par(l) != 0:
            continue
        lo = g.lo(l)
        terms.append((1.0, 0.06, tuple(lo[a] + 0.5 * g.ext(l)[a] * g.dx(l) for a in range(2))))
    return Workload("many_patches_2d_%d_k%d%s" % (N, k, "_d2" if depth2 else ""), g, GaussianSum(terms))

"""ctypes wrapper of the C oracle (nested_oracle.c).  Test infrastructure only.

Arrays are numpy float64, C-contiguous, indexed [k, j, i] (x fastest) in 3-D
and [j, i] in 2-D.  A nested level l is a padded array of n_l + 4 points per
axis; a multigrid level L is an array of N^L + 2 points per axis.
"""
import ctypes
import os

import numpy as np

from . import build as _build

MAXLEV = 16
MAXMG = 32

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class OrcConfig(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("nlevels", ctypes.c_int),
        ("n", (ctypes.c_int * 3) * MAXLEV),
        ("off", (ctypes.c_int * 3) * MAXLEV),
        ("dx0", ctypes.c_double),
        ("G", ctypes.c_double),
        ("n_pre", ctypes.c_int),
        ("n_post", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("max_cycles", ctypes.c_int),
        ("stop_rule", ctypes.c_int),
        ("ghost_literal", ctypes.c_int),
        ("buffer_interp", ctypes.c_int),
        ("parent", ctypes.c_int * MAXLEV),
        ("coarse_post", ctypes.c_int),
    ]


_lib = None
_native = False


def use_native(on=True):
    """Switch every following call to the -O3 -march=native build of the same
    source (built here on first use), or back to the portable build."""
    global _lib, _native
    if bool(on) != _native:
        _lib = None
        _native = bool(on)
        if _native:
            _build.build_native()


def build_flags():
    return " ".join(_build.NATIVE_FLAGS) if _native else "-O2 (generic x86-64)"


def lib():
    """Load oracle/liboracle.so (or the native build), building it with gcc if it is not there."""
    global _lib
    if _lib is None:
        path = _build.LIB_NATIVE if _native else _build.LIB
        if not os.path.exists(path):
            _build.build_native() if _native else _build.build()
        L = ctypes.CDLL(path)
        _i3 = ctypes.POINTER(ctypes.c_int)
        L.orc_plan.argtypes = [ctypes.c_int, _ip, ctypes.c_int]
        L.orc_plan.restype = ctypes.c_int
        L.orc_plan3.argtypes = [ctypes.c_int, _i3, _ip, ctypes.c_int]
        L.orc_plan3.restype = ctypes.c_int
        L.orc_plan_stable.argtypes = [ctypes.c_int, _i3, _ip, ctypes.c_int]
        L.orc_plan_stable.restype = ctypes.c_int
        L.orc_ghost_rule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _dp]
        L.orc_ghost_fill.argtypes = [ctypes.c_int, _i3, ctypes.c_int, _i3, _dp, ctypes.c_int]
        L.orc_rb_sweep.argtypes = [ctypes.c_int, _i3, ctypes.c_int, _i3, ctypes.c_double, _dp, _dp, ctypes.c_int]
        L.orc_residual.argtypes = [ctypes.c_int, _i3, ctypes.c_double, _dp, _dp, _dp]
        L.orc_residual_norm.argtypes = [ctypes.c_int, _i3, ctypes.c_double, _dp, _dp]
        L.orc_residual_norm.restype = ctypes.c_double
        L.orc_restrict.argtypes = [ctypes.c_int, _i3, _dp, _i3, _dp]
        L.orc_prolong_add.argtypes = [ctypes.c_int, _i3, _dp, _i3, _dp]
        L.orc_interface_fill.argtypes = [ctypes.c_int, _i3, _dp, _dp, _i3, _i3, _dp, ctypes.c_double, _dp, _dp]
        L.orc_forces.argtypes = [ctypes.c_int, _i3, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.orc_validate.argtypes = [ctypes.POINTER(OrcConfig)]
        L.orc_validate.restype = ctypes.c_int
        L.orc_solve.argtypes = [ctypes.POINTER(OrcConfig), ctypes.POINTER(_dp), _dp, ctypes.POINTER(_dp), _ip,
                                _ip, _dp, _dp]
        L.orc_solve.restype = ctypes.c_int
        L.orc_vcycle_patch.argtypes = [ctypes.c_int, _i3, ctypes.c_double, _dp, _dp, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_vcycle_patch.restype = ctypes.c_int
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _i3(v):
    """Three ints (x, y, z) for the C side; missing axes are 1."""
    v = list(v) + [1] * (3 - len(v))
    return (ctypes.c_int * 3)(*[int(x) for x in v])


def _act(dim, a, pad):
    """Active points per axis (x, y[, z]) of an array [k, j, i] with `pad` ghost layers."""
    return tuple(a.shape[dim - 1 - ax] - 2 * pad for ax in range(dim))


def _ax(dim, v):
    """An int (the same on every axis) or a per-axis sequence, as a tuple."""
    return tuple(v) if isinstance(v, (tuple, list)) else (int(v),) * dim


# ---------------------------------------------------------------- operators
def plan(N0):
    """Active cells per axis of every multigrid level of a cube (Sec. 2.2)."""
    buf = (ctypes.c_int * MAXMG)()
    m = lib().orc_plan(int(N0), buf, MAXMG)
    if m < 1:
        raise ValueError("bad N0")
    return [buf[i] for i in range(m)]


def plan3(dim, N0):
    """Per-axis hierarchy of a box with N0 = (x, y[, z]) cells: one tuple per
    multigrid level, ending on the first level with one cell along some axis."""
    buf = (ctypes.c_int * (3 * MAXMG))()
    m = lib().orc_plan3(dim, _i3(N0), buf, MAXMG)
    if m < 1:
        raise ValueError("bad N0")
    return [tuple(buf[3 * L + a] for a in range(dim)) for L in range(m)]


def plan_stable(dim, N0):
    """False when some level's right-ghost gain |c_L| / (2d) exceeds the
    bound the oracle accepts (such hierarchies are refused)."""
    buf = (ctypes.c_int * (3 * MAXMG))()
    m = lib().orc_plan3(dim, _i3(N0), buf, MAXMG)
    if m < 1:
        raise ValueError("bad N0")
    return bool(lib().orc_plan_stable(dim, _i3(N0), buf, m))


def ghost_rule(N0, L, N, literal=False):
    one = ctypes.c_int()
    c = ctypes.c_double()
    lib().orc_ghost_rule(N0, L, N, int(literal), ctypes.byref(one), ctypes.byref(c))
    return bool(one.value), c.value


def ghost_fill(dim, N0, L, e, literal=False):
    lib().orc_ghost_fill(dim, _i3(_ax(dim, N0)), L, _i3(_act(dim, e, 1)), _p(e), int(literal))


def rb_sweep(dim, N0, L, h, u, f, literal=False):
    lib().orc_rb_sweep(dim, _i3(_ax(dim, N0)), L, _i3(_act(dim, u, 1)), h, _p(u), _p(f), int(literal))


def residual(dim, h, u, f):
    r = np.zeros_like(u)
    lib().orc_residual(dim, _i3(_act(dim, u, 1)), h, _p(u), _p(f), _p(r))
    return r


def residual_norm(dim, h, u, f):
    return lib().orc_residual_norm(dim, _i3(_act(dim, u, 1)), h, _p(u), _p(f))


def restrict(dim, r, Nc):
    Nc = _ax(dim, Nc)
    fc = np.zeros(tuple(v + 2 for v in reversed(Nc)))
    lib().orc_restrict(dim, _i3(_act(dim, r, 1)), _p(r), _i3(Nc), _p(fc))
    return fc


def prolong_add(dim, ec, uf):
    lib().orc_prolong_add(dim, _i3(_act(dim, ec, 1)), _p(ec), _i3(_act(dim, uf, 1)), _p(uf))


def interface_fill(dim, phic, fc, nf, off, rho, fourpiG):
    """Coarse-to-fine fill of a level l >= 1 (nf: cells per axis, an int or
    a tuple): returns (phi_f, f_f), padded."""
    nf = _ax(dim, nf)
    phif = np.zeros(tuple(v + 4 for v in reversed(nf)))
    ff = np.zeros_like(phif)
    offa = (ctypes.c_int * 3)(*(list(off) + [0] * (3 - len(off))))
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    lib().orc_interface_fill(dim, _i3(_act(dim, phic, 2)), _p(phic), _p(fc), _i3(nf), offa, _p(rho), fourpiG,
                             _p(phif), _p(ff))
    return phif, ff


def forces(dim, dx, phi):
    """F = -grad(Phi) on Omega of a padded level array (fourth-order stencil)."""
    n = _act(dim, phi, 2)
    shp = tuple(reversed(n))
    fx, fy, fz = np.zeros(shp), np.zeros(shp), np.zeros(shp if dim == 3 else (1,))
    lib().orc_forces(dim, _i3(n), dx, _p(phi), _p(fx), _p(fy), _p(fz))
    return (fx, fy, fz) if dim == 3 else (fx, fy)


def num_threads():
    return lib().orc_num_threads()


def set_threads(n):
    lib().orc_set_threads(int(n))


def vcycle_patch(dim, h0, u, f, n_pre=2, n_post=1, literal=False, coarse_post=None):
    rc = lib().orc_vcycle_patch(dim, _i3(_act(dim, u, 1)), h0, _p(u), _p(f), n_pre, n_post,
                                -1 if coarse_post is None else int(coarse_post), int(literal))
    if rc:
        raise RuntimeError("vcycle_patch failed")


# ---------------------------------------------------------------- nested solve
STATUS = {0: "ok", -1: "invalid", -2: "nonfinite", -3: "not converged", -4: "diverged"}


def make_config(geom, n_pre=2, n_post=1, tol=1e-10, max_cycles=50, stop_rule=0, ghost_literal=False,
                buffer_interp=False, coarse_post=None):
    c = OrcConfig()
    c.dim = geom.dim
    c.nlevels = geom.nlevels
    for l in range(geom.nlevels):
        e = list(geom.ext(l)) + [1] * (3 - geom.dim)
        for a in range(3):
            c.n[l][a] = int(e[a])
        for a in range(3):
            c.off[l][a] = geom.off[l][a] if a < len(geom.off[l]) else 0
    c.dx0 = geom.dx0
    c.G = geom.G
    c.n_pre, c.n_post = n_pre, n_post
    c.tol = tol
    c.max_cycles = max_cycles
    c.stop_rule = stop_rule
    c.ghost_literal = int(ghost_literal)
    c.buffer_interp = int(buffer_interp)
    c.coarse_post = -1 if coarse_post is None else int(coarse_post)
    parent = getattr(geom, "parent", None)
    for l in range(geom.nlevels):
        c.parent[l] = int(parent[l]) if parent is not None else l - 1
    return c


def validate(geom):
    c = make_config(geom)
    return lib().orc_validate(ctypes.byref(c)) == 0


def solve(geom, rho, phi_outer, fixed_cycles=None, **kw):
    """Nested solve.  rho[0]: n0_a + 2 per axis, rho[l>=1]: n_l,a per axis,
    phi_outer: n0_a + 4 per axis ([k, j, i] arrays).
    buffer_interp=True: the comparison scheme of Sec. 4 on levels l >= 1 (both
    buffer layers interpolated from level l-1, only Omega^l relaxed).

    Returns dict(phi=[padded arrays], cycles, final_rel, hist, status)."""
    cfg = make_config(geom, **kw)
    d = geom.dim
    nl = geom.nlevels
    rho = [np.ascontiguousarray(r, dtype=np.float64) for r in rho]
    phi_outer = np.ascontiguousarray(phi_outer, dtype=np.float64)
    phi = [np.zeros(geom.shape(l, 2)) for l in range(nl)]
    rho_p = (_dp * nl)(*[_p(r) for r in rho])
    phi_p = (_dp * nl)(*[_p(a) for a in phi])
    fixed = None
    if fixed_cycles is not None:
        fixed = (ctypes.c_int * nl)(*[int(x) for x in fixed_cycles])
    cycles = (ctypes.c_int * nl)()
    final = (ctypes.c_double * nl)()
    hist = np.full(nl * (cfg.max_cycles + 1), np.nan)
    st = lib().orc_solve(ctypes.byref(cfg), rho_p, _p(phi_outer), phi_p, fixed, cycles, final, _p(hist))
    return dict(phi=phi, cycles=[cycles[l] for l in range(nl)], final_rel=[final[l] for l in range(nl)],
                hist=hist.reshape(nl, cfg.max_cycles + 1), status=st, status_name=STATUS.get(st, str(st)))

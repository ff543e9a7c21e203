"""Composite error norms of Sec. 3 (test infrastructure).

||e||_p = (integral over Omega of |e|^p)^(1/p) and ||e||_inf = sup |e| over
the whole calculation domain.  On a nested grid every point of Omega^0 is
counted once, on the finest level that covers it (the cells of Omega^l not
covered by Omega^{l+1}), with cell volume dx_l^d; errors are taken at cell
centres.  No division by |Omega| (the paper's domains have unit measure).
"""
import numpy as np


def _children(geom, l):
    parent = getattr(geom, "parent", None)
    return [m for m in range(1, geom.nlevels) if (parent[m] if parent is not None else m - 1) == l]


def uncovered_mask(geom, l):
    """Boolean mask (shape of Omega^l) of the cells of patch l not covered by a finer patch
    refined out of it (Omega^{l+1} for the stack of one patch per level)."""
    m = np.ones(geom.shape(l), dtype=bool)
    for c in _children(geom, l):
        o = geom.off[c]
        h = [v // 2 for v in geom.ext(c)]
        sl = tuple(slice(o[a], o[a] + h[a]) for a in reversed(range(geom.dim)))  # [k, j, i]
        m[sl] = False
    return m


def composite_norms(geom, err_levels):
    """err_levels[l]: n_l^d array of pointwise errors.  Returns (L1, L2, Linf)."""
    s1 = 0.0
    s2 = 0.0
    mx = 0.0
    for l, e in enumerate(err_levels):
        e = np.abs(np.asarray(e, dtype=np.float64))
        m = uncovered_mask(geom, l)
        vol = geom.dx(l) ** geom.dim
        s1 += e[m].sum() * vol
        s2 += (e[m] ** 2).sum() * vol
        if m.any():
            mx = max(mx, float(e[m].max()))
    return s1, np.sqrt(s2), mx


def order(e_coarse, e_fine):
    """Observed order log2(e_N / e_2N) (Tables 1-2)."""
    return float(np.log2(e_coarse / e_fine))

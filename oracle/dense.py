"""Direct solve of the nested discrete system: the plain definition of the
fixed point the multigrid iteration converges to (test infrastructure).

For each level (patch) l in order (one-way scheme, Sec. 2.1; the parent of
patch l is l-1 for the stack of one patch per level, geom.parent[l] for a tree):
  * unknowns: Phi at the centres of Gamma^l = Omega^l plus its inner buffer
    layer ((n_l+2)^d cells);
  * Dirichlet data at the outer buffer layer: the caller's potential for
    l = 0, the multilinear interpolant of the parent's Phi for l >= 1;
  * right-hand side 4 pi G rho on Omega^l, and on the inner buffer layer the
    multilinear interpolant of the parent's right-hand side (l >= 1) or the
    caller's density (l = 0);
  * operator: the 5-/7-point Laplacian (eqn:Laplacian2D/3D) with the outer
    layer moved to the right-hand side.
With buffer_interp (the comparison scheme of Sec. 4, levels l >= 1) the
unknowns are the cells of Omega^l alone and the inner buffer layer keeps the
interpolant of the parent's Phi, as Dirichlet data next to the outer layer's.
The interpolation is evaluated from physical cell-centre coordinates (the
bilinear/trilinear formula of Appendix A at the fine centre), not from index
tables, so it is an independent route to the same weights.  The linear system
is solved with scipy's sparse direct solver.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _parent(geom, l):
    return geom.parent[l] if getattr(geom, "parent", None) is not None else l - 1


def _interp(geom, l, coarse_padded, first, count):
    """Multilinear interpolation of the padded array of patch l's parent at the
    centres of patch-l cells first..first+count_a-1 along each axis a (index
    -2 = outer layer); `count` is one count per axis (x, y[, z]) or an int."""
    d = geom.dim
    if not isinstance(count, (tuple, list)):
        count = (count,) * d
    p = _parent(geom, l)
    lo_c = geom.lo(p)
    lo_f = geom.lo(l)
    dxc, dxf = geom.dx(p), geom.dx(l)
    idx = []
    wts = []
    for a in range(d):
        i = np.arange(first, first + count[a])
        x = lo_f[a] + (i + 0.5) * dxf
        t = (x - lo_c[a]) / dxc - 0.5          # continuous coarse cell index
        il = np.floor(t).astype(int)
        w = t - il
        idx.append(il + 2)                      # padded coarse index
        wts.append(w)
    out = np.zeros(tuple(reversed(count)))
    for corner in range(1 << d):
        sel = [(corner >> a) & 1 for a in range(d)]
        # weights along each axis
        wa = [wts[a] if sel[a] else 1.0 - wts[a] for a in range(d)]
        ia = [idx[a] + sel[a] for a in range(d)]
        if d == 3:
            vals = coarse_padded[np.ix_(ia[2], ia[1], ia[0])]
            w = wa[2][:, None, None] * wa[1][None, :, None] * wa[0][None, None, :]
        else:
            vals = coarse_padded[np.ix_(ia[1], ia[0])]
            w = wa[1][:, None] * wa[0][None, :]
        out += w * vals
    return out


def _laplacian_system(d, m, h):
    """Sparse matrix of the Laplacian on m = (m_x, m_y[, m_z]) cells with
    homogeneous Dirichlet data outside (the boundary values are added to the
    right-hand side separately); unknowns in [k, j, i] order (x fastest)."""
    def T(k):
        one = np.ones(k)
        return sp.diags([one[:-1], -2 * one, one[:-1]], [-1, 0, 1], shape=(k, k))

    def I(k):
        return sp.identity(k)

    if d == 2:
        A = sp.kron(I(m[1]), T(m[0])) + sp.kron(T(m[1]), I(m[0]))
    else:
        A = (sp.kron(sp.kron(I(m[2]), I(m[1])), T(m[0])) + sp.kron(sp.kron(I(m[2]), T(m[1])), I(m[0]))
             + sp.kron(sp.kron(T(m[2]), I(m[1])), I(m[0])))
    return (A / (h * h)).tocsc()


def _boundary_term(d, phi_padded, h):
    """Contribution of the outer-layer values to the Laplacian of each cell
    inside them (the array minus its outermost layer)."""
    P = phi_padded.shape
    b = np.zeros(tuple(v - 2 for v in P))
    ring = phi_padded.copy()
    inner = tuple(slice(1, v - 1) for v in P)
    ring[inner] = 0.0
    # sum of the face neighbours that are outer-layer points
    for a in range(d):
        for s in (-1, 1):
            sl = []
            for ax in range(d):
                if ax == a:
                    sl.append(slice(1 + s, P[ax] - 1 + s))
                else:
                    sl.append(slice(1, P[ax] - 1))
            b += ring[tuple(sl)]
    return b / (h * h)


def solve(geom, rho, phi_outer, buffer_interp=False):
    """Exact nested solution.  Returns (phi_padded list, f_padded list)."""
    d = geom.dim
    fourpiG = 4 * math.pi * geom.G
    phis, fs = [], []
    for l in range(geom.nlevels):
        n = geom.ext(l)                       # cells per axis (x, y[, z])
        h = geom.dx(l)
        phi = np.zeros(geom.shape(l, 2))
        f = np.zeros(geom.shape(l, 2))
        core = tuple(slice(2, v + 2) for v in reversed(n))
        gam = tuple(slice(1, v + 3) for v in reversed(n))
        if l == 0:
            phi[...] = np.asarray(phi_outer)
            f[gam] = fourpiG * np.asarray(rho[0])
        else:
            p = _parent(geom, l)
            phi[...] = _interp(geom, l, phis[p], -2, tuple(v + 4 for v in n))
            f[gam] = _interp(geom, l, fs[p], -1, tuple(v + 2 for v in n))
            f[core] = fourpiG * np.asarray(rho[l])
        if l > 0 and buffer_interp:
            # unknowns on Omega^l; the inner layer is the boundary of the sub-box
            sub = phi[gam]
            A = _laplacian_system(d, n, h)
            rhs = f[core] - _boundary_term(d, sub, h)
            x = spla.spsolve(A, rhs.reshape(-1))
            phi[core] = x.reshape(tuple(reversed(n)))
        else:
            m = tuple(v + 2 for v in n)
            A = _laplacian_system(d, m, h)
            rhs = f[gam] - _boundary_term(d, phi, h)
            x = spla.spsolve(A, rhs.reshape(-1))
            phi[gam] = x.reshape(tuple(reversed(m)))
        phis.append(phi)
        fs.append(f)
    return phis, fs


def forces(dim, dx, phi):
    """F = -grad(Phi) on Omega from a padded array, fourth-order central
    difference (Eqn:force_evaluation), written with array slices."""
    P = phi.shape
    out = []
    for a in range(dim):
        ax = dim - 1 - a  # numpy axis of physical axis a ([k, j, i] order)

        def sh(off):
            sl = [slice(2, v - 2) for v in P]
            sl[ax] = slice(2 + off, P[ax] - 2 + off)
            return phi[tuple(sl)]

        g = 8.0 * (sh(1) - sh(-1)) - (sh(2) - sh(-2))
        out.append(-g / (12.0 * dx))
    return tuple(out)

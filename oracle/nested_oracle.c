/*
 * Plain FP64 CPU oracle for the nested-grid multigrid Poisson solver of
 * Wang & Yen, "Self-gravitational Force Calculation of Second Order Accuracy
 * Using Multigrid Method on Nested Grids" (arXiv:2001.02327).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * Everything is plain loops over natural (x-fastest) arrays, in the order the
 * paper states the steps.  No blocking, fusion or colour-split layout.
 *
 * Array conventions
 *   Nested level l: Omega^l has n_a cells along axis a (Sec. 2.1 gives the
 *   cell counts per direction; the cells are cubes).  Its padded array has
 *   P_a = n_a + 4 points along axis a: index 0 / P_a-1 = outer buffer layer
 *   (Dirichlet potential interpolated from level l-1), 1 / P_a-2 = inner
 *   buffer layer (relaxed with the patch), 2..n_a+1 = Omega^l.  Sec. 2.1,
 *   Fig. 1b-c.  Multigrid level L of that patch: N^L_a active cells along
 *   axis a, arrays of N^L_a + 2 points per axis, active 1..N^L_a, one ghost
 *   layer.  Sec. 2.2.  Multigrid level 0 of patch l *is* the padded level
 *   array (N^0_a = n_a + 2, Gamma^l = Omega^l plus the inner buffer layer).
 *   A 2-D array is one plane (third extent 1, k = 0).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXLEV 16  /* nested patches (entries) */
#define ORC_MAXMG 32   /* multigrid levels per patch */

/* ------------------------------------------------------------------ */
/* configuration passed in from Python (ctypes mirror in oracle/core.py) */
typedef struct {
    int dim;                    /* 2 or 3 */
    int nlevels;                /* number of nested levels */
    int n[ORC_MAXLEV][3];       /* cells of Omega^l along x, y, z (z unused in 2-D) */
    int off[ORC_MAXLEV][3];     /* l>=1: lower corner of Omega^l, in cells of its parent */
    double dx0;                 /* cell size of level 0 */
    double G;                   /* gravitational constant */
    int n_pre, n_post;          /* smoothing counts (Sec. 3: 2 and 1) */
    double tol;                 /* stop tolerance */
    int max_cycles;
    int stop_rule;              /* 0: ||r||_inf <= tol*||f||_inf ; 1: max|F^q - F^{q-1}| < tol */
    int ghost_literal;          /* 1: use the right-ghost factor exactly as printed (negative tests) */
    int buffer_interp;          /* 1: comparison scheme of Sec. 4 on levels l >= 1: both buffer layers
                                   keep the interpolated potential and only Omega^l is relaxed */
    int parent[ORC_MAXLEV];     /* l>=1: the patch Omega^l is refined out of (earlier entry); the
                                   stack of Sec. 2.1 has parent[l] = l-1, a tree gives several
                                   disjoint patches per level */
    int coarse_post;            /* post-smoothing sweeps on multigrid levels L >= 1; -1: n_post
                                   (Sec. 2.3 smooths every level alike) */
} orc_config;

/* refinement depth of entry l: number of parent links down to the base level */
static int depth_of(const orc_config *cfg, int l)
{
    int k = 0;
    while (l > 0) {
        l = cfg->parent[l];
        k++;
    }
    return k;
}

/* ------------------------------------------------------------------ */
/* An array of q[0] x q[1] x q[2] points, x fastest (q[2] = 1 in 2-D). */
static size_t idx3(const int *q, int i, int j, int k) { return ((size_t)k * q[1] + j) * q[0] + i; }

static size_t npts(const int *q) { return (size_t)q[0] * q[1] * q[2]; }

/* points per axis of an array with `act[a]` active points and `pad` extra
 * points on each side along the axes of a dim-dimensional grid */
static void extents(int dim, const int *act, int pad, int *q)
{
    for (int a = 0; a < 3; a++) q[a] = a < dim ? act[a] + 2 * pad : 1;
}

/* ------------------------------------------------------------------ */
/* Multigrid hierarchy, Sec. 2.2 items 1-4.
 * h^0 = 1/N^0, h^L = 2 h^{L-1}, N^L = round(1/h^L) with ties rounded up,
 * stop once N^L = 1.  1/h^L = N^0 / 2^L exactly, so the rounding is done in
 * integers: floor((N^0 + 2^{L-1}) / 2^L).  Returns the number of levels. */
int orc_plan(int N0, int *NL, int maxlev)
{
    if (N0 < 1 || maxlev < 1) return -1;
    NL[0] = N0;
    int L = 0;
    while (NL[L] > 1) {
        L++;
        if (L >= maxlev) return -1;
        long num = (long)N0 + (1L << (L - 1));
        NL[L] = (int)(num >> L);
    }
    return L + 1;
}

/* The hierarchy of a patch with N^0_a cells along each axis: items 1-3 of
 * Sec. 2.2 along every axis with the same doubling of h, so the cells stay
 * cubes on every level; item 4's test N^L = 1 is met by the axes at
 * different levels, and the hierarchy ends at the first level on which some
 * axis has one active cell (for a cube: the one-cell level).  NL[L*3 + a].
 * Returns the number of levels. */
int orc_plan3(int dim, const int *N0, int *NL, int maxlev)
{
    for (int a = 0; a < dim; a++)
        if (N0[a] < 1) return -1;
    if (maxlev < 1) return -1;
    for (int a = 0; a < 3; a++) NL[a] = a < dim ? N0[a] : 1;
    int L = 0;
    for (;;) {
        int one = 0;
        for (int a = 0; a < dim; a++)
            if (NL[3 * L + a] <= 1) one = 1;
        if (one) break;
        L++;
        if (L >= maxlev) return -1;
        for (int a = 0; a < 3; a++) {
            long num = (long)N0[a] + (1L << (L - 1));
            NL[3 * L + a] = a < dim ? (int)(num >> L) : 1;
        }
    }
    return L + 1;
}

/* Right-ghost rule of Sec. 2.4 for multigrid level L >= 1 (one axis).
 * The right-most active centre is x_N = (N - 1/2) h^L with h^L = 2^L / N^0.
 * If x_N == 1: ghost = -e_{N-1}.  Otherwise the ghost is the value at
 * x_N + h^L of the straight line through (x_N, e_N) that vanishes at x = 1:
 *     e_{N+1} = e_N (1 - x_N - h^L) / (1 - x_N).
 * (The printed factor (1 - h)/(1 - x_N) is a misprint: it does not vanish at
 * x = 1 and its gain exceeds one; it is kept behind `literal` so the tests
 * can show that it diverges.) */
void orc_ghost_rule(int N0, int L, int N, int literal, int *xn_is_one, double *coef)
{
    *xn_is_one = ((long)(2 * N - 1) * (1L << (L - 1)) == (long)N0);
    if (literal) {
        double h = ldexp(1.0, L) / (double)N0;
        double xN = ((double)N - 0.5) * h;
        *coef = (1.0 - h) / (1.0 - xN);
    } else {
        /* multiply numerator and denominator by 2 N^0: both are integers, so the
         * factor is a single correctly rounded division */
        double num = 2.0 * N0 - (double)(2 * N + 1) * ldexp(1.0, L);
        double den = 2.0 * N0 - (double)(2 * N - 1) * ldexp(1.0, L);
        *coef = num / den;
    }
}

/* Fill the ghost layer of a multigrid level L >= 1 (Sec. 2.4): left
 * e_0 = -e_1, right per orc_ghost_rule of that axis (its own N^0 and N^L);
 * the 1-D rule is applied along x over the active y,z range, then along y
 * over the x range including ghosts, then along z over the full x,y range, so
 * edges and corners receive the rule of every axis on which they are ghosts.
 * N0 and N: per axis. */
void orc_ghost_fill(int dim, const int *N0, int L, const int *N, double *e, int literal)
{
    int q[3];
    extents(dim, N, 1, q);
    int one[3] = {0, 0, 0};
    double c[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; a++) orc_ghost_rule(N0[a], L, N[a], literal, &one[a], &c[a]);
    const int Nx = N[0], Ny = N[1], Nz = dim == 3 ? N[2] : 0;
    int klo = dim == 3 ? 1 : 0, khi = dim == 3 ? Nz : 0;
    /* x */
    for (int k = klo; k <= khi; k++)
        for (int j = 1; j <= Ny; j++) {
            e[idx3(q, 0, j, k)] = -e[idx3(q, 1, j, k)];
            e[idx3(q, Nx + 1, j, k)] = one[0] ? -e[idx3(q, Nx - 1, j, k)] : c[0] * e[idx3(q, Nx, j, k)];
        }
    /* y */
    for (int k = klo; k <= khi; k++)
        for (int i = 0; i <= Nx + 1; i++) {
            e[idx3(q, i, 0, k)] = -e[idx3(q, i, 1, k)];
            e[idx3(q, i, Ny + 1, k)] = one[1] ? -e[idx3(q, i, Ny - 1, k)] : c[1] * e[idx3(q, i, Ny, k)];
        }
    /* z */
    if (dim == 3)
        for (int j = 0; j <= Ny + 1; j++)
            for (int i = 0; i <= Nx + 1; i++) {
                e[idx3(q, i, j, 0)] = -e[idx3(q, i, j, 1)];
                e[idx3(q, i, j, Nz + 1)] = one[2] ? -e[idx3(q, i, j, Nz - 1)] : c[2] * e[idx3(q, i, j, Nz)];
            }
}

/* ------------------------------------------------------------------ */
/* Discrete Laplacian, eqn:Laplacian2D / eqn:Laplacian3D: sum of the 2d face
 * neighbours minus 2d times the centre, over (Delta x^L_MG)^2. */
static double laplacian(int dim, const int *q, const double *u, int i, int j, int k, double h)
{
    if (dim == 3)
        return (u[idx3(q, i - 1, j, k)] + u[idx3(q, i + 1, j, k)] + u[idx3(q, i, j - 1, k)] +
                u[idx3(q, i, j + 1, k)] + u[idx3(q, i, j, k - 1)] + u[idx3(q, i, j, k + 1)] -
                6.0 * u[idx3(q, i, j, k)]) / (h * h);
    return (u[idx3(q, i - 1, j, 0)] + u[idx3(q, i + 1, j, 0)] + u[idx3(q, i, j - 1, 0)] +
            u[idx3(q, i, j + 1, 0)] - 4.0 * u[idx3(q, i, j, 0)]) / (h * h);
}

/* One Gauss-Seidel half sweep over the cells of one colour.  Red (colour 0)
 * cells have an even sum of 0-based active indices.  Solving the discrete
 * Poisson equation at a cell for its own value, with the neighbours held,
 * gives u_c = (sum of neighbours - h^2 f_c) / (2d).  Cells of one colour only
 * read cells of the other colour, so the loop order inside a colour does not
 * matter. */
static void half_sweep(int dim, const int *N, double h, double *u, const double *f, int colour)
{
    int q[3];
    extents(dim, N, 1, q);
    int klo = dim == 3 ? 1 : 0, khi = dim == 3 ? N[2] : 0;
#pragma omp parallel for schedule(static)
    for (int k = klo; k <= khi; k++)
        for (int j = 1; j <= N[1]; j++)
            for (int i = 1; i <= N[0]; i++) {
                int par = ((i - 1) + (j - 1) + (dim == 3 ? k - 1 : 0)) & 1;
                if (par != colour) continue;
                double s;
                if (dim == 3)
                    s = u[idx3(q, i - 1, j, k)] + u[idx3(q, i + 1, j, k)] + u[idx3(q, i, j - 1, k)] +
                        u[idx3(q, i, j + 1, k)] + u[idx3(q, i, j, k - 1)] + u[idx3(q, i, j, k + 1)];
                else
                    s = u[idx3(q, i - 1, j, 0)] + u[idx3(q, i + 1, j, 0)] + u[idx3(q, i, j - 1, 0)] +
                        u[idx3(q, i, j + 1, 0)];
                size_t c = idx3(q, i, j, k);
                u[c] = (s - h * h * f[c]) / (2.0 * dim);
            }
}

/* A full red-black sweep.  Multigrid level 0 keeps its ghost layer fixed
 * (Dirichlet data of the patch); levels L >= 1 refresh their ghosts from the
 * current interior before each half sweep (Sec. 2.4, last paragraph).
 * N0, N: per axis. */
void orc_rb_sweep(int dim, const int *N0, int L, const int *N, double h, double *u, const double *f, int literal)
{
    for (int colour = 0; colour < 2; colour++) {
        if (L > 0) orc_ghost_fill(dim, N0, L, N, u, literal);
        half_sweep(dim, N, h, u, f, colour);
    }
}

/* Residual r = f - lap(u) on active cells; zero on ghosts.  The paper's
 * density residual (step 4) is lap(u) - 4 pi G rho and its coarse problem
 * (step 6) carries a minus sign, so the coarse right-hand side is R(r) with
 * this r. */
void orc_residual(int dim, const int *N, double h, const double *u, const double *f, double *r)
{
    int q[3];
    extents(dim, N, 1, q);
    memset(r, 0, npts(q) * sizeof(double));
    int klo = dim == 3 ? 1 : 0, khi = dim == 3 ? N[2] : 0;
#pragma omp parallel for schedule(static)
    for (int k = klo; k <= khi; k++)
        for (int j = 1; j <= N[1]; j++)
            for (int i = 1; i <= N[0]; i++) {
                size_t c = idx3(q, i, j, k);
                r[c] = f[c] - laplacian(dim, q, u, i, j, k, h);
            }
}

/* max over active cells of |f - lap(u)| */
double orc_residual_norm(int dim, const int *N, double h, const double *u, const double *f)
{
    int q[3];
    extents(dim, N, 1, q);
    int klo = dim == 3 ? 1 : 0, khi = dim == 3 ? N[2] : 0;
    double m = 0.0;
    int bad = 0;
    for (int k = klo; k <= khi; k++)
        for (int j = 1; j <= N[1]; j++)
            for (int i = 1; i <= N[0]; i++) {
                double a = fabs(f[idx3(q, i, j, k)] - laplacian(dim, q, u, i, j, k, h));
                if (!isfinite(a)) bad = 1;
                if (a > m) m = a;
            }
    return bad ? NAN : m;
}

double orc_active_absmax(int dim, const int *N, const double *f)
{
    int q[3];
    extents(dim, N, 1, q);
    int klo = dim == 3 ? 1 : 0, khi = dim == 3 ? N[2] : 0;
    double m = 0.0;
    for (int k = klo; k <= khi; k++)
        for (int j = 1; j <= N[1]; j++)
            for (int i = 1; i <= N[0]; i++) {
                double a = fabs(f[idx3(q, i, j, k)]);
                if (a > m) m = a;
            }
    return m;
}

/* Restriction, eqn:restriction2D/3D: coarse value = mean of the 2^d fine
 * children.  Coarse active cell I covers fine cells 2I-1 and 2I per axis.
 * Children outside the fine active range 1..Nf hold no residual and count as
 * zero (the coarse grids' right edges float, Sec. 2.2). */
void orc_restrict(int dim, const int *Nf, const double *r, const int *Nc, double *fc)
{
    int qf[3], qc[3];
    extents(dim, Nf, 1, qf);
    extents(dim, Nc, 1, qc);
    memset(fc, 0, npts(qc) * sizeof(double));
    int klo = dim == 3 ? 1 : 0, khi = dim == 3 ? Nc[2] : 0;
#pragma omp parallel for schedule(static)
    for (int K = klo; K <= khi; K++)
        for (int J = 1; J <= Nc[1]; J++)
            for (int I = 1; I <= Nc[0]; I++) {
                double sum = 0.0;
                int kc0 = dim == 3 ? 2 * K - 1 : 0, kc1 = dim == 3 ? 2 * K : 0;
                for (int k = kc0; k <= kc1; k++)
                    for (int j = 2 * J - 1; j <= 2 * J; j++)
                        for (int i = 2 * I - 1; i <= 2 * I; i++) {
                            int inside = i <= Nf[0] && j <= Nf[1] && (dim == 2 || k <= Nf[2]);
                            if (inside) sum += r[idx3(qf, i, j, k)];
                        }
                fc[idx3(qc, I, J, K)] = sum / (dim == 3 ? 8.0 : 4.0);
            }
}

/* Multilinear interpolation of eqn:prolongation2D/3D, in the paper's integer
 * form: the nearest coarse value carries 9/16 (2-D) or 27/64 (3-D), each value
 * displaced along one axis 3/16 or 9/64, along two axes 1/16 or 3/64, along
 * three axes 1/64 (Appendix A: bilinear/trilinear interpolation at the
 * quarter points).  `ci/cj/ck` are the nearest coarse indices and `si/sj/sk`
 * the direction (+1/-1) toward the fine point along each axis. */
static double interp_point(int dim, const int *qc, const double *c, int ci, int cj, int ck, int si, int sj,
                           int sk)
{
    if (dim == 2) {
        double A = c[idx3(qc, ci, cj, 0)];
        double B = c[idx3(qc, ci + si, cj, 0)];
        double D = c[idx3(qc, ci, cj + sj, 0)];
        double C = c[idx3(qc, ci + si, cj + sj, 0)];
        return (9.0 * A + 3.0 * B + C + 3.0 * D) / 16.0;
    }
    double near = c[idx3(qc, ci, cj, ck)];
    double face = c[idx3(qc, ci + si, cj, ck)] + c[idx3(qc, ci, cj + sj, ck)] + c[idx3(qc, ci, cj, ck + sk)];
    double edge = c[idx3(qc, ci + si, cj + sj, ck)] + c[idx3(qc, ci + si, cj, ck + sk)] +
                  c[idx3(qc, ci, cj + sj, ck + sk)];
    double corner = c[idx3(qc, ci + si, cj + sj, ck + sk)];
    return (27.0 * near + 9.0 * face + 3.0 * edge + corner) / 64.0;
}

/* Prolongation and correction, step 10: u^{L-1} += P(e^L) on the active
 * cells of level L-1.  Fine active cell a lies in coarse cell ceil(a/2); an
 * odd a is the left child, so its second coarse neighbour is on the left. */
void orc_prolong_add(int dim, const int *Nc, const double *ec, const int *Nf, double *uf)
{
    int qf[3], qc[3];
    extents(dim, Nf, 1, qf);
    extents(dim, Nc, 1, qc);
    int klo = dim == 3 ? 1 : 0, khi = dim == 3 ? Nf[2] : 0;
#pragma omp parallel for schedule(static)
    for (int k = klo; k <= khi; k++)
        for (int j = 1; j <= Nf[1]; j++)
            for (int i = 1; i <= Nf[0]; i++) {
                int ci = (i + 1) / 2, cj = (j + 1) / 2, ck = dim == 3 ? (k + 1) / 2 : 0;
                int si = (i & 1) ? -1 : 1, sj = (j & 1) ? -1 : 1, sk = (k & 1) ? -1 : 1;
                uf[idx3(qf, i, j, k)] += interp_point(dim, qc, ec, ci, cj, ck, si, sj, sk);
            }
}

/* ------------------------------------------------------------------ */
/* One V-cycle, steps 2-13 of Sec. 2.3, on patch storage:
 *   mg_u[0] = potential (level array), mg_f[0] = 4 pi G rho,
 *   mg_u[L], mg_f[L] (L >= 1) = correction and its right-hand side,
 *   mg_r[L] = residual scratch.
 * Coarse corrections start from zero each cycle.  The coarsest level gets
 * only the N_pre sweeps (steps 6-8). */
typedef struct {
    int dim, nmg;
    int N0[3];
    int N[ORC_MAXMG][3];
    double h[ORC_MAXMG];
    double *u[ORC_MAXMG], *f[ORC_MAXMG], *r[ORC_MAXMG];
    int literal;
} orc_mg;

static size_t mg_points(int dim, const int *N)
{
    int q[3];
    extents(dim, N, 1, q);
    return npts(q);
}

/* One V-cycle (Sec. 2.3 steps 2-13): n_pre sweeps before the restriction on
 * every level, n_post after the prolongation on level 0 and n_post_coarse on
 * the levels below it. */
static void vcycle(orc_mg *m, int n_pre, int n_post, int n_post_coarse)
{
    int d = m->dim;
    for (int s = 0; s < n_pre; s++) orc_rb_sweep(d, m->N0, 0, m->N[0], m->h[0], m->u[0], m->f[0], m->literal);
    int L = 0;
    while (L + 1 < m->nmg) {
        if (L > 0) orc_ghost_fill(d, m->N0, L, m->N[L], m->u[L], m->literal);
        orc_residual(d, m->N[L], m->h[L], m->u[L], m->f[L], m->r[L]);
        orc_restrict(d, m->N[L], m->r[L], m->N[L + 1], m->f[L + 1]);
        memset(m->u[L + 1], 0, mg_points(d, m->N[L + 1]) * sizeof(double));
        for (int s = 0; s < n_pre; s++)
            orc_rb_sweep(d, m->N0, L + 1, m->N[L + 1], m->h[L + 1], m->u[L + 1], m->f[L + 1], m->literal);
        L++;
    }
    while (L > 0) {
        orc_ghost_fill(d, m->N0, L, m->N[L], m->u[L], m->literal);
        orc_prolong_add(d, m->N[L], m->u[L], m->N[L - 1], m->u[L - 1]);
        for (int s = 0; s < (L - 1 > 0 ? n_post_coarse : n_post); s++)
            orc_rb_sweep(d, m->N0, L - 1, m->N[L - 1], m->h[L - 1], m->u[L - 1], m->f[L - 1], m->literal);
        L--;
    }
}

/* Largest right-ghost gain |c_L| / (2d) accepted.  The refresh before each
 * half sweep is explicit (lagged), so an error at the last active cell of a
 * multigrid level comes back through its ghost amplified by c_L / (2d); when
 * x_N lies just below 1 the line through zero at x_MG = 1 is steep and c_L
 * large (e.g. -63 for N^0 = 194 at L = 7).  Measured on single patches: the
 * V-cycle keeps its contraction (~0.25) up to gains of about 5 and slows or
 * diverges from 7.75 (2-D) or 10.5 (3-D) on; hierarchies beyond 6 are refused
 * (the printed factor, kept for the negative tests, is not checked). */
#define ORC_MAX_GHOST_GAIN 6.0

int orc_plan_stable(int dim, const int *N0, const int *NL, int nmg)
{
    for (int L = 1; L < nmg; L++)
        for (int a = 0; a < dim; a++) {
            int one;
            double c;
            orc_ghost_rule(N0[a], L, NL[3 * L + a], 0, &one, &c);
            if (!one && fabs(c) > ORC_MAX_GHOST_GAIN * 2.0 * dim) return 0;
        }
    return 1;
}

/* Multigrid hierarchy of a patch whose level-0 grid has N0[a] cells per axis. */
static int mg_plan(orc_mg *m, int dim, const int *N0)
{
    int NL[ORC_MAXMG * 3];
    m->dim = dim;
    for (int a = 0; a < 3; a++) m->N0[a] = a < dim ? N0[a] : 1;
    m->nmg = orc_plan3(dim, m->N0, NL, ORC_MAXMG);
    if (m->nmg < 1) return -1;
    if (!m->literal && !orc_plan_stable(dim, m->N0, NL, m->nmg)) return -1;
    for (int L = 0; L < m->nmg; L++)
        for (int a = 0; a < 3; a++) m->N[L][a] = NL[3 * L + a];
    return 0;
}

/* ------------------------------------------------------------------ */
/* Coarse-to-fine fill of patch l >= 1 (Sec. 2.1, Sec. 2.4 first paragraph):
 * the potential on every padded point (outer buffer = Dirichlet data, the
 * rest = initial guess) and the right-hand side on the inner buffer layer are
 * interpolated from level l-1; Omega^l takes the caller's density.  Fine
 * padded index p along an axis is fine cell p-2, which sits in coarse cell
 * off + floor((p-2)/2), i.e. coarse padded index q = off + 2 + floor((p-2)/2);
 * an even p-2 is a left child, so the second coarse point is q-1.
 * Interpolating f = 4 pi G rho is the same linear map as interpolating rho.
 * nc, nf: cells per axis of the coarse and the fine patch. */
void orc_interface_fill(int dim, const int *nc, const double *phic, const double *fc, const int *nf, const int *off,
                        const double *rho, double fourpiG, double *phif, double *ff)
{
    int Pc[3], Pf[3];
    extents(dim, nc, 2, Pc);
    extents(dim, nf, 2, Pf);
    int kmax = dim == 3 ? Pf[2] - 1 : 0;
    for (int k = 0; k <= kmax; k++)
        for (int j = 0; j < Pf[1]; j++)
            for (int i = 0; i < Pf[0]; i++) {
                int p[3] = {i, j, k}, q[3] = {0, 0, 0}, s[3] = {0, 0, 0};
                for (int a = 0; a < dim; a++) {
                    int fine = p[a] - 2;
                    int fl = (fine >= 0) ? fine / 2 : -((1 - fine) / 2); /* floor(fine/2) */
                    q[a] = off[a] + 2 + fl;
                    s[a] = (fine % 2 == 0) ? -1 : 1;
                }
                size_t c = idx3(Pf, i, j, k);
                phif[c] = interp_point(dim, Pc, phic, q[0], q[1], q[2], s[0], s[1], s[2]);
                int ring = 0, omega = 1;
                for (int a = 0; a < dim; a++) {
                    if (p[a] == 0 || p[a] == Pf[a] - 1) ring = 2;
                    else if ((p[a] == 1 || p[a] == Pf[a] - 2) && ring < 1) ring = 1;
                    if (p[a] < 2 || p[a] > nf[a] + 1) omega = 0;
                }
                if (omega) {
                    size_t ri = dim == 3 ? (((size_t)(k - 2) * nf[1] + (j - 2)) * nf[0] + (i - 2))
                                         : ((size_t)(j - 2) * nf[0] + (i - 2));
                    ff[c] = fourpiG * rho[ri];
                } else if (ring == 1) {
                    ff[c] = interp_point(dim, Pc, fc, q[0], q[1], q[2], s[0], s[1], s[2]);
                } else {
                    ff[c] = 0.0;
                }
            }
}

/* Forces F = -grad(Phi) on Omega^l with the fourth-order central difference
 * of Eqn:force_evaluation: dPhi/dx = (4/3)(Phi_{i+1}-Phi_{i-1})/(2 dx)
 *                                  - (1/3)(Phi_{i+2}-Phi_{i-2})/(4 dx).
 * Output arrays are n_z x n_y x n_x (n_y x n_x in 2-D), natural order. */
void orc_forces(int dim, const int *n, double dx, const double *phi, double *fx, double *fy, double *fz)
{
    int P[3];
    extents(dim, n, 2, P);
    int kmax = dim == 3 ? n[2] - 1 : 0;
    for (int k = 0; k <= kmax; k++)
        for (int j = 0; j < n[1]; j++)
            for (int i = 0; i < n[0]; i++) {
                int pi = i + 2, pj = j + 2, pk = dim == 3 ? k + 2 : 0;
                size_t o = dim == 3 ? (((size_t)k * n[1] + j) * n[0] + i) : ((size_t)j * n[0] + i);
                double dpx = (4.0 / 3.0) * (phi[idx3(P, pi + 1, pj, pk)] - phi[idx3(P, pi - 1, pj, pk)]) / (2.0 * dx) -
                             (1.0 / 3.0) * (phi[idx3(P, pi + 2, pj, pk)] - phi[idx3(P, pi - 2, pj, pk)]) / (4.0 * dx);
                double dpy = (4.0 / 3.0) * (phi[idx3(P, pi, pj + 1, pk)] - phi[idx3(P, pi, pj - 1, pk)]) / (2.0 * dx) -
                             (1.0 / 3.0) * (phi[idx3(P, pi, pj + 2, pk)] - phi[idx3(P, pi, pj - 2, pk)]) / (4.0 * dx);
                fx[o] = -dpx;
                fy[o] = -dpy;
                if (dim == 3) {
                    double dpz = (4.0 / 3.0) * (phi[idx3(P, pi, pj, pk + 1)] - phi[idx3(P, pi, pj, pk - 1)]) / (2.0 * dx) -
                                 (1.0 / 3.0) * (phi[idx3(P, pi, pj, pk + 2)] - phi[idx3(P, pi, pj, pk - 2)]) / (4.0 * dx);
                    fz[o] = -dpz;
                }
            }
}

/* ------------------------------------------------------------------ */
/* Validation of the nested geometry: returns 0 or a negative code.  Every
 * patch has an even number (>= 4) of cells along each axis, sits on whole
 * cells of its parent with one parent cell of margin on every side, and does
 * not overlap its siblings. */
int orc_validate(const orc_config *cfg)
{
    if (cfg->dim != 2 && cfg->dim != 3) return -1;
    if (cfg->nlevels < 1 || cfg->nlevels > ORC_MAXLEV) return -1;
    for (int l = 0; l < cfg->nlevels; l++) {
        for (int a = 0; a < cfg->dim; a++)
            if (cfg->n[l][a] < 4 || (cfg->n[l][a] & 1)) return -1;
        if (l == 0) continue;
        int p = cfg->parent[l];
        if (p < 0 || p >= l) return -1;
        for (int a = 0; a < cfg->dim; a++) {
            int o = cfg->off[l][a];
            if (o < 1 || o + cfg->n[l][a] / 2 > cfg->n[p][a] - 1) return -1;
        }
        /* siblings (same parent) must not overlap */
        for (int m = 1; m < l; m++) {
            if (cfg->parent[m] != p) continue;
            int apart = 0;
            for (int a = 0; a < cfg->dim; a++) {
                int lo1 = cfg->off[l][a], hi1 = lo1 + cfg->n[l][a] / 2;
                int lo2 = cfg->off[m][a], hi2 = lo2 + cfg->n[m][a] / 2;
                if (hi1 <= lo2 || hi2 <= lo1) apart = 1;
            }
            if (!apart) return -1;
        }
    }
    if (!(cfg->dx0 > 0.0)) return -1;
    if (cfg->buffer_interp && cfg->stop_rule != 0) return -1;
    return 0;
}

static double maxabs_diff(size_t m, const double *a, const double *b)
{
    double x = 0.0;
    for (size_t i = 0; i < m; i++) {
        double t = fabs(a[i] - b[i]);
        if (!(t <= x)) x = t; /* propagates NaN */
    }
    return x;
}

/* Nested solve, one-way scheme (Sec. 2.1): level 0 first, each finer level
 * from the converged coarser one.
 *   rho[0]  : (n0_a + 2) per axis, Omega^0 plus its inner buffer layer (caller data)
 *   rho[l]  : n_l,a per axis on Omega^l (l >= 1)
 *   phi_outer: (n0_a + 4) per axis, only its outer layer is read (Dirichlet data of level 0)
 *   phi[l]  : out, (n_l,a + 4) per axis padded potential
 *   fixed_cycles: NULL, or per-level cycle counts to run instead of the stop rule
 *   cycles, final_rel: out per level; hist: NULL or out, nlevels*(max_cycles+1)
 *     relative residual before the first cycle and after each cycle.
 * Returns 0, -2 (non-finite), -3 (cap reached without convergence),
 * -4 (diverged), -1 (invalid geometry or allocation failure). */
int orc_solve(const orc_config *cfg, const double *const *rho, const double *phi_outer, double **phi,
              const int *fixed_cycles, int *cycles, double *final_rel, double *hist)
{
    if (orc_validate(cfg)) return -1;
    int d = cfg->dim;
    double fourpiG = 4.0 * M_PI * cfg->G;
    int status = 0;
    double *fl[ORC_MAXLEV] = {0};
    for (int l = 0; l < cfg->nlevels; l++) {
        int P[3];
        extents(d, cfg->n[l], 2, P);
        fl[l] = calloc(npts(P), sizeof(double));
        if (!fl[l]) { status = -1; goto done; }
    }
    for (int l = 0; l < cfg->nlevels; l++) {
        const int *n = cfg->n[l];
        int P[3];
        extents(d, n, 2, P);
        double dx = ldexp(cfg->dx0, -depth_of(cfg, l));
        size_t m0 = npts(P);
        double *f0 = fl[l];
        double *u0 = phi[l];
        if (l == 0) {
            /* Dirichlet data from the caller; Gamma^0 starts from zero */
            memcpy(u0, phi_outer, m0 * sizeof(double));
            int kmin = d == 3 ? 1 : 0, kmax = d == 3 ? P[2] - 2 : 0;
            for (int k = kmin; k <= kmax; k++)
                for (int j = 1; j <= P[1] - 2; j++)
                    for (int i = 1; i <= P[0] - 2; i++) {
                        size_t c = idx3(P, i, j, k);
                        u0[c] = 0.0;
                        size_t ri = d == 3 ? (((size_t)(k - 1) * (n[1] + 2) + (j - 1)) * (n[0] + 2) + (i - 1))
                                           : ((size_t)(j - 1) * (n[0] + 2) + (i - 1));
                        f0[c] = fourpiG * rho[0][ri];
                    }
        } else {
            int p = cfg->parent[l];
            orc_interface_fill(d, cfg->n[p], phi[p], fl[p], n, cfg->off[l], rho[l], fourpiG, u0, f0);
        }

        /* The relaxed domain: Gamma^l (N^0 = n + 2 per axis) with the outer
         * buffer layer as its ghost layer, which is the level array itself; or,
         * for the comparison scheme of Sec. 4 (Fig. 4: the buffer values come
         * from the coarse level by linear interpolation), Omega^l alone
         * (N^0 = n) in an array of its own whose ghost layer is the
         * interpolated inner buffer layer.  Its active values go back into the
         * level array afterwards. */
        int interp_buffer = l > 0 && cfg->buffer_interp;
        int N0[3], Ps[3];
        for (int a = 0; a < 3; a++) N0[a] = a < d ? (interp_buffer ? n[a] : n[a] + 2) : 1;
        extents(d, N0, 1, Ps);
        size_t ms = npts(Ps);
        double *us = u0, *fs = f0;
        if (interp_buffer) {
            us = malloc(ms * sizeof(double));
            fs = malloc(ms * sizeof(double));
            if (!us || !fs) {
                free(us);
                free(fs);
                status = -1;
                goto done;
            }
            int kmax = d == 3 ? Ps[2] - 1 : 0;
            for (int k = 0; k <= kmax; k++)
                for (int j = 0; j < Ps[1]; j++)
                    for (int i = 0; i < Ps[0]; i++) {
                        size_t src = idx3(P, i + 1, j + 1, d == 3 ? k + 1 : 0);
                        us[idx3(Ps, i, j, k)] = u0[src];
                        fs[idx3(Ps, i, j, k)] = f0[src];
                    }
        }

        orc_mg m;
        memset(&m, 0, sizeof m);
        m.literal = cfg->ghost_literal;
        if (mg_plan(&m, d, N0)) {
            if (interp_buffer) {
                free(us);
                free(fs);
            }
            status = -1;
            goto done;
        }
        m.u[0] = us;
        m.f[0] = fs;
        int oom = 0;
        for (int L = 0; L < m.nmg; L++) {
            m.h[L] = dx * ldexp(1.0, L);
            size_t mm = mg_points(d, m.N[L]);
            if (L > 0) {
                m.u[L] = calloc(mm, sizeof(double));
                m.f[L] = calloc(mm, sizeof(double));
                if (!m.u[L] || !m.f[L]) oom = 1;
            }
            m.r[L] = calloc(mm, sizeof(double));
            if (!m.r[L]) oom = 1;
        }

        /* reference scale of the stop test: ||f||_inf over Gamma^l, or, for a
         * zero density, the residual of the zero potential */
        double scale = orc_active_absmax(d, m.N[0], fs);
        if (!(scale > 0.0) && !oom) {
            double *z = malloc(ms * sizeof(double));
            if (!z) oom = 1;
            else {
                memcpy(z, us, ms * sizeof(double));
                int kmin = d == 3 ? 1 : 0, kmax = d == 3 ? Ps[2] - 2 : 0;
                for (int k = kmin; k <= kmax; k++)
                    for (int j = 1; j <= Ps[1] - 2; j++)
                        for (int i = 1; i <= Ps[0] - 2; i++) z[idx3(Ps, i, j, k)] = 0.0;
                scale = orc_residual_norm(d, m.N[0], m.h[0], z, fs);
                free(z);
            }
        }

        size_t nf = (size_t)n[0] * n[1] * (d == 3 ? n[2] : 1);
        double *Fprev = NULL, *Fcur = NULL;
        if (cfg->stop_rule == 1 && !oom) {
            Fprev = calloc(3 * nf, sizeof(double));
            Fcur = calloc(3 * nf, sizeof(double));
            if (!Fprev || !Fcur) oom = 1;
            else orc_forces(d, n, dx, u0, Fprev, Fprev + nf, Fprev + 2 * nf);
        }

        int lvl_status = 0, q = 0;
        double r = 0.0;
        if (oom) lvl_status = -1;
        else {
            r = orc_residual_norm(d, m.N[0], m.h[0], us, fs);
            double r0 = r;
            double *hl = hist ? hist + (size_t)l * (cfg->max_cycles + 1) : NULL;
            if (hl) hl[0] = scale > 0 ? r / scale : r;
            int pinned = fixed_cycles && fixed_cycles[l] >= 0;
            for (;;) {
                if (!isfinite(r)) { lvl_status = -2; break; }
                if (pinned) {
                    if (q >= fixed_cycles[l]) break;
                } else if (cfg->stop_rule == 0 && r <= cfg->tol * scale) {
                    break;
                }
                if (q >= cfg->max_cycles) { lvl_status = -3; break; }
                vcycle(&m, cfg->n_pre, cfg->n_post, cfg->coarse_post >= 0 ? cfg->coarse_post : cfg->n_post);
                q++;
                r = orc_residual_norm(d, m.N[0], m.h[0], us, fs);
                if (hl && q <= cfg->max_cycles) hl[q] = scale > 0 ? r / scale : r;
                if (!isfinite(r)) { lvl_status = -2; break; }
                if (r0 > 0 && r > 1e3 * r0) { lvl_status = -4; break; }
                if (cfg->stop_rule == 1 && !pinned) {
                    orc_forces(d, n, dx, u0, Fcur, Fcur + nf, Fcur + 2 * nf);
                    double dF = maxabs_diff((size_t)d * nf, Fcur, Fprev);
                    double *t = Fprev; Fprev = Fcur; Fcur = t;
                    if (dF < cfg->tol) break;
                }
            }
        }
        if (interp_buffer) {
            int kmin = d == 3 ? 1 : 0, kmax = d == 3 ? n[2] : 0;
            for (int k = kmin; k <= kmax; k++)
                for (int j = 1; j <= n[1]; j++)
                    for (int i = 1; i <= n[0]; i++) u0[idx3(P, i + 1, j + 1, d == 3 ? k + 1 : 0)] = us[idx3(Ps, i, j, k)];
            free(us);
            free(fs);
        }
        cycles[l] = q;
        final_rel[l] = scale > 0 ? r / scale : r;
        free(Fprev);
        free(Fcur);
        for (int L = 0; L < m.nmg; L++) {
            if (L > 0) { free(m.u[L]); free(m.f[L]); }
            free(m.r[L]);
        }
        if (lvl_status && !status) status = lvl_status;
        if (lvl_status == -1 || lvl_status == -2 || lvl_status == -4) goto done;
    }
done:
    for (int l = 0; l < cfg->nlevels; l++) free(fl[l]);
    return status;
}

/* ------------------------------------------------------------------ */
/* Single-patch entry points used by the operator tests. */

/* one V-cycle on a single patch with caller-provided level-0 arrays
 * (N0[a] + 2 points per axis: potential with fixed ghosts, and f); the levels
 * below level 0 take n_post_coarse post-smoothing sweeps (-1: n_post) */
int orc_vcycle_patch(int dim, const int *N0, double h0, double *u, const double *f, int n_pre, int n_post,
                     int n_post_coarse, int literal)
{
    orc_mg m;
    memset(&m, 0, sizeof m);
    m.literal = literal;
    if (mg_plan(&m, dim, N0)) return -1;
    m.u[0] = u;
    m.f[0] = (double *)f;
    for (int L = 0; L < m.nmg; L++) {
        m.h[L] = h0 * ldexp(1.0, L);
        size_t mm = mg_points(dim, m.N[L]);
        if (L > 0) {
            m.u[L] = calloc(mm, sizeof(double));
            m.f[L] = calloc(mm, sizeof(double));
        }
        m.r[L] = calloc(mm, sizeof(double));
    }
    vcycle(&m, n_pre, n_post, n_post_coarse >= 0 ? n_post_coarse : n_post);
    for (int L = 0; L < m.nmg; L++) {
        if (L > 0) { free(m.u[L]); free(m.f[L]); }
        free(m.r[L]);
    }
    return 0;
}

/* threads the OpenMP loops of the oracle use */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* thread count of the parallel loops (timing at 1 thread and at all cores);
 * results do not depend on it: every parallel loop updates independent points */
void orc_set_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
}

// Host runtime of the nested-grid multigrid solver: geometry validation,
// multigrid planning, device storage, the V-cycle schedule and the C ABI
// declared in include/nested_poisson.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/nested_poisson.h"
#include "np_internal.h"

using namespace np;

// Entries solved together: patches of one refinement depth with the same
// extents, whose V-cycles and stop-test norms run as one launch per operator
// over the group (one grid row per patch), or a single entry.
struct PatchGroup {
    int n;
    int member[NP_MAX_LEVELS];
};

namespace {

// ------------------------------------------------------------------ planning
// Cells of level l along axis a (Sec. 2.1: counts per direction; a cube when
// the per-axis extents are not given).
int level_n(const np_config* c, int l, int a)
{
    if (a >= c->dim) return 1;
    return c->extent[l][0] > 0 ? c->extent[l][a] : c->n[l];
}

// Validation of the nested geometry (Sec. 2.1): even cell counts of at least
// 4, patches on whole coarse cells with one coarse cell of margin.
bool validate(const np_config* c, char* why, size_t nwhy)
{
    auto fail = [&](const char* fmt, auto... args) {
        if constexpr (sizeof...(args) == 0)
            snprintf(why, nwhy, "%s", fmt);
        else
            snprintf(why, nwhy, fmt, args...);
        return false;
    };
    if (!c) return fail("null config");
    if (c->dim != 2 && c->dim != 3) return fail("dim must be 2 or 3 (got %d)", c->dim);
    if (c->nlevels < 1 || c->nlevels > NP_MAX_LEVELS) return fail("nlevels must be 1..%d (got %d)", NP_MAX_LEVELS, c->nlevels);
    for (int l = 0; l < c->nlevels; l++) {
        for (int a = 0; a < c->dim; a++) {
            const int n = level_n(c, l, a);
            if (n < 4 || (n & 1)) return fail("level %d: cells along axis %d must be even and >= 4 (got %d)", l, a, n);
            if (n > 1 << 14) return fail("level %d: too many cells along axis %d (%d)", l, a, n);
        }
        if (l == 0) continue;
        const int p = c->parent[l];
        if (p < 0 || p >= l) return fail("level %d: parent %d must name an earlier entry", l, p);
        for (int a = 0; a < c->dim; a++) {
            int o = c->offset[l][a];
            if (o < 1 || o + level_n(c, l, a) / 2 > level_n(c, p, a) - 1)
                return fail("level %d: offset leaves less than one coarse cell of margin on axis %d", l, a);
        }
        // patches refined out of the same parent do not overlap
        for (int m = 1; m < l; m++) {
            if (c->parent[m] != p) continue;
            bool overlap = true;
            for (int a = 0; a < c->dim; a++) {
                const int lo1 = c->offset[l][a], hi1 = lo1 + level_n(c, l, a) / 2;
                const int lo2 = c->offset[m][a], hi2 = lo2 + level_n(c, m, a) / 2;
                if (hi1 <= lo2 || hi2 <= lo1) overlap = false;
            }
            if (overlap) return fail("levels %d and %d: patches of the same parent overlap", m, l);
        }
    }
    if (!(c->dx0 > 0.0) || !std::isfinite(c->dx0)) return fail("dx0 must be positive");
    if (!std::isfinite(c->G)) return fail("G must be finite");
    if (c->n_pre < 0 || c->n_pre > 16 || c->n_post < 0 || c->n_post > 16)
        return fail("n_pre/n_post must be 0..16 (got %d, %d)", c->n_pre, c->n_post);
    if (!(c->tol > 0.0)) return fail("tol must be positive");
    if (c->max_cycles < 1 || c->max_cycles > NP_MAX_CYCLES) return fail("max_cycles must be 1..%d (got %d)", NP_MAX_CYCLES, c->max_cycles);
    if (c->stop_rule != NP_STOP_RESIDUAL && c->stop_rule != NP_STOP_FORCE_DELTA) return fail("bad stop_rule %d", c->stop_rule);
    if (c->precision != NP_PREC_FP64 && c->precision != NP_PREC_FP32_DC && c->precision != NP_PREC_FP16S_DC)
        return fail("bad precision %d", c->precision);
    if (c->guess != NP_GUESS_INTERP && c->guess != NP_GUESS_LEARNED) return fail("bad guess %d", c->guess);
    if (c->guess == NP_GUESS_LEARNED && c->dim != 3) return fail("the learned guess is 3-D only (dim %d)", c->dim);
    if (c->inner_cycles < 0 || c->inner_cycles > 8)
        return fail("inner_cycles must be 0 (adaptive) or 1..8 (got %d)", c->inner_cycles);
    if (c->buffer != NP_BUFFER_RELAXED && c->buffer != NP_BUFFER_INTERP) return fail("bad buffer %d", c->buffer);
    if (c->buffer == NP_BUFFER_INTERP &&
        (c->precision != NP_PREC_FP64 || c->guess != NP_GUESS_INTERP || c->stop_rule != NP_STOP_RESIDUAL))
        return fail("the interpolated buffer runs with FP64, the interpolated guess and the residual stop "
                    "rule only");
    if (c->batch != 0 && c->batch != 1) return fail("batch must be 0 or 1 (got %d)", c->batch);
    if (c->guess_gate != 0 && c->guess_gate != 1) return fail("guess_gate must be 0 or 1 (got %d)", c->guess_gate);
    if (c->coarse_post < -1 || c->coarse_post > 16) return fail("coarse_post must be -1..16 (got %d)", c->coarse_post);
    if (c->sweep != NP_SWEEP_FULL && c->sweep != NP_SWEEP_HALF && c->sweep != NP_SWEEP_FUSED &&
        c->sweep != NP_SWEEP_FULL_ALL)
        return fail("bad sweep %d", c->sweep);
    return true;
}

// Whether patches of one depth and extents are solved as one batch: with
// batch = 1 in FP64, with the interpolated guess, the relaxed buffer and the
// residual stop rule (their per-patch state is the potential, the right-hand
// side and the stop test only).
bool batching(const np_config* c)
{
    return c->batch == 1 && c->precision == NP_PREC_FP64 && c->guess == NP_GUESS_INTERP &&
           c->buffer == NP_BUFFER_RELAXED && c->stop_rule == NP_STOP_RESIDUAL;
}

// Sec. 2.2 along every axis: N^0_a = n_a + 2; N^L_a = round(N^0_a / 2^L),
// halves up (the same doubling of h on every axis); the hierarchy ends on the
// first level with one active cell along some axis.  NL[L][a]; returns the
// number of levels.
int plan_levels(int dim, const int* N0, int (*NL)[3])
{
    for (int a = 0; a < 3; a++) NL[0][a] = a < dim ? N0[a] : 1;
    int L = 0;
    for (;;) {
        bool one = false;
        for (int a = 0; a < dim; a++)
            if (NL[L][a] <= 1) one = true;
        if (one) break;
        if (L + 1 >= NP_MAX_MG) return -1;
        L++;
        for (int a = 0; a < 3; a++)
            NL[L][a] = a < dim ? (int)(((long long)N0[a] + (1LL << (L - 1))) >> L) : 1;
    }
    return L + 1;
}

// Sec. 2.4 right ghost of level L: the line through (x_N, e_N) vanishing at
// x_MG = 1, evaluated at x_N + h^L; with x_N = (N - 1/2) 2^L / N^0 the factor
// is (2 N^0 - (2N+1) 2^L) / (2 N^0 - (2N-1) 2^L).  x_N = 1 exactly when
// (2N - 1) 2^(L-1) = N^0, where the rule is e_{N+1} = -e_{N-1}.
void ghost_rule(int N0, int L, int N, int* one, double* coef)
{
    long long twoL = 1LL << L;
    *one = ((long long)(2 * N - 1) * (twoL / 2) == (long long)N0) ? 1 : 0;
    double num = 2.0 * N0 - (double)((2LL * N + 1) * twoL);
    double den = 2.0 * N0 - (double)((2LL * N - 1) * twoL);
    *coef = *one ? -1.0 : num / den;
}

// The kernels index coarse grids from fine ones; these bounds (per axis) are
// what keeps every access inside the padded arrays:
//   prolongation: fine active a in 1..Nf reads coarse ceil(a/2) and its
//     neighbour towards a, so ceil(Nf/2) <= Nc + 1 and floor(Nf/2) <= Nc;
//   restriction: coarse I in 1..Nc has children 2I-1, 2I <= Nf + 1;
//   the x_N = 1 rule reads e_{N-1}, so N >= 2 there.
bool plan_in_bounds(const np_plan* p, int l, int dim)
{
    for (int a = 0; a < dim; a++) {
        for (int L = 0; L + 1 < p->nmg[l]; L++) {
            int Nf = p->N[l][L][a], Nc = p->N[l][L + 1][a];
            if ((Nf + 1) / 2 > Nc + 1 || Nf / 2 > Nc || 2 * Nc > Nf + 1) return false;
        }
        for (int L = 1; L < p->nmg[l]; L++)
            if (p->xn_is_one[l][L][a] && p->N[l][L][a] < 2) return false;
    }
    return true;
}

// N^0 of nested level l along axis a: the patch and its inner buffer layer, or
// the patch alone where the buffer keeps its interpolated values (levels l >= 1)
int level_N0(const np_config* c, int l, int a)
{
    return (l > 0 && c->buffer == NP_BUFFER_INTERP) ? level_n(c, l, a) : level_n(c, l, a) + 2;
}

// refinement depth of entry l (0 for the base level) and its cell size dx0 / 2^depth
int level_depth(const np_config* c, int l)
{
    int k = 0;
    while (l > 0) {
        l = c->parent[l];
        k++;
    }
    return k;
}

// Solve order: with batching, the entries by depth (then index), grouped by
// extents within a depth; every parent lies at a smaller depth, so it is
// solved in an earlier group (one-way scheme).  Otherwise one entry per group
// in entry order (a parent is always an earlier entry).
int make_groups(const np_config* c, PatchGroup* g)
{
    int ng = 0;
    if (!batching(c)) {
        for (int l = 0; l < c->nlevels; l++) {
            g[ng].n = 1;
            g[ng].member[0] = l;
            ng++;
        }
        return ng;
    }
    int maxd = 0;
    for (int l = 0; l < c->nlevels; l++) maxd = std::max(maxd, level_depth(c, l));
    for (int dep = 0; dep <= maxd; dep++) {
        const int first = ng;
        for (int l = 0; l < c->nlevels; l++) {
            if (level_depth(c, l) != dep) continue;
            int k = first;
            for (; k < ng; k++) {
                const int m = g[k].member[0];
                bool same = true;
                for (int a = 0; a < c->dim; a++)
                    if (level_n(c, l, a) != level_n(c, m, a)) same = false;
                if (same) break;
            }
            if (k == ng) {
                g[ng].n = 0;
                ng++;
            }
            g[k].member[g[k].n++] = l;
        }
    }
    return ng;
}
double level_dx(const np_config* c, int l) { return std::ldexp(c->dx0, -level_depth(c, l)); }

// Returns NP_OK, or NP_EINVAL with the reason in `why`.
int make_plan(const np_config* c, np_plan* p, char* why, size_t nwhy)
{
    memset(p, 0, sizeof(*p));
    const int d = c->dim;
    for (int l = 0; l < c->nlevels; l++) {
        int N0[3];
        for (int a = 0; a < 3; a++) N0[a] = a < d ? level_N0(c, l, a) : 1;
        int m = plan_levels(d, N0, p->N[l]);
        if (m < 2) {
            snprintf(why, nwhy, "level %d: multigrid hierarchy too deep", l);
            return NP_EINVAL;
        }
        p->nmg[l] = m;
        for (int L = 1; L < m; L++)
            for (int a = 0; a < 3; a++) {
                if (a < d) {
                    ghost_rule(N0[a], L, p->N[l][L][a], &p->xn_is_one[l][L][a], &p->ghost_coef[l][L][a]);
                    if (!p->xn_is_one[l][L][a] && std::fabs(p->ghost_coef[l][L][a]) > NP_MAX_GHOST_GAIN * 2.0 * d) {
                        snprintf(why, nwhy,
                                 "level %d: right-ghost coefficient %.3g of multigrid level %d on axis %d exceeds "
                                 "%g x 2d (the explicit ghost refresh would make the V-cycle diverge)",
                                 l, p->ghost_coef[l][L][a], L, a, NP_MAX_GHOST_GAIN);
                        return NP_EINVAL;
                    }
                } else {
                    p->xn_is_one[l][L][a] = 0;
                    p->ghost_coef[l][L][a] = 0.0;
                }
            }
        if (!plan_in_bounds(p, l, d)) {
            snprintf(why, nwhy, "level %d: multigrid hierarchy out of the kernels' index bounds", l);
            return NP_EINVAL;
        }
    }
    return NP_OK;
}

double bits_to_double(unsigned long long b)
{
    double d;
    memcpy(&d, &b, sizeof d);
    return d;
}

thread_local char g_last_error[256] = "";

}  // namespace

namespace np {
void set_last_error(const char* msg) { snprintf(g_last_error, sizeof g_last_error, "%s", msg); }
}  // namespace np

// ------------------------------------------------------------------ handle
// device reduction slots: 0 norm, 1 force change, 2 max |f| of a fill,
// 3 restricted residual; kBatchSlot + b the norm of batch member b
constexpr int kBatchSlot = 8;
constexpr int kBitSlots = kBatchSlot + NP_MAX_LEVELS;

struct np_solver {
    np_config cfg;
    np_plan plan;
    int ngroups = 0;
    PatchGroup groups[NP_MAX_LEVELS];
    bool owns[NP_MAX_LEVELS] = {};  // phi[l] and f[l] own their allocation (else inside a group's)
    int* d_act = nullptr;           // device flags of the batch members still iterating
    int* h_act = nullptr;           // pinned host copy
    hipStream_t stream = nullptr;
    int device = 0;
    SGrid lg[NP_MAX_LEVELS];          // level grids (= multigrid level 0)
    double* phi[NP_MAX_LEVELS] = {};  // split potential per level
    double* f[NP_MAX_LEVELS] = {};    // split right-hand side per level
    // multigrid scratch for L >= 1, shared by the levels (sized for the largest)
    double* mg_u[NP_MAX_MG] = {};
    double* mg_f[NP_MAX_MG] = {};
    double* force_scratch = nullptr;  // FORCE_DELTA stop rule
    unsigned long long* d_bits = nullptr;  // device reduction slots
    unsigned long long* h_bits = nullptr;  // pinned host copy
    int fixed[NP_MAX_LEVELS];
    bool has_fixed = false;
    bool solved = false;
    std::vector<double> hist[NP_MAX_LEVELS];
    char err[512] = {0};
    // kernel-class timing with HIP events on the handle's stream
    bool prof = false;
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    std::vector<int> ev_cls;
    std::vector<int> ev_n;  // kernel launches inside each interval
    int ev_used = 0;
    int cur_cls = 0;
    long prof_count[NP_NKCLASS] = {};
    double prof_ms[NP_NKCLASS] = {};
    // coarse part of the V-cycle as one HIP graph per nested level
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t coarse_exec[NP_MAX_LEVELS] = {};
    // mixed-precision defect correction: level-0 correction and defect in
    // FP32 or FP16 (colour-split, sized for the largest level), FP32 coarse levels
    // e_lo is the correction the inner cycles work on, e_nx the one the next
    // outer pass starts; phi_alt is the second FP64 potential buffer the outer
    // pass writes the updated potential into (the pointers rotate)
    void* e_lo = nullptr;
    void* e_nx = nullptr;
    void* r_lo = nullptr;
    // the grid whose ghost layers in e_lo, e_nx and r_lo are known to be zero
    // (no kernel writes a ghost point of these arrays; -1: not cleared yet)
    SGrid lo_ghost_grid{-1, -1, -1, 0, 0, 0};
    // f - lap phi of a level's starting potential in FP32 (active points; zero
    // elsewhere, cleared when the grid changes: r32_grid), from which its first
    // scaled defect is formed
    float* r32 = nullptr;
    SGrid r32_grid{-1, -1, -1, 0, 0, 0};
    size_t lo_bytes = 0;
    double* phi_alt = nullptr;
    size_t alt_cap = 0;
    int fs_rev = 0;  // z order of the next full sweep (alternates; cache reuse only)
    size_t phi_cap[NP_MAX_LEVELS] = {};
    float* mg_u32[NP_MAX_MG] = {};
    float* mg_f32[NP_MAX_MG] = {};
    hipGraphExec_t coarse_exec32[NP_MAX_LEVELS] = {};
    // learned initial guess: weights (bfloat16 per layer, FP32 biases) and
    // activations on Gamma of the largest level
    bool have_weights = false;
    // contraction per V-cycle measured on each level's last solve (the keep
    // test of a child's learned guess), and the restricted-residual ratio of
    // each level's learned guess against the interpolated one
    double rho_meas[NP_MAX_LEVELS] = {};
    double guess_box_ratio[NP_MAX_LEVELS] = {};
    // levels on which the learned guess was found not to pay (guess_gate)
    bool guess_off[NP_MAX_LEVELS] = {};
    uint16_t* net_w[3] = {};
    float* net_b[3] = {};
    uint16_t* net_x = nullptr;
    uint16_t* net_a1 = nullptr;
    uint16_t* net_a2 = nullptr;
    float* net_out = nullptr;
    // training-feature scratch (interpolated guess of one level), on demand
    double* feat_phi = nullptr;
    double* feat_f = nullptr;
    // NP_BUFFER_INTERP: the relaxed domain of a level l >= 1 (Omega^l, its ghost
    // layer the inner buffer layer), (n + 2)^d colour-split, sized for the largest level
    SGrid ag[NP_MAX_LEVELS];
    double* ab_phi = nullptr;
    double* ab_f = nullptr;
};

namespace {

int set_err(np_solver* s, int code, const char* fmt, ...)
{
    if (s) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(s->err, sizeof s->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIPCHK(s, call)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return set_err((s), NP_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

SGrid mg_grid(const np_solver* s, int l, int L)
{
    const int* N = s->plan.N[l][L];
    return make_grid(s->cfg.dim, N[0] + 2, N[1] + 2, N[2] + 2);
}

// padded grid of nested level l (n_a + 4 points per axis)
SGrid level_grid(const np_config* c, int l)
{
    return make_grid(c->dim, level_n(c, l, 0) + 4, level_n(c, l, 1) + 4, level_n(c, l, 2) + 4);
}

// right-ghost rule of multigrid level L of nested level l, per axis
Rule3 rule_of(const np_solver* s, int l, int L)
{
    Rule3 r{};
    for (int a = 0; a < 3; a++) {
        r.xn1[a] = s->plan.xn_is_one[l][L][a];
        r.coef[a] = s->plan.ghost_coef[l][L][a];
    }
    return r;
}

bool same_grid(const SGrid& a, const SGrid& b) { return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz; }

// Fold the recorded event pairs into the per-class totals (synchronises).
int prof_flush(np_solver* s)
{
    if (!s->ev_used) return NP_OK;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int i = 0; i + 1 < s->ev_used; i += 2) {
        float ms = 0.f;
        HIPCHK(s, hipEventElapsedTime(&ms, s->ev[i], s->ev[i + 1]));
        int c = s->ev_cls[i / 2];
        s->prof_ms[c] += ms;
        s->prof_count[c] += s->ev_n[i / 2];
    }
    s->ev_used = 0;
    return NP_OK;
}

void prof_begin(np_solver* s, int cls)
{
    if (!s->prof) return;
    if (s->ev_used + 2 > (int)s->ev.size()) prof_flush(s);
    s->cur_cls = cls;
    (void)hipEventRecord(s->ev[s->ev_used], s->stream);
}

// closes the interval opened by prof_begin; it held `launches` kernels of the
// class (back to back on the stream), whose average duration the profile reports
void prof_end(np_solver* s, int launches = 1)
{
    if (!s->prof) return;
    (void)hipEventRecord(s->ev[s->ev_used + 1], s->stream);
    s->ev_cls[s->ev_used / 2] = s->cur_cls;
    s->ev_n[s->ev_used / 2] = launches;
    s->ev_used += 2;
}

void prof_release(np_solver* s)
{
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    s->ev.clear();
    s->ev_cls.clear();
    s->ev_n.clear();
    s->ev_used = 0;
    s->prof = false;
}

// Pointers, grids and spacings of the multigrid levels L >= 1 of nested level
// l (entry 0 describes multigrid level 0 for grid and spacing only).
template <typename T>
struct MGView {
    int nmg;
    T* u[NP_MAX_MG];
    T* f[NP_MAX_MG];
    SGrid g[NP_MAX_MG];
    double h[NP_MAX_MG];
};

template <typename T>
MGView<T> mg_view(const np_solver* s, int l, T* const* mu, T* const* mf)
{
    MGView<T> v;
    v.nmg = s->plan.nmg[l];
    double dx = level_dx(&s->cfg, l);
    for (int L = 0; L < v.nmg; L++) {
        v.u[L] = L == 0 ? nullptr : mu[L];
        v.f[L] = L == 0 ? nullptr : mf[L];
        v.g[L] = L == 0 ? s->lg[l] : mg_grid(s, l, L);
        v.h[L] = std::ldexp(dx, L);
    }
    return v;
}

// One red-black sweep on multigrid level L >= 1.  The ghost layer is the
// level's rule (Sec. 2.4), evaluated by the kernels where they read it; that is
// the same as refreshing it before each half sweep.
template <typename T>
void coarse_sweep(const np_solver* s, int l, const MGView<T>& v, int L, hipStream_t st, int first_colour = 0)
{
    const int d = s->cfg.dim;
    const Rule3 rule = rule_of(s, l, L);
    for (int colour = first_colour; colour < 2; colour++)
        launch_half_sweep<T>(d, st, v.g[L], v.u[L], v.f[L], colour, v.h[L] * v.h[L], 0, rule);
}

// First multigrid level of the coarse tail of nested level l (the levels from
// there to the coarsest level fit in LDS together, elements of esz bytes),
// or 0 if none does.
int tail_level(const np_solver* s, int l, size_t esz)
{
    const int nmg = s->plan.nmg[l];
    for (int L = 1; L < nmg; L++) {
        const int nlev = nmg - L;
        if (nlev <= kTailMaxLevels &&
            coarse_tail_lds_bytes(s->cfg.dim, &s->plan.N[l][L], nlev, esz) <= kTailLdsBytes)
            return L;
    }
    return 0;
}

// Everything a V-cycle does on levels L >= 1 (Sec. 2.3 steps 6-13 below the
// finest multigrid level): from the pre-smoothing of level 1 down to the
// coarsest level and back up to the post-smoothing of level 1, which precedes
// the prolongation into level 0; the levels from the tail level down run as one
// kernel.  The sequence is the same in every cycle of a nested level, so it is
// captured once into a HIP graph.
template <typename T>
void coarse_part(const np_solver* s, int l, const MGView<T>& v, hipStream_t st)
{
    const np_config& c = s->cfg;
    const int d = c.dim;
    const int Lt = tail_level(s, l, sizeof(T));
    const int npost = c.coarse_post >= 0 ? c.coarse_post : c.n_post;  // post-smoothing below level 0
    auto tail = [&](int L0) {
        const int nlev = s->plan.nmg[l] - L0;
        double h[kTailMaxLevels];
        Rule3 rules[kTailMaxLevels];
        for (int a = 0; a < nlev; a++) {
            rules[a] = rule_of(s, l, L0 + a);
            h[a] = v.h[L0 + a];
        }
        launch_coarse_tail<T>(d, st, nlev, &s->plan.N[l][L0], h, rules, c.n_pre, npost, v.g[L0], v.f[L0],
                              v.u[L0]);
    };
    if (Lt == 1) {
        tail(1);
        return;
    }
    // the restriction into a level that the tail does not take has already done
    // that level's first red half sweep (seeded correction)
    for (int it = 0; it < c.n_pre; it++) coarse_sweep(s, l, v, 1, st, it == 0 ? 1 : 0);
    int L = 1;
    while (L + 1 < s->plan.nmg[l]) {
        const bool seed = c.n_pre > 0 && L + 1 != Lt;
        launch_resid_restrict<T, T>(d, st, v.g[L], v.u[L], v.f[L], 1.0 / (v.h[L] * v.h[L]), 1.0, v.g[L + 1], v.f[L + 1],
                                    v.u[L + 1], 1, rule_of(s, l, L), seed ? v.h[L + 1] * v.h[L + 1] : 0.0);
        if (L + 1 == Lt) {
            tail(Lt);
            L = Lt;
            break;
        }
        for (int it = 0; it < c.n_pre; it++) coarse_sweep(s, l, v, L + 1, st, it == 0 ? 1 : 0);
        L++;
    }
    while (L > 1) {
        launch_prolong_add<T, T>(d, st, v.g[L], v.u[L], v.g[L - 1], v.u[L - 1], 0, rule_of(s, l, L));
        for (int it = 0; it < npost; it++) coarse_sweep(s, l, v, L - 1, st);
        L--;
    }
}

template <typename T>
int run_coarse(np_solver* s, int l, const MGView<T>& v, hipGraphExec_t* exec)
{
    if (!s->cap_stream) {
        coarse_part(s, l, v, s->stream);
        HIPCHK(s, hipGetLastError());
        return NP_OK;
    }
    if (!exec[l]) {
        HIPCHK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        coarse_part(s, l, v, s->cap_stream);
        hipGraph_t graph = nullptr;
        HIPCHK(s, hipStreamEndCapture(s->cap_stream, &graph));
        hipError_t e = hipGraphInstantiate(&exec[l], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            exec[l] = nullptr;
            return set_err(s, NP_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
    }
    HIPCHK(s, hipGraphLaunch(exec[l], s->stream));
    return NP_OK;
}

// One V-cycle (Sec. 2.3 steps 2-13) on nested level l.  Multigrid level 0 is
// (u0, f0) of type T0 with half-sweep factor h2_0 and residual factor
// inv_h2_0; the restricted right-hand side is multiplied by out_scale_0; the
// coarse levels are of type TC.
// With red_done the first red half sweep has already been done (by the
// defect-correction outer pass) and the cycle starts with black.
template <typename T0, typename TC>
int vcycle_t(np_solver* s, int l, T0* u0, const T0* f0, double h2_0, double inv_h2_0, double out_scale_0,
             const MGView<TC>& v, hipGraphExec_t* exec, bool red_done = false, bool red_unstored = false)
{
    const np_config& c = s->cfg;
    const int d = c.dim;
    hipStream_t st = s->stream;
    // the half sweeps of one smoothing step run back to back: one profiling
    // interval over all of them (launch count recorded), so the per-launch
    // average carries no event overhead between the sweeps
    // (the seeded black half sweep, whose bytes differ, has an interval and a
    // class of its own)
    int nsweep = 0;
    // NP_SWEEP_FUSED with 2-byte storage: the last pre-smoothing black half sweep
    // runs inside the restriction (launch_black_restrict); fused_seed: it is
    // the step's seeded first half sweep
    bool fuse = false, fused_seed = false;
    if constexpr (std::is_same<T0, __half>::value && std::is_same<TC, float>::value)
        fuse = d == 3 && c.n_pre > 0 && c.sweep == NP_SWEEP_FUSED && black_restrict_fits(v.g[0], v.g[1]);
    auto sweep0 = [&](bool fuse_black) {
        for (int colour = red_done ? 1 : 0; colour < 2; colour++) {
            if (colour == 1 && fuse_black) {
                fused_seed = red_done && red_unstored;
                red_done = false;
                break;
            }
            bool seeded = false;
            if constexpr (sizeof(T0) <= 4) {
                if (red_done && red_unstored) {
                    // with one pre-smoothing sweep the restriction reads the red values next
                    prof_begin(s, NP_KCLASS_SEEDED);
                    launch_half_sweep_seeded<T0>(st, v.g[0], u0, f0, h2_0, c.n_pre == 1);
                    prof_end(s);
                    seeded = true;
                }
            }
            if (!seeded) {
                if (nsweep == 0) prof_begin(s, NP_KCLASS_SMOOTH);
                launch_half_sweep<T0>(d, st, v.g[0], u0, f0, colour, h2_0, 1, Rule3{});
                nsweep++;
            }
            red_done = false;
        }
    };
    auto smooth0 = [&](int sweeps, bool fuse_last) {
        if (sweeps <= 0) return;
        nsweep = 0;
        for (int it = 0; it < sweeps; it++) sweep0(fuse_last && it == sweeps - 1);
        if (nsweep) prof_end(s, nsweep);
    };
    smooth0(c.n_pre, fuse);
    // the restriction does multigrid level 1's first red half sweep unless the
    // coarse tail starts at level 1 (coarse_part then skips it)
    const bool seed1 = c.n_pre > 0 && tail_level(s, l, sizeof(TC)) != 1;
    if constexpr (std::is_same<T0, __half>::value && std::is_same<TC, float>::value) {
        if (fuse) {
            prof_begin(s, NP_KCLASS_BLACK_RESTRICT);
            launch_black_restrict(st, v.g[0], u0, f0, h2_0, inv_h2_0, out_scale_0, v.g[1], v.f[1], v.u[1],
                                  seed1 ? v.h[1] * v.h[1] : 0.0, fused_seed);
            prof_end(s);
        }
    }
    if (!fuse) {
        prof_begin(s, NP_KCLASS_RESTRICT);
        launch_resid_restrict<T0, TC>(d, st, v.g[0], u0, f0, inv_h2_0, out_scale_0, v.g[1], v.f[1], v.u[1], 0,
                                      Rule3{}, seed1 ? v.h[1] * v.h[1] : 0.0);
        prof_end(s);
    }
    prof_begin(s, NP_KCLASS_COARSE);
    int rc = run_coarse(s, l, v, exec);
    prof_end(s);
    if (rc) return rc;
    prof_begin(s, NP_KCLASS_PROLONG);
    // on level 0 (fixed ghost layer) the red corrections are dead when a
    // post-smoothing red half sweep follows: it reads only black points
    launch_prolong_add<TC, T0>(d, st, v.g[1], v.u[1], v.g[0], u0, c.n_post > 0, rule_of(s, l, 1));
    prof_end(s);
    smooth0(c.n_post, false);
    return NP_OK;
}

// Plain FP64 V-cycle on the level's potential.
int vcycle(np_solver* s, int l)
{
    MGView<double> v = mg_view<double>(s, l, s->mg_u, s->mg_f);
    double h = v.h[0];
    return vcycle_t<double, double>(s, l, s->phi[l], s->f[l], h * h, 1.0 / (h * h), 1.0, v, s->coarse_exec);
}

// Whether nested level l (solved on its own) runs full sweeps on multigrid level 0.
// A full sweep's thread takes a pair of columns times five rows times a chunk
// of 16 planes and needs registers for one wave per SIMD, so a launch of fewer
// than about four waves per SIMD leaves the chip partly idle: the paper's
// 3 x 128^3 stack took 15.2 ms per solve with full sweeps and 8.6 ms with half
// sweeps, eight 64^3 patches one after another 46.7 and 27.3 ms, a 512 x 512 x
// 64 slab (1080 waves) 150 us per full sweep against two half sweeps of 48 us;
// 2 x 256^3 (952 waves) alike, 512^3 (7128 waves) faster with full sweeps.
constexpr long kFullSweepMinWaves = 4096;

bool full_sweeps(const np_solver* s, int l)
{
    const np_config& c = s->cfg;
    const SGrid& g = s->lg[l];
    const bool big = full_sweep_waves(g) >= kFullSweepMinWaves;
    return c.dim == 3 && c.precision == NP_PREC_FP64 && c.sweep != NP_SWEEP_HALF &&
           (big || c.sweep == NP_SWEEP_FULL_ALL) && s->phi_alt && c.n_pre >= 1 && c.n_post >= 1 &&
           !(l > 0 && c.buffer == NP_BUFFER_INTERP);
}

// One full sweep of level l's multigrid level 0 from the potential into the
// spare buffer, which then becomes the potential (mode: kSweepRes* bits).
void full_sweep(np_solver* s, int l, int mode)
{
    const double h = level_dx(&s->cfg, l);
    launch_full_sweep<double>(s->stream, s->lg[l], s->phi[l], s->phi_alt, s->f[l], h * h, 1.0 / (h * h), mode,
                              s->fs_rev, s->d_bits);
    s->fs_rev ^= 1;
    std::swap(s->phi[l], s->phi_alt);
    std::swap(s->phi_cap[l], s->alt_cap);
}

// Plain FP64 V-cycle (Sec. 2.3 steps 2-13) with full sweeps on multigrid level
// 0.  The last post-smoothing sweep takes the residual norm of its black points
// into slot 0 (zeroed here); full_sweep_norm_sync completes it.  With
// first_done the first pre-smoothing sweep has already run (by
// full_sweep_norm_sync, its result in the spare buffer).
int vcycle_full(np_solver* s, int l, bool first_done)
{
    const np_config& c = s->cfg;
    const int d = c.dim;
    hipStream_t st = s->stream;
    MGView<double> v = mg_view<double>(s, l, s->mg_u, s->mg_f);
    const double h = v.h[0];
    int it = 0;
    if (first_done) {
        std::swap(s->phi[l], s->phi_alt);
        std::swap(s->phi_cap[l], s->alt_cap);
        it = 1;
    }
    if (it < c.n_pre) {
        prof_begin(s, NP_KCLASS_FULL);
        const int n = c.n_pre - it;
        for (; it < c.n_pre; it++) full_sweep(s, l, 0);
        prof_end(s, n);
    }
    const bool seed1 = tail_level(s, l, sizeof(double)) != 1;
    prof_begin(s, NP_KCLASS_RESTRICT);
    launch_resid_restrict<double, double>(d, st, v.g[0], s->phi[l], s->f[l], 1.0 / (h * h), 1.0, v.g[1], v.f[1],
                                          v.u[1], 0, Rule3{}, seed1 ? v.h[1] * v.h[1] : 0.0);
    prof_end(s);
    prof_begin(s, NP_KCLASS_COARSE);
    int rc = run_coarse(s, l, v, s->coarse_exec);
    prof_end(s);
    if (rc) return rc;
    // the post-smoothing sweeps read only the black values: the prolongation
    // corrects the black points
    prof_begin(s, NP_KCLASS_PROLONG);
    launch_prolong_add<double, double>(d, st, v.g[1], v.u[1], v.g[0], s->phi[l], 1, rule_of(s, l, 1));
    prof_end(s);
    launch_set_u64(st, s->d_bits, 1, 0ULL);
    prof_begin(s, NP_KCLASS_FULL);
    for (it = 0; it < c.n_post; it++) full_sweep(s, l, it == c.n_post - 1 ? kSweepResOut : 0);
    prof_end(s, c.n_post);
    return NP_OK;
}

// Completes the residual norm of the potential after vcycle_full: the next
// cycle's first pre-smoothing sweep, into the spare buffer (the potential is
// not replaced), also takes the norm over the red points (host-synchronous).
int full_sweep_norm_sync(np_solver* s, int l, double* out)
{
    const double h = level_dx(&s->cfg, l);
    prof_begin(s, NP_KCLASS_FULL_RES);
    launch_full_sweep<double>(s->stream, s->lg[l], s->phi[l], s->phi_alt, s->f[l], h * h, 1.0 / (h * h), kSweepResIn,
                              s->fs_rev, s->d_bits);
    prof_end(s);
    s->fs_rev ^= 1;
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(s->h_bits, s->d_bits, sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *out = bits_to_double(s->h_bits[0]);
    return NP_OK;
}

// Inner V-cycle of the defect correction, on the scaled level-0 problem
// L e'' = r'' (L = h^2 lap, the integer stencil, r'' = r / ||r||) in low
// precision TL, with FP32 coarse levels: the coarse right-hand side is
// R(r'' - L e'') / h^2, in the same units as e''.
// Whether the outer pass leaves the next correction's start unstored: its
// first black half sweep then forms the red values (the red half sweep from
// zero) from the defect, and stores them when no red half sweep follows that
// black one (n_pre = 1).  Needs the paired level-0 sweep.
bool dc_seed_black(const np_solver* s, int l)
{
    const np_config& c = s->cfg;
    return c.precision != NP_PREC_FP64 && c.dim == 3 && c.n_pre >= 1 && (s->lg[l].hx % 2) == 0;
}

template <typename TL>
int vcycle_lo(np_solver* s, int l, bool red_done)
{
    MGView<float> v = mg_view<float>(s, l, s->mg_u32, s->mg_f32);
    double h = v.h[0];
    return vcycle_t<TL, float>(s, l, (TL*)s->e_lo, (const TL*)s->r_lo, 1.0, 1.0, 1.0 / (h * h), v, s->coarse_exec32,
                               red_done, red_done && dc_seed_black(s, l));
}

// Queue a norm into slot `slot` and return it (host-synchronous).
int norm_sync(np_solver* s, int l, int mode, double* out)
{
    double dx = level_dx(&s->cfg, l);
    launch_set_u64(s->stream, s->d_bits, 1, 0ULL);
    prof_begin(s, NP_KCLASS_NORM);
    launch_norm(s->cfg.dim, s->stream, s->lg[l], s->phi[l], s->f[l], 1.0 / (dx * dx), mode, s->d_bits);
    prof_end(s);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(s->h_bits, s->d_bits, sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *out = bits_to_double(s->h_bits[0]);
    return NP_OK;
}

int force_delta_sync(np_solver* s, int l, double* out)
{
    double dx = level_dx(&s->cfg, l);
    launch_set_u64(s->stream, s->d_bits + 1, 1, 0ULL);
    prof_begin(s, NP_KCLASS_NORM);
    launch_force_delta(s->cfg.dim, s->stream, s->lg[l], dx, s->phi[l], s->force_scratch, s->d_bits + 1);
    prof_end(s);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(s->h_bits + 1, s->d_bits + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *out = bits_to_double(s->h_bits[1]);
    return NP_OK;
}

// Outer pass of the defect correction on level l (host-synchronous): with
// update, phi += factor * e'' into the other potential buffer and the buffers
// rotate; then r'' = (f - lap phi) * rscale into the low-precision defect and
// the next correction's start (its first red half sweep when n_pre > 0).
// Returns ||f - lap phi||_inf of the (updated) potential.
int dc_outer_sync(np_solver* s, int l, bool update, double factor, double rscale, double* out)
{
    const np_config& c = s->cfg;
    double dx = level_dx(&c, l);
    int first_red = c.n_pre > 0;
    void* e_in = update ? s->e_lo : nullptr;
    void* e_out = dc_seed_black(s, l) ? nullptr : (update ? s->e_nx : s->e_lo);
    double* p_out = update ? s->phi_alt : nullptr;
    launch_set_u64(s->stream, s->d_bits, 1, 0ULL);
    prof_begin(s, NP_KCLASS_DC);
    if (c.precision == NP_PREC_FP16S_DC)
        launch_dc_outer<__half>(c.dim, s->stream, s->lg[l], s->phi[l], (const __half*)e_in, factor, p_out, s->f[l],
                                1.0 / (dx * dx), rscale, (__half*)s->r_lo, (__half*)e_out, first_red, s->d_bits);
    else
        launch_dc_outer<float>(c.dim, s->stream, s->lg[l], s->phi[l], (const float*)e_in, factor, p_out, s->f[l],
                               1.0 / (dx * dx), rscale, (float*)s->r_lo, (float*)e_out, first_red, s->d_bits);
    prof_end(s);
    HIPCHK(s, hipGetLastError());
    if (update) {
        std::swap(s->e_lo, s->e_nx);
        std::swap(s->phi[l], s->phi_alt);
        std::swap(s->phi_cap[l], s->alt_cap);
    }
    HIPCHK(s, hipMemcpyAsync(s->h_bits, s->d_bits, sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *out = bits_to_double(s->h_bits[0]);
    return NP_OK;
}

// The level's starting residual for the defect correction: one pass of the
// outer kernel without update that keeps f - lap phi in FP32 (r32) and returns
// its max norm, so that the first scaled defect needs no second pass over phi
// and f (dc_scale_defect).
int dc_first_residual(np_solver* s, int l, double* out)
{
    const np_config& c = s->cfg;
    double dx = level_dx(&c, l);
    if (!same_grid(s->lg[l], s->r32_grid)) {
        HIPCHK(s, hipMemsetAsync(s->r32, 0, 2 * s->lg[l].cs * sizeof(float), s->stream));
        s->r32_grid = s->lg[l];
    }
    launch_set_u64(s->stream, s->d_bits, 1, 0ULL);
    prof_begin(s, NP_KCLASS_NORM);
    launch_dc_outer<float>(c.dim, s->stream, s->lg[l], s->phi[l], nullptr, 0.0, nullptr, s->f[l], 1.0 / (dx * dx), 1.0,
                           s->r32, nullptr, 0, s->d_bits);
    prof_end(s);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(s->h_bits, s->d_bits, sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *out = bits_to_double(s->h_bits[0]);
    return NP_OK;
}

// The first defect of a level from r32: r'' = r32 * rscale and the next
// correction's start, as the outer pass without update writes them.
int dc_scale_defect(np_solver* s, int l, double rscale)
{
    const np_config& c = s->cfg;
    void* e_out = dc_seed_black(s, l) ? nullptr : s->e_lo;
    prof_begin(s, NP_KCLASS_DC_SCALE);
    if (c.precision == NP_PREC_FP16S_DC)
        launch_dc_scale<__half>(c.dim, s->stream, s->lg[l], s->r32, rscale, (__half*)s->r_lo, (__half*)e_out,
                                c.n_pre > 0);
    else
        launch_dc_scale<float>(c.dim, s->stream, s->lg[l], s->r32, rscale, (float*)s->r_lo, (float*)e_out,
                               c.n_pre > 0);
    prof_end(s);
    HIPCHK(s, hipGetLastError());
    return NP_OK;
}

// Inner cycles of one defect-correction step (extension of Sec. 2.3 with FP32
// or FP16-stored inner cycles): k low-precision V-cycles on the scaled defect
// r'' = r / r_scale, the first one starting from the state the outer pass left
// (e'' = 0, red points relaxed when n_pre > 0).
int dc_inner(np_solver* s, int l, int k)
{
    const np_config& c = s->cfg;
    for (int it = 0; it < k; it++) {
        const bool red_done = it == 0 && c.n_pre > 0;
        int rc = c.precision == NP_PREC_FP16S_DC ? vcycle_lo<__half>(s, l, red_done) : vcycle_lo<float>(s, l, red_done);
        if (rc) return rc;
    }
    return NP_OK;
}

// Inner V-cycles of the next defect-correction step: inner_cycles, or with
// NP_INNER_ADAPTIVE the number that the contraction per cycle rho measured on
// the previous step says brings the residual r down to the target, between 1
// and a maximum (an outer pass costs about as much as a V-cycle, so the
// estimate is rounded down unless it is a quarter cycle past an integer).  The
// maximum is 4 with FP32 storage and 3 with FP16 storage, whose rounding (2^-11
// relative) starts to limit what one step gains after about three cycles of
// contraction ~0.3.  Never runs past `limit` (a pinned count or the cap).
constexpr double kAdaptiveRho0 = 0.3;

int dc_cycles(const np_config& c, double r, double target, double rho, int q, int limit)
{
    int k = c.inner_cycles;
    if (k == NP_INNER_ADAPTIVE) {
        const int kmax = c.precision == NP_PREC_FP16S_DC ? 3 : 4;
        double need = kmax;
        if (r > target && target > 0.0) need = std::log(target / r) / std::log(rho);
        k = (int)std::ceil(need - 0.25);
        k = k < 1 ? 1 : (k > kmax ? kmax : k);
    }
    if (q + k > limit) k = limit - q > 1 ? limit - q : 1;
    return k;
}

// End of a level's defect correction: the level's potential must live in a
// buffer of the level's own capacity unless every buffer is as large as the
// spare one; otherwise copy it back into the level's own buffer.
int dc_settle(np_solver* s, int l)
{
    if (s->alt_cap >= s->phi_cap[l]) return NP_OK;
    size_t bytes = 2 * s->lg[l].cs * sizeof(double);
    HIPCHK(s, hipMemcpyAsync(s->phi_alt, s->phi[l], bytes, hipMemcpyDeviceToDevice, s->stream));
    std::swap(s->phi[l], s->phi_alt);
    std::swap(s->phi_cap[l], s->alt_cap);
    return NP_OK;
}

// Max norm of the residual of level l's potential restricted twice (its mean
// over boxes of 4^3 points; host-synchronous, slot 3).
int box_resid_sync(np_solver* s, int l, double* out)
{
    const double dx = level_dx(&s->cfg, l);
    launch_set_u64(s->stream, s->d_bits + 3, 1, 0ULL);
    launch_box_resid_norm3(s->stream, s->lg[l], s->phi[l], s->f[l], 1.0 / (dx * dx), s->d_bits + 3);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(s->h_bits + 3, s->d_bits + 3, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    *out = bits_to_double(s->h_bits[3]);
    return NP_OK;
}

// Learned initial guess of level l >= 1 (3-D): the network's prediction from
// the interpolated guess, kept only where it is expected to save a V-cycle.
// The cycle count is set by the error the smoother does not remove, whose
// residual survives restriction: the guess is kept if it lowers the residual
// restricted twice (mean over 4^3 boxes) by at least the contraction of one
// V-cycle, `rho` (measured on the parent level), and its point-wise residual
// is finite; otherwise the interpolated guess is restored.  *r is the max-norm
// residual of the guess in effect on return.
int learned_guess(np_solver* s, int l, const double* rho_l, double fourpiG, double fnorm, double rho, double* r,
                  int* used, int* ran)
{
    *used = 0;
    *ran = 0;
    if (!s->have_weights || !(fnorm > 0.0) || !std::isfinite(*r)) return NP_OK;
    *ran = 1;
    const np_config& c = s->cfg;
    hipStream_t st = s->stream;
    SGrid g = s->lg[l];
    const int X = g.nx - 2, Y = g.ny - 2, Z = g.nz - 2;
    const double dx = level_dx(&c, l);
    double rb_interp = 0.0;
    int rc = box_resid_sync(s, l, &rb_interp);
    if (rc) return rc;
    prof_begin(s, NP_KCLASS_GUESS);
    net_features_bf16(st, g, s->phi[l], s->f[l], 1.0 / fnorm, 1.0 / (dx * dx), s->net_x);
    net_conv_mfma(st, s->net_x, 2, s->net_w[0], s->net_b[0], 16, 1, 1, Z, Y, X, s->net_a1);
    net_conv_mfma(st, s->net_a1, 16, s->net_w[1], s->net_b[1], 16, 1, 1, Z, Y, X, s->net_a2);
    net_conv_mfma(st, s->net_a2, 16, s->net_w[2], s->net_b[2], 1, 0, 1, Z, Y, X, s->net_out);
    net_apply(st, g, s->phi[l], s->net_out, fnorm * dx * dx);
    prof_end(s);
    HIPCHK(s, hipGetLastError());
    double rl = 0.0, rb = 0.0;
    rc = norm_sync(s, l, 0, &rl);
    if (rc) return rc;
    rc = box_resid_sync(s, l, &rb);
    if (rc) return rc;
    s->guess_box_ratio[l] = rb_interp > 0.0 ? rb / rb_interp : 0.0;
    if (std::isfinite(rl) && std::isfinite(rb) && rb <= rho * rb_interp) {
        *r = rl;
        *used = 1;
        return NP_OK;
    }
    // fallback: restore the interpolated guess
    launch_interface_fill(c.dim, st, s->lg[c.parent[l]], s->phi[c.parent[l]], s->f[c.parent[l]], g, c.offset[l][0],
                          c.offset[l][1], c.offset[l][2], rho_l, fourpiG, s->phi[l], s->f[l], nullptr);
    HIPCHK(s, hipGetLastError());
    return NP_OK;
}

// NP_BUFFER_INTERP on a level l >= 1: for the duration of the level's solve
// the level's grid and arrays are those of the relaxed domain (Omega^l, whose
// ghost layer is the interpolated inner buffer layer), so the V-cycle and norm
// code runs unchanged on it; the level's own storage comes back on scope exit.
struct RelaxedDomain {
    np_solver* s;
    int l;
    bool on;
    SGrid g{};
    double* phi = nullptr;
    double* f = nullptr;
    RelaxedDomain(np_solver* s_, int l_, bool on_) : s(s_), l(l_), on(on_)
    {
        if (!on) return;
        g = s->lg[l];
        phi = s->phi[l];
        f = s->f[l];
        s->lg[l] = s->ag[l];
        s->phi[l] = s->ab_phi;
        s->f[l] = s->ab_f;
    }
    ~RelaxedDomain()
    {
        if (!on) return;
        s->lg[l] = g;
        s->phi[l] = phi;
        s->f[l] = f;
    }
    RelaxedDomain(const RelaxedDomain&) = delete;
    RelaxedDomain& operator=(const RelaxedDomain&) = delete;
};

// A batch of patches (one depth, one set of extents; FP64, interpolated
// guess, residual stop rule): each member is filled from its parent, then the
// V-cycles and the stop-test norms run as one launch per operator over the
// members still iterating (device flags d_act), each member stopping at its
// own count, with the arithmetic of a single-patch solve.
int solve_batch(np_solver* s, const PatchGroup& G, const double* const* rho, double fourpiG, np_stats& st,
                int& status)
{
    const np_config& c = s->cfg;
    const int d = c.dim;
    const int n = G.n, m0 = G.member[0];
    hipStream_t stm = s->stream;
    auto t0 = std::chrono::steady_clock::now();
    unsigned long long* slots = s->d_bits + kBatchSlot;
    // the members' fills (each from its own parent), max |f| of member b into slot b
    prof_begin(s, NP_KCLASS_FILL);
    launch_set_u64(stm, slots, n, 0ULL);
    for (int b = 0; b < n; b++) {
        const int l = G.member[b];
        s->hist[l].clear();
        launch_interface_fill(d, stm, s->lg[c.parent[l]], s->phi[c.parent[l]], s->f[c.parent[l]], s->lg[l],
                              c.offset[l][0], c.offset[l][1], d == 3 ? c.offset[l][2] : 0, rho[l], fourpiG, s->phi[l],
                              s->f[l], slots + b);
    }
    prof_end(s, n);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(s->h_bits + kBatchSlot, slots, n * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             stm));
    HIPCHK(s, hipStreamSynchronize(stm));
    double scale[NP_MAX_LEVELS], r[NP_MAX_LEVELS], r0[NP_MAX_LEVELS];
    int q[NP_MAX_LEVELS] = {}, lvl[NP_MAX_LEVELS] = {};
    for (int b = 0; b < n; b++) {
        scale[b] = bits_to_double(s->h_bits[kBatchSlot + b]);
        if (!std::isfinite(scale[b])) return set_err(s, NP_ENONFINITE, "level %d: non-finite density", G.member[b]);
    }
    for (int b = 0; b < n; b++) {
        if (scale[b] > 0.0) continue;
        // zero density: the residual of the zero potential sets the scale
        int rc = norm_sync(s, G.member[b], 2, &scale[b]);
        if (rc) return rc;
        if (!std::isfinite(scale[b]))
            return set_err(s, NP_ENONFINITE, "level %d: non-finite boundary data", G.member[b]);
    }
    // the batch's grids: level 0 and the multigrid levels, one row per member
    const double dx = level_dx(&c, m0);
    MGView<double> v = mg_view<double>(s, m0, s->mg_u, s->mg_f);
    for (int L = 0; L < v.nmg; L++) v.g[L] = batched(v.g[L], n, s->d_act);
    const SGrid g0 = v.g[0];
    // stop-test norms of the members still iterating into their slots
    auto norms = [&](bool first) -> int {
        launch_set_u64(stm, slots, n, 0ULL);
        prof_begin(s, NP_KCLASS_NORM);
        launch_norm(d, stm, g0, s->phi[m0], s->f[m0], 1.0 / (dx * dx), 0, slots);
        prof_end(s);
        HIPCHK(s, hipGetLastError());
        HIPCHK(s, hipMemcpyAsync(s->h_bits + kBatchSlot, slots, n * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                 stm));
        HIPCHK(s, hipStreamSynchronize(stm));
        for (int b = 0; b < n; b++)
            if (first || s->h_act[b]) r[b] = bits_to_double(s->h_bits[kBatchSlot + b]);
        return NP_OK;
    };
    // which members go on: the rule of a single-patch solve, member by member
    auto update = [&]() -> bool {
        bool any = false;
        for (int b = 0; b < n; b++) {
            if (!s->h_act[b]) continue;
            const int l = G.member[b];
            const bool pinned = s->has_fixed && s->fixed[l] >= 0;
            bool go = true;
            if (!std::isfinite(r[b])) {
                lvl[b] = NP_ENONFINITE;
                go = false;
            } else if (q[b] > 0 && r0[b] > 0 && r[b] > 1e3 * r0[b]) {
                lvl[b] = NP_EDIVERGED;
                go = false;
            } else if (pinned ? q[b] >= s->fixed[l] : r[b] <= c.tol * scale[b]) {
                go = false;
            } else if (q[b] >= c.max_cycles) {
                lvl[b] = NP_ENOTCONV;
                go = false;
            }
            s->h_act[b] = go ? 1 : 0;
            any = any || go;
        }
        return any;
    };
    for (int b = 0; b < n; b++) s->h_act[b] = 1;
    HIPCHK(s, hipMemcpyAsync(s->d_act, s->h_act, n * sizeof(int), hipMemcpyHostToDevice, stm));
    int rc = norms(true);
    if (rc) return rc;
    for (int b = 0; b < n; b++) {
        r0[b] = r[b];
        s->hist[G.member[b]].push_back(scale[b] > 0 ? r[b] / scale[b] : r[b]);
        st.interp_rel_residual[G.member[b]] = scale[b] > 0 ? r[b] / scale[b] : r[b];
    }
    bool any = update();
    while (any) {
        HIPCHK(s, hipMemcpyAsync(s->d_act, s->h_act, n * sizeof(int), hipMemcpyHostToDevice, stm));
        rc = vcycle_t<double, double>(s, m0, s->phi[m0], s->f[m0], dx * dx, 1.0 / (dx * dx), 1.0, v,
                                      s->coarse_exec);
        if (rc) return rc;
        HIPCHK(s, hipGetLastError());
        for (int b = 0; b < n; b++) q[b] += s->h_act[b];
        rc = norms(false);
        if (rc) return rc;
        for (int b = 0; b < n; b++)
            if (s->h_act[b]) s->hist[G.member[b]].push_back(scale[b] > 0 ? r[b] / scale[b] : r[b]);
        any = update();
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int b = 0; b < n; b++) {
        const int l = G.member[b];
        st.cycles[l] = q[b];
        st.outer_steps[l] = 0;
        st.scale[l] = scale[b];
        st.initial_rel_residual[l] = s->hist[l].front();
        st.final_rel_residual[l] = scale[b] > 0 ? r[b] / scale[b] : r[b];
        st.level_ms[l] = ms;
        if (q[b] > 0 && r0[b] > 0.0 && r[b] > 0.0 && r[b] < r0[b]) {
            const double m = std::pow(r[b] / r0[b], 1.0 / q[b]);
            s->rho_meas[l] = m < 0.02 ? 0.02 : (m > 0.95 ? 0.95 : m);
        } else {
            s->rho_meas[l] = 0.0;
        }
    }
    for (int b = 0; b < n; b++) {
        const int l = G.member[b];
        if (lvl[b] == NP_ENONFINITE || lvl[b] == NP_EDIVERGED)
            return set_err(s, lvl[b], "level %d: %s after %d cycles", l,
                           lvl[b] == NP_ENONFINITE ? "non-finite residual" : "residual diverged", q[b]);
        if (lvl[b] == NP_ENOTCONV && status == NP_OK) {
            status = NP_ENOTCONV;
            set_err(s, NP_ENOTCONV, "level %d: not converged in %d cycles (rel. residual %.3e)", l, q[b],
                    st.final_rel_residual[l]);
        }
    }
    return NP_OK;
}

void free_all(np_solver* s)
{
    for (int l = 0; l < NP_MAX_LEVELS; l++) {
        if (s->coarse_exec[l]) (void)hipGraphExecDestroy(s->coarse_exec[l]);
        s->coarse_exec[l] = nullptr;
    }
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    s->cap_stream = nullptr;
    for (int l = 0; l < NP_MAX_LEVELS; l++) {
        if (s->owns[l]) {
            if (s->phi[l]) (void)hipFree(s->phi[l]);
            if (s->f[l]) (void)hipFree(s->f[l]);
        }
        s->owns[l] = false;
        s->phi[l] = s->f[l] = nullptr;
    }
    if (s->d_act) (void)hipFree(s->d_act);
    if (s->h_act) (void)hipHostFree(s->h_act);
    s->d_act = nullptr;
    s->h_act = nullptr;
    for (int L = 0; L < NP_MAX_MG; L++) {
        if (s->mg_u[L]) (void)hipFree(s->mg_u[L]);
        if (s->mg_f[L]) (void)hipFree(s->mg_f[L]);
        if (s->mg_u32[L]) (void)hipFree(s->mg_u32[L]);
        if (s->mg_f32[L]) (void)hipFree(s->mg_f32[L]);
        s->mg_u[L] = s->mg_f[L] = nullptr;
        s->mg_u32[L] = s->mg_f32[L] = nullptr;
    }
    for (int l = 0; l < NP_MAX_LEVELS; l++) {
        if (s->coarse_exec32[l]) (void)hipGraphExecDestroy(s->coarse_exec32[l]);
        s->coarse_exec32[l] = nullptr;
    }
    if (s->e_lo) (void)hipFree(s->e_lo);
    if (s->e_nx) (void)hipFree(s->e_nx);
    if (s->r_lo) (void)hipFree(s->r_lo);
    if (s->r32) (void)hipFree(s->r32);
    s->r32 = nullptr;
    if (s->phi_alt) (void)hipFree(s->phi_alt);
    s->e_lo = s->e_nx = s->r_lo = nullptr;
    s->phi_alt = nullptr;
    for (int k = 0; k < 3; k++) {
        if (s->net_w[k]) (void)hipFree(s->net_w[k]);
        if (s->net_b[k]) (void)hipFree(s->net_b[k]);
        s->net_w[k] = nullptr;
        s->net_b[k] = nullptr;
    }
    void* net[] = {s->net_x, s->net_a1, s->net_a2, s->net_out, s->feat_phi, s->feat_f};
    for (void* p : net)
        if (p) (void)hipFree(p);
    s->net_x = s->net_a1 = s->net_a2 = nullptr;
    s->net_out = nullptr;
    s->feat_phi = s->feat_f = nullptr;
    if (s->ab_phi) (void)hipFree(s->ab_phi);
    if (s->ab_f) (void)hipFree(s->ab_f);
    s->ab_phi = s->ab_f = nullptr;
    if (s->force_scratch) (void)hipFree(s->force_scratch);
    if (s->d_bits) (void)hipFree(s->d_bits);
    if (s->h_bits) (void)hipHostFree(s->h_bits);
    s->force_scratch = nullptr;
    s->d_bits = nullptr;
    s->h_bits = nullptr;
}

int alloc_dev(np_solver* s, void** p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_err(s, NP_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    return NP_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

void nested_poisson_default_config(np_config* c)
{
    if (!c) return;
    memset(c, 0, sizeof(*c));
    c->G = 1.0;
    c->n_pre = 2;
    c->n_post = 1;
    c->tol = 1e-10;
    c->max_cycles = 50;
    c->stop_rule = NP_STOP_RESIDUAL;
    c->precision = NP_PREC_FP64;
    c->inner_cycles = 1;
    c->guess = NP_GUESS_INTERP;
    c->buffer = NP_BUFFER_RELAXED;
    c->batch = 1;
    c->guess_gate = 1;
    c->coarse_post = -1;
    for (int l = 0; l < NP_MAX_LEVELS; l++) c->parent[l] = l - 1;
}

int nested_poisson_plan(const np_config* cfg, np_plan* out)
{
    if (!out) return NP_EINVAL;
    if (!validate(cfg, g_last_error, sizeof g_last_error)) return NP_EINVAL;
    return make_plan(cfg, out, g_last_error, sizeof g_last_error);
}

int nested_poisson_create(const np_config* cfg, void* hip_stream, np_solver** out)
{
    if (!out) return NP_EINVAL;
    *out = nullptr;
    if (!validate(cfg, g_last_error, sizeof g_last_error)) return NP_EINVAL;
    np_solver* s = new (std::nothrow) np_solver();
    if (!s) return NP_ENOMEM;
    s->cfg = *cfg;
    if (make_plan(cfg, &s->plan, g_last_error, sizeof g_last_error) != NP_OK) {
        delete s;
        return NP_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        snprintf(g_last_error, sizeof g_last_error, "no HIP device");
        delete s;
        return NP_ENODEV;
    }
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return NP_EHIP;
    }
    s->stream = (hipStream_t)hip_stream;
    const int d = cfg->dim;
    int rc = NP_OK;
    size_t max_cells = 0;  // largest Omega^l
    s->ngroups = make_groups(cfg, s->groups);
    for (int l = 0; l < cfg->nlevels; l++) {
        s->lg[l] = level_grid(cfg, l);
        const size_t cells = (size_t)level_n(cfg, l, 0) * level_n(cfg, l, 1) * level_n(cfg, l, 2);
        if (cells > max_cells) max_cells = cells;
    }
    // the level arrays; a batch's members lie 2 cs apart in one allocation
    for (int gi = 0; gi < s->ngroups && rc == NP_OK; gi++) {
        const PatchGroup& G = s->groups[gi];
        const int m0 = G.member[0];
        const size_t bytes = 2 * s->lg[m0].cs * sizeof(double);
        rc = alloc_dev(s, (void**)&s->phi[m0], G.n * bytes);
        if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->f[m0], G.n * bytes);
        s->owns[m0] = true;
        for (int b = 0; b < G.n && rc == NP_OK; b++) {
            const int m = G.member[b];
            s->phi[m] = s->phi[m0] + b * 2 * s->lg[m0].cs;
            s->f[m] = s->f[m0] + b * 2 * s->lg[m0].cs;
            s->phi_cap[m] = bytes;
        }
    }
    // multigrid scratch: per level L the largest grid over the nested levels,
    // FP64 for the plain solve, FP32 for the defect correction's inner cycles
    const bool dc = cfg->precision != NP_PREC_FP64;
    for (int L = 1; L < NP_MAX_MG && rc == NP_OK; L++) {
        size_t best = 0;
        for (int gi = 0; gi < s->ngroups; gi++) {
            const int l = s->groups[gi].member[0];
            if (L < s->plan.nmg[l]) {
                size_t b = 2 * mg_grid(s, l, L).cs * s->groups[gi].n;
                if (b > best) best = b;
            }
        }
        if (!best) break;
        if (dc) {
            rc = alloc_dev(s, (void**)&s->mg_u32[L], best * sizeof(float));
            if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->mg_f32[L], best * sizeof(float));
        } else {
            rc = alloc_dev(s, (void**)&s->mg_u[L], best * sizeof(double));
            if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->mg_f[L], best * sizeof(double));
        }
    }
    if (rc == NP_OK && cfg->buffer == NP_BUFFER_INTERP && cfg->nlevels > 1) {
        size_t best = 0;
        for (int l = 1; l < cfg->nlevels; l++) {
            s->ag[l] = make_grid(d, level_n(cfg, l, 0) + 2, level_n(cfg, l, 1) + 2, level_n(cfg, l, 2) + 2);
            if (2 * s->ag[l].cs > best) best = 2 * s->ag[l].cs;
        }
        rc = alloc_dev(s, (void**)&s->ab_phi, best * sizeof(double));
        if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->ab_f, best * sizeof(double));
    }
    if (rc == NP_OK && dc) {
        size_t best = 0;
        for (int l = 0; l < cfg->nlevels; l++)
            if (2 * s->lg[l].cs > best) best = 2 * s->lg[l].cs;
        size_t esz = cfg->precision == NP_PREC_FP16S_DC ? sizeof(__half) : sizeof(float);
        s->lo_bytes = best * esz;
        rc = alloc_dev(s, &s->e_lo, s->lo_bytes);
        if (rc == NP_OK) rc = alloc_dev(s, &s->e_nx, s->lo_bytes);
        if (rc == NP_OK) rc = alloc_dev(s, &s->r_lo, s->lo_bytes);
        if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->r32, best * sizeof(float));
        s->alt_cap = best * sizeof(double);
        if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->phi_alt, s->alt_cap);
    }
    if (rc == NP_OK && !dc && d == 3 && cfg->sweep != NP_SWEEP_HALF && cfg->n_pre >= 1 && cfg->n_post >= 1) {
        // the second potential buffer of the full sweeps
        size_t best = 0;
        for (int l = 0; l < cfg->nlevels; l++)
            if (2 * s->lg[l].cs > best) best = 2 * s->lg[l].cs;
        s->alt_cap = best * sizeof(double);
        rc = alloc_dev(s, (void**)&s->phi_alt, s->alt_cap);
    }
    if (rc == NP_OK && cfg->guess == NP_GUESS_LEARNED) {
        size_t vox = 0;
        for (int l = 1; l < cfg->nlevels; l++) {
            const size_t m = ((size_t)level_n(cfg, l, 0) + 2) * (level_n(cfg, l, 1) + 2) * (level_n(cfg, l, 2) + 2);
            if (m > vox) vox = m;
        }
        const int cin[3] = {2, 16, 16}, cout[3] = {16, 16, 1};
        for (int k = 0; k < 3 && rc == NP_OK; k++) {
            rc = alloc_dev(s, (void**)&s->net_w[k], 27 * cin[k] * cout[k] * sizeof(uint16_t));
            if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->net_b[k], 16 * sizeof(float));
        }
        if (rc == NP_OK && vox) {
            rc = alloc_dev(s, (void**)&s->net_x, vox * 2 * sizeof(uint16_t));
            if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->net_a1, vox * 16 * sizeof(uint16_t));
            if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->net_a2, vox * 16 * sizeof(uint16_t));
            if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->net_out, vox * sizeof(float));
        }
    }
    if (rc == NP_OK && cfg->stop_rule == NP_STOP_FORCE_DELTA)
        rc = alloc_dev(s, (void**)&s->force_scratch, (size_t)d * max_cells * sizeof(double));
    if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->d_bits, kBitSlots * sizeof(unsigned long long));
    if (rc == NP_OK && hipHostMalloc((void**)&s->h_bits, kBitSlots * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        s->h_bits = nullptr;
        rc = NP_ENOMEM;
    }
    if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->d_act, NP_MAX_LEVELS * sizeof(int));
    if (rc == NP_OK && hipHostMalloc((void**)&s->h_act, NP_MAX_LEVELS * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        s->h_act = nullptr;
        rc = NP_ENOMEM;
    }
    if (rc != NP_OK) {
        snprintf(g_last_error, sizeof g_last_error, "%s", s->err);
        free_all(s);
        delete s;
        return rc;
    }
    for (int l = 0; l < NP_MAX_LEVELS; l++) s->fixed[l] = -1;
    // private stream used only to record the coarse-cycle graphs (nothing runs on it)
    if (hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        s->cap_stream = nullptr;  // launch the coarse part directly instead
    }
    *out = s;
    return NP_OK;
}

int nested_poisson_set_fixed_cycles(np_solver* s, const int* cycles)
{
    if (!s) return NP_EINVAL;
    if (!cycles) {
        s->has_fixed = false;
        for (int l = 0; l < NP_MAX_LEVELS; l++) s->fixed[l] = -1;
        return NP_OK;
    }
    for (int l = 0; l < s->cfg.nlevels; l++) {
        if (cycles[l] > NP_MAX_CYCLES) return set_err(s, NP_EINVAL, "fixed cycle count %d too large", cycles[l]);
        s->fixed[l] = cycles[l];
    }
    s->has_fixed = true;
    return NP_OK;
}

int nested_poisson_solve(np_solver* s, const double* const* rho, const double* phi_outer, np_stats* stats)
{
    if (!s) return NP_EINVAL;
    if (!rho || !phi_outer) return set_err(s, NP_EINVAL, "null input pointer");
    for (int l = 0; l < s->cfg.nlevels; l++)
        if (!rho[l]) return set_err(s, NP_EINVAL, "rho[%d] is null", l);
    HIPCHK(s, hipSetDevice(s->device));
    const np_config& c = s->cfg;
    const int d = c.dim;
    const double fourpiG = 4.0 * M_PI * c.G;
    np_stats st;
    memset(&st, 0, sizeof st);
    s->solved = false;
    int status = NP_OK;
    auto t_all = std::chrono::steady_clock::now();
    for (int gi = 0; gi < s->ngroups; gi++) {
        if (s->groups[gi].n > 1) {
            int rc = solve_batch(s, s->groups[gi], rho, fourpiG, st, status);
            if (rc) {
                if (stats) *stats = st;
                return rc;
            }
            continue;
        }
        const int l = s->groups[gi].member[0];
        auto t0 = std::chrono::steady_clock::now();
        s->hist[l].clear();
        prof_begin(s, NP_KCLASS_FILL);
        // the fill also reduces max |f| into slot 2
        launch_set_u64(s->stream, s->d_bits + 2, 1, 0ULL);
        if (l == 0) {
            launch_level0_init(d, s->stream, s->lg[0], rho[0], phi_outer, fourpiG, s->phi[0], s->f[0], s->d_bits + 2);
        } else {
            launch_interface_fill(d, s->stream, s->lg[c.parent[l]], s->phi[c.parent[l]], s->f[c.parent[l]], s->lg[l],
                                  c.offset[l][0], c.offset[l][1], d == 3 ? c.offset[l][2] : 0, rho[l], fourpiG,
                                  s->phi[l], s->f[l], s->d_bits + 2);
        }
        prof_end(s);
        HIPCHK(s, hipGetLastError());
        HIPCHK(s, hipMemcpyAsync(s->h_bits + 2, s->d_bits + 2, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                 s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        const double fnorm = bits_to_double(s->h_bits[2]);
        int rc = NP_OK;
        if (!std::isfinite(fnorm)) return set_err(s, NP_ENONFINITE, "level %d: non-finite density", l);
        double scale = fnorm;
        // comparison scheme: Omega^l alone is relaxed, with the interpolated inner
        // buffer layer as its Dirichlet data; its |f| sets the stop test's scale
        const bool interp_buffer = l > 0 && c.buffer == NP_BUFFER_INTERP;
        // last padded index of Omega^l in the relaxed domain's array, per axis
        const int box_hi[3] = {level_n(&c, l, 0) + 1, level_n(&c, l, 1) + 1, level_n(&c, l, 2) + 1};
        if (interp_buffer) {
            prof_begin(s, NP_KCLASS_FILL);
            launch_copy_box(d, s->stream, s->lg[l], s->phi[l], s->ag[l], s->ab_phi, 0, box_hi, 1);
            launch_copy_box(d, s->stream, s->lg[l], s->f[l], s->ag[l], s->ab_f, 0, box_hi, 1);
            prof_end(s);
            HIPCHK(s, hipGetLastError());
        }
        RelaxedDomain dom(s, l, interp_buffer);
        if (interp_buffer) {
            rc = norm_sync(s, l, 1, &scale);
            if (rc) return rc;
        }
        if (!(scale > 0.0)) {
            rc = norm_sync(s, l, 2, &scale);
            if (rc) return rc;
            if (!std::isfinite(scale)) return set_err(s, NP_ENONFINITE, "level %d: non-finite boundary data", l);
        }
        // with the defect correction the starting residual pass also keeps
        // f - lap phi in FP32, the source of the level's first scaled defect
        // (unless the learned guess changes phi after it)
        const bool dc = c.precision != NP_PREC_FP64;
        // the learned guess runs unless it was found not to pay on this level
        const bool net = l > 0 && c.guess == NP_GUESS_LEARNED && s->have_weights && !(c.guess_gate && s->guess_off[l]);
        const bool r32_start = dc && !net;
        double r = 0.0;
        rc = r32_start ? dc_first_residual(s, l, &r) : norm_sync(s, l, 0, &r);
        if (rc) return rc;
        st.interp_rel_residual[l] = scale > 0 ? r / scale : r;
        const double rho_p = l > 0 && s->rho_meas[c.parent[l]] > 0.0 ? s->rho_meas[c.parent[l]] : kAdaptiveRho0;
        double t_guess = 0.0;
        if (net) {
            const auto tg = std::chrono::steady_clock::now();
            rc = learned_guess(s, l, rho[l], fourpiG, fnorm, rho_p, &r, &st.learned_used[l], &st.learned_ran[l]);
            if (rc) return rc;
            t_guess = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tg).count();
            st.guess_ms[l] = t_guess;
            st.guess_box_ratio[l] = s->guess_box_ratio[l];
        }
        double Fdelta = 0.0;
        bool pinned = s->has_fixed && s->fixed[l] >= 0;
        if (c.stop_rule == NP_STOP_FORCE_DELTA && !pinned) {
            rc = force_delta_sync(s, l, &Fdelta);  // seeds the previous-force buffer
            if (rc) return rc;
        }
        const double r0 = r;
        s->hist[l].push_back(scale > 0 ? r / scale : r);
        int q = 0;
        int lvl = NP_OK;
        // defect correction: r_lo holds (f - lap phi) / r_scale for the current phi
        bool have_defect = false;
        double r_scale = 1.0;
        double rho = kAdaptiveRho0;
        int outer = 0;
        if (dc) {
            // multigrid level 0 of the correction has a zero ghost layer, and the
            // defect's ghost layer stands in for it where a black half sweep forms
            // the red values from the defect.  The arrays are shared by the levels:
            // cleared whole when this level's grid differs from the one they were
            // last cleared for (every kernel writes their active points only, and
            // each active point is written before it is read within a level)
            if (!same_grid(s->lg[l], s->lo_ghost_grid)) {
                size_t esz = c.precision == NP_PREC_FP16S_DC ? sizeof(__half) : sizeof(float);
                HIPCHK(s, hipMemsetAsync(s->e_lo, 0, 2 * s->lg[l].cs * esz, s->stream));
                HIPCHK(s, hipMemsetAsync(s->e_nx, 0, 2 * s->lg[l].cs * esz, s->stream));
                HIPCHK(s, hipMemsetAsync(s->r_lo, 0, 2 * s->lg[l].cs * esz, s->stream));
                s->lo_ghost_grid = s->lg[l];
            }
            // the outer pass writes only active points of the other potential
            // buffer: give it this level's fixed ghost layer
            launch_copy_ghosts(c.dim, s->stream, s->lg[l], s->phi[l], s->phi_alt);
        }
        // full sweeps write the active points of the spare buffer: the same
        const bool fs = !dc && full_sweeps(s, l);
        bool first_done = false;  // the next cycle's first pre-smoothing sweep has run
        if (fs) launch_copy_ghosts(c.dim, s->stream, s->lg[l], s->phi[l], s->phi_alt);
        for (;;) {
            if (!std::isfinite(r)) { lvl = NP_ENONFINITE; break; }
            if (pinned) {
                if (q >= s->fixed[l]) break;
            } else if (c.stop_rule == NP_STOP_RESIDUAL && r <= c.tol * scale) {
                break;
            }
            if (q >= c.max_cycles) { lvl = NP_ENOTCONV; break; }
            if (dc) {
                if (!have_defect) {
                    double same = 0.0;
                    r_scale = r > 0 ? r : 1.0;
                    rc = r32_start ? dc_scale_defect(s, l, 1.0 / r_scale)
                                   : dc_outer_sync(s, l, false, 0.0, 1.0 / r_scale, &same);
                    if (rc) return rc;
                    have_defect = true;
                }
                const int k = dc_cycles(c, r, c.tol * scale, rho, q, pinned ? s->fixed[l] : c.max_cycles);
                rc = dc_inner(s, l, k);
                if (rc) return rc;
                q += k;
                outer++;
                // phi += h^2 r_scale e'', then the residual of the updated potential,
                // scaled by the previous norm (the new one is not known until the pass ends)
                double rprev = r > 0 ? r : 1.0;
                double dx = level_dx(&c, l);
                rc = dc_outer_sync(s, l, true, dx * dx * r_scale, 1.0 / rprev, &r);
                if (rc) return rc;
                r_scale = rprev;
                if (r > 0.0 && r < rprev) {
                    const double m = std::pow(r / rprev, 1.0 / k);
                    rho = m < 0.02 ? 0.02 : (m > 0.95 ? 0.95 : m);
                }
            } else if (fs) {
                rc = vcycle_full(s, l, first_done);
                if (rc) return rc;
                HIPCHK(s, hipGetLastError());
                q++;
                rc = full_sweep_norm_sync(s, l, &r);
                if (rc) return rc;
                first_done = true;
            } else {
                rc = vcycle(s, l);
                if (rc) return rc;
                HIPCHK(s, hipGetLastError());
                q++;
                rc = norm_sync(s, l, 0, &r);
                if (rc) return rc;
            }
            s->hist[l].push_back(scale > 0 ? r / scale : r);
            if (!std::isfinite(r)) { lvl = NP_ENONFINITE; break; }
            if (r0 > 0 && r > 1e3 * r0) { lvl = NP_EDIVERGED; break; }
            if (c.stop_rule == NP_STOP_FORCE_DELTA && !pinned) {
                rc = force_delta_sync(s, l, &Fdelta);
                if (rc) return rc;
                if (Fdelta < c.tol) break;
            }
        }
        if (dc || fs) {
            rc = dc_settle(s, l);
            if (rc) return rc;
        }
        if (interp_buffer) {
            // the relaxed values back into Omega^l of the level's array
            prof_begin(s, NP_KCLASS_FILL);
            launch_copy_box(d, s->stream, s->lg[l], s->phi[l], dom.g, dom.phi, 2, box_hi, -1);
            prof_end(s);
            HIPCHK(s, hipGetLastError());
        }
        st.cycles[l] = q;
        st.outer_steps[l] = outer;
        // contraction per V-cycle of this level (geometric mean), clamped
        if (q > 0 && r0 > 0.0 && r > 0.0 && r < r0) {
            const double m = std::pow(r / r0, 1.0 / q);
            s->rho_meas[l] = m < 0.02 ? 0.02 : (m > 0.95 ? 0.95 : m);
        } else {
            s->rho_meas[l] = 0.0;
        }
        st.scale[l] = scale;
        st.initial_rel_residual[l] = s->hist[l].front();
        st.final_rel_residual[l] = scale > 0 ? r / scale : r;
        st.level_ms[l] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (net && c.guess_gate) {
            // V-cycles the kept guess is predicted to save (its restricted
            // residual over the interpolated guess's, in contractions of one
            // cycle, the keep test's terms) at this level's time per cycle,
            // against the time the learned guess took
            const double ratio = st.guess_box_ratio[l];
            double n_save = 0.0;
            if (st.learned_used[l] && ratio > 0.0 && ratio < 1.0 && rho_p > 0.0 && rho_p < 1.0)
                n_save = std::log(ratio) / std::log(rho_p);
            const double per_cycle = q > 0 ? (st.level_ms[l] - t_guess) / q : 0.0;
            if (!(n_save * per_cycle > t_guess)) s->guess_off[l] = true;
        }
        if (lvl == NP_ENONFINITE || lvl == NP_EDIVERGED) {
            if (stats) *stats = st;
            return set_err(s, lvl, "level %d: %s after %d cycles", l,
                           lvl == NP_ENONFINITE ? "non-finite residual" : "residual diverged", q);
        }
        if (lvl == NP_ENOTCONV && status == NP_OK) {
            status = NP_ENOTCONV;
            set_err(s, NP_ENOTCONV, "level %d: not converged in %d cycles (rel. residual %.3e)", l, q,
                    st.final_rel_residual[l]);
        }
    }
    st.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_all).count();
    if (stats) *stats = st;
    s->solved = true;
    return status;
}

int nested_poisson_history(const np_solver* s, int level, double* out, int cap)
{
    if (!s || !out || cap < 0 || level < 0 || level >= s->cfg.nlevels) return NP_EINVAL;
    int m = (int)s->hist[level].size();
    if (m > cap) m = cap;
    for (int i = 0; i < m; i++) out[i] = s->hist[level][i];
    return m;
}

int nested_poisson_forces(np_solver* s, int level, double* fx, double* fy, double* fz)
{
    if (!s) return NP_EINVAL;
    if (level < 0 || level >= s->cfg.nlevels) return set_err(s, NP_EINVAL, "level %d out of range", level);
    if (!fx || !fy || (s->cfg.dim == 3 && !fz)) return set_err(s, NP_EINVAL, "null force pointer");
    if (!s->solved) return set_err(s, NP_ESTATE, "forces requested before a successful solve");
    HIPCHK(s, hipSetDevice(s->device));
    prof_begin(s, NP_KCLASS_FORCES);
    launch_forces(s->cfg.dim, s->stream, s->lg[level], level_dx(&s->cfg, level), s->phi[level], fx, fy, fz);
    prof_end(s);
    HIPCHK(s, hipGetLastError());
    return NP_OK;
}

int nested_poisson_potential(np_solver* s, int level, double* phi_padded)
{
    if (!s) return NP_EINVAL;
    if (level < 0 || level >= s->cfg.nlevels) return set_err(s, NP_EINVAL, "level %d out of range", level);
    if (!phi_padded) return set_err(s, NP_EINVAL, "null output pointer");
    if (!s->solved) return set_err(s, NP_ESTATE, "potential requested before a successful solve");
    HIPCHK(s, hipSetDevice(s->device));
    launch_export(s->cfg.dim, s->stream, s->lg[level], s->phi[level], phi_padded);
    HIPCHK(s, hipGetLastError());
    return NP_OK;
}

void nested_poisson_destroy(np_solver* s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    prof_release(s);
    free_all(s);
    delete s;
}

// Parameter blob of the learned guess (layout in nested_poisson.h).
static const unsigned kBlobCin[3] = {2, 16, 16}, kBlobCout[3] = {16, 16, 1};

static uint16_t host_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

int nested_poisson_pack_guess_weights(const float* theta, size_t n, void* blob, size_t nbytes)
{
    if (!theta || !blob || n != NP_NET_PARAMS || nbytes < NP_GUESS_BLOB_BYTES) {
        snprintf(g_last_error, sizeof g_last_error, "pack: need %d parameters and a blob of %d bytes",
                 NP_NET_PARAMS, (int)NP_GUESS_BLOB_BYTES);
        return NP_EINVAL;
    }
    unsigned char* out = (unsigned char*)blob;
    const uint32_t hdr[10] = {NP_GUESS_BLOB_MAGIC, NP_GUESS_BLOB_VERSION, 3, kBlobCin[0], kBlobCout[0],
                              kBlobCin[1], kBlobCout[1], kBlobCin[2], kBlobCout[2], 0};
    memcpy(out, hdr, sizeof hdr);
    size_t o = NP_GUESS_BLOB_HEADER, k = 0;
    for (int L = 0; L < 3; L++) {
        const size_t nw = 27 * (size_t)kBlobCin[L] * kBlobCout[L];
        for (size_t i = 0; i < nw; i++) {
            const uint16_t b = host_bf16(theta[k + i]);
            memcpy(out + o + 2 * i, &b, 2);
        }
        o += 2 * nw;
        memcpy(out + o, theta + k + nw, 4 * (size_t)kBlobCout[L]);
        o += 4 * (size_t)kBlobCout[L];
        k += nw + kBlobCout[L];
    }
    return NP_OK;
}

int nested_poisson_check_guess_weights(const void* blob, size_t nbytes)
{
    auto bad = [](const char* why) {
        snprintf(g_last_error, sizeof g_last_error, "guess weights: %s", why);
        return NP_EINVAL;
    };
    if (!blob) return bad("null blob");
    if (nbytes != NP_GUESS_BLOB_BYTES) return bad("size mismatch");
    uint32_t hdr[10];
    memcpy(hdr, blob, sizeof hdr);
    if (hdr[0] != NP_GUESS_BLOB_MAGIC) return bad("wrong magic");
    if (hdr[1] != NP_GUESS_BLOB_VERSION) return bad("unsupported version");
    if (hdr[2] != 3) return bad("layer count is not 3");
    for (int L = 0; L < 3; L++)
        if (hdr[3 + 2 * L] != kBlobCin[L] || hdr[4 + 2 * L] != kBlobCout[L]) return bad("layer shape mismatch");
    const unsigned char* in = (const unsigned char*)blob;
    size_t o = NP_GUESS_BLOB_HEADER;
    for (int L = 0; L < 3; L++) {
        o += 2 * 27 * (size_t)kBlobCin[L] * kBlobCout[L];
        for (unsigned c = 0; c < kBlobCout[L]; c++) {
            float b;
            memcpy(&b, in + o + 4 * c, 4);
            if (!std::isfinite(b)) return bad("non-finite bias");
        }
        o += 4 * (size_t)kBlobCout[L];
    }
    return NP_OK;
}

int nested_poisson_set_guess_weights(np_solver* s, const void* blob, size_t nbytes)
{
    if (!s) return NP_EINVAL;
    if (nested_poisson_check_guess_weights(blob, nbytes) != NP_OK)
        return set_err(s, NP_EINVAL, "%s", g_last_error);
    if (s->cfg.guess != NP_GUESS_LEARNED) return set_err(s, NP_ESTATE, "handle created without the learned guess");
    HIPCHK(s, hipSetDevice(s->device));
    const unsigned char* in = (const unsigned char*)blob;
    size_t o = NP_GUESS_BLOB_HEADER;
    for (int k = 0; k < 3; k++) {
        const size_t nw = 27 * (size_t)kBlobCin[k] * kBlobCout[k];
        HIPCHK(s, hipMemcpyAsync(s->net_w[k], in + o, 2 * nw, hipMemcpyHostToDevice, s->stream));
        o += 2 * nw;
        HIPCHK(s, hipMemcpyAsync(s->net_b[k], in + o, 4 * (size_t)kBlobCout[k], hipMemcpyHostToDevice, s->stream));
        o += 4 * (size_t)kBlobCout[k];
    }
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->have_weights = true;
    for (int l = 0; l < NP_MAX_LEVELS; l++) s->guess_off[l] = false;
    return NP_OK;
}

int nested_poisson_guess_features(np_solver* s, int level, float* x, float* target)
{
    if (!s) return NP_EINVAL;
    const np_config& c = s->cfg;
    if (c.dim != 3 || level < 1 || level >= c.nlevels || !x)
        return set_err(s, NP_EINVAL, "features need a 3-D level >= 1 and an output array");
    if (!s->solved) return set_err(s, NP_ESTATE, "features requested before a successful solve");
    HIPCHK(s, hipSetDevice(s->device));
    if (!s->feat_phi) {
        size_t best = 0;
        for (int l = 0; l < c.nlevels; l++)
            if (2 * s->lg[l].cs > best) best = 2 * s->lg[l].cs;
        int rc = alloc_dev(s, (void**)&s->feat_phi, best * sizeof(double));
        if (rc == NP_OK) rc = alloc_dev(s, (void**)&s->feat_f, best * sizeof(double));
        if (rc) return rc;
    }
    // the interpolated guess of this level, rebuilt from the converged coarser level;
    // the density of the patch itself does not enter Phi_interp, so the level's own
    // right-hand side serves as the density argument (only f_tmp's patch part uses it)
    const int l = level;
    double dx = level_dx(&c, l);
    double fourpiG = 4.0 * M_PI * c.G;
    launch_interface_fill(c.dim, s->stream, s->lg[c.parent[l]], s->phi[c.parent[l]], s->f[c.parent[l]], s->lg[l],
                          c.offset[l][0], c.offset[l][1], c.offset[l][2], s->f[l], 0.0, s->feat_phi, s->feat_f,
                          nullptr);
    double fnorm = 0.0;
    int rc = norm_sync(s, l, 1, &fnorm);
    if (rc) return rc;
    if (!(fnorm > 0.0)) return set_err(s, NP_EINVAL, "level %d has zero density", l);
    (void)fourpiG;
    net_features_f32(s->stream, s->lg[l], s->feat_phi, s->f[l], 1.0 / fnorm, 1.0 / (dx * dx), x);
    if (target) net_target(s->stream, s->lg[l], s->phi[l], s->feat_phi, 1.0 / (fnorm * dx * dx), target);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return NP_OK;
}

int nested_poisson_set_profiling(np_solver* s, int enable)
{
    if (!s) return NP_EINVAL;
    HIPCHK(s, hipSetDevice(s->device));
    if (s->prof) {
        int rc = prof_flush(s);
        if (rc) return rc;
    }
    for (int c = 0; c < NP_NKCLASS; c++) {
        s->prof_count[c] = 0;
        s->prof_ms[c] = 0.0;
    }
    if (!enable) {
        prof_release(s);
        return NP_OK;
    }
    if (s->ev.empty()) {
        const int pool = 4096;
        s->ev.resize(pool);
        s->ev_cls.resize(pool / 2);
        s->ev_n.resize(pool / 2);
        for (int i = 0; i < pool; i++) {
            if (hipEventCreate(&s->ev[i]) != hipSuccess) {
                s->ev.resize(i);
                prof_release(s);
                return set_err(s, NP_EHIP, "hipEventCreate failed");
            }
        }
    }
    s->ev_used = 0;
    s->prof = true;
    return NP_OK;
}

int nested_poisson_get_profile(np_solver* s, np_profile* out)
{
    if (!s || !out) return NP_EINVAL;
    if (!s->prof) return set_err(s, NP_ESTATE, "profiling is not enabled");
    HIPCHK(s, hipSetDevice(s->device));
    int rc = prof_flush(s);
    if (rc) return rc;
    for (int c = 0; c < NP_NKCLASS; c++) {
        out->count[c] = s->prof_count[c];
        out->ms[c] = s->prof_ms[c];
    }
    return NP_OK;
}

const char* nested_poisson_strerror(int code)
{
    switch (code) {
    case NP_OK: return "ok";
    case NP_EINVAL: return "invalid argument";
    case NP_ENOMEM: return "out of memory";
    case NP_EHIP: return "HIP runtime error";
    case NP_ENONFINITE: return "non-finite value";
    case NP_ENOTCONV: return "not converged";
    case NP_EDIVERGED: return "diverged";
    case NP_ESTATE: return "call out of order";
    case NP_ENODEV: return "no HIP device";
    default: return "unknown error";
    }
}

const char* nested_poisson_last_error(const np_solver* s) { return s ? s->err : g_last_error; }

}  // extern "C"

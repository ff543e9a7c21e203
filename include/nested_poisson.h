/*
 * nested_poisson.h -- C ABI of the MI355X (gfx950) nested-grid multigrid
 * self-gravity solver.
 *
 * Method: H.-H. Wang & C.-C. Yen, "Self-gravitational Force Calculation of
 * Second Order Accuracy Using Multigrid Method on Nested Grids"
 * (arXiv:2001.02327).  The solver computes the potential of
 *     lap(Phi) = 4 pi G rho          (Sec. 1, first equation)
 * on a stack of nested Cartesian patches with refinement ratio 2 (Sec. 2.1),
 * level by level from coarse to fine (one-way interface scheme), and the
 * forces F = -grad(Phi) with the fourth-order central difference
 * (Eqn:force_evaluation).
 *
 * Geometry (Sec. 2.1).  The entries l = 0 .. nlevels-1 ("levels") are
 * patches: entry 0 is the base level; every other entry l is refined out of
 * its parent p = parent[l] (0 <= p < l), with cell size dx_p / 2, so the cell
 * size of entry l is dx0 / 2^depth(l).  nested_poisson_default_config sets
 * parent[l] = l - 1, the paper's stack of one patch per level; a tree gives
 * several disjoint patches per level (the patch-based setting of Sec. 4).
 * Entry l is a box of n_a = extent[l][a] cells along axis a (Sec. 2.1 gives
 * the cell counts per direction; the cells are cubes), or a cube (square in
 * 2-D) of n[l] cells per axis when extent[l][0] is 0.  Its lower corner lies
 * offset[l][a] cells of p above p's lower corner along axis a; it must keep
 * at least one coarse cell of margin on every side:
 *     1 <= offset[l][a]  and  offset[l][a] + n_a/2 <= n_a(p) - 1,
 * and patches with the same parent must not overlap.  Patches are solved in
 * entry order, each from its converged parent (one-way scheme).
 * Each level carries a two-cell buffer.  Its padded array has n_a + 4
 * points along axis a: index 0 and n_a+3 are the outer buffer layer
 * (Dirichlet potential), 1 and n_a+2 the inner buffer layer (relaxed together
 * with the patch), 2..n_a+1 the patch itself.  Cell i of the patch is centred
 * at lo_l + (i + 1/2) dx_l.
 *
 * Memory.  Every array crossing this ABI is row-major with x fastest
 * ([k][j][i] in 3-D, [j][i] in 2-D), FP64, in DEVICE memory of the device
 * that was current at create time.  The library allocates and owns all of
 * its working storage; the caller owns every pointer it passes and must keep
 * it valid until the call returns (solve) or until the work queued on the
 * handle's stream has completed (forces, potential).
 *
 * Errors.  Every function returns 0 on success or a negative NP_E* code; no
 * C++ exception or abort crosses the ABI.  nested_poisson_last_error() gives a
 * message for the last failure on a handle.  A handle is not thread-safe:
 * use one handle per host thread and stream.
 */
#ifndef NESTED_POISSON_H
#define NESTED_POISSON_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NP_MAX_LEVELS 16  /* nested patches (entries) per solver */
#define NP_MAX_MG 32      /* multigrid levels per patch */
#define NP_MAX_CYCLES 200 /* cap on max_cycles */

/* return codes */
#define NP_OK 0
#define NP_EINVAL (-1)      /* invalid argument or geometry */
#define NP_ENOMEM (-2)      /* device or host allocation failed */
#define NP_EHIP (-3)        /* a HIP runtime call failed */
#define NP_ENONFINITE (-4)  /* NaN/Inf in the input or the residual */
#define NP_ENOTCONV (-5)    /* max_cycles reached; the potential is still valid */
#define NP_EDIVERGED (-6)   /* residual grew beyond 1e3 x its initial value */
#define NP_ESTATE (-7)      /* call out of order (e.g. forces before solve) */
#define NP_ENODEV (-8)      /* no HIP device available */

/* stop rules (Sec. 2.3 step 14 and Sec. 3.1) */
#define NP_STOP_RESIDUAL 0    /* ||f - lap Phi||_inf <= tol * ||f||_inf over the relaxed points */
#define NP_STOP_FORCE_DELTA 1 /* max over the patch of |F^q - F^{q-1}| < tol (the paper's rule) */

/* arithmetic of the V-cycles */
#define NP_PREC_FP64 0     /* every operator in FP64 */
#define NP_PREC_FP32_DC 1  /* FP32 V-cycles inside FP64 defect correction */
#define NP_PREC_FP16S_DC 2 /* FP16-stored, FP32-computed finest-level V-cycle arrays inside FP64 defect correction */
#define NP_INNER_ADAPTIVE 0 /* inner_cycles: chosen per step from the measured contraction */

/* initial guess of levels l >= 1 */
#define NP_GUESS_INTERP 0  /* interpolated from the parent patch (Sec. 2.4) */
#define NP_GUESS_LEARNED 1 /* interpolated guess plus the correction predicted by the conv net */

/* buffer zone of levels l >= 1 (Sec. 2.1 and Sec. 4, Fig. 4) */
#define NP_BUFFER_RELAXED 0 /* the paper's method: the inner buffer layer is relaxed with the patch */
#define NP_BUFFER_INTERP 1  /* comparison scheme of Sec. 4: both buffer layers keep the potential
                               interpolated from the parent and only Omega^l is relaxed (the inner
                               layer is its Dirichlet data); FP64, interpolated guess and the
                               residual stop rule only */

/* How multigrid level 0 of a 3-D FP64 solve is smoothed (np_config.sweep).
 * NP_SWEEP_FULL: on level grids whose full sweep starts at least 4096
 * wavefronts (cubic levels from about 420^3 cells; on smaller or thin grids
 * the half sweeps, which occupy the chip better, run), each
 * red-black sweep is one pass from the level's potential
 * into a second buffer (the handle's; the buffers then trade roles), and the
 * stop test's residual norm is taken inside the sweeps: over the black points
 * by the last post-smoothing sweep, over the red points by the next cycle's
 * first pre-smoothing sweep, which runs before the test and is dropped when
 * the level stops (needs n_pre >= 1 and n_post >= 1, the relaxed buffer on
 * levels l >= 1 and a level solved on its own; elsewhere the half sweeps run).
 * NP_SWEEP_HALF: two half sweeps in place and a separate residual pass.
 * NP_SWEEP_FULL_ALL: as NP_SWEEP_FULL on every level, whatever its size.
 * NP_SWEEP_FUSED: as NP_SWEEP_FULL, and in the defect correction with 2-byte
 * storage (3-D) the last pre-smoothing black half sweep of multigrid level 0
 * runs inside the restriction that follows it (Sec. 2.3 steps 2-5 in one pass;
 * needs N^0 = 2 N^1 along every axis and an odd N^1_x, elsewhere they run
 * apart).  On MI355X this pass is slower than the two kernels it replaces, so
 * it is not the default.  The iterates are the same in all four. */
#define NP_SWEEP_FULL 0
#define NP_SWEEP_HALF 1
#define NP_SWEEP_FUSED 2
#define NP_SWEEP_FULL_ALL 3

typedef struct np_config {
    int dim;                        /* 2 or 3 */
    int nlevels;                    /* 1..NP_MAX_LEVELS */
    int n[NP_MAX_LEVELS];           /* cells per axis of level l: even, >= 4 */
    int offset[NP_MAX_LEVELS][3];   /* l >= 1: corner offset in cells of the parent (see above) */
    double dx0;                     /* cell size of level 0, > 0 */
    double G;                       /* gravitational constant */
    int n_pre;                      /* pre-smoothing sweeps (the paper uses 2), 0..16 */
    int n_post;                     /* post-smoothing sweeps (the paper uses 1), 0..16 */
    double tol;                     /* stop tolerance, > 0 */
    int max_cycles;                 /* 1..NP_MAX_CYCLES */
    int stop_rule;                  /* NP_STOP_* */
    int precision;                  /* NP_PREC_* */
    int inner_cycles;               /* low-precision V-cycles per defect-correction step: 1..8,
                                       or NP_INNER_ADAPTIVE (0): 1..4 per step (1..3 with FP16
                                       storage), as many as the contraction measured so far
                                       says the stop test needs */
    int guess;                      /* NP_GUESS_* */
    int buffer;                     /* NP_BUFFER_* */
    int parent[NP_MAX_LEVELS];      /* l >= 1: the entry patch l is refined out of, 0 <= parent[l] < l */
    int extent[NP_MAX_LEVELS][3];   /* cells of level l along x, y (, z): each even, >= 4; all zero:
                                       n[l] along every axis */
    int batch;                      /* 1 (default): patches of one refinement depth with the same
                                       extents are solved together, one launch per operator over
                                       all of them, each patch stopping at its own cycle count (FP64,
                                       interpolated guess, relaxed buffer, residual stop rule;
                                       otherwise one after another); 0: one after another */
    int sweep;                      /* NP_SWEEP_* (default NP_SWEEP_FULL) */
    int guess_gate;                 /* NP_GUESS_LEARNED: 1 (default) runs the network on a level only
                                       while it pays.  After each inference the solve compares the
                                       host time the learned guess took with the V-cycles it is
                                       predicted to save (log of its restricted-residual ratio over
                                       log of the parent's measured contraction per cycle, the keep
                                       test's terms) times the level's time per V-cycle; where it
                                       does not pay, later solves of the handle start that level from
                                       the interpolated guess without running the network
                                       (nested_poisson_set_guess_weights re-arms every level).
                                       0: the network runs in every solve */
    int coarse_post;                /* post-smoothing sweeps on the multigrid levels below level 0
                                       (the coarse part of every V-cycle, coarse tail included),
                                       0..16; -1 (default): n_post.  The defect correction's inner
                                       V-cycles only precondition its FP64 iteration, so their
                                       schedule is free; the FP64 V-cycle of Sec. 2.3 is V(n_pre,
                                       n_post) on every level */
} np_config;

/* Fills `cfg` with the paper's solver settings (N_pre = 2, N_post = 1,
 * Sec. 3) and tol = 1e-10, max_cycles = 50, FP64, residual stop,
 * interpolated guess, relaxed buffer, parent[l] = l - 1, batch = 1,
 * guess_gate = 1, coarse_post = -1.  The other
 * geometry fields (extent included: cubic patches) are zeroed. */
void nested_poisson_default_config(np_config* cfg);

/* Multigrid hierarchy of one patch (Sec. 2.2), along each axis a: N^0_a =
 * n_a + 2 (patch plus its inner buffer layer; N^0_a = n_a on levels l >= 1
 * with NP_BUFFER_INTERP, where the patch alone is relaxed), N^L_a =
 * round(N^0_a / 2^L) with halves rounded up (every axis doubles its mesh size,
 * so the cells stay cubes); the hierarchy ends on the first level with one
 * active cell along some axis (for a cube: N^L = 1).  For L >= 1, right-ghost
 * rule of Sec. 2.4 per axis: xn_is_one[L][a] is 1 when the right-most active
 * centre sits exactly at x_MG = 1 (ghost = -e_{N-1}), otherwise ghost =
 * ghost_coef[L][a] * e_N, the value at x_N + h^L of the line through
 * (x_N, e_N) that vanishes at x_MG = 1.  The ghost refresh is explicit, so an
 * error at the last active cell returns amplified by ghost_coef / (2 dim);
 * hierarchies where that gain exceeds NP_MAX_GHOST_GAIN (x_N just below 1,
 * e.g. N^0 = 194 at L = 7 with ghost_coef = -63) make the V-cycle diverge and
 * are refused (NP_EINVAL). */
#define NP_MAX_GHOST_GAIN 6.0
typedef struct np_plan {
    int nmg[NP_MAX_LEVELS];                      /* multigrid levels of each nested level */
    int N[NP_MAX_LEVELS][NP_MAX_MG][3];          /* active cells along x, y, z (z: 1 in 2-D) */
    int xn_is_one[NP_MAX_LEVELS][NP_MAX_MG][3];
    double ghost_coef[NP_MAX_LEVELS][NP_MAX_MG][3];
} np_plan;

/* Validates `cfg` and computes the hierarchy on the host; touches no device.
 * Returns NP_EINVAL for an invalid configuration. */
int nested_poisson_plan(const np_config* cfg, np_plan* out);

typedef struct np_solver np_solver;

/* Creates a solver on the current HIP device.  `hip_stream` is a hipStream_t
 * (NULL = the null stream); all device work of the handle is queued on it.
 * Allocates the per-level potential and right-hand side and the multigrid
 * scratch.  Errors: NP_EINVAL (cfg invalid; checked before any device call),
 * NP_ENODEV, NP_ENOMEM, NP_EHIP. */
int nested_poisson_create(const np_config* cfg, void* hip_stream, np_solver** out);

/* Nested solve (Sec. 2.1 one-way scheme, Sec. 2.3 V-cycle).
 *   rho[0]    : n_a(0) + 2 points per axis: density of level 0 including its
 *               inner buffer layer
 *   rho[l>=1] : n_a(l) points per axis: density of level l (the inner buffer
 *               layer of l >= 1 gets the density interpolated from its parent)
 *   phi_outer : n_a(0) + 4 points per axis; only the outer layer is read
 *               (Dirichlet data of level 0)
 * Level 0 starts from Phi = 0; level l >= 1 from the potential interpolated
 * from its parent (plus the learned correction with NP_GUESS_LEARNED).
 * Returns after the last stop test of the finest level (host-synchronous).
 * `stats` may be NULL.  Errors: NP_EINVAL, NP_ENONFINITE, NP_ENOTCONV (the
 * cap was hit on some level; results are valid), NP_EDIVERGED, NP_EHIP. */
typedef struct np_stats {
    int cycles[NP_MAX_LEVELS];                /* V-cycles per level (inner ones for DC) */
    double initial_rel_residual[NP_MAX_LEVELS];
    double final_rel_residual[NP_MAX_LEVELS]; /* ||r||_inf / scale at exit */
    double scale[NP_MAX_LEVELS];              /* reference norm of the stop test */
    double level_ms[NP_MAX_LEVELS];           /* host wall time per level */
    double total_ms;
    int learned_used[NP_MAX_LEVELS];          /* 1 where the learned guess was kept */
    double interp_rel_residual[NP_MAX_LEVELS];/* relative residual of the interpolated guess */
    int outer_steps[NP_MAX_LEVELS];           /* defect-correction steps (0 for NP_PREC_FP64) */
    double guess_box_ratio[NP_MAX_LEVELS];    /* learned guess: its residual restricted twice (mean over
                                                 4^3 boxes, max norm) over the interpolated guess's */
    int learned_ran[NP_MAX_LEVELS];           /* 1 where the network ran in this solve */
    double guess_ms[NP_MAX_LEVELS];           /* host time of the learned guess (inference, its
                                                 residual norms and a rejected guess's refill) */
} np_stats;
int nested_poisson_solve(np_solver* s, const double* const* rho, const double* phi_outer, np_stats* stats);

/* Runs exactly cycles[l] V-cycles on level l instead of the stop rule
 * (cycles[l] < 0 keeps the stop rule for that level).  NULL clears.  Used to
 * compare iterates at equal cycle counts.  The array has nlevels entries. */
int nested_poisson_set_fixed_cycles(np_solver* s, const int* cycles);

/* Relative residual after each cycle (each outer step for the defect
 * correction) of the last solve on `level`: out[0] is before the first one.  Writes min(cap, cycles+1) values and
 * returns their count (or a negative error). */
int nested_poisson_history(const np_solver* s, int level, double* out, int cap);

/* F = -grad(Phi) on the cells of level `level` (Eqn:force_evaluation),
 * written to device arrays fx, fy (and fz in 3-D; ignored in 2-D), each of
 * the level's shape (n_z x n_y x n_x, x fastest).
 * Queued on the handle's stream; does not synchronise.
 * Errors: NP_EINVAL (level out of range, null pointer), NP_ESTATE (no solve). */
int nested_poisson_forces(np_solver* s, int level, double* fx, double* fy, double* fz);

/* Copies the padded potential of `level` (n_a + 4 points per axis) into the
 * device array `phi_padded` (both buffer layers included).  Queued on the stream.
 * Errors: as nested_poisson_forces. */
int nested_poisson_potential(np_solver* s, int level, double* phi_padded);

/* Kernel-class timing.  With profiling enabled the handle records a HIP
 * event pair on its stream around each launch (or group of launches) of a
 * class and accumulates the elapsed device time; classes: */
#define NP_KCLASS_SMOOTH 0   /* red-black half sweeps on the nested-level arrays (multigrid level 0) */
#define NP_KCLASS_RESTRICT 1 /* fused residual + restriction out of multigrid level 0 */
#define NP_KCLASS_PROLONG 2  /* prolongation + correction into multigrid level 0 */
#define NP_KCLASS_COARSE 3   /* all work on multigrid levels >= 1 (one interval per V-cycle) */
#define NP_KCLASS_NORM 4     /* max-norm reductions of the stop test (residual, or force change) */
#define NP_KCLASS_FILL 5     /* level-0 setup and coarse-to-fine fills */
#define NP_KCLASS_FORCES 6   /* force evaluation */
#define NP_KCLASS_DC 7       /* FP64 residual / correction passes of the defect correction */
#define NP_KCLASS_GUESS 8    /* learned initial guess (features, three convolutions, update) */
#define NP_KCLASS_SEEDED 9   /* first black half sweep of a defect-correction step, which forms its red
                              * neighbours from the defect (and stores them with one pre-smoothing sweep) */
#define NP_KCLASS_FULL 10    /* full red-black sweeps of multigrid level 0 (NP_SWEEP_FULL) */
#define NP_KCLASS_FULL_RES 11 /* the full sweep that also completes the stop test's residual norm */
#define NP_KCLASS_DC_SCALE 12 /* first scaled defect of a level from its starting residual */
#define NP_KCLASS_BLACK_RESTRICT 13 /* last pre-smoothing black half sweep of multigrid level 0 fused with
                                     * the residual restriction (NP_SWEEP_FUSED, 2-byte storage) */
#define NP_NKCLASS 16
typedef struct np_profile {
    long count[NP_NKCLASS]; /* launches (intervals) recorded */
    double ms[NP_NKCLASS];  /* summed device time */
} np_profile;
/* enable != 0 starts (and zeroes) the counters, 0 stops and frees the events. */
int nested_poisson_set_profiling(np_solver* s, int enable);
/* Synchronises the stream and returns the totals since profiling was enabled.
 * Errors: NP_EINVAL, NP_ESTATE (profiling off), NP_EHIP. */
int nested_poisson_get_profile(np_solver* s, np_profile* out);

/* ------------------------------------------------------------------ learned initial guess
 * A 3-D convolution network predicts, for a level l >= 1, the correction of
 * the interpolated initial guess (an extension; the paper interpolates only):
 *   input  x = (f / ||f||_inf, r0 / ||f||_inf) on Gamma^l, r0 = f - lap(Phi_interp),
 *   output y on Gamma^l, guess = Phi_interp + ||f||_inf dx_l^2 y,
 * network conv3x3x3(2->16) -> ReLU -> conv3x3x3(16->16) -> ReLU ->
 * conv3x3x3(16->1), zero padding, same size.  The V-cycles then iterate to the
 * same tolerance.  The guess is kept only where it should save a V-cycle:
 * the cycle count is set by the error the smoother leaves, whose residual
 * survives restriction, so the guess is kept if its residual restricted twice
 * (the mean over boxes of 4^3 points, max norm) is at most rho times that of
 * the interpolated guess, rho being the contraction per V-cycle measured on
 * the parent level's solve (0.3 before any); otherwise, or if non-finite, it
 * is discarded.
 * Parameter vector (NP_NET_PARAMS floats): for each layer its weights
 * [27 taps][cout][cin] (taps ordered dz, dy, dx in -1..1, dx fastest) then its
 * cout biases.  Activations of the np_net_* kernels are FP32 (or bfloat16 as
 * stated) channel-last [batch][z][y][x][channel] device arrays; weights are
 * bfloat16 device arrays; every call is queued on `stream` (hipStream_t). */
#define NP_NET_PARAMS 8241

/* Versioned parameter blob of the network (host memory, little-endian):
 *   header, NP_GUESS_BLOB_HEADER bytes of uint32: magic NP_GUESS_BLOB_MAGIC
 *     ("NPGW"), version NP_GUESS_BLOB_VERSION, layer count 3, then cin and
 *     cout of each layer (2,16), (16,16), (16,1), then 0;
 *   per layer: its bfloat16 weights [27 taps][cout][cin] (taps ordered
 *     dz, dy, dx in -1..1, dx fastest), then its cout FP32 biases.
 * NP_GUESS_BLOB_BYTES in all. */
#define NP_GUESS_BLOB_MAGIC 0x5747504eu /* "NPGW" */
#define NP_GUESS_BLOB_VERSION 1
#define NP_GUESS_BLOB_HEADER 40
#define NP_GUESS_BLOB_BYTES (NP_GUESS_BLOB_HEADER + 2 * (27 * (2 * 16 + 16 * 16 + 16 * 1)) + 4 * (16 + 16 + 1))

/* Packs a parameter vector (FP32, NP_NET_PARAMS values, the layout above with
 * FP32 weights) into a blob of nbytes >= NP_GUESS_BLOB_BYTES, rounding the
 * weights to bfloat16 (nearest even).  Host only; touches no device.
 * Errors: NP_EINVAL (null pointer, n != NP_NET_PARAMS, blob too small). */
int nested_poisson_pack_guess_weights(const float* theta, size_t n, void* blob, size_t nbytes);

/* Checks a blob's header, layer shapes and size (nbytes must equal
 * NP_GUESS_BLOB_BYTES) and that every bias is finite.  Host only.
 * Errors: NP_EINVAL with a message in nested_poisson_last_error(NULL). */
int nested_poisson_check_guess_weights(const void* blob, size_t nbytes);

/* Copies a blob (host memory, checked as above before any device work) into
 * the handle; required before a solve with guess = NP_GUESS_LEARNED.
 * Errors: NP_EINVAL (bad blob: wrong magic, version, shapes or size),
 * NP_ESTATE (handle created without the learned guess), NP_EHIP. */
int nested_poisson_set_guess_weights(np_solver* s, const void* blob, size_t nbytes);

/* Training data of level `level` >= 1 after a successful solve: the network
 * input x ((n_z+2) x (n_y+2) x (n_x+2) x 2 FP32, channel-last) built from the
 * interpolated guess, and target = (Phi_converged - Phi_interp) /
 * (||f||_inf dx_l^2) (one value per point of Gamma^l, FP32, may be NULL).
 * Device arrays.  Errors: NP_EINVAL, NP_ESTATE, NP_ENOMEM. */
int nested_poisson_guess_features(np_solver* s, int level, float* x, float* target);

/* Workspace (bytes) needed by np_net_conv3d_bwd_weight for (cin, cout) and by
 * np_net_mse for n values. */
size_t np_net_workspace_bytes(int cin, int cout, long nvox);
/* out = conv(in) + bias (ReLU if relu != 0); FP32 activations, bfloat16
 * weights, FP32 accumulation; 1 <= cin, cout <= 16. */
int np_net_conv3d_fwd(const float* in, int cin, const unsigned short* w_bf16, const float* bias, int cout, int relu,
                      int batch, int nz, int ny, int nx, float* out, void* stream);
/* A layer of the network on the matrix cores (the inference path), for
 * (cin, cout) = (2, 16), (16, 16) or (16, 1): bfloat16 activations in,
 * bfloat16 out (cout 16) or FP32 out (cout 1), FP32 accumulation
 * (v_mfma_f32_16x16x16 bf16); `in` aligned to 4 * cin bytes.  Other shapes:
 * NP_EINVAL. */
int np_net_conv3d_fwd_mfma(const unsigned short* in_bf16, int cin, const unsigned short* w_bf16, const float* bias,
                           int cout, int relu, int batch, int nz, int ny, int nx, void* out, void* stream);
/* gin = d loss / d in given gout = d loss / d out. */
int np_net_conv3d_bwd_data(const float* gout, int cout, const unsigned short* w_bf16, int cin, int batch, int nz,
                           int ny, int nx, float* gin, void* stream);
/* gw [27][cout][cin] and gb [cout] (FP32), summed in a fixed order (deterministic). */
int np_net_conv3d_bwd_weight(const float* in, int cin, const float* gout, int cout, int batch, int nz, int ny, int nx,
                             float* gw, float* gb, float* workspace, size_t workspace_bytes, void* stream);
/* grad *= (act > 0) */
int np_net_relu_bwd(const float* act, float* grad, long n, void* stream);
/* loss[0] = sum(mask (pred - target)^2) / count, grad = 2 mask (pred - target) / count
 * (mask may be NULL = all ones). */
int np_net_mse(const float* pred, const float* target, const float* mask, long n, float count, float* grad,
               float* loss, float* workspace, size_t workspace_bytes, void* stream);
/* np_net_mse without the workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops):
 * the partial sums live in a static device array of the library, so the
 * call allocates nothing.  n <= NP_NET_MSE_NOALLOC_MAX (2^28 values, 4 MiB
 * of partials held by each device the library runs on until the process
 * ends); larger n: NP_EINVAL with a message in nested_poisson_last_error(NULL).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (different streams or threads) race and must be serialised by
 * the caller.  Same results as np_net_mse.  NP_ENODEV / NP_EHIP if the
 * device's copy of the array cannot be located. */
#define NP_NET_MSE_NOALLOC_MAX (1L << 28)
int np_net_mse_noalloc(const float* pred, const float* target, const float* mask, long n, float count, float* grad,
                       float* loss, void* stream);
/* Adam with bias correction (step >= 1) on FP32 master weights; refreshes the
 * bfloat16 copy when w_bf16 is not NULL. */
int np_net_adam(float* w, const float* g, float* m, float* v, long n, float lr, float beta1, float beta2, float eps,
                int step, unsigned short* w_bf16, void* stream);
/* bfloat16 copy (round to nearest even). */
int np_net_to_bf16(const float* a, unsigned short* b, long n, void* stream);
/* a = bfloat16(a) in place, kept as FP32 (the training forward pass stores its
 * inputs and hidden activations at the precision the inference path uses). */
int np_net_round_bf16(float* a, long n, void* stream);
/* out = the 7-point stencil of eqn:Laplacian3D without the 1/dx^2 factor (sum
 * of the six face neighbours minus six times the centre), zero outside the
 * box, on one-channel [batch][z][y][x] FP32 arrays (in != out).  The
 * stencil is symmetric, so it is also its own adjoint (the backward pass of
 * the residual training objective). */
int np_net_lap7(const float* in, int batch, int nz, int ny, int nx, float* out, void* stream);

/* Frees every library allocation of the handle.  NULL-safe. */
void nested_poisson_destroy(np_solver* s);

/* Static text of an NP_* code. */
const char* nested_poisson_strerror(int code);
/* Message of the last failure on `s`; with s == NULL, of the last failed
 * nested_poisson_plan or nested_poisson_create on the calling thread. */
const char* nested_poisson_last_error(const np_solver* s);

#ifdef __cplusplus
}
#endif

#endif /* NESTED_POISSON_H */

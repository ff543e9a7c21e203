// Internal declarations of the nested-grid multigrid library (gfx950).
//
// Storage: every grid (a nested level's padded array, or one multigrid level)
// is a box of nx x ny x nz points (nz = 1 in 2-D) in "colour-split" form: the
// red points (even sum of 0-based active indices) and the black points are
// stored in two separate arrays, each holding hx = (nx+1)/2 points per row:
//     value(pi, pj, pk) = a[c * cs + pk * ps + pj * hx + (pi >> 1)],
//     c = (pi + pj + pk + dim) & 1          (0 = red),
// with pi, pj, pk padded indices (0 = ghost / outer buffer layer).  A
// red-black half sweep then reads one colour and writes the other with unit
// stride, so one full sweep streams each array once.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstddef>
#include <cstdint>

namespace np {

struct SGrid {
    int nx;     // padded points along x
    int ny;     // padded points along y
    int nz;     // padded points along z (1 in 2-D)
    int hx;     // compact points per row and colour
    size_t ps;  // elements per plane of one colour: ny rows of hx, rounded up to a
                // multiple of 128 in 3-D so that every plane starts 256-byte aligned
    size_t cs;  // elements per colour array (nz planes)
    // a batch of nb patches with identical grids (the multigrid kernels launch
    // one grid row per patch, blockIdx.y): patch b's array starts b * bs
    // elements after patch 0's, and act (device array, may be null) flags the
    // patches still iterating; nb = 1, bs = 0, act = null for a single grid
    int nb;
    size_t bs;
    const int* act;
};

inline SGrid make_grid(int dim, int nx, int ny, int nz)
{
    SGrid g;
    g.nx = nx;
    g.ny = ny;
    g.nz = dim == 3 ? nz : 1;
    g.hx = (nx + 1) / 2;
    g.ps = (size_t)g.hx * ny;
    if (dim == 3) g.ps = (g.ps + 127) / 128 * 128;
    g.cs = g.ps * g.nz;
    g.nb = 1;
    g.bs = 0;
    g.act = nullptr;
    return g;
}

// the same grid over a batch of nb patches whose arrays lie 2 cs apart
inline SGrid batched(SGrid g, int nb, const int* act)
{
    g.nb = nb;
    g.bs = nb > 1 ? 2 * g.cs : 0;
    g.act = nb > 1 ? act : nullptr;
    return g;
}

// a grid of n points along every axis
inline SGrid make_grid(int dim, int n) { return make_grid(dim, n, n, n); }

// padded points per axis as an array (x, y, z)
inline void grid_extent(const SGrid& g, int* q)
{
    q[0] = g.nx;
    q[1] = g.ny;
    q[2] = g.nz;
}

// Right-ghost rule of a multigrid level L >= 1 (Sec. 2.4), one per axis:
// xn1[a] = 1 when the last active centre along axis a sits at x_MG = 1, else
// the ghost is coef[a] times the last active value.
struct Rule3 {
    int xn1[3];
    double coef[3];
};

// message returned by nested_poisson_last_error(NULL) on the calling thread
void set_last_error(const char* msg);

// ------------------------------------------------------------------ launches
// All launches are asynchronous on `st`.  Grids and sizes are checked by the
// caller (the runtime) before any launch.

// FP64 level operators (nested-level arrays, multigrid level 0)
// fmax: device slot, zeroed by the caller, that receives the bit pattern of
// max |f| over the level (atomic maximum)
void launch_level0_init(int dim, hipStream_t st, SGrid g, const double* rho0, const double* phi_outer,
                        double fourpiG, double* phi, double* f, unsigned long long* fmax);
// fmax (may be null): device slot, zeroed by the caller, that receives the bit
// pattern of max |f| over the level (atomic maximum)
// (gf is the fine level's padded grid: nf_a = gf.n_a - 4 cells per axis)
void launch_interface_fill(int dim, hipStream_t st, SGrid gc, const double* phic, const double* fc, SGrid gf,
                           int offx, int offy, int offz, const double* rho, double fourpiG, double* phif,
                           double* ff, unsigned long long* fmax);
// forces on Omega (g.n_a - 4 cells per axis; arrays n_z x n_y x n_x)
void launch_forces(int dim, hipStream_t st, SGrid g, double dx, const double* phi, double* fx, double* fy,
                   double* fz);
void launch_force_delta(int dim, hipStream_t st, SGrid g, double dx, const double* phi, double* F,
                        unsigned long long* maxbits);
void launch_export(int dim, hipStream_t st, SGrid g, const double* a, double* out);

// norms over the active points 1..nx-2 (mode 0: |f - lap u|, 1: |f|, 2: |f - lap u| with
// the active part of u taken as zero); result is max of the bit patterns of |value|
void launch_norm(int dim, hipStream_t st, SGrid g, const double* u, const double* f, double inv_h2, int mode,
                 unsigned long long* maxbits);
void launch_set_u64(hipStream_t st, unsigned long long* p, int count, unsigned long long v);
// 3-D: max over boxes of 4^3 active points of |mean of f - lap u| (the residual
// restricted twice), as a bit pattern into maxbits (atomic maximum)
void launch_box_resid_norm3(hipStream_t st, SGrid g, const double* u, const double* f, double inv_h2,
                            unsigned long long* maxbits);

// multigrid operators, templated on the storage type (double, float; __half
// only on multigrid level 0 of the FP16-storage defect correction)
// fine != 0: the nested-level arrays (multigrid level 0, ghost layer in
// memory); fine == 0: a multigrid level L >= 1 whose ghost values follow the
// rule of each axis where they are read
template <typename T>
void launch_half_sweep(int dim, hipStream_t st, SGrid g, T* u, const T* f, int colour, double h2, int fine,
                       const Rule3& rule);
// Black half sweep of a 3-D multigrid level 0 (even hx, 2- or 4-byte storage)
// whose red points hold the red half sweep from zero, (0 - h2 f) / 6, unstored:
// the red values are formed from f (and stored into u with store_red)
template <typename T>
void launch_half_sweep_seeded(hipStream_t st, SGrid g, T* u, const T* f, double h2, int store_red);
// One red-black sweep of a 3-D multigrid level 0 (ghost layer in memory) from
// P into Q (Q's ghost layer must equal P's; P is not written).  mode bit 0:
// max |f - lap P| over P's red points into maxbits; bit 1: max |f - lap Q| over
// Q's black points (atomic maxima of the bit patterns; slot zeroed by the
// caller).  rev: order of the z-chunks (cache reuse only)
constexpr int kSweepResIn = 1, kSweepResOut = 2;
template <typename T>
void launch_full_sweep(hipStream_t st, SGrid g, const T* P, T* Q, const T* f, double h2, double inv_h2, int mode,
                       int rev, unsigned long long* maxbits);
// wavefronts one launch_full_sweep on grid g starts
long full_sweep_waves(const SGrid& g);
// fine grid of type TF, coarse of type TC; the coarse right-hand side is
// multiplied by out_scale; rule != 0: the fine grid is a level L >= 1.  The
// coarse correction is cleared, or with seed_h2 > 0 (the coarse level's h^2)
// set to the result of its first red half sweep from zero, which the caller
// then does not launch
template <typename TF, typename TC>
void launch_resid_restrict(int dim, hipStream_t st, SGrid gf, const TF* u, const TF* f, double inv_h2, double out_scale,
                           SGrid gc, TC* fc, TC* ec, int rule, const Rule3& fine_rule, double seed_h2);
// Black half sweep of a 3-D multigrid level 0 in 2-byte storage followed by
// the residual restriction of launch_resid_restrict (FP32 coarse level, fixed
// ghost layer), in one pass, with the same results.  seed != 0: the red points
// hold the red half sweep from zero, unstored; the red values are formed from f
// and stored (as launch_half_sweep_seeded with store_red).  Applies where
// black_restrict_fits: N_fine = 2 N_coarse along every axis, even hx
bool black_restrict_fits(const SGrid& gf, const SGrid& gc);
void launch_black_restrict(hipStream_t st, SGrid gf, __half* u, const __half* f, double h2, double inv_h2,
                           double out_scale, SGrid gc, float* fc, float* ec, double seed_h2, int seed);
// black_only != 0 corrects only the black points; coarse_rule: the coarse level's rule
template <typename TC, typename TF>
void launch_prolong_add(int dim, hipStream_t st, SGrid gc, const TC* ec, SGrid gf, TF* u, int black_only,
                        const Rule3& coarse_rule);

// coarse tail: levels Lt .. Lt+nlev-1 of one V-cycle (active points N[a][axis],
// spacing h[a], rule[a]; the last level has one point along some axis) in one
// workgroup with the levels in LDS; reads f and writes the correction u of
// level Lt (grid g0).  Returns -1 without launching when the levels do not fit
// (coarse_tail_lds_bytes).
constexpr int kTailMaxLevels = 8;
constexpr size_t kTailLdsBytes = 64 * 1024;
size_t coarse_tail_lds_bytes(int dim, const int (*N)[3], int nlev, size_t esz);
template <typename T>
int launch_coarse_tail(int dim, hipStream_t st, int nlev, const int (*N)[3], const double* h, const Rule3* rule,
                       int n_pre, int n_post, SGrid g0, const T* f0, T* u0);

// defect correction, one fused outer pass: phi_out = phi_in + factor * e_in
// (no update and no write of phi_out when e_in is null), r = (f - lap phi_out)
// * rscale in low precision (+ its FP64 max norm into maxbits), and the next
// correction e_out (not written when null): zero, or with first_red the first
// red half sweep from zero
template <typename TL>
void launch_dc_outer(int dim, hipStream_t st, SGrid g, const double* phi_in, const TL* e_in, double factor,
                     double* phi_out, const double* f, double inv_h2, double rscale, TL* r, TL* e_out, int first_red,
                     unsigned long long* maxbits);
// r = (TL)(r32 * rscale) on the active points (r32: f - lap phi in FP32 from a
// pass of launch_dc_outer<float> with rscale 1), and the next correction's start
// into e_out (may be null) as launch_dc_outer writes it.  In 3-D the whole
// arrays are scaled: r32 must be zero at every point that is not active
template <typename TL>
void launch_dc_scale(int dim, hipStream_t st, SGrid g, const float* r32, double rscale, TL* r, TL* e_out,
                     int first_red);
// ghost layer of a nested-level array copied from src to dst
void launch_copy_ghosts(int dim, hipStream_t st, SGrid g, const double* src, double* dst);
// dst(p) = src(p + shift) for the points p of grid gd with lo <= p_a <= hi[a]
// on every axis (padded indices of each grid; the caller keeps p + shift
// inside gs)
void launch_copy_box(int dim, hipStream_t st, SGrid gs, const double* src, SGrid gd, double* dst, int lo,
                     const int* hi, int shift);

// learned initial guess network (np_net.hip); activations channel-last,
// weights bfloat16 [27][cout][cin]
void net_conv_fwd_f32(hipStream_t st, const float* in, int cin, const uint16_t* w, const float* bias, int cout, int relu,
                      int B, int Z, int Y, int X, float* out);
void net_conv_fwd_bf16(hipStream_t st, const uint16_t* in, int cin, const uint16_t* w, const float* bias, int cout,
                       int relu, int B, int Z, int Y, int X, uint16_t* out);
void net_conv_fwd_bf16_to_f32(hipStream_t st, const uint16_t* in, int cin, const uint16_t* w, const float* bias,
                              int cout, int relu, int B, int Z, int Y, int X, float* out);
// matrix-core inference of a layer (cin, cout) in {(2, 16), (16, 16), (16, 1)}:
// bfloat16 input, bfloat16 output (cout 16) or FP32 output (cout 1)
void net_conv_mfma(hipStream_t st, const uint16_t* in, int cin, const uint16_t* w, const float* bias, int cout, int relu,
                   int B, int Z, int Y, int X, void* out);
void net_conv_bwd_data(hipStream_t st, const float* gout, int cout, const uint16_t* w, int cin, int B, int Z, int Y,
                       int X, float* gin);
size_t net_bwd_weight_workspace(int cin, int cout);
void net_conv_bwd_weight(hipStream_t st, const float* in, int cin, const float* gout, int cout, int B, int Z, int Y,
                         int X, float* gw, float* gb, float* part);
void net_relu_bwd(hipStream_t st, const float* act, float* g, long n);
size_t net_mse_workspace(long n);
void net_mse(hipStream_t st, const float* pred, const float* target, const float* mask, long n, float count,
             float* grad, float* part, float* loss);
void net_adam(hipStream_t st, float* w, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
              float eps, int step, uint16_t* wb);
void net_to_bf16(hipStream_t st, const float* a, uint16_t* b, long n);
// solver glue on a nested level's Gamma ((n_x+2) x (n_y+2) x (n_z+2) points)
void net_features_bf16(hipStream_t st, SGrid g, const double* phi, const double* f, double inv_fnorm, double inv_h2,
                       uint16_t* x);
void net_features_f32(hipStream_t st, SGrid g, const double* phi, const double* f, double inv_fnorm, double inv_h2,
                      float* x);
void net_apply(hipStream_t st, SGrid g, double* phi, const float* out, double s);
void net_target(hipStream_t st, SGrid g, const double* pa, const double* pb, double inv_s, float* t);

}  // namespace np

// HIP kernels of the nested-grid multigrid solver for gfx950 (MI355X).
//
// Every kernel is a bandwidth-bound stencil sweep over colour-split storage
// (see np_internal.h).  One thread handles one compact (h, pj, pk) position;
// consecutive threads take consecutive h, so each wavefront of 64 lanes reads
// and writes 64 consecutive elements of a colour array.
#include "np_internal.h"

namespace np {

namespace {

constexpr int kBlock = 256;

__host__ __device__ inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Workgroups are dealt to the 8 XCDs of the chip round-robin (workgroup b runs
// on XCD b % 8).  Renumber them so that XCD x processes one contiguous run of
// logical blocks: stencil neighbours (rows above/below, planes in front/behind)
// are then fetched into the same XCD's L2 instead of eight different ones.
__device__ __forceinline__ long xcd_block()
{
    long nb = gridDim.x, b = blockIdx.x;
    long q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Strip ordering of a 3-D box of points (x fastest): the y range is cut into
// strips of R rows and logical blocks run over (strip, z, block of the strip
// plane).  With the XCD-contiguous numbering above, every XCD walks whole
// strips plane by plane, so the planes a stencil revisits (z-neighbours) and
// the rows it shares (y-neighbours) are still in that XCD's L2.
struct Strip {
    int nxa, nya, nza;  // box extents
    int R;              // rows per strip
    int B;              // blocks per strip plane
};

inline Strip make_strip(int nxa, int nya, int nza, int nstrip)
{
    Strip s;
    s.nxa = nxa;
    s.nya = nya;
    s.nza = nza;
    s.R = (nya + nstrip - 1) / nstrip;
    s.B = (int)(((long)s.R * nxa + kBlock - 1) / kBlock);
    return s;
}

inline long strip_blocks(const Strip& s)
{
    long nstrip = (s.nya + s.R - 1) / s.R;
    return nstrip * s.nza * s.B;
}

__device__ __forceinline__ bool strip_point(const Strip& s, int& x, int& y, int& z)
{
    const long lb = xcd_block();
    const long per = (long)s.nza * s.B;
    const int st = (int)(lb / per);
    const long rem = lb - st * per;
    z = (int)(rem / s.B);
    const int blk = (int)(rem - (long)z * s.B);
    const int tin = blk * kBlock + threadIdx.x;
    const int rr = tin / s.nxa;
    x = tin - rr * s.nxa;
    y = st * s.R + rr;
    return rr < s.R && y < s.nya;
}

template <int D>
__device__ __forceinline__ int colour_of(int pi, int pj, int pk)
{
    return (pi + pj + pk + D) & 1;
}

__device__ __forceinline__ size_t row_base(const SGrid& g, int pj, int pk)
{
    return ((size_t)pk * g.nx + pj) * g.hx;
}

template <int D, typename T>
__device__ __forceinline__ T at(const T* __restrict__ a, const SGrid& g, int pi, int pj, int pk)
{
    return a[(size_t)colour_of<D>(pi, pj, pk) * g.cs + row_base(g, pj, pk) + (pi >> 1)];
}

template <int D, typename T>
__device__ __forceinline__ size_t pos(const SGrid& g, int pi, int pj, int pk)
{
    return (size_t)colour_of<D>(pi, pj, pk) * g.cs + row_base(g, pj, pk) + (pi >> 1);
}

// Maximum of non-negative doubles through their bit patterns: the unsigned
// order of the patterns is the numeric order, +inf above every finite value
// and a (positive) NaN above +inf, so NaN and Inf survive the reduction.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ void block_max_to(unsigned long long v, unsigned long long* out)
{
    __shared__ unsigned long long red[kBlock / 64];
    v = wave_max_u64(v);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = red[0];
        for (int w = 1; w < kBlock / 64; w++) m = red[w] > m ? red[w] : m;
        atomicMax(out, m);
    }
}

__device__ __forceinline__ unsigned long long abs_bits(double a)
{
    return (unsigned long long)__double_as_longlong(fabs(a));
}

// ------------------------------------------------------------------ level setup
// Level 0: potential = caller's outer layer on the ring, zero on Gamma^0;
// right-hand side = 4 pi G rho on Gamma^0 (caller gives Omega^0 plus its inner
// layer, (n+2)^d points).
template <int D>
__global__ void __launch_bounds__(kBlock) k_level0_init(SGrid g, const double* __restrict__ rho0,
                                                        const double* __restrict__ phi_outer, double fourpiG,
                                                        double* __restrict__ phi, double* __restrict__ f)
{
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = (long)g.nx * g.nx * g.nz;
    if (t >= total) return;
    int pi = (int)(t % g.nx);
    long r = t / g.nx;
    int pj = (int)(r % g.nx);
    int pk = (int)(r / g.nx);
    int last = g.nx - 1;
    bool ring = pi == 0 || pi == last || pj == 0 || pj == last || (D == 3 && (pk == 0 || pk == last));
    size_t p = pos<D, double>(g, pi, pj, pk);
    if (ring) {
        phi[p] = phi_outer[t];
        f[p] = 0.0;
    } else {
        int m = g.nx - 2;
        size_t ri = D == 3 ? (((size_t)(pk - 1) * m + (pj - 1)) * m + (pi - 1)) : ((size_t)(pj - 1) * m + (pi - 1));
        phi[p] = 0.0;
        f[p] = fourpiG * rho0[ri];
    }
}

// Interpolation weight pair along one axis for fine padded index p of a
// level whose corner sits `off` coarse cells into the coarse patch: the fine
// cell p-2 lies in coarse cell off + floor((p-2)/2) (padded q = that + 2);
// the second coarse point is on the side of the fine centre.
__device__ __forceinline__ void fine_to_coarse(int p, int off, int& q, int& s)
{
    int fine = p - 2;
    q = off + 2 + (fine >> 1);  // arithmetic shift = floor for negatives
    s = (fine & 1) ? 1 : -1;
}

template <int D>
__device__ __forceinline__ double interp_tensor(const double* __restrict__ c, const SGrid& gc, int qi, int qj, int qk,
                                                int si, int sj, int sk)
{
    const double w0 = 0.75, w1 = 0.25;
    double y0 = w0 * at<D>(c, gc, qi, qj, qk) + w1 * at<D>(c, gc, qi + si, qj, qk);
    double y1 = w0 * at<D>(c, gc, qi, qj + sj, qk) + w1 * at<D>(c, gc, qi + si, qj + sj, qk);
    double z0 = w0 * y0 + w1 * y1;
    if (D == 2) return z0;
    double y2 = w0 * at<D>(c, gc, qi, qj, qk + sk) + w1 * at<D>(c, gc, qi + si, qj, qk + sk);
    double y3 = w0 * at<D>(c, gc, qi, qj + sj, qk + sk) + w1 * at<D>(c, gc, qi + si, qj + sj, qk + sk);
    double z1 = w0 * y2 + w1 * y3;
    return w0 * z0 + w1 * z1;
}

// Level l >= 1 from level l-1: potential everywhere (outer layer = Dirichlet
// data, rest = initial guess) and right-hand side of the inner layer
// interpolated; Omega^l takes 4 pi G rho from the caller (n^d points).
template <int D>
__global__ void __launch_bounds__(kBlock) k_interface_fill(SGrid gc, const double* __restrict__ phic,
                                                           const double* __restrict__ fc, SGrid gf, int nf, int offx,
                                                           int offy, int offz, const double* __restrict__ rho,
                                                           double fourpiG, double* __restrict__ phif,
                                                           double* __restrict__ ff)
{
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = (long)gf.nx * gf.nx * gf.nz;
    if (t >= total) return;
    int pi = (int)(t % gf.nx);
    long r = t / gf.nx;
    int pj = (int)(r % gf.nx);
    int pk = (int)(r / gf.nx);
    int qi, qj, qk = 0, si, sj, sk = 1;
    fine_to_coarse(pi, offx, qi, si);
    fine_to_coarse(pj, offy, qj, sj);
    if (D == 3) fine_to_coarse(pk, offz, qk, sk);
    size_t p = pos<D, double>(gf, pi, pj, pk);
    phif[p] = interp_tensor<D>(phic, gc, qi, qj, qk, si, sj, sk);
    int last = gf.nx - 1;
    bool outer = pi == 0 || pi == last || pj == 0 || pj == last || (D == 3 && (pk == 0 || pk == last));
    bool omega = pi >= 2 && pi <= nf + 1 && pj >= 2 && pj <= nf + 1 && (D == 2 || (pk >= 2 && pk <= nf + 1));
    double v;
    if (outer) {
        v = 0.0;
    } else if (omega) {
        size_t ri = D == 3 ? (((size_t)(pk - 2) * nf + (pj - 2)) * nf + (pi - 2)) : ((size_t)(pj - 2) * nf + (pi - 2));
        v = fourpiG * rho[ri];
    } else {
        v = interp_tensor<D>(fc, gc, qi, qj, qk, si, sj, sk);
    }
    ff[p] = v;
}

// ------------------------------------------------------------------ forces
// F = -grad Phi with the fourth-order central difference:
// dPhi/dx = [8 (Phi_{i+1} - Phi_{i-1}) - (Phi_{i+2} - Phi_{i-2})] / (12 dx).
template <int D>
__device__ __forceinline__ double d4(const double* __restrict__ phi, const SGrid& g, int pi, int pj, int pk, int ax,
                                     double m12dx)
{
    int e[3] = {0, 0, 0};
    e[ax] = 1;
    double p1 = at<D>(phi, g, pi + e[0], pj + e[1], pk + e[2]);
    double m1 = at<D>(phi, g, pi - e[0], pj - e[1], pk - e[2]);
    double p2 = at<D>(phi, g, pi + 2 * e[0], pj + 2 * e[1], pk + 2 * e[2]);
    double m2 = at<D>(phi, g, pi - 2 * e[0], pj - 2 * e[1], pk - 2 * e[2]);
    return (8.0 * (p1 - m1) - (p2 - m2)) * m12dx;
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_forces(SGrid g, int n, double m12dx, const double* __restrict__ phi,
                                                   double* __restrict__ fx, double* __restrict__ fy,
                                                   double* __restrict__ fz, Strip sp)
{
    int i, j, k = 0;
    long t;
    if (D == 3) {
        if (!strip_point(sp, i, j, k)) return;
        t = ((long)k * n + j) * n + i;
    } else {
        t = xcd_block() * kBlock + threadIdx.x;
        if (t >= (long)n * n) return;
        i = (int)(t % n);
        j = (int)(t / n);
    }
    int pi = i + 2, pj = j + 2, pk = D == 3 ? k + 2 : 0;
    fx[t] = d4<D>(phi, g, pi, pj, pk, 0, m12dx);
    fy[t] = d4<D>(phi, g, pi, pj, pk, 1, m12dx);
    if (D == 3) fz[t] = d4<D>(phi, g, pi, pj, pk, 2, m12dx);
}

// Forces into F (d arrays of n^d) and the maximum change against the values
// F held before (the stop rule of Sec. 3.1).
template <int D>
__global__ void __launch_bounds__(kBlock) k_force_delta(SGrid g, int n, double m12dx, const double* __restrict__ phi,
                                                        double* __restrict__ F, unsigned long long* maxbits)
{
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = D == 3 ? (long)n * n * n : (long)n * n;
    unsigned long long m = 0;
    if (t < total) {
        int i = (int)(t % n);
        long r = t / n;
        int j = (int)(r % n);
        int k = (int)(r / n);
        int pi = i + 2, pj = j + 2, pk = D == 3 ? k + 2 : 0;
        for (int ax = 0; ax < D; ax++) {
            double v = d4<D>(phi, g, pi, pj, pk, ax, m12dx);
            double old = F[ax * total + t];
            F[ax * total + t] = v;
            unsigned long long b = abs_bits(v - old);
            m = b > m ? b : m;
        }
    }
    block_max_to(m, maxbits);
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_export(SGrid g, const double* __restrict__ a, double* __restrict__ out)
{
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = (long)g.nx * g.nx * g.nz;
    if (t >= total) return;
    int pi = (int)(t % g.nx);
    long r = t / g.nx;
    int pj = (int)(r % g.nx);
    int pk = (int)(r / g.nx);
    out[t] = at<D>(a, g, pi, pj, pk);
}

// ------------------------------------------------------------------ norms
// Grid-stride loop over a bounded grid so that only a few thousand blocks
// meet in the final atomic maximum.
template <int D>
__global__ void __launch_bounds__(kBlock) k_norm(SGrid g, const double* __restrict__ u, const double* __restrict__ f,
                                                 double inv_h2, int mode, unsigned long long* maxbits)
{
    int m = g.nx - 2;
    long total = (long)g.hx * m * (D == 3 ? m : 1);
    long stride = (long)gridDim.x * kBlock;
    size_t ny = (size_t)g.hx, nz = (size_t)g.nx * g.hx;
    unsigned long long best = 0;
    for (long t = xcd_block() * kBlock + threadIdx.x; t < total; t += stride) {
        int h = (int)(t % g.hx);
        long r = t / g.hx;
        int pj = 1 + (int)(r % m);
        int pk = D == 3 ? 1 + (int)(r / m) : 0;
        size_t row = row_base(g, pj, pk);
        for (int c = 0; c < 2; c++) {
            int pi = 2 * h + ((c + pj + pk + D) & 1);
            if (pi < 1 || pi > g.nx - 2) continue;
            const double* o = u + (size_t)(c ^ 1) * g.cs;
            size_t self = (size_t)c * g.cs + row + h;
            double val;
            if (mode == 1) {
                val = f[self];
            } else if (mode == 2) {
                // the active part of u taken as zero: only ghost-layer neighbours remain
                double s = 0.0;
                if (pi - 1 == 0) s += o[row + ((pi - 1) >> 1)];
                if (pi + 1 == g.nx - 1) s += o[row + ((pi + 1) >> 1)];
                if (pj - 1 == 0) s += o[row - ny + h];
                if (pj + 1 == g.nx - 1) s += o[row + ny + h];
                if (D == 3 && pk - 1 == 0) s += o[row - nz + h];
                if (D == 3 && pk + 1 == g.nx - 1) s += o[row + nz + h];
                val = f[self] - s * inv_h2;
            } else {
                double s = o[row + ((pi - 1) >> 1)];
                s = s + o[row + ((pi + 1) >> 1)];
                s = s + o[row - ny + h];
                s = s + o[row + ny + h];
                if (D == 3) {
                    s = s + o[row - nz + h];
                    s = s + o[row + nz + h];
                }
                val = f[self] - (s - (2.0 * D) * u[self]) * inv_h2;
            }
            unsigned long long b = abs_bits(val);
            best = b > best ? b : best;
        }
    }
    block_max_to(best, maxbits);
}

// 3-D residual max-norm on a nested-level array, marching along z like
// k_smooth_fine3: a thread owns compact (h, pj), treats the red and the black
// point of that position on every plane of its chunk, and keeps both colours'
// values at pk-1, pk, pk+1 of its column in registers.
constexpr int kNormChunk = 8;

__global__ void __launch_bounds__(kBlock) k_resid_norm3(SGrid g, const double* __restrict__ u,
                                                        const double* __restrict__ f, double inv_h2, int pblocks,
                                                        unsigned long long* maxbits)
{
    const int m = g.nx - 2;
    const long lb = xcd_block();
    const int zc = (int)(lb / pblocks);
    const long t = (lb - (long)zc * pblocks) * kBlock + threadIdx.x;
    unsigned long long best = 0;
    if (t < (long)g.hx * m) {
        const int h = (int)(t % g.hx);
        const int pj = 1 + (int)(t / g.hx);
        const int k0 = 1 + zc * kNormChunk;
        const int k1 = min(k0 + kNormChunk - 1, m);
        const size_t plane = (size_t)g.nx * g.hx;
        const size_t col = (size_t)pj * g.hx + h;
        const double* __restrict__ a[2] = {u, u + g.cs};
        double below[2], cur[2];
        for (int c = 0; c < 2; c++) {
            below[c] = a[c][(size_t)(k0 - 1) * plane + col];
            cur[c] = a[c][(size_t)k0 * plane + col];
        }
        for (int pk = k0; pk <= k1; pk++) {
            const size_t here = (size_t)pk * plane + col;
            double above[2] = {a[0][here + plane], a[1][here + plane]};
            for (int c = 0; c < 2; c++) {
                const int o = c ^ 1;
                const int par = (c + pj + pk + 3) & 1;
                const int pi = 2 * h + par;
                if (pi < 1 || pi > g.nx - 2) continue;
                double xm = par ? cur[o] : a[o][here - 1];
                double xp = par ? a[o][here + 1] : cur[o];
                double s = xm + xp;
                s = s + a[o][here - g.hx];
                s = s + a[o][here + g.hx];
                s = s + below[o];
                s = s + above[o];
                double r = f[(size_t)c * g.cs + here] - (s - 6.0 * cur[c]) * inv_h2;
                unsigned long long b = abs_bits(r);
                best = b > best ? b : best;
            }
            for (int c = 0; c < 2; c++) {
                below[c] = cur[c];
                cur[c] = above[c];
            }
        }
    }
    block_max_to(best, maxbits);
}

__global__ void k_set_u64(unsigned long long* p, int count, unsigned long long v)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = v;
}

// ------------------------------------------------------------------ multigrid
template <typename T>
struct Compute { using type = T; };
template <>
struct Compute<__half> { using type = float; };

// Red-black Gauss-Seidel half sweep: u_c = (sum of the 2d neighbours - h^2 f_c) / (2d)
// over the active points of one colour; the neighbours are all of the other colour.
// k_smooth_fine runs it on the nested-level arrays (multigrid level 0, whose
// ghost layer is the fixed outer buffer), k_half_sweep on the coarse levels.
template <int D, typename T>
__device__ __forceinline__ void half_sweep_body(T* __restrict__ u, const T* __restrict__ f, SGrid g,
                                                       int colour, typename Compute<T>::type h2,
                                                       typename Compute<T>::type inv2d)
{
    using C = typename Compute<T>::type;
    long t = xcd_block() * kBlock + threadIdx.x;
    int m = g.nx - 2;
    long total = (long)g.hx * m * (D == 3 ? m : 1);
    if (t >= total) return;
    int h = (int)(t % g.hx);
    long r = t / g.hx;
    int pj = 1 + (int)(r % m);
    int pk = D == 3 ? 1 + (int)(r / m) : 0;
    int pi = 2 * h + ((colour + pj + pk + D) & 1);
    if (pi < 1 || pi > g.nx - 2) return;
    const T* __restrict__ o = u + (size_t)(colour ^ 1) * g.cs;
    size_t row = row_base(g, pj, pk);
    size_t ny = (size_t)g.hx, nz = (size_t)g.nx * g.hx;
    C s = (C)o[row + ((pi - 1) >> 1)];
    s = s + (C)o[row + ((pi + 1) >> 1)];
    s = s + (C)o[row - ny + h];
    s = s + (C)o[row + ny + h];
    if (D == 3) {
        s = s + (C)o[row - nz + h];
        s = s + (C)o[row + nz + h];
    }
    size_t self = (size_t)colour * g.cs + row + h;
    u[self] = (T)((s - h2 * (C)f[self]) * inv2d);
}


template <int D, typename T>
__global__ void __launch_bounds__(kBlock) k_smooth_fine(T* __restrict__ u, const T* __restrict__ f, SGrid g, int colour,
                                                        typename Compute<T>::type h2, typename Compute<T>::type inv2d)
{
    half_sweep_body<D, T>(u, f, g, colour, h2, inv2d);
}

// 3-D level-0 half sweep marching along z.  A thread owns one compact (h, pj)
// position and walks kZChunk planes, keeping the other colour's values at
// planes pk-1, pk, pk+1 of its own column in registers: each value of the
// other colour is loaded once per chunk as the "plane above" and reused as the
// centre's x-neighbour and the next planes' z-neighbours.  Logical blocks run
// over the flattened (pj, h) plane fastest, so the blocks resident on one XCD
// cover adjacent rows of the same planes and the y-neighbour rows come from
// its L2.
constexpr int kZChunk = 8;

template <typename T, int TAG>
__global__ void __launch_bounds__(kBlock) k_smooth_zmarch3(T* __restrict__ u, const T* __restrict__ f, SGrid g, int colour,
                                                           typename Compute<T>::type h2,
                                                           typename Compute<T>::type inv2d, int pblocks)
{
    using C = typename Compute<T>::type;
    const int m = g.nx - 2;
    const long lb = xcd_block();
    const int zc = (int)(lb / pblocks);
    const long t = (lb - (long)zc * pblocks) * kBlock + threadIdx.x;
    if (t >= (long)g.hx * m) return;
    const int h = (int)(t % g.hx);
    const int pj = 1 + (int)(t / g.hx);
    const int k0 = 1 + zc * kZChunk;
    const int k1 = min(k0 + kZChunk - 1, m);
    const size_t plane = (size_t)g.nx * g.hx;
    const size_t col = (size_t)pj * g.hx + h;  // offset of (h, pj) inside a plane
    const T* __restrict__ o = u + (size_t)(colour ^ 1) * g.cs;
    T* __restrict__ uc = u + (size_t)colour * g.cs;
    const T* __restrict__ fc = f + (size_t)colour * g.cs;
    C below = (C)o[(size_t)(k0 - 1) * plane + col];
    C cur = (C)o[(size_t)k0 * plane + col];
    int pk = k0;
    // groups of 4 planes: every load of the group is issued before the first
    // update so that each wave keeps ~20 loads in flight.  Loads at inactive
    // (ghost) positions stay inside the arrays: h-1 / h+1 fall in the
    // neighbouring row of the same plane and f covers the whole padded grid.
    for (; pk + 3 <= k1; pk += 4) {
        C ab[4], xo[4], ym[4], yp[4], fv[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const size_t here = (size_t)(pk + q) * plane + col;
            const int par = (colour + pj + pk + q + 3) & 1;
            ab[q] = (C)o[here + plane];
            xo[q] = (C)o[par ? here + 1 : here - 1];
            ym[q] = (C)o[here - g.hx];
            yp[q] = (C)o[here + g.hx];
            fv[q] = (C)fc[here];
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const size_t here = (size_t)(pk + q) * plane + col;
            const int par = (colour + pj + pk + q + 3) & 1;
            const int pi = 2 * h + par;
            if (pi >= 1 && pi <= g.nx - 2) {
                C xm = par ? cur : xo[q];
                C xp = par ? xo[q] : cur;
                C s = xm + xp;
                s = s + ym[q];
                s = s + yp[q];
                s = s + below;
                s = s + ab[q];
                uc[here] = (T)((s - h2 * fv[q]) * inv2d);
            }
            below = cur;
            cur = ab[q];
        }
    }
    for (; pk <= k1; pk++) {
        const size_t here = (size_t)pk * plane + col;
        C above = (C)o[here + plane];
        const int par = (colour + pj + pk + 3) & 1;  // pi = 2h + par
        const int pi = 2 * h + par;
        if (pi >= 1 && pi <= g.nx - 2) {
            // x-neighbours pi-1, pi+1: compact h-1 and h (par 0) or h and h+1 (par 1)
            C xm = par ? cur : (C)o[here - 1];
            C xp = par ? (C)o[here + 1] : cur;
            C s = xm + xp;
            s = s + (C)o[here - g.hx];
            s = s + (C)o[here + g.hx];
            s = s + below;
            s = s + above;
            uc[here] = (T)((s - h2 * (C)fc[here]) * inv2d);
        }
        below = cur;
        cur = above;
    }
}

template <int D, typename T>
__global__ void __launch_bounds__(kBlock) k_half_sweep(T* __restrict__ u, const T* __restrict__ f, SGrid g, int colour,
                                                       typename Compute<T>::type h2, typename Compute<T>::type inv2d)
{
    half_sweep_body<D, T>(u, f, g, colour, h2, inv2d);
}

// Paired form of the level-0 z-march for 2- and 4-byte storage: a thread owns
// the two compact points h0 = 2 hp and h0 + 1 of a row and moves them with
// one 2-element load or store; the extra x-neighbour (h0 - 1 or h0 + 2) is a
// single load.  Same arithmetic, in the same order, as k_smooth_zmarch3.
// Requires an even row length hx (so pairs never straddle rows and stay
// aligned).
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
    T a, b;
};

template <typename T>
__global__ void __launch_bounds__(kBlock) k_smooth_zmarch3_pair(T* __restrict__ u, const T* __restrict__ f, SGrid g,
                                                                int colour, typename Compute<T>::type h2,
                                                                typename Compute<T>::type inv2d, int pblocks)
{
    using C = typename Compute<T>::type;
    const int m = g.nx - 2;
    const int hp_n = g.hx >> 1;
    const long lb = xcd_block();
    const int zc = (int)(lb / pblocks);
    const long t = (lb - (long)zc * pblocks) * kBlock + threadIdx.x;
    if (t >= (long)hp_n * m) return;
    const int h0 = 2 * (int)(t % hp_n);
    const int pj = 1 + (int)(t / hp_n);
    const int k0 = 1 + zc * kZChunk;
    const int k1 = min(k0 + kZChunk - 1, m);
    const size_t plane = (size_t)g.nx * g.hx;
    const size_t col = (size_t)pj * g.hx + h0;
    const T* __restrict__ o = u + (size_t)(colour ^ 1) * g.cs;
    T* __restrict__ uc = u + (size_t)colour * g.cs;
    const T* __restrict__ fc = f + (size_t)colour * g.cs;
    Pair<T> below = *(const Pair<T>*)(o + (size_t)(k0 - 1) * plane + col);
    Pair<T> cur = *(const Pair<T>*)(o + (size_t)k0 * plane + col);
    for (int pk = k0; pk <= k1; pk++) {
        const size_t here = (size_t)pk * plane + col;
        const Pair<T> above = *(const Pair<T>*)(o + here + plane);
        const Pair<T> ym = *(const Pair<T>*)(o + here - g.hx);
        const Pair<T> yp = *(const Pair<T>*)(o + here + g.hx);
        const Pair<T> fv = *(const Pair<T>*)(fc + here);
        const int par = (colour + pj + pk + 3) & 1;
        // the extra x-neighbour stays inside the plane (neighbouring row at the row ends)
        const C ex = (C)o[par ? here + 2 : here - 1];
        C xm0, xp0, xm1, xp1;
        if (par) {
            xm0 = (C)cur.a;
            xp0 = (C)cur.b;
            xm1 = (C)cur.b;
            xp1 = ex;
        } else {
            xm0 = ex;
            xp0 = (C)cur.a;
            xm1 = (C)cur.a;
            xp1 = (C)cur.b;
        }
        C s0 = xm0 + xp0;
        s0 = s0 + (C)ym.a;
        s0 = s0 + (C)yp.a;
        s0 = s0 + (C)below.a;
        s0 = s0 + (C)above.a;
        C s1 = xm1 + xp1;
        s1 = s1 + (C)ym.b;
        s1 = s1 + (C)yp.b;
        s1 = s1 + (C)below.b;
        s1 = s1 + (C)above.b;
        Pair<T> r;
        r.a = (T)((s0 - h2 * (C)fv.a) * inv2d);
        r.b = (T)((s1 - h2 * (C)fv.b) * inv2d);
        const int pi0 = 2 * h0 + par;
        const bool a0 = pi0 >= 1, a1 = pi0 + 2 <= g.nx - 2;
        if (a0 && a1) {
            *(Pair<T>*)(uc + here) = r;
        } else {
            if (a0) uc[here] = r.a;
            if (a1) uc[here + 1] = r.b;
        }
        below = cur;
        cur = above;
    }
}

// Ghost layer of a multigrid level L >= 1 (Sec. 2.4): left e_0 = -e_1; right
// -e_{N-1} when x_N = 1, else coef * e_N; edges and corners compose the rule
// of each axis they are ghosts on, applied in the order x, y, z.
// blockIdx.y = face (2 per axis).
template <int D, typename T>
__global__ void __launch_bounds__(kBlock) k_ghost_fill(T* __restrict__ u, SGrid g, int xn_is_one,
                                                       typename Compute<T>::type coef)
{
    using C = typename Compute<T>::type;
    int Q = g.nx, N = Q - 2;
    int t = blockIdx.x * kBlock + threadIdx.x;
    int per = D == 3 ? Q * Q : Q;
    if (t >= per) return;
    int face = blockIdx.y;
    int axis = face >> 1, side = face & 1;
    int p[3] = {0, 0, 0};
    int a = t % Q, b = t / Q;
    if (D == 3) {
        p[axis] = side ? Q - 1 : 0;
        p[(axis + 1) % 3] = a;
        p[(axis + 2) % 3] = b;
    } else {
        p[axis] = side ? Q - 1 : 0;
        p[1 - axis] = a;
    }
    int src[3] = {p[0], p[1], p[2]};
    C fac[3] = {1, 1, 1};
    bool scaled[3] = {false, false, false};
    for (int ax = 0; ax < D; ax++) {
        if (src[ax] == 0) {
            src[ax] = 1;
            fac[ax] = -1;
            scaled[ax] = true;
        } else if (src[ax] == Q - 1) {
            if (xn_is_one) {
                src[ax] = N - 1;
                fac[ax] = -1;
            } else {
                src[ax] = N;
                fac[ax] = coef;
            }
            scaled[ax] = true;
        }
    }
    C v = (C)at<D>(u, g, src[0], src[1], src[2]);
    for (int ax = 0; ax < D; ax++)
        if (scaled[ax]) v = fac[ax] * v;
    u[pos<D, T>(g, p[0], p[1], p[2])] = (T)v;
}

// Residual r = f - lap(u) on the 2^d children of each coarse active point and
// their mean (eqn:restriction2D/3D) into the coarse right-hand side, times
// out_scale (1 except below a scaled level-0 defect problem); children beyond
// the fine active range count as zero.  Also clears the coarse correction.
// TF: fine storage, TC: coarse storage.
template <int D, typename TF, typename TC>
__global__ void __launch_bounds__(kBlock) k_resid_restrict(const TF* __restrict__ u, const TF* __restrict__ f, SGrid gf,
                                                           typename Compute<TC>::type inv_h2,
                                                           typename Compute<TC>::type out_scale, SGrid gc,
                                                           TC* __restrict__ fc, TC* __restrict__ ec)
{
    using C = typename Compute<TC>::type;
    int Nc = gc.nx - 2, Nf = gf.nx - 2;
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = D == 3 ? (long)Nc * Nc * Nc : (long)Nc * Nc;
    if (t >= total) return;
    int I = 1 + (int)(t % Nc);
    long r = t / Nc;
    int J = 1 + (int)(r % Nc);
    int K = D == 3 ? 1 + (int)(r / Nc) : 0;
    C sum = 0;
    int k0 = D == 3 ? 2 * K - 1 : 0, k1 = D == 3 ? 2 * K : 0;
    for (int k = k0; k <= k1; k++)
        for (int j = 2 * J - 1; j <= 2 * J; j++)
            for (int i = 2 * I - 1; i <= 2 * I; i++) {
                if (i > Nf || j > Nf || (D == 3 && k > Nf)) continue;
                C s = (C)at<D>(u, gf, i - 1, j, k);
                s = s + (C)at<D>(u, gf, i + 1, j, k);
                s = s + (C)at<D>(u, gf, i, j - 1, k);
                s = s + (C)at<D>(u, gf, i, j + 1, k);
                if (D == 3) {
                    s = s + (C)at<D>(u, gf, i, j, k - 1);
                    s = s + (C)at<D>(u, gf, i, j, k + 1);
                }
                C uc = (C)at<D>(u, gf, i, j, k);
                sum += (C)at<D>(f, gf, i, j, k) - (s - (C)(2 * D) * uc) * inv_h2;
            }
    size_t pc = pos<D, TC>(gc, I, J, K);
    fc[pc] = (TC)(sum * ((C)(D == 3 ? 0.125 : 0.25) * out_scale));
    ec[pc] = (TC)0;
}

// u += P(e) on the fine active points (eqn:prolongation2D/3D as the tensor
// product of (3/4, 1/4) along each axis: the coarse parent ceil(p/2) weighs
// 3/4, its neighbour on the side of the fine centre 1/4).  Each thread does
// the red and the black point of one compact position; with black_only the
// red points are left alone (used when a red half sweep that reads only
// black values follows on a grid with a fixed ghost layer).
template <int D, typename TC, typename TF>
__global__ void __launch_bounds__(kBlock) k_prolong_add(const TC* __restrict__ e, SGrid gc, TF* __restrict__ u, SGrid gf,
                                                        int black_only)
{
    using C = typename Compute<TC>::type;
    int m = gf.nx - 2;
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = (long)gf.hx * m * (D == 3 ? m : 1);
    if (t >= total) return;
    int h = (int)(t % gf.hx);
    long r = t / gf.hx;
    int pj = 1 + (int)(r % m);
    int pk = D == 3 ? 1 + (int)(r / m) : 0;
    const C w0 = (C)0.75, w1 = (C)0.25;
    int qj = (pj + 1) >> 1, sj = (pj & 1) ? -1 : 1;
    int qk = D == 3 ? (pk + 1) >> 1 : 0, sk = (pk & 1) ? -1 : 1;
    for (int c = black_only; c < 2; c++) {
        int pi = 2 * h + ((c + pj + pk + D) & 1);
        if (pi < 1 || pi > gf.nx - 2) continue;
        int qi = (pi + 1) >> 1, si = (pi & 1) ? -1 : 1;
        C y0 = w0 * (C)at<D>(e, gc, qi, qj, qk) + w1 * (C)at<D>(e, gc, qi + si, qj, qk);
        C y1 = w0 * (C)at<D>(e, gc, qi, qj + sj, qk) + w1 * (C)at<D>(e, gc, qi + si, qj + sj, qk);
        C v = w0 * y0 + w1 * y1;
        if (D == 3) {
            C y2 = w0 * (C)at<D>(e, gc, qi, qj, qk + sk) + w1 * (C)at<D>(e, gc, qi + si, qj, qk + sk);
            C y3 = w0 * (C)at<D>(e, gc, qi, qj + sj, qk + sk) + w1 * (C)at<D>(e, gc, qi + si, qj + sj, qk + sk);
            v = w0 * v + w1 * (w0 * y2 + w1 * y3);
        }
        size_t p = (size_t)c * gf.cs + row_base(gf, pj, pk) + h;
        u[p] = (TF)((C)u[p] + v);
    }
}

// ------------------------------------------------------------------ defect correction
// Outer FP64 step of the mixed-precision solve: r64 = f - lap(phi) on the
// level-0 active points (same arithmetic as the stop-test norm), its max
// norm, and the scaled low-precision copy r = r64 * rscale; the correction e
// is cleared where the first relaxation reads it (black only when a red half
// sweep comes first, both colours otherwise).
template <int D, typename TL>
__global__ void __launch_bounds__(kBlock) k_dc_residual(SGrid g, const double* __restrict__ phi,
                                                        const double* __restrict__ f, double inv_h2, double rscale,
                                                        TL* __restrict__ r, TL* __restrict__ e, int clear_red,
                                                        unsigned long long* maxbits)
{
    int m = g.nx - 2;
    long total = (long)g.hx * m * (D == 3 ? m : 1);
    long stride = (long)gridDim.x * kBlock;
    size_t ny = (size_t)g.hx, nz = (size_t)g.nx * g.hx;
    unsigned long long best = 0;
    for (long t = xcd_block() * kBlock + threadIdx.x; t < total; t += stride) {
        int h = (int)(t % g.hx);
        long rr = t / g.hx;
        int pj = 1 + (int)(rr % m);
        int pk = D == 3 ? 1 + (int)(rr / m) : 0;
        size_t row = row_base(g, pj, pk);
        for (int c = 0; c < 2; c++) {
            int pi = 2 * h + ((c + pj + pk + D) & 1);
            if (pi < 1 || pi > g.nx - 2) continue;
            const double* o = phi + (size_t)(c ^ 1) * g.cs;
            size_t self = (size_t)c * g.cs + row + h;
            double s = o[row + ((pi - 1) >> 1)];
            s = s + o[row + ((pi + 1) >> 1)];
            s = s + o[row - ny + h];
            s = s + o[row + ny + h];
            if (D == 3) {
                s = s + o[row - nz + h];
                s = s + o[row + nz + h];
            }
            double v = f[self] - (s - (2.0 * D) * phi[self]) * inv_h2;
            r[self] = (TL)(float)(v * rscale);
            if (c == 1 || clear_red) e[self] = (TL)0.0f;
            unsigned long long b = abs_bits(v);
            best = b > best ? b : best;
        }
    }
    block_max_to(best, maxbits);
}

// 3-D form of k_dc_residual marching along z like k_resid_norm3 (both colours
// of one compact column per thread, z-neighbours from registers).
template <typename TL>
__global__ void __launch_bounds__(kBlock) k_dc_residual3(SGrid g, const double* __restrict__ u,
                                                         const double* __restrict__ f, double inv_h2, double rscale,
                                                         TL* __restrict__ r, TL* __restrict__ e, int clear_red,
                                                         int pblocks, unsigned long long* maxbits)
{
    const int m = g.nx - 2;
    const long lb = xcd_block();
    const int zc = (int)(lb / pblocks);
    const long t = (lb - (long)zc * pblocks) * kBlock + threadIdx.x;
    unsigned long long best = 0;
    if (t < (long)g.hx * m) {
        const int h = (int)(t % g.hx);
        const int pj = 1 + (int)(t / g.hx);
        const int k0 = 1 + zc * kNormChunk;
        const int k1 = min(k0 + kNormChunk - 1, m);
        const size_t plane = (size_t)g.nx * g.hx;
        const size_t col = (size_t)pj * g.hx + h;
        const double* __restrict__ a[2] = {u, u + g.cs};
        double below[2], cur[2];
        for (int c = 0; c < 2; c++) {
            below[c] = a[c][(size_t)(k0 - 1) * plane + col];
            cur[c] = a[c][(size_t)k0 * plane + col];
        }
        for (int pk = k0; pk <= k1; pk++) {
            const size_t here = (size_t)pk * plane + col;
            double above[2] = {a[0][here + plane], a[1][here + plane]};
            for (int c = 0; c < 2; c++) {
                const int o = c ^ 1;
                const int par = (c + pj + pk + 3) & 1;
                const int pi = 2 * h + par;
                if (pi < 1 || pi > g.nx - 2) continue;
                double xm = par ? cur[o] : a[o][here - 1];
                double xp = par ? a[o][here + 1] : cur[o];
                double s = xm + xp;
                s = s + a[o][here - g.hx];
                s = s + a[o][here + g.hx];
                s = s + below[o];
                s = s + above[o];
                const size_t self = (size_t)c * g.cs + here;
                double v = f[self] - (s - 6.0 * cur[c]) * inv_h2;
                r[self] = (TL)(float)(v * rscale);
                if (c == 1 || clear_red) e[self] = (TL)0.0f;
                unsigned long long b = abs_bits(v);
                best = b > best ? b : best;
            }
            for (int c = 0; c < 2; c++) {
                below[c] = cur[c];
                cur[c] = above[c];
            }
        }
    }
    block_max_to(best, maxbits);
}

// phi += factor * e on the level-0 active points (the FP64 correction update).
template <int D, typename TL>
__global__ void __launch_bounds__(kBlock) k_dc_update(SGrid g, double* __restrict__ phi, const TL* __restrict__ e,
                                                      double factor)
{
    int m = g.nx - 2;
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = (long)g.hx * m * (D == 3 ? m : 1);
    if (t >= total) return;
    int h = (int)(t % g.hx);
    long rr = t / g.hx;
    int pj = 1 + (int)(rr % m);
    int pk = D == 3 ? 1 + (int)(rr / m) : 0;
    size_t row = row_base(g, pj, pk);
    for (int c = 0; c < 2; c++) {
        int pi = 2 * h + ((c + pj + pk + D) & 1);
        if (pi < 1 || pi > g.nx - 2) continue;
        size_t self = (size_t)c * g.cs + row + h;
        phi[self] += factor * (double)(float)e[self];
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers
#define NP_DISPATCH(dim, KERNEL, grid, block, st, ...)                                    \
    do {                                                                                  \
        if ((dim) == 3) hipLaunchKernelGGL((KERNEL<3>), (grid), (block), 0, (st), __VA_ARGS__); \
        else hipLaunchKernelGGL((KERNEL<2>), (grid), (block), 0, (st), __VA_ARGS__);           \
    } while (0)

static long npoints(const SGrid& g) { return (long)g.nx * g.nx * g.nz; }
static long ncompact_active(int dim, const SGrid& g)
{
    long m = g.nx - 2;
    return (long)g.hx * m * (dim == 3 ? m : 1);
}

void launch_level0_init(int dim, hipStream_t st, SGrid g, const double* rho0, const double* phi_outer,
                        double fourpiG, double* phi, double* f)
{
    NP_DISPATCH(dim, k_level0_init, dim3(ceil_div(npoints(g), kBlock)), dim3(kBlock), st, g, rho0, phi_outer, fourpiG,
                phi, f);
}

void launch_interface_fill(int dim, hipStream_t st, SGrid gc, const double* phic, const double* fc, SGrid gf,
                           int nf, int offx, int offy, int offz, const double* rho, double fourpiG, double* phif,
                           double* ff)
{
    NP_DISPATCH(dim, k_interface_fill, dim3(ceil_div(npoints(gf), kBlock)), dim3(kBlock), st, gc, phic, fc, gf, nf,
                offx, offy, offz, rho, fourpiG, phif, ff);
}

void launch_forces(int dim, hipStream_t st, SGrid g, int n, double dx, const double* phi, double* fx, double* fy,
                   double* fz)
{
    double m12dx = -1.0 / (12.0 * dx);
    Strip sp = make_strip(n, n, dim == 3 ? n : 1, 16);
    long blocks = dim == 3 ? strip_blocks(sp) : ceil_div((long)n * n, kBlock);
    NP_DISPATCH(dim, k_forces, dim3(blocks), dim3(kBlock), st, g, n, m12dx, phi, fx, fy, fz, sp);
}

void launch_force_delta(int dim, hipStream_t st, SGrid g, int n, double dx, const double* phi, double* F,
                        unsigned long long* maxbits)
{
    long total = dim == 3 ? (long)n * n * n : (long)n * n;
    double m12dx = -1.0 / (12.0 * dx);
    NP_DISPATCH(dim, k_force_delta, dim3(ceil_div(total, kBlock)), dim3(kBlock), st, g, n, m12dx, phi, F, maxbits);
}

void launch_export(int dim, hipStream_t st, SGrid g, const double* a, double* out)
{
    NP_DISPATCH(dim, k_export, dim3(ceil_div(npoints(g), kBlock)), dim3(kBlock), st, g, a, out);
}

void launch_norm(int dim, hipStream_t st, SGrid g, const double* u, const double* f, double inv_h2, int mode,
                 unsigned long long* maxbits)
{
    if (dim == 3 && mode == 0) {
        long m = g.nx - 2;
        int pblocks = ceil_div((long)g.hx * m, kBlock);
        int chunks = ceil_div(m, kNormChunk);
        hipLaunchKernelGGL(k_resid_norm3, dim3(pblocks * chunks), dim3(kBlock), 0, st, g, u, f, inv_h2, pblocks,
                           maxbits);
        return;
    }
    int blocks = ceil_div(ncompact_active(dim, g), kBlock);
    if (blocks > 2048) blocks = 2048;
    NP_DISPATCH(dim, k_norm, dim3(blocks), dim3(kBlock), st, g, u, f, inv_h2, mode, maxbits);
}

void launch_set_u64(hipStream_t st, unsigned long long* p, int count, unsigned long long v)
{
    hipLaunchKernelGGL(k_set_u64, dim3(ceil_div(count, 64)), dim3(64), 0, st, p, count, v);
}

template <typename T>
void launch_half_sweep(int dim, hipStream_t st, SGrid g, T* u, const T* f, int colour, double h2, int fine)
{
    using C = typename Compute<T>::type;
    dim3 grid(ceil_div(ncompact_active(dim, g), kBlock));
    C inv2d = (C)(1.0 / (2.0 * dim));
    if (dim == 3 && fine && sizeof(T) <= 4 && (g.hx % 2) == 0) {
        // 2- and 4-byte storage: two compact points per thread, paired loads
        long m = g.nx - 2;
        int pblocks = ceil_div((long)(g.hx / 2) * m, kBlock);
        int chunks = ceil_div(m, kZChunk);
        hipLaunchKernelGGL((k_smooth_zmarch3_pair<T>), dim3(pblocks * chunks), dim3(kBlock), 0, st, u, f, g, colour,
                           (C)h2, inv2d, pblocks);
        return;
    }
    if (dim == 3 && (fine || g.nx >= 34)) {
        // z-march; the level-0 instance (TAG 0) is kept apart from the
        // coarse-level one (TAG 1) so that profiles separate them
        long m = g.nx - 2;
        int pblocks = ceil_div((long)g.hx * m, kBlock);
        int chunks = ceil_div(m, kZChunk);
        if (fine)
            hipLaunchKernelGGL((k_smooth_zmarch3<T, 0>), dim3(pblocks * chunks), dim3(kBlock), 0, st, u, f, g, colour,
                               (C)h2, inv2d, pblocks);
        else
            hipLaunchKernelGGL((k_smooth_zmarch3<T, 1>), dim3(pblocks * chunks), dim3(kBlock), 0, st, u, f, g, colour,
                               (C)h2, inv2d, pblocks);
        return;
    }
    if (fine) {
        hipLaunchKernelGGL((k_smooth_fine<2, T>), grid, dim3(kBlock), 0, st, u, f, g, colour, (C)h2, inv2d);
    } else {
        if (dim == 3)
            hipLaunchKernelGGL((k_half_sweep<3, T>), grid, dim3(kBlock), 0, st, u, f, g, colour, (C)h2, inv2d);
        else
            hipLaunchKernelGGL((k_half_sweep<2, T>), grid, dim3(kBlock), 0, st, u, f, g, colour, (C)h2, inv2d);
    }
}

template <typename T>
void launch_ghost_fill(int dim, hipStream_t st, SGrid g, T* u, int xn_is_one, double coef)
{
    using C = typename Compute<T>::type;
    int per = dim == 3 ? g.nx * g.nx : g.nx;
    dim3 grid(ceil_div(per, kBlock), 2 * dim);
    if (dim == 3)
        hipLaunchKernelGGL((k_ghost_fill<3, T>), grid, dim3(kBlock), 0, st, u, g, xn_is_one, (C)coef);
    else
        hipLaunchKernelGGL((k_ghost_fill<2, T>), grid, dim3(kBlock), 0, st, u, g, xn_is_one, (C)coef);
}

template <typename TF, typename TC>
void launch_resid_restrict(int dim, hipStream_t st, SGrid gf, const TF* u, const TF* f, double inv_h2, double out_scale,
                           SGrid gc, TC* fc, TC* ec)
{
    using C = typename Compute<TC>::type;
    long Nc = gc.nx - 2;
    long total = dim == 3 ? Nc * Nc * Nc : Nc * Nc;
    dim3 grid(ceil_div(total, kBlock));
    if (dim == 3)
        hipLaunchKernelGGL((k_resid_restrict<3, TF, TC>), grid, dim3(kBlock), 0, st, u, f, gf, (C)inv_h2, (C)out_scale,
                           gc, fc, ec);
    else
        hipLaunchKernelGGL((k_resid_restrict<2, TF, TC>), grid, dim3(kBlock), 0, st, u, f, gf, (C)inv_h2, (C)out_scale,
                           gc, fc, ec);
}

template <typename TC, typename TF>
void launch_prolong_add(int dim, hipStream_t st, SGrid gc, const TC* ec, SGrid gf, TF* u, int black_only)
{
    dim3 grid(ceil_div(ncompact_active(dim, gf), kBlock));
    if (dim == 3)
        hipLaunchKernelGGL((k_prolong_add<3, TC, TF>), grid, dim3(kBlock), 0, st, ec, gc, u, gf, black_only);
    else
        hipLaunchKernelGGL((k_prolong_add<2, TC, TF>), grid, dim3(kBlock), 0, st, ec, gc, u, gf, black_only);
}

template <typename TL>
void launch_dc_residual(int dim, hipStream_t st, SGrid g, const double* phi, const double* f, double inv_h2,
                        double rscale, TL* r, TL* e, int clear_red, unsigned long long* maxbits)
{
    int blocks = ceil_div(ncompact_active(dim, g), kBlock);
    if (blocks > 4096) blocks = 4096;
    if (dim == 3) {
        long m = g.nx - 2;
        int pblocks = ceil_div((long)g.hx * m, kBlock);
        int chunks = ceil_div(m, kNormChunk);
        hipLaunchKernelGGL((k_dc_residual3<TL>), dim3(pblocks * chunks), dim3(kBlock), 0, st, g, phi, f, inv_h2,
                           rscale, r, e, clear_red, pblocks, maxbits);
    } else
        hipLaunchKernelGGL((k_dc_residual<2, TL>), dim3(blocks), dim3(kBlock), 0, st, g, phi, f, inv_h2, rscale, r, e,
                           clear_red, maxbits);
}

template <typename TL>
void launch_dc_update(int dim, hipStream_t st, SGrid g, double* phi, const TL* e, double factor)
{
    dim3 grid(ceil_div(ncompact_active(dim, g), kBlock));
    if (dim == 3)
        hipLaunchKernelGGL((k_dc_update<3, TL>), grid, dim3(kBlock), 0, st, g, phi, e, factor);
    else
        hipLaunchKernelGGL((k_dc_update<2, TL>), grid, dim3(kBlock), 0, st, g, phi, e, factor);
}

template void launch_half_sweep<double>(int, hipStream_t, SGrid, double*, const double*, int, double, int);
template void launch_half_sweep<float>(int, hipStream_t, SGrid, float*, const float*, int, double, int);
template void launch_half_sweep<__half>(int, hipStream_t, SGrid, __half*, const __half*, int, double, int);
template void launch_ghost_fill<double>(int, hipStream_t, SGrid, double*, int, double);
template void launch_ghost_fill<float>(int, hipStream_t, SGrid, float*, int, double);
template void launch_resid_restrict<double, double>(int, hipStream_t, SGrid, const double*, const double*, double,
                                                    double, SGrid, double*, double*);
template void launch_resid_restrict<float, float>(int, hipStream_t, SGrid, const float*, const float*, double, double,
                                                  SGrid, float*, float*);
template void launch_resid_restrict<__half, float>(int, hipStream_t, SGrid, const __half*, const __half*, double,
                                                   double, SGrid, float*, float*);
template void launch_prolong_add<double, double>(int, hipStream_t, SGrid, const double*, SGrid, double*, int);
template void launch_prolong_add<float, float>(int, hipStream_t, SGrid, const float*, SGrid, float*, int);
template void launch_prolong_add<float, __half>(int, hipStream_t, SGrid, const float*, SGrid, __half*, int);
template void launch_dc_residual<float>(int, hipStream_t, SGrid, const double*, const double*, double, double, float*,
                                        float*, int, unsigned long long*);
template void launch_dc_residual<__half>(int, hipStream_t, SGrid, const double*, const double*, double, double,
                                         __half*, __half*, int, unsigned long long*);
template void launch_dc_update<float>(int, hipStream_t, SGrid, double*, const float*, double);
template void launch_dc_update<__half>(int, hipStream_t, SGrid, double*, const __half*, double);

}  // namespace np

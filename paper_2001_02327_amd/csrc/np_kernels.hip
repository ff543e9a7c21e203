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
// block sizes measured per kernel at 514^3 (128 / 256 / 512 threads): the paired
// level-0 half sweep 92.8 / 84.3 / 82.5 us, the forces 1217 / 1248 / 2805 us;
// every other kernel is fastest at kBlock
constexpr int kSmoothPairBlock = 512;
constexpr int kForceBlock = 128;

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

// Two consecutive elements moved by one load or store of twice the width.
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
    T a, b;
};

// Stores marked non-temporal, for FP64 data written once and not read again
// before much more than the caches hold has passed through them (the updated
// potential of the defect-correction pass, the forces, the coarse-to-fine
// fill): they then do not displace what the next kernels read.
__device__ __forceinline__ void store_nt(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_nt(Pair<double>* p, const Pair<double>& v)
{
    typedef double d2_t __attribute__((ext_vector_type(2)));
    const d2_t x = {v.a, v.b};
    __builtin_nontemporal_store(x, (d2_t*)p);
}
constexpr bool kFillNt = true;  // non-temporal stores in the level setup kernels as well
// load of FP64 data read once and not again soon (the right-hand side in the
// defect-correction pass)
__device__ __forceinline__ Pair<double> load_nt(const Pair<double>* p)
{
    typedef double d2_t __attribute__((ext_vector_type(2)));
    const d2_t x = __builtin_nontemporal_load((const d2_t*)p);
    return Pair<double>{x.x, x.y};
}
constexpr bool kDcLoadNt = true;

// Consecutive level-0 kernels of a V-cycle run their z-chunks in alternating
// directions (rev: the logical block order reversed), so that each starts on
// the planes the previous one touched last, which the memory-side cache still
// holds.  The direction changes the order of the work only, never its result.
constexpr bool kAlternateZ = true;

__device__ __forceinline__ int zmarch_block(int rev)
{
    const int lb = (int)xcd_block();
    return (kAlternateZ && rev) ? (int)gridDim.x - 1 - lb : lb;
}

// Value of the previous (lane - 1) and next (lane + 1) lane of the wave by a
// DPP wave shift; lane 0 (previous) and lane 63 (next) get 0.
__device__ __forceinline__ unsigned dpp_prev(unsigned v)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}
__device__ __forceinline__ unsigned dpp_next(unsigned v)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}
__device__ __forceinline__ float dpp_prev(float x) { return __uint_as_float(dpp_prev(__float_as_uint(x))); }
__device__ __forceinline__ float dpp_next(float x) { return __uint_as_float(dpp_next(__float_as_uint(x))); }
__device__ __forceinline__ double dpp_prev(double x)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long lo = dpp_prev((unsigned)b), hi = dpp_prev((unsigned)(b >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}
__device__ __forceinline__ double dpp_next(double x)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long lo = dpp_next((unsigned)b), hi = dpp_next((unsigned)(b >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
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

__device__ __forceinline__ bool strip_point(const Strip& s, int& x, int& y, int& z)
{
    const int lb = (int)xcd_block();
    const int per = s.nza * s.B;
    const int st = lb / per;
    const int rem = lb - st * per;
    z = rem / s.B;
    const int blk = rem - z * s.B;
    const int tin = blk * kBlock + threadIdx.x;
    const int rr = tin / s.nxa;
    x = tin - rr * s.nxa;
    y = st * s.R + rr;
    return rr < s.R && y < s.nya;
}

// Patch batches (SGrid::nb): a multigrid launch over nb patches of one grid
// runs patch blockIdx.y; its arrays start blockIdx.y * bs elements in, and a
// patch whose flag in act is 0 has stopped iterating: its blocks return at
// once (a block-uniform exit, before any barrier).
__device__ __forceinline__ bool batch_idle(const SGrid& g) { return g.act && !g.act[blockIdx.y]; }

template <typename T>
__device__ __forceinline__ T* batch_at(T* p, const SGrid& g)
{
    return p ? p + (size_t)blockIdx.y * g.bs : p;
}

template <int D>
__device__ __forceinline__ int colour_of(int pi, int pj, int pk)
{
    return (pi + pj + pk + D) & 1;
}

__device__ __forceinline__ size_t row_base(const SGrid& g, int pj, int pk)
{
    return (size_t)pk * g.ps + (size_t)pj * g.hx;
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

// Atomic maximum of v over a block of NW wavefronts into *out.
template <int NW>
__device__ __forceinline__ void block_max_to_w(unsigned long long v, unsigned long long* out)
{
    __shared__ unsigned long long red[NW];
    v = wave_max_u64(v);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = red[0];
        for (int w = 1; w < NW; w++) m = red[w] > m ? red[w] : m;
        atomicMax(out, m);
    }
}

__device__ __forceinline__ void block_max_to(unsigned long long v, unsigned long long* out)
{
    block_max_to_w<kBlock / 64>(v, out);
}

__device__ __forceinline__ unsigned long long abs_bits(double a)
{
    return (unsigned long long)__double_as_longlong(fabs(a));
}

// Residual f - (s - 2d u) / h^2 at a point (s: the sum of its 2d neighbours)
// with the rounding every residual-norm pass uses: one fused multiply-add
// forms s - 2d u, a second f - (s - 2d u) inv_h2.
__device__ __forceinline__ double resid(double f, double s, double u, double two_d, double inv_h2)
{
    return __fma_rn(-inv_h2, __fma_rn(-two_d, u, s), f);
}

// ------------------------------------------------------------------ level setup
// Level 0: potential = caller's outer layer on the ring, zero on Gamma^0;
// right-hand side = 4 pi G rho on Gamma^0 (caller gives Omega^0 plus its inner
// layer, (n+2)^d points).
// Also reduces max |f| into *fmax (grid-stride loop, one atomic per block).
constexpr int kInitBlocks = 16384;
template <int D>
__global__ void __launch_bounds__(kBlock) k_level0_init(SGrid g, const double* __restrict__ rho0,
                                                        const double* __restrict__ phi_outer, double fourpiG,
                                                        double* __restrict__ phi, double* __restrict__ f,
                                                        unsigned long long* fmax)
{
    const long total = (long)g.nx * g.ny * g.nz;
    const long stride = (long)gridDim.x * kBlock;
    unsigned long long best = 0;
    // 32-bit index arithmetic where the grid allows (a 64-bit division costs
    // several times a 32-bit one, per point)
    const bool narrow = total <= 0xffffffffL;
    for (long t = xcd_block() * kBlock + threadIdx.x; t < total; t += stride) {
        int pi, pj, pk;
        if (narrow) {
            const unsigned tu = (unsigned)t, r = tu / (unsigned)g.nx;
            pi = (int)(tu - r * (unsigned)g.nx);
            pj = (int)(r % (unsigned)g.ny);
            pk = (int)(r / (unsigned)g.ny);
        } else {
            pi = (int)(t % g.nx);
            const long r = t / g.nx;
            pj = (int)(r % g.ny);
            pk = (int)(r / g.ny);
        }
        bool ring = pi == 0 || pi == g.nx - 1 || pj == 0 || pj == g.ny - 1 || (D == 3 && (pk == 0 || pk == g.nz - 1));
        size_t p = pos<D, double>(g, pi, pj, pk);
        if (ring) {
            phi[p] = phi_outer[t];
            f[p] = 0.0;
        } else {
            const int mx = g.nx - 2, my = g.ny - 2;
            size_t ri = D == 3 ? (((size_t)(pk - 1) * my + (pj - 1)) * mx + (pi - 1)) : ((size_t)(pj - 1) * mx + (pi - 1));
            const double v = fourpiG * rho0[ri];
            if (kFillNt) {
                store_nt(phi + p, 0.0);
                store_nt(f + p, v);
            } else {
                phi[p] = 0.0;
                f[p] = v;
            }
            const unsigned long long b = abs_bits(v);
            best = b > best ? b : best;
        }
    }
    block_max_to(best, fmax);
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
                                                           const double* __restrict__ fc, SGrid gf, int offx,
                                                           int offy, int offz, const double* __restrict__ rho,
                                                           double fourpiG, double* __restrict__ phif,
                                                           double* __restrict__ ff, unsigned long long* fmax)
{
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = (long)gf.nx * gf.ny * gf.nz;
    const int nfx = gf.nx - 4, nfy = gf.ny - 4, nfz = gf.nz - 4;
    unsigned long long best = 0;
    if (t < total) {
    int pi = (int)(t % gf.nx);
    long r = t / gf.nx;
    int pj = (int)(r % gf.ny);
    int pk = (int)(r / gf.ny);
    int qi, qj, qk = 0, si, sj, sk = 1;
    fine_to_coarse(pi, offx, qi, si);
    fine_to_coarse(pj, offy, qj, sj);
    if (D == 3) fine_to_coarse(pk, offz, qk, sk);
    size_t p = pos<D, double>(gf, pi, pj, pk);
    phif[p] = interp_tensor<D>(phic, gc, qi, qj, qk, si, sj, sk);
    bool outer = pi == 0 || pi == gf.nx - 1 || pj == 0 || pj == gf.ny - 1 || (D == 3 && (pk == 0 || pk == gf.nz - 1));
    bool omega = pi >= 2 && pi <= nfx + 1 && pj >= 2 && pj <= nfy + 1 && (D == 2 || (pk >= 2 && pk <= nfz + 1));
    double v;
    if (outer) {
        v = 0.0;
    } else if (omega) {
        size_t ri = D == 3 ? (((size_t)(pk - 2) * nfy + (pj - 2)) * nfx + (pi - 2)) : ((size_t)(pj - 2) * nfx + (pi - 2));
        v = fourpiG * rho[ri];
    } else {
        v = interp_tensor<D>(fc, gc, qi, qj, qk, si, sj, sk);
    }
    ff[p] = v;
    best = abs_bits(v);
    }
    if (fmax) block_max_to(best, fmax);
}

// 3-D form of k_interface_fill marching along the coarse z axis: a thread owns
// one coarse column and a chunk of coarse planes, keeps the 3 x 3 x 3 coarse
// potential around the current coarse cell in registers and writes the 8 fine
// points whose interpolation parent is that cell (fine padded p = 2a + d,
// d = 0, 1, for the a-th parent from offset + 1).  The right-hand side of the
// inner layer (rare) is interpolated with direct loads.  Same values as
// k_interface_fill.
constexpr int kFillChunk = 8;

__global__ void __launch_bounds__(kBlock) k_interface_fill3_zm(SGrid gc, const double* __restrict__ phic,
                                                               const double* __restrict__ fc, SGrid gf,
                                                               int offx, int offy, int offz,
                                                               const double* __restrict__ rho, double fourpiG,
                                                               double* __restrict__ phif, double* __restrict__ ff,
                                                               int pblocks, unsigned long long* fmax)
{
    // parents per axis: fine padded points 0 .. n_a + 3 in pairs
    const int Mx = (gf.nx + 1) / 2, My = (gf.ny + 1) / 2, Mz = (gf.nz + 1) / 2;
    const int nfx = gf.nx - 4, nfy = gf.ny - 4, nfz = gf.nz - 4;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    unsigned long long best = 0;  // max |f| written (the outer layer's 0 does not raise it)
    if (t < Mx * My) {
    const int a = (int)(t % Mx), b = (int)(t / Mx);
    const int c0 = zc * kFillChunk, c1 = min(c0 + kFillChunk, Mz) - 1;
    const int qi = offx + 1 + a, qj = offy + 1 + b;
    double cv[3][3][3];  // [z][y][x]: coarse planes qk-1 .. qk+1, rows qj-1 .., columns qi-1 ..
    auto load_plane = [&](int qk, double (&pl)[3][3]) {
#pragma unroll
        for (int y = 0; y < 3; y++)
#pragma unroll
            for (int x = 0; x < 3; x++) pl[y][x] = at<3>(phic, gc, qi - 1 + x, qj - 1 + y, qk);
    };
    load_plane(offz + c0, cv[0]);
    load_plane(offz + c0 + 1, cv[1]);
    load_plane(offz + c0 + 2, cv[2]);
    const double w0 = 0.75, w1 = 0.25;
    for (int cc = c0; cc <= c1; cc++) {
        const int qk = offz + 1 + cc;
        // issued before this step's arithmetic: the next step's coarse plane and
        // the density of this step's children inside Omega
        double nxt[3][3];
        if (cc < c1) load_plane(qk + 2, nxt);
        double rv[2][2][2];
#pragma unroll
        for (int dz = 0; dz < 2; dz++)
#pragma unroll
            for (int dy = 0; dy < 2; dy++)
#pragma unroll
                for (int dx = 0; dx < 2; dx++) {
                    const int pi = 2 * a + dx, pj = 2 * b + dy, pk = 2 * cc + dz;
                    const bool omega =
                        pi >= 2 && pi <= nfx + 1 && pj >= 2 && pj <= nfy + 1 && pk >= 2 && pk <= nfz + 1;
                    rv[dz][dy][dx] = omega ? rho[((size_t)(pk - 2) * nfy + (pj - 2)) * nfx + (pi - 2)] : 0.0;
                }
#pragma unroll
        for (int dz = 0; dz < 2; dz++) {
            const int pk = 2 * cc + dz;
            if (pk > gf.nz - 1) continue;
            const int zs = dz ? 2 : 0;  // side of the fine centre: -1 for d = 0, +1 for d = 1
#pragma unroll
            for (int dy = 0; dy < 2; dy++) {
                const int pj = 2 * b + dy;
                if (pj > gf.ny - 1) continue;
                const int ys = dy ? 2 : 0;
#pragma unroll
                for (int dx = 0; dx < 2; dx++) {
                    const int pi = 2 * a + dx;
                    if (pi > gf.nx - 1) continue;
                    const int xs = dx ? 2 : 0;
                    const double y0 = w0 * cv[1][1][1] + w1 * cv[1][1][xs];
                    const double y1 = w0 * cv[1][ys][1] + w1 * cv[1][ys][xs];
                    const double z0 = w0 * y0 + w1 * y1;
                    const double y2 = w0 * cv[zs][1][1] + w1 * cv[zs][1][xs];
                    const double y3 = w0 * cv[zs][ys][1] + w1 * cv[zs][ys][xs];
                    const double z1 = w0 * y2 + w1 * y3;
                    const size_t p = pos<3, double>(gf, pi, pj, pk);
                    phif[p] = w0 * z0 + w1 * z1;
                    const bool outer = pi == 0 || pi == gf.nx - 1 || pj == 0 || pj == gf.ny - 1 || pk == 0 ||
                                       pk == gf.nz - 1;
                    const bool omega =
                        pi >= 2 && pi <= nfx + 1 && pj >= 2 && pj <= nfy + 1 && pk >= 2 && pk <= nfz + 1;
                    double v;
                    if (outer) {
                        v = 0.0;
                    } else if (omega) {
                        v = fourpiG * rv[dz][dy][dx];
                    } else {
                        v = interp_tensor<3>(fc, gc, qi, qj, qk, dx ? 1 : -1, dy ? 1 : -1, dz ? 1 : -1);
                    }
                    ff[p] = v;
                    const unsigned long long bv = abs_bits(v);
                    best = bv > best ? bv : best;
                }
            }
        }
#pragma unroll
        for (int y = 0; y < 3; y++)
#pragma unroll
            for (int x = 0; x < 3; x++) {
                cv[0][y][x] = cv[1][y][x];
                cv[1][y][x] = cv[2][y][x];
                cv[2][y][x] = nxt[y][x];
            }
    }
    }
    if (fmax) block_max_to(best, fmax);
}

// 3-D coarse-to-fine fill in the paired form of the level-0 kernels: a thread
// owns the compact pair (h0, h0 + 1) of one fine row pj in both colours (the
// four fine points x = 2 h0 .. 2 h0 + 3), numbered flat over the padded plane
// (aligned waves), and a chunk of fine-plane pairs (2c + 2, 2c + 3), which share
// the coarse parent plane.  Their parents and neighbours lie among the coarse
// columns offx + h0 .. offx + h0 + 3 of two coarse rows; per coarse plane the
// four x-interpolants of each row are formed once.  Potential and right-hand
// side go out as paired stores, the density comes in 16-byte loads.  Same
// values, in the same order of operations, as k_interface_fill.  Requires an
// even row length hx and a coarse array of fewer than 2^31 elements.
constexpr int kFillPairChunk = 4;  // fine-plane pairs per thread

__global__ void __launch_bounds__(kBlock) k_interface_fill3_pair(SGrid gc, const double* __restrict__ phic,
                                                                 const double* __restrict__ fc, SGrid gf,
                                                                 int offx, int offy, int offz,
                                                                 const double* __restrict__ rho, double fourpiG,
                                                                 double* __restrict__ phif, double* __restrict__ ff,
                                                                 int pblocks, unsigned long long* fmax)
{
    const int nfx = gf.nx - 4, nfy = gf.ny - 4, nfz = gf.nz - 4;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    const int q = 2 * t;
    const int pj = q / gf.hx;
    const int h0 = q - pj * gf.hx;
    unsigned long long best = 0;  // max |f| written (the outer layer's 0 does not raise it)
    if (pj < gf.ny) {
        const int c0 = -1 + zc * kFillPairChunk;
        const int c1 = min(c0 + kFillPairChunk, gf.nz / 2 - 1);  // pairs c0 .. c1 - 1
        const int fyy = pj - 2;
        const int qy = offy + 2 + (fyy >> 1), sy = (fyy & 1) ? 1 : -1;
        const int cxb = offx + h0;  // coarse columns cxb .. cxb + 3
        // offsets inside a coarse plane of (row y, column x) for an even / odd plane index
        unsigned off[2][2][4];
#pragma unroll
        for (int y = 0; y < 2; y++)
#pragma unroll
            for (int x = 0; x < 4; x++) {
                const int cyv = y ? qy + sy : qy, cxv = cxb + x;
                const unsigned o = (unsigned)(cyv * gc.hx + (cxv >> 1));
                const bool ce = ((cxv + cyv + 3) & 1) != 0;  // colour on an even plane
                off[0][y][x] = o + (ce ? (unsigned)gc.cs : 0u);
                off[1][y][x] = o + (ce ? 0u : (unsigned)gc.cs);
            }
        const double w0 = 0.75, w1 = 0.25;
        // X[y][a]: x-interpolant of coarse plane qz, row y (parent, side), for the fine point 2 h0 + a
        auto load_X = [&](int qz, double (&X)[2][4]) {
            const double* __restrict__ cp = phic + (size_t)qz * gc.ps;
            double cv[2][4];
#pragma unroll
            for (int y = 0; y < 2; y++)
#pragma unroll
                for (int x = 0; x < 4; x++) cv[y][x] = cp[(qz & 1) ? off[1][y][x] : off[0][y][x]];
#pragma unroll
            for (int y = 0; y < 2; y++) {
                X[y][0] = w0 * cv[y][1] + w1 * cv[y][0];
                X[y][1] = w0 * cv[y][1] + w1 * cv[y][2];
                X[y][2] = w0 * cv[y][2] + w1 * cv[y][1];
                X[y][3] = w0 * cv[y][2] + w1 * cv[y][3];
            }
        };
        double Xm[2][4], X0[2][4], Xp[2][4];  // coarse planes qk - 1, qk, qk + 1
        load_X(offz + 1 + c0, Xm);
        load_X(offz + 2 + c0, X0);
        load_X(offz + 3 + c0, Xp);
        const bool yomega = pj >= 2 && pj <= nfy + 1;
        const size_t prow = (size_t)pj * gf.hx + h0;
        for (int c = c0; c < c1; c++) {
            const int qk = offz + 2 + c;
            double Xn[2][4];
            if (c + 1 < c1) load_X(qk + 2, Xn);
#pragma unroll
            for (int d = 0; d < 2; d++) {
                const int p = 2 * c + 2 + d;  // fine plane; its side coarse plane is qk - 1 (d = 0) or qk + 1
                const bool omega_row = yomega && p >= 2 && p <= nfz + 1;
                double rv[4] = {0.0, 0.0, 0.0, 0.0};
                if (omega_row) {
                    const int x0 = 2 * h0 - 2;  // natural x of the pair's first point
                    const double* __restrict__ rr = rho + ((size_t)(p - 2) * nfy + (pj - 2)) * nfx;
                    if (x0 >= 0 && x0 + 1 <= nfx - 1) {
                        const Pair<double> v = *(const Pair<double>*)(rr + x0);
                        rv[0] = v.a;
                        rv[1] = v.b;
                    }
                    if (x0 + 2 >= 0 && x0 + 3 <= nfx - 1) {
                        const Pair<double> v = *(const Pair<double>*)(rr + x0 + 2);
                        rv[2] = v.a;
                        rv[3] = v.b;
                    }
                }
                double ph[4], fv[4];
#pragma unroll
                for (int a = 0; a < 4; a++) {
                    const double(&S)[2][4] = d ? Xp : Xm;
                    const double z0 = w0 * X0[0][a] + w1 * X0[1][a];
                    const double z1 = w0 * S[0][a] + w1 * S[1][a];
                    ph[a] = w0 * z0 + w1 * z1;
                    const int pi = 2 * h0 + a;
                    const bool outer =
                        pi == 0 || pi == gf.nx - 1 || pj == 0 || pj == gf.ny - 1 || p == 0 || p == gf.nz - 1;
                    const bool omega = omega_row && pi >= 2 && pi <= nfx + 1;
                    double v;
                    if (outer) {
                        v = 0.0;
                    } else if (omega) {
                        v = fourpiG * rv[a];
                    } else {
                        v = interp_tensor<3>(fc, gc, offx + 1 + h0 + (a >> 1), qy, qk, (a & 1) ? 1 : -1, sy,
                                             d ? 1 : -1);
                    }
                    fv[a] = v;
                    const unsigned long long bv = abs_bits(v);
                    best = bv > best ? bv : best;
                }
                // colour of the even-x points 2 h0, 2 h0 + 2 in this row and plane
                const int ce = (pj + p + 1) & 1;
                const size_t base = (size_t)p * gf.ps + prow;
                Pair<double> pe{ph[0], ph[2]}, po{ph[1], ph[3]}, fe{fv[0], fv[2]}, fo{fv[1], fv[3]};
                if (kFillNt) {
                    store_nt((Pair<double>*)(phif + (size_t)ce * gf.cs + base), pe);
                    store_nt((Pair<double>*)(phif + (size_t)(ce ^ 1) * gf.cs + base), po);
                    store_nt((Pair<double>*)(ff + (size_t)ce * gf.cs + base), fe);
                    store_nt((Pair<double>*)(ff + (size_t)(ce ^ 1) * gf.cs + base), fo);
                } else {
                    *(Pair<double>*)(phif + (size_t)ce * gf.cs + base) = pe;
                    *(Pair<double>*)(phif + (size_t)(ce ^ 1) * gf.cs + base) = po;
                    *(Pair<double>*)(ff + (size_t)ce * gf.cs + base) = fe;
                    *(Pair<double>*)(ff + (size_t)(ce ^ 1) * gf.cs + base) = fo;
                }
            }
#pragma unroll
            for (int y = 0; y < 2; y++)
#pragma unroll
                for (int x = 0; x < 4; x++) {
                    Xm[y][x] = X0[y][x];
                    X0[y][x] = Xp[y][x];
                    Xp[y][x] = Xn[y][x];
                }
        }
    }
    if (fmax) block_max_to(best, fmax);
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
__global__ void __launch_bounds__(kBlock) k_forces(SGrid g, double m12dx, const double* __restrict__ phi,
                                                   double* __restrict__ fx, double* __restrict__ fy,
                                                   double* __restrict__ fz, Strip sp)
{
    const int nx = g.nx - 4, ny = g.ny - 4;
    int i, j, k = 0;
    long t;
    if (D == 3) {
        if (!strip_point(sp, i, j, k)) return;
        t = ((long)k * ny + j) * nx + i;
    } else {
        t = xcd_block() * kBlock + threadIdx.x;
        if (t >= (long)nx * ny) return;
        i = (int)(t % nx);
        j = (int)(t / nx);
    }
    int pi = i + 2, pj = j + 2, pk = D == 3 ? k + 2 : 0;
    fx[t] = d4<D>(phi, g, pi, pj, pk, 0, m12dx);
    fy[t] = d4<D>(phi, g, pi, pj, pk, 1, m12dx);
    if (D == 3) fz[t] = d4<D>(phi, g, pi, pj, pk, 2, m12dx);
}

// 3-D forces marching along z: a thread owns kForceRows columns (i, j0 .. j0+3)
// of Omega and a chunk of kForceChunk planes; the potential along its columns
// (planes k-2 .. k+2) stays in registers for the z-derivative and serves the
// y-derivatives of the neighbouring columns, so only two rows on each side are
// loaded for y; every load of the chunk is issued before the first difference.
// The x-neighbours i-2 .. i+2 are the adjacent lanes' column values, moved by DPP
// shifts: a wave owns the kForceOwn columns between its two first and two last
// lanes, which only supply values; at the ends of a row (the buffer columns) the
// lanes load them.  Same arithmetic as k_forces.  DELTA: the force-change stop
// test (Sec. 3.1): the arrays hold the previous iterate's forces, each point's
// new value replaces the old one and max |F_new - F_old| over the points and
// components goes to maxbits (as k_force_delta, value for value).
// planes and rows per thread: (8, 4) measured best of (4, 1), (4, 2), (2, 4), (4, 4),
// (4, 8), (2, 8) at 512^3 (1.61 -> 1.28 ms, with every x-neighbour loaded)
constexpr int kForceChunk = 8;
constexpr int kForceRows = 4;
constexpr int kForceOwn = 60;  // columns a wave owns (lanes 2..61)

template <bool DELTA>
__global__ void __launch_bounds__(kForceBlock) k_forces3_zm(SGrid g, double m12dx, const double* __restrict__ phi,
                                                       double* __restrict__ fx, double* __restrict__ fy,
                                                       double* __restrict__ fz, int pblocks,
                                                       unsigned long long* maxbits)
{
    unsigned long long best = 0;
    constexpr int R = kForceRows;
    constexpr int KC = kForceChunk;
    const int nx = g.nx - 4, ny = g.ny - 4, nz = g.nz - 4;
    const int nrb = (ny + R - 1) / R;
    const long total = (long)nx * nrb;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const long wave = (long)(lb - zc * pblocks) * (kForceBlock / 64) + (threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const long t = wave * kForceOwn + lane - 2;
    const bool owner = lane >= 2 && lane < 2 + kForceOwn && t >= 0 && t < total;
    const long tc = t < 0 ? 0 : (t >= total ? total - 1 : t);
    const int i = (int)(tc % nx), j0 = R * (int)(tc / nx);
    const int k0 = zc * KC;
    const int nk = min(KC, nz - k0);
    const int pi = i + 2;
    const bool xload = i < 2 || i >= nx - 2;  // an x-neighbour lies in the buffer columns
    // padded rows j0 + 2 - 2 .. j0 + 2 + R + 1: the thread's rows and two on each side
    // (rows past the array are clamped; they are never differenced)
    auto prow = [&](int q) { return min(j0 + q, ny + 3); };  // q = 0 .. R + 3
    double col[R][KC + 4];  // padded planes k0 .. k0 + nk + 3 of each of the thread's rows
    double yh[4][KC];       // rows j0, j0 + 1 (below) and j0 + R + 2, j0 + R + 3 (above), padded
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int q = 0; q < KC + 4; q++)
            if (q < nk + 4) col[r][q] = at<3>(phi, g, pi, prow(r + 2), k0 + q);
#pragma unroll
    for (int q = 0; q < KC; q++) {
        if (q < nk) {
            const int pk = k0 + q + 2;
            yh[0][q] = at<3>(phi, g, pi, prow(0), pk);
            yh[1][q] = at<3>(phi, g, pi, prow(1), pk);
            yh[2][q] = at<3>(phi, g, pi, prow(R + 2), pk);
            yh[3][q] = at<3>(phi, g, pi, prow(R + 3), pk);
        }
    }
    // value of padded row j0 + w (w = 0 .. R + 3) at padded plane k0 + q + 2
    auto yv = [&](int w, int q) -> double {
        if (w < 2) return yh[w][q];
        if (w >= R + 2) return yh[w - R][q];
        return col[w - 2][q + 2];
    };
#pragma unroll
    for (int q = 0; q < KC; q++) {
        if (q < nk) {
#pragma unroll
            for (int r = 0; r < R; r++) {
                const double c = col[r][q + 2];
                double xm1 = dpp_prev(c), xp1 = dpp_next(c);
                double xm2 = dpp_prev(xm1), xp2 = dpp_next(xp1);
                if (xload) {
                    const int pj = prow(r + 2), pk = k0 + q + 2;
                    xm1 = at<3>(phi, g, pi - 1, pj, pk);
                    xp1 = at<3>(phi, g, pi + 1, pj, pk);
                    xm2 = at<3>(phi, g, pi - 2, pj, pk);
                    xp2 = at<3>(phi, g, pi + 2, pj, pk);
                }
                if (!owner || j0 + r >= ny) continue;
                const long o = ((long)(k0 + q) * ny + (j0 + r)) * nx + i;
                const int w = r + 2;
                const double vx = (8.0 * (xp1 - xm1) - (xp2 - xm2)) * m12dx;
                const double vy = (8.0 * (yv(w + 1, q) - yv(w - 1, q)) - (yv(w + 2, q) - yv(w - 2, q))) * m12dx;
                const double vz = (8.0 * (col[r][q + 3] - col[r][q + 1]) - (col[r][q + 4] - col[r][q])) * m12dx;
                if (DELTA) {
                    const double ox = fx[o], oy = fy[o], oz = fz[o];
                    unsigned long long b = abs_bits(vx - ox);
                    best = b > best ? b : best;
                    b = abs_bits(vy - oy);
                    best = b > best ? b : best;
                    b = abs_bits(vz - oz);
                    best = b > best ? b : best;
                }
                store_nt(fx + o, vx);
                store_nt(fy + o, vy);
                store_nt(fz + o, vz);
            }
        }
    }
    if (DELTA) block_max_to_w<kForceBlock / 64>(best, maxbits);
}

// Forces into F (d arrays of n^d) and the maximum change against the values
// F held before (the stop rule of Sec. 3.1).
template <int D>
__global__ void __launch_bounds__(kBlock) k_force_delta(SGrid g, double m12dx, const double* __restrict__ phi,
                                                        double* __restrict__ F, unsigned long long* maxbits)
{
    const int nx = g.nx - 4, ny = g.ny - 4, nz = D == 3 ? g.nz - 4 : 1;
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = (long)nx * ny * nz;
    unsigned long long m = 0;
    if (t < total) {
        int i = (int)(t % nx);
        long r = t / nx;
        int j = (int)(r % ny);
        int k = (int)(r / ny);
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
    long total = (long)g.nx * g.ny * g.nz;
    if (t >= total) return;
    int pi = (int)(t % g.nx);
    long r = t / g.nx;
    int pj = (int)(r % g.ny);
    int pk = (int)(r / g.ny);
    out[t] = at<D>(a, g, pi, pj, pk);
}

// ------------------------------------------------------------------ norms
// Grid-stride loop over a bounded grid so that only a few thousand blocks
// meet in the final atomic maximum.
template <int D>
__global__ void __launch_bounds__(kBlock) k_norm(SGrid g, const double* __restrict__ u, const double* __restrict__ f,
                                                 double inv_h2, int mode, unsigned long long* maxbits)
{
    if (batch_idle(g)) return;
    u = batch_at(u, g);
    f = batch_at(f, g);
    maxbits += blockIdx.y;
    const int my = g.ny - 2, mz = g.nz - 2;
    long total = (long)g.hx * my * (D == 3 ? mz : 1);
    long stride = (long)gridDim.x * kBlock;
    size_t ny = (size_t)g.hx, nz = g.ps;
    unsigned long long best = 0;
    for (long t = xcd_block() * kBlock + threadIdx.x; t < total; t += stride) {
        int h = (int)(t % g.hx);
        long r = t / g.hx;
        int pj = 1 + (int)(r % my);
        int pk = D == 3 ? 1 + (int)(r / my) : 0;
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
                if (pj + 1 == g.ny - 1) s += o[row + ny + h];
                if (D == 3 && pk - 1 == 0) s += o[row - nz + h];
                if (D == 3 && pk + 1 == g.nz - 1) s += o[row + nz + h];
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
                val = resid(f[self], s, u[self], 2.0 * D, inv_h2);
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
constexpr int kNormChunk = 8;  // 2, 4, 16 measured slower (more blocks, more atomics)

__global__ void __launch_bounds__(kBlock) k_resid_norm3(SGrid g, const double* __restrict__ u,
                                                        const double* __restrict__ f, double inv_h2, int pblocks,
                                                        unsigned long long* maxbits)
{
    if (batch_idle(g)) return;
    u = batch_at(u, g);
    f = batch_at(f, g);
    maxbits += blockIdx.y;
    const int my = g.ny - 2, mz = g.nz - 2;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    unsigned long long best = 0;
    // flat index over the whole (padded) plane: aligned wave segments; the ghost
    // rows and the padding have no work
    const int pj = t / g.hx;
    const int h = t - pj * g.hx;
    if (pj >= 1 && pj <= my) {
        const int k0 = 1 + zc * kNormChunk;
        const int k1 = min(k0 + kNormChunk - 1, mz);
        const size_t plane = g.ps;
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
                double r = resid(f[(size_t)c * g.cs + here], s, cur[c], 6.0, inv_h2);
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

// Max norm of the residual's mean over boxes of 4^3 active points of a 3-D
// nested-level array (boxes at the far end keep their full volume; points
// past the active range count as zero): the residual restricted twice
// (eqn:restriction3D applied to multigrid levels 0 -> 1 -> 2), i.e. its part
// that the smoother does not remove and that sets the number of V-cycles.  A
// thread owns one box.
constexpr int kBox = 4;

__global__ void __launch_bounds__(kBlock) k_box_resid_norm3(SGrid g, const double* __restrict__ u,
                                                            const double* __restrict__ f, double inv_h2,
                                                            unsigned long long* maxbits)
{
    const int mx = g.nx - 2, my = g.ny - 2, mz = g.nz - 2;
    const int nbx = (mx + kBox - 1) / kBox, nby = (my + kBox - 1) / kBox, nbz = (mz + kBox - 1) / kBox;
    const long t = xcd_block() * kBlock + threadIdx.x;
    unsigned long long best = 0;
    if (t < (long)nbx * nby * nbz) {
        const int bx = (int)(t % nbx), by = (int)((t / nbx) % nby), bz = (int)(t / ((long)nbx * nby));
        {
            double sum = 0.0;
            for (int dz = 0; dz < kBox; dz++) {
                const int pk = 1 + kBox * bz + dz;
                if (pk > mz) break;
                for (int dy = 0; dy < kBox; dy++) {
                    const int pj = 1 + kBox * by + dy;
                    if (pj > my) break;
                    for (int dx = 0; dx < kBox; dx++) {
                        const int pi = 1 + kBox * bx + dx;
                        if (pi > mx) break;
                        double s6 = at<3>(u, g, pi - 1, pj, pk) + at<3>(u, g, pi + 1, pj, pk);
                        s6 = s6 + at<3>(u, g, pi, pj - 1, pk);
                        s6 = s6 + at<3>(u, g, pi, pj + 1, pk);
                        s6 = s6 + at<3>(u, g, pi, pj, pk - 1);
                        s6 = s6 + at<3>(u, g, pi, pj, pk + 1);
                        sum += at<3>(f, g, pi, pj, pk) - (s6 - 6.0 * at<3>(u, g, pi, pj, pk)) * inv_h2;
                    }
                }
            }
            const unsigned long long b = abs_bits(sum * (1.0 / (kBox * kBox * kBox)));
            best = b > best ? b : best;
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

// Ghost rule of a multigrid level L >= 1 (Sec. 2.4): the layer outside the
// active points 1..N is anti-symmetric, e_0 = -e_1 on the left and on the right
// e_{N+1} = -e_{N-1} when x_N = 1, else coef * e_N; points outside along several
// axes compose the rule of each axis in the order x, y, z.  The kernels never
// store this layer: they evaluate it where they read it.  That gives the values
// a refresh before every half sweep would: a face ghost next to an active
// point p depends only on p itself or on the point beyond p on the same axis,
// which has the other colour, and neither changes before p's own update.
template <typename C>
struct GRule {
    int xn1[3];  // per axis: the last active centre sits at x_MG = 1
    C coef[3];   // per axis: the right-ghost coefficient otherwise
};

template <typename C>
GRule<C> grule(const Rule3& r)
{
    return GRule<C>{{r.xn1[0], r.xn1[1], r.xn1[2]}, {(C)r.coef[0], (C)r.coef[1], (C)r.coef[2]}};
}

// Value at padded point p of a level with a rule ghost layer (any point, ghost
// along any number of axes).  Factors are applied per axis in x, y, z order.
template <int D, typename T, typename C>
__device__ __forceinline__ C rule_at(const T* __restrict__ a, const SGrid& g, int pi, int pj, int pk,
                                     const GRule<C>& gr)
{
    const int Na[3] = {g.nx - 2, g.ny - 2, g.nz - 2};
    int p[3] = {pi, pj, pk};
    C fac[3] = {(C)1, (C)1, (C)1};
    bool sc[3] = {false, false, false};
    for (int ax = 0; ax < D; ax++) {
        const int N = Na[ax];
        if (p[ax] == 0) {
            p[ax] = 1;
            fac[ax] = (C)-1;
            sc[ax] = true;
        } else if (p[ax] == N + 1) {
            p[ax] = gr.xn1[ax] ? N - 1 : N;
            fac[ax] = gr.xn1[ax] ? (C)-1 : gr.coef[ax];
            sc[ax] = true;
        }
    }
    C v = (C)at<D>(a, g, p[0], p[1], p[2]);
    for (int ax = 0; ax < D; ax++)
        if (sc[ax]) v = fac[ax] * v;
    return v;
}

// Face-ghost substitution for a 7-point stencil at active index q (1..N) along
// axis ax: the neighbour below (q = 1) is -self; the neighbour above (q = N)
// is -(the neighbour below) when x_N = 1, else coef * self.
template <typename C>
__device__ __forceinline__ void rule_pair(int q, int N, C self, C& lo, C& hi, const GRule<C>& gr, int ax)
{
    if (q == 1) lo = -self;
    if (q == N) hi = gr.xn1[ax] ? -lo : gr.coef[ax] * self;
}

// Red-black Gauss-Seidel half sweep: u_c = (sum of the 2d neighbours - h^2 f_c) / (2d)
// over the active points of one colour; the neighbours are all of the other colour.
// k_smooth_fine runs it on the nested-level arrays (multigrid level 0, whose
// ghost layer is the fixed outer buffer), k_half_sweep on the coarse levels.
template <int D, typename T, bool RULE>
__device__ __forceinline__ void half_sweep_body(T* __restrict__ u, const T* __restrict__ f, SGrid g,
                                                       int colour, typename Compute<T>::type h2,
                                                       typename Compute<T>::type inv2d,
                                                       GRule<typename Compute<T>::type> gr)
{
    using C = typename Compute<T>::type;
    if (batch_idle(g)) return;
    u = batch_at(u, g);
    f = batch_at(f, g);
    long t = xcd_block() * kBlock + threadIdx.x;
    const int my = g.ny - 2, mz = g.nz - 2;
    long total = (long)g.hx * my * (D == 3 ? mz : 1);
    if (t >= total) return;
    int h = (int)(t % g.hx);
    long r = t / g.hx;
    int pj = 1 + (int)(r % my);
    int pk = D == 3 ? 1 + (int)(r / my) : 0;
    int pi = 2 * h + ((colour + pj + pk + D) & 1);
    if (pi < 1 || pi > g.nx - 2) return;
    const T* __restrict__ o = u + (size_t)(colour ^ 1) * g.cs;
    size_t row = row_base(g, pj, pk);
    size_t ny = (size_t)g.hx, nz = g.ps;
    size_t self = (size_t)colour * g.cs + row + h;
    C xm = (C)o[row + ((pi - 1) >> 1)], xp = (C)o[row + ((pi + 1) >> 1)];
    C ym = (C)o[row - ny + h], yp = (C)o[row + ny + h];
    C zm = 0, zp = 0;
    if (D == 3) {
        zm = (C)o[row - nz + h];
        zp = (C)o[row + nz + h];
    }
    if (RULE) {
        const int Nx = g.nx - 2;
        if (pi == 1 || pi == Nx || pj == 1 || pj == my || (D == 3 && (pk == 1 || pk == mz))) {
            const C me = (C)u[self];
            rule_pair(pi, Nx, me, xm, xp, gr, 0);
            rule_pair(pj, my, me, ym, yp, gr, 1);
            if (D == 3) rule_pair(pk, mz, me, zm, zp, gr, 2);
        }
    }
    C s = xm + xp;
    s = s + ym;
    s = s + yp;
    if (D == 3) {
        s = s + zm;
        s = s + zp;
    }
    u[self] = (T)((s - h2 * (C)f[self]) * inv2d);
}


template <int D, typename T>
__global__ void __launch_bounds__(kBlock) k_smooth_fine(T* __restrict__ u, const T* __restrict__ f, SGrid g, int colour,
                                                        typename Compute<T>::type h2, typename Compute<T>::type inv2d)
{
    half_sweep_body<D, T, false>(u, f, g, colour, h2, inv2d, GRule<typename Compute<T>::type>{});
}

// 3-D level-0 half sweep marching along z.  A thread owns one compact (h, pj)
// position and walks kZChunk planes, keeping the other colour's values at
// planes pk-1, pk, pk+1 of its own column in registers: each value of the
// other colour is loaded once per chunk as the "plane above" and reused as the
// centre's x-neighbour and the next planes' z-neighbours.  Logical blocks run
// over the flattened (pj, h) plane fastest, so the blocks resident on one XCD
// cover adjacent rows of the same planes and the y-neighbour rows come from
// its L2.
// planes per thread on multigrid level 0 and on the coarse levels (4/4, 8/8,
// 8/4, 4/2, 4/1 measured at 514^3: 4/4 best)
constexpr int kZChunk0 = 4;
constexpr bool kDppExtra = true;  // pair sweep: extra x-neighbour from the adjacent lane
constexpr int kZChunk1 = 4;
constexpr int kZChunkSmall = 1;  // coarse levels of at most kSmallPlanes planes: more threads, shorter chains
constexpr int kSmallPlanes = 64;

// TAG 0: level 0 (ghost layer in memory); TAG 1: coarse levels, whose ghost
// values come from the rule (GRule) where a boundary point reads them.
template <typename T, int TAG>
__global__ void __launch_bounds__(kBlock) k_smooth_zmarch3(T* __restrict__ u, const T* __restrict__ f, SGrid g, int colour,
                                                           typename Compute<T>::type h2,
                                                           typename Compute<T>::type inv2d, int pblocks,
                                                           GRule<typename Compute<T>::type> gr)
{
    using C = typename Compute<T>::type;
    constexpr bool RULE = TAG >= 1;
    constexpr int kZChunk = TAG == 0 ? kZChunk0 : (TAG == 1 ? kZChunk1 : kZChunkSmall);
    constexpr int kZGroup = kZChunk;  // planes whose loads are issued together
    if (batch_idle(g)) return;
    u = batch_at(u, g);
    f = batch_at(f, g);
    const int mx = g.nx - 2, my = g.ny - 2, mz = g.nz - 2;
    const int lb = zmarch_block(TAG == 0 ? colour : 0);  // level 0: red half sweeps up, black down
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    // flat index over the whole (padded) plane: aligned wave segments
    const int pj = t / g.hx;
    const int h = t - pj * g.hx;
    if (pj < 1 || pj > my) return;
    const int k0 = 1 + zc * kZChunk;
    const int k1 = min(k0 + kZChunk - 1, mz);
    const size_t plane = g.ps;
    const size_t col = (size_t)pj * g.hx + h;  // offset of (h, pj) inside a plane
    const T* __restrict__ o = u + (size_t)(colour ^ 1) * g.cs;
    T* __restrict__ uc = u + (size_t)colour * g.cs;
    const T* __restrict__ fc = f + (size_t)colour * g.cs;
    C below = (C)o[(size_t)(k0 - 1) * plane + col];
    C cur = (C)o[(size_t)k0 * plane + col];
    int pk = k0;
    // groups of kZGroup planes: every load of the group is issued before the
    // first update so that each wave keeps many loads in flight.  Loads at
    // inactive (ghost) positions stay inside the arrays: h-1 / h+1 fall in the
    // neighbouring row of the same plane and f covers the whole padded grid.
    // level 0: the other colour's x-neighbour that is not the thread's own compact
    // slot (h + 1 for par 1, h - 1 for par 0) is the adjacent lane's value of the
    // same plane (flat numbering), moved by a DPP wave shift; only the wave's edge
    // lanes load it.  Lanes of other rows are used only for ghost points.  (On
    // the coarse levels the exchange measured slower and every lane loads.)
    constexpr bool XDPP = TAG == 0;
    const int lane = (int)(threadIdx.x & 63);
    const auto own_load = [&](int par) { return !XDPP || (par ? lane == 63 : lane == 0); };
    for (; pk + kZGroup - 1 <= k1; pk += kZGroup) {
        C ab[kZGroup], xo[kZGroup], ym[kZGroup], yp[kZGroup], fv[kZGroup];
#pragma unroll
        for (int q = 0; q < kZGroup; q++) {
            const size_t here = (size_t)(pk + q) * plane + col;
            const int par = (colour + pj + pk + q + 3) & 1;
            ab[q] = (C)o[here + plane];
            if (own_load(par)) xo[q] = (C)o[par ? here + 1 : here - 1];
            ym[q] = (C)o[here - g.hx];
            yp[q] = (C)o[here + g.hx];
            fv[q] = (C)fc[here];
        }
#pragma unroll
        for (int q = 0; q < kZGroup; q++) {
            const size_t here = (size_t)(pk + q) * plane + col;
            const int par = (colour + pj + pk + q + 3) & 1;
            const int pi = 2 * h + par;
            if constexpr (XDPP) {
                const C nb = par ? dpp_next(cur) : dpp_prev(cur);
                if (!own_load(par)) xo[q] = nb;
            }
            if (pi >= 1 && pi <= mx) {
                C xm = par ? cur : xo[q];
                C xp = par ? xo[q] : cur;
                C y0 = ym[q], y1 = yp[q], z0 = below, z1 = ab[q];
                if (RULE) {
                    const int kk = pk + q;
                    if (pi == 1 || pi == mx || pj == 1 || pj == my || kk == 1 || kk == mz) {
                        const C me = (C)uc[here];
                        rule_pair(pi, mx, me, xm, xp, gr, 0);
                        rule_pair(pj, my, me, y0, y1, gr, 1);
                        rule_pair(kk, mz, me, z0, z1, gr, 2);
                    }
                }
                C s = xm + xp;
                s = s + y0;
                s = s + y1;
                s = s + z0;
                s = s + z1;
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
        if (pi >= 1 && pi <= mx) {
            // x-neighbours pi-1, pi+1: compact h-1 and h (par 0) or h and h+1 (par 1)
            C xm = par ? cur : (C)o[here - 1];
            C xp = par ? (C)o[here + 1] : cur;
            C y0 = (C)o[here - g.hx], y1 = (C)o[here + g.hx], z0 = below, z1 = above;
            if (RULE) {
                if (pi == 1 || pi == mx || pj == 1 || pj == my || pk == 1 || pk == mz) {
                    const C me = (C)uc[here];
                    rule_pair(pi, mx, me, xm, xp, gr, 0);
                    rule_pair(pj, my, me, y0, y1, gr, 1);
                    rule_pair(pk, mz, me, z0, z1, gr, 2);
                }
            }
            C s = xm + xp;
            s = s + y0;
            s = s + y1;
            s = s + z0;
            s = s + z1;
            uc[here] = (T)((s - h2 * (C)fc[here]) * inv2d);
        }
        below = cur;
        cur = above;
    }
}

template <int D, typename T>
__global__ void __launch_bounds__(kBlock) k_half_sweep(T* __restrict__ u, const T* __restrict__ f, SGrid g, int colour,
                                                       typename Compute<T>::type h2, typename Compute<T>::type inv2d,
                                                       GRule<typename Compute<T>::type> gr)
{
    half_sweep_body<D, T, true>(u, f, g, colour, h2, inv2d, gr);
}

// FP32 sums of FP16 halves of packed 32-bit words in one v_fma_mix_f32 each
// (h * 1.0 + s with the FP16 operand converted exactly inside the instruction):
// the same single rounding as a conversion followed by an FP32 add, one
// instruction instead of two.  H selects the low (0) or high (1) half.
template <int H>
__device__ __forceinline__ float mix_add(float s, uint32_t w)
{
    float r;
    if constexpr (H == 0)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(s));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(s));
    return r;
}

// half HA of a plus half HB of b, both FP16, summed in FP32
template <int HA, int HB>
__device__ __forceinline__ float mix_add2(uint32_t a, uint32_t b)
{
    float r;
    if constexpr (HA == 0 && HB == 1)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    else if constexpr (HA == 1 && HB == 0)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    else if constexpr (HA == 0 && HB == 0)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Gauss-Seidel value of a point in storage type T from the sum s of its 2d
// neighbours: (s - h^2 f) / (2d) in the compute type C, rounded to T, written
// as k_smooth_zmarch3_pair writes it (there inline, so that the compiler keeps
// building the pair in one register for a 4-byte store).
template <typename T, typename C>
__device__ __forceinline__ T gs_value(C s, T fv, C h2, C inv2d)
{
    return (T)((s - h2 * (C)fv) * inv2d);
}

// Paired form of the level-0 z-march for 2- and 4-byte storage: a thread owns
// the two compact points h0 = 2 hp and h0 + 1 of a row and moves them with
// one 2-element load or store; the extra x-neighbour (h0 - 1 or h0 + 2) is a
// single load.  Same arithmetic, in the same order, as k_smooth_zmarch3.
// Requires an even row length hx (so pairs never straddle rows and stay
// aligned).
// SEED (1 or 2): the first black half sweep of a defect-correction step whose
// red points hold the result of a red half sweep from zero, e = (0 - h2 r) /
// (2d), which is not stored: the red values are formed from the defect f (red)
// here, in the same arithmetic (its ghost layer is zero, as is the
// correction's).  With SEED = 2 they are also stored, for a restriction that
// reads them next (one pre-smoothing sweep); with 1 a red half sweep rewrites
// them first.
template <typename T, int SEED = 0>
__global__ void __launch_bounds__(kSmoothPairBlock) k_smooth_zmarch3_pair(T* __restrict__ u, const T* __restrict__ f, SGrid g,
                                                                int colour, typename Compute<T>::type h2,
                                                                typename Compute<T>::type inv2d, int pblocks)
{
    using C = typename Compute<T>::type;
    const auto sv = [&](T v) -> T { return SEED ? (T)(((C)0 - h2 * (C)v) * inv2d) : v; };
    const auto sp = [&](Pair<T> v) -> Pair<T> {
        if (SEED) {
            v.a = sv(v.a);
            v.b = sv(v.b);
        }
        return v;
    };
    if (batch_idle(g)) return;
    u = batch_at(u, g);
    f = batch_at(f, g);
    const int my = g.ny - 2, mz = g.nz - 2;
    const int lb = zmarch_block(colour);  // red half sweeps up, black down
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kSmoothPairBlock + (int)threadIdx.x;
    // flat pair index over the whole (padded) plane: each wave covers 128
    // consecutive compact elements, an aligned segment; the ghost rows and the
    // plane padding have no work
    const int q = 2 * t;
    const int pj = q / g.hx;
    const int h0 = q - pj * g.hx;
    if (pj < 1 || pj > my) return;
    constexpr int kZChunk = kZChunk0;
    const int k0 = 1 + zc * kZChunk;
    const int k1 = min(k0 + kZChunk - 1, mz);
    const size_t plane = g.ps;
    const size_t col = (size_t)pj * g.hx + h0;
    const T* __restrict__ o = (SEED ? f : u) + (size_t)(colour ^ 1) * g.cs;
    T* __restrict__ uc = u + (size_t)colour * g.cs;
    T* __restrict__ uo = u + (size_t)(colour ^ 1) * g.cs;  // written with SEED = 2 only
    const T* __restrict__ fc = f + (size_t)colour * g.cs;
    Pair<T> below = sp(*(const Pair<T>*)(o + (size_t)(k0 - 1) * plane + col));
    Pair<T> cur = sp(*(const Pair<T>*)(o + (size_t)k0 * plane + col));
    auto step = [&](int pk, const Pair<T>& above, const Pair<T>& ym, const Pair<T>& yp, const Pair<T>& fv, T exh) {
        const C ex = (C)exh;
        const size_t here = (size_t)pk * plane + col;
        const int par = (colour + pj + pk + 3) & 1;
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
        C s0, s1;
        if constexpr (sizeof(T) == 2) {
            // the same sums on the packed FP16 words: x-neighbours are the
            // point's compact partner and the extra value (one rounding each)
            const uint32_t c = __builtin_bit_cast(uint32_t, cur);
            const uint32_t xw = __builtin_bit_cast(uint16_t, exh);
            s0 = mix_add2<0, 1>(c, par ? c : (xw << 16));  // a + (par ? b : extra)
            s1 = mix_add2<1, 0>(c, par ? xw : c);          // b + (par ? extra : a)
            const uint32_t wym = __builtin_bit_cast(uint32_t, ym), wyp = __builtin_bit_cast(uint32_t, yp);
            const uint32_t wbl = __builtin_bit_cast(uint32_t, below), wab = __builtin_bit_cast(uint32_t, above);
            s0 = mix_add<0>(s0, wym);
            s0 = mix_add<0>(s0, wyp);
            s0 = mix_add<0>(s0, wbl);
            s0 = mix_add<0>(s0, wab);
            s1 = mix_add<1>(s1, wym);
            s1 = mix_add<1>(s1, wyp);
            s1 = mix_add<1>(s1, wbl);
            s1 = mix_add<1>(s1, wab);
        } else {
            s0 = xm0 + xp0;
            s0 = s0 + (C)ym.a;
            s0 = s0 + (C)yp.a;
            s0 = s0 + (C)below.a;
            s0 = s0 + (C)above.a;
            s1 = xm1 + xp1;
            s1 = s1 + (C)ym.b;
            s1 = s1 + (C)yp.b;
            s1 = s1 + (C)below.b;
            s1 = s1 + (C)above.b;
        }
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
        // the pair's red values formed from the defect (0 on its ghost columns,
        // as the correction's ghost layer)
        if (SEED == 2) *(Pair<T>*)(uo + here) = cur;
        below = cur;
        cur = above;
    };
    // the extra x-neighbour stays inside the plane (neighbouring row at the row ends)
    auto extra = [&](int pk, size_t here) -> T { return sv(o[((colour + pj + pk + 3) & 1) ? here + 2 : here - 1]); };
    if (k1 - k0 + 1 == kZChunk) {
        // a full chunk: every load of its planes is issued before the first
        // update, so that each wave keeps ~20 loads in flight
        Pair<T> ab[kZChunk], ym[kZChunk], yp[kZChunk], fv[kZChunk];
        T ex[kZChunk];
        if constexpr (sizeof(T) <= 4 && kDppExtra) {
            // the extra x-neighbour of plane pk is an element of the neighbouring
            // lane's pair in the same plane (flat numbering: lane - 1 holds slots
            // h0 - 2, h0 - 1 and lane + 1 slots h0 + 2, h0 + 3), moved across lanes
            // with a DPP wave shift; only the wave's edge lanes, whose neighbour is
            // in another wave, load it
            const int lane = (int)(threadIdx.x & 63);
#pragma unroll
            for (int q = 0; q < kZChunk; q++) {
                const size_t here = (size_t)(k0 + q) * plane + col;
                ab[q] = sp(*(const Pair<T>*)(o + here + plane));
                ym[q] = sp(*(const Pair<T>*)(o + here - g.hx));
                yp[q] = sp(*(const Pair<T>*)(o + here + g.hx));
                fv[q] = *(const Pair<T>*)(fc + here);
                const int par = (colour + pj + k0 + q + 3) & 1;
                if (par ? lane == 63 : lane == 0) ex[q] = extra(k0 + q, here);
            }
#pragma unroll
            for (int q = 0; q < kZChunk; q++) {
                const int par = (colour + pj + k0 + q + 3) & 1;
                T xv;
                if constexpr (sizeof(T) == 2) {
                    const unsigned w = __builtin_bit_cast(uint32_t, cur);
                    xv = __builtin_bit_cast(T, par ? (uint16_t)(dpp_next(w) & 0xffffu) : (uint16_t)(dpp_prev(w) >> 16));
                } else {
                    xv = par ? dpp_next(cur.a) : dpp_prev(cur.b);
                }
                const T e = (par ? lane == 63 : lane == 0) ? ex[q] : xv;
                step(k0 + q, ab[q], ym[q], yp[q], fv[q], e);
            }
            return;
        }
#pragma unroll
        for (int q = 0; q < kZChunk; q++) {
            const size_t here = (size_t)(k0 + q) * plane + col;
            ab[q] = sp(*(const Pair<T>*)(o + here + plane));
            ym[q] = sp(*(const Pair<T>*)(o + here - g.hx));
            yp[q] = sp(*(const Pair<T>*)(o + here + g.hx));
            fv[q] = *(const Pair<T>*)(fc + here);
            ex[q] = extra(k0 + q, here);
        }
#pragma unroll
        for (int q = 0; q < kZChunk; q++) step(k0 + q, ab[q], ym[q], yp[q], fv[q], ex[q]);
        return;
    }
    for (int pk = k0; pk <= k1; pk++) {
        const size_t here = (size_t)pk * plane + col;
        step(pk, sp(*(const Pair<T>*)(o + here + plane)), sp(*(const Pair<T>*)(o + here - g.hx)),
             sp(*(const Pair<T>*)(o + here + g.hx)), *(const Pair<T>*)(fc + here), extra(pk, here));
    }
}

// ------------------------------------------------------------------ full sweep
// One red-black sweep of multigrid level 0 of a 3-D level (ghost layer in
// memory) in a single pass, from the potential P into a second array Q whose
// ghost layer is P's: red points first, then black, each with the arithmetic
// of the half sweeps above, so Q ends up holding what the two half sweeps in
// place would leave (bit for bit).  The black update of a point reads the new
// red values of the rows beside it, which belong to other threads, so a
// thread relaxes the red points of its G rows and of one row on either side of
// them, and of one plane beyond either end of its chunk of planes, and keeps
// them in registers; it stores only its own.  The x-neighbour in the other
// compact slot comes from the adjacent lane by a DPP shift; a wave owns the
// kFsOwn columns between its first and its last lane, which only supply red
// values to their neighbours.  No thread reads what another writes.
// MODE & kFsResIn: also max |f - lap P| over the red points owned.  P's black
// points are exact (their residual was taken by the black update of the sweep
// that produced P, MODE & kFsResOut), so together they give P's residual norm,
// with the operations of the residual pass (k_dc_outer3_pair) per point.
constexpr int kFsBlock = 256;
constexpr int kFsOwn = 62;   // columns a wave owns (lanes 1..62)
constexpr int kFsRows = 3;   // rows per thread (1, 2, 3, 4 measured: 3 fastest)
constexpr int kFsChunk = 16; // planes per thread
constexpr int kFsResIn = kSweepResIn, kFsResOut = kSweepResOut;

template <typename T, int G, int KCH, int MODE>
__global__ void __launch_bounds__(kFsBlock) k_full_sweep3(const T* __restrict__ P, T* __restrict__ Q,
                                                          const T* __restrict__ f, SGrid g, double h2, double inv2d,
                                                          double inv_h2, int nrg, int wblocks, int rev,
                                                          unsigned long long* maxbits)
{
    using C = typename Compute<T>::type;
    constexpr int R = G + 2;  // rows whose red points the thread relaxes
    const C h2c = (C)h2, inv2dc = (C)inv2d;
    const int mx = g.nx - 2, my = g.ny - 2, mz = g.nz - 2;
    const int lb = zmarch_block(rev);
    const int zc = lb / wblocks;
    const long wave = (long)(lb - zc * wblocks) * (kFsBlock / 64) + (threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const long total = (long)nrg * g.hx;
    const long t = wave * kFsOwn + lane - 1;
    const bool owner = lane >= 1 && lane <= kFsOwn && t >= 0 && t < total;
    const long tc = t < 0 ? 0 : (t >= total ? total - 1 : t);
    const int rg = (int)(tc / g.hx);
    const int h = (int)(tc - (long)rg * g.hx);
    const int j0 = 1 + G * rg;  // first own row
    const int k0 = 1 + zc * KCH;
    const int k1 = min(k0 + KCH - 1, mz);
    const size_t cs = g.cs, ps = g.ps;
    const int hm = h > 0 ? h - 1 : 0, hp = h + 1 < g.hx ? h + 1 : g.hx - 1;
    // element offsets inside a plane (32-bit; plane bases are uniform) of the red
    // rows j0-1 .. j0+G and of the rows j0-2 and j0+G+1 (rows clamped into the
    // array: values of rows outside it are never used)
    auto rowc = [&](int r) { return r < 0 ? 0 : (r > my + 1 ? my + 1 : r); };
    auto planec = [&](int k) { return (size_t)(k < 0 ? 0 : (k > mz + 1 ? mz + 1 : k)) * ps; };
    unsigned ro[R];
#pragma unroll
    for (int i = 0; i < R; i++) ro[i] = (unsigned)(rowc(j0 - 1 + i) * g.hx + h);
    const unsigned ry0 = (unsigned)(rowc(j0 - 2) * g.hx + h), ry1 = (unsigned)(rowc(j0 + G + 1) * g.hx + h);
    const int dm = hm - h, dp = hp - h;  // the other compact slot of the edge lanes
    const T* __restrict__ Pr = P;
    const T* __restrict__ Pb = P + cs;
    const T* __restrict__ fr = f;
    const T* __restrict__ fb = f + cs;
    T* __restrict__ Qr = Q;
    T* __restrict__ Qb = Q + cs;
    C b0[R], b1[R];  // P's black values of the red rows at planes k - 1 and k
    C rn[R];         // new red values at plane k - 1
    C rp[G];         // new red values of the own rows at plane k - 2
    {
        const T* __restrict__ pa = Pb + planec(k0 - 2);
        const T* __restrict__ pb = Pb + planec(k0 - 1);
#pragma unroll
        for (int i = 0; i < R; i++) {
            b0[i] = (C)pa[ro[i]];
            b1[i] = (C)pb[ro[i]];
        }
    }
#pragma unroll
    for (int i = 0; i < R; i++) rn[i] = (C)0;
#pragma unroll
    for (int i = 0; i < G; i++) rp[i] = (C)0;
    unsigned long long best = 0;
    // the loads of step k (red points of plane k, black points of plane k - 1),
    // all issued before the step computes
    struct Loads {
        C ba[R], fv[R], ex[R], gh[R], fbv[G], prv[G], y0, y1;
    };
    auto load = [&](int k, Loads& L) {
        const T* __restrict__ pbk = Pb + planec(k);
        const T* __restrict__ pba = Pb + planec(k + 1);
        const T* __restrict__ prk = Pr + planec(k);
        const T* __restrict__ frk = fr + planec(k);
        const T* __restrict__ fbk = fb + planec(k - 1);
        const bool kact = k >= 1 && k <= mz;
        L.y0 = (C)pbk[ry0];
        L.y1 = (C)pbk[ry1];
#pragma unroll
        for (int i = 0; i < R; i++) {
            const int r = j0 - 1 + i;
            const int par = (r + k + 3) & 1;  // red point pi = 2h + par
            const int pi = 2 * h + par;
            L.ba[i] = (C)pba[ro[i]];
            L.fv[i] = (C)frk[ro[i]];
            L.ex[i] = (C)0;
            if (par ? lane == 63 : lane == 0) L.ex[i] = (C)pbk[(int)ro[i] + (par ? dp : dm)];
            L.gh[i] = (C)0;
            const bool act = kact && r >= 1 && r <= my && pi >= 1 && pi <= mx;
            if (!act) L.gh[i] = (C)prk[ro[i]];
        }
        const bool bstep = k - 1 >= k0;
        const bool red_own = k >= k0 && k <= k1;
#pragma unroll
        for (int i = 0; i < G; i++) {
            L.fbv[i] = bstep ? (C)fbk[ro[i + 1]] : (C)0;
            L.prv[i] = ((MODE & kFsResIn) && red_own) ? (C)prk[ro[i + 1]] : (C)0;
        }
    };
    auto step = [&](int k, const Loads& L) {
        const size_t pk = planec(k), pkb = planec(k - 1);
        const bool red_own = k >= k0 && k <= k1;
        const bool bstep = k - 1 >= k0;
        const bool kact = k >= 1 && k <= mz;
        // red points of plane k
        C rk[R];
#pragma unroll
        for (int i = 0; i < R; i++) {
            const int r = j0 - 1 + i;
            const int par = (r + k + 3) & 1;
            const int pi = 2 * h + par;
            const C sh = par ? dpp_next(b1[i]) : dpp_prev(b1[i]);
            const C e = (par ? lane == 63 : lane == 0) ? L.ex[i] : sh;
            const C xm = par ? b1[i] : e;
            const C xp = par ? e : b1[i];
            const C y0 = i == 0 ? L.y0 : b1[i - 1];
            const C y1 = i == R - 1 ? L.y1 : b1[i + 1];
            C s = xm + xp;
            s = s + y0;
            s = s + y1;
            s = s + b0[i];
            s = s + L.ba[i];
            const bool act = kact && r >= 1 && r <= my && pi >= 1 && pi <= mx;
            const T v = (T)((s - h2c * L.fv[i]) * inv2dc);
            rk[i] = act ? (C)v : L.gh[i];
            if (i >= 1 && i <= G && red_own && owner && act) {
                (Qr + pk)[ro[i]] = v;
                if (MODE & kFsResIn) {
                    const double res = resid(L.fv[i], s, L.prv[i - 1], 6.0, inv_h2);
                    const unsigned long long bb = abs_bits(res);
                    best = bb > best ? bb : best;
                }
            }
        }
        // black points of plane k - 1
        if (bstep) {
#pragma unroll
            for (int i = 0; i < G; i++) {
                const int r = j0 + i;
                const int kb = k - 1;
                const int par = (r + kb + 4) & 1;
                const int pi = 2 * h + par;
                const C sh = par ? dpp_next(rn[i + 1]) : dpp_prev(rn[i + 1]);
                const C xm = par ? rn[i + 1] : sh;
                const C xp = par ? sh : rn[i + 1];
                C s = xm + xp;
                s = s + rn[i];
                s = s + rn[i + 2];
                s = s + rp[i];
                s = s + rk[i + 1];
                const T v = (T)((s - h2c * L.fbv[i]) * inv2dc);
                if (owner && r <= my && pi >= 1 && pi <= mx) {
                    (Qb + pkb)[ro[i + 1]] = v;
                    if (MODE & kFsResOut) {
                        const double res = resid(L.fbv[i], s, (C)v, 6.0, inv_h2);
                        const unsigned long long bb = abs_bits(res);
                        best = bb > best ? bb : best;
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < G; i++) rp[i] = rn[i + 1];
#pragma unroll
        for (int i = 0; i < R; i++) {
            rn[i] = rk[i];
            b0[i] = b1[i];
            b1[i] = L.ba[i];
        }
    };
    for (int k = k0 - 1; k <= k1 + 1; k++) {
        Loads L;
        load(k, L);
        step(k, L);
    }
    if (MODE) block_max_to(best, maxbits);
}

// Paired form of k_full_sweep3 (even row length hx): a lane owns the compact
// points h0 = 2 hp and h0 + 1 of its rows, moves each pair with one 16-byte
// access, and takes the compact slot past its pair (h0 - 1 or h0 + 2) from the
// adjacent lane's pair; a wave owns the kFsOwn pairs between its first and
// last lane.  Same arithmetic per point, in the same order, as the single form
// and the paired half sweep.
constexpr int kFsPairRows = 5;    // rows per thread (1..8 measured at 514^3: 5 fastest)
constexpr int kFsPairChunk = 16;  // planes per thread

template <typename T, int G, int KCH, int MODE>
__global__ void __launch_bounds__(kFsBlock) k_full_sweep3_pair(const T* __restrict__ P, T* __restrict__ Q,
                                                               const T* __restrict__ f, SGrid g, double h2,
                                                               double inv2d, double inv_h2, int nrg, int wblocks,
                                                               int rev, unsigned long long* maxbits)
{
    using C = typename Compute<T>::type;
    using PT = Pair<T>;
    constexpr int R = G + 2;
    const C h2c = (C)h2, inv2dc = (C)inv2d;
    const int mx = g.nx - 2, my = g.ny - 2, mz = g.nz - 2;
    const int lb = zmarch_block(rev);
    const int zc = lb / wblocks;
    const long wave = (long)(lb - zc * wblocks) * (kFsBlock / 64) + (threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int hp2 = g.hx / 2;  // pairs per row
    const long total = (long)nrg * hp2;
    const long t = wave * kFsOwn + lane - 1;
    const bool owner = lane >= 1 && lane <= kFsOwn && t >= 0 && t < total;
    const long tc = t < 0 ? 0 : (t >= total ? total - 1 : t);
    const int rg = (int)(tc / hp2);
    const int h0 = 2 * (int)(tc - (long)rg * hp2);
    const int j0 = 1 + G * rg;
    const int k0 = 1 + zc * KCH;
    const int k1 = min(k0 + KCH - 1, mz);
    const size_t cs = g.cs, ps = g.ps;
    auto rowc = [&](int r) { return r < 0 ? 0 : (r > my + 1 ? my + 1 : r); };
    auto planec = [&](int k) { return (size_t)(k < 0 ? 0 : (k > mz + 1 ? mz + 1 : k)) * ps; };
    unsigned ro[R];
#pragma unroll
    for (int i = 0; i < R; i++) ro[i] = (unsigned)(rowc(j0 - 1 + i) * g.hx + h0);
    const unsigned ry0 = (unsigned)(rowc(j0 - 2) * g.hx + h0), ry1 = (unsigned)(rowc(j0 + G + 1) * g.hx + h0);
    const T* __restrict__ Pr = P;
    const T* __restrict__ Pb = P + cs;
    const T* __restrict__ fr = f;
    const T* __restrict__ fb = f + cs;
    T* __restrict__ Qr = Q;
    T* __restrict__ Qb = Q + cs;
    auto ldp = [](const T* p, unsigned o) { return *(const PT*)(p + o); };
    PT b0[R], b1[R];  // P's black pairs of the red rows at planes k - 1 and k
    PT rn[R];         // new red pairs at plane k - 1
    PT rp[G];         // new red pairs of the own rows at plane k - 2
    {
        const T* pa = Pb + planec(k0 - 2);
        const T* pb = Pb + planec(k0 - 1);
#pragma unroll
        for (int i = 0; i < R; i++) {
            b0[i] = ldp(pa, ro[i]);
            b1[i] = ldp(pb, ro[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < R; i++) rn[i] = PT{(T)0, (T)0};
#pragma unroll
    for (int i = 0; i < G; i++) rp[i] = PT{(T)0, (T)0};
    unsigned long long best = 0;
    auto take = [&](unsigned long long b) { best = b > best ? b : best; };
    for (int k = k0 - 1; k <= k1 + 1; k++) {
        const T* __restrict__ pbk = Pb + planec(k);
        const T* __restrict__ pba = Pb + planec(k + 1);
        const T* __restrict__ prk = Pr + planec(k);
        const T* __restrict__ frk = fr + planec(k);
        const T* __restrict__ fbk = fb + planec(k - 1);
        const bool kact = k >= 1 && k <= mz;
        const bool red_own = k >= k0 && k <= k1;
        const bool bstep = k - 1 >= k0;
        // every load of the step first
        PT ba[R], fv[R], gh[R], fbv[G], prv[G];
        T ex[R];
        const PT y0v = ldp(pbk, ry0), y1v = ldp(pbk, ry1);
#pragma unroll
        for (int i = 0; i < R; i++) {
            const int r = j0 - 1 + i;
            const int par = (r + k + 3) & 1;  // red points pi = 2 h0 + par, + 2
            const int pi0 = 2 * h0 + par;
            ba[i] = ldp(pba, ro[i]);
            fv[i] = ldp(frk, ro[i]);
            const bool ract = kact && r >= 1 && r <= my;
            // the slot past the pair: the adjacent lane's, loaded by the wave's edge
            // lanes only where the point reading it is active (so it lies in the row)
            ex[i] = (T)0;
            if (par ? (lane == 63 && ract && pi0 + 2 <= mx) : (lane == 0 && ract && pi0 >= 1))
                ex[i] = pbk[(int)ro[i] + (par ? 2 : -1)];
            gh[i] = PT{(T)0, (T)0};
            if (!(ract && pi0 >= 1 && pi0 + 2 <= mx)) gh[i] = ldp(prk, ro[i]);
        }
#pragma unroll
        for (int i = 0; i < G; i++) {
            fbv[i] = bstep ? ldp(fbk, ro[i + 1]) : PT{(T)0, (T)0};
            prv[i] = ((MODE & kFsResIn) && red_own) ? ldp(prk, ro[i + 1]) : PT{(T)0, (T)0};
        }
        // red points of plane k
        PT rk[R];
#pragma unroll
        for (int i = 0; i < R; i++) {
            const int r = j0 - 1 + i;
            const int par = (r + k + 3) & 1;
            const int pi0 = 2 * h0 + par;
            const C nx = (C)dpp_next(b1[i].a), pv = (C)dpp_prev(b1[i].b);
            const C e = (par ? lane == 63 : lane == 0) ? (C)ex[i] : (par ? nx : pv);
            C xm0, xp0, xm1, xp1;
            if (par) {
                xm0 = (C)b1[i].a;
                xp0 = (C)b1[i].b;
                xm1 = (C)b1[i].b;
                xp1 = e;
            } else {
                xm0 = e;
                xp0 = (C)b1[i].a;
                xm1 = (C)b1[i].a;
                xp1 = (C)b1[i].b;
            }
            const PT y0 = i == 0 ? y0v : b1[i - 1];
            const PT y1 = i == R - 1 ? y1v : b1[i + 1];
            C s0 = xm0 + xp0;
            s0 = s0 + (C)y0.a;
            s0 = s0 + (C)y1.a;
            s0 = s0 + (C)b0[i].a;
            s0 = s0 + (C)ba[i].a;
            C s1 = xm1 + xp1;
            s1 = s1 + (C)y0.b;
            s1 = s1 + (C)y1.b;
            s1 = s1 + (C)b0[i].b;
            s1 = s1 + (C)ba[i].b;
            const bool ract = kact && r >= 1 && r <= my;
            const bool a0 = ract && pi0 >= 1 && pi0 <= mx, a1 = ract && pi0 + 2 <= mx;
            const T v0 = (T)((s0 - h2c * (C)fv[i].a) * inv2dc), v1 = (T)((s1 - h2c * (C)fv[i].b) * inv2dc);
            rk[i].a = a0 ? v0 : gh[i].a;
            rk[i].b = a1 ? v1 : gh[i].b;
            if (i >= 1 && i <= G && red_own && owner) {
                T* q = Qr + planec(k) + ro[i];
                if (a0 && a1)
                    *(PT*)q = PT{v0, v1};
                else {
                    if (a0) q[0] = v0;
                    if (a1) q[1] = v1;
                }
                if (MODE & kFsResIn) {
                    if (a0) take(abs_bits(resid((double)fv[i].a, (double)s0, (double)prv[i - 1].a, 6.0, inv_h2)));
                    if (a1) take(abs_bits(resid((double)fv[i].b, (double)s1, (double)prv[i - 1].b, 6.0, inv_h2)));
                }
            }
        }
        // black points of plane k - 1
        if (bstep) {
#pragma unroll
            for (int i = 0; i < G; i++) {
                const int r = j0 + i;
                const int kb = k - 1;
                const int par = (r + kb + 4) & 1;
                const int pi0 = 2 * h0 + par;
                const PT cur = rn[i + 1];
                const C nx = (C)dpp_next(cur.a), pv = (C)dpp_prev(cur.b);
                C xm0, xp0, xm1, xp1;
                if (par) {
                    xm0 = (C)cur.a;
                    xp0 = (C)cur.b;
                    xm1 = (C)cur.b;
                    xp1 = nx;
                } else {
                    xm0 = pv;
                    xp0 = (C)cur.a;
                    xm1 = (C)cur.a;
                    xp1 = (C)cur.b;
                }
                C s0 = xm0 + xp0;
                s0 = s0 + (C)rn[i].a;
                s0 = s0 + (C)rn[i + 2].a;
                s0 = s0 + (C)rp[i].a;
                s0 = s0 + (C)rk[i + 1].a;
                C s1 = xm1 + xp1;
                s1 = s1 + (C)rn[i].b;
                s1 = s1 + (C)rn[i + 2].b;
                s1 = s1 + (C)rp[i].b;
                s1 = s1 + (C)rk[i + 1].b;
                const T v0 = (T)((s0 - h2c * (C)fbv[i].a) * inv2dc), v1 = (T)((s1 - h2c * (C)fbv[i].b) * inv2dc);
                const bool a0 = owner && r <= my && pi0 >= 1 && pi0 <= mx, a1 = owner && r <= my && pi0 + 2 <= mx;
                T* q = Qb + planec(kb) + ro[i + 1];
                if (a0 && a1)
                    *(PT*)q = PT{v0, v1};
                else {
                    if (a0) q[0] = v0;
                    if (a1) q[1] = v1;
                }
                if (MODE & kFsResOut) {
                    if (a0) take(abs_bits(resid((double)fbv[i].a, (double)s0, (double)v0, 6.0, inv_h2)));
                    if (a1) take(abs_bits(resid((double)fbv[i].b, (double)s1, (double)v1, 6.0, inv_h2)));
                }
            }
        }
#pragma unroll
        for (int i = 0; i < G; i++) rp[i] = rn[i + 1];
#pragma unroll
        for (int i = 0; i < R; i++) {
            rn[i] = rk[i];
            b0[i] = b1[i];
            b1[i] = ba[i];
        }
    }
    if (MODE) block_max_to(best, maxbits);
}

// Coarse right-hand side and correction of one coarse point.  With seed_h2 > 0
// the correction is not cleared but set to the result of the coarse level's
// first red half sweep from zero, (0 - h^2 f) / (2d) on red points (black
// neighbours and rule ghosts are all zero then), in the sweep's arithmetic, so
// that sweep is not launched; black points get 0.
template <int D, typename TC, typename C>
__device__ __forceinline__ void coarse_out(TC* __restrict__ fc, TC* __restrict__ ec, size_t q, int I, int J, int K, C val,
                                           C seed_h2, C inv2d)
{
    const TC fv = (TC)val;
    fc[q] = fv;
    TC e = (TC)0;
    if (seed_h2 > (C)0 && colour_of<D>(I, J, K) == 0) e = (TC)(((C)0 - seed_h2 * (C)fv) * inv2d);
    ec[q] = e;
}

// Residual r = f - lap(u) on the 2^d children of each coarse active point and
// their mean (eqn:restriction2D/3D) into the coarse right-hand side, times
// out_scale (1 except below a scaled level-0 defect problem); children beyond
// the fine active range count as zero.  Also clears the coarse correction.
// TF: fine storage, TC: coarse storage; RULE: the fine level is a coarse
// multigrid level whose ghost values come from its rule.
template <int D, typename TF, typename TC, bool RULE>
__global__ void __launch_bounds__(kBlock) k_resid_restrict(const TF* __restrict__ u, const TF* __restrict__ f, SGrid gf,
                                                           typename Compute<TC>::type inv_h2,
                                                           typename Compute<TC>::type out_scale, SGrid gc,
                                                           TC* __restrict__ fc, TC* __restrict__ ec,
                                                           GRule<typename Compute<TC>::type> gr,
                                                           typename Compute<TC>::type seed_h2,
                                                           typename Compute<TC>::type inv2d)
{
    using C = typename Compute<TC>::type;
    if (batch_idle(gf)) return;
    u = batch_at(u, gf);
    f = batch_at(f, gf);
    fc = batch_at(fc, gc);
    ec = batch_at(ec, gc);
    const int Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    const int Nfx = gf.nx - 2, Nfy = gf.ny - 2, Nfz = gf.nz - 2;
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = D == 3 ? (long)Ncx * Ncy * Ncz : (long)Ncx * Ncy;
    if (t >= total) return;
    int I = 1 + (int)(t % Ncx);
    long r = t / Ncx;
    int J = 1 + (int)(r % Ncy);
    int K = D == 3 ? 1 + (int)(r / Ncy) : 0;
    C sum = 0;
    int k0 = D == 3 ? 2 * K - 1 : 0, k1 = D == 3 ? 2 * K : 0;
    for (int k = k0; k <= k1; k++)
        for (int j = 2 * J - 1; j <= 2 * J; j++)
            for (int i = 2 * I - 1; i <= 2 * I; i++) {
                if (i > Nfx || j > Nfy || (D == 3 && k > Nfz)) continue;
                C xm = (C)at<D>(u, gf, i - 1, j, k), xp = (C)at<D>(u, gf, i + 1, j, k);
                C ym = (C)at<D>(u, gf, i, j - 1, k), yp = (C)at<D>(u, gf, i, j + 1, k);
                C zm = 0, zp = 0;
                if (D == 3) {
                    zm = (C)at<D>(u, gf, i, j, k - 1);
                    zp = (C)at<D>(u, gf, i, j, k + 1);
                }
                C uc = (C)at<D>(u, gf, i, j, k);
                if (RULE) {
                    rule_pair(i, Nfx, uc, xm, xp, gr, 0);
                    rule_pair(j, Nfy, uc, ym, yp, gr, 1);
                    if (D == 3) rule_pair(k, Nfz, uc, zm, zp, gr, 2);
                }
                C s = xm + xp;
                s = s + ym;
                s = s + yp;
                if (D == 3) {
                    s = s + zm;
                    s = s + zp;
                }
                sum += (C)at<D>(f, gf, i, j, k) - (s - (C)(2 * D) * uc) * inv_h2;
            }
    size_t pc = pos<D, TC>(gc, I, J, K);
    coarse_out<D, TC, C>(fc, ec, pc, I, J, K, sum * ((C)(D == 3 ? 0.125 : 0.25) * out_scale), seed_h2, inv2d);
}

// 3-D restriction marching along the coarse z axis: a thread owns one coarse
// column (I, J) and a chunk of coarse planes K.  For each fine plane it loads
// the 2 x 2 children of its column and their x/y neighbours (a cross of 12
// values) once; the z neighbours of a child plane are the centres of the
// planes before and after it, kept in registers.  Per child and in the sum
// over children the arithmetic and order are those of k_resid_restrict.
// Fine indices beyond N_f + 1 (beside children past the active range, which
// count as zero) are clamped into the array and never used.
template <typename TF, typename TC, bool RULE>
__global__ void __launch_bounds__(kBlock) k_restrict3_zm(const TF* __restrict__ u, const TF* __restrict__ f, SGrid gf,
                                                         typename Compute<TC>::type inv_h2,
                                                         typename Compute<TC>::type out_scale, SGrid gc,
                                                         TC* __restrict__ fc, TC* __restrict__ ec,
                                                         GRule<typename Compute<TC>::type> gr, int pblocks, int kch,
                                                         typename Compute<TC>::type seed_h2,
                                                         typename Compute<TC>::type inv2d)
{
    using C = typename Compute<TC>::type;
    if (batch_idle(gf)) return;
    u = batch_at(u, gf);
    f = batch_at(f, gf);
    fc = batch_at(fc, gc);
    ec = batch_at(ec, gc);
    const int Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    const int Nfx = gf.nx - 2, Nfy = gf.ny - 2, Nfz = gf.nz - 2;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    if (t >= (long)Ncx * Ncy) return;
    const int I = 1 + (int)(t % Ncx), J = 1 + (int)(t / Ncx);
    const int K0 = 1 + zc * kch;
    const int K1 = min(K0 + kch - 1, Ncz);
    auto clx = [&](int a) { return a > Nfx + 1 ? Nfx + 1 : a; };
    auto cly = [&](int a) { return a > Nfy + 1 ? Nfy + 1 : a; };
    auto cl = [&](int a) { return a > Nfz + 1 ? Nfz + 1 : a; };
    int xi[4], yj[4];
    for (int a = 0; a < 4; a++) {
        xi[a] = clx(2 * I - 2 + a);
        yj[a] = cly(2 * J - 2 + a);
    }
    // cross of fine plane k: P[r][c] = u(2I-2+c, 2J-2+r, k); the corners are not loaded
    auto load_cross = [&](int k, C (&P)[4][4]) {
        const int kk = cl(k);
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 4; c++) {
                if ((r == 0 || r == 3) && (c == 0 || c == 3)) continue;
                P[r][c] = (C)at<3>(u, gf, xi[c], yj[r], kk);
            }
    };
    C pc[2][2];       // centres of the plane below the current pair
    C p1[4][4], p2[4][4], p3[4][4];
    {
        const int kk = cl(2 * K0 - 2);
        for (int r = 0; r < 2; r++)
            for (int c = 0; c < 2; c++) pc[r][c] = (C)at<3>(u, gf, xi[1 + c], yj[1 + r], kk);
    }
    load_cross(2 * K0 - 1, p1);
    for (int K = K0; K <= K1; K++) {
        load_cross(2 * K, p2);
        load_cross(2 * K + 1, p3);
        C fv[2][2][2];
#pragma unroll
        for (int dz = 0; dz < 2; dz++)
#pragma unroll
            for (int dy = 0; dy < 2; dy++)
#pragma unroll
                for (int dx = 0; dx < 2; dx++)
                    fv[dz][dy][dx] = (C)at<3>(f, gf, xi[1 + dx], yj[1 + dy], cl(2 * K - 1 + dz));
        C sum = 0;
#pragma unroll
        for (int dz = 0; dz < 2; dz++) {
            const int k = 2 * K - 1 + dz;
            if (k > Nfz) continue;
#pragma unroll
            for (int dy = 0; dy < 2; dy++) {
                const int j = 2 * J - 1 + dy;
                if (j > Nfy) continue;
#pragma unroll
                for (int dx = 0; dx < 2; dx++) {
                    const int i = 2 * I - 1 + dx;
                    if (i > Nfx) continue;
                    const C(&P)[4][4] = dz ? p2 : p1;
                    const C uc = P[1 + dy][1 + dx];
                    C xm = P[1 + dy][dx], xp = P[1 + dy][2 + dx];
                    C ym = P[dy][1 + dx], yp = P[2 + dy][1 + dx];
                    C zm = dz ? p1[1 + dy][1 + dx] : pc[dy][dx];
                    C zp = dz ? p3[1 + dy][1 + dx] : p2[1 + dy][1 + dx];
                    if (RULE) {
                        rule_pair(i, Nfx, uc, xm, xp, gr, 0);
                        rule_pair(j, Nfy, uc, ym, yp, gr, 1);
                        rule_pair(k, Nfz, uc, zm, zp, gr, 2);
                    }
                    C s = xm + xp;
                    s = s + ym;
                    s = s + yp;
                    s = s + zm;
                    s = s + zp;
                    sum += fv[dz][dy][dx] - (s - (C)6 * uc) * inv_h2;
                }
            }
        }
        const size_t q = pos<3, TC>(gc, I, J, K);
        coarse_out<3, TC, C>(fc, ec, q, I, J, K, sum * ((C)0.125 * out_scale), seed_h2, inv2d);
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int c = 0; c < 2; c++) pc[r][c] = p2[1 + r][1 + c];
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 4; c++) p1[r][c] = p3[r][c];
    }
}

// Residual and restriction out of multigrid level 0 (ghost layer in memory),
// the z-march of k_restrict3_zm (thread per coarse column (I, J), a chunk of
// coarse planes, the 12-point cross of each fine plane loaded once) with every
// address split into a uniform part and one per-lane offset: the fine points a
// thread reads are (2I - 2 + c, 2J - 2 + r, k), whose colour
// (c + r + k + 1) & 1 and in-plane offset r hx + (c >> 1) beyond the lane's
// base (2J - 2) hx + I - 1 are the same for every lane of the block (the chunk,
// hence k, is uniform).  So each load is a scalar pointer plus the lane's fixed
// byte offset, with no per-load address arithmetic.  Same arithmetic in the
// same order as k_restrict3_zm.  Requires N_f = 2 N_c along every axis (every
// child active) and arrays of fewer than 2^31 bytes.
template <typename TF, typename TC>
__global__ void __launch_bounds__(kBlock) k_restrict3_l0(const TF* __restrict__ u, const TF* __restrict__ f, SGrid gf,
                                                          typename Compute<TC>::type inv_h2,
                                                          typename Compute<TC>::type out_scale, SGrid gc,
                                                          TC* __restrict__ fc, TC* __restrict__ ec, int pblocks, int kch,
                                                          typename Compute<TC>::type seed_h2,
                                                          typename Compute<TC>::type inv2d)
{
    using C = typename Compute<TC>::type;
    if (batch_idle(gf)) return;
    u = batch_at(u, gf);
    f = batch_at(f, gf);
    fc = batch_at(fc, gc);
    ec = batch_at(ec, gc);
    const int Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    if (t >= Ncx * Ncy) return;
    const int I = 1 + t % Ncx, J = 1 + t / Ncx;
    const int K0 = 1 + zc * kch;
    const int K1 = min(K0 + kch - 1, Ncz);
    const unsigned boff = (unsigned)(((2 * J - 2) * gf.hx + (I - 1)) * (int)sizeof(TF));
    const size_t fplane = gf.ps;
    // value at (2I - 2 + c, 2J - 2 + r, k) of array a
    auto ld = [&](const TF* __restrict__ a, int c, int r, int k) -> C {
        const TF* p = a + (size_t)k * fplane + (((c + r + k + 1) & 1) ? gf.cs : 0) + (size_t)r * gf.hx + (c >> 1);
        return (C) * (const TF*)((const char*)p + boff);
    };
    // cross of fine plane k: P[r][c] = u(2I-2+c, 2J-2+r, k); the corners are not loaded
    auto load_cross = [&](int k, C (&P)[4][4]) {
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 4; c++) {
                if ((r == 0 || r == 3) && (c == 0 || c == 3)) continue;
                P[r][c] = ld(u, c, r, k);
            }
    };
    C pc[2][2];  // centres of the plane below the current pair
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
        for (int c = 0; c < 2; c++) pc[r][c] = ld(u, 1 + c, 1 + r, 2 * K0 - 2);
    C p1[4][4], p2[4][4], p3[4][4];
    load_cross(2 * K0 - 1, p1);
    for (int K = K0; K <= K1; K++) {
        load_cross(2 * K, p2);
        load_cross(2 * K + 1, p3);
        C fv[2][2][2];
#pragma unroll
        for (int dz = 0; dz < 2; dz++)
#pragma unroll
            for (int dy = 0; dy < 2; dy++)
#pragma unroll
                for (int dx = 0; dx < 2; dx++) fv[dz][dy][dx] = ld(f, 1 + dx, 1 + dy, 2 * K - 1 + dz);
        C sum = 0;
#pragma unroll
        for (int dz = 0; dz < 2; dz++) {
#pragma unroll
            for (int dy = 0; dy < 2; dy++) {
#pragma unroll
                for (int dx = 0; dx < 2; dx++) {
                    const C(&P)[4][4] = dz ? p2 : p1;
                    const C uc = P[1 + dy][1 + dx];
                    C s = P[1 + dy][dx] + P[1 + dy][2 + dx];
                    s = s + P[dy][1 + dx];
                    s = s + P[2 + dy][1 + dx];
                    s = s + (dz ? p1[1 + dy][1 + dx] : pc[dy][dx]);
                    s = s + (dz ? p3[1 + dy][1 + dx] : p2[1 + dy][1 + dx]);
                    sum += fv[dz][dy][dx] - (s - (C)6 * uc) * inv_h2;
                }
            }
        }
        const size_t q = pos<3, TC>(gc, I, J, K);
        coarse_out<3, TC, C>(fc, ec, q, I, J, K, sum * ((C)0.125 * out_scale), seed_h2, inv2d);
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
            for (int c = 0; c < 2; c++) pc[r][c] = p2[1 + r][1 + c];
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 4; c++) p1[r][c] = p3[r][c];
    }
}

// Residual and restriction out of multigrid level 0 in the paired layout of
// the level-0 sweeps.  A thread owns coarse row J (fine rows 2J - 1, 2J and
// their neighbours 2J - 2, 2J + 1) and the compact pair (h0, h0 + 1) of those
// rows, i.e. the fine points x = 2 h0 .. 2 h0 + 3 of both colours, and forms
// the coarse points I = h0 + 1 and h0 + 2 (children x = 2 h0 + 1 .. 2 h0 + 4)
// of a chunk of coarse planes.  Fine values come in paired loads; x = 2 h0 + 4
// and 2 h0 + 5 are the first pair elements of the next lane, moved by a DPP
// wave shift.  Lanes run over (J, pair) flat, 63 new pairs per wave: lane 63
// repeats the next wave's lane 0 so that the shift has a source, and stores
// nothing.  At a row's end the shifted values come from the next row; they
// feed only I = N_c + 1, which is not stored.  Per child and in the sum over
// children the arithmetic and order are those of k_restrict3_l0, with a
// third of its memory instructions (the 2-byte loads of the FP16 form kept
// the texture address unit busy).  Requires N_f = 2 N_c along every axis, an
// even row length hx and arrays of fewer than 2^31 elements.  Used for 2-byte
// storage: 206 -> 162 us at 514^3; the FP32 and FP64 forms (138 and 230 VGPRs)
// measured slower than k_restrict3_l0 (325 vs 278 us, 597 vs 537 us).
constexpr int kRestrictPairChunk = 4;  // coarse planes per thread
constexpr int kRestrictPairGroup = 4;  // coarse planes whose loads are issued together (divides the chunk; 1, 2, 4: 163, 161, 159 us)

// One fine row of a pair of coarse points in packed FP16 words: x = 2 h0 + m
// for m = 0..5 is the lower (m = 0, 1, 4, 5) or upper (m = 2, 3) half of A (even
// x = 2 h0, 2 h0 + 2), B (odd x), An and Bn (the next lane's A and B: x =
// 2 h0 + 4, 2 h0 + 5).  The residual arithmetic below takes the halves straight
// from the words (v_fma_mix converts them exactly), so no value is converted on
// its own.
struct HRow {
    uint32_t A, B, An, Bn;
};
__device__ __forceinline__ HRow hrow(uint32_t A, uint32_t B) { return HRow{A, B, dpp_next(A), dpp_next(B)}; }
template <int M>
__device__ __forceinline__ uint32_t hw(const HRow& r)
{
    return (M == 0 || M == 2) ? r.A : ((M == 1 || M == 3) ? r.B : (M == 4 ? r.An : r.Bn));
}
template <int M>
constexpr int kHalfOf = (M == 2 || M == 3) ? 1 : 0;

// c * (half H of w) + s, one rounding
template <int H>
__device__ __forceinline__ float mix_fma_w(uint32_t w, float c, float s)
{
    float r;
    if constexpr (H == 0)
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(c), "v"(s));
    else
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(w), "v"(c), "v"(s));
    return r;
}
// c * t + (half H of w), one rounding
template <int H>
__device__ __forceinline__ float mix_fma_to(float c, float t, uint32_t w)
{
    float r;
    if constexpr (H == 0)
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[0,0,1]" : "=v"(r) : "v"(c), "v"(t), "v"(w));
    else
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[0,0,1] op_sel_hi:[0,0,1]" : "=v"(r) : "v"(c), "v"(t), "v"(w));
    return r;
}

// Residual f - lap u at x = 2 h0 + M of fine row 2J - 1 + DY: the neighbour
// sum in the order x, y, z (one rounding per addition), then s - 6 u and f -
// (s - 6 u) / h^2 as fused multiply-adds.  c: rows 2J - 1, 2J of the plane, y0,
// y3: rows 2J - 2, 2J + 1, zm / zp: rows 2J - 1, 2J of the planes below and
// above, fr: the right-hand side; m6 = -6, ninv_h2 = -1 / h^2.
template <int M, int DY>
__device__ __forceinline__ float resid_h(const HRow (&zm)[2], const HRow (&c)[2], const HRow (&zp)[2], const HRow& y0,
                                         const HRow& y3, const HRow (&fr)[2], float m6, float ninv_h2)
{
    constexpr int H = kHalfOf<M>;
    float s = mix_add2<kHalfOf<M - 1>, kHalfOf<M + 1>>(hw<M - 1>(c[DY]), hw<M + 1>(c[DY]));
    s = mix_add<H>(s, hw<M>(DY ? c[0] : y0));
    s = mix_add<H>(s, hw<M>(DY ? y3 : c[1]));
    s = mix_add<H>(s, hw<M>(zm[DY]));
    s = mix_add<H>(s, hw<M>(zp[DY]));
    const float t = mix_fma_w<H>(hw<M>(c[DY]), m6, s);
    return mix_fma_to<H>(ninv_h2, t, hw<M>(fr[DY]));
}

// The residuals of one fine plane of a pair of coarse points (rows 2J - 1 + dy,
// x = 2 h0 + 1 + j) added to their two sums in the order dy, dx.
__device__ __forceinline__ void pair_plane_sums(const HRow (&zm)[2], const HRow (&c)[2], const HRow (&zp)[2],
                                                const HRow& y0, const HRow& y3, const HRow (&fr)[2], float m6,
                                                float ninv_h2, float& sa, float& sb)
{
    sa = sa + resid_h<1, 0>(zm, c, zp, y0, y3, fr, m6, ninv_h2);
    sa = sa + resid_h<2, 0>(zm, c, zp, y0, y3, fr, m6, ninv_h2);
    sa = sa + resid_h<1, 1>(zm, c, zp, y0, y3, fr, m6, ninv_h2);
    sa = sa + resid_h<2, 1>(zm, c, zp, y0, y3, fr, m6, ninv_h2);
    sb = sb + resid_h<3, 0>(zm, c, zp, y0, y3, fr, m6, ninv_h2);
    sb = sb + resid_h<4, 0>(zm, c, zp, y0, y3, fr, m6, ninv_h2);
    sb = sb + resid_h<3, 1>(zm, c, zp, y0, y3, fr, m6, ninv_h2);
    sb = sb + resid_h<4, 1>(zm, c, zp, y0, y3, fr, m6, ninv_h2);
}

// The paired restriction described above (FP16 fine level, FP32 coarse level).
template <typename TF, typename TC>
__global__ void __launch_bounds__(kBlock) k_restrict3_pair(const TF* __restrict__ u, const TF* __restrict__ f, SGrid gf,
                                                            float inv_h2, float out_scale, SGrid gc,
                                                            TC* __restrict__ fc, TC* __restrict__ ec, int pblocks,
                                                            float seed_h2, float inv2d)
{
    static_assert(sizeof(TF) == 2 && sizeof(TC) == 4, "FP16 fine level, FP32 coarse level");
    using C = float;
    if (batch_idle(gf)) return;
    u = batch_at(u, gf);
    f = batch_at(f, gf);
    fc = batch_at(fc, gc);
    ec = batch_at(ec, gc);
    const int Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int lane = (int)(threadIdx.x & 63);
    const int w = (lb - zc * pblocks) * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int e = 63 * w + lane;
    const int P = gf.hx >> 1;  // pairs per fine row
    const int J = 1 + e / P;
    if (J > Ncy) return;
    const int hp = e - (J - 1) * P;
    const int h0 = 2 * hp;
    const int K0 = 1 + zc * kRestrictPairChunk;
    const int K1 = min(K0 + kRestrictPairChunk - 1, Ncz);
    const size_t fplane = gf.ps;
    const unsigned row0 = (unsigned)((2 * J - 2) * gf.hx + h0);
    // fine row 2J - 2 + r of plane z: x = 2 h0 + 2 i is in colour (y + z + 1) & 1
    // at compact h0 + i, the odd x in the other colour
    auto seg = [&](const TF* __restrict__ a, int r, int z) -> HRow {
        const int y = 2 * J - 2 + r;
        const bool ca = ((y + z + 1) & 1) != 0;
        const TF* __restrict__ pl = a + (size_t)z * fplane + (row0 + (unsigned)(r * gf.hx));
        return hrow(*(const uint32_t*)(pl + (ca ? gf.cs : 0)), *(const uint32_t*)(pl + (ca ? 0 : gf.cs)));
    };
    const C scale = (C)0.125 * out_scale;
    const C m6 = -6.0f, ninv_h2 = -inv_h2;
    const int I = h0 + 1;
    const bool store_b = lane != 63 && I + 1 <= Ncx, store_a = lane != 63;
    HRow lo[2], mid[2];  // rows 2J - 1, 2J of fine planes 2K - 2, 2K - 1
#pragma unroll
    for (int r = 0; r < 2; r++) {
        lo[r] = seg(u, 1 + r, 2 * K0 - 2);
        mid[r] = seg(u, 1 + r, 2 * K0 - 1);
    }
    // the packed words of one coarse plane's fine rows, loaded before any of
    // them is used (the DPP shifts of hrow come with the arithmetic)
    struct Raw {
        uint32_t n1[2][2], n2[2][2], fa[2][2], fb[2][2], y[4][2];
    };
    auto segw = [&](const TF* __restrict__ a, int r, int z, uint32_t (&w)[2]) {
        const int y = 2 * J - 2 + r;
        const bool ca = ((y + z + 1) & 1) != 0;
        const TF* __restrict__ pl = a + (size_t)z * fplane + (row0 + (unsigned)(r * gf.hx));
        w[0] = *(const uint32_t*)(pl + (ca ? gf.cs : 0));
        w[1] = *(const uint32_t*)(pl + (ca ? 0 : gf.cs));
    };
    auto load = [&](int K, Raw& d) {
#pragma unroll
        for (int r = 0; r < 2; r++) {
            segw(u, 1 + r, 2 * K, d.n1[r]);
            segw(u, 1 + r, 2 * K + 1, d.n2[r]);
            segw(f, 1 + r, 2 * K - 1, d.fa[r]);
            segw(f, 1 + r, 2 * K, d.fb[r]);
        }
        segw(u, 0, 2 * K - 1, d.y[0]);
        segw(u, 3, 2 * K - 1, d.y[1]);
        segw(u, 0, 2 * K, d.y[2]);
        segw(u, 3, 2 * K, d.y[3]);
    };
    auto step = [&](int K, const Raw& d) {
        HRow n1[2], n2[2], fa[2], fb[2];
#pragma unroll
        for (int r = 0; r < 2; r++) {
            n1[r] = hrow(d.n1[r][0], d.n1[r][1]);
            n2[r] = hrow(d.n2[r][0], d.n2[r][1]);
            fa[r] = hrow(d.fa[r][0], d.fa[r][1]);
            fb[r] = hrow(d.fb[r][0], d.fb[r][1]);
        }
        const HRow ya = hrow(d.y[0][0], d.y[0][1]), yb = hrow(d.y[1][0], d.y[1][1]);
        const HRow yc = hrow(d.y[2][0], d.y[2][1]), yd = hrow(d.y[3][0], d.y[3][1]);
        C sa = 0, sb = 0;
        pair_plane_sums(lo, mid, n1, ya, yb, fa, m6, ninv_h2, sa, sb);
        pair_plane_sums(mid, n1, n2, yc, yd, fb, m6, ninv_h2, sa, sb);
        if (store_a) coarse_out<3, TC, C>(fc, ec, pos<3, TC>(gc, I, J, K), I, J, K, sa * scale, seed_h2, inv2d);
        if (store_b)
            coarse_out<3, TC, C>(fc, ec, pos<3, TC>(gc, I + 1, J, K), I + 1, J, K, sb * scale, seed_h2, inv2d);
#pragma unroll
        for (int r = 0; r < 2; r++) {
            lo[r] = n1[r];
            mid[r] = n2[r];
        }
    };
    if (K1 - K0 + 1 == kRestrictPairChunk) {
        // a full chunk in groups of kRestrictPairGroup coarse planes, every load
        // of a group issued before its first residual
#pragma unroll
        for (int i = 0; i < kRestrictPairChunk; i += kRestrictPairGroup) {
            Raw d[kRestrictPairGroup];
#pragma unroll
            for (int q = 0; q < kRestrictPairGroup; q++) load(K0 + i + q, d[q]);
#pragma unroll
            for (int q = 0; q < kRestrictPairGroup; q++) step(K0 + i + q, d[q]);
        }
    } else {
        for (int K = K0; K <= K1; K++) {
            Raw d;
            load(K, d);
            step(K, d);
        }
    }
}

// ------------------------------------------------------------------ black sweep + restriction
// The last pre-smoothing black half sweep of multigrid level 0 in 2-byte
// storage, fused with the residual and its restriction (Sec. 2.3 steps 2-5:
// the sweep, then eqn:restriction3D of f - lap u).  Threads are laid out as in
// k_restrict3_pair (a pair of coarse points I = h0 + 1, I + 1 of coarse row J,
// a chunk of coarse planes), except that a wave owns the 62 pairs of its lanes
// 1..62: lane 0 only supplies red values to lane 1 and lane 63 the first values
// of its pair to lane 62.  The residuals of a thread read the final values of
// fine rows 2J - 2 .. 2J + 1 of the fine planes 2K0 - 2 .. 2K1 + 1; the thread
// forms their black values itself from the red values and the right-hand
// side, with the arithmetic of k_smooth_zmarch3_pair (the red values are not
// changed by a black half sweep), keeps them in registers and stores the black
// points it owns (fine rows 2J - 1, 2J, planes 2K0 - 1 .. 2K1, compact slots
// h0, h0 + 1).  The residual and the sums are those of k_restrict3_pair, so
// the result equals the black half sweep followed by that restriction, bit for
// bit.  No thread reads what another writes: black values are read only on the
// ghost layer, which no kernel writes.
// SEED: the red values are those of a red half sweep from zero, formed from the
// defect f (red) as k_smooth_zmarch3_pair<T, 2> forms them, and stored.
constexpr int kBrChunk = 4;  // coarse planes per thread

template <int SEED>
__global__ void __launch_bounds__(kBlock) k_black_restrict3_pair(__half* __restrict__ u, const __half* __restrict__ f,
                                                                  SGrid gf, float h2, float inv_h2, float out_scale,
                                                                  SGrid gc, float* __restrict__ fc,
                                                                  float* __restrict__ ec, int pblocks, float seed_h2,
                                                                  float inv2d)
{
    using T = __half;
    using C = float;
    typedef uint32_t W;  // a pair of compact FP16 values, the lower one first
    if (batch_idle(gf)) return;
    u = batch_at(u, gf);
    f = batch_at(f, gf);
    fc = batch_at(fc, gc);
    ec = batch_at(ec, gc);
    const int Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    const int Nfx = gf.nx - 2, Nfy = gf.ny - 2, Nfz = gf.nz - 2;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int lane = (int)(threadIdx.x & 63);
    const int w = (lb - zc * pblocks) * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int P = gf.hx >> 1;  // pairs per fine row
    const int e = max(62 * w + lane - 1, 0);
    if (e >= P * Ncy) return;
    const bool own = lane >= 1 && lane <= 62;
    const int J = 1 + e / P;
    const int hp = e - (J - 1) * P;
    const int h0 = 2 * hp;
    const int K0 = 1 + zc * kBrChunk;
    const int K1 = min(K0 + kBrChunk - 1, Ncz);
    const size_t ps = gf.ps;
    const T* __restrict__ rsrc = SEED ? f : u;  // red values (colour 0), formed from f with SEED
    const T* __restrict__ fblk = f + gf.cs;
    T* __restrict__ ublk = u + gf.cs;
    const auto half_of = [](W v, int hi) -> T { return __builtin_bit_cast(T, (uint16_t)(hi ? v >> 16 : v & 0xffffu)); };
    const auto pack = [](T a, T b) -> W {
        return (W)__builtin_bit_cast(uint16_t, a) | ((W)__builtin_bit_cast(uint16_t, b) << 16);
    };
    // word at compact h0 of fine row y (clamped to the grid) of plane z
    const auto ld = [&](const T* __restrict__ a, int z, int y) -> W {
        y = min(max(y, 0), Nfy + 1);
        return *(const W*)(a + (size_t)z * ps + (unsigned)(y * gf.hx + h0));
    };
    // red words of rows 2J - 3 .. 2J + 2 of plane z; outside the grid (needed only
    // by the ghost planes, whose black values are not formed) the nearest plane's,
    // so that every load is unconditional
    const auto red_plane = [&](int z, W (&r)[6]) {
        z = min(max(z, 0), Nfz + 1);
#pragma unroll
        for (int i = 0; i < 6; i++) {
            W v = ld(rsrc, z, 2 * J - 3 + i);
            if (SEED)
                v = pack(gs_value<T, C>((C)0, half_of(v, 0), h2, inv2d), gs_value<T, C>((C)0, half_of(v, 1), h2, inv2d));
            r[i] = v;
        }
    };
    // right-hand side of the black points of rows 2J - 2 .. 2J + 1 of plane z
    const auto fblk_plane = [&](int z, W (&b)[4]) {
#pragma unroll
        for (int i = 0; i < 4; i++) b[i] = ld(fblk, z, 2 * J - 2 + i);
    };
    // Final values of rows 2J - 2 .. 2J + 1 of plane z (as k_restrict3_pair reads
    // them) and its black words, from the red words of planes z - 1, z, z + 1
    // and the black right-hand side of z.
    const auto produce = [&](int z, const W (&rm)[6], const W (&rc)[6], const W (&rp)[6], const W (&fb)[4],
                             HRow (&v)[4], W (&bw)[4]) {
        const bool gz = z == 0 || z == Nfz + 1;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int y = 2 * J - 2 + r;
            const int o = (y + z + 1) & 1;  // x offset of the red points in this row
            const W rw = rc[r + 1];
            const W pw = dpp_prev(rw), nw = dpp_next(rw);
            // the black points x = 2 h0 + 1 - o and x + 2: their x-neighbours
            // (the previous lane's upper red value or this lane's, and this
            // lane's lower one or the next lane's), then rows y - 1, y + 1 and
            // planes z - 1, z + 1, one rounding per addition, as the half sweep
            C sa = mix_add2<1, 0>(o ? pw : rw, rw);
            C sb = mix_add2<1, 0>(rw, o ? rw : nw);
            sa = mix_add<0>(sa, rc[r]);
            sb = mix_add<1>(sb, rc[r]);
            sa = mix_add<0>(sa, rc[r + 2]);
            sb = mix_add<1>(sb, rc[r + 2]);
            sa = mix_add<0>(sa, rm[r + 1]);
            sb = mix_add<1>(sb, rm[r + 1]);
            sa = mix_add<0>(sa, rp[r + 1]);
            sb = mix_add<1>(sb, rp[r + 1]);
            W b = pack(gs_value<T, C>(sa, half_of(fb[r], 0), h2, inv2d), gs_value<T, C>(sb, half_of(fb[r], 1), h2, inv2d));
            // ghost points keep their stored values
            const int xa = 2 * h0 + 1 - o;
            const bool gr = gz || y == 0 || y == Nfy + 1;
            const bool ga = gr || xa == 0 || xa == Nfx + 1, gb = gr || xa + 2 == Nfx + 1;
            if (ga || gb) {
                const W g = ld(ublk, z, y);
                b = (ga ? (g & 0xffffu) : (b & 0xffffu)) | (gb ? (g & 0xffff0000u) : (b & 0xffff0000u));
            }
            bw[r] = b;
            v[r] = hrow(o ? b : rw, o ? rw : b);  // even x, odd x
        }
    };
    // right-hand side of rows 2J - 1, 2J of plane z as k_restrict3_pair reads it
    const auto rhs = [&](int z, const W (&fr)[2], const W (&fb)[2], HRow (&v)[2]) {
#pragma unroll
        for (int dy = 0; dy < 2; dy++) {
            const int o = (2 * J - 1 + dy + z + 1) & 1;
            v[dy] = hrow(o ? fb[dy] : fr[dy], o ? fr[dy] : fb[dy]);
        }
    };
    // stores of the owned points of rows 2J - 1, 2J of an active plane z
    const auto store_plane = [&](int z, const W (&bw)[4], const W (&rw)[6]) {
        if (!own) return;
#pragma unroll
        for (int dy = 0; dy < 2; dy++) {
            const int y = 2 * J - 1 + dy;
            const size_t here = (size_t)z * ps + (unsigned)(y * gf.hx + h0);
            const int xa = 2 * h0 + 1 - ((y + z + 1) & 1);
            const bool a0 = xa >= 1, a1 = xa + 2 <= Nfx;
            if (a0 && a1) {
                *(W*)(ublk + here) = bw[1 + dy];
            } else {
                if (a0) ublk[here] = half_of(bw[1 + dy], 0);
                if (a1) ublk[here + 1] = half_of(bw[1 + dy], 1);
            }
            if (SEED) *(W*)(u + here) = rw[2 + dy];
        }
    };
    const C scale = (C)0.125 * out_scale;
    const C m6 = -6.0f, ninv_h2 = -inv_h2;
    const int I = h0 + 1;
    const bool store_b = own && I + 1 <= Ncx;
    // planes 2K0 - 2 and 2K0 - 1
    W rA[6], rB[6], rC[6], rD[6], fA[4], fB[4];
    red_plane(2 * K0 - 3, rA);
    red_plane(2 * K0 - 2, rB);
    red_plane(2 * K0 - 1, rC);
    red_plane(2 * K0, rD);
    fblk_plane(2 * K0 - 2, fA);
    fblk_plane(2 * K0 - 1, fB);
    HRow v0[4], v1[4];
    W b0[4], b1[4];
    produce(2 * K0 - 2, rA, rB, rC, fA, v0, b0);
    produce(2 * K0 - 1, rB, rC, rD, fB, v1, b1);
    // carried between coarse planes: final rows 2J - 1, 2J of fine plane 2K - 2,
    // all four rows of 2K - 1 and its black words, red words and black
    // right-hand side, and the red words of plane 2K
    HRow zlo[2] = {v0[1], v0[2]};
    W rp1[6], rc0[6], fbp[2];
#pragma unroll
    for (int i = 0; i < 6; i++) {
        rp1[i] = rC[i];
        rc0[i] = rD[i];
    }
    fbp[0] = fB[1];
    fbp[1] = fB[2];
    auto step = [&](int K) {
        // fine planes 2K, 2K + 1 produced; residuals of 2K - 1, 2K
        W rn1[6], rn2[6], fn0[4], fn1[4], fr0[2], fr1[2];
        red_plane(2 * K + 1, rn1);
        red_plane(2 * K + 2, rn2);
        fblk_plane(2 * K, fn0);
        fblk_plane(2 * K + 1, fn1);
#pragma unroll
        for (int dy = 0; dy < 2; dy++) {
            fr0[dy] = ld(f, 2 * K - 1, 2 * J - 1 + dy);
            fr1[dy] = ld(f, 2 * K, 2 * J - 1 + dy);
        }
        HRow v2[4], v3[4], fa[2], fbv[2];
        W b2[4], b3[4];
        produce(2 * K, rp1, rc0, rn1, fn0, v2, b2);
        const HRow c1[2] = {v1[1], v1[2]}, c2[2] = {v2[1], v2[2]};
        rhs(2 * K - 1, fr0, fbp, fa);
        C sa = 0, sb = 0;
        pair_plane_sums(zlo, c1, c2, v1[0], v1[3], fa, m6, ninv_h2, sa, sb);
        store_plane(2 * K - 1, b1, rp1);
        produce(2 * K + 1, rc0, rn1, rn2, fn1, v3, b3);
        const HRow z3[2] = {v3[1], v3[2]};
        const W fbc[2] = {fn0[1], fn0[2]};
        rhs(2 * K, fr1, fbc, fbv);
        pair_plane_sums(c1, c2, z3, v2[0], v2[3], fbv, m6, ninv_h2, sa, sb);
        store_plane(2 * K, b2, rc0);
        if (own) coarse_out<3, float, C>(fc, ec, pos<3, float>(gc, I, J, K), I, J, K, sa * scale, seed_h2, inv2d);
        if (store_b)
            coarse_out<3, float, C>(fc, ec, pos<3, float>(gc, I + 1, J, K), I + 1, J, K, sb * scale, seed_h2, inv2d);
        // advance by two fine planes
        zlo[0] = c2[0];
        zlo[1] = c2[1];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            v1[r] = v3[r];
            b1[r] = b3[r];
        }
#pragma unroll
        for (int i = 0; i < 6; i++) {
            rp1[i] = rn1[i];
            rc0[i] = rn2[i];
        }
        fbp[0] = fn1[1];
        fbp[1] = fn1[2];
    };
#pragma unroll 1
    for (int K = K0; K <= K1; K++) step(K);
}

// u += P(e) on the fine active points (eqn:prolongation2D/3D as the tensor
// product of (3/4, 1/4) along each axis: the coarse parent ceil(p/2) weighs
// 3/4, its neighbour on the side of the fine centre 1/4).  Each thread does
// the red and the black point of one compact position; with black_only the
// red points are left alone (used when a red half sweep that reads only
// black values follows on a grid with a fixed ghost layer).  The coarse level
// is a multigrid level L >= 1: where the parent q or its neighbour q + s is a
// ghost (the parent of the last fine point is one when N_f = 2 N_c + 1), its
// value comes from the rule.
template <typename C>
struct AxisNb {
    int q;       // neighbour index after the rule
    C fac;       // rule factor
    bool ghost;  // the factor applies
};

template <typename C>
__device__ __forceinline__ AxisNb<C> axis_nb(int q, int N, const GRule<C>& gr, int ax)
{
    AxisNb<C> a{q, (C)1, false};
    if (q == 0) {
        a.q = 1;
        a.fac = (C)-1;
        a.ghost = true;
    } else if (q == N + 1) {
        a.q = gr.xn1[ax] ? N - 1 : N;
        a.fac = gr.xn1[ax] ? (C)-1 : gr.coef[ax];
        a.ghost = true;
    }
    return a;
}

template <int D, typename TC, typename TF>
__global__ void __launch_bounds__(kBlock) k_prolong_add(const TC* __restrict__ e, SGrid gc, TF* __restrict__ u, SGrid gf,
                                                        int black_only, GRule<typename Compute<TC>::type> gr)
{
    using C = typename Compute<TC>::type;
    if (batch_idle(gf)) return;
    e = batch_at(e, gc);
    u = batch_at(u, gf);
    const int my = gf.ny - 2, mz = gf.nz - 2;
    long t = xcd_block() * kBlock + threadIdx.x;
    long total = (long)gf.hx * my * (D == 3 ? mz : 1);
    if (t >= total) return;
    int h = (int)(t % gf.hx);
    long r = t / gf.hx;
    int pj = 1 + (int)(r % my);
    int pk = D == 3 ? 1 + (int)(r / my) : 0;
    const C w0 = (C)0.75, w1 = (C)0.25;
    const int Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    int qj = (pj + 1) >> 1, sj = (pj & 1) ? -1 : 1;
    int qk = D == 3 ? (pk + 1) >> 1 : 0, sk = (pk & 1) ? -1 : 1;
    const AxisNb<C> pj_ = axis_nb(qj, Ncy, gr, 1), nj = axis_nb(qj + sj, Ncy, gr, 1);
    const AxisNb<C> none{0, (C)1, false};
    const AxisNb<C> pk_ = D == 3 ? axis_nb(qk, Ncz, gr, 2) : none, nk = D == 3 ? axis_nb(qk + sk, Ncz, gr, 2) : none;
    for (int c = black_only; c < 2; c++) {
        int pi = 2 * h + ((c + pj + pk + D) & 1);
        if (pi < 1 || pi > gf.nx - 2) continue;
        int qi = (pi + 1) >> 1, si = (pi & 1) ? -1 : 1;
        const AxisNb<C> pi_ = axis_nb(qi, Ncx, gr, 0), ni = axis_nb(qi + si, Ncx, gr, 0);
        // coarse value at (parent or neighbour) per axis, rule factors in x, y, z order
        auto E = [&](bool bx, bool by, bool bz) -> C {
            const AxisNb<C>& ax = bx ? ni : pi_;
            const AxisNb<C>& ay = by ? nj : pj_;
            const AxisNb<C>& az = bz ? nk : pk_;
            C v = (C)at<D>(e, gc, ax.q, ay.q, az.q);
            if (ax.ghost) v = ax.fac * v;
            if (ay.ghost) v = ay.fac * v;
            if (az.ghost) v = az.fac * v;
            return v;
        };
        C y0 = w0 * E(false, false, false) + w1 * E(true, false, false);
        C y1 = w0 * E(false, true, false) + w1 * E(true, true, false);
        C v = w0 * y0 + w1 * y1;
        if (D == 3) {
            C y2 = w0 * E(false, false, true) + w1 * E(true, false, true);
            C y3 = w0 * E(false, true, true) + w1 * E(true, true, true);
            v = w0 * v + w1 * (w0 * y2 + w1 * y3);
        }
        size_t p = (size_t)c * gf.cs + row_base(gf, pj, pk) + h;
        u[p] = (TF)((C)u[p] + v);
    }
}

// 3-D prolongation marching along the coarse z axis: a thread owns one coarse
// column (I, J) and a chunk of coarse planes K, keeps the 3 x 3 x 3 coarse
// neighbourhood of (I, J, K) in registers (each step loads the 3 x 3 values of
// plane K + 1, with the rule applied where they are ghosts) and corrects the
// 2 x 2 x 2 fine children of (I, J, K), or the black ones with black_only.  The
// coarse index runs to ceil(N_f / 2), which is N_c + 1 when N_f = 2 N_c + 1
// (a ghost parent with one active child).  Per child the arithmetic is that
// of k_prolong_add.
template <typename C>
__device__ __forceinline__ AxisNb<C> axis_nb_clamped(int q, int N, const GRule<C>& gr, int ax)
{
    // q = N + 2 only beside a ghost parent, on the side it has no child: any
    // in-bounds value serves
    return axis_nb(q > N + 1 ? N + 1 : q, N, gr, ax);
}

template <typename TC, typename TF>
__global__ void __launch_bounds__(kBlock) k_prolong3_zm(const TC* __restrict__ e, SGrid gc, TF* __restrict__ u,
                                                         SGrid gf, int black_only, GRule<typename Compute<TC>::type> gr,
                                                         int pblocks, int kch)
{
    using C = typename Compute<TC>::type;
    if (batch_idle(gf)) return;
    e = batch_at(e, gc);
    u = batch_at(u, gf);
    const int Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    const int Nfx = gf.nx - 2, Nfy = gf.ny - 2, Nfz = gf.nz - 2;
    // coarse parents per axis
    const int Mx = (Nfx + 1) >> 1, My = (Nfy + 1) >> 1, Mz = (Nfz + 1) >> 1;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    if (t >= (long)Mx * My) return;
    const int I = 1 + (int)(t % Mx), J = 1 + (int)(t / Mx);
    const int K0 = 1 + zc * kch;
    const int K1 = min(K0 + kch - 1, Mz);
    AxisNb<C> mx[3], my[3];
    for (int a = 0; a < 3; a++) {
        mx[a] = axis_nb_clamped(I - 1 + a, Ncx, gr, 0);
        my[a] = axis_nb_clamped(J - 1 + a, Ncy, gr, 1);
    }
    // coarse values, index [z][y][x] = plane K-1+z, row J-1+y, column I-1+x
    C cv[3][3][3];
    auto load_plane = [&](int kk, C (&pl)[3][3]) {
        const AxisNb<C> mz = axis_nb_clamped(kk, Ncz, gr, 2);
#pragma unroll
        for (int y = 0; y < 3; y++)
#pragma unroll
            for (int x = 0; x < 3; x++) {
                C v = (C)at<3>(e, gc, mx[x].q, my[y].q, mz.q);
                if (mx[x].ghost) v = mx[x].fac * v;
                if (my[y].ghost) v = my[y].fac * v;
                if (mz.ghost) v = mz.fac * v;
                pl[y][x] = v;
            }
    };
    load_plane(K0 - 1, cv[0]);
    load_plane(K0, cv[1]);
    const C w0 = (C)0.75, w1 = (C)0.25;
    // the loads of one coarse step K: the children's positions and current
    // values, and the coarse plane K + 1
    struct Step {
        C pl[3][3];
        size_t pos8[8];
        bool live[8];
        TF old[8];
    };
    auto load = [&](int K, Step& st) {
#pragma unroll
        for (int c8 = 0; c8 < 8; c8++) {
            const int dz = c8 >> 2, dy = (c8 >> 1) & 1, dx = c8 & 1;
            const int pk = 2 * K - 1 + dz, pj = 2 * J - 1 + dy, pi = 2 * I - 1 + dx;
            const int colour = (pi + pj + pk + 3) & 1;
            st.live[c8] = pi <= Nfx && pj <= Nfy && pk <= Nfz && !(black_only && colour == 0);
            st.pos8[c8] = (size_t)colour * gf.cs + row_base(gf, pj, pk) + (pi >> 1);
            if (st.live[c8]) st.old[c8] = u[st.pos8[c8]];
        }
        load_plane(K + 1, st.pl);
    };
    auto apply = [&](const Step& st) {
#pragma unroll
        for (int y = 0; y < 3; y++)
#pragma unroll
            for (int x = 0; x < 3; x++) cv[2][y][x] = st.pl[y][x];
#pragma unroll
        for (int c8 = 0; c8 < 8; c8++) {
            if (!st.live[c8]) continue;
            const int dz = c8 >> 2, dy = (c8 >> 1) & 1, dx = c8 & 1;
            const int zs = 1 + (dz ? 1 : -1), ys = 1 + (dy ? 1 : -1), xs = 1 + (dx ? 1 : -1);
            C y0 = w0 * cv[1][1][1] + w1 * cv[1][1][xs];
            C y1 = w0 * cv[1][ys][1] + w1 * cv[1][ys][xs];
            C v = w0 * y0 + w1 * y1;
            C y2 = w0 * cv[zs][1][1] + w1 * cv[zs][1][xs];
            C y3 = w0 * cv[zs][ys][1] + w1 * cv[zs][ys][xs];
            v = w0 * v + w1 * (w0 * y2 + w1 * y3);
            u[st.pos8[c8]] = (TF)((C)st.old[c8] + v);
        }
#pragma unroll
        for (int y = 0; y < 3; y++)
#pragma unroll
            for (int x = 0; x < 3; x++) {
                cv[0][y][x] = cv[1][y][x];
                cv[1][y][x] = cv[2][y][x];
            }
    };
    // two coarse steps at a time: all loads of both before the first correction
    int K = K0;
    for (; K + 1 <= K1; K += 2) {
        Step s0, s1;
        load(K, s0);
        load(K + 1, s1);
        apply(s0);
        apply(s1);
    }
    if (K <= K1) {
        Step s0;
        load(K, s0);
        apply(s0);
    }
}

// Prolongation into the black points of multigrid level 0 (the red ones are
// left alone: a red half sweep that reads only black values follows), paired
// form: a thread owns the compact pair (h0, h0 + 1) of one fine row pj and a
// chunk of coarse planes.  The two black points of the pair in any fine plane
// have their x parents and neighbours among the coarse columns h0 .. h0 + 2,
// and every fine point of row pj has the same y parent and neighbour, so a
// coarse plane contributes 2 x 3 values (rule applied where they are ghosts).
// Per coarse plane and row the four x-interpolants the pair can need are
// formed once (which column is parent and which neighbour depends only on the
// parity of the fine plane); each coarse plane K then corrects the pair in
// fine planes 2K - 1 and 2K with one paired load and store each.  Per point
// the arithmetic is that of k_prolong3_zm (same products, same order).  The
// chunk's plane index is uniform over the block, so plane bases are scalar and
// each lane keeps fixed 32-bit offsets inside a plane.  Requires an even row
// length hx and arrays of fewer than 2^31 elements.
constexpr int kProlongPairChunk = 8;  // coarse planes per thread: 2, 4, 8 measured 103, 86, 83 us (FP16 storage, 514^3)

template <typename TC, typename TF, int KCH>
__global__ void __launch_bounds__(kBlock) k_prolong3_pair(const TC* __restrict__ e, SGrid gc, TF* __restrict__ u,
                                                           SGrid gf, GRule<typename Compute<TC>::type> gr, int pblocks)
{
    using C = typename Compute<TC>::type;
    if (batch_idle(gf)) return;
    e = batch_at(e, gc);
    u = batch_at(u, gf);
    const int Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    const int Nfx = gf.nx - 2, Nfy = gf.ny - 2, Nfz = gf.nz - 2;
    const int Mz = (Nfz + 1) >> 1;  // coarse parents along z
    const int lb = zmarch_block(1);  // after the restriction, which runs up
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    // flat pair index over the whole (padded) fine plane: aligned wave segments
    const int q0 = 2 * t;
    const int pj = q0 / gf.hx;
    const int h0 = q0 - pj * gf.hx;
    if (pj < 1 || pj > Nfy) return;
    const int K0 = 1 + zc * KCH;
    const int nk = min(KCH, Mz - K0 + 1);
    const int qj = (pj + 1) >> 1, sj = (pj & 1) ? -1 : 1;
    const AxisNb<C> my[2] = {axis_nb_clamped(qj, Ncy, gr, 1), axis_nb_clamped(qj + sj, Ncy, gr, 1)};
    AxisNb<C> mx[3];
#pragma unroll
    for (int a = 0; a < 3; a++) mx[a] = axis_nb_clamped(h0 + a, Ncx, gr, 0);
    const bool edge = my[0].ghost || my[1].ghost || mx[0].ghost || mx[2].ghost;
    // offsets inside a coarse plane of slot (y, x) for an even / odd plane index
    // (the colour of a coarse point flips with the plane's parity)
    unsigned off[2][2][3];
#pragma unroll
    for (int y = 0; y < 2; y++)
#pragma unroll
        for (int x = 0; x < 3; x++) {
            const unsigned o = (unsigned)(my[y].q * gc.hx + (mx[x].q >> 1));
            const int c0 = (mx[x].q + my[y].q + 3) & 1;  // colour on an even plane
            off[0][y][x] = o + (c0 ? (unsigned)gc.cs : 0u);
            off[1][y][x] = o + (c0 ? 0u : (unsigned)gc.cs);
        }
    const size_t cplane = gc.ps;
    const size_t fplane = gf.ps;
    const unsigned row = (unsigned)(pj * gf.hx + h0);
    TF* __restrict__ ub = u + gf.cs;  // black colour array
    // Every load of the chunk is issued before the first use, with no branch
    // between them (the planes past the chunk's end read clamped, in-bounds
    // indices and feed no stored value): with the loads of each coarse plane
    // behind a condition, each plane cost a full memory round trip.
    // coarse planes K0 - 1 .. K0 + KCH (the index clamped to the ghost plane)
    AxisNb<C> mzs[KCH + 2];
    TC raw[KCH + 2][2][3];
#pragma unroll
    for (int z = 0; z < KCH + 2; z++) {
        mzs[z] = axis_nb_clamped(K0 - 1 + z, Ncz, gr, 2);
        const TC* __restrict__ ep = e + (size_t)mzs[z].q * cplane;
        const bool odd = (mzs[z].q & 1) != 0;
#pragma unroll
        for (int y = 0; y < 2; y++)
#pragma unroll
            for (int x = 0; x < 3; x++) raw[z][y][x] = ep[odd ? off[1][y][x] : off[0][y][x]];
    }
    // fine black pairs of planes 2K - 1 and 2K (past the last active plane the
    // ghost plane Nfz + 1 is read and nothing is stored)
    Pair<TF> old[KCH][2];
#pragma unroll
    for (int z = 0; z < KCH; z++)
#pragma unroll
        for (int d = 0; d < 2; d++) {
            const int pk = min(2 * (K0 + z) - 1 + d, Nfz + 1);
            old[z][d] = *(const Pair<TF>*)(ub + (size_t)pk * fplane + row);
        }
    const C w0 = (C)0.75, w1 = (C)0.25;
    // par0: parity term of the black points in the odd fine plane 2K - 1
    // (pi = 2 h + par); the even plane 2K has the other one
    const bool par0 = ((pj + 1) & 1) != 0;
    // X[z][d][b][y]: x-interpolant of coarse plane K0 - 1 + z, row y, for the
    // pair point b in the fine plane of parity d (0: 2K - 1, 1: 2K)
    C X[KCH + 2][2][2][2];
#pragma unroll
    for (int z = 0; z < KCH + 2; z++) {
        const AxisNb<C>& mz = mzs[z];
        C cv[2][3];
#pragma unroll
        for (int y = 0; y < 2; y++)
#pragma unroll
            for (int x = 0; x < 3; x++) cv[y][x] = (C)raw[z][y][x];
        if (edge || mz.ghost) {
#pragma unroll
            for (int y = 0; y < 2; y++)
#pragma unroll
                for (int x = 0; x < 3; x++) {
                    C v = cv[y][x];
                    if (mx[x].ghost) v = mx[x].fac * v;
                    if (my[y].ghost) v = my[y].fac * v;
                    if (mz.ghost) v = mz.fac * v;
                    cv[y][x] = v;
                }
        }
#pragma unroll
        for (int y = 0; y < 2; y++) {
            // par = 1: point 0 has parent column 1 and neighbour 0, point 1
            // parent 2 and neighbour 1; par = 0: (0, 1) and (1, 2)
            const C A = par0 ? cv[y][1] : cv[y][0], B = par0 ? cv[y][0] : cv[y][1];
            const C P = par0 ? cv[y][2] : cv[y][1], Q = par0 ? cv[y][1] : cv[y][2];
            X[z][0][0][y] = w0 * A + w1 * B;
            X[z][1][0][y] = w0 * B + w1 * A;
            X[z][0][1][y] = w0 * P + w1 * Q;
            X[z][1][1][y] = w0 * Q + w1 * P;
        }
    }
#pragma unroll
    for (int z = 0; z < KCH; z++) {
#pragma unroll
        for (int d = 0; d < 2; d++) {
            const int pk = 2 * (K0 + z) - 1 + d;
            if (z >= nk || pk > Nfz) continue;
            const int zs = d ? z + 2 : z;  // the z neighbour: plane K + 1 or K - 1
            C r[2];
#pragma unroll
            for (int b = 0; b < 2; b++) {
                C v = w0 * X[z + 1][d][b][0] + w1 * X[z + 1][d][b][1];
                r[b] = w0 * v + w1 * (w0 * X[zs][d][b][0] + w1 * X[zs][d][b][1]);
            }
            const Pair<TF> o = old[z][d];
            Pair<TF> nv;
            nv.a = (TF)((C)o.a + r[0]);
            nv.b = (TF)((C)o.b + r[1]);
            const int pi0 = 2 * h0 + (d ? !par0 : par0);
            const bool a0 = pi0 >= 1, a1 = pi0 + 2 <= Nfx;
            TF* q = ub + (size_t)pk * fplane + row;
            if (a0 && a1) {
                *(Pair<TF>*)q = nv;
            } else {
                if (a0) q[0] = nv.a;
                if (a1) q[1] = nv.b;
            }
        }
    }
}

// ------------------------------------------------------------------ coarse tail
// The smallest multigrid levels of a V-cycle, from a level Lt whose data and
// that of every coarser level fit in LDS together, down to the one-point level
// and back, in one workgroup: as separate launches their cost would be launch
// latency, not work.  Same operations in the same order and arithmetic as the
// per-level kernels: n_pre sweeps on Lt; per level down, the restriction
// (correction cleared) and n_pre sweeps; per level up, the prolongation and
// n_post sweeps.  Each level lives in LDS in natural order (x fastest) on its
// box of N_a + 2 points per axis; the ghost slots are never written, the rule
// supplies their values.
constexpr int kTailThreads = 1024;

template <typename C>
struct TailParams {
    int nlev;                   // levels Lt .. Lt + nlev - 1 (the last has one point along some axis)
    int N[kTailMaxLevels][3];   // active points per axis
    int off[kTailMaxLevels];    // LDS element offset of level a's u; its f follows one box later
    C h2[kTailMaxLevels];       // smoother factor (2^L h)^2
    C inv_h2[kTailMaxLevels];   // residual factor 1 / (2^L h)^2
    GRule<C> gr[kTailMaxLevels];
    float rN[kTailMaxLevels][3];  // 1 / N per axis (index decoding)
    float rS[kTailMaxLevels];     // 1 / ((N_x + 1) / 2), the slots of one colour per row
    int n_pre, n_post;
};

// points of a level's box in LDS ((N_x+2) x (N_y+2) [x (N_z+2)])
template <int D>
__device__ __forceinline__ int box_size(const int* N)
{
    return D == 3 ? (N[0] + 2) * (N[1] + 2) * (N[2] + 2) : (N[0] + 2) * (N[1] + 2);
}

template <int D>
__device__ __forceinline__ int box_active(const int* N)
{
    return D == 3 ? N[0] * N[1] * N[2] : N[0] * N[1];
}

// q = a / N and a % N for 0 <= a < 2^22 through a float reciprocal (rN = 1/N,
// loop-invariant) corrected by one step, instead of an integer division
__device__ __forceinline__ int divmod_small(int a, int N, float rN, int& rem)
{
    int q = (int)((float)a * rN);
    int r = a - q * N;
    if (r < 0) {
        q--;
        r += N;
    } else if (r >= N) {
        q++;
        r -= N;
    }
    rem = r;
    return q;
}

template <int D>
__device__ __forceinline__ void tail_point(int t, const int* N, const float* rN, int& i, int& j, int& k)
{
    int ri;
    const int r = divmod_small(t, N[0], rN[0], ri);
    i = 1 + ri;
    if (D == 3) {
        int rj;
        k = 1 + divmod_small(r, N[1], rN[1], rj);
        j = 1 + rj;
    } else {
        j = 1 + r;
        k = 0;
    }
}

// element index of (i, j, k) in a level box with active points N
__device__ __forceinline__ int box_idx(const int* N, int i, int j, int k)
{
    return (k * (N[1] + 2) + j) * (N[0] + 2) + i;
}

// One half sweep; the threads run over the points of the colour only: row
// (j, k) holds (N_x + 1) / 2 slots, slot s is i = i0 + 2 s with i0 = 1 or 2
// by the row's parity (a slot past N_x has no point).
template <int D, typename C>
__device__ __forceinline__ void tail_sweep(C* U, const C* F, const int* N, const float* rN, float rS, C h2, C inv2d,
                                           const GRule<C>& gr, int colour)
{
    const int Qx = N[0] + 2, Qxy = Qx * (N[1] + 2);
    const int hs = (N[0] + 1) >> 1;
    const int total = hs * N[1] * (D == 3 ? N[2] : 1);
    for (int t = threadIdx.x; t < total; t += kTailThreads) {
        int sl;
        const int row = divmod_small(t, hs, rS, sl);
        int j, k;
        if (D == 3) {
            int rj;
            k = 1 + divmod_small(row, N[1], rN[1], rj);
            j = 1 + rj;
        } else {
            j = 1 + row;
            k = 0;
        }
        const int i = 1 + ((1 + j + k + D + colour) & 1) + 2 * sl;
        if (i > N[0]) continue;
        const int idx = box_idx(N, i, j, k);
        C xm = U[idx - 1], xp = U[idx + 1], ym = U[idx - Qx], yp = U[idx + Qx], zm = 0, zp = 0;
        if (D == 3) {
            zm = U[idx - Qxy];
            zp = U[idx + Qxy];
        }
        const C me = U[idx];
        rule_pair(i, N[0], me, xm, xp, gr, 0);
        rule_pair(j, N[1], me, ym, yp, gr, 1);
        if (D == 3) rule_pair(k, N[2], me, zm, zp, gr, 2);
        C s = xm + xp;
        s = s + ym;
        s = s + yp;
        if (D == 3) {
            s = s + zm;
            s = s + zp;
        }
        U[idx] = (s - h2 * F[idx]) * inv2d;
    }
}

template <int D, typename C>
__device__ __forceinline__ void tail_restrict(const C* U, const C* F, const int* Nf, C inv_h2, const GRule<C>& gr,
                                              C* Uc, C* Fc, const int* Nc, const float* rNc)
{
    const int Qx = Nf[0] + 2, Qxy = Qx * (Nf[1] + 2), total = box_active<D>(Nc);
    for (int t = threadIdx.x; t < total; t += kTailThreads) {
        int I, J, K;
        tail_point<D>(t, Nc, rNc, I, J, K);
        C sum = 0;
        const int k0 = D == 3 ? 2 * K - 1 : 0, k1 = D == 3 ? 2 * K : 0;
        for (int k = k0; k <= k1; k++)
            for (int j = 2 * J - 1; j <= 2 * J; j++)
                for (int i = 2 * I - 1; i <= 2 * I; i++) {
                    if (i > Nf[0] || j > Nf[1] || (D == 3 && k > Nf[2])) continue;
                    const int idx = box_idx(Nf, i, j, k);
                    C xm = U[idx - 1], xp = U[idx + 1], ym = U[idx - Qx], yp = U[idx + Qx], zm = 0, zp = 0;
                    if (D == 3) {
                        zm = U[idx - Qxy];
                        zp = U[idx + Qxy];
                    }
                    const C uc = U[idx];
                    rule_pair(i, Nf[0], uc, xm, xp, gr, 0);
                    rule_pair(j, Nf[1], uc, ym, yp, gr, 1);
                    if (D == 3) rule_pair(k, Nf[2], uc, zm, zp, gr, 2);
                    C s = xm + xp;
                    s = s + ym;
                    s = s + yp;
                    if (D == 3) {
                        s = s + zm;
                        s = s + zp;
                    }
                    sum += F[idx] - (s - (C)(2 * D) * uc) * inv_h2;
                }
        const int pc = box_idx(Nc, I, J, K);
        Fc[pc] = sum * ((C)(D == 3 ? 0.125 : 0.25) * (C)1);
        Uc[pc] = (C)0;
    }
}

template <int D, typename C>
__device__ __forceinline__ void tail_prolong(const C* Ue, const int* Nc, const GRule<C>& gr, C* U, const int* Nf,
                                             const float* rNf)
{
    const int total = box_active<D>(Nf);
    const C w0 = (C)0.75, w1 = (C)0.25;
    const AxisNb<C> none{0, (C)1, false};
    for (int t = threadIdx.x; t < total; t += kTailThreads) {
        int i, j, k;
        tail_point<D>(t, Nf, rNf, i, j, k);
        const int qi = (i + 1) >> 1, si = (i & 1) ? -1 : 1;
        const int qj = (j + 1) >> 1, sj = (j & 1) ? -1 : 1;
        const int qk = D == 3 ? (k + 1) >> 1 : 0, sk = (k & 1) ? -1 : 1;
        const AxisNb<C> pi_ = axis_nb(qi, Nc[0], gr, 0), ni = axis_nb(qi + si, Nc[0], gr, 0);
        const AxisNb<C> pj_ = axis_nb(qj, Nc[1], gr, 1), nj = axis_nb(qj + sj, Nc[1], gr, 1);
        const AxisNb<C> pk_ = D == 3 ? axis_nb(qk, Nc[2], gr, 2) : none;
        const AxisNb<C> nk = D == 3 ? axis_nb(qk + sk, Nc[2], gr, 2) : none;
        auto E = [&](bool bx, bool by, bool bz) -> C {
            const AxisNb<C>& ax = bx ? ni : pi_;
            const AxisNb<C>& ay = by ? nj : pj_;
            const AxisNb<C>& az = bz ? nk : pk_;
            C v = Ue[box_idx(Nc, ax.q, ay.q, az.q)];
            if (ax.ghost) v = ax.fac * v;
            if (ay.ghost) v = ay.fac * v;
            if (az.ghost) v = az.fac * v;
            return v;
        };
        C y0 = w0 * E(false, false, false) + w1 * E(true, false, false);
        C y1 = w0 * E(false, true, false) + w1 * E(true, true, false);
        C v = w0 * y0 + w1 * y1;
        if (D == 3) {
            C y2 = w0 * E(false, false, true) + w1 * E(true, false, true);
            C y3 = w0 * E(false, true, true) + w1 * E(true, true, true);
            v = w0 * v + w1 * (w0 * y2 + w1 * y3);
        }
        const int idx = box_idx(Nf, i, j, k);
        U[idx] = U[idx] + v;
    }
}

template <int D, typename C>
__global__ void __launch_bounds__(kTailThreads) k_coarse_tail(TailParams<C> P, SGrid g0, const C* __restrict__ fg,
                                                              C* __restrict__ ug)
{
    extern __shared__ __align__(16) unsigned char tail_lds[];
    if (batch_idle(g0)) return;
    fg = batch_at(fg, g0);
    ug = batch_at(ug, g0);
    C* const lds = reinterpret_cast<C*>(tail_lds);
    const C inv2d = (C)(1.0 / (2.0 * D));
    auto U = [&](int a) { return lds + P.off[a]; };
    auto F = [&](int a) { return lds + P.off[a] + box_size<D>(P.N[a]); };
    auto sweep = [&](int a) {
        for (int colour = 0; colour < 2; colour++) {
            tail_sweep<D, C>(U(a), F(a), P.N[a], P.rN[a], P.rS[a], P.h2[a], inv2d, P.gr[a], colour);
            __syncthreads();
        }
    };
    {
        const int* N = P.N[0];
        const int total = box_active<D>(N);
        C* u = U(0);
        C* f = F(0);
        for (int t = threadIdx.x; t < total; t += kTailThreads) {
            int i, j, k;
            tail_point<D>(t, N, P.rN[0], i, j, k);
            const int idx = box_idx(N, i, j, k);
            f[idx] = fg[pos<D, C>(g0, i, j, k)];
            u[idx] = (C)0;
        }
        __syncthreads();
    }
    for (int it = 0; it < P.n_pre; it++) sweep(0);
    int a = 0;
    while (a + 1 < P.nlev) {
        tail_restrict<D, C>(U(a), F(a), P.N[a], P.inv_h2[a], P.gr[a], U(a + 1), F(a + 1), P.N[a + 1], P.rN[a + 1]);
        __syncthreads();
        for (int it = 0; it < P.n_pre; it++) sweep(a + 1);
        a++;
    }
    while (a > 0) {
        tail_prolong<D, C>(U(a), P.N[a], P.gr[a], U(a - 1), P.N[a - 1], P.rN[a - 1]);
        __syncthreads();
        for (int it = 0; it < P.n_post; it++) sweep(a - 1);
        a--;
    }
    {
        const int* N = P.N[0];
        const int total = box_active<D>(N);
        const C* u = U(0);
        for (int t = threadIdx.x; t < total; t += kTailThreads) {
            int i, j, k;
            tail_point<D>(t, N, P.rN[0], i, j, k);
            ug[pos<D, C>(g0, i, j, k)] = u[box_idx(N, i, j, k)];
        }
    }
}

// ------------------------------------------------------------------ defect correction
// Outer FP64 pass of the mixed-precision solve, fused into one sweep over the
// level-0 active points:
//   1. phi_out = phi_in + factor * e_in (only when UPD; e_in is zero on the
//      ghost layer, so the updated potential there is phi_in's);
//   2. r64 = f - lap(phi_out), the stop test's residual, and its max norm;
//   3. r = r64 * rscale in the low precision TL (the next inner right-hand side);
//   4. the next correction's start e_out: zero, except that with first_red the
//      first red half sweep from e = 0 is done here (e = -h2 r / 2d on red
//      points, in the smoother's arithmetic), so the inner cycle starts with black.
// phi_out and e_out are other buffers than phi_in and e_in: neighbours read the
// old values while the pass writes the new ones.
template <typename TL, bool UPD>
struct DcIn {
    const double* __restrict__ p;
    const TL* __restrict__ e;
    double factor;
    __device__ __forceinline__ double operator()(size_t i) const
    {
        double v = p[i];
        if (UPD) v = __fma_rn(factor, (double)(float)e[i], v);
        return v;
    }
};

template <typename TL>
__device__ __forceinline__ void dc_out(size_t self, int colour, double v, double rscale, TL* __restrict__ r,
                                       TL* __restrict__ eout, int first_red, float h2l, float inv2d)
{
    const TL rl = (TL)(float)(v * rscale);
    r[self] = rl;
    TL e0 = (TL)0.0f;
    if (colour == 0 && first_red) e0 = (TL)((0.0f - h2l * (float)rl) * inv2d);
    if (eout) eout[self] = e0;
}

// r'' = r32 * rscale on the active points of a level (r32: f - lap phi kept in
// FP32 by the level's first residual pass), rounded through FP32 as the outer
// pass rounds, and the next correction's start as the outer pass writes it (the
// red half sweep from zero on red points, zero on black) when e is not null
template <int D, typename TL>
__global__ void __launch_bounds__(kBlock) k_dc_scale(SGrid g, const float* __restrict__ r32, double rscale,
                                                     TL* __restrict__ r, TL* __restrict__ e, int first_red,
                                                     float h2l, float inv2d)
{
    const int my = g.ny - 2, mz = g.nz - 2;
    const long total = (long)g.hx * my * (D == 3 ? mz : 1);
    const long stride = (long)gridDim.x * kBlock;
    for (long t = xcd_block() * kBlock + threadIdx.x; t < total; t += stride) {
        const int h = (int)(t % g.hx);
        const long rr = t / g.hx;
        const int pj = 1 + (int)(rr % my);
        const int pk = D == 3 ? 1 + (int)(rr / my) : 0;
        const size_t row = row_base(g, pj, pk);
        for (int c = 0; c < 2; c++) {
            const int pi = 2 * h + ((c + pj + pk + D) & 1);
            if (pi < 1 || pi > g.nx - 2) continue;
            const size_t self = (size_t)c * g.cs + row + h;
            dc_out<TL>(self, c, (double)r32[self], rscale, r, e, first_red, h2l, inv2d);
        }
    }
}

template <int D, typename TL, bool UPD>
__global__ void __launch_bounds__(kBlock) k_dc_outer(SGrid g, DcIn<TL, UPD> in, double* __restrict__ pout,
                                                     const double* __restrict__ f, double inv_h2, double rscale,
                                                     TL* __restrict__ r, TL* __restrict__ eout, int first_red,
                                                     float h2l, float inv2d, unsigned long long* maxbits)
{
    const int my = g.ny - 2, mz = g.nz - 2;
    long total = (long)g.hx * my * (D == 3 ? mz : 1);
    long stride = (long)gridDim.x * kBlock;
    size_t ny = (size_t)g.hx, nz = g.ps;
    unsigned long long best = 0;
    for (long t = xcd_block() * kBlock + threadIdx.x; t < total; t += stride) {
        int h = (int)(t % g.hx);
        long rr = t / g.hx;
        int pj = 1 + (int)(rr % my);
        int pk = D == 3 ? 1 + (int)(rr / my) : 0;
        size_t row = row_base(g, pj, pk);
        for (int c = 0; c < 2; c++) {
            int pi = 2 * h + ((c + pj + pk + D) & 1);
            if (pi < 1 || pi > g.nx - 2) continue;
            size_t o = (size_t)(c ^ 1) * g.cs + row;
            size_t self = (size_t)c * g.cs + row + h;
            double s = in(o + ((pi - 1) >> 1));
            s = s + in(o + ((pi + 1) >> 1));
            s = s + in(o - ny + h);
            s = s + in(o + ny + h);
            if (D == 3) {
                s = s + in(o - nz + h);
                s = s + in(o + nz + h);
            }
            const double cen = in(self);
            if (UPD) pout[self] = cen;
            double v = resid(f[self], s, cen, 2.0 * D, inv_h2);
            dc_out<TL>(self, c, v, rscale, r, eout, first_red, h2l, inv2d);
            unsigned long long b = abs_bits(v);
            best = b > best ? b : best;
        }
    }
    block_max_to(best, maxbits);
}

// 3-D form marching along z like k_resid_norm3: a thread owns both colours of
// one compact column of a chunk of planes and keeps the updated potential at
// pk-1, pk, pk+1 in registers.
template <typename TL, bool UPD>
__global__ void __launch_bounds__(kBlock) k_dc_outer3(SGrid g, DcIn<TL, UPD> in, double* __restrict__ pout,
                                                      const double* __restrict__ f, double inv_h2, double rscale,
                                                      TL* __restrict__ r, TL* __restrict__ eout, int first_red,
                                                      float h2l, float inv2d, int pblocks,
                                                      unsigned long long* maxbits)
{
    const int my = g.ny - 2, mz = g.nz - 2;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    unsigned long long best = 0;
    // flat index over the whole (padded) plane: aligned wave segments; the ghost
    // rows and the padding have no work
    const int pj = t / g.hx;
    const int h = t - pj * g.hx;
    if (pj >= 1 && pj <= my) {
        const int k0 = 1 + zc * kNormChunk;
        const int k1 = min(k0 + kNormChunk - 1, mz);
        const size_t plane = g.ps;
        const size_t col = (size_t)pj * g.hx + h;
        const size_t cs = g.cs;
        double below[2], cur[2];
        for (int c = 0; c < 2; c++) {
            below[c] = in(c * cs + (size_t)(k0 - 1) * plane + col);
            cur[c] = in(c * cs + (size_t)k0 * plane + col);
        }
        for (int pk = k0; pk <= k1; pk++) {
            const size_t here = (size_t)pk * plane + col;
            double above[2] = {in(here + plane), in(cs + here + plane)};
            for (int c = 0; c < 2; c++) {
                const int o = c ^ 1;
                const int par = (c + pj + pk + 3) & 1;
                const int pi = 2 * h + par;
                if (pi < 1 || pi > g.nx - 2) continue;
                const size_t oh = o * cs + here;
                double xm = par ? cur[o] : in(oh - 1);
                double xp = par ? in(oh + 1) : cur[o];
                double s = xm + xp;
                s = s + in(oh - g.hx);
                s = s + in(oh + g.hx);
                s = s + below[o];
                s = s + above[o];
                const size_t self = c * cs + here;
                if (UPD) pout[self] = cur[c];
                double v = resid(f[self], s, cur[c], 6.0, inv_h2);
                dc_out<TL>(self, c, v, rscale, r, eout, first_red, h2l, inv2d);
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

// Paired form of k_dc_outer3 (row length hx even): a thread owns the compact
// points h0 = 2 hp and h0 + 1 of both colours and moves each pair of the
// potential with one 16-byte access and each pair of e, r with one 2- or
// 4-byte access; the extra x-neighbour (h0 - 1 or h0 + 2) is a single load,
// or, in the pass without the update, comes from the adjacent lane by a DPP
// shift (a load at a wave's edge).  Same arithmetic per point as k_dc_outer3.
template <typename TL, bool UPD>
__device__ __forceinline__ Pair<double> dc_pair(const DcIn<TL, UPD>& in, size_t i)
{
    Pair<double> v = *(const Pair<double>*)(in.p + i);
    if (UPD) {
        const Pair<TL> e = *(const Pair<TL>*)(in.e + i);
        v.a = __fma_rn(in.factor, (double)(float)e.a, v.a);
        v.b = __fma_rn(in.factor, (double)(float)e.b, v.b);
    }
    return v;
}

constexpr int kDcChunk = 8;  // planes per thread of the paired DC pass (aligned layout: 2, 4, 8 give 1.02, 0.93, 0.91 ms)
constexpr int kDcGroup = 2;  // planes of the DC pass whose loads are issued together (1, 2, 4 measured alike)
// residual pass without the update (UPD = false): extra x-neighbour from the
// adjacent lane, edge lanes load it (611 -> 587 us at 514^3); with the update
// the shifts measured slower (881 -> 945 us) and the load stays
template <bool UPD>
constexpr bool kDcDppExtra = !UPD;

// OUT = false: only the max norm of the residual (the stop test's residual
// pass), no outputs.  eout == nullptr: the next correction's start is not
// stored (its first black half sweep forms the red values from r).
template <typename TL, bool UPD, bool OUT = true>
__global__ void __launch_bounds__(kBlock) k_dc_outer3_pair(SGrid g, DcIn<TL, UPD> in, double* __restrict__ pout,
                                                           const double* __restrict__ f, double inv_h2, double rscale,
                                                           TL* __restrict__ r, TL* __restrict__ eout, int first_red,
                                                           float h2l, float inv2d, int pblocks,
                                                           unsigned long long* maxbits)
{
    if (batch_idle(g)) return;
    in.p = batch_at(in.p, g);
    if (UPD) in.e = batch_at(in.e, g);
    pout = batch_at(pout, g);
    f = batch_at(f, g);
    r = batch_at(r, g);
    eout = batch_at(eout, g);
    maxbits += blockIdx.y;
    const int my = g.ny - 2, mz = g.nz - 2;
    const int lb = (int)xcd_block();
    const int zc = lb / pblocks;
    const int t = (lb - zc * pblocks) * kBlock + (int)threadIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    unsigned long long best = 0;
    // flat pair index over the whole (padded) plane, as in k_smooth_zmarch3_pair
    const int q = 2 * t;
    const int pj = q / g.hx;
    const int h0 = q - pj * g.hx;
    if (pj >= 1 && pj <= my) {
        const int k0 = 1 + zc * kDcChunk;
        const int k1 = min(k0 + kDcChunk - 1, mz);
        const size_t plane = g.ps;
        const size_t col = (size_t)pj * g.hx + h0;
        const size_t cs = g.cs;
        Pair<double> below[2], cur[2];
        for (int c = 0; c < 2; c++) {
            below[c] = dc_pair(in, c * cs + (size_t)(k0 - 1) * plane + col);
            cur[c] = dc_pair(in, c * cs + (size_t)k0 * plane + col);
        }
        // the loads of one plane: updated potential above and in the rows
        // beside, the extra x-neighbour of each colour, and f
        struct Plane {
            Pair<double> above[2], ym[2], yp[2], fv[2];
            double ex[2];
        };
        auto load = [&](int pk, Plane& d) {
            const size_t here = (size_t)pk * plane + col;
            for (int c = 0; c < 2; c++) {
                d.above[c] = dc_pair(in, c * cs + here + plane);
                d.ym[c] = dc_pair(in, c * cs + here - g.hx);
                d.yp[c] = dc_pair(in, c * cs + here + g.hx);
                d.fv[c] = kDcLoadNt ? load_nt((const Pair<double>*)(f + c * cs + here))
                                    : *(const Pair<double>*)(f + c * cs + here);
                // the extra x-neighbour of colour c's points (other colour o), inside
                // the plane (neighbouring row at the row ends); with kDcDppExtra<UPD>
                // only a wave's edge lane loads it, the others take it from the
                // adjacent lane's pair in step
                const int par = (c + pj + pk + 3) & 1;
                d.ex[c] = 0.0;
                if (!kDcDppExtra<UPD> || (par ? lane == 63 : lane == 0))
                    d.ex[c] = in((c ^ 1) * cs + (par ? here + 2 : here - 1));
            }
        };
        auto step = [&](int pk, const Plane& d) {
            const size_t here = (size_t)pk * plane + col;
            for (int c = 0; c < 2; c++) {
                const int o = c ^ 1;
                const int par = (c + pj + pk + 3) & 1;
                const int pi0 = 2 * h0 + par;
                const bool a0 = pi0 >= 1, a1 = pi0 + 2 <= g.nx - 2;
                double ex = d.ex[c];
                if (kDcDppExtra<UPD>) {
                    // flat numbering: lane + 1 holds slots h0 + 2, h0 + 3 of colour o
                    // in this plane and lane - 1 slots h0 - 2, h0 - 1 (the same
                    // updated values the load would form); across a row end the
                    // shifted value feeds only a point outside the active box
                    const double nx = dpp_next(cur[o].a), pv = dpp_prev(cur[o].b);
                    if (!(par ? lane == 63 : lane == 0)) ex = par ? nx : pv;
                }
                double xm0, xp0, xm1, xp1;
                if (par) {
                    xm0 = cur[o].a;
                    xp0 = cur[o].b;
                    xm1 = cur[o].b;
                    xp1 = ex;
                } else {
                    xm0 = ex;
                    xp0 = cur[o].a;
                    xm1 = cur[o].a;
                    xp1 = cur[o].b;
                }
                double s0 = xm0 + xp0;
                s0 = s0 + d.ym[o].a;
                s0 = s0 + d.yp[o].a;
                s0 = s0 + below[o].a;
                s0 = s0 + d.above[o].a;
                double s1 = xm1 + xp1;
                s1 = s1 + d.ym[o].b;
                s1 = s1 + d.yp[o].b;
                s1 = s1 + below[o].b;
                s1 = s1 + d.above[o].b;
                const size_t self = c * cs + here;
                const Pair<double> fv = d.fv[c];
                const double v0 = resid(fv.a, s0, cur[c].a, 6.0, inv_h2);
                const double v1 = resid(fv.b, s1, cur[c].b, 6.0, inv_h2);
                Pair<TL> rl, el;
                rl.a = (TL)(float)(v0 * rscale);
                rl.b = (TL)(float)(v1 * rscale);
                el.a = el.b = (TL)0.0f;
                if (c == 0 && first_red) {
                    el.a = (TL)((0.0f - h2l * (float)rl.a) * inv2d);
                    el.b = (TL)((0.0f - h2l * (float)rl.b) * inv2d);
                }
                if (a0 && a1) {
                    if (UPD) store_nt((Pair<double>*)(pout + self), cur[c]);
                    if (OUT) {
                        *(Pair<TL>*)(r + self) = rl;
                        if (eout) *(Pair<TL>*)(eout + self) = el;
                    }
                    unsigned long long b0 = abs_bits(v0), b1 = abs_bits(v1);
                    b0 = b1 > b0 ? b1 : b0;
                    best = b0 > best ? b0 : best;
                } else {
                    if (a0) {
                        if (UPD) store_nt(pout + self, cur[c].a);
                        if (OUT) {
                            r[self] = rl.a;
                            if (eout) eout[self] = el.a;
                        }
                        unsigned long long b0 = abs_bits(v0);
                        best = b0 > best ? b0 : best;
                    }
                    if (a1) {
                        if (UPD) store_nt(pout + self + 1, cur[c].b);
                        if (OUT) {
                            r[self + 1] = rl.b;
                            if (eout) eout[self + 1] = el.b;
                        }
                        unsigned long long b1 = abs_bits(v1);
                        best = b1 > best ? b1 : best;
                    }
                }
            }
            for (int c = 0; c < 2; c++) {
                below[c] = cur[c];
                cur[c] = d.above[c];
            }
        };
        int pk = k0;
        // groups of kDcGroup planes: every load of the group is issued before its
        // first update
        for (; pk + kDcGroup - 1 <= k1; pk += kDcGroup) {
            Plane d[kDcGroup];
#pragma unroll
            for (int q = 0; q < kDcGroup; q++) load(pk + q, d[q]);
#pragma unroll
            for (int q = 0; q < kDcGroup; q++) step(pk + q, d[q]);
        }
        for (; pk <= k1; pk++) {
            Plane d;
            load(pk, d);
            step(pk, d);
        }
    }
    block_max_to(best, maxbits);
}

// Copy of the ghost layer (the points outside the active box) of a nested-level
// array: gives a second potential buffer the same fixed outer values.
template <int D>
__global__ void __launch_bounds__(kBlock) k_copy_ghosts(SGrid g, const double* __restrict__ src, double* __restrict__ dst)
{
    const int Q[3] = {g.nx, g.ny, g.nz};
    int t = blockIdx.x * kBlock + threadIdx.x;
    int face = blockIdx.y;
    int axis = face >> 1, side = face & 1;
    const int a1 = D == 3 ? (axis + 1) % 3 : (axis ^ 1), a2 = (axis + 2) % 3;
    int per = D == 3 ? Q[a1] * Q[a2] : Q[a1];
    if (t >= per) return;
    int p[3] = {0, 0, 0};
    p[axis] = side ? Q[axis] - 1 : 0;
    if (D == 3) {
        p[a1] = t % Q[a1];
        p[a2] = t / Q[a1];
    } else {
        p[a1] = t;
    }
    size_t i = pos<D, double>(g, p[0], p[1], D == 3 ? p[2] : 0);
    dst[i] = src[i];
}

// dst(p) = src(p + shift) over the box lo <= p_a <= hi of grid gd (colour and
// compact position taken in each grid's own padded indices): moves the relaxed
// domain of a level between the level array and an array of its own
template <int D>
__global__ void __launch_bounds__(kBlock) k_copy_box(SGrid gs, const double* __restrict__ src, SGrid gd,
                                                     double* __restrict__ dst, int lo, int wx, int wy, int wz,
                                                     int shift)
{
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    const long total = D == 3 ? (long)wx * wy * wz : (long)wx * wy;
    if (t >= total) return;
    const int i = lo + (int)(t % wx);
    const long r = t / wx;
    const int j = lo + (int)(r % wy);
    const int k = D == 3 ? lo + (int)(r / wy) : 0;
    dst[pos<D, double>(gd, i, j, k)] = at<D>(src, gs, i + shift, j + shift, D == 3 ? k + shift : 0);
}

}  // namespace

// ------------------------------------------------------------------ launchers
#define NP_DISPATCH(dim, KERNEL, grid, block, st, ...)                                    \
    do {                                                                                  \
        if ((dim) == 3) hipLaunchKernelGGL((KERNEL<3>), (grid), (block), 0, (st), __VA_ARGS__); \
        else hipLaunchKernelGGL((KERNEL<2>), (grid), (block), 0, (st), __VA_ARGS__);           \
    } while (0)

static long npoints(const SGrid& g) { return (long)g.nx * g.ny * g.nz; }
static long ncompact_active(int dim, const SGrid& g)
{
    return (long)g.hx * (g.ny - 2) * (dim == 3 ? g.nz - 2 : 1);
}

void launch_level0_init(int dim, hipStream_t st, SGrid g, const double* rho0, const double* phi_outer,
                        double fourpiG, double* phi, double* f, unsigned long long* fmax)
{
    int blocks = ceil_div(npoints(g), kBlock);
    if (blocks > kInitBlocks) blocks = kInitBlocks;
    NP_DISPATCH(dim, k_level0_init, dim3(blocks), dim3(kBlock), st, g, rho0, phi_outer, fourpiG, phi, f, fmax);
}

void launch_interface_fill(int dim, hipStream_t st, SGrid gc, const double* phic, const double* fc, SGrid gf,
                           int offx, int offy, int offz, const double* rho, double fourpiG, double* phif,
                           double* ff, unsigned long long* fmax)
{
    if (dim == 3 && gf.hx % 2 == 0 && 2 * gc.cs < (1ull << 31)) {
        const int pblocks = ceil_div((long)(gf.ps / 2), kBlock);
        const int chunks = ceil_div(gf.nz / 2, kFillPairChunk);
        hipLaunchKernelGGL(k_interface_fill3_pair, dim3(pblocks * chunks), dim3(kBlock), 0, st, gc, phic, fc, gf, offx,
                           offy, offz, rho, fourpiG, phif, ff, pblocks, fmax);
        return;
    }
    if (dim == 3) {
        const long Mx = (gf.nx + 1) / 2, My = (gf.ny + 1) / 2, Mz = (gf.nz + 1) / 2;
        const int pblocks = ceil_div(Mx * My, kBlock);
        hipLaunchKernelGGL(k_interface_fill3_zm, dim3(pblocks * ceil_div(Mz, kFillChunk)), dim3(kBlock), 0, st, gc, phic,
                           fc, gf, offx, offy, offz, rho, fourpiG, phif, ff, pblocks, fmax);
        return;
    }
    NP_DISPATCH(dim, k_interface_fill, dim3(ceil_div(npoints(gf), kBlock)), dim3(kBlock), st, gc, phic, fc, gf,
                offx, offy, offz, rho, fourpiG, phif, ff, fmax);
}

void launch_forces(int dim, hipStream_t st, SGrid g, double dx, const double* phi, double* fx, double* fy,
                   double* fz)
{
    double m12dx = -1.0 / (12.0 * dx);
    const long nx = g.nx - 4, ny = g.ny - 4, nz = g.nz - 4;
    if (dim == 3) {
        const long waves = ceil_div(nx * ((ny + kForceRows - 1) / kForceRows), kForceOwn);
        const int pblocks = ceil_div(waves, kForceBlock / 64);
        hipLaunchKernelGGL(k_forces3_zm<false>, dim3(pblocks * ceil_div(nz, kForceChunk)), dim3(kForceBlock), 0, st,
                           g, m12dx, phi, fx, fy, fz, pblocks, nullptr);
        return;
    }
    Strip sp = make_strip((int)nx, (int)ny, 1, 16);
    NP_DISPATCH(dim, k_forces, dim3(ceil_div(nx * ny, kBlock)), dim3(kBlock), st, g, m12dx, phi, fx, fy, fz, sp);
}

void launch_force_delta(int dim, hipStream_t st, SGrid g, double dx, const double* phi, double* F,
                        unsigned long long* maxbits)
{
    long total = (long)(g.nx - 4) * (g.ny - 4) * (dim == 3 ? g.nz - 4 : 1);
    double m12dx = -1.0 / (12.0 * dx);
    if (dim == 3) {
        // the z-march force kernel with the comparison (components at F, F + total, F + 2 total)
        const long nx = g.nx - 4, ny = g.ny - 4, nz = g.nz - 4;
        const long waves = ceil_div(nx * ((ny + kForceRows - 1) / kForceRows), kForceOwn);
        const int pblocks = ceil_div(waves, kForceBlock / 64);
        hipLaunchKernelGGL(k_forces3_zm<true>, dim3(pblocks * ceil_div(nz, kForceChunk)), dim3(kForceBlock), 0, st, g,
                           m12dx, phi, F, F + total, F + 2 * total, pblocks, maxbits);
        return;
    }
    NP_DISPATCH(dim, k_force_delta, dim3(ceil_div(total, kBlock)), dim3(kBlock), st, g, m12dx, phi, F, maxbits);
}

void launch_export(int dim, hipStream_t st, SGrid g, const double* a, double* out)
{
    NP_DISPATCH(dim, k_export, dim3(ceil_div(npoints(g), kBlock)), dim3(kBlock), st, g, a, out);
}

void launch_norm(int dim, hipStream_t st, SGrid g, const double* u, const double* f, double inv_h2, int mode,
                 unsigned long long* maxbits)
{
    if (dim == 3 && mode == 0 && g.hx % 2 == 0) {
        // the paired DC pass without outputs: same residual, same order of operations
        const long mz = g.nz - 2;
        const int pblocks = ceil_div((long)(g.ps / 2), kBlock);
        hipLaunchKernelGGL((k_dc_outer3_pair<float, false, false>), dim3(pblocks * ceil_div(mz, kDcChunk), g.nb), dim3(kBlock), 0,
                           st, g, DcIn<float, false>{u, nullptr, 0.0}, nullptr, f, inv_h2, 0.0, nullptr, nullptr, 0, 0.0f,
                           0.0f, pblocks, maxbits);
        return;
    }
    if (dim == 3 && mode == 0) {
        long mz = g.nz - 2;
        int pblocks = ceil_div((long)g.ps, kBlock);
        int chunks = ceil_div(mz, kNormChunk);
        hipLaunchKernelGGL(k_resid_norm3, dim3(pblocks * chunks, g.nb), dim3(kBlock), 0, st, g, u, f, inv_h2, pblocks,
                           maxbits);
        return;
    }
    int blocks = ceil_div(ncompact_active(dim, g), kBlock);
    if (blocks > 2048) blocks = 2048;
    NP_DISPATCH(dim, k_norm, dim3(blocks, g.nb), dim3(kBlock), st, g, u, f, inv_h2, mode, maxbits);
}

void launch_box_resid_norm3(hipStream_t st, SGrid g, const double* u, const double* f, double inv_h2,
                            unsigned long long* maxbits)
{
    const long nb = (long)((g.nx - 2 + kBox - 1) / kBox) * ((g.ny - 2 + kBox - 1) / kBox) *
                    ((g.nz - 2 + kBox - 1) / kBox);
    hipLaunchKernelGGL(k_box_resid_norm3, dim3(ceil_div(nb, kBlock)), dim3(kBlock), 0, st, g, u, f, inv_h2, maxbits);
}

void launch_set_u64(hipStream_t st, unsigned long long* p, int count, unsigned long long v)
{
    hipLaunchKernelGGL(k_set_u64, dim3(ceil_div(count, 64)), dim3(64), 0, st, p, count, v);
}

template <typename T>
void launch_half_sweep(int dim, hipStream_t st, SGrid g, T* u, const T* f, int colour, double h2, int fine,
                       const Rule3& rule)
{
    using C = typename Compute<T>::type;
    dim3 grid(ceil_div(ncompact_active(dim, g), kBlock), g.nb);
    C inv2d = (C)(1.0 / (2.0 * dim));
    const GRule<C> gr = grule<C>(rule);
    if (dim == 3 && fine && sizeof(T) <= 4 && (g.hx % 2) == 0) {
        // 2- and 4-byte storage: two compact points per thread, paired loads
        // (on the coarse levels, with the ghost rule, this form measured slower
        // than k_smooth_zmarch3)
        long mz = g.nz - 2;
        int pblocks = ceil_div((long)(g.ps / 2), kSmoothPairBlock);
        int chunks = ceil_div(mz, kZChunk0);
        hipLaunchKernelGGL((k_smooth_zmarch3_pair<T>), dim3(pblocks * chunks, g.nb), dim3(kSmoothPairBlock), 0, st, u, f, g,
                           colour, (C)h2, inv2d, pblocks);
        return;
    }
    if (dim == 3 && (fine || g.nz >= 34)) {
        // z-march; the level-0 instance (TAG 0) is kept apart from the
        // coarse-level one (TAG 1) so that profiles separate them
        long mz = g.nz - 2;
        int pblocks = ceil_div((long)g.ps, kBlock);
        const bool small = !fine && mz <= kSmallPlanes;
        int chunks = ceil_div(mz, fine ? kZChunk0 : (small ? kZChunkSmall : kZChunk1));
        if (fine)
            hipLaunchKernelGGL((k_smooth_zmarch3<T, 0>), dim3(pblocks * chunks, g.nb), dim3(kBlock), 0, st, u, f, g, colour,
                               (C)h2, inv2d, pblocks, gr);
        else if (small)
            hipLaunchKernelGGL((k_smooth_zmarch3<T, 2>), dim3(pblocks * chunks, g.nb), dim3(kBlock), 0, st, u, f, g, colour,
                               (C)h2, inv2d, pblocks, gr);
        else
            hipLaunchKernelGGL((k_smooth_zmarch3<T, 1>), dim3(pblocks * chunks, g.nb), dim3(kBlock), 0, st, u, f, g, colour,
                               (C)h2, inv2d, pblocks, gr);
        return;
    }
    if (fine) {
        hipLaunchKernelGGL((k_smooth_fine<2, T>), grid, dim3(kBlock), 0, st, u, f, g, colour, (C)h2, inv2d);
    } else {
        if (dim == 3)
            hipLaunchKernelGGL((k_half_sweep<3, T>), grid, dim3(kBlock), 0, st, u, f, g, colour, (C)h2, inv2d, gr);
        else
            hipLaunchKernelGGL((k_half_sweep<2, T>), grid, dim3(kBlock), 0, st, u, f, g, colour, (C)h2, inv2d, gr);
    }
}

template <typename T>
void launch_half_sweep_seeded(hipStream_t st, SGrid g, T* u, const T* f, double h2, int store_red)
{
    using C = typename Compute<T>::type;
    const long mz = g.nz - 2;
    const int pblocks = ceil_div((long)(g.ps / 2), kSmoothPairBlock);
    const int chunks = ceil_div(mz, kZChunk0);
    if (store_red)
        hipLaunchKernelGGL((k_smooth_zmarch3_pair<T, 2>), dim3(pblocks * chunks, g.nb), dim3(kSmoothPairBlock), 0, st,
                           u, f, g, 1, (C)h2, (C)(1.0 / 6.0), pblocks);
    else
        hipLaunchKernelGGL((k_smooth_zmarch3_pair<T, 1>), dim3(pblocks * chunks, g.nb), dim3(kSmoothPairBlock), 0, st,
                           u, f, g, 1, (C)h2, (C)(1.0 / 6.0), pblocks);
}

long full_sweep_waves(const SGrid& g)
{
    const int my = g.ny - 2, mz = g.nz - 2;
    const bool paired = g.hx % 2 == 0;
    const int nrg = ceil_div(my, paired ? kFsPairRows : kFsRows);
    const long waves = ceil_div((long)nrg * (paired ? g.hx / 2 : g.hx), kFsOwn);
    return (long)ceil_div(waves, kFsBlock / 64) * (kFsBlock / 64) * ceil_div(mz, paired ? kFsPairChunk : kFsChunk);
}

template <typename T>
void launch_full_sweep(hipStream_t st, SGrid g, const T* P, T* Q, const T* f, double h2, double inv_h2, int mode,
                       int rev, unsigned long long* maxbits)
{
    const int my = g.ny - 2, mz = g.nz - 2;
    const double inv2d = 1.0 / 6.0;
    if (g.hx % 2 == 0) {
        const int nrg = ceil_div(my, kFsPairRows);
        const long waves = ceil_div((long)nrg * (g.hx / 2), kFsOwn);
        const int wblocks = ceil_div(waves, kFsBlock / 64);
        const dim3 grid(wblocks * ceil_div(mz, kFsPairChunk));
#define NP_FSP(M)                                                                                                      \
    hipLaunchKernelGGL((k_full_sweep3_pair<T, kFsPairRows, kFsPairChunk, M>), grid, dim3(kFsBlock), 0, st, P, Q, f, g, h2, \
                       inv2d, inv_h2, nrg, wblocks, rev, maxbits)
        switch (mode & 3) {
        case 0: NP_FSP(0); break;
        case 1: NP_FSP(1); break;
        case 2: NP_FSP(2); break;
        default: NP_FSP(3); break;
        }
#undef NP_FSP
        return;
    }
    const int nrg = ceil_div(my, kFsRows);
    const long waves = ceil_div((long)nrg * g.hx, kFsOwn);
    const int wblocks = ceil_div(waves, kFsBlock / 64);
    const dim3 grid(wblocks * ceil_div(mz, kFsChunk));
#define NP_FS(M)                                                                                                    \
    hipLaunchKernelGGL((k_full_sweep3<T, kFsRows, kFsChunk, M>), grid, dim3(kFsBlock), 0, st, P, Q, f, g, h2, inv2d, \
                       inv_h2, nrg, wblocks, rev, maxbits)
    switch (mode & 3) {
    case 0: NP_FS(0); break;
    case 1: NP_FS(1); break;
    case 2: NP_FS(2); break;
    default: NP_FS(3); break;
    }
#undef NP_FS
}

template <typename TF, typename TC>
void launch_resid_restrict(int dim, hipStream_t st, SGrid gf, const TF* u, const TF* f, double inv_h2, double out_scale,
                           SGrid gc, TC* fc, TC* ec, int rule, const Rule3& fine_rule, double seed_h2)
{
    using C = typename Compute<TC>::type;
    const C sh2 = (C)seed_h2, inv2d = (C)(1.0 / (2.0 * dim));
    const long Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    long total = dim == 3 ? Ncx * Ncy * Ncz : Ncx * Ncy;
    dim3 grid(ceil_div(total, kBlock), gf.nb);
    const GRule<C> gr = grule<C>(fine_rule);
    if (dim == 3) {
        // z-march: 4 coarse planes per thread on large grids, 1 on small ones
        // (there the column count alone does not fill the chip)
        const int kch = Ncx * Ncy >= 128 * 128 ? 4 : 1;
        const int pblocks = ceil_div(Ncx * Ncy, kBlock);
        const dim3 zgrid(pblocks * ceil_div(Ncz, kch), gf.nb);
        if constexpr (sizeof(TF) == 2) {
            if (!rule && gf.nx - 2 == 2 * Ncx && gf.ny - 2 == 2 * Ncy && gf.nz - 2 == 2 * Ncz && gf.hx % 2 == 0 &&
                2 * gf.cs < (1ull << 31)) {
                // multigrid level 0 in 2-byte storage, paired layout
                const long waves = ceil_div((long)(gf.hx / 2) * Ncy, 63);
                const int pb = ceil_div(waves, kBlock / 64);
                const dim3 pgrid(pb * ceil_div(Ncz, kRestrictPairChunk), gf.nb);
                hipLaunchKernelGGL((k_restrict3_pair<TF, TC>), pgrid, dim3(kBlock), 0, st, u, f, gf, (C)inv_h2,
                                   (C)out_scale, gc, fc, ec, pb, sh2, inv2d);
                return;
            }
        }
        if (!rule && gf.nx - 2 == 2 * Ncx && gf.ny - 2 == 2 * Ncy && gf.nz - 2 == 2 * Ncz &&
            2 * gf.cs * sizeof(TF) < (1ull << 31)) {
            // multigrid level 0: uniform addressing
            hipLaunchKernelGGL((k_restrict3_l0<TF, TC>), zgrid, dim3(kBlock), 0, st, u, f, gf, (C)inv_h2, (C)out_scale,
                               gc, fc, ec, pblocks, kch, sh2, inv2d);
            return;
        }
        if (rule)
            hipLaunchKernelGGL((k_restrict3_zm<TF, TC, true>), zgrid, dim3(kBlock), 0, st, u, f, gf, (C)inv_h2,
                               (C)out_scale, gc, fc, ec, gr, pblocks, kch, sh2, inv2d);
        else
            hipLaunchKernelGGL((k_restrict3_zm<TF, TC, false>), zgrid, dim3(kBlock), 0, st, u, f, gf, (C)inv_h2,
                               (C)out_scale, gc, fc, ec, gr, pblocks, kch, sh2, inv2d);
    } else {
        if (rule)
            hipLaunchKernelGGL((k_resid_restrict<2, TF, TC, true>), grid, dim3(kBlock), 0, st, u, f, gf, (C)inv_h2,
                               (C)out_scale, gc, fc, ec, gr, sh2, inv2d);
        else
            hipLaunchKernelGGL((k_resid_restrict<2, TF, TC, false>), grid, dim3(kBlock), 0, st, u, f, gf, (C)inv_h2,
                               (C)out_scale, gc, fc, ec, gr, sh2, inv2d);
    }
}

bool black_restrict_fits(const SGrid& gf, const SGrid& gc)
{
    const long Ncx = gc.nx - 2, Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    return gf.nz > 1 && gf.nx - 2 == 2 * Ncx && gf.ny - 2 == 2 * Ncy && gf.nz - 2 == 2 * Ncz && gf.hx % 2 == 0 &&
           2 * gf.cs < (1ull << 31);
}

void launch_black_restrict(hipStream_t st, SGrid gf, __half* u, const __half* f, double h2, double inv_h2,
                           double out_scale, SGrid gc, float* fc, float* ec, double seed_h2, int seed)
{
    const long Ncy = gc.ny - 2, Ncz = gc.nz - 2;
    const long waves = ceil_div((long)(gf.hx / 2) * Ncy, 62);
    const int pb = ceil_div(waves, kBlock / 64);
    const dim3 grid(pb * ceil_div(Ncz, kBrChunk), gf.nb);
    const float inv2d = (float)(1.0 / 6.0);
    if (seed)
        hipLaunchKernelGGL((k_black_restrict3_pair<1>), grid, dim3(kBlock), 0, st, u, f, gf, (float)h2, (float)inv_h2,
                           (float)out_scale, gc, fc, ec, pb, (float)seed_h2, inv2d);
    else
        hipLaunchKernelGGL((k_black_restrict3_pair<0>), grid, dim3(kBlock), 0, st, u, f, gf, (float)h2, (float)inv_h2,
                           (float)out_scale, gc, fc, ec, pb, (float)seed_h2, inv2d);
}

template <typename TC, typename TF>
void launch_prolong_add(int dim, hipStream_t st, SGrid gc, const TC* ec, SGrid gf, TF* u, int black_only,
                        const Rule3& coarse_rule)
{
    using C = typename Compute<TC>::type;
    const GRule<C> gr = grule<C>(coarse_rule);
    dim3 grid(ceil_div(ncompact_active(dim, gf), kBlock), gf.nb);
    if (dim == 3 && black_only && (gf.hx % 2) == 0 && 2 * gf.cs < (1ull << 31) && 2 * gc.cs < (1ull << 31)) {
        // paired form: one paired load and store per fine plane and pair
        const long Mz = (gf.nz - 1) / 2;
        const int pblocks = ceil_div((long)(gf.ps / 2), kBlock);
        const int chunks = ceil_div(Mz, kProlongPairChunk);
        hipLaunchKernelGGL((k_prolong3_pair<TC, TF, kProlongPairChunk>), dim3(pblocks * chunks, gf.nb), dim3(kBlock), 0, st,
                           ec, gc, u, gf, gr, pblocks);
        return;
    }
    if (dim == 3) {
        // ceil(N_f / 2) coarse parents per axis
        const long Mx = (gf.nx - 1) / 2, My = (gf.ny - 1) / 2, Mz = (gf.nz - 1) / 2;
        // 8 coarse planes per thread on large grids, 4 from 100^2 columns (129^2
        // under a 514^3 level: coarse part 325 -> 320 us per cycle against 2), 2
        // or 1 on small ones (there the column count alone does not fill the chip)
        const int kch = Mx * My >= 200 * 200 ? 8 : (Mx * My >= 100 * 100 ? 4 : (Mz <= kSmallPlanes / 2 ? 1 : 2));
        const int pblocks = ceil_div(Mx * My, kBlock);
        const int chunks = ceil_div(Mz, kch);
        hipLaunchKernelGGL((k_prolong3_zm<TC, TF>), dim3(pblocks * chunks, gf.nb), dim3(kBlock), 0, st, ec, gc, u, gf,
                           black_only, gr, pblocks, kch);
    } else
        hipLaunchKernelGGL((k_prolong_add<2, TC, TF>), grid, dim3(kBlock), 0, st, ec, gc, u, gf, black_only, gr);
}

static size_t tail_box(int dim, const int* N)
{
    const size_t qx = (size_t)N[0] + 2, qy = (size_t)N[1] + 2, qz = (size_t)N[2] + 2;
    return dim == 3 ? qx * qy * qz : qx * qy;
}

size_t coarse_tail_lds_bytes(int dim, const int (*N)[3], int nlev, size_t esz)
{
    size_t e = 0;
    for (int a = 0; a < nlev; a++) e += 2 * tail_box(dim, N[a]);
    return e * esz;
}

template <typename T>
int launch_coarse_tail(int dim, hipStream_t st, int nlev, const int (*N)[3], const double* h, const Rule3* rule,
                       int n_pre, int n_post, SGrid g0, const T* f0, T* u0)
{
    if (nlev < 1 || nlev > kTailMaxLevels) return -1;
    const size_t bytes = coarse_tail_lds_bytes(dim, N, nlev, sizeof(T));
    if (bytes > kTailLdsBytes) return -1;
    TailParams<T> P{};
    P.nlev = nlev;
    P.n_pre = n_pre;
    P.n_post = n_post;
    int off = 0;
    for (int a = 0; a < nlev; a++) {
        for (int ax = 0; ax < 3; ax++) P.N[a][ax] = ax < dim ? N[a][ax] : 0;
        P.off[a] = off;
        off += 2 * (int)tail_box(dim, N[a]);
        P.h2[a] = (T)(h[a] * h[a]);
        P.inv_h2[a] = (T)(1.0 / (h[a] * h[a]));
        P.gr[a] = grule<T>(rule[a]);
        for (int ax = 0; ax < 3; ax++) P.rN[a][ax] = ax < dim ? 1.0f / (float)N[a][ax] : 0.0f;
        P.rS[a] = 1.0f / (float)((N[a][0] + 1) / 2);
    }
    if (dim == 3)
        hipLaunchKernelGGL((k_coarse_tail<3, T>), dim3(1, g0.nb), dim3(kTailThreads), bytes, st, P, g0, f0, u0);
    else
        hipLaunchKernelGGL((k_coarse_tail<2, T>), dim3(1, g0.nb), dim3(kTailThreads), bytes, st, P, g0, f0, u0);
    return 0;
}

template <typename TL>
void launch_dc_outer(int dim, hipStream_t st, SGrid g, const double* phi_in, const TL* e_in, double factor,
                     double* phi_out, const double* f, double inv_h2, double rscale, TL* r, TL* e_out, int first_red,
                     unsigned long long* maxbits)
{
    const float h2l = 1.0f, inv2d = (float)(1.0 / (2.0 * dim));
    const bool upd = e_in != nullptr;
    if (dim == 3 && g.hx % 2 == 0 && g.cs % 2 == 0) {
        long mz = g.nz - 2;
        int pblocks = ceil_div((long)(g.ps / 2), kBlock);
        dim3 grid(pblocks * ceil_div(mz, kDcChunk), g.nb);
        if (upd)
            hipLaunchKernelGGL((k_dc_outer3_pair<TL, true>), grid, dim3(kBlock), 0, st, g,
                               DcIn<TL, true>{phi_in, e_in, factor}, phi_out, f, inv_h2, rscale, r, e_out, first_red,
                               h2l, inv2d, pblocks, maxbits);
        else
            hipLaunchKernelGGL((k_dc_outer3_pair<TL, false>), grid, dim3(kBlock), 0, st, g,
                               DcIn<TL, false>{phi_in, nullptr, 0.0}, phi_out, f, inv_h2, rscale, r, e_out, first_red,
                               h2l, inv2d, pblocks, maxbits);
        return;
    }
    if (dim == 3) {
        long mz = g.nz - 2;
        int pblocks = ceil_div((long)g.ps, kBlock);
        dim3 grid(pblocks * ceil_div(mz, kNormChunk));
        if (upd)
            hipLaunchKernelGGL((k_dc_outer3<TL, true>), grid, dim3(kBlock), 0, st, g, DcIn<TL, true>{phi_in, e_in, factor},
                               phi_out, f, inv_h2, rscale, r, e_out, first_red, h2l, inv2d, pblocks, maxbits);
        else
            hipLaunchKernelGGL((k_dc_outer3<TL, false>), grid, dim3(kBlock), 0, st, g,
                               DcIn<TL, false>{phi_in, nullptr, 0.0}, phi_out, f, inv_h2, rscale, r, e_out, first_red,
                               h2l, inv2d, pblocks, maxbits);
        return;
    }
    int blocks = ceil_div(ncompact_active(dim, g), kBlock);
    if (blocks > 4096) blocks = 4096;
    if (upd)
        hipLaunchKernelGGL((k_dc_outer<2, TL, true>), dim3(blocks), dim3(kBlock), 0, st, g,
                           DcIn<TL, true>{phi_in, e_in, factor}, phi_out, f, inv_h2, rscale, r, e_out, first_red, h2l,
                           inv2d, maxbits);
    else
        hipLaunchKernelGGL((k_dc_outer<2, TL, false>), dim3(blocks), dim3(kBlock), 0, st, g,
                           DcIn<TL, false>{phi_in, nullptr, 0.0}, phi_out, f, inv_h2, rscale, r, e_out, first_red, h2l,
                           inv2d, maxbits);
}

// k_dc_scale over whole arrays, 8 consecutive elements per thread: with r32
// zero at every point that is not active (cleared with the level's other
// low-precision arrays; the residual pass writes active points only) the
// ghost points of r and e come out zero, as the point-wise form leaves them.
// Needs cs a multiple of 8 (3-D planes are padded to 128 elements).
template <typename TL>
__global__ void __launch_bounds__(kBlock) k_dc_scale_flat(long n8, size_t cs, const float* __restrict__ r32,
                                                          double rscale, TL* __restrict__ r, TL* __restrict__ e,
                                                          int first_red, float h2l, float inv2d)
{
    const long stride = (long)gridDim.x * kBlock;
    for (long t = xcd_block() * kBlock + threadIdx.x; t < n8; t += stride) {
        const size_t i = (size_t)t * 8;
        const int colour = i < cs ? 0 : 1;
        const float4 a = *(const float4*)(r32 + i);
        const float4 b = *(const float4*)(r32 + i + 4);
        const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        // the eight values of r (and e) go out in 16-byte stores
        union Out {
            TL v[8];
            uint4 w[sizeof(TL) / 2];
        } rl, el;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            rl.v[k] = (TL)(float)((double)v[k] * rscale);
            el.v[k] = (colour == 0 && first_red) ? (TL)((0.0f - h2l * (float)rl.v[k]) * inv2d) : (TL)0.0f;
        }
#pragma unroll
        for (int k = 0; k < (int)(sizeof(TL) / 2); k++) {
            ((uint4*)(r + i))[k] = rl.w[k];
            if (e) ((uint4*)(e + i))[k] = el.w[k];
        }
    }
}

template <typename TL>
void launch_dc_scale(int dim, hipStream_t st, SGrid g, const float* r32, double rscale, TL* r, TL* e_out,
                     int first_red)
{
    const float h2l = 1.0f, inv2d = (float)(1.0 / (2.0 * dim));
    if (dim == 3 && g.cs % 8 == 0) {
        const long n8 = (long)(2 * g.cs / 8);
        int blocks = ceil_div(n8, kBlock);
        if (blocks > 16384) blocks = 16384;
        hipLaunchKernelGGL((k_dc_scale_flat<TL>), dim3(blocks), dim3(kBlock), 0, st, n8, g.cs, r32, rscale, r, e_out,
                           first_red, h2l, inv2d);
        return;
    }
    int blocks = ceil_div(ncompact_active(dim, g), kBlock);
    if (blocks > 16384) blocks = 16384;
    if (dim == 3)
        hipLaunchKernelGGL((k_dc_scale<3, TL>), dim3(blocks), dim3(kBlock), 0, st, g, r32, rscale, r, e_out, first_red,
                           h2l, inv2d);
    else
        hipLaunchKernelGGL((k_dc_scale<2, TL>), dim3(blocks), dim3(kBlock), 0, st, g, r32, rscale, r, e_out, first_red,
                           h2l, inv2d);
}
template void launch_dc_scale<float>(int, hipStream_t, SGrid, const float*, double, float*, float*, int);
template void launch_dc_scale<__half>(int, hipStream_t, SGrid, const float*, double, __half*, __half*, int);

void launch_copy_ghosts(int dim, hipStream_t st, SGrid g, const double* src, double* dst)
{
    // the largest face
    const int m = g.nx > g.ny ? (g.nx > g.nz ? g.nx : g.nz) : (g.ny > g.nz ? g.ny : g.nz);
    int per = dim == 3 ? m * m : m;
    dim3 grid(ceil_div(per, kBlock), 2 * dim);
    if (dim == 3)
        hipLaunchKernelGGL((k_copy_ghosts<3>), grid, dim3(kBlock), 0, st, g, src, dst);
    else
        hipLaunchKernelGGL((k_copy_ghosts<2>), grid, dim3(kBlock), 0, st, g, src, dst);
}

void launch_copy_box(int dim, hipStream_t st, SGrid gs, const double* src, SGrid gd, double* dst, int lo,
                     const int* hi, int shift)
{
    const long wx = hi[0] - lo + 1, wy = hi[1] - lo + 1, wz = dim == 3 ? hi[2] - lo + 1 : 1;
    if (wx <= 0 || wy <= 0 || wz <= 0) return;
    dim3 grid(ceil_div(wx * wy * wz, kBlock));
    if (dim == 3)
        hipLaunchKernelGGL((k_copy_box<3>), grid, dim3(kBlock), 0, st, gs, src, gd, dst, lo, (int)wx, (int)wy, (int)wz,
                           shift);
    else
        hipLaunchKernelGGL((k_copy_box<2>), grid, dim3(kBlock), 0, st, gs, src, gd, dst, lo, (int)wx, (int)wy, 1,
                           shift);
}

template void launch_half_sweep<double>(int, hipStream_t, SGrid, double*, const double*, int, double, int, const Rule3&);
template void launch_full_sweep<double>(hipStream_t, SGrid, const double*, double*, const double*, double, double, int,
                                        int, unsigned long long*);
template void launch_half_sweep<float>(int, hipStream_t, SGrid, float*, const float*, int, double, int, const Rule3&);
template void launch_half_sweep<__half>(int, hipStream_t, SGrid, __half*, const __half*, int, double, int,
                                        const Rule3&);
template void launch_half_sweep_seeded<float>(hipStream_t, SGrid, float*, const float*, double, int);
template void launch_half_sweep_seeded<__half>(hipStream_t, SGrid, __half*, const __half*, double, int);
template void launch_resid_restrict<double, double>(int, hipStream_t, SGrid, const double*, const double*, double,
                                                    double, SGrid, double*, double*, int, const Rule3&, double);
template void launch_resid_restrict<float, float>(int, hipStream_t, SGrid, const float*, const float*, double, double,
                                                  SGrid, float*, float*, int, const Rule3&, double);
template void launch_resid_restrict<__half, float>(int, hipStream_t, SGrid, const __half*, const __half*, double,
                                                   double, SGrid, float*, float*, int, const Rule3&, double);
template void launch_prolong_add<double, double>(int, hipStream_t, SGrid, const double*, SGrid, double*, int,
                                                 const Rule3&);
template void launch_prolong_add<float, float>(int, hipStream_t, SGrid, const float*, SGrid, float*, int, const Rule3&);
template void launch_prolong_add<float, __half>(int, hipStream_t, SGrid, const float*, SGrid, __half*, int,
                                                const Rule3&);
template int launch_coarse_tail<float>(int, hipStream_t, int, const int (*)[3], const double*, const Rule3*, int, int,
                                       SGrid, const float*, float*);
template int launch_coarse_tail<double>(int, hipStream_t, int, const int (*)[3], const double*, const Rule3*, int,
                                        int, SGrid, const double*, double*);
template void launch_dc_outer<float>(int, hipStream_t, SGrid, const double*, const float*, double, double*,
                                     const double*, double, double, float*, float*, int, unsigned long long*);
template void launch_dc_outer<__half>(int, hipStream_t, SGrid, const double*, const __half*, double, double*,
                                      const double*, double, double, __half*, __half*, int, unsigned long long*);

}  // namespace np

// Kernels of the learned initial-guess network (gfx950).
//
// Network: conv3x3x3(2->16) -> ReLU -> conv3x3x3(16->16) -> ReLU ->
// conv3x3x3(16->1), zero padding, same-size output.  Activations are
// channel-last [batch][z][y][x][c]; the weights of a layer are bfloat16
// [27 taps][cout][cin] with taps ordered (dz, dy, dx), dx fastest, offsets
// -1..1; biases FP32.  Training keeps FP32 master weights (Adam) and runs the
// convolutions with the bfloat16 weights and FP32 activations and
// accumulation; inference of the 16->16 layer runs on the matrix cores
// (bfloat16 x bfloat16 -> FP32 MFMA).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>

#include "../../include/nested_poisson.h"
#include "np_internal.h"

namespace np {

namespace {

constexpr int kNB = 256;

__host__ __device__ inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even; NaN stays NaN
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename T>
__device__ __forceinline__ float ld(const T* p);
template <>
__device__ __forceinline__ float ld<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float ld<uint16_t>(const uint16_t* p) { return bf16_to_f32(*p); }

template <typename T>
__device__ __forceinline__ void st(T* p, float v);
template <>
__device__ __forceinline__ void st<float>(float* p, float v) { *p = v; }
template <>
__device__ __forceinline__ void st<uint16_t>(uint16_t* p, float v) { *p = f32_to_bf16(v); }

// ------------------------------------------------------------------ convolution, FP32 accumulate
// Thread per output voxel; the layer's weights are staged in LDS as FP32.
template <typename TI, typename TO>
__global__ void __launch_bounds__(kNB) k_conv_fwd(const TI* __restrict__ in, int cin, const uint16_t* __restrict__ w,
                                                 const float* __restrict__ bias, int cout, int relu, int B, int Z, int Y,
                                                 int X, TO* __restrict__ out)
{
    __shared__ float ws[27 * 16 * 16];
    const int nw = 27 * cout * cin;
    for (int i = threadIdx.x; i < nw; i += kNB) ws[i] = bf16_to_f32(w[i]);
    __syncthreads();
    const long nvox = (long)B * Z * Y * X;
    const long v = (long)blockIdx.x * kNB + threadIdx.x;
    if (v >= nvox) return;
    const int x = (int)(v % X);
    long r = v / X;
    const int y = (int)(r % Y);
    r /= Y;
    const int z = (int)(r % Z);
    const int b = (int)(r / Z);
    float acc[16];
    for (int o = 0; o < cout; o++) acc[o] = bias[o];
    int t = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++, t++) {
                const int zz = z + dz, yy = y + dy, xx = x + dx;
                if (zz < 0 || zz >= Z || yy < 0 || yy >= Y || xx < 0 || xx >= X) continue;
                const TI* src = in + ((((long)b * Z + zz) * Y + yy) * X + xx) * cin;
                const float* wt = ws + t * cout * cin;
                for (int i = 0; i < cin; i++) {
                    const float a = ld(src + i);
                    for (int o = 0; o < cout; o++) acc[o] = fmaf(wt[o * cin + i], a, acc[o]);
                }
            }
    TO* dst = out + v * cout;
    for (int o = 0; o < cout; o++) st(dst + o, relu ? fmaxf(acc[o], 0.0f) : acc[o]);
}

// The same convolution for the network's own channel counts, fixed at compile
// time: the accumulators stay in registers, the input channels of a tap come in
// with 8- to 16-byte loads and the outputs leave the same way.  Same
// arithmetic in the same order as k_conv_fwd.
template <int N, typename T>
__device__ __forceinline__ void ld_vec(const T* p, float (&a)[N])
{
    if constexpr (sizeof(T) == 2 && N % 8 == 0) {
#pragma unroll
        for (int q = 0; q < N / 8; q++) {
            const uint4 u = ((const uint4*)p)[q];
            const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int e = 0; e < 4; e++) {
                a[8 * q + 2 * e] = __uint_as_float(w4[e] << 16);
                a[8 * q + 2 * e + 1] = __uint_as_float(w4[e] & 0xffff0000u);
            }
        }
    } else if constexpr (sizeof(T) == 2 && N == 2) {
        const uint32_t u = *(const uint32_t*)p;
        a[0] = __uint_as_float(u << 16);
        a[1] = __uint_as_float(u & 0xffff0000u);
    } else if constexpr (sizeof(T) == 4 && N % 4 == 0) {
#pragma unroll
        for (int q = 0; q < N / 4; q++) {
            const float4 u = ((const float4*)p)[q];
            a[4 * q] = u.x;
            a[4 * q + 1] = u.y;
            a[4 * q + 2] = u.z;
            a[4 * q + 3] = u.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; i++) a[i] = ld(p + i);
    }
}

template <int N, typename T>
__device__ __forceinline__ void st_vec(T* p, const float (&a)[N])
{
    if constexpr (sizeof(T) == 2 && N % 8 == 0) {
#pragma unroll
        for (int q = 0; q < N / 8; q++) {
            uint32_t w4[4];
#pragma unroll
            for (int e = 0; e < 4; e++)
                w4[e] = (uint32_t)f32_to_bf16(a[8 * q + 2 * e]) | ((uint32_t)f32_to_bf16(a[8 * q + 2 * e + 1]) << 16);
            ((uint4*)p)[q] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
        }
    } else if constexpr (sizeof(T) == 4 && N % 4 == 0) {
#pragma unroll
        for (int q = 0; q < N / 4; q++) ((float4*)p)[q] = make_float4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < N; i++) st(p + i, a[i]);
    }
}

template <int CIN, int COUT, typename TI, typename TO>
__global__ void __launch_bounds__(kNB) k_conv_fwd_t(const TI* __restrict__ in, const uint16_t* __restrict__ w,
                                                   const float* __restrict__ bias, int relu, int B, int Z, int Y, int X,
                                                   TO* __restrict__ out)
{
    __shared__ float ws[27 * COUT * CIN];
    for (int i = threadIdx.x; i < 27 * COUT * CIN; i += kNB) ws[i] = bf16_to_f32(w[i]);
    __syncthreads();
    const long nvox = (long)B * Z * Y * X;
    const long v = (long)blockIdx.x * kNB + threadIdx.x;
    if (v >= nvox) return;
    const int x = (int)(v % X);
    long r = v / X;
    const int y = (int)(r % Y);
    r /= Y;
    const int z = (int)(r % Z);
    const int b = (int)(r / Z);
    float acc[COUT];
#pragma unroll
    for (int o = 0; o < COUT; o++) acc[o] = bias[o];
    int t = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++, t++) {
                const int zz = z + dz, yy = y + dy, xx = x + dx;
                if (zz < 0 || zz >= Z || yy < 0 || yy >= Y || xx < 0 || xx >= X) continue;
                float a[CIN];
                ld_vec<CIN>(in + ((((long)b * Z + zz) * Y + yy) * X + xx) * CIN, a);
                const float* wt = ws + t * COUT * CIN;
#pragma unroll
                for (int i = 0; i < CIN; i++)
#pragma unroll
                    for (int o = 0; o < COUT; o++) acc[o] = fmaf(wt[o * CIN + i], a[i], acc[o]);
            }
    if (relu) {
#pragma unroll
        for (int o = 0; o < COUT; o++) acc[o] = fmaxf(acc[o], 0.0f);
    }
    st_vec<COUT>(out + v * COUT, acc);
}

// Data gradient: gin[v][i] = sum_taps sum_o w[t][o][i] * gout[v - tap][o].
__global__ void __launch_bounds__(kNB) k_conv_bwd_data(const float* __restrict__ gout, int cout,
                                                      const uint16_t* __restrict__ w, int cin, int B, int Z, int Y, int X,
                                                      float* __restrict__ gin)
{
    __shared__ float ws[27 * 16 * 16];
    const int nw = 27 * cout * cin;
    for (int i = threadIdx.x; i < nw; i += kNB) ws[i] = bf16_to_f32(w[i]);
    __syncthreads();
    const long nvox = (long)B * Z * Y * X;
    const long v = (long)blockIdx.x * kNB + threadIdx.x;
    if (v >= nvox) return;
    const int x = (int)(v % X);
    long r = v / X;
    const int y = (int)(r % Y);
    r /= Y;
    const int z = (int)(r % Z);
    const int b = (int)(r / Z);
    float acc[16];
    for (int i = 0; i < cin; i++) acc[i] = 0.0f;
    int t = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++, t++) {
                const int zz = z - dz, yy = y - dy, xx = x - dx;
                if (zz < 0 || zz >= Z || yy < 0 || yy >= Y || xx < 0 || xx >= X) continue;
                const float* g = gout + ((((long)b * Z + zz) * Y + yy) * X + xx) * cout;
                const float* wt = ws + t * cout * cin;
                for (int o = 0; o < cout; o++) {
                    const float go = g[o];
                    for (int i = 0; i < cin; i++) acc[i] = fmaf(wt[o * cin + i], go, acc[i]);
                }
            }
    float* dst = gin + v * cin;
    for (int i = 0; i < cin; i++) dst[i] = acc[i];
}

// Weight and bias gradients, first stage: block `blk` sums over the voxel rows
// blk, blk + gridDim.x, ... and writes its partial (27*cout*cin weights, then
// cout biases) to part[blk].  Each thread owns weight entries
// e = threadIdx.x, threadIdx.x + 256, ...; the row's inputs (3x3 neighbour
// rows with a one-voxel halo) and output gradients are staged in LDS.
constexpr int kRowMax = 64;  // longest row segment staged at once (longer rows are split)

__global__ void __launch_bounds__(kNB) k_conv_bwd_weight_part(const float* __restrict__ in, int cin,
                                                             const float* __restrict__ gout, int cout, int B, int Z,
                                                             int Y, int X, float* __restrict__ part)
{
    __shared__ float sin[9][kRowMax + 2][16];
    __shared__ float sg[kRowMax][16];
    const int nw = 27 * cout * cin;
    const int ne = nw + cout;
    float acc[28];  // ceil((27*16*16 + 16) / 256) = 28 entries per thread at most
    for (int q = 0; q < 28; q++) acc[q] = 0.0f;
    const int nseg = (X + kRowMax - 1) / kRowMax;
    const long nrows = (long)B * Z * Y * nseg;
    for (long row = blockIdx.x; row < nrows; row += gridDim.x) {
        const int seg = (int)(row % nseg);
        long rr = row / nseg;
        const int y = (int)(rr % Y);
        rr /= Y;
        const int z = (int)(rr % Z);
        const int b = (int)(rr / Z);
        const int x0 = seg * kRowMax;
        const int len = min(kRowMax, X - x0);
        __syncthreads();
        // stage 9 neighbour rows (dz, dy) with x in [x0-1, x0+len] and the output gradients
        for (int idx = threadIdx.x; idx < 9 * (len + 2) * cin; idx += kNB) {
            const int i = idx % cin;
            const int xs = (idx / cin) % (len + 2);
            const int nr = idx / (cin * (len + 2));
            const int zz = z + nr / 3 - 1, yy = y + nr % 3 - 1, xx = x0 + xs - 1;
            float vv = 0.0f;
            if (zz >= 0 && zz < Z && yy >= 0 && yy < Y && xx >= 0 && xx < X)
                vv = in[((((long)b * Z + zz) * Y + yy) * X + xx) * cin + i];
            sin[nr][xs][i] = vv;
        }
        for (int idx = threadIdx.x; idx < len * cout; idx += kNB) {
            const int o = idx % cout, xs = idx / cout;
            sg[xs][o] = gout[((((long)b * Z + z) * Y + y) * X + x0 + xs) * cout + o];
        }
        __syncthreads();
        int q = 0;
        for (int e = threadIdx.x; e < ne; e += kNB, q++) {
            float s = 0.0f;
            if (e < nw) {
                const int i = e % cin;
                const int o = (e / cin) % cout;
                const int t = e / (cin * cout);
                const int nr = t / 3, dx = t % 3;  // (dz, dy) row index and x offset + 1
                for (int xs = 0; xs < len; xs++) s = fmaf(sg[xs][o], sin[nr][xs + dx][i], s);
            } else {
                const int o = e - nw;
                for (int xs = 0; xs < len; xs++) s += sg[xs][o];
            }
            acc[q] += s;
        }
    }
    int q = 0;
    for (int e = threadIdx.x; e < ne; e += kNB, q++) part[(long)blockIdx.x * ne + e] = acc[q];
}

// Second stage: gw/gb = sum over the partials, in a fixed order.
__global__ void k_sum_parts(const float* __restrict__ part, int nparts, int ne, int nw, float* __restrict__ gw,
                            float* __restrict__ gb)
{
    const int e = blockIdx.x * kNB + threadIdx.x;
    if (e >= ne) return;
    float s = 0.0f;
    for (int p = 0; p < nparts; p++) s += part[(long)p * ne + e];
    if (e < nw) gw[e] = s;
    else gb[e - nw] = s;
}

__global__ void k_relu_bwd(const float* __restrict__ act, float* __restrict__ g, long n)
{
    const long i = (long)blockIdx.x * kNB + threadIdx.x;
    if (i < n && !(act[i] > 0.0f)) g[i] = 0.0f;
}

// Masked mean squared error: grad = 2 mask (pred - target) / sum(mask), and
// per-block partial sums of mask (pred - target)^2 and of mask.
__global__ void k_mse(const float* __restrict__ pred, const float* __restrict__ target, const float* __restrict__ mask,
                      long n, float inv_count, float* __restrict__ grad, float* __restrict__ part)
{
    __shared__ float red[kNB];
    const long i = (long)blockIdx.x * kNB + threadIdx.x;
    float d = 0.0f;
    if (i < n) {
        const float m = mask ? mask[i] : 1.0f;
        const float diff = (pred[i] - target[i]) * m;
        grad[i] = 2.0f * diff * inv_count;
        d = diff * diff;
    }
    red[threadIdx.x] = d;
    __syncthreads();
    for (int s = kNB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum(const float* __restrict__ part, int n, float scale, float* __restrict__ out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float s = 0.0f;
        for (int i = 0; i < n; i++) s += part[i];
        out[0] = s * scale;
    }
}

// Adam (Kingma & Ba) with bias correction on FP32 master weights; the
// bfloat16 copy used by the convolutions is refreshed.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long n, float lr, float b1, float b2, float eps, float c1, float c2, uint16_t* __restrict__ wb)
{
    const long i = (long)blockIdx.x * kNB + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f32_to_bf16(wi);
}

__global__ void k_to_bf16(const float* __restrict__ a, uint16_t* __restrict__ b, long n)
{
    const long i = (long)blockIdx.x * kNB + threadIdx.x;
    if (i < n) b[i] = f32_to_bf16(a[i]);
}

// a = bfloat16(a), kept in FP32 storage: the training forward pass rounds its
// inputs and hidden activations as the bfloat16 inference path stores them
__global__ void k_round_bf16(float* __restrict__ a, long n)
{
    const long i = (long)blockIdx.x * kNB + threadIdx.x;
    if (i < n) a[i] = bf16_to_f32(f32_to_bf16(a[i]));
}

// out = h^2 lap(in) with the 7-point stencil of eqn:Laplacian3D (the sum of
// the six face neighbours minus six times the centre), zero outside the box;
// one channel, [batch][z][y][x].  The stencil is symmetric, so the same kernel
// applies its transpose in the backward pass of the residual objective.
__global__ void k_lap7(const float* __restrict__ in, int B, int Z, int Y, int X, float* __restrict__ out)
{
    const long v = (long)blockIdx.x * kNB + threadIdx.x;
    const long nv = (long)B * Z * Y * X;
    if (v >= nv) return;
    const int x = (int)(v % X);
    long r = v / X;
    const int y = (int)(r % Y);
    r /= Y;
    const int z = (int)(r % Z);
    float s = x > 0 ? in[v - 1] : 0.0f;
    s += x + 1 < X ? in[v + 1] : 0.0f;
    s += y > 0 ? in[v - X] : 0.0f;
    s += y + 1 < Y ? in[v + X] : 0.0f;
    s += z > 0 ? in[v - (long)X * Y] : 0.0f;
    s += z + 1 < Z ? in[v + (long)X * Y] : 0.0f;
    out[v] = s - 6.0f * in[v];
}

// ------------------------------------------------------------------ inference on the matrix cores
// Operand layout of v_mfma_f32_16x16x16 bf16: lane l supplies A[row l%16][k
// 4(l/16)..+3] and B[k 4(l/16)..+3][col l%16], and receives D[rows
// 4(l/16)..+3][col l%16].  Rows are 16 consecutive voxels along x, columns the
// output channels.
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Matrix-core convolution with the input block staged in LDS (the inference
// path of all three layers).  A workgroup loads its weights once and then runs
// a contiguous range of 16 (x) x 4 (y) x 4 (z) blocks of output voxels: for
// each it copies the 18 x 6 x 6 input voxels around the block (zero outside the
// volume) into LDS, and each of its 4 wavefronts produces 4 rows of 16 voxels,
// taking the A operand of every tap from LDS, so that an input voxel is read
// from memory about 2.5 times instead of 27.  The
// K dimension of the products: CIN = 16, one tap's 16 channels per MFMA (27
// products, in tap order); CIN = 2, (tap, channel) pairs,
// 16 per MFMA (4 products, taps past 27 zero).  COUT = 1 pads the weight
// columns with zeros and writes FP32; COUT = 16 writes bfloat16.
constexpr int kCTx = 16, kCTy = 4, kCTz = 4;
constexpr long kConvWorkgroups = 2048;

template <int CIN, int COUT, typename TO>
__global__ void __launch_bounds__(256) k_conv_mfma_lds(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias, int relu, int B, int Z, int Y,
                                                      int X, TO* __restrict__ out, long per_block)
{
    constexpr int SX = kCTx + 2, SY = kCTy + 2, SZ = kCTz + 2, NV = SX * SY * SZ;
    constexpr int NMF = CIN == 16 ? 27 : 4;
    // LDS stride per voxel in bfloat16 elements: 16 channels padded to 24 so that
    // the 16 voxels of an A-operand read fall into different banks
    constexpr int VS = CIN == 16 ? 24 : 2;
    __shared__ __align__(16) uint16_t tile[NV * VS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int ntx = (X + kCTx - 1) / kCTx, nty = (Y + kCTy - 1) / kCTy, ntz = (Z + kCTz - 1) / kCTz;
    const long ntiles = (long)B * ntz * nty * ntx;
    // weights of the lane's B operand for every product (once per workgroup,
    // which then runs a contiguous range of output blocks)
    v4s bw[NMF];
#pragma unroll
    for (int sI = 0; sI < NMF; sI++) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            int t, c;
            if (CIN == 16) {
                t = sI;
                c = 4 * kq + e;
            } else {
                t = 8 * sI + 2 * kq + (e >> 1);
                c = e & 1;
            }
            bw[sI][e] = (row < COUT && t < 27) ? (short)w[(t * COUT + row) * CIN + c] : (short)0;
        }
    }
    const float bo = row < COUT ? bias[row] : 0.0f;
    const long first = (long)blockIdx.x * per_block;
    const long last = first + per_block < ntiles ? first + per_block : ntiles;
    for (long bid = first; bid < last; bid++) {
        long rem = bid;
        const int bx = (int)(rem % ntx);
        rem /= ntx;
        const int by = (int)(rem % nty);
        rem /= nty;
        const int bz = (int)(rem % ntz);
        const int b = (int)(rem / ntz);
        const int x0 = bx * kCTx, y0 = by * kCTy, z0 = bz * kCTz;
        __syncthreads();  // the previous block's operands have been read
        // stage the input block
        for (int v = threadIdx.x; v < NV; v += 256) {
            const int lx = v % SX, ly = (v / SX) % SY, lz = v / (SX * SY);
            const int gx = x0 - 1 + lx, gy = y0 - 1 + ly, gz = z0 - 1 + lz;
            const bool inside = gx >= 0 && gx < X && gy >= 0 && gy < Y && gz >= 0 && gz < Z;
            const uint16_t* src = in + ((((long)b * Z + gz) * Y + gy) * X + gx) * CIN;
            if (CIN == 16) {
                uint4 q0 = make_uint4(0, 0, 0, 0), q1 = q0;
                if (inside) {
                    q0 = ((const uint4*)src)[0];
                    q1 = ((const uint4*)src)[1];
                }
                ((uint4*)(tile + v * VS))[0] = q0;
                ((uint4*)(tile + v * VS))[1] = q1;
            } else {
                ((uint32_t*)tile)[v] = inside ? *(const uint32_t*)src : 0u;
            }
        }
        __syncthreads();
        // A operand of product sI for the wave's output row it (rows of 16 voxels
        // at (y0 + ly, z0 + lz)); rows outside the volume read zeros and are not stored
        auto afrag = [&](int it, int sI) -> v4s {
            const int rid = wave * 4 + it;
            const int ly = rid % kCTy, lz = rid / kCTy;
            if (CIN == 16) {
                const int dz = sI / 9, dy = (sI / 3) % 3, dx = sI % 3;
                const int lv = ((lz + dz) * SY + (ly + dy)) * SX + (row + dx);
                return *(const v4s*)(tile + lv * VS + 4 * kq);
            }
            short e4[4] = {0, 0, 0, 0};
    #pragma unroll
            for (int h = 0; h < 2; h++) {
                const int t = 8 * sI + 2 * kq + h;
                if (t < 27) {
                    const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
                    const int lv = ((lz + dz) * SY + (ly + dy)) * SX + (row + dx);
                    const uint32_t pr = ((const uint32_t*)tile)[lv];
                    e4[2 * h] = (short)(pr & 0xffffu);
                    e4[2 * h + 1] = (short)(pr >> 16);
                }
            }
            return v4s{e4[0], e4[1], e4[2], e4[3]};
        };
        auto store = [&](int it, const v4f& acc) {
            const int rid = wave * 4 + it;
            const int y = y0 + rid % kCTy, z = z0 + rid / kCTy;
            if (y >= Y || z >= Z) return;
            // lane holds D[voxels 4 kq .. 4 kq + 3][channel row]
            const long base = (((long)b * Z + z) * Y + y) * X;
            for (int q = 0; q < 4; q++) {
                const int x = x0 + 4 * kq + q;
                if (x >= X || row >= COUT) continue;
                float v = acc[q] + bo;
                if (relu) v = fmaxf(v, 0.0f);
                st(out + (base + x) * COUT + row, v);
            }
        };
        // two rows at a time on two independent accumulation chains; the A
        // operands of a plane of taps (9 products) are read before its products
        for (int p = 0; p < 4; p += 2) {
            v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
            constexpr int G = CIN == 16 ? 9 : NMF;
    #pragma unroll
            for (int g0 = 0; g0 < NMF; g0 += G) {
                v4s a0[G], a1[G];
    #pragma unroll
                for (int q = 0; q < G; q++) {
                    a0[q] = afrag(p, g0 + q);
                    a1[q] = afrag(p + 1, g0 + q);
                }
    #pragma unroll
                for (int q = 0; q < G; q++) {
                    acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0[q], bw[g0 + q], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[q], bw[g0 + q], acc1, 0, 0, 0);
                }
            }
            store(p, acc0);
            store(p + 1, acc1);
        }
    }
}

// ------------------------------------------------------------------ solver glue
// Features of a nested level's Gamma ((n+2)^3 points, channel-last, 2 channels):
// f / ||f|| and r0 / ||f|| with r0 = f - lap(phi) of the interpolated guess.
template <typename TA>
__global__ void __launch_bounds__(kNB) k_net_features(SGrid g, const double* __restrict__ phi,
                                                     const double* __restrict__ f, double inv_fnorm, double inv_h2,
                                                     TA* __restrict__ x)
{
    const int mx = g.nx - 2, my = g.ny - 2, mz = g.nz - 2;
    const long nv = (long)mx * my * mz;
    const long v = (long)blockIdx.x * kNB + threadIdx.x;
    if (v >= nv) return;
    const int i = (int)(v % mx) + 1;
    const int j = (int)((v / mx) % my) + 1;
    const int k = (int)(v / ((long)mx * my)) + 1;
    auto at = [&](const double* a, int pi, int pj, int pk) {
        return a[(size_t)((pi + pj + pk + 3) & 1) * g.cs + ((size_t)pk * g.ps + (size_t)pj * g.hx) + (pi >> 1)];
    };
    const double lap = (at(phi, i - 1, j, k) + at(phi, i + 1, j, k) + at(phi, i, j - 1, k) + at(phi, i, j + 1, k) +
                        at(phi, i, j, k - 1) + at(phi, i, j, k + 1) - 6.0 * at(phi, i, j, k)) * inv_h2;
    const double fv = at(f, i, j, k);
    st(x + 2 * v, (float)(fv * inv_fnorm));
    st(x + 2 * v + 1, (float)((fv - lap) * inv_fnorm));
}

// phi += s * out on Gamma (out: (n+2)^3 FP32)
__global__ void __launch_bounds__(kNB) k_net_apply(SGrid g, double* __restrict__ phi, const float* __restrict__ out,
                                                  double s)
{
    const int mx = g.nx - 2, my = g.ny - 2, mz = g.nz - 2;
    const long nv = (long)mx * my * mz;
    const long v = (long)blockIdx.x * kNB + threadIdx.x;
    if (v >= nv) return;
    const int i = (int)(v % mx) + 1;
    const int j = (int)((v / mx) % my) + 1;
    const int k = (int)(v / ((long)mx * my)) + 1;
    phi[(size_t)((i + j + k + 3) & 1) * g.cs + ((size_t)k * g.ps + (size_t)j * g.hx) + (i >> 1)] += s * (double)out[v];
}

// target = (phi_a - phi_b) * inv_s on Gamma
__global__ void __launch_bounds__(kNB) k_net_target(SGrid g, const double* __restrict__ pa,
                                                   const double* __restrict__ pb, double inv_s, float* __restrict__ t)
{
    const int mx = g.nx - 2, my = g.ny - 2, mz = g.nz - 2;
    const long nv = (long)mx * my * mz;
    const long v = (long)blockIdx.x * kNB + threadIdx.x;
    if (v >= nv) return;
    const int i = (int)(v % mx) + 1;
    const int j = (int)((v / mx) % my) + 1;
    const int k = (int)(v / ((long)mx * my)) + 1;
    const size_t p = (size_t)((i + j + k + 3) & 1) * g.cs + ((size_t)k * g.ps + (size_t)j * g.hx) + (i >> 1);
    t[v] = (float)((pa[p] - pb[p]) * inv_s);
}

}  // namespace

// ------------------------------------------------------------------ launchers
constexpr int kNetParts = 2048;  // blocks (partial sums) of the weight-gradient reduction

// The network's layer shapes (2 -> 16, 16 -> 16, 16 -> 1) run on the
// compile-time kernel; returns false for other shapes.
template <typename TI, typename TO>
static bool conv_fwd_fixed(hipStream_t st, const TI* in, int cin, const uint16_t* w, const float* bias, int cout, int relu,
                    int B, int Z, int Y, int X, TO* out)
{
    const dim3 grid(cdiv((long)B * Z * Y * X, kNB));
    if (cin == 2 && cout == 16)
        hipLaunchKernelGGL((k_conv_fwd_t<2, 16, TI, TO>), grid, dim3(kNB), 0, st, in, w, bias, relu, B, Z, Y, X, out);
    else if (cin == 16 && cout == 16)
        hipLaunchKernelGGL((k_conv_fwd_t<16, 16, TI, TO>), grid, dim3(kNB), 0, st, in, w, bias, relu, B, Z, Y, X, out);
    else if (cin == 16 && cout == 1)
        hipLaunchKernelGGL((k_conv_fwd_t<16, 1, TI, TO>), grid, dim3(kNB), 0, st, in, w, bias, relu, B, Z, Y, X, out);
    else
        return false;
    return true;
}

void net_conv_fwd_f32(hipStream_t st, const float* in, int cin, const uint16_t* w, const float* bias, int cout, int relu,
                      int B, int Z, int Y, int X, float* out)
{
    long nv = (long)B * Z * Y * X;
    if (conv_fwd_fixed(st, in, cin, w, bias, cout, relu, B, Z, Y, X, out)) return;
    hipLaunchKernelGGL((k_conv_fwd<float, float>), dim3(cdiv(nv, kNB)), dim3(kNB), 0, st, in, cin, w, bias, cout, relu, B,
                       Z, Y, X, out);
}

void net_conv_fwd_bf16(hipStream_t st, const uint16_t* in, int cin, const uint16_t* w, const float* bias, int cout,
                       int relu, int B, int Z, int Y, int X, uint16_t* out)
{
    long nv = (long)B * Z * Y * X;
    if (conv_fwd_fixed(st, in, cin, w, bias, cout, relu, B, Z, Y, X, out)) return;
    hipLaunchKernelGGL((k_conv_fwd<uint16_t, uint16_t>), dim3(cdiv(nv, kNB)), dim3(kNB), 0, st, in, cin, w, bias, cout,
                       relu, B, Z, Y, X, out);
}

void net_conv_fwd_bf16_to_f32(hipStream_t st, const uint16_t* in, int cin, const uint16_t* w, const float* bias,
                              int cout, int relu, int B, int Z, int Y, int X, float* out)
{
    long nv = (long)B * Z * Y * X;
    if (conv_fwd_fixed(st, in, cin, w, bias, cout, relu, B, Z, Y, X, out)) return;
    hipLaunchKernelGGL((k_conv_fwd<uint16_t, float>), dim3(cdiv(nv, kNB)), dim3(kNB), 0, st, in, cin, w, bias, cout,
                       relu, B, Z, Y, X, out);
}

void net_conv_mfma(hipStream_t st, const uint16_t* in, int cin, const uint16_t* w, const float* bias, int cout, int relu,
                   int B, int Z, int Y, int X, void* out)
{
    const long tiles = (long)B * ((Z + kCTz - 1) / kCTz) * ((Y + kCTy - 1) / kCTy) * ((X + kCTx - 1) / kCTx);
    // persistent workgroups, each over a contiguous range of output blocks
    const long per = (tiles + kConvWorkgroups - 1) / kConvWorkgroups;
    const dim3 grid((unsigned)((tiles + per - 1) / per));
    if (cin == 16 && cout == 16)
        hipLaunchKernelGGL((k_conv_mfma_lds<16, 16, uint16_t>), grid, dim3(256), 0, st, in, w, bias, relu, B, Z, Y, X,
                           (uint16_t*)out, per);
    else if (cin == 2 && cout == 16)
        hipLaunchKernelGGL((k_conv_mfma_lds<2, 16, uint16_t>), grid, dim3(256), 0, st, in, w, bias, relu, B, Z, Y, X,
                           (uint16_t*)out, per);
    else if (cin == 16 && cout == 1)
        hipLaunchKernelGGL((k_conv_mfma_lds<16, 1, float>), grid, dim3(256), 0, st, in, w, bias, relu, B, Z, Y, X,
                           (float*)out, per);
}

void net_conv_bwd_data(hipStream_t st, const float* gout, int cout, const uint16_t* w, int cin, int B, int Z, int Y,
                       int X, float* gin)
{
    long nv = (long)B * Z * Y * X;
    hipLaunchKernelGGL(k_conv_bwd_data, dim3(cdiv(nv, kNB)), dim3(kNB), 0, st, gout, cout, w, cin, B, Z, Y, X, gin);
}

size_t net_bwd_weight_workspace(int cin, int cout) { return (size_t)kNetParts * (27 * cin * cout + cout) * sizeof(float); }

void net_conv_bwd_weight(hipStream_t st, const float* in, int cin, const float* gout, int cout, int B, int Z, int Y,
                         int X, float* gw, float* gb, float* part)
{
    int ne = 27 * cin * cout + cout;
    hipLaunchKernelGGL(k_conv_bwd_weight_part, dim3(kNetParts), dim3(kNB), 0, st, in, cin, gout, cout, B, Z, Y, X, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(cdiv(ne, kNB)), dim3(kNB), 0, st, part, kNetParts, ne, 27 * cin * cout, gw, gb);
}

void net_relu_bwd(hipStream_t st, const float* act, float* g, long n)
{
    hipLaunchKernelGGL(k_relu_bwd, dim3(cdiv(n, kNB)), dim3(kNB), 0, st, act, g, n);
}

size_t net_mse_workspace(long n) { return (size_t)cdiv(n, kNB) * sizeof(float); }

void net_mse(hipStream_t st, const float* pred, const float* target, const float* mask, long n, float count,
             float* grad, float* part, float* loss)
{
    int nb = cdiv(n, kNB);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kNB), 0, st, pred, target, mask, n, 1.0f / count, grad, part);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1), 0, st, part, nb, 1.0f / count, loss);
}

void net_adam(hipStream_t st, float* w, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
              float eps, int step, uint16_t* wb)
{
    float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(cdiv(n, kNB)), dim3(kNB), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2, wb);
}

void net_to_bf16(hipStream_t st, const float* a, uint16_t* b, long n)
{
    hipLaunchKernelGGL(k_to_bf16, dim3(cdiv(n, kNB)), dim3(kNB), 0, st, a, b, n);
}

void net_features_bf16(hipStream_t st, SGrid g, const double* phi, const double* f, double inv_fnorm, double inv_h2,
                       uint16_t* x)
{
    const long nvox = (long)(g.nx - 2) * (g.ny - 2) * (g.nz - 2);
    hipLaunchKernelGGL((k_net_features<uint16_t>), dim3(cdiv(nvox, kNB)), dim3(kNB), 0, st, g, phi, f, inv_fnorm,
                       inv_h2, x);
}

void net_features_f32(hipStream_t st, SGrid g, const double* phi, const double* f, double inv_fnorm, double inv_h2,
                      float* x)
{
    const long nvox = (long)(g.nx - 2) * (g.ny - 2) * (g.nz - 2);
    hipLaunchKernelGGL((k_net_features<float>), dim3(cdiv(nvox, kNB)), dim3(kNB), 0, st, g, phi, f, inv_fnorm,
                       inv_h2, x);
}

void net_apply(hipStream_t st, SGrid g, double* phi, const float* out, double s)
{
    const long nvox = (long)(g.nx - 2) * (g.ny - 2) * (g.nz - 2);
    hipLaunchKernelGGL(k_net_apply, dim3(cdiv(nvox, kNB)), dim3(kNB), 0, st, g, phi, out, s);
}

void net_target(hipStream_t st, SGrid g, const double* pa, const double* pb, double inv_s, float* t)
{
    const long nvox = (long)(g.nx - 2) * (g.ny - 2) * (g.nz - 2);
    hipLaunchKernelGGL(k_net_target, dim3(cdiv(nvox, kNB)), dim3(kNB), 0, st, g, pa, pb, inv_s, t);
}

}  // namespace np

// ------------------------------------------------------------------ C ABI (include/nested_poisson.h)
using namespace np;

static bool net_ok(int cin, int cout) { return cin >= 1 && cin <= 16 && cout >= 1 && cout <= 16; }
static bool dims_ok(int b, int z, int y, int x) { return b >= 1 && z >= 1 && y >= 1 && x >= 1; }

extern "C" {

size_t np_net_workspace_bytes(int cin, int cout, long nvox)
{
    size_t a = net_ok(cin, cout) ? net_bwd_weight_workspace(cin, cout) : 0;
    size_t b = nvox > 0 ? net_mse_workspace(nvox) : 0;
    return a > b ? a : b;
}

int np_net_conv3d_fwd(const float* in, int cin, const unsigned short* w, const float* bias, int cout, int relu,
                      int batch, int nz, int ny, int nx, float* out, void* stream)
{
    if (!in || !w || !bias || !out || !net_ok(cin, cout) || !dims_ok(batch, nz, ny, nx)) return NP_EINVAL;
    net_conv_fwd_f32((hipStream_t)stream, in, cin, w, bias, cout, relu, batch, nz, ny, nx, out);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

int np_net_conv3d_fwd_mfma(const unsigned short* in, int cin, const unsigned short* w, const float* bias, int cout,
                           int relu, int batch, int nz, int ny, int nx, void* out, void* stream)
{
    if (!in || !w || !bias || !out || !dims_ok(batch, nz, ny, nx)) return NP_EINVAL;
    if (!((cin == 2 && cout == 16) || (cin == 16 && cout == 16) || (cin == 16 && cout == 1))) return NP_EINVAL;
    if ((uintptr_t)in & (uintptr_t)(4 * cin - 1)) return NP_EINVAL;
    net_conv_mfma((hipStream_t)stream, in, cin, w, bias, cout, relu, batch, nz, ny, nx, out);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

int np_net_conv3d_bwd_data(const float* gout, int cout, const unsigned short* w, int cin, int batch, int nz, int ny,
                           int nx, float* gin, void* stream)
{
    if (!gout || !w || !gin || !net_ok(cin, cout) || !dims_ok(batch, nz, ny, nx)) return NP_EINVAL;
    net_conv_bwd_data((hipStream_t)stream, gout, cout, w, cin, batch, nz, ny, nx, gin);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

int np_net_conv3d_bwd_weight(const float* in, int cin, const float* gout, int cout, int batch, int nz, int ny, int nx,
                             float* gw, float* gb, float* workspace, size_t workspace_bytes, void* stream)
{
    if (!in || !gout || !gw || !gb || !workspace || !net_ok(cin, cout) || !dims_ok(batch, nz, ny, nx)) return NP_EINVAL;
    if (workspace_bytes < net_bwd_weight_workspace(cin, cout)) return NP_EINVAL;
    net_conv_bwd_weight((hipStream_t)stream, in, cin, gout, cout, batch, nz, ny, nx, gw, gb, workspace);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

int np_net_relu_bwd(const float* act, float* grad, long n, void* stream)
{
    if (!act || !grad || n < 0) return NP_EINVAL;
    if (n) net_relu_bwd((hipStream_t)stream, act, grad, n);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

int np_net_mse(const float* pred, const float* target, const float* mask, long n, float count, float* grad,
               float* loss, float* workspace, size_t workspace_bytes, void* stream)
{
    if (!pred || !target || !grad || !loss || !workspace || n < 1 || !(count > 0)) return NP_EINVAL;
    if (workspace_bytes < net_mse_workspace(n)) return NP_EINVAL;
    net_mse((hipStream_t)stream, pred, target, mask, n, count, grad, workspace, loss);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

// Partial sums of np_net_mse_noalloc: one file-scope device array, never
// allocated at run time.  Each device holds its own copy at its own address,
// looked up once per device (hipGetSymbolAddress) and kept in mse_scratch_dev;
// host code uses only those addresses, never the array's name.
static __device__ __align__(256) float scratch[NP_NET_MSE_NOALLOC_MAX / 256];
static float* mse_scratch_dev[64];
static std::mutex mse_scratch_mu;

static int mse_scratch(float** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        set_last_error("np_net_mse_noalloc: no current HIP device (or device index >= 64)");
        return NP_ENODEV;
    }
    std::lock_guard<std::mutex> lock(mse_scratch_mu);
    if (!mse_scratch_dev[dev]) {
        float* p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            char msg[160];
            snprintf(msg, sizeof msg, "np_net_mse_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            set_last_error(msg);
            return NP_EHIP;
        }
        mse_scratch_dev[dev] = p;
    }
    *out = mse_scratch_dev[dev];
    return NP_OK;
}

int np_net_mse_noalloc(const float* pred, const float* target, const float* mask, long n, float count, float* grad,
                       float* loss, void* stream)
{
    if (!pred || !target || !grad || !loss || n < 1 || !(count > 0)) return NP_EINVAL;
    if (n > NP_NET_MSE_NOALLOC_MAX) {
        char msg[160];
        snprintf(msg, sizeof msg, "np_net_mse_noalloc: n = %ld exceeds the maximum %ld", n,
                 (long)NP_NET_MSE_NOALLOC_MAX);
        set_last_error(msg);
        return NP_EINVAL;
    }
    float* part = nullptr;
    const int rc = mse_scratch(&part);
    if (rc) return rc;
    // every partial k_sum reads (blocks 0 .. ceil(n/256) - 1) is written by k_mse
    // first, so nothing needs clearing between calls
    net_mse((hipStream_t)stream, pred, target, mask, n, count, grad, part, loss);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

int np_net_adam(float* w, const float* g, float* m, float* v, long n, float lr, float beta1, float beta2, float eps,
                int step, unsigned short* w_bf16, void* stream)
{
    if (!w || !g || !m || !v || n < 0 || step < 1) return NP_EINVAL;
    if (n) net_adam((hipStream_t)stream, w, g, m, v, n, lr, beta1, beta2, eps, step, w_bf16);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

int np_net_round_bf16(float* a, long n, void* stream)
{
    if (!a || n < 0) return NP_EINVAL;
    if (n) hipLaunchKernelGGL(k_round_bf16, dim3(cdiv(n, kNB)), dim3(kNB), 0, (hipStream_t)stream, a, n);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

int np_net_lap7(const float* in, int batch, int nz, int ny, int nx, float* out, void* stream)
{
    if (!in || !out || in == out || !dims_ok(batch, nz, ny, nx)) return NP_EINVAL;
    const long nv = (long)batch * nz * ny * nx;
    hipLaunchKernelGGL(k_lap7, dim3(cdiv(nv, kNB)), dim3(kNB), 0, (hipStream_t)stream, in, batch, nz, ny, nx, out);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

int np_net_to_bf16(const float* a, unsigned short* b, long n, void* stream)
{
    if (!a || !b || n < 0) return NP_EINVAL;
    if (n) net_to_bf16((hipStream_t)stream, a, b, n);
    return hipGetLastError() == hipSuccess ? NP_OK : NP_EHIP;
}

}  // extern "C"

// cnn_kernels.hip -- learned GS seed: a 5-layer 3x3 convolutional network
// (1 -> 32 -> 32 -> 32 -> 32 -> 2 channels, circular padding, ReLU on layers
// 1..4) mapping a target amplitude to a replay-plane unit phasor that replaces
// the LUT phasor in R_0 of Gerchberg-Saxton.  Not part of the paper's method:
// it is the learned extension of its LUT seed, trained on the project's own
// GS output; the LUT seed remains the fallback.
//
// Arithmetic: BF16 weights and activations, FP32 accumulation.  The 32->32
// layers (forward and backward-data) are implicit GEMMs on gfx950 MFMA
// (v_mfma_f32_32x32x16_bf16: 32 pixels x 32 channels per wave, K = 9 taps x 32
// input channels); the 1->32 and 32->2 layers, the weight gradients, the loss
// and Adam run on the vector ALUs.  FP64 only for the loss sums.
//
// Layouts: target FP32 [ny][nx]; hidden activations and their gradients BF16
// channel-last [ny][nx][32] (the MFMA operand of one pixel is 8 consecutive
// channels = one 16-byte load); layer-5 output FP32 [ny][nx][2]; master
// parameters FP32 in the order of the oracle: per layer w[co][ci][3][3] then
// b[co]; tap t = (dy+1)*3 + (dx+1) reads input (y+dy, x+dx) mod (ny, nx).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cnn.hpp"
#include "fft_engine.hpp"

namespace holo {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even (inputs are finite)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float bfround(float f) { return bf2f(f2bf(f)); }

// ---------------------------------------------------------------------------
// Layer 1 (1 -> 32), VALU: out[y][x][co] = relu(b + sum_t w[co][t] T[y+dy][x+dx])
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv1(const float* __restrict__ target, int ny, int nx,
                                               const float* __restrict__ w /* [32][9] */,
                                               const float* __restrict__ b, uint16_t* __restrict__ out)
{
    __shared__ float ws[32 * 9 + 32];
    for (int i = threadIdx.x; i < 32 * 9; i += blockDim.x) ws[i] = bfround(w[i]);
    if (threadIdx.x < 32) ws[32 * 9 + threadIdx.x] = b[threadIdx.x];
    __syncthreads();
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nx * ny) return;
    const int y = p / nx, x = p - y * nx;
    float v[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = (y + t / 3 - 1 + ny) & (ny - 1), xx = (x + t % 3 - 1 + nx) & (nx - 1);
        v[t] = target[yy * nx + xx];
    }
    uint16_t o[32];
#pragma unroll
    for (int co = 0; co < 32; ++co) {
        float a = ws[32 * 9 + co];
#pragma unroll
        for (int t = 0; t < 9; ++t) a = fmaf(ws[co * 9 + t], v[t], a);
        o[co] = f2bf(a > 0.0f ? a : 0.0f);
    }
    uint4* dst = reinterpret_cast<uint4*>(out + (size_t)p * 32);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint4 u;
        u.x = o[8 * q] | ((uint32_t)o[8 * q + 1] << 16);
        u.y = o[8 * q + 2] | ((uint32_t)o[8 * q + 3] << 16);
        u.z = o[8 * q + 4] | ((uint32_t)o[8 * q + 5] << 16);
        u.w = o[8 * q + 6] | ((uint32_t)o[8 * q + 7] << 16);
        dst[q] = u;
    }
}

// ---------------------------------------------------------------------------
// 32 -> 32 layer on MFMA.  Block = 4 waves = 4 output rows y0..y0+3 of one
// 32-pixel segment x0..x0+31; each wave computes D[32 px][32 ch] with 18
// MFMA steps of K = 16 (tap t = step/2, channels 16*(step%2) .. +15).
// MODE 0 (forward): input = activation, weights Wk[co][t][ci], epilogue
//   relu(acc + b[co]).
// MODE 1 (backward data): input = dY, weights Wk[ci][8-t][co] (transposed,
//   taps reversed), epilogue acc * (act_prev > 0).
// LDS: input halo tile [6 rows][34 px][32 ch] and weights [32][9][32], BF16.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_conv32(const uint16_t* __restrict__ in, int ny, int nx,
                                                const uint16_t* __restrict__ wk, const float* __restrict__ bias,
                                                const uint16_t* __restrict__ act_prev, uint16_t* __restrict__ out)
{
    __shared__ __attribute__((aligned(16))) uint16_t tile[6 * 34 * 32];
    __shared__ __attribute__((aligned(16))) uint16_t wl[32 * 9 * 32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nseg = nx / 32;
    const int x0 = (blockIdx.x % nseg) * 32;
    const int y0 = (blockIdx.x / nseg) * 4;
    // stage weights (18 KiB) and the halo tile: 6*34 pixels x 64 bytes
    {
        const uint4* src = reinterpret_cast<const uint4*>(wk);
        uint4* dst = reinterpret_cast<uint4*>(wl);
        for (int i = threadIdx.x; i < 32 * 9 * 32 / 8; i += 256) dst[i] = src[i];
    }
    for (int i = threadIdx.x; i < 6 * 34 * 4; i += 256) {
        const int q = i & 3, pix = i >> 2;
        const int r = pix / 34, c = pix - r * 34;
        const int yy = (y0 + r - 1 + ny) & (ny - 1), xx = (x0 + c - 1 + nx) & (nx - 1);
        reinterpret_cast<uint4*>(tile)[pix * 4 + q] =
            reinterpret_cast<const uint4*>(in + ((size_t)yy * nx + xx) * 32)[q];
    }
    __syncthreads();
    f32x16 acc = {};
    const int i = lane & 31, kh = lane >> 5;   // pixel row of A / channel column of B; K half
#pragma unroll
    for (int step = 0; step < 18; ++step) {
        const int t = step >> 1, c0 = 16 * (step & 1) + 8 * kh;
        const int dy = t / 3, dx = t % 3;   // tile offsets (halo origin at -1)
        const uint4 a = *reinterpret_cast<const uint4*>(tile + ((wave + dy) * 34 + (i + dx)) * 32 + c0);
        const uint4 bw = *reinterpret_cast<const uint4*>(wl + (i * 9 + t) * 32 + c0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, bw),
                                                      acc, 0, 0, 0);
    }
    // D[px][ch]: register r holds pixel 8*(r/4) + 4*kh + (r%4), channel i
    const int y = y0 + wave;
    const float bb = MODE == 0 ? bias[i] : 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int px = 8 * (r >> 2) + 4 * kh + (r & 3);
        const size_t o = ((size_t)y * nx + x0 + px) * 32 + i;
        float v = acc[r];
        if (MODE == 0) {
            v += bb;
            v = v > 0.0f ? v : 0.0f;
        } else {
            v = act_prev[o] != 0 ? v : 0.0f;   // ReLU gate (activations are >= 0)
        }
        out[o] = f2bf(v);
    }
}

// ---------------------------------------------------------------------------
// Layer 5 (32 -> 2), VALU, and the phasor normalisation p = o/|o|.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv5(const uint16_t* __restrict__ in, int ny, int nx,
                                               const float* __restrict__ w /* [2][32][9] */,
                                               const float* __restrict__ b, float2* __restrict__ o5,
                                               float2* __restrict__ phasor)
{
    __shared__ float ws[2 * 32 * 9];
    for (int j = threadIdx.x; j < 2 * 32 * 9; j += blockDim.x) ws[j] = bfround(w[j]);
    __syncthreads();
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nx * ny) return;
    const int y = p / nx, x = p - y * nx;
    float a0 = b[0], a1 = b[1];
    for (int t = 0; t < 9; ++t) {
        const int yy = (y + t / 3 - 1 + ny) & (ny - 1), xx = (x + t % 3 - 1 + nx) & (nx - 1);
        const uint4* src = reinterpret_cast<const uint4*>(in + ((size_t)yy * nx + xx) * 32);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 u = src[q];
            const uint32_t wds[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const float v = bf2f((uint16_t)(wds[h >> 1] >> (16 * (h & 1))));
                const int ci = 8 * q + h;
                a0 = fmaf(ws[(0 * 32 + ci) * 9 + t], v, a0);
                a1 = fmaf(ws[(1 * 32 + ci) * 9 + t], v, a1);
            }
        }
    }
    o5[p] = make_float2(a0, a1);
    const float m = sqrtf(a0 * a0 + a1 * a1);
    phasor[p] = m > 0.0f ? make_float2(a0 / m, a1 / m) : make_float2(1.0f, 0.0f);
}

// ---------------------------------------------------------------------------
// Loss L = 1 - |Z| / W, Z = sum w p conj(q), W = sum w, w = T^2 (FP64 sums).
// The label may be any complex field (e.g. a GS replay field); its phasor
// q/|q| is used (0 -> 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 unit(float2 q)
{
    const float m = sqrtf(q.x * q.x + q.y * q.y);
    return m > 0.0f ? make_float2(q.x / m, q.y / m) : make_float2(1.0f, 0.0f);
}

__global__ __launch_bounds__(256) void k_loss_partial(const float2* __restrict__ ph, const float2* __restrict__ lab,
                                                      const float* __restrict__ target, int n,
                                                      double* __restrict__ part /* [blocks][3] */)
{
    __shared__ double red[3 * 8];
    double a[3] = {0.0, 0.0, 0.0};
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const double w = (double)target[p] * (double)target[p];
        const float2 pp = ph[p], q = unit(lab[p]);
        a[0] += w * ((double)pp.x * q.x + (double)pp.y * q.y);
        a[1] += w * ((double)pp.y * q.x - (double)pp.x * q.y);
        a[2] += w;
    }
    double s[3];
    block_sum<3>(a, red, s);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[blockIdx.x * 3 + k] = s[k];
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, int nb,
                                                    double* __restrict__ zsum /* zr, zi, W, loss */)
{
    __shared__ double red[3 * 8];
    double a[3] = {0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < nb; j += blockDim.x)
        for (int k = 0; k < 3; ++k) a[k] += part[j * 3 + k];
    double s[3];
    block_sum<3>(a, red, s);
    if (threadIdx.x == 0) {
        zsum[0] = s[0];
        zsum[1] = s[1];
        zsum[2] = s[2];
        zsum[3] = s[2] > 0.0 ? 1.0 - sqrt(s[0] * s[0] + s[1] * s[1]) / s[2] : 0.0;
    }
}

// dL/do for the raw layer-5 output: g = dL/dp = -(w / (W |Z|)) Z q, then
// through p = o/|o|: (g - (g.p) p) / |o|.
__global__ __launch_bounds__(256) void k_loss_grad(const float2* __restrict__ o5, const float2* __restrict__ lab,
                                                   const float* __restrict__ target, int n,
                                                   const double* __restrict__ zsum, float2* __restrict__ d5)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double zr = zsum[0], zi = zsum[1], W = zsum[2];
    const double zm = sqrt(zr * zr + zi * zi);
    const float w = target[p] * target[p];
    const float k = (W > 0.0 && zm > 0.0) ? (float)(-(double)w / (W * zm)) : 0.0f;
    const float2 q = unit(lab[p]);
    const float gr = k * ((float)zr * q.x - (float)zi * q.y), gi = k * ((float)zr * q.y + (float)zi * q.x);
    const float2 o = o5[p];
    const float m = sqrtf(o.x * o.x + o.y * o.y);
    float2 d = make_float2(0.0f, 0.0f);
    if (m > 0.0f) {
        const float pr = o.x / m, pi = o.y / m, dd = gr * pr + gi * pi;
        d = make_float2((gr - dd * pr) / m, (gi - dd * pi) / m);
    }
    d5[p] = d;
}

// Backward data of layer 5: dX4[y][x][ci] = (sum_{co,t} w5[co][ci][t] d5[y-dy][x-dx][co]) * (act4 > 0)
__global__ __launch_bounds__(256) void k_conv5_bwd_data(const float2* __restrict__ d5, int ny, int nx,
                                                        const float* __restrict__ w,
                                                        const uint16_t* __restrict__ act4,
                                                        uint16_t* __restrict__ dx)
{
    __shared__ float ws[2 * 32 * 9];
    for (int j = threadIdx.x; j < 2 * 32 * 9; j += blockDim.x) ws[j] = bfround(w[j]);
    __syncthreads();
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nx * ny) return;
    const int y = p / nx, x = p - y * nx;
    float g[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        // input (y, x) reaches output (y - dy, x - dx) through tap t
        const int yy = (y - (t / 3 - 1) + ny) & (ny - 1), xx = (x - (t % 3 - 1) + nx) & (nx - 1);
        const float2 d = d5[yy * nx + xx];
        g[t][0] = d.x;
        g[t][1] = d.y;
    }
    uint16_t o[32];
#pragma unroll
    for (int ci = 0; ci < 32; ++ci) {
        float a = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) a = fmaf(ws[ci * 9 + t], g[t][0], fmaf(ws[(32 + ci) * 9 + t], g[t][1], a));
        o[ci] = f2bf(act4[(size_t)p * 32 + ci] != 0 ? a : 0.0f);
    }
    uint4* dst = reinterpret_cast<uint4*>(dx + (size_t)p * 32);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint4 u;
        u.x = o[8 * q] | ((uint32_t)o[8 * q + 1] << 16);
        u.y = o[8 * q + 2] | ((uint32_t)o[8 * q + 3] << 16);
        u.z = o[8 * q + 4] | ((uint32_t)o[8 * q + 5] << 16);
        u.w = o[8 * q + 6] | ((uint32_t)o[8 * q + 7] << 16);
        dst[q] = u;
    }
}

// ---------------------------------------------------------------------------
// Weight gradients (VALU, FP32 accumulation), per-block partials over a
// contiguous range of rows, reduced by k_grad_reduce in a fixed order.
// 32 -> 32: thread = (tap, 4 output channels, 4 input channels): 576 threads;
// per pixel one 8-byte LDS read of dY and one of X, 16 FMAs.
// partial layout per block: [co][ci][t] (oracle order) then bias [co].
// ---------------------------------------------------------------------------
constexpr int kSeg = 256;   // pixels per row segment staged in LDS
__global__ __launch_bounds__(576) void k_dw32(const uint16_t* __restrict__ x /* act_{l-1} */,
                                              const uint16_t* __restrict__ dy, int ny, int nx,
                                              int rows_per_block, float* __restrict__ part)
{
    // one row segment of `seg` pixels: dY [seg][32] and X [3][seg + 2][32]
    __shared__ __attribute__((aligned(16))) uint16_t sdy[kSeg * 32];
    __shared__ __attribute__((aligned(16))) uint16_t sx[3 * (kSeg + 2) * 32];
    const int seg = nx < kSeg ? nx : kSeg;
    const int tid = threadIdx.x;
    const int t = tid / 64, cog = (tid >> 3) & 7, cig = tid & 7;
    const int dyo = t / 3, dxo = t % 3;
    float acc[4][4] = {};
    float accb = 0.0f;   // bias gradient: threads 0..31 own channel tid
    const int ybeg = blockIdx.x * rows_per_block;
    for (int y = ybeg; y < ybeg + rows_per_block && y < ny; ++y)
        for (int xs = 0; xs < nx; xs += seg) {
            __syncthreads();
            for (int i = tid; i < seg * 4; i += 576)
                reinterpret_cast<uint4*>(sdy)[i] =
                    reinterpret_cast<const uint4*>(dy + ((size_t)y * nx + xs) * 32)[i];
            for (int i = tid; i < 3 * (seg + 2) * 4; i += 576) {
                const int q = i & 3, pix = i >> 2;
                const int r = pix / (seg + 2), c = pix - r * (seg + 2);
                const int yy = (y + r - 1 + ny) & (ny - 1), xx = (xs + c - 1 + nx) & (nx - 1);
                reinterpret_cast<uint4*>(sx)[pix * 4 + q] =
                    reinterpret_cast<const uint4*>(x + ((size_t)yy * nx + xx) * 32)[q];
            }
            __syncthreads();
            for (int px = 0; px < seg; ++px) {
                const uint2 gd = *reinterpret_cast<const uint2*>(sdy + px * 32 + 4 * cog);
                const uint2 gx = *reinterpret_cast<const uint2*>(sx + (dyo * (seg + 2) + px + dxo) * 32 + 4 * cig);
                const float d[4] = {bf2f(gd.x & 0xFFFF), bf2f(gd.x >> 16), bf2f(gd.y & 0xFFFF), bf2f(gd.y >> 16)};
                const float v[4] = {bf2f(gx.x & 0xFFFF), bf2f(gx.x >> 16), bf2f(gx.y & 0xFFFF), bf2f(gx.y >> 16)};
#pragma unroll
                for (int a2 = 0; a2 < 4; ++a2)
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[a2][c] = fmaf(d[a2], v[c], acc[a2][c]);
            }
            if (tid < 32)
                for (int px = 0; px < seg; ++px) accb += bf2f(sdy[px * 32 + tid]);
        }
    float* o = part + (size_t)blockIdx.x * (32 * 32 * 9 + 32);
#pragma unroll
    for (int a2 = 0; a2 < 4; ++a2)
#pragma unroll
        for (int c = 0; c < 4; ++c) o[((4 * cog + a2) * 32 + 4 * cig + c) * 9 + t] = acc[a2][c];
    if (tid < 32) o[32 * 32 * 9 + tid] = accb;
}

// Layer 1 weight gradient: dW1[co][t] = sum_p dY1[p][co] T[p + d(t)]; thread
// (co, t) = 288 threads, loops over the block's rows.
__global__ __launch_bounds__(320) void k_dw1(const float* __restrict__ target, const uint16_t* __restrict__ dy,
                                             int ny, int nx, int rows_per_block, float* __restrict__ part)
{
    const int tid = threadIdx.x;
    const int co = tid / 10, t = tid % 10;   // t == 9: bias
    float acc = 0.0f;
    if (co < 32) {
        const int ybeg = blockIdx.x * rows_per_block;
        for (int y = ybeg; y < ybeg + rows_per_block && y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const float d = bf2f(dy[((size_t)y * nx + x) * 32 + co]);
                float v = 1.0f;
                if (t < 9) {
                    const int yy = (y + t / 3 - 1 + ny) & (ny - 1), xx = (x + t % 3 - 1 + nx) & (nx - 1);
                    v = target[yy * nx + xx];
                }
                acc = fmaf(d, v, acc);
            }
        float* o = part + (size_t)blockIdx.x * (32 * 9 + 32);
        if (t < 9) o[co * 9 + t] = acc;
        else o[32 * 9 + co] = acc;
    }
}

// Layer 5 weight gradient: dW5[co][ci][t] = sum_p d5[p][co] X4[p + d(t)][ci];
// thread (ci, t) handles both output channels: 288 threads (+2 bias).
__global__ __launch_bounds__(320) void k_dw5(const uint16_t* __restrict__ x4, const float2* __restrict__ d5,
                                             int ny, int nx, int rows_per_block, float* __restrict__ part)
{
    const int tid = threadIdx.x;
    const int ci = tid / 9, t = tid % 9;
    float a0 = 0.0f, a1 = 0.0f;
    const int ybeg = blockIdx.x * rows_per_block;
    for (int y = ybeg; y < ybeg + rows_per_block && y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const float2 d = d5[(size_t)y * nx + x];
            if (tid < 288) {
                const int yy = (y + t / 3 - 1 + ny) & (ny - 1), xx = (x + t % 3 - 1 + nx) & (nx - 1);
                const float v = bf2f(x4[((size_t)yy * nx + xx) * 32 + ci]);
                a0 = fmaf(d.x, v, a0);
                a1 = fmaf(d.y, v, a1);
            } else if (tid == 288) {
                a0 += d.x;
            } else if (tid == 289) {
                a1 += d.y;
            }
        }
    float* o = part + (size_t)blockIdx.x * (2 * 32 * 9 + 2);
    if (tid < 288) {
        o[(0 * 32 + ci) * 9 + t] = a0;
        o[(1 * 32 + ci) * 9 + t] = a1;
    } else if (tid == 288) {
        o[2 * 32 * 9] = a0;
    } else if (tid == 289) {
        o[2 * 32 * 9 + 1] = a1;
    }
}

// grad[j] = sum over blocks of part[b][j], fixed order.
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ part, int nblocks, int n,
                                                     float* __restrict__ grad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * n + j];
    grad[j] = s;
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int n, float lr, float b1,
                                              float b2, float eps, float c1, float c2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.0f - b1) * gj;
    const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    p[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// BF16 MFMA weight copies of a 32->32 layer from its master [co][ci][t]:
// forward Wk[co][t][ci]; backward-data Wt[ci][8-t][co].
__global__ __launch_bounds__(256) void k_pack32(const float* __restrict__ w, uint16_t* __restrict__ wf,
                                                uint16_t* __restrict__ wt)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= 32 * 32 * 9) return;
    const int co = j / 288, ci = (j / 9) % 32, t = j % 9;
    const uint16_t h = f2bf(w[j]);
    wf[(co * 9 + t) * 32 + ci] = h;
    wt[(ci * 9 + (8 - t)) * 32 + co] = h;
}

}  // namespace cnn

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t cnn_launch_forward(const CnnBuffers& b, const float* target, int ny, int nx, float2* phasor,
                              hipStream_t s)
{
    using namespace cnn;
    const int npx = nx * ny;
    const int g256 = (npx + 255) / 256;
    const dim3 gmf((nx / 32) * (ny / 4));
    hipLaunchKernelGGL(k_conv1, dim3(g256), dim3(256), 0, s, target, ny, nx, b.params + b.off[0],
                       b.params + b.off[0] + 32 * 9, b.act[0]);
    for (int l = 1; l <= 3; ++l)
        hipLaunchKernelGGL(k_conv32<0>, gmf, dim3(256), 0, s, b.act[l - 1], ny, nx, b.wf[l - 1],
                           b.params + b.off[l] + 32 * 32 * 9, nullptr, b.act[l]);
    hipLaunchKernelGGL(k_conv5, dim3(g256), dim3(256), 0, s, b.act[3], ny, nx, b.params + b.off[4],
                       b.params + b.off[4] + 2 * 32 * 9, b.o5, phasor);
    return hipGetLastError();
}

hipError_t cnn_launch_loss(const CnnBuffers& b, const float* target, const float2* label, const float2* phasor,
                           int n, hipStream_t s)
{
    using namespace cnn;
    const int nb = 256;
    hipLaunchKernelGGL(k_loss_partial, dim3(nb), dim3(256), 0, s, phasor, label, target, n, b.loss_part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, b.loss_part, nb, b.zsum);
    return hipGetLastError();
}

hipError_t cnn_launch_backward(const CnnBuffers& b, const float* target, const float2* label, int ny, int nx,
                               hipStream_t s)
{
    using namespace cnn;
    const int npx = nx * ny;
    const int g256 = (npx + 255) / 256;
    const dim3 gmf((nx / 32) * (ny / 4));
    const int rpb = b.rows_per_block;
    const int nblk = (ny + rpb - 1) / rpb;
    hipLaunchKernelGGL(k_loss_grad, dim3(g256), dim3(256), 0, s, b.o5, label, target, npx, b.zsum, b.d5);
    // layer 5
    hipLaunchKernelGGL(k_dw5, dim3(nblk), dim3(320), 0, s, b.act[3], b.d5, ny, nx, rpb, b.part);
    hipLaunchKernelGGL(k_grad_reduce, dim3((2 * 32 * 9 + 2 + 255) / 256), dim3(256), 0, s, b.part, nblk,
                       2 * 32 * 9 + 2, b.grad + b.off[4]);
    hipLaunchKernelGGL(k_conv5_bwd_data, dim3(g256), dim3(256), 0, s, b.d5, ny, nx, b.params + b.off[4], b.act[3],
                       b.dact[0]);
    // layers 4, 3, 2 (index l = 3, 2, 1): dW from act[l-1] and dY; dX through MFMA
    uint16_t* dcur = b.dact[0];
    uint16_t* dnext = b.dact[1];
    for (int l = 3; l >= 1; --l) {
        hipLaunchKernelGGL(k_dw32, dim3(nblk), dim3(576), 0, s, b.act[l - 1], dcur, ny, nx, rpb, b.part);
        hipLaunchKernelGGL(k_grad_reduce, dim3((32 * 32 * 9 + 32 + 255) / 256), dim3(256), 0, s, b.part, nblk,
                           32 * 32 * 9 + 32, b.grad + b.off[l]);
        hipLaunchKernelGGL(k_conv32<1>, gmf, dim3(256), 0, s, dcur, ny, nx, b.wt[l - 1], nullptr, b.act[l - 1],
                           dnext);
        uint16_t* tmp = dcur;
        dcur = dnext;
        dnext = tmp;
    }
    // layer 1
    hipLaunchKernelGGL(k_dw1, dim3(nblk), dim3(320), 0, s, target, dcur, ny, nx, rpb, b.part);
    hipLaunchKernelGGL(k_grad_reduce, dim3((32 * 9 + 32 + 255) / 256), dim3(256), 0, s, b.part, nblk, 32 * 9 + 32,
                       b.grad + b.off[0]);
    return hipGetLastError();
}

hipError_t cnn_launch_adam(const CnnBuffers& b, int n, float lr, int step, hipStream_t s)
{
    using namespace cnn;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - pow(0.9, step)), c2 = (float)(1.0 - pow(0.999, step));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, b.params, b.grad, b.m, b.v, n, lr, b1, b2,
                       1e-8f, c1, c2);
    return cnn_launch_pack(b, s);
}

hipError_t cnn_launch_pack(const CnnBuffers& b, hipStream_t s)
{
    using namespace cnn;
    for (int l = 1; l <= 3; ++l)
        hipLaunchKernelGGL(k_pack32, dim3((32 * 32 * 9 + 255) / 256), dim3(256), 0, s, b.params + b.off[l],
                           b.wf[l - 1], b.wt[l - 1]);
    return hipGetLastError();
}

}  // namespace holo

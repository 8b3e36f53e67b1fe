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
    __shared__ __attribute__((aligned(16))) uint16_t stage[256 * 40];
    for (int i = threadIdx.x; i < 32 * 9; i += blockDim.x) ws[i] = bfround(w[i]);
    if (threadIdx.x < 32) ws[32 * 9 + threadIdx.x] = b[threadIdx.x];
    __syncthreads();
    const int p = min(blockIdx.x * blockDim.x + threadIdx.x, nx * ny - 1);   // tail lanes recompute the last pixel
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
    // the block's 256 pixels are one contiguous 16 KiB run of the output: stage
    // each pixel's 64 bytes in LDS (80-byte pitch against bank conflicts), then
    // store 16-byte words at consecutive addresses
    uint4* sp = reinterpret_cast<uint4*>(stage + threadIdx.x * 40);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint4 u;
        u.x = o[8 * q] | ((uint32_t)o[8 * q + 1] << 16);
        u.y = o[8 * q + 2] | ((uint32_t)o[8 * q + 3] << 16);
        u.z = o[8 * q + 4] | ((uint32_t)o[8 * q + 5] << 16);
        u.w = o[8 * q + 6] | ((uint32_t)o[8 * q + 7] << 16);
        sp[q] = u;
    }
    __syncthreads();
    const int p0 = blockIdx.x * blockDim.x;
    const int npx = nx * ny - p0 < (int)blockDim.x ? nx * ny - p0 : (int)blockDim.x;   // pixels in this block
    uint4* dst = reinterpret_cast<uint4*>(out + (size_t)p0 * 32);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int w = q * (int)blockDim.x + threadIdx.x;   // 16-byte word of the run
        if (w < npx * 4) dst[w] = *reinterpret_cast<const uint4*>(stage + (w >> 2) * 40 + (w & 3) * 8);
    }
}

// ---------------------------------------------------------------------------
// 32 -> 32 layer on MFMA.  Block = 4 waves over a tile of kConvRows rows x 32
// pixels; wave w computes tile rows w*kConvRows/4 .. +kConvRows/4-1, one 32-pixel x
// 32-channel result per row, from 18 MFMA steps of K = 16 (tap t = step/2,
// input channels 16*(step%2) .. +15).  The weights stay in registers for the
// whole tile (lane l holds the 18 B-operand words of output channel l%32);
// the activations come from an LDS halo tile [18 rows][34 px][32 ch].
// MODE 0 (forward): input = activation, weights Wk[co][t][ci], epilogue
//   relu(acc + b[co]).
// MODE 1 (backward data): input = dY, weights Wk[ci][8-t][co] (transposed,
//   taps reversed), epilogue acc * (act_prev > 0).
// ---------------------------------------------------------------------------
constexpr int kConvRows = 8;
constexpr int kOutPitch = 40;   // u16 per staged output pixel (80-byte rows)
template <int MODE>
__global__ __launch_bounds__(256) void k_conv32(const uint16_t* __restrict__ in, int ny, int nx,
                                                const uint16_t* __restrict__ wk, const float* __restrict__ bias,
                                                const uint16_t* __restrict__ act_prev, uint16_t* __restrict__ out)
{
    __shared__ __attribute__((aligned(16))) uint16_t tile[(kConvRows + 2) * 34 * 32];
    __shared__ __attribute__((aligned(16))) uint16_t opage[4][32 * kOutPitch];   // per-wave output staging
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 31, kh = lane >> 5;   // pixel row of A / channel column of B; K half
    const int nseg = nx / 32;
    const int x0 = (blockIdx.x % nseg) * 32;
    const int y0 = (blockIdx.x / nseg) * kConvRows;
    // weights: B[k][n = i] for step s = 8 channels of tap s/2
    uint4 bw[18];
#pragma unroll
    for (int st = 0; st < 18; ++st)
        bw[st] = *reinterpret_cast<const uint4*>(wk + (i * 9 + (st >> 1)) * 32 + 16 * (st & 1) + 8 * kh);
    const int rows = ny - y0 < kConvRows ? ny - y0 : kConvRows;
    for (int j = threadIdx.x; j < (rows + 2) * 34 * 4; j += 256) {
        const int q = j & 3, pix = j >> 2;
        const int r = pix / 34, c = pix - r * 34;
        const int yy = (y0 + r - 1 + ny) & (ny - 1), xx = (x0 + c - 1 + nx) & (nx - 1);
        reinterpret_cast<uint4*>(tile)[pix * 4 + q] = reinterpret_cast<const uint4*>(in + ((size_t)yy * nx + xx) * 32)[q];
    }
    __syncthreads();
    const float bb = MODE == 0 ? bias[i] : 0.0f;
    for (int rr = 0; rr < kConvRows / 4; ++rr) {
        const int rl = wave * (kConvRows / 4) + rr;   // tile row
        if (rl >= rows) break;
        f32x16 acc = {};
#pragma unroll
        for (int st = 0; st < 18; ++st) {
            const int t = st >> 1, c0 = 16 * (st & 1) + 8 * kh;
            const int dy = t / 3, dx = t % 3;   // tile offsets (halo origin at -1)
            const uint4 a = *reinterpret_cast<const uint4*>(tile + ((rl + dy) * 34 + (i + dx)) * 32 + c0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                          __builtin_bit_cast(bf16x8, bw[st]), acc, 0, 0, 0);
        }
        // D[px][ch]: register r holds pixel 8*(r/4) + 4*kh + (r%4), channel i.
        // Through this wave's LDS page to [px][ch] order, then 16-byte stores
        // (8 channels of one pixel); MODE 1 gates with the matching 16-byte
        // word of act_prev.
        uint16_t* pg = opage[wave];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int px = 8 * (r >> 2) + 4 * kh + (r & 3);
            float v = acc[r];
            if (MODE == 0) {
                v += bb;
                v = v > 0.0f ? v : 0.0f;
            }
            pg[px * kOutPitch + i] = f2bf(v);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int y = y0 + rl;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int w = lane + 64 * h;          // 128 words: pixel w/4, channels 8*(w%4)..
            const int px = w >> 2, q = w & 3;
            uint4 u = *reinterpret_cast<const uint4*>(pg + px * kOutPitch + 8 * q);
            uint4* dst = reinterpret_cast<uint4*>(out + ((size_t)y * nx + x0 + px) * 32) + q;
            if (MODE == 1) {
                const uint4 g = reinterpret_cast<const uint4*>(act_prev + ((size_t)y * nx + x0 + px) * 32)[q];
                auto gate = [](uint32_t val, uint32_t gw) {
                    const uint32_t lo = (gw & 0xFFFFu) ? (val & 0xFFFFu) : 0u;
                    const uint32_t hi = (gw >> 16) ? (val & 0xFFFF0000u) : 0u;
                    return lo | hi;
                };
                u = make_uint4(gate(u.x, g.x), gate(u.y, g.y), gate(u.z, g.z), gate(u.w, g.w));
            }
            *dst = u;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---------------------------------------------------------------------------
// Layer 5 (32 -> 2), VALU, and the phasor normalisation p = o/|o|.
// ---------------------------------------------------------------------------
// 32 -> 2 output layer.  Block = up to 512 pixels: a tile of R = min(512/W,
// ny) rows x W pixels (W = min(nx, 64)), two vertically adjacent pixels per
// thread, whose
// halo [R+2][W+2][32 ch] is staged in LDS with coalesced 16-byte loads; a
// thread reads the 4 x 3 neighbourhood its two pixels share from LDS.
// Activations and weights are both BF16, so each pair of input channels is one
// v_dot2 (two exact products accumulated in FP32); the weights, packed as BF16
// pairs by k_pack5 in [tap][ci/2][co] order, are read with block-uniform
// addresses (scalar loads).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
constexpr int kC5Px = 512;                          // pixels per block
__global__ __launch_bounds__(256) void k_conv5(const uint16_t* __restrict__ in, int ny, int nx,
                                               const uint32_t* __restrict__ w5 /* [9][16][2] BF16 pairs */,
                                               const float* __restrict__ b, float2* __restrict__ o5,
                                               float2* __restrict__ phasor)
{
    __shared__ __attribute__((aligned(16))) uint16_t tile[660 * 32];   // (R+2)(W+2) <= 660 pixels
    const int W = nx < 64 ? nx : 64, R = kC5Px / W < ny ? kC5Px / W : ny;   // launcher: same W, R
    const int nseg = nx / W;
    const int x0 = (blockIdx.x % nseg) * W, y0 = (blockIdx.x / nseg) * R;
    const int hw = W + 2, nchunk = (R + 2) * hw * 4;
    for (int j = threadIdx.x; j < nchunk; j += blockDim.x) {
        const int pix = j >> 2, part = j & 3;
        const int ty = pix / hw, tx = pix - ty * hw;
        const int gy = (y0 + ty - 1 + ny) & (ny - 1), gx = (x0 + tx - 1 + nx) & (nx - 1);
        reinterpret_cast<uint4*>(tile)[j] =
            reinterpret_cast<const uint4*>(in + ((size_t)gy * nx + gx) * 32)[part];
    }
    __syncthreads();
    const int r2 = threadIdx.x / W, c = threadIdx.x - r2 * W;   // pixels at tile rows 2*r2, 2*r2 + 1
    if (2 * r2 >= R) return;                                    // a tile smaller than 512 pixels
    float a0 = b[0], a1 = b[1], b0 = b[0], b1 = b[1];
#pragma unroll
    for (int hr = 0; hr < 4; ++hr) {        // halo row 2*r2 + hr: tap row hr of pixel A, hr - 1 of pixel B
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const uint4* src = reinterpret_cast<const uint4*>(tile + ((2 * r2 + hr) * hw + c + dx) * 32);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 u = src[q];
                const uint32_t wds[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {   // channels 8q + 2k, 8q + 2k + 1
                    const bf16x2_t v = __builtin_bit_cast(bf16x2_t, wds[k]);
                    if (hr < 3) {
                        const int pr = (hr * 3 + dx) * 16 + 4 * q + k;
                        a0 = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w5[pr * 2]), v, a0, false);
                        a1 = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w5[pr * 2 + 1]), v, a1,
                                                             false);
                    }
                    if (hr > 0) {
                        const int pr = ((hr - 1) * 3 + dx) * 16 + 4 * q + k;
                        b0 = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w5[pr * 2]), v, b0, false);
                        b1 = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w5[pr * 2 + 1]), v, b1,
                                                             false);
                    }
                }
            }
        }
    }
    const size_t pa = (size_t)(y0 + 2 * r2) * nx + x0 + c, pb = pa + nx;
    o5[pa] = make_float2(a0, a1);
    o5[pb] = make_float2(b0, b1);
    const float ma = sqrtf(a0 * a0 + a1 * a1), mb = sqrtf(b0 * b0 + b1 * b1);
    phasor[pa] = ma > 0.0f ? make_float2(a0 / ma, a1 / ma) : make_float2(1.0f, 0.0f);
    phasor[pb] = mb > 0.0f ? make_float2(b0 / mb, b1 / mb) : make_float2(1.0f, 0.0f);
}

// Layer-5 weights [co][ci][t] (FP32 master) -> BF16 pairs [t][ci/2][co]
// (channel 2k in the low half, 2k+1 in the high half).
__global__ __launch_bounds__(256) void k_pack5(const float* __restrict__ w, uint32_t* __restrict__ w5)
{
    for (int j = threadIdx.x; j < 9 * 16 * 2; j += blockDim.x) {
        const int co = j & 1, k = (j >> 1) % 16, t = j / 32;
        const uint32_t lo = f2bf(w[(co * 32 + 2 * k) * 9 + t]), hi = f2bf(w[(co * 32 + 2 * k + 1) * 9 + t]);
        w5[j] = lo | (hi << 16);
    }
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
                                                    double* __restrict__ zsum /* zr, zi, W, loss, batch mean */,
                                                    int accumulate, double inv_batch)
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
        zsum[4] = (accumulate ? zsum[4] : 0.0) + zsum[3] * inv_batch;
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
// Weight gradients, FP32 accumulation, one partial per block over a
// contiguous range of image rows, reduced by k_grad_reduce in a fixed order.
// Partial layout per block: [co][ci][t] (the oracle's order), then bias [co].
// ---------------------------------------------------------------------------

// 32 -> 32 on MFMA: for tap t = (dy, dx), dW_t[co][ci] = sum_p dY[p][co] *
// X[p + (dy, dx)][ci] is a 32x32 product with K = pixels.  The pixel axis has
// to be the operand's contiguous axis, so each 32-pixel segment of a row is
// staged in LDS transposed, dYt[co][px] and Xt[dy][ci][halo px], by threads
// that load 8 pixels x 8 channels (eight 16-byte words), transpose the 8x8
// block in registers and write eight 16-byte rows.  Block = 3 waves; wave w
// owns the taps of kernel row dy = w - 1 (three 32x32 accumulators); the
// dx-shifted B operand comes from two aligned 16-byte reads and a funnel
// shift.  D = A B with A[m = co][k = px] and B[k = px][n = ci]; register r of
// lane l holds co = 8*(r/4) + 4*(l/32) + r%4, ci = l%32.  The next segment's
// words are loaded while the current one is multiplied.
constexpr int kDwSeg = 64;                    // output pixels per staged segment
constexpr int kDwGx = (kDwSeg + 2 + 7) / 8;   // 8-pixel groups of a halo row
constexpr int kDwPitch = 8 * kDwGx;           // u16 per LDS channel row (16-byte aligned rows)
constexpr int kDwNx = 3 * 4 * kDwGx;          // X staging threads
constexpr int kDwNd = 4 * (kDwSeg / 8);       // dY staging threads

// 8 pixels x 8 channels (w[p] = channels 0..7 of pixel p) -> channel e's 8
// pixels as one 16-byte word.
__device__ __forceinline__ uint4 transpose_ch(const uint4 (&w)[8], int e)
{
    uint32_t d[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint4 a = w[2 * j], b = w[2 * j + 1];
        const uint32_t av = (e >> 1) == 0 ? a.x : (e >> 1) == 1 ? a.y : (e >> 1) == 2 ? a.z : a.w;
        const uint32_t bv = (e >> 1) == 0 ? b.x : (e >> 1) == 1 ? b.y : (e >> 1) == 2 ? b.z : b.w;
        d[j] = (e & 1) ? ((av >> 16) | (bv & 0xFFFF0000u)) : ((av & 0xFFFFu) | (bv << 16));
    }
    return make_uint4(d[0], d[1], d[2], d[3]);
}

__global__ __launch_bounds__(192) void k_dw32(const uint16_t* __restrict__ x /* act_{l-1} */,
                                              const uint16_t* __restrict__ dy, int ny, int nx,
                                              int rows_per_block, float* __restrict__ part)
{
    __shared__ __attribute__((aligned(16))) uint16_t dyt[32 * kDwPitch];
    __shared__ __attribute__((aligned(16))) uint16_t xt[3 * 32 * kDwPitch];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, half = lane >> 5;
    f32x16 acc[3] = {};
    float accb = 0.0f;   // bias gradient of channel tid (tid < 32)
    const int ybeg = blockIdx.x * rows_per_block;
    const int yend = ybeg + rows_per_block < ny ? ybeg + rows_per_block : ny;
    const int segs_per_row = nx / kDwSeg;
    const int nseg = (yend - ybeg) * segs_per_row;
    // staging roles: tid < kDwNx: X row r, channels 8q.., halo pixels
    // 8g..8g+7 (halo pixel c is x0 - 1 + c); the next kDwNd threads: dY
    // channels 8q.., pixels 8g..
    static_assert(kDwNx + kDwNd <= 192, "staging threads");
    const bool sx = tid < kDwNx, sd = tid >= kDwNx && tid < kDwNx + kDwNd;
    const int j_ = sd ? tid - kDwNx : tid;
    const int r_ = sx ? tid / (4 * kDwGx) : 0;
    const int q_ = sx ? (tid % (4 * kDwGx)) / kDwGx : j_ / (kDwSeg / 8);
    const int g_ = sx ? tid % kDwGx : j_ % (kDwSeg / 8);
    uint4 w[8];
    auto fetch = [&](int sidx) {
        const int y = ybeg + sidx / segs_per_row, x0 = (sidx % segs_per_row) * kDwSeg;
        if (sx) {
            const int yy = (y + r_ - 1 + ny) & (ny - 1);
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const int xx = (x0 + 8 * g_ + p - 1 + nx) & (nx - 1);
                w[p] = reinterpret_cast<const uint4*>(x + ((size_t)yy * nx + xx) * 32)[q_];
            }
        } else if (sd) {
#pragma unroll
            for (int p = 0; p < 8; ++p)
                w[p] = reinterpret_cast<const uint4*>(dy + ((size_t)y * nx + x0 + 8 * g_ + p) * 32)[q_];
        }
    };
    if (nseg > 0) fetch(0);
    for (int sidx = 0; sidx < nseg; ++sidx) {
        __syncthreads();
        if (sx) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *reinterpret_cast<uint4*>(xt + (r_ * 32 + 8 * q_ + e) * kDwPitch + 8 * g_) = transpose_ch(w, e);
        } else if (sd) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *reinterpret_cast<uint4*>(dyt + (8 * q_ + e) * kDwPitch + 8 * g_) = transpose_ch(w, e);
        }
        __syncthreads();
        if (sidx + 1 < nseg) fetch(sidx + 1);   // next segment in flight during the products
#pragma unroll
        for (int ks = 0; ks < kDwSeg / 16; ++ks) {
            const int c0 = 16 * ks + 8 * half;
            const uint4 a = *reinterpret_cast<const uint4*>(dyt + l32 * kDwPitch + c0);
            const uint16_t* xr = xt + (wave * 32 + l32) * kDwPitch + c0;
            const uint4 lo = *reinterpret_cast<const uint4*>(xr);
            const uint4 hi = *reinterpret_cast<const uint4*>(xr + 8);
            // output pixel c0 + e with tap dx reads halo pixel c0 + e + dx
            const uint4 b0 = lo;
            const uint4 b1 = make_uint4(__builtin_amdgcn_alignbit(lo.y, lo.x, 16), __builtin_amdgcn_alignbit(lo.z, lo.y, 16),
                                        __builtin_amdgcn_alignbit(lo.w, lo.z, 16), __builtin_amdgcn_alignbit(hi.x, lo.w, 16));
            const uint4 b2 = make_uint4(lo.y, lo.z, lo.w, hi.x);
            const bf16x8 av = __builtin_bit_cast(bf16x8, a);
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8, b0), acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8, b1), acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, __builtin_bit_cast(bf16x8, b2), acc[2], 0, 0, 0);
        }
        if (tid < 32)
#pragma unroll 8
            for (int px = 0; px < kDwSeg; ++px) accb += bf2f(dyt[tid * kDwPitch + px]);
    }
    float* o = part + (size_t)blockIdx.x * (32 * 32 * 9 + 32);
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int co = 8 * (r >> 2) + 4 * half + (r & 3);
            o[(co * 32 + l32) * 9 + wave * 3 + dx] = acc[dx][r];
        }
    if (tid < 32) o[32 * 32 * 9 + tid] = accb;
}

// Layers 1 and 5 (few outputs, K = all pixels) on the vector ALUs: block = 8
// groups x 32 lanes and one image row; group g runs over pixels
// [g*nx/8, (g+1)*nx/8) with a 3x3 window of its lane's input values in
// registers (one new column per pixel), and the 8 groups' sums are added in
// group order through LDS.
// Layer 5: lane = input channel ci; per pixel 18 FMAs (2 outputs x 9 taps);
// lanes 0, 1 of group 0.. also sum the bias of output channel lane.
__global__ __launch_bounds__(256) void k_dw5(const uint16_t* __restrict__ x4, const float2* __restrict__ d5,
                                             int ny, int nx, int rows_per_block, float* __restrict__ part)
{
    constexpr int NO = 2 * 32 * 9 + 2;
    __shared__ float red[8][NO];
    const int ci = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int seg = nx / 8;
    float a0[9] = {}, a1[9] = {};
    float b0 = 0.0f, b1 = 0.0f;
    const int ybeg = blockIdx.x * rows_per_block;
    for (int y = ybeg; y < ybeg + rows_per_block && y < ny; ++y) {
        size_t rowo[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) rowo[r] = (size_t)((y + r - 1 + ny) & (ny - 1)) * nx;
        const int xs = g * seg;
        float wv[3][3];   // [row][col] = X[y+row-1][x+col-1][ci]
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            wv[r][0] = bf2f(x4[(rowo[r] + ((xs - 1 + nx) & (nx - 1))) * 32 + ci]);
            wv[r][1] = bf2f(x4[(rowo[r] + xs) * 32 + ci]);
        }
        for (int xi = xs; xi < xs + seg; ++xi) {
            const int xn = (xi + 1) & (nx - 1);
#pragma unroll
            for (int r = 0; r < 3; ++r) wv[r][2] = bf2f(x4[(rowo[r] + xn) * 32 + ci]);
            const float2 d = d5[(size_t)y * nx + xi];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                a0[t] = fmaf(d.x, wv[t / 3][t % 3], a0[t]);
                a1[t] = fmaf(d.y, wv[t / 3][t % 3], a1[t]);
            }
            b0 += d.x;
            b1 += d.y;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                wv[r][0] = wv[r][1];
                wv[r][1] = wv[r][2];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        red[g][(0 * 32 + ci) * 9 + t] = a0[t];
        red[g][(1 * 32 + ci) * 9 + t] = a1[t];
    }
    if (ci == 0) {
        red[g][2 * 32 * 9] = b0;
        red[g][2 * 32 * 9 + 1] = b1;
    }
    __syncthreads();
    float* o = part + (size_t)blockIdx.x * NO;
    for (int j = threadIdx.x; j < NO; j += 256) {
        float s = red[0][j];
#pragma unroll
        for (int gg = 1; gg < 8; ++gg) s += red[gg][j];
        o[j] = s;
    }
}

// Layer 1: lane = output channel co; 3x3 window of the target (broadcast
// loads) in registers, per pixel 9 FMAs and the bias sum.
__global__ __launch_bounds__(256) void k_dw1(const float* __restrict__ target, const uint16_t* __restrict__ dy,
                                             int ny, int nx, int rows_per_block, float* __restrict__ part)
{
    constexpr int NO = 32 * 9 + 32;
    __shared__ float red[8][NO];
    const int co = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int seg = nx / 8;
    float a[9] = {};
    float ab = 0.0f;
    const int ybeg = blockIdx.x * rows_per_block;
    for (int y = ybeg; y < ybeg + rows_per_block && y < ny; ++y) {
        size_t rowo[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) rowo[r] = (size_t)((y + r - 1 + ny) & (ny - 1)) * nx;
        const int xs = g * seg;
        float wv[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            wv[r][0] = target[rowo[r] + ((xs - 1 + nx) & (nx - 1))];
            wv[r][1] = target[rowo[r] + xs];
        }
        for (int xi = xs; xi < xs + seg; ++xi) {
            const int xn = (xi + 1) & (nx - 1);
#pragma unroll
            for (int r = 0; r < 3; ++r) wv[r][2] = target[rowo[r] + xn];
            const float d = bf2f(dy[((size_t)y * nx + xi) * 32 + co]);
#pragma unroll
            for (int t = 0; t < 9; ++t) a[t] = fmaf(d, wv[t / 3][t % 3], a[t]);
            ab += d;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                wv[r][0] = wv[r][1];
                wv[r][1] = wv[r][2];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) red[g][co * 9 + t] = a[t];
    red[g][32 * 9 + co] = ab;
    __syncthreads();
    float* o = part + (size_t)blockIdx.x * NO;
    for (int j = threadIdx.x; j < NO; j += 256) {
        float s = red[0][j];
#pragma unroll
        for (int gg = 1; gg < 8; ++gg) s += red[gg][j];
        o[j] = s;
    }
}

// grad[j] (+)= scale * sum over blocks b of part[b][j] in a fixed order: thread (j, s)
// adds blocks s, s+4, s+8, ... (four loads in flight), then the four slices
// are added in slice order.  Block = 64 outputs x 4 slices.
// grad[j] (+)= scale * sum over blocks of part[b][j]: a block takes 16
// parameters and splits the partial rows over 16 slices (slice s sums rows
// s, s+16, ..., then the slices are added in order) -- a fixed order, so the
// gradient is the same run to run.
constexpr int kRedOut = 16, kRedSlices = 16;
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ part, int nblocks, int n,
                                                     float scale, int accumulate, float* __restrict__ grad)
{
    __shared__ float red[kRedSlices][kRedOut];
    const int jl = threadIdx.x % kRedOut, sl = threadIdx.x / kRedOut;
    const int j = blockIdx.x * kRedOut + jl;
    float s = 0.0f;
    if (j < n) {
        int b = sl;
        for (; b + 3 * kRedSlices < nblocks; b += 4 * kRedSlices) {
            const float v0 = part[(size_t)b * n + j], v1 = part[(size_t)(b + kRedSlices) * n + j];
            const float v2 = part[(size_t)(b + 2 * kRedSlices) * n + j];
            const float v3 = part[(size_t)(b + 3 * kRedSlices) * n + j];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; b < nblocks; b += kRedSlices) s += part[(size_t)b * n + j];
    }
    red[sl][jl] = s;
    __syncthreads();
    if (sl == 0 && j < n) {
        float g = red[0][jl];
        for (int q = 1; q < kRedSlices; ++q) g += red[q][jl];
        g *= scale;
        grad[j] = accumulate ? grad[j] + g : g;
    }
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
    const dim3 gmf((nx / 32) * ((ny + kConvRows - 1) / kConvRows));
    hipLaunchKernelGGL(k_conv1, dim3(g256), dim3(256), 0, s, target, ny, nx, b.params + b.off[0],
                       b.params + b.off[0] + 32 * 9, b.act[0]);
    for (int l = 1; l <= 3; ++l)
        hipLaunchKernelGGL(k_conv32<0>, gmf, dim3(256), 0, s, b.act[l - 1], ny, nx, b.wf[l - 1],
                           b.params + b.off[l] + 32 * 32 * 9, nullptr, b.act[l]);
    const int w5c = nx < 64 ? nx : 64, r5 = kC5Px / w5c < ny ? kC5Px / w5c : ny;   // k_conv5's tile
    hipLaunchKernelGGL(k_conv5, dim3((nx / w5c) * (ny / r5)), dim3(256), 0, s, b.act[3], ny, nx, b.w5,
                       b.params + b.off[4] + 2 * 32 * 9, b.o5, phasor);
    return hipGetLastError();
}

hipError_t cnn_launch_loss(const CnnBuffers& b, const float* target, const float2* label, const float2* phasor,
                           int n, int accumulate, double inv_batch, hipStream_t s)
{
    using namespace cnn;
    const int nb = 256;
    hipLaunchKernelGGL(k_loss_partial, dim3(nb), dim3(256), 0, s, phasor, label, target, n, b.loss_part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, b.loss_part, nb, b.zsum, accumulate, inv_batch);
    return hipGetLastError();
}

hipError_t cnn_launch_backward(const CnnBuffers& b, const float* target, const float2* label, int ny, int nx,
                               float scale, int accumulate, hipStream_t s)
{
    using namespace cnn;
    const int npx = nx * ny;
    const int g256 = (npx + 255) / 256;
    const dim3 gmf((nx / 32) * ((ny + kConvRows - 1) / kConvRows));
    const int rpb = b.rows_per_block;
    const int nblk = (ny + rpb - 1) / rpb;
    hipLaunchKernelGGL(k_loss_grad, dim3(g256), dim3(256), 0, s, b.o5, label, target, npx, b.zsum, b.d5);
    // layer 5
    hipLaunchKernelGGL(k_dw5, dim3(nblk), dim3(256), 0, s, b.act[3], b.d5, ny, nx, rpb, b.part);
    hipLaunchKernelGGL(k_grad_reduce, dim3((2 * 32 * 9 + 2 + kRedOut - 1) / kRedOut), dim3(256), 0, s, b.part,
                       nblk, 2 * 32 * 9 + 2, scale, accumulate, b.grad + b.off[4]);
    hipLaunchKernelGGL(k_conv5_bwd_data, dim3(g256), dim3(256), 0, s, b.d5, ny, nx, b.params + b.off[4], b.act[3],
                       b.dact[0]);
    // layers 4, 3, 2 (index l = 3, 2, 1): dW from act[l-1] and dY; dX through MFMA
    uint16_t* dcur = b.dact[0];
    uint16_t* dnext = b.dact[1];
    for (int l = 3; l >= 1; --l) {
        hipLaunchKernelGGL(k_dw32, dim3(nblk), dim3(192), 0, s, b.act[l - 1], dcur, ny, nx, rpb, b.part);
        hipLaunchKernelGGL(k_grad_reduce, dim3((32 * 32 * 9 + 32 + kRedOut - 1) / kRedOut), dim3(256), 0, s,
                           b.part, nblk, 32 * 32 * 9 + 32, scale, accumulate, b.grad + b.off[l]);
        hipLaunchKernelGGL(k_conv32<1>, gmf, dim3(256), 0, s, dcur, ny, nx, b.wt[l - 1], nullptr, b.act[l - 1],
                           dnext);
        uint16_t* tmp = dcur;
        dcur = dnext;
        dnext = tmp;
    }
    // layer 1
    hipLaunchKernelGGL(k_dw1, dim3(nblk), dim3(256), 0, s, target, dcur, ny, nx, rpb, b.part);
    hipLaunchKernelGGL(k_grad_reduce, dim3((32 * 9 + 32 + kRedOut - 1) / kRedOut), dim3(256), 0, s, b.part, nblk,
                       32 * 9 + 32, scale, accumulate, b.grad + b.off[0]);
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
    hipLaunchKernelGGL(k_pack5, dim3(1), dim3(256), 0, s, b.params + b.off[4], b.w5);
    return hipGetLastError();
}

}  // namespace holo

// fft_engine.hpp -- register/LDS Stockham FFT engine for gfx950 (wave64).
//
// Evaluates the 1D factors of the unitary DFT pair of Eq. (1)/(2) (without the
// 1/sqrt(N) scale, which callers fold in where it matters) along one axis of a
// 2D field.  A length-N transform (N = 2^k, 16 <= N <= 2048) is computed by
// T = N/16 cooperating threads that each hold P = 16 points in registers.
//
// Register layout: thread t holds element e = t + T*m in slot m (m < 16) at the
// start of every stage and after the last stage, so:
//   * the first stage reads straight from memory with lane-contiguous addresses
//     (coalesced along rows, or 16 columns at a time along columns);
//   * the last stage leaves results where the next pointwise step (binarise,
//     normalise, |.|^2, amplitude replacement) and a following transform of the
//     same axis expect them -- no shuffle between chained transforms;
//   * only the stage-to-stage exchange goes through LDS.
// Stages (Stockham autosort, natural order in and out): radix 16 as often as
// 16 divides the remaining length, then one radix-2/4/8 stage.  Stage with
// radix R after Ns points have been combined: butterfly j = t + b*T (b < 16/R)
// reads elements j + r*N/R, multiplies by W_{Ns*R}^{(j mod Ns)*r}, does an
// R-point DFT in registers, and writes element (j/Ns)*Ns*R + (j mod Ns) + r*Ns.
//
// Twiddles come from a table W_N^k = exp(-2*pi*i*k/N), k < N, generated once
// per length in FP64 on the device and rounded to FP32 (never by recurrence);
// the inverse direction uses its conjugate.  Radix-16 internal constants are
// the FP32 roundings of cos/sin(2*pi*k/16).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace holo {

constexpr int kP = 16;  // points per thread

template <int N>
struct ilog2 { static constexpr int v = 1 + ilog2<N / 2>::v; };
template <>
struct ilog2<1> { static constexpr int v = 0; };

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}

// cos/sin(2*pi*k/16), k = 0..4 (the rest follow by symmetry).
__device__ __forceinline__ float c16(int k)
{
    switch (k & 15) {
        case 0: return 1.0f;
        case 1: return 0.923879532511286756f;
        case 2: return 0.707106781186547524f;
        case 3: return 0.382683432365089772f;
        case 4: return 0.0f;
        case 5: return -0.382683432365089772f;
        case 6: return -0.707106781186547524f;
        case 7: return -0.923879532511286756f;
        case 8: return -1.0f;
        case 9: return -0.923879532511286756f;
        case 10: return -0.707106781186547524f;
        case 11: return -0.382683432365089772f;
        case 12: return 0.0f;
        case 13: return 0.382683432365089772f;
        case 14: return 0.707106781186547524f;
        default: return 0.923879532511286756f;
    }
}
__device__ __forceinline__ float s16(int k) { return c16(k - 4); }

// x * exp(SIGN * 2*pi*i*k/16) with k a compile-time constant after unrolling;
// exact cases (multiples of pi/2) avoid multiplications.
template <int SIGN>
__device__ __forceinline__ float2 rot16(float2 x, int k)
{
    k &= 15;
    if (k == 0) return x;
    if (k == 8) return make_float2(-x.x, -x.y);
    if (k == 4) return SIGN > 0 ? make_float2(-x.y, x.x) : make_float2(x.y, -x.x);
    if (k == 12) return SIGN > 0 ? make_float2(x.y, -x.x) : make_float2(-x.y, x.x);
    const float c = c16(k), s = SIGN > 0 ? s16(k) : -s16(k);
    if (k == 2 || k == 6 || k == 10 || k == 14) {
        // |c| == |s| == sqrt(1/2): (x.x*c - x.y*s, x.x*s + x.y*c) with one scale
        const float h = 0.707106781186547524f;
        float sc = c > 0 ? 1.0f : -1.0f, ss = s > 0 ? 1.0f : -1.0f;
        return make_float2(h * (sc * x.x - ss * x.y), h * (ss * x.x + sc * x.y));
    }
    return make_float2(fmaf(x.x, c, -x.y * s), fmaf(x.x, s, x.y * c));
}

// R-point DFT (R = 2, 4, 8, 16) of u[0..R) in registers, natural order in and
// out, kernel exp(SIGN*2*pi*i*q*r/R): radix-2 decimation in time.
template <int R, int SIGN>
__device__ __forceinline__ void dft_small(float2 (&u)[R])
{
    constexpr int LR = ilog2<R>::v;
    float2 a[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        int r = 0;
#pragma unroll
        for (int b = 0; b < LR; ++b) r |= ((i >> b) & 1) << (LR - 1 - b);
        a[r] = u[i];
    }
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int j = 0; j < half; ++j) {
#pragma unroll
            for (int i = 0; i < R; i += len) {
                float2 e = a[i + j];
                float2 o = rot16<SIGN>(a[i + j + half], j * (16 / len));
                a[i + j] = cadd(e, o);
                a[i + j + half] = csub(e, o);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) u[i] = a[i];
}

// Padded LDS element offset: one spare slot every 16 elements keeps the
// stride-16 writes of a radix-16 stage off a single bank group.
__device__ __forceinline__ int lds_pad(int e) { return e + (e >> 4); }
template <int N>
struct PadLen { static constexpr int v = N + N / 16; };
__host__ __device__ constexpr int pad_len(int n) { return n + n / 16; }
// The same with one spare slot every P elements, for engines with P points per
// thread (radix-P stages write at strides that are multiples of P).
template <int P>
__device__ __forceinline__ int lds_pad_p(int e) { return e + e / P; }
template <int N, int P>
struct PadLenP { static constexpr int v = N + N / P; };
// Threads per column-transform block: 512 keeps up to 256 VGPRs per lane for
// the two chained transforms; 2048-point columns need 1024 to hold 8 columns.
__host__ __device__ constexpr int col_bound(int n) { return n >= 2048 ? 1024 : 512; }

// u[r] *= W^(step*r) for r = 1..R-1 (conjugated for the inverse kernel),
// where W^k = tw[k] = exp(-2*pi*i*k/N).  Radix 16 reads W^s, W^2s, W^3s and
// W^4s, W^8s, W^12s and forms the other nine as W^4as * W^bs (one FP32 product
// of two correctly rounded table values); radix 8 reads four and forms three.
// Fewer table reads keep register pressure and vector-memory traffic low.
__host__ __device__ constexpr int tw_count(int R) { return R == 16 ? 6 : R == 8 ? 4 : R == 4 ? 3 : 1; }

// The tw_count(R) table values of one butterfly with twiddle step `step`:
// W^s, then W^2s, W^3s (radix >= 4), W^4s (radix >= 8), W^8s, W^12s (radix 16).
template <int R>
__device__ __forceinline__ void read_twiddles(float2* wl, const float2* __restrict__ tw, int step)
{
    wl[0] = tw[step];
    if (R >= 4) {
        wl[1] = tw[2 * step];
        wl[2] = tw[3 * step];
    }
    if (R >= 8) wl[3] = tw[4 * step];
    if (R == 16) {
        wl[4] = tw[8 * step];
        wl[5] = tw[12 * step];
    }
}

template <int R, int SIGN>
__device__ __forceinline__ void apply_read_twiddles(float2 (&u)[R], const float2* wl)
{
    auto mul = [](float2 x, float2 w) { return SIGN < 0 ? cmul(x, w) : cmulc(x, w); };
    if (R == 2) {
        u[1] = mul(u[1], wl[0]);
    } else if (R == 4) {
        u[1] = mul(u[1], wl[0]);
        u[2] = mul(u[2], wl[1]);
        u[3] = mul(u[3], wl[2]);
    } else if (R == 8) {
        u[1] = mul(u[1], wl[0]);
        u[2] = mul(u[2], wl[1]);
        u[3] = mul(u[3], wl[2]);
        u[4] = mul(u[4], wl[3]);
        u[5] = mul(u[5], cmul(wl[3], wl[0]));
        u[6] = mul(u[6], cmul(wl[3], wl[1]));
        u[7] = mul(u[7], cmul(wl[3], wl[2]));
    } else {
        const float2 wb[4] = {make_float2(1.0f, 0.0f), wl[0], wl[1], wl[2]};
        const float2 wa[4] = {make_float2(1.0f, 0.0f), wl[3], wl[4], wl[5]};
#pragma unroll
        for (int b = 1; b < 4; ++b) u[b] = mul(u[b], wb[b]);
#pragma unroll
        for (int a = 1; a < 4; ++a) {
            u[4 * a] = mul(u[4 * a], wa[a]);
#pragma unroll
            for (int b = 1; b < 4; ++b) u[4 * a + b] = mul(u[4 * a + b], cmul(wa[a], wb[b]));
        }
    }
}

template <int R, int SIGN>
__device__ __forceinline__ void apply_twiddles(float2 (&u)[R], const float2* __restrict__ tw, int step)
{
    float2 wl[tw_count(R)];
    read_twiddles<R>(wl, tw, step);
    apply_read_twiddles<R, SIGN>(u, wl);
}

// Stage shape of a length-N transform with P points per thread: radix-P
// stages while P divides the remaining length, then one radix 2^REM stage.
template <int N, int P>
struct StageShape {
    static constexpr int L = ilog2<N>::v;
    static constexpr int LP = ilog2<P>::v;
    static constexpr int NSP = L / LP;
    static constexpr int REM = L % LP;
    static constexpr int NSTAGE = NSP + (REM ? 1 : 0);
    static constexpr int radix(int s) { return s < NSP ? P : (1 << REM); }
    // table values a thread reads over stages 1..NSTAGE-1 (stage 0 has none)
    static constexpr int tw_total()
    {
        int c = 0;
        for (int s = 1; s < NSTAGE; ++s) c += (P / radix(s)) * tw_count(radix(s));
        return c;
    }
};

// The table twiddles of one thread's butterflies over a whole transform, read
// once and kept in registers, for threads that run several transforms of the
// same length and direction set (over sub-frames, or a forward transform and
// its inverse): those transforms then wait on no table reads.  The products
// formed from them are the ones the table path forms, so results are
// bit-identical to it.  The kernels use it at 8 points per thread and up to
// 1024 points: at 16 points per thread and at 2048 points this compiler keeps
// the array in scratch memory (the build test on every kernel's scratch size
// guards against that).
template <int N, int P>
struct TwRegs {
    using S = StageShape<N, P>;
    float2 w[S::tw_total() > 0 ? S::tw_total() : 1];
    __device__ __forceinline__ void read(const float2* __restrict__ tw, int t)
    {
        constexpr int T = N / P;
        int slot = 0, Ns = 1;
#pragma unroll
        for (int s = 0; s < S::NSTAGE; ++s) {
            const int R = S::radix(s);
            const int nb = P / R;
            if (s > 0) {
#pragma unroll
                for (int b = 0; b < nb; ++b) {
                    const int j = t + b * T;
                    const int step = (j & (Ns - 1)) * (N / (Ns * R));
                    float2* d = w + slot + b * tw_count(R);
                    if (R == 16) read_twiddles<16>(d, tw, step);
                    else if (R == 8) read_twiddles<8>(d, tw, step);
                    else if (R == 4) read_twiddles<4>(d, tw, step);
                    else read_twiddles<2>(d, tw, step);
                }
                slot += nb * tw_count(R);
            }
            Ns *= R;
        }
    }
};

// One radix-R stage on butterfly b of thread t (slots b + r*P/R).
// `pre`, when given, holds this butterfly's table values (TwRegs).
template <int N, int R, int SIGN, int P = kP>
__device__ __forceinline__ void stage_butterfly(float2 (&v)[P], int t, int b, int Ns,
                                                const float2* __restrict__ tw, const float2* pre = nullptr)
{
    constexpr int T = N / P;
    constexpr int nb = P / R;
    const int j = t + b * T;
    float2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[b + r * nb];
    if (Ns > 1) {
        if (pre) apply_read_twiddles<R, SIGN>(u, pre);
        else apply_twiddles<R, SIGN>(u, tw, (j & (Ns - 1)) * (N / (Ns * R)));
    }
    dft_small<R, SIGN>(u);
#pragma unroll
    for (int r = 0; r < R; ++r) v[b + r * nb] = u[r];
}

// One transform of length N on T = N/16 threads.  `v` holds slot m = element
// t + T*m on entry and on exit.  LDS addressing is abstracted by `addr(e)` so
// row (one transform per LDS row) and column (C interleaved transforms) layouts
// share the engine.  `tw` is the FP32 table W_N^k; SIGN = -1 for Eq. (1),
// +1 for Eq. (2).  Contains __syncthreads(): every thread of the block must
// call it the same number of times.
// Synchronisation of an LDS exchange.  When every transform lives inside one
// wave (T <= 64 threads, aligned groups), the exchange is private to the wave:
// a wave's LDS operations execute in order, so only the compiler must be kept
// from moving them, and waves of a block stay free to run different phases.
// Otherwise the block barrier is needed.
template <bool WAVE_LOCAL>
__device__ __forceinline__ void exchange_sync()
{
    if (WAVE_LOCAL) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// `pre` (optional): the thread's table twiddles read by TwRegs<N, P>::read.
template <int N, int SIGN, typename Addr, bool WAVE_LOCAL = false, int P = kP>
__device__ __forceinline__ void fft_stages(float2 (&v)[P], int t, float2* lds, Addr addr,
                                           const float2* __restrict__ tw, const float2* pre = nullptr)
{
    static_assert(P == 4 || P == 8 || P == 16, "points per thread");
    constexpr int T = N / P;
    constexpr int NSP = StageShape<N, P>::NSP;        // radix-P stages
    constexpr int REM = StageShape<N, P>::REM;        // bits left for the last small stage
    constexpr int NSTAGE = StageShape<N, P>::NSTAGE;
    auto pad = [](int e) { return P == 16 ? lds_pad(e) : lds_pad_p<P>(e); };
    int Ns = 1, slot = 0;
#pragma unroll
    for (int s = 0; s < NSTAGE; ++s) {
        const bool last = (s == NSTAGE - 1);
        const int R = (s < NSP) ? P : (1 << REM);
        const int nb = P / R;
#pragma unroll
        for (int b = 0; b < nb; ++b) {
            const float2* pb = (pre && s > 0) ? pre + slot + b * tw_count(R) : nullptr;
            if (R == 16) stage_butterfly<N, 16, SIGN, P>(v, t, b, Ns, tw, pb);
            else if (R == 8) stage_butterfly<N, 8, SIGN, P>(v, t, b, Ns, tw, pb);
            else if (R == 4) stage_butterfly<N, 4, SIGN, P>(v, t, b, Ns, tw, pb);
            else stage_butterfly<N, 2, SIGN, P>(v, t, b, Ns, tw, pb);
        }
        if (s > 0) slot += nb * tw_count(R);
        if (!last) {
            // exchange: write outputs at their Stockham positions, read back the
            // t + T*m set for the next stage.  Addresses are padded indices
            // p = e + e/P.  Radix-P stages run first, so Ns is 1 or a multiple
            // of P here and element base + r*Ns pads to pad(base) + r*ps with a
            // compile-time ps; likewise t + T*m pads to pad(t) + m*T*(P+1)/P when
            // P divides T.  The addr functor gets padded indices.
            const int ps = Ns == 1 ? 1 : (Ns / P) * (P + 1);
#pragma unroll
            for (int b = 0; b < nb; ++b) {
                const int j = t + b * T;
                const int pb = pad((j / Ns) * Ns * R + (j & (Ns - 1)));
#pragma unroll
                for (int r = 0; r < R; ++r) lds[addr(pb + r * ps)] = v[b + r * nb];
            }
            exchange_sync<WAVE_LOCAL>();
            if (T % P == 0) {
                const int pt = pad(t);
#pragma unroll
                for (int m = 0; m < P; ++m) v[m] = lds[addr(pt + m * (T / P) * (P + 1))];
            } else {
#pragma unroll
                for (int m = 0; m < P; ++m) v[m] = lds[addr(pad(t + T * m))];
            }
            exchange_sync<WAVE_LOCAL>();
        }
        Ns *= R;
    }
}

// Deterministic sums: butterfly (xor) reduction inside aligned segments of
// `seg` lanes (seg a power of two <= 64); every lane of a segment ends with
// the segment total, added in the same order on every run.
__device__ __forceinline__ double seg_sum(double v, int seg)
{
    for (int off = seg >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum of NV doubles per thread, fixed order: per-wave butterflies,
// then wave totals added in wave order by thread 0 (result valid there).
// `red` needs NV * (blockDim.x / 64 + 1) doubles of LDS.
template <int NV>
__device__ __forceinline__ void block_sum(double (&a)[NV], double* red, double (&out)[NV])
{
    const int n = blockDim.x;
    const int seg = n < 64 ? n : 64;
    const int nw = (n + 63) / 64;
#pragma unroll
    for (int i = 0; i < NV; ++i) a[i] = seg_sum(a[i], seg);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        for (int i = 0; i < NV; ++i) red[(threadIdx.x >> 6) * NV + i] = a[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i < NV; ++i) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[w * NV + i];
            out[i] = s;
        }
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b mod 8), each with its own L2.  This maps the blocks of one XCD onto a
// contiguous range of logical tiles so neighbouring column tiles, which share
// 128-byte lines, meet in the same L2.  A permutation of [0, nblocks).
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    if (nblocks & 7) return b;
    return (b & 7) * (nblocks >> 3) + (b >> 3);
}

// Load / store at a wave-uniform base pointer plus a 32-bit per-lane byte
// offset, so the compiler can use the scalar-base addressing form and keep one
// offset register for a whole set of strided accesses.
template <typename V>
__device__ __forceinline__ V ld_off(const V* base, uint32_t boff)
{
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename V>
__device__ __forceinline__ void st_off(V* base, uint32_t boff, V v)
{
    *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + boff) = v;
}

// LDS addressing for R_ROWS independent row transforms of length N, one per
// padded LDS row.
// (Both take the padded element index p = e + e/16.)
template <int N>
struct RowAddr {
    int row;
    __device__ __forceinline__ int operator()(int p) const { return row * PadLen<N>::v + p; }
};
// LDS addressing for C interleaved column transforms: element e of column c.
template <int C>
struct ColAddr {
    int c;
    __device__ __forceinline__ int operator()(int p) const { return p * C + c; }
};

// Raw buffer access: a descriptor over `bytes` bytes from a wave-uniform base
// (hardware range-checked: loads past the end read 0, stores are dropped),
// a per-lane byte offset and a wave-uniform byte offset, so a strided set of
// accesses needs one offset register and scalar increments.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float2 buf_ld2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float2 x)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, x), r, voff, soff, 0);
}
__device__ __forceinline__ float buf_ld1(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// 16-byte stores take their whole offset in the lane register and a zero
// scalar offset.  A buffer store of more than 8 bytes per lane may read its
// data registers after the next vector instruction has overwritten them; the
// compiler inserts the wait for the form without a scalar-register offset, and
// on gfx950 the form with one (which it leaves unguarded) was seen to lose
// data words (lanes 12..15 of a 16-lane group, now and then).
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 buf_ld4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st4z(__amdgpu_buffer_rsrc_t r, uint32_t voff, float4 x)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, x), r, voff, 0u, 0);
}

}  // namespace holo

// mfma_dft.hpp -- radix-16 DFTs of the register FFT engine on gfx950 matrix
// cores (BF16 or FP16 operands, FP32 accumulation).
//
// The transform is fft_stages of fft_engine.hpp -- same slot contract (thread
// t of a length-N transform holds element t + T*m in slot m on entry and on
// exit, T = N/16), same Stockham factorisation (radix 16 while 16 divides,
// then one radix-2/4/8 stage), same FP32 inter-stage twiddles and LDS
// exchanges -- with one change: the 16-point DFT of each radix-16 butterfly is
// a DFT-matrix product on the matrix cores instead of butterflies on the
// vector ALUs.  A wave's 64 threads are 64 vectors of 16 points; per group of
// 32 vectors v_mfma_f32_32x32x16_{bf16,f16} computes
//
//   D = W^T X^T,  W[r][q] = exp(SIGN*2*pi*i*r*q/16) * sc,
//
// as real products (Re X and Im X against the real and imaginary parts of the
// coefficients), the 32 rows of D being the real and imaginary part of each
// output in turn.  W is split W = W_hi + W_lo (W_hi = rn(W), W_lo = rn(W -
// W_hi) in the operand format, from FP64 values generated on the device), so
// each product is X*W_hi + X*W_lo accumulated in FP32: four MFMAs per 32
// vectors.  The data are rounded to the operand format once per radix-16
// stage (after the FP32 twiddle); the last radix-2/4/8 stage stays FP32.  For
// FP16, sc = 1/16 keeps the data of chained stages in range and is undone
// exactly (x 16^s) after the transform; BF16 has FP32's exponent range and
// sc = 1.  The data stay in registers through the matrix products: operands
// are matched to the threads' own vectors with half-wave lane swaps, and the
// results either go straight to the following LDS exchange or are swapped back
// (after the last stage) -- see fft_stages_mc.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_engine.hpp"

namespace holo {

typedef float mf32x16 __attribute__((ext_vector_type(16)));

template <int PREC>
struct MfmaOp;

// BF16 operands (8 significant bits).
template <>
struct MfmaOp<1> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    // two values rounded to nearest even, the first in bits 0..15, in one
    // instruction (the conversion written out in C++ compiles to two
    // conversions and a merge, or, through a vector conversion, to stack
    // temporaries)
    static __device__ __forceinline__ uint32_t pack(float a, float b)
    {
        uint32_t r;
        asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
        return r;
    }
    static __device__ __forceinline__ mf32x16 mma(v8 a, v8 b, mf32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// FP16 operands (11 significant bits).
template <>
struct MfmaOp<2> {
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    static __device__ __forceinline__ uint32_t pack(float a, float b)
    {
        uint32_t r;
        asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
        return r;
    }
    static __device__ __forceinline__ mf32x16 mma(v8 a, v8 b, mf32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// DFT-matrix operands, generated once per device in FP64 (launch_dft_operand_gen):
// for sign (0: -, 1: +) and part (Re-coefficient hi, lo; Im-coefficient hi,
// lo), lane l holds 8 operand-format values as one 16-byte word: uint4 index
// (si*4 + part)*64 + l.  Row o = l & 31 of W^T is output o >> 1, real part
// (o even) or imaginary part (o odd); column k = 8*(l >> 5) + e is input
// point k.

// Scalar reinterpretation by value.  (Reinterpreting an element of an
// ext_vector value in place with __builtin_bit_cast reads element 0 whatever
// the index, with this compiler, so elements are copied out first.)
__device__ __forceinline__ uint32_t f2u(float f) { return __builtin_bit_cast(uint32_t, f); }
__device__ __forceinline__ float u2f(uint32_t u) { return __builtin_bit_cast(float, u); }

// Register reinterpretation of a whole vector (same size), by value.
template <typename To, typename From>
__device__ __forceinline__ To vcast(From x)
{
    static_assert(sizeof(To) == sizeof(From), "same size");
    return __builtin_bit_cast(To, x);
}

// v_permlane32_swap of (a, b): lanes 32..63 of a trade places with lanes 0..31
// of b (lanes 0..31 of a and 32..63 of b stay).
__device__ __forceinline__ void swap_halves(uint32_t& a, uint32_t& b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}

// The 16-point DFTs of one radix-16 stage for the wave's 64 vectors (u: the
// calling thread's own vector, natural order, twiddled).  Returns g0 for group
// 0 (vectors of lanes 0..31) and g1 for group 1 (lanes 32..63): lane l,
// register r of g_g is row i = 8*(r/4) + 4*h + (r%4) (h = l/32) of
// D for the vector of lane 32*g + l%32, i.e. output i/2, real part for even
// i, imaginary for odd (scaled by 1/16 for FP16).
struct Acc2 {
    mf32x16 g0, g1;
};
template <int SIGN, int PREC>
__device__ __forceinline__ Acc2 mma16(const float2 (&u)[16], const uint4* __restrict__ dftop)
{
    using M = MfmaOp<PREC>;
    typedef typename M::v8 V;
    // DFT-matrix operand (the table layout above, radix 16): Re-coefficient
    // hi, lo; Im-coefficient hi, lo
    const uint4* op = dftop + ((SIGN > 0 ? 1 : 0) * 4) * 64 + (threadIdx.x & 63);
    const V a0 = vcast<V>(op[0]), a1 = vcast<V>(op[64]), a2 = vcast<V>(op[128]), a3 = vcast<V>(op[192]);
    // the lane's points in the operand format, two per register (point 2d in
    // the low half), then halves traded with lane l ^ 32: afterwards lane l
    // holds points 8h..8h+7 of the vector of lane l%32 (r0, i0) and of lane
    // 32 + l%32 (r1, i1), the B-operand layout of the two groups
    uint32_t r0[4], r1[4], i0[4], i1[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        r0[d] = M::pack(u[2 * d].x, u[2 * d + 1].x);
        i0[d] = M::pack(u[2 * d].y, u[2 * d + 1].y);
        r1[d] = M::pack(u[8 + 2 * d].x, u[9 + 2 * d].x);
        i1[d] = M::pack(u[8 + 2 * d].y, u[9 + 2 * d].y);
        swap_halves(r0[d], r1[d]);
        swap_halves(i0[d], i1[d]);
    }
    const V b0r = vcast<V>(u32x4_t{r0[0], r0[1], r0[2], r0[3]});
    const V b0i = vcast<V>(u32x4_t{i0[0], i0[1], i0[2], i0[3]});
    const V b1r = vcast<V>(u32x4_t{r1[0], r1[1], r1[2], r1[3]});
    const V b1i = vcast<V>(u32x4_t{i1[0], i1[1], i1[2], i1[3]});
    mf32x16 acc0 = {}, acc1 = {};
    acc0 = M::mma(a0, b0r, acc0);
    acc1 = M::mma(a0, b1r, acc1);
    acc0 = M::mma(a1, b0r, acc0);
    acc1 = M::mma(a1, b1r, acc1);
    acc0 = M::mma(a2, b0i, acc0);
    acc1 = M::mma(a2, b1i, acc1);
    acc0 = M::mma(a3, b0i, acc0);
    acc1 = M::mma(a3, b1i, acc1);
    return Acc2{acc0, acc1};
}

// Results back to the calling thread's own vector (outputs 0..15 in u): the
// rows of lanes 32..63 in acc0 and of lanes 0..31 in acc1 trade places.
__device__ __forceinline__ void acc_to_own(mf32x16 acc0, mf32x16 acc1, float2 (&u)[16])
{
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int k = 4 * (p >> 1) + (p & 1);
        uint32_t x0 = f2u(acc0[2 * p]), x1 = f2u(acc1[2 * p]);
        uint32_t y0 = f2u(acc0[2 * p + 1]), y1 = f2u(acc1[2 * p + 1]);
        swap_halves(x0, x1);
        swap_halves(y0, y1);
        u[k] = make_float2(u2f(x0), u2f(y0));
        u[k + 2] = make_float2(u2f(x1), u2f(y1));
    }
}

// Transform with the radix-16 DFTs on the matrix cores (PREC 1 = BF16,
// 2 = FP16).  Same contract, factorisation, twiddles and LDS layout as
// fft_stages of the register engine; `addr` must be affine in the padded
// index (addr(p) = addr(0) + p * stride, as the row and column layouts are).
// A radix-16 stage followed by an exchange writes each lane's result rows
// straight to their Stockham positions -- lane l holds outputs 2h, 2h+1,
// 4+2h, .. of two vectors (lanes l%32 and 32 + l%32), whose LDS bases one
// lane swap provides -- instead of first trading them back to their owners.
// The last radix-2/4/8 stage runs in FP32 on the vector ALUs.  Every lane of
// each wave must take part; the block synchronises as fft_stages does.
template <int N, int SIGN, int PREC, typename Addr, bool WAVE_LOCAL = false>
__device__ __forceinline__ void fft_stages_mc(float2 (&v)[kP], int t, float2* lds, Addr addr,
                                              const float2* __restrict__ tw, const uint4* __restrict__ dftop)
{
    constexpr int P = kP;
    constexpr int T = N / P;
    constexpr int L = ilog2<N>::v;
    constexpr int NSP = L / 4;           // radix-16 stages
    constexpr int REM = L % 4;           // bits left for the last small stage
    constexpr int NSTAGE = NSP + (REM ? 1 : 0);
    const int h = (threadIdx.x >> 5) & 1;
    const int stride = addr(1) - addr(0);
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < NSTAGE; ++s) {
        const bool last = (s == NSTAGE - 1);
        if (s < NSP) {
            if (Ns > 1) apply_twiddles<16, SIGN>(v, tw, (t & (Ns - 1)) * (N / (Ns * 16)));
            const Acc2 acc = mma16<SIGN, PREC>(v, dftop);
            const mf32x16 acc0 = acc.g0, acc1 = acc.g1;
            if (last) {
                acc_to_own(acc0, acc1, v);
            } else {
                // output o of the vector of lane w goes to padded index
                // pb(w) + o * ps; this lane holds o = 4q + 2h + b (q < 4, b < 2)
                const int ps = Ns == 1 ? 1 : (Ns / P) * (P + 1);
                uint32_t b0 = (uint32_t)addr(lds_pad((t / Ns) * Ns * P + (t & (Ns - 1))));
                uint32_t b1 = b0;
                swap_halves(b0, b1);   // b0: base of lane l%32's vector, b1: of lane 32 + l%32
                const int off = 2 * h * ps * stride;
                float2* l0 = lds + (int)b0 + off;
                float2* l1 = lds + (int)b1 + off;
                // one group after the other, so that neighbouring outputs of a
                // vector pair into two-address LDS writes
#pragma unroll
                for (int p = 0; p < 8; ++p)
                    l0[(4 * (p >> 1) + (p & 1)) * ps * stride] = make_float2(acc0[2 * p], acc0[2 * p + 1]);
#pragma unroll
                for (int p = 0; p < 8; ++p)
                    l1[(4 * (p >> 1) + (p & 1)) * ps * stride] = make_float2(acc1[2 * p], acc1[2 * p + 1]);
                exchange_sync<WAVE_LOCAL>();
                if (T % P == 0) {
                    const int pt = lds_pad(t);
#pragma unroll
                    for (int m = 0; m < P; ++m) v[m] = lds[addr(pt + m * (T / P) * (P + 1))];
                } else {
#pragma unroll
                    for (int m = 0; m < P; ++m) v[m] = lds[addr(lds_pad(t + T * m))];
                }
                exchange_sync<WAVE_LOCAL>();
            }
            Ns *= 16;
        } else {
            constexpr int R = 1 << (REM ? REM : 1);
#pragma unroll
            for (int b = 0; b < P / R; ++b) stage_butterfly<N, R, SIGN, P>(v, t, b, Ns, tw);
            Ns *= R;
        }
    }
    if constexpr (PREC == 2) {
        // undo the 1/16 of every FP16 radix-16 stage (exact)
        constexpr float sc = (float)(1 << (4 * NSP));
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = make_float2(v[m].x * sc, v[m].y * sc);
    }
}

// One transform through the FP32 register engine (PREC 0, PT = 4, 8 or 16
// points per thread) or with its radix-16 DFTs on the matrix cores (PREC 1 =
// BF16, 2 = FP16, PT = 16; the inter-stage twiddles and the last radix-2/4/8
// stage stay FP32 on the vector ALUs).  `addr` is the calling thread's LDS
// addressing (padded as the engine with PT points per thread pads).  With
// PREC > 0 every lane of each wave must take part (blocks of whole waves, no
// divergence around the call).  `pre` (FP32 only, optional): the thread's
// table twiddles from TwRegs<N, PT>::read.
template <int N, int SIGN, int PREC, bool WAVE_LOCAL = false, int PT = kP, typename Addr>
__device__ __forceinline__ void fft_any(float2 (&v)[PT], int t, float2* lds, Addr addr,
                                        const float2* __restrict__ tw, const uint4* __restrict__ dftop,
                                        const float2* pre = nullptr)
{
    if constexpr (PREC == 0) {
        fft_stages<N, SIGN, Addr, WAVE_LOCAL, PT>(v, t, lds, addr, tw, pre);
    } else {
        static_assert(PT == kP, "the matrix-core transforms take 16 points per thread");
        fft_stages_mc<N, SIGN, PREC, Addr, WAVE_LOCAL>(v, t, lds, addr, tw, dftop);
    }
}

}  // namespace holo

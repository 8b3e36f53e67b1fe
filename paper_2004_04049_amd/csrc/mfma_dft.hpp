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
//   D = W^T X^T,  W[r][q] = exp(SIGN*2*pi*i*r*q/16) / 16,
//
// as real products (Re X and Im X against the real and imaginary parts of the
// coefficients), the 32 rows of D being the real and imaginary part of each
// output in turn.  W is split W = W_hi + W_lo (W_hi = rn(W), W_lo = rn(W -
// W_hi) in the operand format, from FP64 values generated on the device), so
// each product is X*W_hi + X*W_lo accumulated in FP32: four MFMAs per 32
// vectors.  The data are rounded to the operand format once per radix-16
// stage (after the FP32 twiddle); the last radix-2/4/8 stage stays FP32.  The
// 1/16 per stage keeps FP16 operands in range and is undone exactly (x 16^s)
// after the transform.  The data stay in registers: operand and result layouts
// are matched to the threads' own vectors with lane swaps (below).
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
    // two values rounded to nearest even, the first in bits 0..15
    static __device__ __forceinline__ uint32_t pack(float a, float b)
    {
        const __bf16 x = (__bf16)a, y = (__bf16)b;
        return (uint32_t)__builtin_bit_cast(uint16_t, x) | ((uint32_t)__builtin_bit_cast(uint16_t, y) << 16);
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
        const _Float16 x = (_Float16)a, y = (_Float16)b;
        return (uint32_t)__builtin_bit_cast(uint16_t, x) | ((uint32_t)__builtin_bit_cast(uint16_t, y) << 16);
    }
    static __device__ __forceinline__ mf32x16 mma(v8 a, v8 b, mf32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// DFT-matrix operands, generated once per device in FP64 (launch_dft_operand_gen):
// for radix R in {2, 4, 8, 16} (index log2(R) - 1), sign (0: -, 1: +) and part
// (Re-coefficient hi, lo; Im-coefficient hi, lo), lane l holds 8 operand-format
// values as one 16-byte word: uint4 index ((ri*2 + si)*4 + part)*64 + l.
// Row o = l & 31 of W^T is output o >> 1, real part (o even) or imaginary
// part (o odd); column k = 8*(l >> 5) + e is input point k.
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
    To r;
    __builtin_memcpy(&r, &x, sizeof(To));
    return r;
}

// v_permlane32_swap of (a, b): lanes 32..63 of a trade places with lanes 0..31
// of b (lanes 0..31 of a and 32..63 of b stay).
__device__ __forceinline__ void swap_halves(uint32_t& a, uint32_t& b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}

template <int SIGN, int PREC>
struct Dft16Mfma {
    typedef typename MfmaOp<PREC>::v8 V;
    const uint4* dftop;   // operand table (the W_16/16 operand is read per call: 4 KiB, cache-resident)
    __device__ __forceinline__ void operator()(float2 (&u)[16]) const
    {
        using M = MfmaOp<PREC>;
        // DFT-matrix operand (the table layout above, radix 16): Re-coefficient
        // hi, lo; Im-coefficient hi, lo
        const uint4* op = dftop + ((3 * 2 + (SIGN > 0 ? 1 : 0)) * 4) * 64 + (threadIdx.x & 63);
        const V a0 = vcast<V>(op[0]), a1 = vcast<V>(op[64]), a2 = vcast<V>(op[128]), a3 = vcast<V>(op[192]);
        // the lane's points in the operand format, two per register (point 2d
        // in the low half), then halves traded with lane l ^ 32
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
        acc0 = M::mma(a1, b0r, acc0);
        acc0 = M::mma(a2, b0i, acc0);
        acc0 = M::mma(a3, b0i, acc0);
        acc1 = M::mma(a0, b1r, acc1);
        acc1 = M::mma(a1, b1r, acc1);
        acc1 = M::mma(a2, b1i, acc1);
        acc1 = M::mma(a3, b1i, acc1);
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
};

// One transform through the FP32 register engine (PREC 0) or with its radix-16
// DFTs on the matrix cores (PREC 1 = BF16, 2 = FP16; the inter-stage twiddles
// and the last radix-2/4/8 stage stay FP32 on the vector ALUs).  `addr` is the
// calling thread's LDS addressing.  With PREC > 0 every lane of each wave must
// take part (blocks of whole waves, no divergence around the call).
template <int N, int SIGN, int PREC, bool WAVE_LOCAL = false, typename Addr>
__device__ __forceinline__ void fft_any(float2 (&v)[kP], int t, float2* lds, Addr addr,
                                        const float2* __restrict__ tw, const uint4* __restrict__ dftop)
{
    if constexpr (PREC == 0) {
        fft_stages<N, SIGN, Addr, WAVE_LOCAL>(v, t, lds, addr, tw);
    } else {
        const Dft16Mfma<SIGN, PREC> d16{dftop};
        fft_stages<N, SIGN, Addr, WAVE_LOCAL, kP, Dft16Mfma<SIGN, PREC>>(v, t, lds, addr, tw, d16);
        // undo the 1/16 of every radix-16 stage (exact)
        constexpr float sc = (float)(1 << (4 * (ilog2<N>::v / 4)));
#pragma unroll
        for (int m = 0; m < kP; ++m) v[m] = make_float2(v[m].x * sc, v[m].y * sc);
    }
}

}  // namespace holo

// mfma_dft.hpp -- DFT stages as small DFT-matrix products on gfx950 matrix
// cores (BF16 or FP16 operands, FP32 accumulation).
//
// Same contract as fft_stages in fft_engine.hpp (thread t of a length-N
// transform holds element t + T*m in slot m on entry and on exit, T = N/16),
// same Stockham factorisation (radix 16 while 16 divides, then one radix
// 2/4/8 stage), same inter-stage twiddles W_{Ns*R}^{(j mod Ns)*r} from the
// FP32 table, applied on the vector ALUs in FP32.  What changes is the R-point
// DFT itself: the T threads' butterfly sets ("vectors" of 16 points, 16/R
// butterflies of R points) are taken 32 at a time as one operand of
// v_mfma_f32_32x32x16_{bf16,f16}, with the DFT matrix as the other:
//
//   Y[v][k'] = sum_k X[v][k] W[k][k'],  W = blockdiag(W_R, ..., W_R) (16x16),
//   W_R[r][q] = exp(SIGN*2*pi*i*r*q/R) / R,
//
// as two real products per K block (Re X and Im X against [[Re W, Im W],
// [-Im W, Re W]]), 32 output columns = 16 real parts then 16 imaginary
// parts.  W is split W = W_hi + W_lo (W_hi = rn(W), W_lo = rn(W - W_hi) in the
// operand format, from FP64 values generated on the device), so each product
// is X*W_hi + X*W_lo accumulated in FP32:
// four MFMAs per 32 vectors.  The data are rounded to the operand format once
// per stage (after the FP32 twiddle).  The 1/R per stage keeps FP16 operands
// in range and is undone exactly (x N, a power of two) on exit.
//
// Stages run LDS -> registers -> MFMA -> LDS; the engine writes the slot data
// to LDS on entry and reads it back on exit.  Every lane of the block takes
// part (blockDim a multiple of 64; a wave's 64 threads are its 64 vectors).
#pragma once
#include <hip/hip_runtime.h>

#include "fft_engine.hpp"

namespace holo {

typedef float mf32x16 __attribute__((ext_vector_type(16)));
typedef float mf32x8 __attribute__((ext_vector_type(8)));

template <int PREC>
struct MfmaOp;

// BF16 operands (8 significant bits).
template <>
struct MfmaOp<1> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    static __device__ __forceinline__ v8 cvt(mf32x8 x) { return __builtin_convertvector(x, v8); }
    static __device__ __forceinline__ mf32x16 mma(v8 a, v8 b, mf32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// FP16 operands (11 significant bits).
template <>
struct MfmaOp<2> {
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    static __device__ __forceinline__ v8 cvt(mf32x8 x) { return __builtin_convertvector(x, v8); }
    static __device__ __forceinline__ mf32x16 mma(v8 a, v8 b, mf32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// Thread layouts of the kernels, as seen by the engine: slot index t of block
// thread `tid`, and the LDS element (float2) index of padded position p of
// that thread's transform, base(tid) + p * S.
template <int N>
struct RowsOf {   // one transform per T consecutive threads, one padded LDS row each
    static constexpr int T = N / kP;
    static constexpr int S = 1;
    __device__ __forceinline__ int t(int tid) const { return tid & (T - 1); }
    __device__ __forceinline__ int base(int tid) const { return (tid / T) * PadLen<N>::v; }
};
template <int N, int C>
struct ColsOf {   // C interleaved transforms: thread (c, t) = c + C*t
    static constexpr int S = C;
    __device__ __forceinline__ int t(int tid) const { return tid / C; }
    __device__ __forceinline__ int base(int tid) const { return tid & (C - 1); }
};

// DFT-matrix operands, generated once per device in FP64 (launch_dft_operand_gen):
// for radix R in {2, 4, 8, 16} (index log2(R) - 1), sign (0: -, 1: +) and part
// (Re-coefficient hi, lo; Im-coefficient hi, lo), lane l holds 8 operand-format
// values as one 16-byte word: uint4 index ((ri*2 + si)*4 + part)*64 + l.
// Row o = l & 31 of W^T is output o >> 1, real part (o even) or imaginary
// part (o odd); column k = 8*(l >> 5) + e is input point k.
template <int PREC, int R, int SIGN>
__device__ __forceinline__ void load_operand(const uint4* __restrict__ op, int lane, typename MfmaOp<PREC>::v8 (&a)[4])
{
    constexpr int ri = R == 16 ? 3 : R == 8 ? 2 : R == 4 ? 1 : 0;
    const uint4* p = op + ((ri * 2 + (SIGN > 0 ? 1 : 0)) * 4) * 64 + lane;
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = __builtin_bit_cast(typename MfmaOp<PREC>::v8, p[q * 64]);
}

// The DFT-matrix product runs transposed, D = W^T X^T: the A operand holds
// the 32 output rows of W^T (real and imaginary part of each output, in
// turn), the B operand 32 vectors (lane l32 of each half-wave holds points
// 8*half..+7 of vector l32), and registers 2p, 2p+1 of the result hold, for
// the lane's vector, the real and imaginary part of output
// 4*(p>>1) + 2*half + (p&1).  So every LDS access of a lane is a per-lane base
// plus a compile-time offset, and outputs leave as complex pairs straight from
// adjacent accumulator registers.  The
// padded positions (one spare slot per 16, as in the register engine) keep
// the strided accesses on distinct banks; T = N/16 is a multiple of 16, so
// pad(x + 16m) = pad(x) + 17m splits every address that way.
template <int N, int SIGN, int PREC, typename Lay, bool WAVE_LOCAL = false>
__device__ __forceinline__ void fft_stages_mfma(float2 (&v)[kP], float2* lds, const Lay& lay,
                                                const float2* __restrict__ tw, const uint4* __restrict__ dftop)
{
    using M = MfmaOp<PREC>;
    constexpr int T = N / kP;
    static_assert(T % 16 == 0, "matrix-core stages need N >= 256");
    constexpr int T17 = T / 16 * 17;
    constexpr int L = ilog2<N>::v;
    constexpr int NS16 = L / 4;
    constexpr int REM = L % 4;
    constexpr int NSTAGE = NS16 + (REM ? 1 : 0);
    constexpr int S = Lay::S;
    const int tid = threadIdx.x;
    const int lane = tid & 63, half = lane >> 5, l32 = lane & 31;
    const int wbase = tid - lane;
    const auto rtw = make_rsrc(tw, (uint32_t)(N * sizeof(float2)));

    {
        const int b = lay.base(tid) + lds_pad(lay.t(tid)) * S;
#pragma unroll
        for (int m = 0; m < kP; ++m) lds[b + m * T17 * S] = v[m];
    }
    exchange_sync<WAVE_LOCAL>();

    int tt[2], bs[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int vt = wbase + 32 * g + l32;
        tt[g] = lay.t(vt);
        bs[g] = lay.base(vt);
    }
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < NSTAGE; ++s) {
        const int R = (s < NS16) ? 16 : (1 << REM);
        // B operands: points k = 8*half + e of the wave's 64 vectors, FP32
        // twiddle W_{Ns R}^{(j mod Ns) r} first (butterfly j = tt + b*T reads
        // element j + r*N/R)
        typename M::v8 xr[2], xi[2];
        mf32x8 fr, fi;
        const int bh = R == 16 ? 0 : 8 * half / R;   // butterfly offset of this half
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int lb = bs[g] + (lds_pad(tt[g]) + (R == 16 ? 8 * half * T17 : bh * T17)) * S;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int off = R == 16 ? e * T17 : ((e / R) * T + (e % R) * (N / R)) / 16 * 17;
                float2 x = lds[lb + off * S];
                if (Ns > 1) {
                    const int r = R == 16 ? 8 * half + e : e % R;
                    const int j = tt[g] + (bh + (R == 16 ? 0 : e / R)) * T;
                    const float2 w = buf_ld2(rtw, (uint32_t)((j & (Ns - 1)) * (N / (Ns * R)) * r) * 8u, 0);
                    x = SIGN < 0 ? cmul(x, w) : cmulc(x, w);
                }
                fr[e] = x.x;
                fi[e] = x.y;
            }
            xr[g] = M::cvt(fr);
            xi[g] = M::cvt(fi);
        }
        exchange_sync<WAVE_LOCAL>();
        typename M::v8 a[4];
        if (R == 16) load_operand<PREC, 16, SIGN>(dftop, lane, a);
        else load_operand<PREC, (1 << (REM ? REM : 1)), SIGN>(dftop, lane, a);
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            mf32x16 acc = {};
            acc = M::mma(a[0], xr[g], acc);
            acc = M::mma(a[1], xr[g], acc);
            acc = M::mma(a[2], xi[g], acc);
            acc = M::mma(a[3], xi[g], acc);
            // output ko = 4*(p>>1) + 2*half + (p&1) of butterfly j = tt + (ko/R)*T
            // goes to Stockham position (j/Ns)*Ns*R + (j mod Ns) + (ko mod R)*Ns
            int sb;
            if (Ns == 1) {   // first stage, R = 16: 16*tt + ko, padded 17*tt + ko
                sb = bs[g] + (17 * tt[g] + 2 * half) * S;
            } else if (R == 16) {
                const int j = tt[g];
                sb = bs[g] + (lds_pad((j / Ns) * 16 * Ns + (j & (Ns - 1))) + 2 * half * (Ns / 16) * 17) * S;
            } else {         // last stage, j < Ns: position j + q*Ns
                sb = bs[g] + (lds_pad(tt[g]) + ((2 * half / R) * T + (2 * half % R) * Ns) / 16 * 17) * S;
            }
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const int kc = 4 * (p >> 1) + (p & 1);
                const int off = Ns == 1 ? kc
                                : R == 16 ? kc * (Ns / 16) * 17
                                          : ((kc / R) * T + (kc % R) * Ns) / 16 * 17;
                lds[sb + off * S] = make_float2(acc[2 * p], acc[2 * p + 1]);
            }
        }
        exchange_sync<WAVE_LOCAL>();
        Ns *= R;
    }
    {
        const float sc = (float)N;   // undoes the 1/R of every stage (exact)
        const int b = lay.base(tid) + lds_pad(lay.t(tid)) * S;
#pragma unroll
        for (int m = 0; m < kP; ++m) {
            const float2 x = lds[b + m * T17 * S];
            v[m] = make_float2(x.x * sc, x.y * sc);
        }
    }
    exchange_sync<WAVE_LOCAL>();
}

// One transform through the FP32 register engine (PREC 0) or the matrix
// cores (PREC 1 = BF16, 2 = FP16).  `addr` is the calling thread's LDS
// addressing for the register engine; `lay` the block's layout for the
// matrix-core engine.
template <int N, int SIGN, int PREC, bool WAVE_LOCAL = false, typename Addr, typename Lay>
__device__ __forceinline__ void fft_any(float2 (&v)[kP], int t, float2* lds, Addr addr, const Lay& lay,
                                        const float2* __restrict__ tw, const uint4* __restrict__ dftop)
{
    if constexpr (PREC == 0) fft_stages<N, SIGN, Addr, WAVE_LOCAL>(v, t, lds, addr, tw);
    else fft_stages_mfma<N, SIGN, PREC, Lay, WAVE_LOCAL>(v, lds, lay, tw, dftop);
}

}  // namespace holo

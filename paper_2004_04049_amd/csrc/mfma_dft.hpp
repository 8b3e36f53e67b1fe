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
// operand format), so each product is X*W_hi + X*W_lo accumulated in FP32:
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

// cos(2*pi*k/16), FP32 roundings; sin(2*pi*k/16) = entry (k - 4) mod 16.
__device__ __constant__ const float kCos16[16] = {
    1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f,
    0.0f, -0.382683432365089772f, -0.707106781186547524f, -0.923879532511286756f,
    -1.0f, -0.923879532511286756f, -0.707106781186547524f, -0.382683432365089772f,
    0.0f, 0.382683432365089772f, 0.707106781186547524f, 0.923879532511286756f};

template <int PREC>
struct MfmaOp;

// BF16 operands (8 significant bits).
template <>
struct MfmaOp<1> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    static __device__ __forceinline__ v8 cvt(mf32x8 x) { return __builtin_convertvector(x, v8); }
    static __device__ __forceinline__ mf32x8 back(v8 x) { return __builtin_convertvector(x, mf32x8); }
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
    static __device__ __forceinline__ mf32x8 back(v8 x) { return __builtin_convertvector(x, mf32x8); }
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

// This lane's row of W^T for radix R (see below): columns k = 8*half + e as
// coefficients of Re X[k] (a1) and Im X[k] (a2), each split hi + lo.
template <int PREC, int R, int SIGN>
__device__ __forceinline__ void dft_operand(int half, int l32, typename MfmaOp<PREC>::v8& a1h,
                                            typename MfmaOp<PREC>::v8& a1l, typename MfmaOp<PREC>::v8& a2h,
                                            typename MfmaOp<PREC>::v8& a2l)
{
    using M = MfmaOp<PREC>;
    const int ko = l32 & 15;
    const bool im_out = l32 >= 16;
    constexpr float inv_r = 1.0f / (float)R;   // exact
    mf32x8 w1, w2;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * half + e;
        const bool same = (k / R) == (ko / R);
        const int ang = ((k % R) * (ko % R) * (16 / R)) & 15;   // angle 2*pi*ang/16
        const float c = kCos16[ang] * inv_r;
        const float sn = kCos16[(ang - 4) & 15] * (SIGN > 0 ? inv_r : -inv_r);
        w1[e] = same ? (im_out ? sn : c) : 0.0f;
        w2[e] = same ? (im_out ? c : -sn) : 0.0f;
    }
    a1h = M::cvt(w1);
    a1l = M::cvt(w1 - M::back(a1h));
    a2h = M::cvt(w2);
    a2l = M::cvt(w2 - M::back(a2h));
}

// The DFT-matrix product runs transposed, D = W^T X^T: the A operand holds
// the 32 output rows (16 real parts, then 16 imaginary parts) of W^T, the B
// operand 32 vectors (lane l32 of each half-wave holds points 8*half..+7 of
// vector l32), and register i of the result holds, for the lane's vector,
// output 8*((i>>2)&1) + 4*half + (i&3) (real part for i < 8, imaginary part of
// the same output in i + 8).  So every LDS access of a lane is a per-lane base
// plus a compile-time offset, and outputs leave as complex pairs.  The
// padded positions (one spare slot per 16, as in the register engine) keep
// the strided accesses on distinct banks; T = N/16 is a multiple of 16, so
// pad(x + 16m) = pad(x) + 17m splits every address that way.
template <int N, int SIGN, int PREC, typename Lay, bool WAVE_LOCAL = false>
__device__ __forceinline__ void fft_stages_mfma(float2 (&v)[kP], float2* lds, const Lay& lay,
                                                const float2* __restrict__ tw)
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
    typename M::v8 a16[4];   // radix-16 operand, shared by all radix-16 stages
    dft_operand<PREC, 16, SIGN>(half, l32, a16[0], a16[1], a16[2], a16[3]);
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < NSTAGE; ++s) {
        const int R = (s < NS16) ? 16 : (1 << REM);
        typename M::v8 a1h = a16[0], a1l = a16[1], a2h = a16[2], a2l = a16[3];
        if (R != 16) dft_operand<PREC, (1 << (REM ? REM : 1)), SIGN>(half, l32, a1h, a1l, a2h, a2l);
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
                    const float2 w = tw[(j & (Ns - 1)) * (N / (Ns * R)) * r];
                    x = SIGN < 0 ? cmul(x, w) : cmulc(x, w);
                }
                fr[e] = x.x;
                fi[e] = x.y;
            }
            xr[g] = M::cvt(fr);
            xi[g] = M::cvt(fi);
        }
        exchange_sync<WAVE_LOCAL>();
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            mf32x16 acc = {};
            acc = M::mma(a1h, xr[g], acc);
            acc = M::mma(a1l, xr[g], acc);
            acc = M::mma(a2h, xi[g], acc);
            acc = M::mma(a2l, xi[g], acc);
            // output ko = 8*((i>>2)&1) + 4*half + (i&3) of butterfly j = tt + (ko/R)*T
            // goes to Stockham position (j/Ns)*Ns*R + (j mod Ns) + (ko mod R)*Ns
            int sb;
            if (Ns == 1) {   // first stage, R = 16: 16*tt + ko, padded 17*tt + ko
                sb = bs[g] + (17 * tt[g] + 4 * half) * S;
            } else if (R == 16) {
                const int j = tt[g];
                sb = bs[g] + (lds_pad((j / Ns) * 16 * Ns + (j & (Ns - 1))) + 4 * half * (Ns / 16) * 17) * S;
            } else {         // last stage, j < Ns: position j + q*Ns
                sb = bs[g] + (lds_pad(tt[g]) + ((4 * half / R) * T + (4 * half % R) * Ns) / 16 * 17) * S;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int kc = 8 * ((i >> 2) & 1) + (i & 3);
                const int off = Ns == 1 ? kc
                                : R == 16 ? kc * (Ns / 16) * 17
                                          : ((kc / R) * T + (kc % R) * Ns) / 16 * 17;
                lds[sb + off * S] = make_float2(acc[i], acc[i + 8]);
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
                                        const float2* __restrict__ tw)
{
    if constexpr (PREC == 0) fft_stages<N, SIGN, Addr, WAVE_LOCAL>(v, t, lds, addr, tw);
    else fft_stages_mfma<N, SIGN, PREC, Lay, WAVE_LOCAL>(v, lds, lay, tw);
}

}  // namespace holo

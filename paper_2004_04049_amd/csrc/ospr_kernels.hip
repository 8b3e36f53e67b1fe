// ospr_kernels.hip -- OSPR generation, reconstruction and NMSE kernels (FP32
// transforms, FP64 sums) for gfx950.
//
// Data path of one OSPR frame of n_sf sub-frames (Section 2, Section 3):
//   K1 ospr_rows : R_k = T * LUT[(c + k*N + p) mod N_LUT]  (Section 5, Fig. 3)
//                  and the inverse transform along x                (Eq. (2))
//   K2 ospr_cols : inverse transform along y -> H_k; nearest binary value
//                  b = (Re H_k < 0) packed LSB-first; forward transform along y
//                  of the real +-1 column B_k = 1 - 2b                 (Eq. (1))
//                  written for rows v = 0..ny/2 only (B_k is real, so its
//                  spectrum is Hermitian and the other half is redundant)
//   K3 recon_rows: forward transform along x, I_k = |.|^2, the time average
//                  over sub-frames in registers, FP64 NMSE partial sums
//   K4 finalize  : fixed-order FP64 reduction -> {NMSE, NMSE_sym}
// Transforms are unscaled; the unitary 1/sqrt(N) factors of Eq. (1)/(2) are
// folded into the intensity (1/N), since binarisation is invariant to a
// positive scale.
#include "fft_engine.hpp"
#include "kernels.hpp"
#include "mfma_dft.hpp"
#include "quant.hpp"

namespace holo {

#define HOLO_SWITCH_N(n, ...)                              \
    switch (n) {                                           \
        case 16: { constexpr int N_ = 16; __VA_ARGS__; } break;     \
        case 32: { constexpr int N_ = 32; __VA_ARGS__; } break;     \
        case 64: { constexpr int N_ = 64; __VA_ARGS__; } break;     \
        case 128: { constexpr int N_ = 128; __VA_ARGS__; } break;   \
        case 256: { constexpr int N_ = 256; __VA_ARGS__; } break;   \
        case 512: { constexpr int N_ = 512; __VA_ARGS__; } break;   \
        case 1024: { constexpr int N_ = 1024; __VA_ARGS__; } break; \
        case 2048: { constexpr int N_ = 2048; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;              \
    }

// Sizes with a matrix-core variant (blocks of whole waves at every plan).
#define HOLO_SWITCH_NM(n, ...)                             \
    switch (n) {                                           \
        case 256: { constexpr int N_ = 256; __VA_ARGS__; } break;   \
        case 512: { constexpr int N_ = 512; __VA_ARGS__; } break;   \
        case 1024: { constexpr int N_ = 1024; __VA_ARGS__; } break; \
        case 2048: { constexpr int N_ = 2048; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;              \
    }
// Size and DFT-stage precision (0 FP32 registers, 1 BF16 MFMA, 2 FP16 MFMA).
#define HOLO_SWITCH_NP(n, p, ...)                                               \
    if ((p) == 0) {                                                             \
        HOLO_SWITCH_N(n, { constexpr int P_ = 0; __VA_ARGS__; })                \
    } else if ((p) == 1) {                                                      \
        HOLO_SWITCH_NM(n, { constexpr int P_ = 1; __VA_ARGS__; })               \
    } else if ((p) == 2) {                                                      \
        HOLO_SWITCH_NM(n, { constexpr int P_ = 2; __VA_ARGS__; })               \
    } else {                                                                    \
        return hipErrorInvalidValue;                                            \
    }

// Points per thread PT_ of the OSPR row pass, column pass and reconstruction
// row pass: 16 (radix-16 stages, then one radix-2/4/8 stage) or, in FP32, 8
// (radix-8 stages, then one radix-2/4 stage).  The matrix-core forms take 16
// points per thread.
#define HOLO_SWITCH_PT(pt, ...)                                              \
    if ((pt) == 8) {                                                         \
        constexpr int PT_ = P_ ? kP : 8;                                     \
        __VA_ARGS__;                                                         \
    } else {                                                                 \
        constexpr int PT_ = kP;                                              \
        __VA_ARGS__;                                                         \
    }
// The plan's points per thread (8 or 16 for all three passes), or else per
// pass (0 = generation rows, 1 = generation columns, 2 = reconstruction rows)
// and transform length n: 8 for the generation rows, for the generation
// columns up to 1024 points and for the reconstruction rows up to 512; 16
// above (FP32, 24 sub-frames, 1024^2: rows 34.5 against 36.4 us, columns 48.3
// against 50.4, reconstruction 41.0 against 35.9).
static int plan_pts(const LaunchCfg& c, int pass, int n)
{
    if (c.prec != 0) return kP;
    if (c.pts == 8 || c.pts == kP) return c.pts;
    return (pass == 0 || n <= (pass == 1 ? 1024 : 512)) ? 8 : kP;
}

// Column-tile width C (columns transformed side by side by one block).
// Matrix-core variants (P_ != 0) exist for C = 8 (and 4, for the 2048-point
// plain column transform) only, so the other cases map to C = 8.
#define HOLO_SWITCH_C(c, ...)                                                \
    switch (c) {                                                             \
        case 2: { constexpr int C_ = P_ ? 8 : 2; __VA_ARGS__; } break;       \
        case 4: { constexpr int C_ = 4; __VA_ARGS__; } break;                \
        case 8: { constexpr int C_ = 8; __VA_ARGS__; } break;                \
        case 16: { constexpr int C_ = P_ ? 8 : 16; __VA_ARGS__; } break;     \
        default: return hipErrorInvalidValue;                                \
    }
#define HOLO_SWITCH_C816(c, ...)                                             \
    switch (c) {                                                             \
        case 8: { constexpr int C_ = 8; __VA_ARGS__; } break;                \
        case 16: { constexpr int C_ = P_ ? 8 : 16; __VA_ARGS__; } break;     \
        default: return hipErrorInvalidValue;                                \
    }

// Runtime LDS addressing (block shape chosen at launch).
struct RowAddrR {
    int base;
    __device__ __forceinline__ int operator()(int p) const { return base + p; }
};

static int row_block_rows(int n, int nrows, int planned, int prec = 0, int pt = kP)
{
    const int T = n / pt;
    int rows = planned > 0 ? planned : (256 / T > 0 ? 256 / T : 1);
    if (prec && rows * T < 64) rows = 64 / T;   // matrix cores: whole waves
    if (prec && rows * T > 256) rows = 256 / T; // ... and at most 256 threads (register budget)
    if (rows * T > 1024) rows = 1024 / T;
    if (rows < 1) rows = 1;
    while (rows > 1 && (nrows % rows)) rows >>= 1;
    if (rows > nrows) rows = nrows;
    return rows;
}

// Column-tile width C in {2, 4, 8, 16} (at least `cmin`): the plan's value, or
// else the widest tile that still gives >= 512 blocks over the whole launch;
// capped by 1024 threads and 160 KiB of LDS per block.
int col_block_cols(int n, int ncols, int nbatch, int planned, int cmin)
{
    const int T = n / kP;
    int C = planned;
    if (C <= 0) {
        C = 16;
        while (C > cmin && (long)(ncols / C) * nbatch < 512) C >>= 1;
    }
    if (C < cmin) C = cmin;
    if (C > 16) C = 16;
    while (C > cmin && (C * T > 1024 || (size_t)C * pad_len(n) * sizeof(float2) > 160 * 1024)) C >>= 1;
    if (C > ncols) C = ncols;
    return C;
}

// -------------------------------------------------------------------------
// Twiddles: FP64 evaluation on the device, rounded once to FP32.
// -------------------------------------------------------------------------
__global__ void k_twiddle_gen(float2* tw, int n)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double two_pi = 6.283185307179586476925286766559;
    double a = two_pi * ((double)k / (double)n);
    tw[k] = make_float2((float)cos(a), (float)(-sin(a)));
}

hipError_t launch_twiddle_gen(float2* tw, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_twiddle_gen, dim3((n + 255) / 256), dim3(256), 0, s, tw, n);
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// DFT-matrix operands of the matrix-core radix-16 DFTs (layout in
// mfma_dft.hpp): W[r][q] = exp(sign*2*pi*i*r*q/16) * sc evaluated in FP64
// (sincospi: exact at multiples of pi/2), each coefficient split hi = rn(w),
// lo = rn(w - hi) in the operand format.  sc = 1/16 for FP16 (keeps the data
// of chained stages in FP16's range; undone exactly after the transform), 1
// for BF16 (FP32's exponent range).  One thread per (sign, part, lane,
// element).
// -------------------------------------------------------------------------
__global__ void k_dft_operand_gen(uint16_t* __restrict__ out, int prec)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kDftOpElems) return;
    const int e = idx & 7, lane = (idx >> 3) & 63, part = (idx >> 9) & 3, si = (idx >> 11) & 1;
    const int half = lane >> 5, l32 = lane & 31;
    const int ko = l32 >> 1;
    const bool im_out = (l32 & 1) != 0;
    const int k = 8 * half + e;
    const double sc = prec == 2 ? 1.0 / 16.0 : 1.0;
    double sn, cs;
    sincospi(2.0 * (double)((k * ko) % 16) / 16.0, &sn, &cs);
    const double wr = cs * sc, wi = (si ? sn : -sn) * sc;
    // coefficient of Re X[k] (parts 0, 1) and of Im X[k] (parts 2, 3)
    const double w = part < 2 ? (im_out ? wi : wr) : (im_out ? wr : -wi);
    uint16_t bits;
    if (prec == 1) {
        const __bf16 hi = (__bf16)w;
        const __bf16 lo = (__bf16)(w - (double)hi);
        bits = __builtin_bit_cast(uint16_t, (part & 1) ? lo : hi);
    } else {
        const _Float16 hi = (_Float16)w;
        const _Float16 lo = (_Float16)(w - (double)hi);
        bits = __builtin_bit_cast(uint16_t, (part & 1) ? lo : hi);
    }
    out[idx] = bits;
}

hipError_t launch_dft_operand_gen(uint16_t* out, int prec, hipStream_t s)
{
    hipLaunchKernelGGL(k_dft_operand_gen, dim3(kDftOpElems / 256), dim3(256), 0, s, out, prec);
    return hipGetLastError();
}

#define DFTOP(cfg) (reinterpret_cast<const uint4*>((cfg).dftop))

// -------------------------------------------------------------------------
// Plain 2D transform (used by the unitary holo_fft2 entry point and tests).
// -------------------------------------------------------------------------
template <int N, int SIGN, int P>
__global__ __launch_bounds__(P ? 256 : 1024) void k_fft_rows(const float2* __restrict__ in, float2* __restrict__ out,
                                                   int nrows, const float2* __restrict__ tw,
                                                   const uint4* __restrict__ dftop)
{
    extern __shared__ float2 lds[];
    constexpr int T = N / kP;
    const int row = threadIdx.x / T, t = threadIdx.x % T;
    const int rows = blockDim.x / T;
    const size_t y = (size_t)blockIdx.x * rows + row;
    float2 v[kP];
    const float2* src = in + y * N;
#pragma unroll
    for (int m = 0; m < kP; ++m) v[m] = src[t + T * m];
    fft_any<N, SIGN, P, (N / kP <= 64)>(v, t, lds, RowAddrR{row * PadLen<N>::v}, tw, dftop);
    float2* dst = out + y * N;
#pragma unroll
    for (int m = 0; m < kP; ++m) dst[t + T * m] = v[m];
}

template <int N, int SIGN, int C, int P>
__global__ __launch_bounds__(C * (N / kP)) void k_fft_cols(const float2* __restrict__ in, float2* __restrict__ out,
                                                           int nx, float scale, const float2* __restrict__ tw,
                                                           const uint4* __restrict__ dftop)
{
    extern __shared__ float2 lds[];
    constexpr int T = N / kP;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int x0 = xcd_tile(blockIdx.x, gridDim.x) * C;
    const size_t mstride = (size_t)T * nx;
    const uint32_t toff = ((uint32_t)t * (uint32_t)nx + (uint32_t)c) * (uint32_t)sizeof(float2);
    float2 v[kP];
#pragma unroll
    for (int m = 0; m < kP; ++m) v[m] = ld_off(in + x0 + m * mstride, toff);
    fft_any<N, SIGN, P>(v, t, lds, ColAddr<C>{c}, tw, dftop);
#pragma unroll
    for (int m = 0; m < kP; ++m) st_off(out + x0 + m * mstride, toff, make_float2(v[m].x * scale, v[m].y * scale));
}

template <typename K>
static void allow_lds(K kernel, size_t bytes)
{
    if (bytes > 64 * 1024) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_fft2(const float2* in, float2* tmp, float2* out, int nx, int ny, int sign,
                       const float2* tw_x, const float2* tw_y, const LaunchCfg& cfg, hipStream_t s)
{
    {
        const int rows = row_block_rows(nx, ny, cfg.rows_per_block, cfg.prec);
        HOLO_SWITCH_NP(nx, cfg.prec, {
            constexpr int T = N_ / kP;
            size_t lds = (size_t)rows * PadLen<N_>::v * sizeof(float2);
            if (sign < 0) {
                allow_lds(k_fft_rows<N_, -1, P_>, lds);
                hipLaunchKernelGGL((k_fft_rows<N_, -1, P_>), dim3(ny / rows), dim3(rows * T), lds, s, in, tmp, ny,
                                   tw_x, DFTOP(cfg));
            } else {
                allow_lds(k_fft_rows<N_, 1, P_>, lds);
                hipLaunchKernelGGL((k_fft_rows<N_, 1, P_>), dim3(ny / rows), dim3(rows * T), lds, s, in, tmp, ny,
                                   tw_x, DFTOP(cfg));
            }
        });
    }
    {
        // matrix-core columns: 8 per block (4 at 2048, within 128 registers a thread)
        const int C = cfg.prec ? (ny >= 2048 ? 4 : 8) : col_block_cols(ny, nx, 1, cfg.cols_per_block, 2);
        const float scale = (float)(1.0 / sqrt((double)nx * (double)ny));
        HOLO_SWITCH_NP(ny, cfg.prec, HOLO_SWITCH_C(C, {
            constexpr int T = N_ / kP;
            if constexpr (C_ * T > (P_ ? 512 : 1024)) {
                return hipErrorInvalidValue;
            } else {
                size_t lds = (size_t)C_ * PadLen<N_>::v * sizeof(float2);
                if (sign < 0) {
                    allow_lds(k_fft_cols<N_, -1, C_, P_>, lds);
                    hipLaunchKernelGGL((k_fft_cols<N_, -1, C_, P_>), dim3(nx / C_), dim3(C_ * T), lds, s, tmp, out,
                                       nx, scale, tw_y, DFTOP(cfg));
                } else {
                    allow_lds(k_fft_cols<N_, 1, C_, P_>, lds);
                    hipLaunchKernelGGL((k_fft_cols<N_, 1, C_, P_>), dim3(nx / C_), dim3(C_ * T), lds, s, tmp, out,
                                       nx, scale, tw_y, DFTOP(cfg));
                }
            }
        }));
    }
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// K1: LUT phase randomisation fused with the inverse row transform (full
// planes, for the pair and eight-level variants).  A block serves `spb`
// consecutive sub-frames of its rows and loads its target values once.
// Grid: (ny / rows) * ceil(n_sf / spb) blocks of rows * (nx/16) threads.
// -------------------------------------------------------------------------
template <int NX, int P>
__global__ __launch_bounds__(P ? 256 : 512) void k_ospr_rows(const float* __restrict__ target, int ny, int n_sf,
                                                              int spb, PhaseSrc src, uint64_t c0,
                                                              const uint64_t* __restrict__ c0_base,
                                                              float2* __restrict__ x1, const float2* __restrict__ tw,
                                                              int pitch, const uint4* __restrict__ dftop)
{
    extern __shared__ float2 lds[];
    constexpr int T = NX / kP;
    const int rows = blockDim.x / T;
    const int row = threadIdx.x / T, t = threadIdx.x % T;
    const int row_blocks = ny / rows;
    const int kb = blockIdx.x / row_blocks;
    const int y = (blockIdx.x % row_blocks) * rows + row;
    const uint64_t npix = (uint64_t)NX * (uint64_t)ny;
    const auto rt = make_rsrc(target, (uint32_t)(npix * 4));
    const uint32_t toff = ((uint32_t)y * NX + (uint32_t)t) * 4u;
    float a[kP];
#pragma unroll
    for (int m = 0; m < kP; ++m) a[m] = buf_ld1(rt, toff, (uint32_t)(m * T * 4));
    uint32_t* lt = nullptr;
    if (phase_uses_lds(src)) {   // code tables after the transform's LDS rows
        lt = (uint32_t*)(lds + rows * PadLen<NX>::v);
        phase_stage(src, (uint32_t)T, lt);
    }
    const size_t plane = (size_t)ny * pitch;
    const uint32_t ooff = ((uint32_t)y * (uint32_t)pitch + (uint32_t)t) * 8u;
    const int k_end = min(n_sf, (kb + 1) * spb);
    for (int k = kb * spb; k < k_end; ++k) {   // uniform over the block
        // pool position of pixel (t, y) of sub-frame k, then +T per slot; the
        // launch's start is c0 plus a base read from device memory when given
        // (lets a replayed graph follow a cursor that moves per call)
        const uint64_t pos0 = pool_pos(src, c0, c0_base, (uint64_t)k * npix + (uint64_t)y * NX + (uint64_t)t);
        const uint32_t rs = src.kind == SRC_MSEQ ? src.rows[(size_t)k * ny + y] : 0u;
        float2 v[kP];
        phase_slots<kP>(src, pos0, (uint32_t)T, t, rs, v, lt);
#pragma unroll
        for (int m = 0; m < kP; ++m) v[m] = make_float2(a[m] * v[m].x, a[m] * v[m].y);
        fft_any<NX, 1, P, (NX / kP <= 64)>(v, t, lds, RowAddrR{row * PadLen<NX>::v}, tw, dftop);
        const auto ro = make_rsrc(x1 + (size_t)k * plane, (uint32_t)(plane * 8));
#pragma unroll
        for (int m = 0; m < kP; ++m) buf_st2(ro, ooff, (uint32_t)(m * T * 8), v[m]);
    }
}

// Sub-frames per row-pass block: 8 while the launch keeps >= 1024 blocks
// (measured at 1024^2, 24 sub-frames, Hermitian K1: 8 -> 37.5 us,
// 4 -> 38.9 us, 2 -> 39.0 us), fewer for smaller launches.
static int rows_sf_per_block(int row_blocks, int n_sf)
{
    int spb = 8;
    while (spb > 1 && (long)row_blocks * ((n_sf + spb - 1) / spb) < 1024) spb >>= 1;
    return spb;
}

hipError_t launch_ospr_rows(const float* target, int nx, int ny, int n_sf, const PhaseSrc& src, uint64_t c0,
                            const uint64_t* c0_base, float2* x1, const float2* tw_x, const LaunchCfg& cfg,
                            hipStream_t s)
{
    int rows = row_block_rows(nx, ny, cfg.rows_per_block, cfg.prec);
    while (rows > 1 && rows * (nx / kP) > 512) rows >>= 1;   // the FP32 kernel's launch bound
    const int row_blocks = ny / rows;
    const int spb = rows_sf_per_block(row_blocks, n_sf);
    HOLO_SWITCH_NP(nx, cfg.prec, {
        constexpr int T = N_ / kP;
        size_t lds = (size_t)rows * PadLen<N_>::v * sizeof(float2) +
                     (src.kind == SRC_MSEQ || src.kind == SRC_CODES8 ? kPhaseLdsWords * sizeof(uint32_t) : 0);
        allow_lds(k_ospr_rows<N_, P_>, lds);
        hipLaunchKernelGGL((k_ospr_rows<N_, P_>), dim3(row_blocks * ((n_sf + spb - 1) / spb)), dim3(rows * T), lds, s,
                           target, ny, n_sf, spb, src, c0, c0_base, x1, tw_x, row_pitch(nx, cfg), DFTOP(cfg));
    });
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// K1 for binary frames.  Only Re H is binarised, and
// Re IFFT2{R} = IFFT2{R_h} with R_h(x, y) = (R(x, y) + conj R(-x, -y))/2, the
// Hermitian part of R (indices mod nx, ny; the 1/2 is dropped, since only
// signs are read).  Row transforms of a Hermitian field obey
// X(x, -y) = conj X(x, y), so rows y = 0..ny/2 are transformed and stored (a
// half plane of ny/2 + 1 rows, pitch as x1) and the column pass rebuilds the
// others.  Each thread draws its pixels (x, y) and their mirrors (-x, -y):
// for x = t + T*m the mirror column is t' + T*m' with t' = (T - t) mod T and
// m' = PT - 1 - m (t > 0) or (PT - m) mod PT (t = 0), i.e. slot m' of a thread
// t' (PT points per thread, T = nx/PT; PT = 8 or 16 in FP32, 16 with the
// matrix cores).
// A block serves `spb` consecutive sub-frames of its rows, so each thread
// loads its target values once for all of them (the target does not stay in
// L2 between sub-frames of a whole-frame launch).
// Grid: ceil((ny/2 + 1) / rows) * ceil(n_sf / spb) blocks; the surplus rows of
// the last row block repeat row ny/2 and are not stored.
// -------------------------------------------------------------------------

template <int NX, int P, int PT>
__global__ __launch_bounds__(P ? 256 : 512) __attribute__((amdgpu_waves_per_eu(3))) void k_ospr_rows_h(const float* __restrict__ target, int ny, int n_sf,
                                                                int spb, PhaseSrc src, uint64_t c0,
                                                                const uint64_t* __restrict__ c0_base,
                                                                float2* __restrict__ x1, const float2* __restrict__ tw,
                                                                int pitch, const uint4* __restrict__ dftop,
                                                                const GroupFrame* __restrict__ gtab)
{
    if (gtab) {   // grouped launch: this frame's arguments
        const GroupFrame& gf = gtab[blockIdx.y];
        if ((int)blockIdx.x >= gf.k1_blocks) return;
        target = gf.target;
        n_sf = gf.n_sf;
        spb = gf.spb;
        c0 = gf.c0;
        x1 = gf.x1;
    }
    extern __shared__ float2 lds[];
    constexpr int T = NX / PT;
    const int rows = blockDim.x / T;
    const int row = threadIdx.x / T, t = threadIdx.x % T;
    const int nh = ny / 2 + 1;
    const int row_blocks = (nh + rows - 1) / rows;
    const int kb = blockIdx.x / row_blocks;
    const int yr = (blockIdx.x % row_blocks) * rows + row;
    const int y = yr < nh ? yr : nh - 1;
    const int ym = (ny - y) & (ny - 1);
    const int tm = (T - t) & (T - 1);
    const uint64_t npix = (uint64_t)NX * (uint64_t)ny;
    const auto rt = make_rsrc(target, (uint32_t)(npix * 4));
    const uint32_t toff0 = ((uint32_t)y * NX + (uint32_t)t) * 4u;
    const uint32_t toff1 = ((uint32_t)ym * NX + (uint32_t)tm) * 4u;
    float a[PT], b[PT];
#pragma unroll
    for (int m = 0; m < PT; ++m) {
        a[m] = buf_ld1(rt, toff0, (uint32_t)(m * T * 4));
        b[m] = buf_ld1(rt, toff1, (uint32_t)(m * T * 4));
    }
    uint32_t* lt = nullptr;
    if (phase_uses_lds(src)) {
        lt = (uint32_t*)(lds + rows * PadLenP<NX, PT>::v);
        phase_stage(src, (uint32_t)T, lt);
    }
    const bool mseq = src.kind == SRC_MSEQ;
    const bool t0 = t == 0;
    // FP32 at 8 points per thread: the row transforms' table twiddles are read
    // once for all of the block's sub-frames (at 16 the registers are spent)
    constexpr bool kPre = P == 0 && PT == 8 && NX <= 1024;
    TwRegs<NX, PT> twr;
    if constexpr (kPre) twr.read(tw, t);
    const size_t plane = (size_t)nh * pitch;
    const uint32_t ooff = ((uint32_t)y * (uint32_t)pitch + (uint32_t)t) * 8u;
    const int k_end = min(n_sf, (kb + 1) * spb);
    for (int k = kb * spb; k < k_end; ++k) {   // uniform over the block
        const uint64_t pos0 = pool_pos(src, c0, c0_base, (uint64_t)k * npix + (uint64_t)y * NX + (uint64_t)t);
        const uint64_t pos1 = pool_pos(src, c0, c0_base, (uint64_t)k * npix + (uint64_t)ym * NX + (uint64_t)tm);
        const uint32_t rs0 = mseq ? src.rows[(size_t)k * ny + y] : 0u;
        const uint32_t rs1 = mseq ? src.rows[(size_t)k * ny + ym] : 0u;
        float2 v[PT], w[PT];
        phase_slots<PT>(src, pos0, (uint32_t)T, t, rs0, v, lt);
        phase_slots<PT>(src, pos1, (uint32_t)T, tm, rs1, w, lt);
#pragma unroll
        for (int m = 0; m < PT; ++m) {
            const int mi = PT - 1 - m, mz = (PT - m) & (PT - 1);
            const float bm = t0 ? b[mz] : b[mi];
            const float2 wm = t0 ? w[mz] : w[mi];
            // R(x, y) + conj R(-x, -y)
            v[m] = make_float2(fmaf(a[m], v[m].x, bm * wm.x), fmaf(a[m], v[m].y, -bm * wm.y));
        }
        fft_any<NX, 1, P, (NX / PT <= 64), PT>(v, t, lds, RowAddrR{row * PadLenP<NX, PT>::v}, tw, dftop,
                                               kPre ? twr.w : nullptr);
        if (yr < nh) {
            const auto ro = make_rsrc(x1 + (size_t)k * plane, (uint32_t)(plane * 8));
#pragma unroll
            for (int m = 0; m < PT; ++m) buf_st2(ro, ooff, (uint32_t)(m * T * 8), v[m]);
        }
    }
}

static int rows_h_rows(int nx, int ny, const LaunchCfg& cfg, int pt)
{
    int rows = row_block_rows(nx, ny, cfg.rows_per_block, cfg.prec, pt);
    while (rows > 1 && rows * (nx / pt) > 512) rows >>= 1;   // the FP32 kernel's launch bound
    return rows;
}

void ospr_rows_h_shape(int nx, int ny, int n_sf, const LaunchCfg& cfg, int* blocks, int* spb)
{
    const int rows = rows_h_rows(nx, ny, cfg, plan_pts(cfg, 0, nx));
    const int row_blocks = (ny / 2 + 1 + rows - 1) / rows;
    *spb = rows_sf_per_block(row_blocks, n_sf);
    *blocks = row_blocks * ((n_sf + *spb - 1) / *spb);
}

hipError_t launch_ospr_rows_h(const float* target, int nx, int ny, int n_sf, const PhaseSrc& src, uint64_t c0,
                              const uint64_t* c0_base, float2* x1, const float2* tw_x, const LaunchCfg& cfg,
                              hipStream_t s, const GroupFrame* gtab, int ngroup, int grid_x)
{
    const int pt = plan_pts(cfg, 0, nx);
    const int rows = rows_h_rows(nx, ny, cfg, pt);
    int blocks, spb;
    ospr_rows_h_shape(nx, ny, n_sf, cfg, &blocks, &spb);
    const dim3 grid(gtab ? grid_x : blocks, gtab ? ngroup : 1);
    HOLO_SWITCH_NP(nx, cfg.prec, HOLO_SWITCH_PT(pt, {
        constexpr int T = N_ / PT_;
        size_t lds = (size_t)rows * PadLenP<N_, PT_>::v * sizeof(float2) +
                     (src.kind == SRC_MSEQ || src.kind == SRC_CODES8 ? kPhaseLdsWords * sizeof(uint32_t) : 0);
        allow_lds(k_ospr_rows_h<N_, P_, PT_>, lds);
        hipLaunchKernelGGL((k_ospr_rows_h<N_, P_, PT_>), grid, dim3(rows * T), lds, s, target, ny, n_sf, spb, src, c0,
                           c0_base, x1, tw_x, row_pitch(nx, cfg), DFTOP(cfg), gtab);
    }));
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// K2: inverse column transform, binarise + pack, forward column transform of
// the +-1 column; writes the half spectrum rows 0..ny/2.
//
// Columns are taken in pairs, from the half plane of k_ospr_rows_h.  Its
// columns are Hermitian (X(-y) = conj X(y)), so their inverse transforms are
// real: columns a, b of a pair share one inverse transform,
// IFFT{X_a + i X_b} = h_a + i h_b with h_a, h_b real, and only signs are read
// from it.  Likewise their +-1 columns share one forward transform
// Z = F{B_a + i B_b}, separated as F_a(v) = (Z(v) + conj Z(-v))/2,
// F_b(v) = (Z(v) - conj Z(-v))/(2i) (as in the pair variant below).  Signs and
// spectra differ from per-column transforms by rounding only.
// Grid: (nx / C) * n_sf blocks of (C/2) * (ny/PT) threads (PT points per
// thread); thread (q, t) owns columns x0 + 2q and x0 + 2q + 1 (one 16-byte
// load and one 16-byte store per row), rows t + T*m.  Slots m < PT/2 load row
// y = t + T*m; slot m >= PT/2 loads the mirror row ny - y = (T - t) +
// T*(PT - 1 - m) (also for t = 0, where slot PT/2 is row ny/2) and conjugates; rows 0 and ny/2 are real up to rounding, and their real
// parts are taken.  The C/2 lanes of a row segment are adjacent in the wave,
// so two ballots give the row's C bits.  Four waves per SIMD (what the LDS
// tile allows): the matrix-core form would otherwise take 148 registers and
// run three.
// -------------------------------------------------------------------------
// Bits 0..7 of x moved to the even positions 0, 2, .., 14.
__device__ __forceinline__ uint32_t spread_bits8(uint32_t x)
{
    x = (x | (x << 4)) & 0x0F0Fu;
    x = (x | (x << 2)) & 0x3333u;
    return (x | (x << 1)) & 0x5555u;
}

template <int NY, int C, int P, int PT>
__global__ __launch_bounds__((C / 2) * (NY / PT)) __attribute__((amdgpu_waves_per_eu(4))) void k_ospr_cols2(const float2* __restrict__ x1, int nx,
                                                                   uint32_t* __restrict__ bits,
                                                                   float2* __restrict__ x2,
                                                                   const float2* __restrict__ tw, int pitch,
                                                                   const uint4* __restrict__ dftop,
                                                                   const GroupFrame* __restrict__ gtab)
{
    extern __shared__ float2 lds[];
    constexpr int CP = C / 2;
    constexpr int T = NY / PT;
    const int q = threadIdx.x % CP, t = threadIdx.x / CP;
    const int lane = threadIdx.x & 63;
    const int ncb = nx / C;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (gtab) {   // grouped launch: this frame's arguments
        const GroupFrame& gf = gtab[blockIdx.y];
        if (tile >= gf.k2_tiles) return;
        x1 = gf.x1;
        bits = gf.bits;
        x2 = gf.x2;
    }
    const int k = tile / ncb;
    const int x0 = (tile - k * ncb) * C;
    const size_t npix = (size_t)nx * NY;
    const size_t plane = (size_t)(NY / 2 + 1) * pitch;
    const uint32_t voff = ((uint32_t)t * (uint32_t)pitch + (uint32_t)(x0 + 2 * q)) * 8u;
    const uint32_t moff = ((uint32_t)(T - t) * (uint32_t)pitch + (uint32_t)(x0 + 2 * q)) * 8u;
    const uint32_t mst = (uint32_t)T * (uint32_t)pitch * 8u;
    const auto rin = make_rsrc(x1 + (size_t)k * plane, (uint32_t)(plane * 8));
    float2 v[PT];
#pragma unroll
    for (int m = 0; m < PT / 2; ++m) {
        const float4 ab = buf_ld4(rin, voff, m * mst);               // X_a = (x, y), X_b = (z, w) at row y
        v[m] = make_float2(ab.x - ab.w, ab.y + ab.z);                // X_a + i X_b
        const float4 cd = buf_ld4(rin, moff, (PT / 2 - 1 - m) * mst); // slot m + PT/2: row ny - y = (T - t) + T*(PT/2 - 1 - m)
        v[m + PT / 2] = make_float2(cd.x + cd.w, cd.z - cd.y);       // conj X_a + i conj X_b
        if (m == 0 && t == 0) {                                      // rows 0 and ny/2
            v[0] = make_float2(ab.x, ab.z);
            v[PT / 2] = make_float2(cd.x, cd.z);
        }
    }
    // FP32 at 8 points per thread: one read of the table twiddles serves both
    // transforms (at 16 the registers are spent)
    constexpr bool kPre = P == 0 && PT == 8 && NY <= 1024;
    TwRegs<NY, PT> twr;
    if constexpr (kPre) twr.read(tw, t);
    const float2* pre = kPre ? twr.w : nullptr;
    fft_any<NY, 1, P, false, PT>(v, t, lds, ColAddr<CP>{q}, tw, dftop, pre);

    // nearest of {+1, -1}: bit = (Re h < 0); Re h = 0 -> +1.  The CP lanes of
    // a row give the even columns' bits (ballot of .x) and the odd columns'
    // (ballot of .y); interleaved, they are the row's C bits in raster order.
    const auto rbits = make_rsrc(bits + (size_t)k * (npix / 32), (uint32_t)(npix / 8));
    const uint32_t boff = ((uint32_t)t * (uint32_t)nx + (uint32_t)x0) / 8u;
    const uint32_t bst = (uint32_t)T * (uint32_t)nx / 8u;
    const int g0 = lane & ~(CP - 1);
#pragma unroll
    for (int m = 0; m < PT; ++m) {
        const bool na = v[m].x < 0.0f, nb = v[m].y < 0.0f;
        const uint64_t ma = __ballot(na), mb = __ballot(nb);
        if (q == 0) {
            const uint32_t w = spread_bits8((uint32_t)(ma >> g0) & ((1u << CP) - 1u)) |
                               (spread_bits8((uint32_t)(mb >> g0) & ((1u << CP) - 1u)) << 1);
            if (C == 16) __builtin_amdgcn_raw_buffer_store_b16((unsigned short)w, rbits, boff, m * bst, 0);
            else __builtin_amdgcn_raw_buffer_store_b8((unsigned char)w, rbits, boff, m * bst, 0);
        }
        v[m] = make_float2(na ? -1.0f : 1.0f, nb ? -1.0f : 1.0f);
    }
    fft_any<NY, -1, P, false, PT>(v, t, lds, ColAddr<CP>{q}, tw, dftop, pre);

    // separation: rows v <= NY/2 (slots m < PT/2, and m = PT/2 for t = 0) need
    // Z at -v, which lies in slots PT/2..PT-1, or slot 0 for v = 0
    __syncthreads();
#pragma unroll
    for (int m = PT / 2; m < PT; ++m) lds[(t + T * m) * CP + q] = v[m];
    if (t == 0) lds[q] = v[0];
    __syncthreads();
    // one 16-byte store per row: F_a = (Z + conj Zm) / 2, F_b = (Z - conj Zm) / (2i)
    const size_t hplane = (size_t)(NY / 2 + 1) * pitch;
    const auto rout = make_rsrc(x2 + (size_t)k * hplane, (uint32_t)(hplane * 8));
#pragma unroll
    for (int m = 0; m <= PT / 2; ++m) {
        if (m == PT / 2 && t != 0) break;
        const float2 z = v[m];
        const float2 zm = lds[((NY - (t + T * m)) & (NY - 1)) * CP + q];
        buf_st4z(rout, voff + (uint32_t)m * mst,
                 make_float4(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y), 0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x)));
    }
}

// Column-tile width of K2: 8 columns (4 column pairs per block) unless
// planned; measured at 1024^2, 24 sub-frames (FP32, 16 points per thread):
// 50.3 us against 55.2 us for 16-column tiles.  The matrix-core forms use
// 8-column tiles.
static int ospr_cols_width(int nx, int ny, int n_sf, const LaunchCfg& cfg, int pt)
{
    int C = cfg.prec ? 8 : cfg.cols_per_block > 0 ? col_block_cols(ny, nx, n_sf, cfg.cols_per_block, 8) : 8;
    if ((C / 2) * (ny / pt) > 1024) C = 8;   // 2048-point columns at 8 points per thread
    return C;
}

int ospr_cols_tiles(int nx, int ny, int n_sf, const LaunchCfg& cfg)
{
    return (nx / ospr_cols_width(nx, ny, n_sf, cfg, plan_pts(cfg, 1, ny))) * n_sf;
}

hipError_t launch_ospr_cols(const float2* x1, int nx, int ny, int n_sf, uint32_t* bits, float2* x2,
                            const float2* tw_y, const LaunchCfg& cfg, hipStream_t s, const GroupFrame* gtab,
                            int ngroup, int grid_x)
{
    const int pt = plan_pts(cfg, 1, ny);
    const int C = ospr_cols_width(nx, ny, n_sf, cfg, pt);
    HOLO_SWITCH_NP(ny, cfg.prec, HOLO_SWITCH_PT(pt, {
        constexpr int T = N_ / PT_;
        if constexpr (P_ != 0) {
            size_t lds = (size_t)4 * PadLen<N_>::v * sizeof(float2);
            allow_lds(k_ospr_cols2<N_, 8, P_, kP>, lds);
            const dim3 grid(gtab ? grid_x : (nx / 8) * n_sf, gtab ? ngroup : 1);
            hipLaunchKernelGGL((k_ospr_cols2<N_, 8, P_, kP>), grid, dim3(4 * T), lds, s, x1, nx, bits, x2, tw_y,
                               row_pitch(nx, cfg), DFTOP(cfg), gtab);
        } else {
            HOLO_SWITCH_C816(C, {
                if constexpr ((C_ / 2) * T > 1024) {
                    return hipErrorInvalidValue;   // not reached: C is reduced above
                } else {
                    size_t lds = (size_t)(C_ / 2) * PadLenP<N_, PT_>::v * sizeof(float2);
                    allow_lds(k_ospr_cols2<N_, C_, 0, PT_>, lds);
                    const dim3 grid(gtab ? grid_x : (nx / C_) * n_sf, gtab ? ngroup : 1);
                    hipLaunchKernelGGL((k_ospr_cols2<N_, C_, 0, PT_>), grid, dim3((C_ / 2) * T), lds, s, x1, nx, bits,
                                       x2, tw_y, row_pitch(nx, cfg), nullptr, gtab);
                }
            });
        }
    }));
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// K2 variants (not from the paper).
//
// Pairs: field j of the chunk gives sub-frames 2j (from Re H) and 2j+1 (from
// Im H).  Both +-1 columns go through one forward transform as
// Z = F{B_re + i B_im}; B_re, B_im are real, so per column their spectra are
// F_re(v) = (Z(v) + conj Z(-v)) / 2 and F_im(v) = (Z(v) - conj Z(-v)) / (2i),
// and each is written as the usual half spectrum: the reconstruction passes
// see 2*n_fields ordinary binary sub-frames.  Row -v of column c sits in
// thread T - t, slot 15 - m (thread 0: slot (16 - m) mod 16); the exchange
// goes through LDS.
//
// Eight levels: sub-frame k is quantised to the nearest of exp(i*2*pi*m/8)
// (codes, one byte per pixel), and the full column spectrum of its phasors is
// written (the hologram is complex, its spectrum not Hermitian).
// -------------------------------------------------------------------------
template <int NY, int C, int P>
__global__ __launch_bounds__(C * (NY / kP)) void k_ospr_cols_pair(const float2* __restrict__ x1, int nx,
                                                                 uint32_t* __restrict__ bits,
                                                                 float2* __restrict__ x2,
                                                                 const float2* __restrict__ tw, int pitch,
                                                                 const uint4* __restrict__ dftop)
{
    extern __shared__ float2 lds[];
    constexpr int T = NY / kP;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int lane = threadIdx.x & 63;
    const int ncb = nx / C;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int j = tile / ncb;
    const int x0 = (tile - j * ncb) * C;
    const size_t npix = (size_t)nx * NY;
    const size_t plane = (size_t)NY * pitch;
    const uint32_t voff = ((uint32_t)t * (uint32_t)pitch + (uint32_t)(x0 + c)) * 8u;
    const uint32_t mst = (uint32_t)T * (uint32_t)pitch * 8u;
    const auto rin = make_rsrc(x1 + (size_t)j * plane, (uint32_t)(plane * 8));
    float2 v[kP];
#pragma unroll
    for (int m = 0; m < kP; ++m) v[m] = buf_ld2(rin, voff, m * mst);
    fft_any<NY, 1, P>(v, t, lds, ColAddr<C>{c}, tw, dftop);

    // nearest of {+1, -1} for Re H (sub-frame 2j) and Im H (sub-frame 2j+1)
    const auto rb_re = make_rsrc(bits + (size_t)(2 * j) * (npix / 32), (uint32_t)(npix / 8));
    const auto rb_im = make_rsrc(bits + (size_t)(2 * j + 1) * (npix / 32), (uint32_t)(npix / 8));
    const uint32_t boff = ((uint32_t)t * (uint32_t)nx + (uint32_t)x0) / 8u;
    const uint32_t bst = (uint32_t)T * (uint32_t)nx / 8u;
#pragma unroll
    for (int m = 0; m < kP; ++m) {
        const bool nre = v[m].x < 0.0f, nim = v[m].y < 0.0f;
        const uint64_t mre = __ballot(nre), mim = __ballot(nim);
        if (c == 0) {
            const uint32_t cre = (uint32_t)(mre >> (lane & ~(C - 1))), cim = (uint32_t)(mim >> (lane & ~(C - 1)));
            if (C == 16) {
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)cre, rb_re, boff, m * bst, 0);
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)cim, rb_im, boff, m * bst, 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b8((unsigned char)cre, rb_re, boff, m * bst, 0);
                __builtin_amdgcn_raw_buffer_store_b8((unsigned char)cim, rb_im, boff, m * bst, 0);
            }
        }
        v[m] = make_float2(nre ? -1.0f : 1.0f, nim ? -1.0f : 1.0f);
    }
    fft_any<NY, -1, P>(v, t, lds, ColAddr<C>{c}, tw, dftop);

    // mirror rows through LDS (plain [row][C] layout; the engine is done with it)
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kP; ++m) lds[(t + T * m) * C + c] = v[m];
    __syncthreads();
    float2 fre[kP / 2 + 1], fim[kP / 2 + 1];
#pragma unroll
    for (int m = 0; m <= kP / 2; ++m) {
        const int row = t + T * m;
        const float2 z = v[m];
        const float2 zm = lds[((NY - row) & (NY - 1)) * C + c];
        fre[m] = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));   // (Z + conj Zm) / 2
        fim[m] = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));   // (Z - conj Zm) / (2i)
    }
    // rows v = t + T*m <= NY/2: every slot m < 8, and m = 8 for t = 0 only
    const size_t hplane = (size_t)(NY / 2 + 1) * pitch;
    const auto rre = make_rsrc(x2 + (size_t)(2 * j) * hplane, (uint32_t)(hplane * 8));
    const auto rim = make_rsrc(x2 + (size_t)(2 * j + 1) * hplane, (uint32_t)(hplane * 8));
#pragma unroll
    for (int m = 0; m < kP / 2; ++m) {
        buf_st2(rre, voff, m * mst, fre[m]);
        buf_st2(rim, voff, m * mst, fim[m]);
    }
    if (t == 0) {
        buf_st2(rre, voff, (kP / 2) * mst, fre[kP / 2]);
        buf_st2(rim, voff, (kP / 2) * mst, fim[kP / 2]);
    }
}

template <int NY, int C, int P>
__global__ __launch_bounds__(C * (NY / kP)) void k_ospr_cols_l8(const float2* __restrict__ x1, int nx,
                                                               uint8_t* __restrict__ codes,
                                                               float2* __restrict__ x2,
                                                               const float2* __restrict__ tw, int pitch,
                                                               const uint4* __restrict__ dftop)
{
    extern __shared__ float2 lds[];
    constexpr int T = NY / kP;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int ncb = nx / C;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int k = tile / ncb;
    const int x0 = (tile - k * ncb) * C;
    const size_t npix = (size_t)nx * NY;
    const size_t plane = (size_t)NY * pitch;
    const uint32_t voff = ((uint32_t)t * (uint32_t)pitch + (uint32_t)(x0 + c)) * 8u;
    const uint32_t mst = (uint32_t)T * (uint32_t)pitch * 8u;
    const auto rin = make_rsrc(x1 + (size_t)k * plane, (uint32_t)(plane * 8));
    float2 v[kP];
#pragma unroll
    for (int m = 0; m < kP; ++m) v[m] = buf_ld2(rin, voff, m * mst);
    fft_any<NY, 1, P>(v, t, lds, ColAddr<C>{c}, tw, dftop);
    const auto rc = make_rsrc(codes + (size_t)k * npix, (uint32_t)npix);
    const uint32_t coff = (uint32_t)t * (uint32_t)nx + (uint32_t)(x0 + c);
#pragma unroll
    for (int m = 0; m < kP; ++m) {
        const uint8_t q = quant8(v[m]);
        __builtin_amdgcn_raw_buffer_store_b8((unsigned char)q, rc, coff, (uint32_t)(m * T * nx), 0);
        v[m] = level8_phasor(q);
    }
    fft_any<NY, -1, P>(v, t, lds, ColAddr<C>{c}, tw, dftop);
    const auto rout = make_rsrc(x2 + (size_t)k * plane, (uint32_t)(plane * 8));
#pragma unroll
    for (int m = 0; m < kP; ++m) buf_st2(rout, voff, m * mst, v[m]);
}

hipError_t launch_ospr_cols_mode(int mode, const float2* x1, int nx, int ny, int n_fields, void* holo, float2* x2,
                                 const float2* tw_y, const LaunchCfg& cfg, hipStream_t s)
{
    // 8-column tiles unless planned (measured at 1024^2, 12 fields: pairs
    // 57 us against 68 us, eight levels 153 us against 163 us for 16 columns)
    const int C = cfg.prec ? 8 : cfg.cols_per_block > 0 ? col_block_cols(ny, nx, n_fields, cfg.cols_per_block, 8) : 8;
    HOLO_SWITCH_NP(ny, cfg.prec, HOLO_SWITCH_C816(C, {
        constexpr int T = N_ / kP;
        if (C_ * T <= 1024) {
            size_t lds = (size_t)C_ * PadLen<N_>::v * sizeof(float2);
            if (mode == OSPR_PAIRS) {
                allow_lds(k_ospr_cols_pair<N_, C_, P_>, lds);
                hipLaunchKernelGGL((k_ospr_cols_pair<N_, C_, P_>), dim3((nx / C_) * n_fields), dim3(C_ * T), lds, s,
                                   x1, nx, (uint32_t*)holo, x2, tw_y, row_pitch(nx, cfg), DFTOP(cfg));
            } else {
                allow_lds(k_ospr_cols_l8<N_, C_, P_>, lds);
                hipLaunchKernelGGL((k_ospr_cols_l8<N_, C_, P_>), dim3((nx / C_) * n_fields), dim3(C_ * T), lds, s,
                                   x1, nx, (uint8_t*)holo, x2, tw_y, row_pitch(nx, cfg), DFTOP(cfg));
            }
        }
    }));
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// Reconstruction column transform from a quantised hologram.
//   levels 2: packed bits -> B = +-1 -> rows 0..ny/2 of its column spectrum
//   levels 8: codes m -> exp(i*2*pi*m/8) -> full column spectrum
// -------------------------------------------------------------------------

template <int NY, int C, int P>
__global__ __launch_bounds__(C * (NY / kP)) void k_recon_cols(const void* __restrict__ holo, int levels, int nx,
                                                             float2* __restrict__ x2, const float2* __restrict__ tw,
                                                             int pitch, const uint4* __restrict__ dftop)
{
    extern __shared__ float2 lds[];
    constexpr int T = NY / kP;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int ncb = nx / C;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int k = tile / ncb;
    const int x0 = (tile - k * ncb) * C;
    const int x = x0 + c;
    const size_t npix = (size_t)nx * NY;
    float2 v[kP];
    if (levels == 2) {
        const uint32_t* w = reinterpret_cast<const uint32_t*>(holo) + (size_t)k * (npix / 32);
#pragma unroll
        for (int m = 0; m < kP; ++m) {
            const size_t p = (size_t)(t + T * m) * nx + x;
            const uint32_t b = (w[p >> 5] >> (p & 31)) & 1u;
            v[m] = make_float2(b ? -1.0f : 1.0f, 0.0f);
        }
    } else {
        const uint8_t* cd = reinterpret_cast<const uint8_t*>(holo) + (size_t)k * npix;
#pragma unroll
        for (int m = 0; m < kP; ++m) v[m] = level8_phasor(cd[(size_t)(t + T * m) * nx + x]);
    }
    fft_any<NY, -1, P>(v, t, lds, ColAddr<C>{c}, tw, dftop);
    const int vmax = levels == 2 ? NY / 2 : NY - 1;
    float2* dst = x2 + (size_t)k * (vmax + 1) * pitch;
#pragma unroll
    for (int m = 0; m < kP; ++m) {
        const int vv = t + T * m;
        if (vv <= vmax) dst[(size_t)vv * pitch + x] = v[m];
    }
}

hipError_t launch_recon_cols(const void* holo, int levels, int nx, int ny, int n_sf, float2* x2,
                             const float2* tw_y, const LaunchCfg& cfg, hipStream_t s)
{
    const int C = cfg.prec ? 8 : col_block_cols(ny, nx, n_sf, cfg.recon_cols_per_block, 2);
    HOLO_SWITCH_NP(ny, cfg.prec, HOLO_SWITCH_C(C, {
        constexpr int T = N_ / kP;
        if (C_ * T <= 1024) {
            size_t lds = (size_t)C_ * PadLen<N_>::v * sizeof(float2);
            allow_lds(k_recon_cols<N_, C_, P_>, lds);
            hipLaunchKernelGGL((k_recon_cols<N_, C_, P_>), dim3((nx / C_) * n_sf), dim3(C_ * T), lds, s, holo, levels,
                               nx, x2, tw_y, row_pitch(nx, cfg), DFTOP(cfg));
        }
    }));
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// K3: row transform of each sub-frame's column spectrum, intensity, time
// average and FP64 NMSE partial sums.  One block per spectrum row v; its
// G = blockDim/(nx/16) thread groups take sub-frames g, g+G, ... and their
// sums are combined through LDS in a fixed order.
// partials[v*5 + {0..4}] = {S_II, S_IT, S_ITs, S_TT, S_TsTs} over the pixels
// this row stands for (itself and, for the half spectrum, its point mirror).
// -------------------------------------------------------------------------
template <int NX, int P, int PT>
__global__ __launch_bounds__(P ? 256 : 512) __attribute__((amdgpu_waves_per_eu(4))) void k_recon_rows(const float2* __restrict__ x2, int ny, int n_sf, int half,
                                                     const float* __restrict__ target, float* __restrict__ recon,
                                                     double* __restrict__ partials, const float2* __restrict__ tw,
                                                     float inv_scale, int pitch, const uint4* __restrict__ dftop,
                                                     const GroupFrame* __restrict__ gtab)
{
    if (gtab) {   // grouped launch: this frame's arguments (half spectra)
        const GroupFrame& gf = gtab[blockIdx.y];
        x2 = gf.x2;
        n_sf = gf.n_sf;
        target = gf.target;
        recon = gf.recon;
        partials = gf.part;
        inv_scale = gf.inv_scale;
    }
    extern __shared__ float2 lds[];
    constexpr int T = NX / PT;
    const int G = blockDim.x / T;
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    const int v_row = blockIdx.x;
    const int nrows_spec = half ? (ny / 2 + 1) : ny;
    const size_t sf_stride = (size_t)nrows_spec * pitch;
    float acc[PT];
#pragma unroll
    for (int m = 0; m < PT; ++m) acc[m] = 0.0f;
    const int rounds = (n_sf + G - 1) / G;
    // one descriptor per round, based at the round's first spectrum (64-bit
    // pointer arithmetic) and covering the round's min(G, n_sf - r*G) spectra,
    // so the 32-bit record count and lane offsets stay below 2^32 for any
    // n_sf (at most G planes: < 2^30 bytes); loads of sub-frames k >= n_sf
    // fall outside it and read as zero.  No register prefetch of the next
    // sub-frame: capped at 128 VGPRs (4 waves per SIMD) the plain loop is
    // faster (35.8 against 37.2 us at 1024^2, 24 sub-frames, 4 groups)
    const uint32_t kst = (uint32_t)(sf_stride * 8);
    const uint32_t roff = ((uint32_t)v_row * (uint32_t)pitch + (uint32_t)t) * 8u + (uint32_t)g * kst;
    // FP32 at 8 points per thread: the table twiddles read once for all rounds
    // (up to 512 points; at 1024 the extra registers cost a block per CU, and
    // the 513 blocks then take two rounds: 51 against 41 us)
    constexpr bool kPre = P == 0 && PT == 8 && NX <= 512;
    TwRegs<NX, PT> twr;
    if constexpr (kPre) twr.read(tw, t);
    for (int r = 0; r < rounds; ++r) {
        const int k = r * G + g;
        const bool valid = k < n_sf;
        const int in_round = n_sf - r * G < G ? n_sf - r * G : G;
        const auto rx = make_rsrc(x2 + (size_t)r * G * sf_stride, (uint32_t)in_round * kst);
        float2 v[PT];
#pragma unroll
        for (int m = 0; m < PT; ++m) v[m] = buf_ld2(rx, roff, (uint32_t)(m * T * 8));
        fft_any<NX, -1, P, (NX / PT <= 64), PT>(v, t, lds, RowAddrR{g * PadLenP<NX, PT>::v}, tw, dftop,
                                                kPre ? twr.w : nullptr);
        if (valid) {
#pragma unroll
            for (int m = 0; m < PT; ++m) acc[m] = fmaf(v[m].x, v[m].x, fmaf(v[m].y, v[m].y, acc[m]));
        }
    }
    // combine the G groups' sums (group order fixed); the groups' transforms
    // synchronise per wave, so wait for all of them before reusing LDS
    float* ldsf = reinterpret_cast<float*>(lds);
    if (G > 1) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PT; ++m) ldsf[g * NX + t + T * m] = acc[m];
        __syncthreads();
        if (g == 0) {
#pragma unroll
            for (int m = 0; m < PT; ++m) {
                float s = ldsf[t + T * m];
                for (int gg = 1; gg < G; ++gg) s += ldsf[gg * NX + t + T * m];
                acc[m] = s;
            }
        }
        __syncthreads();
    }
    double sums[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (g == 0) {
        const int vm = (ny - v_row) % ny;
        const bool self_mirror = !half || v_row == 0 || v_row == ny / 2;
        const float* trow = target + (size_t)v_row * NX;
        const float* mrow = target + (size_t)vm * NX;
#pragma unroll
        for (int m = 0; m < PT; ++m) {
            const int u = t + T * m;
            const int um = (NX - u) & (NX - 1);
            const double ib = (double)(acc[m] * inv_scale);
            const double ta = (double)trow[u], tb = (double)mrow[um];
            const double t2a = ta * ta, t2b = tb * tb, ts = 0.5 * (t2a + t2b);
            if (half && !self_mirror) {
                sums[0] += 2.0 * ib * ib;
                sums[1] += ib * (t2a + t2b);
                sums[2] += 2.0 * ib * ts;
                sums[3] += t2a * t2a + t2b * t2b;
                sums[4] += 2.0 * ts * ts;
            } else {
                sums[0] += ib * ib;
                sums[1] += ib * t2a;
                sums[2] += ib * ts;
                sums[3] += t2a * t2a;
                sums[4] += ts * ts;
            }
            if (recon) {
                recon[(size_t)v_row * NX + u] = (float)ib;
                if (half && !self_mirror) recon[(size_t)vm * NX + um] = (float)ib;
            }
        }
    }
    double tot[5];
    block_sum<5>(sums, reinterpret_cast<double*>(lds), tot);
    if (threadIdx.x == 0)
        for (int i = 0; i < 5; ++i) partials[(size_t)v_row * 5 + i] = tot[i];
}

int recon_rows_groups(int nx, int n_sf, const LaunchCfg& cfg)
{
    const int T = nx / plan_pts(cfg, 2, nx);
    int G = cfg.ksplit > 0 ? cfg.ksplit : 4;
    while (G > 1 && (G * T > 512 || G > n_sf)) G >>= 1;
    // matrix cores: whole waves (groups past n_sf transform zeros and add
    // nothing), at most 256 threads
    if (cfg.prec && G * T > 256) G = 256 / T;
    if (cfg.prec && G * T < 64) G = 64 / T;
    return G;
}

hipError_t launch_recon_rows(const float2* x2, int nx, int ny, int n_sf, bool half, const float* target,
                             float* recon, double* partials, const float2* tw_x, const LaunchCfg& cfg,
                             hipStream_t s, const GroupFrame* gtab, int ngroup)
{
    const int nrows_spec = half ? ny / 2 + 1 : ny;
    const int pt = plan_pts(cfg, 2, nx);
    const int G = recon_rows_groups(nx, n_sf, cfg);
    HOLO_SWITCH_NP(nx, cfg.prec, HOLO_SWITCH_PT(pt, {
        constexpr int T = N_ / PT_;
        size_t fft_lds = (size_t)G * PadLenP<N_, PT_>::v * sizeof(float2);
        size_t red_lds = (size_t)5 * (G * T / 64 + 1) * sizeof(double);
        size_t lds = fft_lds > red_lds ? fft_lds : red_lds;
        const float inv_scale = (float)(1.0 / ((double)n_sf * (double)nx * (double)ny));
        allow_lds(k_recon_rows<N_, P_, PT_>, lds);
        hipLaunchKernelGGL((k_recon_rows<N_, P_, PT_>), dim3(nrows_spec, gtab ? ngroup : 1), dim3(G * T), lds, s, x2,
                           ny, n_sf, half ? 1 : 0, target, recon, partials, tw_x, inv_scale, row_pitch(nx, cfg),
                           DFTOP(cfg), gtab);
    }));
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// K4: {NMSE, NMSE_sym} = 1 - S_IW^2 / (S_II * S_WW) from the row partials,
// reduced in a fixed order (deterministic run to run): lane l adds rows
// l, l + 64, ... in turn, then a butterfly over the wave.  One wave, no block
// barriers (6.3 against 7.0 us for a 256-thread block at 513 rows).
// -------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_nmse_finalize(const double* __restrict__ partials, int nrows,
                                                       double* __restrict__ out2, const GroupFrame* __restrict__ gtab)
{
    if (gtab) {   // grouped launch: one block per frame
        partials = gtab[blockIdx.x].part;
        out2 = gtab[blockIdx.x].nm;
    }
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = threadIdx.x; r < nrows; r += 64)
        for (int i = 0; i < 5; ++i) a[i] += partials[(size_t)r * 5 + i];
    double s[5];
    for (int i = 0; i < 5; ++i) s[i] = seg_sum(a[i], 64);
    if (threadIdx.x == 0) {
        const double s_ii = s[0], s_it = s[1], s_its = s[2], s_tt = s[3], s_tsts = s[4];
        out2[0] = (s_ii > 0.0 && s_tt > 0.0) ? 1.0 - s_it * s_it / (s_ii * s_tt) : 1.0;
        out2[1] = (s_ii > 0.0 && s_tsts > 0.0) ? 1.0 - s_its * s_its / (s_ii * s_tsts) : 1.0;
    }
}

hipError_t launch_nmse_finalize(const double* partials, int nrows, double* out2, hipStream_t s)
{
    hipLaunchKernelGGL(k_nmse_finalize, dim3(1), dim3(64), 0, s, partials, nrows, out2, nullptr);
    return hipGetLastError();
}

hipError_t launch_ospr_group(const GroupFrame* tab, const GroupFrame* host, int n, int nx, int ny,
                             const PhaseSrc& src, const uint64_t* c0_base, const float2* tw_x, const float2* tw_y,
                             const LaunchCfg& cfg, hipStream_t s)
{
    int k1 = 0, k2 = 0;
    for (int f = 0; f < n; ++f) {
        k1 = host[f].k1_blocks > k1 ? host[f].k1_blocks : k1;
        k2 = host[f].k2_tiles > k2 ? host[f].k2_tiles : k2;
    }
    // the shape arguments of the first frame stand for all (equal by grouping)
    const int ns = host[0].n_sf;
    hipError_t e = launch_ospr_rows_h(nullptr, nx, ny, ns, src, 0, c0_base, nullptr, tw_x, cfg, s, tab, n, k1);
    if (e != hipSuccess) return e;
    if ((e = launch_ospr_cols(nullptr, nx, ny, ns, nullptr, nullptr, tw_y, cfg, s, tab, n, k2)) != hipSuccess) return e;
    if ((e = launch_recon_rows(nullptr, nx, ny, ns, true, nullptr, nullptr, nullptr, tw_x, cfg, s, tab, n)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_nmse_finalize, dim3(n), dim3(64), 0, s, nullptr, ny / 2 + 1, nullptr, tab);
    return hipGetLastError();
}

}  // namespace holo

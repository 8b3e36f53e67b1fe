// gs_kernels.hip -- Gerchberg-Saxton passes (FP32 transforms, FP64 sums).
//
// GS (Section 2; Gerchberg & Saxton 1972) alternates between the hologram
// plane, where the SLM allows phase only, and the replay plane, where only the
// target amplitude is prescribed.  One iteration is two passes over the field:
//   cols pass: inverse transform along y (completing H = F^{-1}{R}, Eq. (2)),
//              optional 8-level codes of H, H' = H/|H| (H = 0 -> 1), forward
//              transform along y (first half of R' = F{H'}, Eq. (1)).
//   rows pass: forward transform along x (R'), FP64 partial sums of the
//              per-iteration NMSE and amplitude error, amplitude replacement
//              R = T * R'/|R'| (R' = 0 -> T), inverse transform along x.
// The first rows pass forms R_0 = T * phasor from the LUT (cyclic address
// (c + p) mod N_LUT, Section 5) or from a caller phasor field, and the last one
// writes the unitary replay field R'_n instead of replacing amplitudes.
#include "fft_engine.hpp"
#include "kernels.hpp"
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

namespace {
struct RowAddrG {
    int base;
    __device__ __forceinline__ int operator()(int p) const { return base + p; }
};

template <typename K>
void allow_lds_g(K kernel, size_t bytes)
{
    // a refusal shows up as the launch's own error
    if (bytes > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Sum over the T threads of each row (rows are aligned groups of T lanes):
// butterflies inside a wave, then the T/64 wave totals of a row in order.
// Result valid in the row's thread t == 0.  Needs NV * blockDim/64 doubles.
template <int NV>
__device__ __forceinline__ void row_sum(double (&a)[NV], double* red, int T, int row, int t)
{
    const int seg = T < 64 ? T : 64;
#pragma unroll
    for (int i = 0; i < NV; ++i) a[i] = seg_sum(a[i], seg);
    if (T > 64) {
        __syncthreads();
        if ((threadIdx.x & 63) == 0)
            for (int i = 0; i < NV; ++i) red[(threadIdx.x >> 6) * NV + i] = a[i];
        __syncthreads();
        if (t == 0) {
            const int w0 = (row * T) >> 6, nw = T >> 6;
            for (int i = 0; i < NV; ++i) {
                double s = 0.0;
                for (int w = 0; w < nw; ++w) s += red[(w0 + w) * NV + i];
                a[i] = s;
            }
        }
    }
}
}  // namespace


// -------------------------------------------------------------------------
// Rows pass.  partials layout: [ny][3] = {S_II, S_IT, E} for ITER/FINAL,
// [ny][2] = {sum T^2, sum T^4} for INIT.
// -------------------------------------------------------------------------
template <int NX, int MODE, int P>
__global__ __launch_bounds__(P == 16 ? 256 : 512) void k_gs_rows(const float* __restrict__ target, int ny,
                                                  PhaseSrc src, uint64_t c0,
                                                  const uint64_t* __restrict__ c0_base,
                                                  const float2* __restrict__ init, float2* __restrict__ state,
                                                  float2* __restrict__ field_out, double* __restrict__ partials,
                                                  const GsConsts* __restrict__ consts, const float2* __restrict__ tw,
                                                  int pitch, const GsFrame* __restrict__ gtab, int part_off)
{
    if (gtab) {   // grouped launch: this frame's arguments
        const GsFrame& gf = gtab[blockIdx.y];
        target = gf.target;
        c0 = gf.c0;
        init = gf.init;
        state = gf.state;
        field_out = gf.field;
        partials = (MODE == GS_INIT ? gf.pinit : gf.piter) + part_off;
        consts = gf.consts;
    }
    extern __shared__ float2 lds[];
    constexpr int T = NX / P;
    const int rows = blockDim.x / T;
    const int row = threadIdx.x / T, t = threadIdx.x % T;
    const int y = blockIdx.x * rows + row;
    float2* srow = state + (size_t)y * pitch;
    float2 v[P];
    float ta[P];
    {
        const auto rt = make_rsrc(target, (uint32_t)((size_t)ny * NX * sizeof(float)));
        const uint32_t toff = ((uint32_t)y * NX + (uint32_t)t) * 4u;
#pragma unroll
        for (int m = 0; m < P; ++m) ta[m] = buf_ld1(rt, toff, (uint32_t)(m * T * 4));
    }

    if (MODE == GS_INIT) {
        double s2 = 0.0, s4 = 0.0;
        if (init) {
            const float2* irow = init + (size_t)y * NX;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const float2 p = irow[t + T * m];
                const float mag = sqrtf(p.x * p.x + p.y * p.y);
                v[m] = mag > 0.0f ? make_float2(ta[m] * (p.x / mag), ta[m] * (p.y / mag)) : make_float2(ta[m], 0.0f);
            }
        } else {
            const uint64_t pos0 = pool_pos(src, c0, c0_base, (uint64_t)y * NX + (uint64_t)t);
            const uint32_t rs = src.kind == SRC_MSEQ ? src.rows[y] : 0u;
            phase_slots<P>(src, pos0, (uint32_t)T, t, rs, v);
#pragma unroll
            for (int m = 0; m < P; ++m) v[m] = make_float2(ta[m] * v[m].x, ta[m] * v[m].y);
        }
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const double q = (double)ta[m] * (double)ta[m];
            s2 += q;
            s4 += q * q;
        }
        fft_stages<NX, 1, RowAddrG, (NX / P <= 64), P>(v, t, lds, RowAddrG{row * PadLenP<NX, P>::v}, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) srow[t + T * m] = v[m];
        double a2[2] = {s2, s4};
        row_sum<2>(a2, reinterpret_cast<double*>(lds), T, row, t);
        if (t == 0) {
            partials[(size_t)y * 2] = a2[0];
            partials[(size_t)y * 2 + 1] = a2[1];
        }
        return;
    }

    // state and target through buffer descriptors: one lane offset, slot m at
    // the uniform offset m*T elements
    const auto rs = make_rsrc(state, (uint32_t)((size_t)ny * pitch * sizeof(float2)));
    const uint32_t soff = ((uint32_t)y * (uint32_t)pitch + (uint32_t)t) * 8u;
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = buf_ld2(rs, soff, (uint32_t)(m * T * 8));
    // an iteration's forward and inverse row transforms share one read of
    // the table twiddles (at 8 points per thread and up to 1024 points; at 16
    // points the registers are spent, at 2048 the values would go to scratch)
    constexpr bool kPre = MODE == GS_ITER && P == 8 && NX <= 1024;
    TwRegs<NX, P> twr;
    if constexpr (kPre) twr.read(tw, t);
    const float2* pre = kPre ? twr.w : nullptr;
    fft_stages<NX, -1, RowAddrG, (NX / P <= 64), P>(v, t, lds, RowAddrG{row * PadLenP<NX, P>::v}, tw, pre);
    // R' (unscaled) = sqrt(N) * R'_unitary; intensity in unitary units
    const float inv_n = 1.0f / (float)((size_t)NX * (size_t)ny);
    const float inv_sqrt_n = (float)(1.0 / sqrt((double)NX * (double)ny));
    const float te = (float)consts->te_scale;
    double s_ii = 0.0, s_it = 0.0, e = 0.0;
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const float i_u = (v[m].x * v[m].x + v[m].y * v[m].y) * inv_n;
        const double ib = (double)i_u;
        const double t2 = (double)ta[m] * (double)ta[m];
        s_ii += ib * ib;
        s_it += ib * t2;
        // amplitude error term in FP32 (relative error ~1e-7), summed in FP64
        const float d = sqrtf(i_u) - ta[m] * te;
        e += (double)(d * d);
    }
    if (MODE == GS_FINAL) {
        float2* frow = field_out + (size_t)y * NX;
#pragma unroll
        for (int m = 0; m < P; ++m) frow[t + T * m] = make_float2(v[m].x * inv_sqrt_n, v[m].y * inv_sqrt_n);
    } else {
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const float m2 = v[m].x * v[m].x + v[m].y * v[m].y;
            const float k = ta[m] * rsqrtf(m2);   // T / |R'|
            v[m] = m2 > 0.0f ? make_float2(k * v[m].x, k * v[m].y) : make_float2(ta[m], 0.0f);
        }
        fft_stages<NX, 1, RowAddrG, (NX / P <= 64), P>(v, t, lds, RowAddrG{row * PadLenP<NX, P>::v}, tw, pre);
#pragma unroll
        for (int m = 0; m < P; ++m) buf_st2(rs, soff, (uint32_t)(m * T * 8), v[m]);
    }
    double a3[3] = {s_ii, s_it, e};
    row_sum<3>(a3, reinterpret_cast<double*>(lds), T, row, t);
    if (t == 0) {
        partials[(size_t)y * 3] = a3[0];
        partials[(size_t)y * 3 + 1] = a3[1];
        partials[(size_t)y * 3 + 2] = a3[2];
    }
}

// Points per thread of the GS passes: the plan's value (4, 8 or 16), or else
// 8 when 16 would give the launch fewer than 2^17 threads (two waves per SIMD
// on 256 CUs; a single 1024^2 field has only 1024 transforms per axis), 16
// otherwise.  4 is never chosen by itself: its five radix-4 stages per 1024
// points round more often, and 50-iteration GS trajectories drift from FP64
// about 2.5x further than with 8 or 16.
static int gs_points(int n, int ntrans, int planned)
{
    if (planned == 4 || planned == 8 || planned == 16) return planned;
    return (long)ntrans * (n / 16) < (1L << 17) ? 8 : 16;
}

#define HOLO_SWITCH_P(p, ...)                                    \
    switch (p) {                                                 \
        case 4: { constexpr int P_ = 4; __VA_ARGS__; } break;    \
        case 8: { constexpr int P_ = 8; __VA_ARGS__; } break;    \
        case 16: { constexpr int P_ = 16; __VA_ARGS__; } break;  \
        default: return hipErrorInvalidValue;                    \
    }

hipError_t launch_gs_rows(int mode, const float* target, int nx, int ny, const PhaseSrc& src, uint64_t c0,
                          const uint64_t* c0_base, const float2* init, float2* state, float2* field_out,
                          double* partials, const GsConsts* consts, const float2* tw_x,
                          const LaunchCfg& cfg, hipStream_t s, const GsFrame* gtab, int ngroup, int part_off)
{
    const int P = gs_points(nx, ny, cfg.pts);
    const int T = nx / P;
    const int bound = P == 16 ? 256 : 512;   // launch bound of k_gs_rows
    if (T > bound) return hipErrorInvalidValue;
    int rows = cfg.rows_per_block;
    if (rows <= 0) {   // widest block that still leaves >= 512 blocks
        rows = 256 / T > 0 ? 256 / T : 1;
        while (rows > 1 && ny / rows < 512) rows >>= 1;
    }
    while (rows > 1 && rows * T > bound) rows >>= 1;
    while (rows > 1 && (ny % rows)) rows >>= 1;
    if (rows > ny) rows = ny;
    HOLO_SWITCH_P(P, HOLO_SWITCH_N(nx, {
        if (N_ >= P_) {
            size_t fft_lds = (size_t)rows * PadLenP<N_, P_>::v * sizeof(float2);
            size_t red_lds = (size_t)3 * (rows * T / 64 + 1) * sizeof(double);
            size_t lds = fft_lds > red_lds ? fft_lds : red_lds;
            if (mode == GS_INIT) {
                allow_lds_g(k_gs_rows<N_, GS_INIT, P_>, lds);
                hipLaunchKernelGGL((k_gs_rows<N_, GS_INIT, P_>), dim3(ny / rows, ngroup), dim3(rows * T), lds, s,
                                   target, ny, src, c0, c0_base, init, state, field_out, partials, consts, tw_x,
                                   row_pitch(nx, cfg), gtab, part_off);
            } else if (mode == GS_ITER) {
                allow_lds_g(k_gs_rows<N_, GS_ITER, P_>, lds);
                hipLaunchKernelGGL((k_gs_rows<N_, GS_ITER, P_>), dim3(ny / rows, ngroup), dim3(rows * T), lds, s,
                                   target, ny, src, c0, c0_base, init, state, field_out, partials, consts, tw_x,
                                   row_pitch(nx, cfg), gtab, part_off);
            } else {
                allow_lds_g(k_gs_rows<N_, GS_FINAL, P_>, lds);
                hipLaunchKernelGGL((k_gs_rows<N_, GS_FINAL, P_>), dim3(ny / rows, ngroup), dim3(rows * T), lds, s,
                                   target, ny, src, c0, c0_base, init, state, field_out, partials, consts, tw_x,
                                   row_pitch(nx, cfg), gtab, part_off);
            }
        }
    }));
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// Columns pass (in place on `state`).
// -------------------------------------------------------------------------
template <int NY, int C, int P>
__global__ __launch_bounds__(C * (NY / P)) void k_gs_cols(float2* __restrict__ state, int nx,
                                                          uint8_t* __restrict__ codes, const float2* __restrict__ tw,
                                                          int pitch, const GsFrame* __restrict__ gtab)
{
    if (gtab) {   // grouped launch: this frame's field (and codes, when asked)
        state = gtab[blockIdx.y].state;
        codes = codes ? gtab[blockIdx.y].codes : nullptr;
    }
    extern __shared__ float2 lds[];
    constexpr int T = NY / P;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int x0 = xcd_tile(blockIdx.x, gridDim.x) * C;
    // buffer descriptors over the whole field: lane offset (t*pitch + x0 + c),
    // slot m at the uniform offset m*T rows
    const auto rs = make_rsrc(state, (uint32_t)((size_t)NY * pitch * sizeof(float2)));
    const uint32_t toff = ((uint32_t)t * (uint32_t)pitch + (uint32_t)(x0 + c)) * 8u;
    const uint32_t mst = (uint32_t)T * (uint32_t)pitch * 8u;
    float2 v[P];
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = buf_ld2(rs, toff, m * mst);
    // one read of the table twiddles for both transforms (at 8 points per
    // thread and up to 1024 points, as in the rows pass)
    constexpr bool kPre = P == 8 && NY <= 1024;
    TwRegs<NY, P> twr;
    if constexpr (kPre) twr.read(tw, t);
    const float2* pre = kPre ? twr.w : nullptr;
    fft_stages<NY, 1, ColAddr<C>, false, P>(v, t, lds, ColAddr<C>{c}, tw, pre);
    if (codes) {
        const auto rc = make_rsrc(codes, (uint32_t)((size_t)NY * nx));
        const uint32_t coff = (uint32_t)t * (uint32_t)nx + (uint32_t)(x0 + c);
#pragma unroll
        for (int m = 0; m < P; ++m)
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)quant8(v[m]), rc, coff, (uint32_t)(m * T * nx), 0);
    }
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const float m2 = v[m].x * v[m].x + v[m].y * v[m].y;
        const float k = rsqrtf(m2);   // 1 / |H|
        v[m] = m2 > 0.0f ? make_float2(k * v[m].x, k * v[m].y) : make_float2(1.0f, 0.0f);
    }
    fft_stages<NY, -1, ColAddr<C>, false, P>(v, t, lds, ColAddr<C>{c}, tw, pre);
#pragma unroll
    for (int m = 0; m < P; ++m) buf_st2(rs, toff, m * mst, v[m]);
}

hipError_t launch_gs_cols(float2* state, int nx, int ny, uint8_t* codes, const float2* tw_y,
                          const LaunchCfg& cfg, hipStream_t s, const GsFrame* gtab, int ngroup)
{
    const int P = gs_points(ny, nx, cfg.pts);
    const int T = ny / P;
    // column-tile width: the plan's, or the widest that keeps >= 512 blocks;
    // at most 1024 threads and 160 KiB of LDS per block
    int C = cfg.cols_per_block > 0 ? cfg.cols_per_block : 16;
    if (cfg.cols_per_block <= 0)
        while (C > 2 && nx / C < 512) C >>= 1;
    if (C > 16) C = 16;
    while (C > 2 && (C * T > 1024 || (size_t)C * (ny + ny / P) * sizeof(float2) > 160 * 1024)) C >>= 1;
    if (C > nx) C = nx;
    if (C * T > 1024) return hipErrorInvalidValue;
#define HOLO_GS_COLS_CASE(CC)                                                                                 \
    case CC: {                                                                                                \
        constexpr int C_ = CC;                                                                                \
        HOLO_SWITCH_P(P, HOLO_SWITCH_N(ny, {                                                                  \
            if (N_ >= P_ && C_ * (N_ / P_) <= 1024) {                                                         \
                size_t lds = (size_t)C_ * PadLenP<N_, P_>::v * sizeof(float2);                               \
                allow_lds_g(k_gs_cols<N_, C_, P_>, lds);                                                      \
                hipLaunchKernelGGL((k_gs_cols<N_, C_, P_>), dim3(nx / C_, ngroup), dim3(C_ * T), lds, s,      \
                                   state, nx, codes, tw_y, row_pitch(nx, cfg), gtab);                         \
            }                                                                                                 \
        }));                                                                                                  \
    } break;
    switch (C) {
        HOLO_GS_COLS_CASE(2)
        HOLO_GS_COLS_CASE(4)
        HOLO_GS_COLS_CASE(8)
        HOLO_GS_COLS_CASE(16)
        default: return hipErrorInvalidValue;
    }
#undef HOLO_GS_COLS_CASE
    return hipGetLastError();
}

// -------------------------------------------------------------------------
// Frame constants from the INIT partials: sum T^2, sum T^4 and the amplitude
// scale Te = T * sqrt(N / sum T^2) that matches a unit-modulus hologram's
// replay energy (Parseval).
// -------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gs_consts(const double* __restrict__ part, int ny, int nx,
                                                   GsConsts* __restrict__ consts, const GsFrame* __restrict__ gtab)
{
    if (gtab) {   // grouped launch: one block per frame
        part = gtab[blockIdx.x].pinit;
        consts = gtab[blockIdx.x].consts;
    }
    __shared__ double red[2 * 8];
    double a[2] = {0.0, 0.0}, out[2];
    for (int r = threadIdx.x; r < ny; r += 256) {
        a[0] += part[(size_t)r * 2];
        a[1] += part[(size_t)r * 2 + 1];
    }
    block_sum<2>(a, red, out);
    if (threadIdx.x == 0) {
        consts->sum_t2 = out[0];
        consts->sum_t4 = out[1];
        consts->te_scale = out[0] > 0.0 ? sqrt((double)nx * (double)ny / out[0]) : 0.0;
    }
}

hipError_t launch_gs_consts(const double* init_partials, int ny, int nx, GsConsts* consts, hipStream_t s,
                            const GsFrame* gtab, int ngroup)
{
    hipLaunchKernelGGL(k_gs_consts, dim3(gtab ? ngroup : 1), dim3(256), 0, s, init_partials, ny, nx, consts, gtab);
    return hipGetLastError();
}

// One block per iteration: NMSE_i = 1 - S_IT^2 / (S_II * S_TT), E_i.
__global__ __launch_bounds__(256) void k_gs_finalize(const double* __restrict__ part, int ny,
                                                     const GsConsts* __restrict__ consts, double* __restrict__ nmse,
                                                     double* __restrict__ err, const GsFrame* __restrict__ gtab)
{
    if (gtab) {   // grouped launch: blockIdx.y selects the frame
        const GsFrame& gf = gtab[blockIdx.y];
        part = gf.piter;
        consts = gf.consts;
        nmse = gf.nmse;
        err = gf.err;
    }
    __shared__ double red[3 * 8];
    const int it = blockIdx.x;
    const double* p = part + (size_t)it * ny * 3;
    double a[3] = {0.0, 0.0, 0.0}, out[3];
    for (int r = threadIdx.x; r < ny; r += 256)
        for (int i = 0; i < 3; ++i) a[i] += p[(size_t)r * 3 + i];
    block_sum<3>(a, red, out);
    if (threadIdx.x == 0) {
        const double s_tt = consts->sum_t4;
        if (nmse) nmse[it] = (out[0] > 0.0 && s_tt > 0.0) ? 1.0 - out[1] * out[1] / (out[0] * s_tt) : 1.0;
        if (err) err[it] = out[2];
    }
}

hipError_t launch_gs_finalize(const double* partials, int n_iter, int ny, const GsConsts* consts,
                              double* nmse_out, double* err_out, hipStream_t s, const GsFrame* gtab, int ngroup)
{
    hipLaunchKernelGGL(k_gs_finalize, dim3(n_iter, gtab ? ngroup : 1), dim3(256), 0, s, partials, ny, consts, nmse_out,
                       err_out, gtab);
    return hipGetLastError();
}

}  // namespace holo

// phase_src.hpp -- where the random phase of pool entry i comes from.
//
// The method (the pool of Section 4, read as in Section 5, Fig. 3) reads a
// fixed pool of random phases cyclically: sub-frame k of a frame that starts at pool position c gives
// pixel p the entry at position c + k*N + p (mod the pool length).  Section 4
// names the alternative a software implementation uses -- a PRNG and the
// trigonometric functions -- and Section 7 a hardware one, an M-sequence that
// still needs sine and cosine tables.  The library keeps the pool-position
// contract for every source, so the generation kernels only differ in how a
// position turns into a unit phasor:
//
//   SRC_TABLE   FP32 phasor table of n entries (the method as published);
//   SRC_CODES8  8-bit phase codes (n bytes), phasor exp(2*pi*i*q/256) from a
//               256-entry table (the byte-per-entry reading of the storage
//               figure of Section 5.2; 8x smaller than SRC_TABLE, so 2^20+
//               entry pools stay cache-resident);
//   SRC_PRNG    no table: SplitMix64 in counter form at the absolute position,
//               x_i = mix(seed + (i+1)*gamma) -- the same x_i that fill
//               SRC_TABLE pools, so a PRNG pool equals an unbounded table of
//               the same seed -- phase 2*pi*u, u = top 24 bits of x_i / 2^24,
//               phasor from the hardware sine/cosine (argument in turns);
//   SRC_MSEQ    binary M-sequence of the primitive trinomial x^31 + x^3 + 1
//               (period 2^31 - 1), eight bits per entry as a phase code into
//               the 256-entry table; behaves as a pool of 2^31 - 1 entries.
//
// M-sequence arithmetic: bit s_n of the sequence is the coefficient of x^30 in
// x^n * S_0 reduced mod P(x) = x^31 + x^3 + 1 (the Galois form of the shift
// register; any fixed linear read-out of x^n * S_0 satisfies the recurrence
// s_{n+31} = s_{n+3} + s_n of P).  For j <= 27 the coefficient of x^30 in
// x^j * S is the coefficient of x^(30-j) in S, so the state S_{8i} holds the
// code of entry i (bits s_{8i} .. s_{8i+7}, the first one most significant) in
// its bits 30..23, and stepping to the next entry is one shift by 8 with a
// two-term fold.  A thread whose pixels are a stride T apart advances by
// multiplication with the constant x^(8T), done as four byte-table lookups.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_engine.hpp"

namespace holo {

enum : int { SRC_TABLE = 0, SRC_CODES8 = 1, SRC_PRNG = 2, SRC_MSEQ = 3 };

constexpr uint32_t kMseqM = 0x7FFFFFFFu;   // 2^31 - 1: the period, and the 31-bit element mask
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// Kernel argument (by value).  `rows` is set per launch.
struct PhaseSrc {
    const float2* tab;      // TABLE: n phasors; CODES8, MSEQ: 256 phasors exp(2*pi*i*q/256)
    const uint8_t* codes;   // CODES8: n codes
    const uint32_t* jump;   // MSEQ: [12][4][256] tables v*x^(8b) * x^(8*2^j) mod P for strides 2^j, j < 12
    const uint32_t* rows;   // MSEQ: Galois state at the first pixel of each (sub-frame, row)
    uint64_t seed;          // PRNG
    uint32_t n;             // pool length of the cyclic kinds (MSEQ: 2^31 - 1); PRNG: unused
    int kind;
};

// x^k * s mod P for 1 <= k <= 28: the k bits pushed past x^30 fold back as
// h*(x^3 + 1), which stays below x^31 for k <= 28.
__device__ __forceinline__ uint32_t gf_xshift(uint32_t s, int k)
{
    const uint32_t h = s >> (31 - k);
    return ((s << k) & kMseqM) ^ (h << 3) ^ h;
}

// General product in GF(2)[x] / P (carry-less multiply, then two folds).
__device__ __forceinline__ uint32_t gf_mul(uint32_t a, uint32_t b)
{
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < 31; ++i) acc ^= (uint64_t)(a & (0u - ((b >> i) & 1u))) << i;
    uint64_t hi = acc >> 31;
    acc = (acc & kMseqM) ^ (hi << 3) ^ hi;
    hi = acc >> 31;
    return (uint32_t)((acc & kMseqM) ^ (hi << 3) ^ hi);
}

__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Words of LDS that phase_stage fills: the jump table of one stride (MSEQ),
// then the 256 code phasors (MSEQ, CODES8).
constexpr int kPhaseLdsWords = 1024 + 512;

__device__ __forceinline__ bool phase_uses_lds(const PhaseSrc& src)
{
    return src.kind == SRC_MSEQ || src.kind == SRC_CODES8;
}

// Copies the code tables of `src` into LDS `lt` (kPhaseLdsWords words); every
// thread of the block calls it, for kinds where phase_uses_lds holds.
__device__ __forceinline__ void phase_stage(const PhaseSrc& src, uint32_t T, uint32_t* lt)
{
    if (src.kind == SRC_MSEQ) {
        const uint32_t* j = src.jump + 1024u * (uint32_t)(31 - __builtin_clz(T));
        for (int i = threadIdx.x; i < 1024; i += blockDim.x) lt[i] = j[i];
    }
    const uint32_t* ph = (const uint32_t*)src.tab;
    for (int i = threadIdx.x; i < 512; i += blockDim.x) lt[1024 + i] = ph[i];
    __syncthreads();
}

// Phasors of the pool positions pos0 + T*m, m = 0..P-1, for a thread whose
// slot-0 pixel is pixel t of its row.  pos0: the cyclic kinds take it reduced
// mod n; PRNG takes the absolute position.  `rs`: MSEQ only, the Galois state
// of the row's first pixel; `lt`: code tables staged by phase_stage, or NULL
// to read them from global memory.
template <int P>
__device__ __forceinline__ void phase_slots(const PhaseSrc& src, uint64_t pos0, uint32_t T, int t, uint32_t rs,
                                            float2 (&ph)[P], const uint32_t* lt = nullptr)
{
    if (src.kind == SRC_PRNG) {
        uint64_t z = src.seed + (pos0 + 1) * kGolden;
        const uint64_t dz = (uint64_t)T * kGolden;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const uint64_t x = splitmix_mix(z);
            const float u = (float)(uint32_t)(x >> 40) * 0x1.0p-24f;   // exact: 24 bits
            ph[m] = make_float2(__builtin_amdgcn_cosf(u), __builtin_amdgcn_sinf(u));
            z += dz;
        }
    } else if (src.kind == SRC_MSEQ) {
        const auto rt = make_rsrc(src.tab, 256u * 8u);
        // the [4][256] table of this stride (a power of two): stride 2^j at j * 1024 words
        const auto rj = make_rsrc(src.jump + 1024u * (uint32_t)(31 - __builtin_clz(T)), 1024u * 4u);
        uint32_t s = rs;
        for (int k = 8 * t; k > 0;) {   // x^(8t): shifts of at most 24
            const int d = k > 24 ? 24 : k;
            s = gf_xshift(s, d);
            k -= d;
        }
        if (lt) {
            const float2* lph = (const float2*)(lt + 1024);
#pragma unroll
            for (int m = 0; m < P; ++m) {
                ph[m] = lph[s >> 23];
                if (m + 1 < P)
                    s = lt[s & 255u] ^ lt[256 + ((s >> 8) & 255u)] ^ lt[512 + ((s >> 16) & 255u)] ^ lt[768 + (s >> 24)];
            }
        } else {
#pragma unroll
            for (int m = 0; m < P; ++m) {
                ph[m] = buf_ld2(rt, (s >> 23) * 8u, 0);
                if (m + 1 < P) {
                    const uint32_t b0 = s & 255u, b1 = (s >> 8) & 255u, b2 = (s >> 16) & 255u, b3 = s >> 24;
                    s = __builtin_bit_cast(uint32_t, buf_ld1(rj, b0 * 4u, 0)) ^
                        __builtin_bit_cast(uint32_t, buf_ld1(rj, b1 * 4u, 1024u)) ^
                        __builtin_bit_cast(uint32_t, buf_ld1(rj, b2 * 4u, 2048u)) ^
                        __builtin_bit_cast(uint32_t, buf_ld1(rj, b3 * 4u, 3072u));
                }
            }
        }
    } else {
        const uint32_t n = src.n;
        uint32_t idx = (uint32_t)pos0;
        const uint32_t step = T % n;
        if (src.kind == SRC_CODES8) {
            const auto rc = make_rsrc(src.codes, n);
            const auto rt = make_rsrc(src.tab, 256u * 8u);
            uint32_t q[P];
#pragma unroll
            for (int m = 0; m < P; ++m) {
                q[m] = __builtin_amdgcn_raw_buffer_load_b8(rc, idx, 0, 0);
                idx += step;
                if (idx >= n) idx -= n;
            }
            const float2* lph = lt ? (const float2*)(lt + 1024) : nullptr;
#pragma unroll
            for (int m = 0; m < P; ++m) ph[m] = lph ? lph[q[m]] : buf_ld2(rt, q[m] * 8u, 0);
        } else {
            const auto rl = make_rsrc(src.tab, n * 8u);
#pragma unroll
            for (int m = 0; m < P; ++m) {
                ph[m] = buf_ld2(rl, idx * 8u, 0);
                idx += step;
                if (idx >= n) idx -= n;
            }
        }
    }
}

// Pool position of pixel p of sub-frame k for a launch starting at c0 (+ the
// device word *c0_base when given): cyclic kinds mod n, PRNG absolute.
__device__ __forceinline__ uint64_t pool_pos(const PhaseSrc& src, uint64_t c0, const uint64_t* c0_base,
                                             uint64_t offset)
{
    const uint64_t cb = c0_base ? *c0_base : 0;
    const uint64_t p = cb + c0 + offset;
    return src.kind == SRC_PRNG ? p : p % src.n;
}

}  // namespace holo

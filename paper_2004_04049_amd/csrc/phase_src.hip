// phase_src.hip -- M-sequence row states and the phase-mask fill.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "phase_src.hpp"

namespace holo {

// One thread per (sub-frame k, row y): Galois state of the row's first pixel,
// x^e * S_0 with e = 8 * pos mod (2^31 - 1) (x has order 2^31 - 1 because P
// is primitive), by square-and-multiply over the table x^(2^j), j < 31.
// aux: [0, 31) the powers x^(2^j), [31] S_0.
__global__ void k_mseq_rows(const uint32_t* __restrict__ aux, uint64_t c0, const uint64_t* __restrict__ c0_base,
                            uint64_t npix, int nx, int ny, int n_sf, uint32_t* __restrict__ rows)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_sf * ny) return;
    const int k = g / ny, y = g - (g / ny) * ny;
    const uint64_t cb = c0_base ? *c0_base : 0;
    const uint64_t pos = (cb + c0 + (uint64_t)k * npix + (uint64_t)y * (uint64_t)nx) % kMseqM;
    const uint32_t e = (uint32_t)((pos * 8u) % kMseqM);
    uint32_t s = aux[31];
    for (int j = 0; j < 31; ++j)
        if ((e >> j) & 1u) s = gf_mul(s, aux[j]);
    rows[g] = s;
}

hipError_t launch_mseq_rows(const uint32_t* aux, uint64_t c0, const uint64_t* c0_base, int nx, int ny, int n_sf,
                            uint32_t* rows, hipStream_t s)
{
    const int n = n_sf * ny;
    hipLaunchKernelGGL(k_mseq_rows, dim3((n + 255) / 256), dim3(256), 0, s, aux, c0, c0_base,
                       (uint64_t)nx * (uint64_t)ny, nx, ny, n_sf, rows);
    return hipGetLastError();
}

// The phasor each generation kernel multiplies into pixel (k, y, x): the same
// thread layout as the row pass of the OSPR generation (T = nx/16 threads per
// row, thread t holding pixels t + T*m) and the same phase_slots call.
__global__ __launch_bounds__(256) void k_phase_mask(PhaseSrc src, uint64_t c0, int nx, int ny, int n_sf,
                                                    float2* __restrict__ out)
{
    const int T = nx / 16;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)n_sf * ny * T) return;
    const int t = (int)(gid % T);
    const int64_t r = gid / T;
    const int k = (int)(r / ny), y = (int)(r % ny);
    const uint64_t npix = (uint64_t)nx * (uint64_t)ny;
    const uint64_t pos0 = pool_pos(src, c0, nullptr, (uint64_t)k * npix + (uint64_t)y * nx + (uint64_t)t);
    const uint32_t rs = src.kind == SRC_MSEQ ? src.rows[r] : 0u;
    float2 ph[16];
    phase_slots<16>(src, pos0, (uint32_t)T, t, rs, ph);
    float2* o = out + (size_t)k * npix + (size_t)y * nx + t;
#pragma unroll
    for (int m = 0; m < 16; ++m) o[(size_t)m * T] = ph[m];
}

hipError_t launch_phase_mask(const PhaseSrc& src, uint64_t c0, int nx, int ny, int n_sf, float2* out, hipStream_t s)
{
    const int64_t n = (int64_t)n_sf * ny * (nx / 16);
    hipLaunchKernelGGL(k_phase_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, c0, nx, ny, n_sf, out);
    return hipGetLastError();
}

}  // namespace holo

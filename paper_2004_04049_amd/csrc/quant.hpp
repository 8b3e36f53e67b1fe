// quant.hpp -- the eight phase levels exp(i*2*pi*m/8) of the 8-level
// quantiser (Section 2: each pixel goes to the nearest value the display can
// show) and their phasors.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace holo {

// Nearest of the 8 phase levels exp(i*2*pi*m/8) to h, m = round(8*arg(h)/(2*pi))
// mod 8, decided by comparing |Im| and |Re| against tan(pi/8) without atan2.
__device__ __forceinline__ uint8_t quant8(float2 h)
{
    if (h.x == 0.0f && h.y == 0.0f) return 0;
    const float t8 = 0.414213562373095049f;   // tan(pi/8)
    const float ax = fabsf(h.x), ay = fabsf(h.y);
    int d;                                     // 0: along Re axis, 1: diagonal, 2: along Im axis
    if (ay < ax * t8) d = 0;
    else if (ax < ay * t8) d = 2;
    else d = 1;
    const bool re_neg = h.x < 0.0f, im_neg = h.y < 0.0f;
    int m;
    if (!re_neg && !im_neg) m = d;             // [0, pi/2]
    else if (re_neg && !im_neg) m = 4 - d;     // (pi/2, pi]
    else if (re_neg && im_neg) m = 4 + d;      // (pi, 3pi/2)
    else m = (8 - d) & 7;                      // (3pi/2, 2pi)
    return (uint8_t)m;
}

__device__ __forceinline__ float2 level8_phasor(int m)
{
    const float h = 0.707106781186547524f;
    switch (m & 7) {
        case 0: return make_float2(1.0f, 0.0f);
        case 1: return make_float2(h, h);
        case 2: return make_float2(0.0f, 1.0f);
        case 3: return make_float2(-h, h);
        case 4: return make_float2(-1.0f, 0.0f);
        case 5: return make_float2(-h, -h);
        case 6: return make_float2(0.0f, -1.0f);
        default: return make_float2(h, -h);
    }
}

}  // namespace holo

// cnn.hpp -- device buffers and launchers of the learned GS seed network
// (internal; the boundary is include/holo.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace holo {

constexpr int kCnnC = 32;   // hidden channels

// Parameter offsets of the 5 layers in the flat FP32 vector (per layer
// w[co][ci][3][3] then b[co]).
struct CnnLayout {
    int off[5];
    int n;
    CnnLayout()
    {
        int o = 0;
        for (int l = 0; l < 5; ++l) {
            const int ci = l == 0 ? 1 : kCnnC, co = l == 4 ? 2 : kCnnC;
            off[l] = o;
            o += co * ci * 9 + co;
        }
        n = o;
    }
};

struct CnnBuffers {
    // parameters (FP32 master), Adam moments, gradient, BF16 MFMA copies
    float *params, *m, *v, *grad;
    uint16_t* wf[3];   // forward weights of layers 2..4, [co][t][ci]
    uint16_t* wt[3];   // backward-data weights, [ci][8-t][co]
    uint32_t* w5;      // layer-5 weights as BF16 pairs, [t][ci/2][co]
    int off[5];
    // per-image activations (sized for the largest image seen)
    uint16_t* act[4];  // post-ReLU layers 1..4, [ny][nx][32] BF16
    uint16_t* dact[2]; // gradient ping-pong, [ny][nx][32] BF16
    float2* o5;        // raw layer-5 output
    float2* d5;        // its gradient
    float* part;       // weight-gradient partials
    double* loss_part; // [256][3]
    double* zsum;      // {Re Z, Im Z, W, loss, batch mean loss}
    int rows_per_block;
};

hipError_t cnn_launch_forward(const CnnBuffers& b, const float* target, int ny, int nx, float2* phasor,
                              hipStream_t s);
// loss of one image into zsum[0..3]; zsum[4] (+)= loss * inv_batch
hipError_t cnn_launch_loss(const CnnBuffers& b, const float* target, const float2* label, const float2* phasor,
                           int n, int accumulate, double inv_batch, hipStream_t s);
// gradient of one image: grad (+)= scale * dL/dparams
hipError_t cnn_launch_backward(const CnnBuffers& b, const float* target, const float2* label, int ny, int nx,
                               float scale, int accumulate, hipStream_t s);
hipError_t cnn_launch_adam(const CnnBuffers& b, int n, float lr, int step, hipStream_t s);
hipError_t cnn_launch_pack(const CnnBuffers& b, hipStream_t s);

}  // namespace holo

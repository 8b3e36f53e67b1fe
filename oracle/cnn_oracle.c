/*
 * cnn_oracle.c -- FP64 CPU oracle for the learned GS seed: a small
 * convolutional network mapping a target amplitude to an initial replay-plane
 * phasor for Gerchberg-Saxton.  The paper does not contain this network; it
 * is the learned extension of its LUT seed (the LUT stays the fallback).
 *
 * TEST INFRASTRUCTURE ONLY (see holo_oracle.c).  Shares no code with the HIP
 * path.
 *
 * Network: 5 layers of 3x3 convolution with circular padding,
 *   1 -> C -> C -> C -> C -> 2 channels, bias, ReLU after layers 1..4,
 *   output phasor p = (o0, o1) / |(o0, o1)| per pixel ((1, 0) where o = 0).
 * Tensors are [channels][ny][nx] (double); weights of a layer are
 * [cout][cin][3][3] with tap (dy, dx) at index (dy + 1, dx + 1):
 *   out[co][y][x] = b[co] + sum_{ci, dy, dx} w[co][ci][dy+1][dx+1] *
 *                   in[ci][(y + dy) mod ny][(x + dx) mod nx].
 *
 * Storage model (bf16_store != 0): the hidden activations, and in the
 * backward pass the hidden-layer gradients after the ReLU gate, are rounded
 * to BF16 (8 significant bits, round to nearest, ties to even) where they are
 * stored, as a device implementation that keeps them in BF16 does; all sums
 * stay FP64.  bf16_store = 0 is the exact network.
 *
 * Loss (global-phase invariant, target-intensity weighted): with w = T^2,
 * label phasor q and Z = sum w p conj(q), W = sum w,
 *   L = 1 - |Z| / W
 * which equals the weighted mean of 1 - cos(phi_p - phi_q - c*) at the best
 * global offset c* = arg Z.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Round to the nearest BF16 value (the upper 16 bits of an IEEE binary32),
 * ties to even, via binary32.  Finite inputs only. */
double orc_bf16(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* one 3x3 circular convolution layer */
void orc_conv3x3(const double *in, int cin, int ny, int nx, const double *w, const double *b, int cout,
                 double *out)
{
    for (int co = 0; co < cout; ++co)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double acc = b ? b[co] : 0.0;
                for (int ci = 0; ci < cin; ++ci)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int yy = (y + dy + ny) % ny, xx = (x + dx + nx) % nx;
                            acc += w[((co * cin + ci) * 3 + dy + 1) * 3 + dx + 1] * in[(ci * ny + yy) * nx + xx];
                        }
                out[(co * ny + y) * nx + x] = acc;
            }
}

/* Layer shapes of the 5-layer network with C hidden channels. */
static void layer_shape(int l, int C, int *cin, int *cout)
{
    *cin = l == 0 ? 1 : C;
    *cout = l == 4 ? 2 : C;
}

/* Parameter count; parameters are laid out layer by layer as weights then
 * biases. */
int orc_cnn_nparams(int C)
{
    int n = 0;
    for (int l = 0; l < 5; ++l) {
        int ci, co;
        layer_shape(l, C, &ci, &co);
        n += co * ci * 9 + co;
    }
    return n;
}

/* Forward pass.  acts (may be NULL) receives the post-ReLU activations of
 * layers 1..4 ([4][C][ny][nx]); out2 the raw 2-channel output, phasor the
 * normalised output ([ny][nx] interleaved re, im). */
void orc_cnn_forward(const double *params, int C, const float *target, int ny, int nx, int bf16_store,
                     double *acts, double *out2, double *phasor)
{
    const size_t np = (size_t)ny * nx;
    double *a = (double *)malloc(sizeof(double) * np * (size_t)C);
    double *bufb = (double *)malloc(sizeof(double) * np * (size_t)C);
    double *t = (double *)malloc(sizeof(double) * np);
    for (size_t p = 0; p < np; ++p) t[p] = (double)target[p];
    const double *in = t;
    const double *pp = params;
    for (int l = 0; l < 5; ++l) {
        int ci, co;
        layer_shape(l, C, &ci, &co);
        const double *w = pp, *b = pp + co * ci * 9;
        pp += co * ci * 9 + co;
        double *dst = l == 4 ? out2 : (in == a ? bufb : a);
        orc_conv3x3(in, ci, ny, nx, w, b, co, dst);
        if (l < 4) {
            for (size_t i = 0; i < np * (size_t)co; ++i) {
                const double r = dst[i] > 0.0 ? dst[i] : 0.0;
                dst[i] = bf16_store ? orc_bf16(r) : r;
            }
            if (acts) memcpy(acts + (size_t)l * np * C, dst, sizeof(double) * np * C);
        }
        in = dst;
    }
    for (size_t p = 0; p < np; ++p) {
        double c = out2[p], s = out2[np + p], m = sqrt(c * c + s * s);
        phasor[2 * p] = m > 0.0 ? c / m : 1.0;
        phasor[2 * p + 1] = m > 0.0 ? s / m : 0.0;
    }
    free(a);
    free(bufb);
    free(t);
}

/* Loss L = 1 - |sum w p conj(q)| / sum w with w = T^2. */
double orc_cnn_loss(const double *phasor, const double *label, const float *target, size_t np)
{
    double zr = 0.0, zi = 0.0, W = 0.0;
    for (size_t p = 0; p < np; ++p) {
        double w = (double)target[p] * (double)target[p];
        double pr = phasor[2 * p], pi = phasor[2 * p + 1], qr = label[2 * p], qi = label[2 * p + 1];
        zr += w * (pr * qr + pi * qi);
        zi += w * (pi * qr - pr * qi);
        W += w;
    }
    return W > 0.0 ? 1.0 - sqrt(zr * zr + zi * zi) / W : 0.0;
}

/* Gradient of the loss with respect to all parameters (analytic backward
 * pass).  Returns the loss.  The label is used as given (a unit phasor). */
double orc_cnn_backward(const double *params, int C, const float *target, const double *label, int ny, int nx,
                        int bf16_store, double *grad)
{
    const size_t np = (size_t)ny * nx;
    double *acts = (double *)malloc(sizeof(double) * np * (size_t)C * 4);
    double *out2 = (double *)malloc(sizeof(double) * np * 2);
    double *ph = (double *)malloc(sizeof(double) * np * 2);
    orc_cnn_forward(params, C, target, ny, nx, bf16_store, acts, out2, ph);

    /* dL/dp = -(w / (W |Z|)) * Z q (complex product), then through the
     * normalisation p = o/|o|: dL/do = (g - (g.p) p) / |o|. */
    double zr = 0.0, zi = 0.0, W = 0.0;
    for (size_t p = 0; p < np; ++p) {
        double w = (double)target[p] * (double)target[p];
        zr += w * (ph[2 * p] * label[2 * p] + ph[2 * p + 1] * label[2 * p + 1]);
        zi += w * (ph[2 * p + 1] * label[2 * p] - ph[2 * p] * label[2 * p + 1]);
        W += w;
    }
    const double zm = sqrt(zr * zr + zi * zi);
    const double loss = W > 0.0 ? 1.0 - zm / W : 0.0;
    double *dcur = (double *)malloc(sizeof(double) * np * (size_t)C);
    double *dprev = (double *)malloc(sizeof(double) * np * (size_t)C);
    memset(grad, 0, sizeof(double) * (size_t)orc_cnn_nparams(C));
    for (size_t p = 0; p < np; ++p) {
        double w = (double)target[p] * (double)target[p];
        double k = (W > 0.0 && zm > 0.0) ? -w / (W * zm) : 0.0;
        double qr = label[2 * p], qi = label[2 * p + 1];
        double gr = k * (zr * qr - zi * qi), gi = k * (zr * qi + zi * qr);
        double c = out2[p], s = out2[np + p], m = sqrt(c * c + s * s);
        if (m > 0.0) {
            double pr = c / m, pi = s / m, d = gr * pr + gi * pi;
            dcur[p] = (gr - d * pr) / m;
            dcur[np + p] = (gi - d * pi) / m;
        } else {
            dcur[p] = dcur[np + p] = 0.0;
        }
    }
    /* parameter offsets */
    int off[5], o = 0;
    for (int l = 0; l < 5; ++l) {
        int ci, co;
        layer_shape(l, C, &ci, &co);
        off[l] = o;
        o += co * ci * 9 + co;
    }
    double *tin = (double *)malloc(sizeof(double) * np);
    for (size_t p = 0; p < np; ++p) tin[p] = (double)target[p];
    for (int l = 4; l >= 0; --l) {
        int ci, co;
        layer_shape(l, C, &ci, &co);
        const double *in = l == 0 ? tin : acts + (size_t)(l - 1) * np * C;
        const double *w = params + off[l];
        double *gw = grad + off[l], *gb = grad + off[l] + co * ci * 9;
        /* dcur holds dL/d(pre-activation output) of layer l, [co][ny][nx] */
        for (int c2 = 0; c2 < co; ++c2) {
            double sb = 0.0;
            for (size_t p = 0; p < np; ++p) sb += dcur[(size_t)c2 * np + p];
            gb[c2] = sb;
            for (int c1 = 0; c1 < ci; ++c1)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        double s = 0.0;
                        for (int y = 0; y < ny; ++y)
                            for (int x = 0; x < nx; ++x) {
                                int yy = (y + dy + ny) % ny, xx = (x + dx + nx) % nx;
                                s += dcur[((size_t)c2 * ny + y) * nx + x] * in[((size_t)c1 * ny + yy) * nx + xx];
                            }
                        gw[((c2 * ci + c1) * 3 + dy + 1) * 3 + dx + 1] = s;
                    }
        }
        if (l == 0) break;
        /* dL/d(input of layer l) = transposed convolution, then ReLU mask of
         * the previous layer's output */
        for (int c1 = 0; c1 < ci; ++c1)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    double s = 0.0;
                    for (int c2 = 0; c2 < co; ++c2)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                /* input (y, x) feeds output (y - dy, x - dx) via tap (dy, dx) */
                                int yo = (y - dy + ny) % ny, xo = (x - dx + nx) % nx;
                                s += w[((c2 * ci + c1) * 3 + dy + 1) * 3 + dx + 1] *
                                     dcur[((size_t)c2 * ny + yo) * nx + xo];
                            }
                    size_t i = ((size_t)c1 * ny + y) * nx + x;
                    dprev[i] = in[i] > 0.0 ? (bf16_store ? orc_bf16(s) : s) : 0.0;
                }
        double *tmp = dcur;
        dcur = dprev;
        dprev = tmp;
    }
    free(acts);
    free(out2);
    free(ph);
    free(dcur);
    free(dprev);
    free(tin);
    return loss;
}

/* One Adam step (Kingma & Ba 2015) on n parameters, step count t >= 1. */
void orc_adam(double *params, const double *grad, double *m, double *v, int n, int t, double lr, double b1,
              double b2, double eps)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        params[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

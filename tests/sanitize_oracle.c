/*
 * sanitize_oracle.c -- drives every routine of the FP64 oracle on small
 * inputs in one process, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitize.py compiles it together with
 * oracle/*.c using gcc -fsanitize=address,undefined and runs it on the CPU).
 * Any out-of-bounds access, leak, use after free or undefined operation in the
 * oracle makes the run fail.  Test infrastructure only.
 *
 * Sizes cover square and non-square frames, a ragged word count of the packed
 * bits (N not a multiple of 32), pair and eight-level OSPR modes, GS with and
 * without codes, the brute-force DFT, the seed network's forward, backward and
 * Adam step, and the other phase sources.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* the oracle's exported routines (oracle/holo_oracle.c, cnn_oracle.c, phase_oracle.c) */
uint64_t orc_splitmix64_next(uint64_t *state);
void orc_lut_phases(uint64_t n, uint64_t seed, double *phi);
void orc_lut_phasor_field(const double *phi, uint64_t n_lut, uint64_t cursor, uint64_t k, int64_t nx, int64_t ny,
                          double *out);
void orc_dft2_brute(const double *in, int64_t nx, int64_t ny, int sign, double *out);
void orc_fft2(double *data, int64_t nx, int64_t ny, int sign);
double orc_nmse(const double *Iv, const double *W, uint64_t n);
double orc_nmse_direct(const double *Iv, const double *W, uint64_t n);
void orc_nmse_pair(const double *Iv, const float *T, int64_t nx, int64_t ny, double nmse2[2]);
int orc_quant8(double re, double im);
void orc_reconstruct(const void *holo, int levels, int64_t nx, int64_t ny, int n_sf, double *ibar);
void orc_ospr(const float *T, int64_t nx, int64_t ny, int n_sf, const double *phi, uint64_t n_lut, uint64_t cursor,
              uint32_t *bits, double *reH, double *ibar, double *nmse2);
void orc_ospr_mode(const float *T, int64_t nx, int64_t ny, int n_sf, const double *phi, uint64_t n_lut,
                   uint64_t cursor, int mode, void *holo, double *hval, double *ibar, double *nmse2);
void orc_gs(const float *T, int64_t nx, int64_t ny, int n_iter, const double *init, double *nmse_iter,
            double *err_iter, double *final_field, uint8_t *codes, double *nmse_final2);
int orc_cnn_nparams(int C);
void orc_cnn_forward(const double *params, int C, const float *target, int ny, int nx, int bf16_store, double *acts,
                     double *out2, double *phasor);
double orc_cnn_backward(const double *params, int C, const float *target, const double *label, int ny, int nx,
                        int bf16_store, double *grad);
void orc_adam(double *params, const double *grad, double *m, double *v, int n, int t, double lr, double b1,
              double b2, double eps);
void orc_prng_phases(uint64_t seed, uint64_t start, uint64_t n, double *phi);
void orc_codes8_phases(uint64_t n, uint64_t seed, double *phi);
int orc_mseq_phases(uint64_t seed, uint64_t start, uint64_t n, double *phi);

static uint64_t g_state = 12345;
static double uni(void) { return (double)(orc_splitmix64_next(&g_state) >> 11) * 0x1.0p-53; }

static void frame(int64_t nx, int64_t ny, int n_sf, uint64_t n_lut)
{
    const uint64_t n = (uint64_t)(nx * ny), words = (n + 31) / 32;
    float *T = malloc(sizeof(float) * n);
    for (uint64_t p = 0; p < n; ++p) T[p] = (float)uni();
    double *phi = malloc(sizeof(double) * (n_lut ? n_lut : 1));
    orc_lut_phases(n_lut, 1, phi);
    uint32_t *bits = malloc(sizeof(uint32_t) * words * (uint64_t)n_sf);
    double *reh = malloc(sizeof(double) * n * (uint64_t)n_sf);
    double *ibar = malloc(sizeof(double) * n);
    double *ib2 = malloc(sizeof(double) * n);
    double nm[2];
    orc_ospr(T, nx, ny, n_sf, phi, n_lut, 7, bits, reh, ibar, nm);
    orc_reconstruct(bits, 2, nx, ny, n_sf, ib2);
    orc_nmse_pair(ib2, T, nx, ny, nm);
    const int npair = n_sf & ~1;
    if (npair) {
        uint32_t *pb = malloc(sizeof(uint32_t) * words * (uint64_t)npair);
        double *hv = malloc(sizeof(double) * 2 * n * (uint64_t)npair);
        orc_ospr_mode(T, nx, ny, npair, phi, n_lut, 3, 1, pb, hv, ibar, nm);
        free(pb);
        free(hv);
    }
    uint8_t *codes = malloc(n * (uint64_t)n_sf);
    double *hv8 = malloc(sizeof(double) * 2 * n * (uint64_t)n_sf);
    orc_ospr_mode(T, nx, ny, n_sf, phi, n_lut, 5, 2, codes, hv8, ibar, nm);
    orc_reconstruct(codes, 8, nx, ny, n_sf, ib2);
    double *init = malloc(sizeof(double) * 2 * n);
    orc_lut_phasor_field(phi, n_lut, 0, 0, nx, ny, init);
    double gi[3], ge[3], gf[2];
    double *field = malloc(sizeof(double) * 2 * n);
    uint8_t *gc = malloc(n);
    orc_gs(T, nx, ny, 3, init, gi, ge, field, gc, gf);
    orc_gs(T, nx, ny, 2, init, NULL, NULL, NULL, NULL, NULL);
    printf("frame %lldx%lld n_sf %d lut %llu: nmse %.6f gs %.6f\n", (long long)nx, (long long)ny, n_sf,
           (unsigned long long)n_lut, nm[0], gi[2]);
    free(T); free(phi); free(bits); free(reh); free(ibar); free(ib2); free(codes); free(hv8);
    free(init); free(field); free(gc);
}

int main(void)
{
    frame(16, 16, 3, 17);
    frame(8, 4, 2, 5);       /* N = 32: one packed word per sub-frame */
    frame(4, 2, 3, 0);       /* N = 8: a partial word, flat phase */
    frame(32, 8, 1, 1);
    /* transforms: brute force and radix-2 on a non-square field */
    {
        const int64_t nx = 8, ny = 4, n = nx * ny;
        double *a = malloc(sizeof(double) * 2 * n), *b = malloc(sizeof(double) * 2 * n);
        for (int64_t i = 0; i < 2 * n; ++i) a[i] = uni() - 0.5;
        orc_dft2_brute(a, nx, ny, -1, b);
        orc_fft2(a, nx, ny, -1);
        orc_fft2(a, nx, ny, 1);
        double w[32], iv[32];
        for (int i = 0; i < 32; ++i) { w[i] = uni(); iv[i] = uni(); }
        printf("nmse %.6f %.6f quant8 %d\n", orc_nmse(iv, w, 32), orc_nmse_direct(iv, w, 32), orc_quant8(-1.0, 0.1));
        free(a);
        free(b);
    }
    /* seed network: forward, backward, Adam on an 8x8 image with 3 channels */
    {
        const int C = 3, ny = 8, nx = 8, np_ = ny * nx;
        const int n = orc_cnn_nparams(C);
        double *p = malloc(sizeof(double) * n), *g = malloc(sizeof(double) * n);
        double *m = calloc((size_t)n, sizeof(double)), *v = calloc((size_t)n, sizeof(double));
        for (int i = 0; i < n; ++i) p[i] = uni() - 0.5;
        float T[64];
        double lab[128], acts[4 * 3 * 64], out2[128], ph[128];
        for (int i = 0; i < np_; ++i) {
            T[i] = (float)uni();
            lab[2 * i] = 1.0;
            lab[2 * i + 1] = 0.0;
        }
        orc_cnn_forward(p, C, T, ny, nx, 1, acts, out2, ph);
        orc_cnn_forward(p, C, T, ny, nx, 0, NULL, out2, ph);
        double loss = orc_cnn_backward(p, C, T, lab, ny, nx, 0, g);
        orc_adam(p, g, m, v, n, 1, 1e-3, 0.9, 0.999, 1e-8);
        printf("cnn params %d loss %.6f\n", n, loss);
        free(p); free(g); free(m); free(v);
    }
    /* other phase sources */
    {
        double phi[300];
        orc_prng_phases(1, (uint64_t)1 << 63, 300, phi);
        orc_codes8_phases(300, 1, phi);
        int rc = orc_mseq_phases(1, 1000, 300, phi);
        printf("phase sources ok (mseq rc %d)\n", rc);
    }
    puts("SANITIZE_OK");
    return 0;
}

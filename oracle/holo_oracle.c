/*
 * holo_oracle.c -- plain FP64 CPU oracle for LUT phase randomisation in
 * Gerchberg-Saxton (GS) and One-Step Phase-Retrieval (OSPR) hologram
 * generation (Christopher & Wilkinson, "Lookup tables for phase
 * randomisation in hardware generated holograms", arXiv:2004.04049).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP path.
 *
 * Every routine is written for obviousness, not speed: a radix-2 FFT with
 * directly evaluated twiddles, a brute-force DFT for tiny sizes, and the
 * algorithm steps in the order the paper describes them.  Outer loops carry
 * OpenMP pragmas only so that full-size cases finish in seconds; they do not
 * change any arithmetic (each output element is computed by one thread in a
 * fixed order, so results are identical for any thread count).
 *
 * Conventions (readings of the paper where it is silent are marked READING):
 *   - Images are row-major [ny][nx], raster index p = y*nx + x (READING: the
 *     only order under which a LUT as long as one row gives every row the
 *     same phases, as Section 5.2 reports for N_LUT = 256 at 256x256).
 *   - Transforms are the unitary DFT pair of Eq. (1) (forward, e^{-}) and
 *     Eq. (2) (inverse, e^{+}), with the 1/sqrt(NxNy) factor, no fftshift.
 *   - Complex fields are passed as interleaved (re, im) double pairs.
 *
 * Pinned by tests/test_oracle_*.py: brute-force DFT, numpy.fft, closed forms
 * (delta/constant/shift/Parseval/square-wave grating), invariants of the LUT
 * indexing, brute-force nearest-value quantisers, the GS fixed point and the
 * error-reduction property, and finite differences for the CNN routines.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double TWO_PI = 6.283185307179586476925286766559; /* rounds to 2*M_PI */

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number    */
/* generators", OOPSLA 2014): add the golden gamma, then the variant-13      */
/* mixing function.  Used for the LUT contents, which the paper generates    */
/* "at compile time" from a random source (Section 4).                        */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64_next(uint64_t *state)
{
    uint64_t z;
    *state += 0x9E3779B97F4A7C15ull;
    z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* LUT phases phi_j = 2*pi*u_j, u_j = (x_j >> 11) * 2^-53, j = 0..n-1: uniform
 * on [0, 2*pi) as the workload specifies; the product is one correctly rounded
 * FP64 multiply, so the phases are bit-reproducible.  n = 0 means no table:
 * flat phase (READING of "error is very high when N_LUT is 0", Section 5.2). */
void orc_lut_phases(uint64_t n, uint64_t seed, double *phi)
{
    uint64_t s = seed;
    for (uint64_t j = 0; j < n; ++j) {
        uint64_t x = orc_splitmix64_next(&s);
        double u = (double)(x >> 11) * 0x1.0p-53;
        phi[j] = TWO_PI * u;
    }
}

/* Cyclic LUT address (Section 5, Fig. 3): the pool is read sequentially and
 * successive sub-frames and frames continue where the previous left off, so
 * sub-frame k of a frame that starts at cursor c reads, for raster pixel p,
 * entry (c + k*N + p) mod N_LUT, N = nx*ny.  Computed without overflow. */
uint64_t orc_lut_index(uint64_t cursor, uint64_t k, uint64_t npix, uint64_t p, uint64_t n_lut)
{
    if (n_lut == 0) return 0;
    unsigned __int128 i = (unsigned __int128)cursor + (unsigned __int128)k * npix + p;
    return (uint64_t)(i % n_lut);
}

/* Unit phasor field for one sub-frame: out[p] = exp(i*phi_{index(p)}), or 1 for
 * the flat-phase case n_lut == 0. */
void orc_lut_phasor_field(const double *phi, uint64_t n_lut, uint64_t cursor, uint64_t k,
                          int64_t nx, int64_t ny, double *out /* [2N] */)
{
    uint64_t npix = (uint64_t)(nx * ny);
    for (uint64_t p = 0; p < npix; ++p) {
        double a = 0.0;
        if (n_lut) a = phi[orc_lut_index(cursor, k, npix, p, n_lut)];
        out[2 * p] = cos(a);
        out[2 * p + 1] = sin(a);
    }
}

/* ------------------------------------------------------------------------ */
/* Eq. (1)/(2) by direct summation: F_{u,v} = 1/sqrt(NxNy) sum_{x,y} f_{x,y}  */
/* exp(sign*2*pi*i*(ux/Nx + vy/Ny)).  sign = -1 is Eq. (1), +1 is Eq. (2).    */
/* The phase is reduced exactly as integers before scaling.  Tiny sizes only. */
/* ------------------------------------------------------------------------ */
void orc_dft2_brute(const double *in, int64_t nx, int64_t ny, int sign, double *out)
{
    const double scale = 1.0 / sqrt((double)nx * (double)ny);
    for (int64_t v = 0; v < ny; ++v)
        for (int64_t u = 0; u < nx; ++u) {
            cplx acc = 0.0;
            for (int64_t y = 0; y < ny; ++y)
                for (int64_t x = 0; x < nx; ++x) {
                    /* ux/Nx + vy/Ny = ((ux mod Nx)*Ny + (vy mod Ny)*Nx) / (Nx*Ny) */
                    int64_t num = ((u * x) % nx) * ny + ((v * y) % ny) * nx;
                    double ang = sign * TWO_PI * (double)num / ((double)nx * (double)ny);
                    cplx f = in[2 * (y * nx + x)] + I * in[2 * (y * nx + x) + 1];
                    acc += f * (cos(ang) + I * sin(ang));
                }
            out[2 * (v * nx + u)] = creal(acc) * scale;
            out[2 * (v * nx + u) + 1] = cimag(acc) * scale;
        }
}

/* In-place unscaled radix-2 decimation-in-time FFT of n = 2^k points with
 * stride `stride`; kernel exp(sign*2*pi*i*j*k/n).  Twiddles are evaluated
 * directly from cos/sin of 2*pi*j/n (never by recurrence). */
static void fft1d(cplx *a, int64_t n, int64_t stride, int sign, cplx *tmp)
{
    for (int64_t i = 0; i < n; ++i) tmp[i] = a[i * stride];
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < n; ++i) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = tmp[i]; tmp[i] = tmp[j]; tmp[j] = t; }
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len >> 1;
        for (int64_t j = 0; j < half; ++j) {
            double ang = sign * TWO_PI * (double)j / (double)len;
            cplx w = cos(ang) + I * sin(ang);
            for (int64_t i = 0; i < n; i += len) {
                cplx e = tmp[i + j], o = tmp[i + j + half] * w;
                tmp[i + j] = e + o;
                tmp[i + j + half] = e - o;
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) a[i * stride] = tmp[i];
}

/* Unitary 2D FFT of a [ny][nx] field, in place (Eq. (1) for sign = -1,
 * Eq. (2) for sign = +1): rows, then columns, then one 1/sqrt(NxNy) scale.
 * nx and ny must be powers of two. */
void orc_fft2(double *data, int64_t nx, int64_t ny, int sign)
{
    cplx *a = (cplx *)data;
    const double scale = 1.0 / sqrt((double)nx * (double)ny);
    #pragma omp parallel
    {
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)(nx > ny ? nx : ny));
        #pragma omp for schedule(static)
        for (int64_t y = 0; y < ny; ++y) fft1d(a + y * nx, nx, 1, sign, tmp);
        #pragma omp for schedule(static)
        for (int64_t x = 0; x < nx; ++x) fft1d(a + x, ny, nx, sign, tmp);
        #pragma omp for schedule(static)
        for (int64_t p = 0; p < nx * ny; ++p) a[p] *= scale;
        free(tmp);
    }
}

/* ------------------------------------------------------------------------ */
/* Error metric.  The paper reports "time averaged errors" as MSE without    */
/* defining it (Section 5.2).  READING: the optimal-scale intensity NMSE     */
/*   NMSE(I, W) = min_a ||a*I - W||^2 / ||W||^2 = 1 - S_IW^2 / (S_II * S_WW)  */
/* with W the target intensity T^2; it is scale-free and lies in [0, 1].     */
/* ------------------------------------------------------------------------ */
double orc_nmse(const double *Iv, const double *W, uint64_t n)
{
    double s_iw = 0.0, s_ii = 0.0, s_ww = 0.0;
    for (uint64_t p = 0; p < n; ++p) {
        s_iw += Iv[p] * W[p];
        s_ii += Iv[p] * Iv[p];
        s_ww += W[p] * W[p];
    }
    if (s_ii == 0.0 || s_ww == 0.0) return 1.0;
    return 1.0 - (s_iw * s_iw) / (s_ii * s_ww);
}

/* The same quantity by its definition: best scale a* = S_IW/S_II, then the
 * residual norm.  Kept as a self-check of the closed form. */
double orc_nmse_direct(const double *Iv, const double *W, uint64_t n)
{
    double s_iw = 0.0, s_ii = 0.0, s_ww = 0.0, r = 0.0;
    for (uint64_t p = 0; p < n; ++p) { s_iw += Iv[p] * W[p]; s_ii += Iv[p] * Iv[p]; s_ww += W[p] * W[p]; }
    double a = (s_ii > 0.0) ? s_iw / s_ii : 0.0;
    for (uint64_t p = 0; p < n; ++p) { double d = a * Iv[p] - W[p]; r += d * d; }
    return (s_ww > 0.0) ? r / s_ww : 1.0;
}

/* Target intensity T^2 and its point-symmetrised form
 * Ts^2(u,v) = (T^2(u,v) + T^2(-u mod nx, -v mod ny)) / 2.  A binary (real)
 * hologram has a centro-symmetric replay, so Ts^2 is the best it can reach. */
static void target_intensities(const float *T, int64_t nx, int64_t ny, double *t2, double *ts2)
{
    for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
            double a = (double)T[y * nx + x];
            double b = (double)T[((ny - y) % ny) * nx + (nx - x) % nx];
            t2[y * nx + x] = a * a;
            ts2[y * nx + x] = 0.5 * (a * a + b * b);
        }
}

/* NMSE of an intensity against T^2 and against Ts^2. */
void orc_nmse_pair(const double *Iv, const float *T, int64_t nx, int64_t ny, double nmse2[2])
{
    uint64_t n = (uint64_t)(nx * ny);
    double *t2 = (double *)malloc(sizeof(double) * n);
    double *ts2 = (double *)malloc(sizeof(double) * n);
    target_intensities(T, nx, ny, t2, ts2);
    nmse2[0] = orc_nmse(Iv, t2, n);
    nmse2[1] = orc_nmse(Iv, ts2, n);
    free(t2);
    free(ts2);
}

/* ------------------------------------------------------------------------ */
/* Quantisers: each pixel becomes the nearest value the SLM allows          */
/* (Section 2, "initial hologram").                                           */
/* ------------------------------------------------------------------------ */
/* Binary phase {0, pi} = {+1, -1}: |H-1|^2 - |H+1|^2 = -4 Re H, so the nearest
 * is -1 exactly when Re H < 0.  READING: the tie Re H = 0 goes to +1.
 * Returns the bit (1 = phase pi). */
int orc_binarise(double re) { return re < 0.0 ? 1 : 0; }

/* Eight phase levels exp(i*2*pi*m/8): theta = arg H in [0, 2*pi), m =
 * floor(8*theta/(2*pi) + 1/2) mod 8.  H = 0 gives m = 0. */
int orc_quant8(double re, double im)
{
    double th = atan2(im, re);
    if (th < 0.0) th += TWO_PI;
    int m = (int)floor(8.0 * th / TWO_PI + 0.5);
    return m & 7;
}

/* ------------------------------------------------------------------------ */
/* Reconstruction: replay field R' = F{H'} of a quantised hologram (Section  */
/* 2), its intensity, time-averaged over sub-frames (Section 3).             */
/*   levels == 2: holo is packed bits, uint32[n_sf][ceil(N/32)], bit p%32 of  */
/*                word p/32 (LSB first, raster order); 1 = phase pi.          */
/*   levels == 8: holo is uint8 codes m in 0..7, [n_sf][N].                   */
/* ibar[N] receives (1/n_sf) * sum_k |F{H'_k}|^2 in unitary units.            */
/* ------------------------------------------------------------------------ */
void orc_reconstruct(const void *holo, int levels, int64_t nx, int64_t ny, int n_sf, double *ibar)
{
    uint64_t n = (uint64_t)(nx * ny), words = (n + 31) / 32;
    double *f = (double *)malloc(sizeof(double) * 2 * n);
    memset(ibar, 0, sizeof(double) * n);
    for (int k = 0; k < n_sf; ++k) {
        for (uint64_t p = 0; p < n; ++p) {
            if (levels == 2) {
                const uint32_t *w = (const uint32_t *)holo + (uint64_t)k * words;
                int b = (w[p >> 5] >> (p & 31)) & 1u;
                f[2 * p] = b ? -1.0 : 1.0;
                f[2 * p + 1] = 0.0;
            } else {
                int m = ((const uint8_t *)holo)[(uint64_t)k * n + p] & 7;
                f[2 * p] = cos(TWO_PI * m / 8.0);
                f[2 * p + 1] = sin(TWO_PI * m / 8.0);
            }
        }
        orc_fft2(f, nx, ny, -1);
        for (uint64_t p = 0; p < n; ++p)
            ibar[p] += (f[2 * p] * f[2 * p] + f[2 * p + 1] * f[2 * p + 1]) / (double)n_sf;
    }
    free(f);
}

/* ------------------------------------------------------------------------ */
/* OSPR (Section 2 and 3; Cable et al. 2004): for each of n_sf sub-frames,   */
/* randomise the target's phase from the LUT, back-propagate with Eq. (2),   */
/* binarise to the nearest of {+1, -1}, and time-average the replay          */
/* intensities |F{H'_k}|^2 of Eq. (1).                                        */
/*   bits  [n_sf][ceil(N/32)]  packed binary holograms (required)            */
/*   reH   [n_sf][N] or NULL   Re H before binarisation (unitary units)      */
/*   ibar  [N] or NULL          time-averaged replay intensity                 */
/*   nmse2 [2] or NULL          {NMSE vs T^2, NMSE vs Ts^2}                    */
/* The frame starts at LUT cursor `cursor`; the caller advances it by         */
/* n_sf*N afterwards (Section 5: frames continue where the last left off).   */
/* ------------------------------------------------------------------------ */
void orc_ospr(const float *T, int64_t nx, int64_t ny, int n_sf, const double *phi, uint64_t n_lut,
              uint64_t cursor, uint32_t *bits, double *reH, double *ibar, double *nmse2)
{
    uint64_t n = (uint64_t)(nx * ny), words = (n + 31) / 32;
    double *h = (double *)malloc(sizeof(double) * 2 * n);
    double *ph = (double *)malloc(sizeof(double) * 2 * n);
    memset(bits, 0, sizeof(uint32_t) * words * (uint64_t)n_sf);
    for (int k = 0; k < n_sf; ++k) {
        /* R = T * exp(i*phi): target amplitude with LUT-randomised phase */
        orc_lut_phasor_field(phi, n_lut, cursor, (uint64_t)k, nx, ny, ph);
        for (uint64_t p = 0; p < n; ++p) {
            h[2 * p] = (double)T[p] * ph[2 * p];
            h[2 * p + 1] = (double)T[p] * ph[2 * p + 1];
        }
        /* H = F^{-1}{R} */
        orc_fft2(h, nx, ny, +1);
        uint32_t *w = bits + (uint64_t)k * words;
        for (uint64_t p = 0; p < n; ++p) {
            if (reH) reH[(uint64_t)k * n + p] = h[2 * p];
            if (orc_binarise(h[2 * p])) w[p >> 5] |= 1u << (p & 31);
        }
    }
    free(h);
    free(ph);
    double *ib = ibar ? ibar : (double *)malloc(sizeof(double) * n);
    orc_reconstruct(bits, 2, nx, ny, n_sf, ib);
    if (nmse2) orc_nmse_pair(ib, T, nx, ny, nmse2);
    if (!ibar) free(ib);
}

/* ------------------------------------------------------------------------ */
/* OSPR variants (not from the paper; they change how sub-frames are drawn    */
/* from the randomised fields, the pool is read as in orc_ospr):              */
/*   mode 1, pairs: field j = 0..n_sf/2-1 reads the pool at k = j; its        */
/*     H_j = F^{-1}{T exp(i phi)} gives two binary sub-frames, 2j from Re H_j */
/*     and 2j+1 from Im H_j (nearest of {+1, -1} to each part); holo is       */
/*     packed bits as in orc_ospr, hval[k][p] the decided value (Re or Im).    */
/*   mode 2, eight levels: sub-frame k reads the pool at k and is quantised   */
/*     to the nearest of exp(i*2*pi*m/8) (orc_quant8); holo is uint8 codes    */
/*     [n_sf][N], hval[k][2p..2p+1] = H_k.                                    */
/* Then the time-averaged replay of the quantised sub-frames and the NMSE     */
/* pair, as for the binary frame.  n_sf must be even in mode 1.              */
/* ------------------------------------------------------------------------ */
void orc_ospr_mode(const float *T, int64_t nx, int64_t ny, int n_sf, const double *phi, uint64_t n_lut,
                   uint64_t cursor, int mode, void *holo, double *hval, double *ibar, double *nmse2)
{
    uint64_t n = (uint64_t)(nx * ny), words = (n + 31) / 32;
    double *h = (double *)malloc(sizeof(double) * 2 * n);
    double *ph = (double *)malloc(sizeof(double) * 2 * n);
    int n_fields = mode == 1 ? n_sf / 2 : n_sf;
    if (mode == 1) memset(holo, 0, sizeof(uint32_t) * words * (uint64_t)n_sf);
    for (int j = 0; j < n_fields; ++j) {
        orc_lut_phasor_field(phi, n_lut, cursor, (uint64_t)j, nx, ny, ph);
        for (uint64_t p = 0; p < n; ++p) {
            h[2 * p] = (double)T[p] * ph[2 * p];
            h[2 * p + 1] = (double)T[p] * ph[2 * p + 1];
        }
        orc_fft2(h, nx, ny, +1);
        if (mode == 1) {
            uint32_t *wr = (uint32_t *)holo + (uint64_t)(2 * j) * words;
            uint32_t *wi = (uint32_t *)holo + (uint64_t)(2 * j + 1) * words;
            for (uint64_t p = 0; p < n; ++p) {
                if (hval) {
                    hval[(uint64_t)(2 * j) * n + p] = h[2 * p];
                    hval[(uint64_t)(2 * j + 1) * n + p] = h[2 * p + 1];
                }
                if (orc_binarise(h[2 * p])) wr[p >> 5] |= 1u << (p & 31);
                if (orc_binarise(h[2 * p + 1])) wi[p >> 5] |= 1u << (p & 31);
            }
        } else {
            uint8_t *c = (uint8_t *)holo + (uint64_t)j * n;
            for (uint64_t p = 0; p < n; ++p) {
                if (hval) {
                    hval[2 * ((uint64_t)j * n + p)] = h[2 * p];
                    hval[2 * ((uint64_t)j * n + p) + 1] = h[2 * p + 1];
                }
                c[p] = (uint8_t)orc_quant8(h[2 * p], h[2 * p + 1]);
            }
        }
    }
    free(h);
    free(ph);
    double *ib = ibar ? ibar : (double *)malloc(sizeof(double) * n);
    orc_reconstruct(holo, mode == 1 ? 2 : 8, nx, ny, n_sf, ib);
    if (nmse2) orc_nmse_pair(ib, T, nx, ny, nmse2);
    if (!ibar) free(ib);
}

/* ------------------------------------------------------------------------ */
/* Gerchberg-Saxton (Section 2; Gerchberg & Saxton 1972) with a phase-only   */
/* hologram constraint and an amplitude-only replay constraint.              */
/*   R_0 = T * init/|init|            (init = 0 -> 1)                         */
/*   repeat i = 1..n_iter:                                                    */
/*     H_i  = F^{-1}{R_{i-1}};  H'_i = H_i/|H_i|  (H = 0 -> 1)               */
/*     R'_i = F{H'_i};  record NMSE(|R'_i|^2, T^2) and the amplitude error     */
/*          E_i = sum (|R'_i| - Te)^2, Te = T*sqrt(N / sum T^2)               */
/*     R_i  = T * R'_i/|R'_i|          (R' = 0 -> T)                          */
/*   codes = 8-level quantisation of H_n; replay of the codes; its NMSE pair. */
/* The LUT seeds only R_0 (READING: the paper's GS constraints in Section 8   */
/* concern the initial random phase).                                         */
/*   init    [2N] phasor field (need not be normalised)                       */
/*   nmse_iter/err_iter [n_iter] or NULL; final_field [2N] or NULL gets R'_n  */
/*   codes [N] or NULL; nmse_final2 [2] or NULL (NMSE pair of the codes)      */
/* ------------------------------------------------------------------------ */
void orc_gs(const float *T, int64_t nx, int64_t ny, int n_iter, const double *init,
            double *nmse_iter, double *err_iter, double *final_field, uint8_t *codes,
            double *nmse_final2)
{
    uint64_t n = (uint64_t)(nx * ny);
    double *r = (double *)malloc(sizeof(double) * 2 * n);
    double *h = (double *)malloc(sizeof(double) * 2 * n);
    double *t2 = (double *)malloc(sizeof(double) * n);
    double *iv = (double *)malloc(sizeof(double) * n);
    double sum_t2 = 0.0;
    for (uint64_t p = 0; p < n; ++p) { t2[p] = (double)T[p] * (double)T[p]; sum_t2 += t2[p]; }
    const double te_scale = sum_t2 > 0.0 ? sqrt((double)n / sum_t2) : 0.0;

    for (uint64_t p = 0; p < n; ++p) {
        double a = init[2 * p], b = init[2 * p + 1], m = sqrt(a * a + b * b);
        double c = m > 0.0 ? a / m : 1.0, s = m > 0.0 ? b / m : 0.0;
        r[2 * p] = (double)T[p] * c;
        r[2 * p + 1] = (double)T[p] * s;
    }
    for (int it = 0; it < n_iter; ++it) {
        memcpy(h, r, sizeof(double) * 2 * n);
        orc_fft2(h, nx, ny, +1);                         /* H = F^{-1}{R} */
        if (it == n_iter - 1 && codes)
            for (uint64_t p = 0; p < n; ++p) codes[p] = (uint8_t)orc_quant8(h[2 * p], h[2 * p + 1]);
        for (uint64_t p = 0; p < n; ++p) {               /* phase-only hologram */
            double a = h[2 * p], b = h[2 * p + 1], m = sqrt(a * a + b * b);
            h[2 * p] = m > 0.0 ? a / m : 1.0;
            h[2 * p + 1] = m > 0.0 ? b / m : 0.0;
        }
        orc_fft2(h, nx, ny, -1);                         /* R' = F{H'} */
        double err = 0.0;
        for (uint64_t p = 0; p < n; ++p) {
            double a = h[2 * p], b = h[2 * p + 1];
            iv[p] = a * a + b * b;
            double d = sqrt(iv[p]) - (double)T[p] * te_scale;
            err += d * d;
        }
        if (nmse_iter) nmse_iter[it] = orc_nmse(iv, t2, n);
        if (err_iter) err_iter[it] = err;
        for (uint64_t p = 0; p < n; ++p) {               /* amplitude replacement */
            double a = h[2 * p], b = h[2 * p + 1], m = sqrt(a * a + b * b);
            r[2 * p] = m > 0.0 ? (double)T[p] * a / m : (double)T[p];
            r[2 * p + 1] = m > 0.0 ? (double)T[p] * b / m : 0.0;
        }
    }
    if (final_field) memcpy(final_field, h, sizeof(double) * 2 * n);
    if (codes && nmse_final2) {
        orc_reconstruct(codes, 8, nx, ny, 1, iv);
        orc_nmse_pair(iv, T, nx, ny, nmse_final2);
    }
    free(r); free(h); free(t2); free(iv);
}

/* Threads the OpenMP loops above use (reported with CPU timings); setting
 * them changes scheduling only, never a result. */
#ifdef _OPENMP
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
int orc_num_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif

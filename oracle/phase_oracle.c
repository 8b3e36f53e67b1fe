/*
 * phase_oracle.c -- plain FP64 CPU oracle for the phase sources compared
 * against the LUT: the software route of Section 4 (a PRNG plus trigonometric
 * functions), the M-sequence route of Section 7 (a shift-register sequence
 * feeding sine/cosine tables), and an 8-bit-code table.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP path:
 * the M-sequence is stepped one bit at a time by its recurrence, where the
 * library jumps through polynomial arithmetic.
 *
 * Every source fills "pool positions" i = start .. start+n-1 with a phase;
 * an OSPR frame starting at cursor c reads position c + k*N + p for pixel p
 * of sub-frame k (Section 5, Fig. 3), exactly as with a table.
 *
 * Pinned by tests/test_oracle_phase_sources.py: SplitMix64 against its
 * sequential form (itself pinned to a published vector), the M-sequence
 * against a hand-derived impulse response of its recurrence, the
 * primitivity of x^31 + x^3 + 1 in independent GF(2) arithmetic (so the
 * period is 2^31 - 1), and code/phase assembly against worked examples.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static const double TWO_PI_P = 6.283185307179586476925286766559;

/* SplitMix64 output i of the stream seeded with `seed`, directly: the state
 * after i+1 additions of the golden gamma, then the variant-13 finaliser
 * (Steele, Lea & Flood, OOPSLA 2014). */
static uint64_t splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64_at(uint64_t seed, uint64_t i) { return splitmix64_at(seed, i); }

/* PRNG source: phi_i = 2*pi * (x_i >> 40) / 2^24, the top 24 bits of the
 * SplitMix64 output x_i as a fraction of a turn. */
void orc_prng_phases(uint64_t seed, uint64_t start, uint64_t n, double *phi)
{
    for (uint64_t j = 0; j < n; ++j) {
        uint64_t x = splitmix64_at(seed, start + j);
        phi[j] = TWO_PI_P * ((double)(x >> 40) / 16777216.0);
    }
}

/* 8-bit-code table: code q_j = x_j >> 56 (top byte of SplitMix64 output j),
 * phase 2*pi*q_j/256. */
void orc_codes8_phases(uint64_t n, uint64_t seed, double *phi)
{
    for (uint64_t j = 0; j < n; ++j) {
        unsigned q = (unsigned)(splitmix64_at(seed, j) >> 56);
        phi[j] = TWO_PI_P * ((double)q / 256.0);
    }
}

/* M-sequence bits of x^31 + x^3 + 1: s_0..s_30 are bits 30..0 of `window`,
 * then s_{m+31} = s_{m+3} xor s_m, i.e. s_n = s_{n-28} xor s_{n-31}. */
void orc_mseq_bits(uint32_t window, uint64_t nbits, uint8_t *s)
{
    for (uint64_t j = 0; j < 31 && j < nbits; ++j) s[j] = (uint8_t)((window >> (30 - j)) & 1u);
    for (uint64_t k = 31; k < nbits; ++k) s[k] = s[k - 28] ^ s[k - 31];
}

/* Codes of positions start..start+n-1 from a given window: q_i collects bits
 * s_{8i} .. s_{8i+7}, the first one most significant. */
int orc_mseq_codes(uint32_t window, uint64_t start, uint64_t n, uint8_t *codes)
{
    uint64_t nbits = 8 * (start + n);
    uint8_t *s = (uint8_t *)malloc(nbits ? nbits : 1);
    if (!s) return -1;
    orc_mseq_bits(window, nbits, s);
    for (uint64_t i = 0; i < n; ++i) {
        unsigned q = 0;
        for (int j = 0; j < 8; ++j) q = (q << 1) | s[8 * (start + i) + (uint64_t)j];
        codes[i] = (uint8_t)q;
    }
    free(s);
    return 0;
}

/* The M-sequence source of a seed: window = (SplitMix64 output 0) mod 2^31
 * (1 if that is 0); phases 2*pi*q_i/256. */
uint32_t orc_mseq_window(uint64_t seed)
{
    uint32_t w = (uint32_t)(splitmix64_at(seed, 0) & 0x7FFFFFFFull);
    return w ? w : 1u;
}

int orc_mseq_phases(uint64_t seed, uint64_t start, uint64_t n, double *phi)
{
    uint8_t *q = (uint8_t *)malloc(n ? n : 1);
    if (!q) return -1;
    if (orc_mseq_codes(orc_mseq_window(seed), start, n, q)) {
        free(q);
        return -1;
    }
    for (uint64_t i = 0; i < n; ++i) phi[i] = TWO_PI_P * ((double)q[i] / 256.0);
    free(q);
    return 0;
}

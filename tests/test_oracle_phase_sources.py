"""Pins for the oracle's other phase sources: the software route of Section 3
(a PRNG with trigonometric functions), the M-sequence route of Section 7
(a shift-register sequence with sine/cosine tables) and the 8-bit-code
table.  CPU only."""
import numpy as np

import synth

M31 = (1 << 31) - 1
POLY = (1 << 31) | (1 << 3) | 1     # x^31 + x^3 + 1


def _seq(seed, n):
    return [int(v) for v in synth.splitmix64_stream(seed, n)]


def test_prng_counter_form_matches_sequential_stream(orc):
    # the counter form must give output i of the stream (pinned against the
    # published vector in test_oracle_lut.py), not output i+1 or i-1
    seq = _seq(99, 600)
    assert [orc.splitmix64_at(99, i) for i in range(600)] == seq
    phi = orc.prng_phases(99, 100, 500)
    turns = phi / (2 * np.pi) * 2.0 ** 24
    assert np.array_equal(np.round(turns), [x >> 40 for x in seq[100:600]])
    assert np.abs(turns - np.round(turns)).max() < 1e-6     # 24-bit phase grid
    assert phi.min() >= 0 and phi.max() < 2 * np.pi


def test_codes8_are_top_bytes(orc):
    seq = _seq(5, 2000)
    phi = orc.codes8_phases(2000, 5)
    q = phi / (2 * np.pi) * 256
    assert np.abs(q - np.round(q)).max() < 1e-9              # multiples of 2*pi/256
    assert np.array_equal(np.round(q).astype(int), [x >> 56 for x in seq])
    h = np.bincount(np.round(q).astype(int) // 32, minlength=8)         # roughly uniform
    assert h.min() > 180 and h.max() < 330


def test_mseq_impulse_response_by_hand(orc):
    # window with only s_30 set.  The recurrence s_n = s_{n-28} xor s_{n-31}
    # is 0 until s_58 = s_30; s_61 = s_33 xor s_30 = 1; s_86 = s_58 xor s_55 = 1;
    # s_89 = s_61 xor s_58 = 0; s_92 = s_64 xor s_61 = 1; all else below 93 is 0.
    s = orc.mseq_bits(1, 93)
    assert list(np.nonzero(s)[0]) == [30, 58, 61, 86, 92]
    # codes take 8 bits, the first most significant: s_30 is bit 6 of code 3
    # (value 2); s_58, s_61 are bits 2 and 5 of code 7 (32 + 4); s_86 is bit 6
    # of code 10 (2); s_92 is bit 4 of code 11 (8)
    assert list(orc.mseq_codes(1, 0, 12)) == [0, 0, 0, 2, 0, 0, 0, 36, 0, 0, 2, 8]
    assert list(orc.mseq_codes(1, 7, 5)) == [36, 0, 0, 2, 8]     # an offset start reads the same bits


def _gf2_mulmod(a, b, m):
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a >> 31 & 1:
            a ^= m
    return r


def test_trinomial_is_primitive():
    # x^31 + x^3 + 1 has no root in GF(2) (P(0) = P(1) = 1) and x^(2^31) = x
    # mod P; with 31 prime this makes P irreducible, and since 2^31 - 1 is
    # prime every element but 1 of GF(2^31)* -- x included -- has order
    # 2^31 - 1: the sequence period
    x = 2
    y = x
    for _ in range(31):
        y = _gf2_mulmod(y, y, POLY)
    assert y == x
    z = x
    for _ in range(30):
        z = _gf2_mulmod(z, z, POLY)
    assert z != x                                            # and not already at 2^30


def test_mseq_is_the_sequence_of_the_trinomial(orc):
    # Independent route: any fixed linear read-out of x^n * S mod P is a
    # sequence with characteristic polynomial P.  With the read-out
    # "coefficient of x^30" and S chosen so the first 31 read-outs are the
    # window, the two must agree everywhere.
    w = orc.mseq_window(2024)
    s = orc.mseq_bits(w, 4000)
    # S with read-outs s_0..s_30: bits 30..3 are s_0..s_27 and the last three
    # fold in s_28..s_30 (x^j * S for j = 28..30 wraps once)
    S = (w & ~7) | ((w >> 28) ^ w) & 7
    st = S
    for n in range(4000):
        assert (st >> 30) & 1 == s[n], n
        st = _gf2_mulmod(st, 2, POLY)


def test_mseq_window_from_seed(orc):
    for seed in (1, 7, 2024):
        w = _seq(seed, 1)[0] & M31
        assert orc.mseq_window(seed) == (w if w else 1)
    ph = orc.mseq_phases(7, 1000, 300)
    q = ph / (2 * np.pi) * 256
    assert np.abs(q - np.round(q)).max() < 1e-9
    assert np.array_equal(np.round(q).astype(np.uint8), orc.mseq_codes(orc.mseq_window(7), 1000, 300))

"""The paper's LUT-length findings (Section 5.2, Figs. 4-5) as asserted checks
on the FP64 oracle (CPU, 64x64 frames so the sweep takes seconds).

Binary OSPR, 24 sub-frames, six seeded blob/rectangle targets (standing in for
the paper's test images) chained through one pool, several pool seeds per
length; added error = mean NMSE / mean NMSE of the non-repeating pool - 1.
Checked:
  * a pool no longer than the sub-frame count gives a very large error
    (2 <= 24: well above 50%);
  * a pool exactly one row long (N_LUT = nx) spikes: every row (and every
    sub-frame) gets the same phases, so it is far worse than the primes on
    either side of it;
  * the paper's N_LUT = 10007 adds less than 5%.
The GPU counterpart at the paper's 256x256 size is tests/test_gpu_lut_claims.py.
"""
import numpy as np

import synth

N, NSF, NT, SEEDS = 64, 24, 6, 4


def _added(orc, lengths):
    targets = [synth.blob_target(N, N, synth.SEED_LUT_STUDY0 + i) for i in range(NT)]
    full = N * N * NSF * NT
    res = {}
    for L in list(lengths) + ["nonrepeating"]:
        length = full if L == "nonrepeating" else L
        per_seed = []
        for s in range(SEEDS):
            phi = orc.lut_phases(length, 1 + s)
            cur = 0
            nm = []
            for t in targets:
                nm.append(orc.ospr(t, NSF, phi, length, cur, want_reh=False, want_ibar=False)["nmse2"])
                cur += N * N * NSF
            per_seed.append(np.mean(nm, axis=0))
        res[L] = np.mean(per_seed, axis=0)
    ref = res.pop("nonrepeating")
    return {L: 100 * (m / ref - 1) for L, m in res.items()}


def test_section_5_2_claims_on_the_oracle(orc):
    added = _added(orc, [2, 61, 64, 67, 10007])
    print({L: [round(v, 2) for v in a] for L, a in added.items()})
    nm = {L: a[0] for L, a in added.items()}          # full-frame NMSE
    assert nm[2] > 50.0
    assert nm[64] > 2 * max(nm[61], nm[67])
    assert nm[64] > 50.0
    assert abs(nm[10007]) < 5.0

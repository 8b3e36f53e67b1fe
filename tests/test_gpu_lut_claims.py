"""The paper's LUT-length findings (Section 5.2, Figs. 4-5) at its own frame
size, 256x256, on the library's batched path (GPU).

Binary OSPR, 24 sub-frames, six seeded blob/rectangle targets chained through
one pool per call, 16 pool seeds per length; added error = mean NMSE / mean
NMSE of the non-repeating pool (every pixel of every sub-frame its own entry)
- 1.  Checked:
  * pools no longer than the sub-frame count (2, 23 <= 24) give very large
    errors;
  * N_LUT = nx = 256 spikes: every row gets the same phases, so it is worse
    than the primes 251 and 263 on either side;
  * the paper's N_LUT = 10007 adds less than 5% (full-frame NMSE).
"""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def test_section_5_2_claims_at_256():
    import paper_2004_04049_amd as h
    from paper_2004_04049_amd import lut_study
    n, nsf = 256, 24
    targets = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_LUT_STUDY0 + i)).cuda() for i in range(6)]
    print("lut claims 256x256: sweep", flush=True)
    res = lut_study.sweep(targets, nsf, [2, 23, 251, 256, 263, 10007], 16)
    sm = lut_study.summarize(res, n, nsf)
    added = {r["n_lut"]: r["added_pct"] for r in sm["rows"]}
    added_sym = {r["n_lut"]: r["added_sym_pct"] for r in sm["rows"]}
    print("added error % (NMSE):", {k: round(v, 2) for k, v in added.items()})
    print("added error % (NMSE_sym):", {k: round(v, 2) for k, v in added_sym.items()})
    assert added[2] > 50.0 and added[23] > 50.0
    # (measured: 256 -> +122%, 251 -> +82%, 263 -> +71%; the neighbours sit
    # on the shoulder of the spike, which the paper also reports near
    # multiples of the resolution)
    assert added[256] > 1.2 * max(added[251], added[263]) and added[256] > 100.0
    assert abs(added[10007]) < 5.0

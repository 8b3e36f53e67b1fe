"""LUT-length study (Section 5.2, Figs. 4-5): time-averaged error of binary OSPR
frames as a function of the phase-pool length N_LUT, on seeded synthetic
targets standing in for the paper's test images.

For every hologram side n, prime N_LUT and LUT seed, the library generates one
batch of frames (one per target, 24 sub-frames each, cursor chained across the
batch as Section 5 prescribes) with `holo_ospr_generate_batched` and returns
their NMSE pair; the reference is the non-repeating pool (N_LUT = n*n*n_sf:
every pixel of every sub-frame gets its own phase, the PRNG-equivalent case of
Section 5.1).  The added error of a pool length is mean NMSE / mean NMSE of the
reference - 1, averaged over targets and seeds.  All arithmetic runs in the
library; this module only sequences calls and keeps the books.

Run:  python -m paper_2004_04049_amd.lut_study --sizes 64,128,256 --seeds 100
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import FP32, Lut, lut_check, ospr_generate_batched, set_graphs


def primes_upto(n: int):
    sieve = np.ones(n + 1, dtype=bool)
    sieve[:2] = False
    for i in range(2, int(n ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = False
    return np.nonzero(sieve)[0]


def default_primes(n: int, hi: int = 100003):
    """About 40 log-spaced primes up to `hi`, the paper's 10007, and the
    primes next to n, n/2 and 2n (where the paper sees error spikes)."""
    ps = primes_upto(hi)
    picks = set(int(ps[np.searchsorted(ps, v)]) for v in np.geomspace(2, hi, 40))
    picks.add(10007)
    for m in (n // 2, n, 2 * n, 4 * n):
        i = np.searchsorted(ps, m)
        picks.update(int(p) for p in ps[max(i - 1, 0):i + 1])
    return sorted(picks)


def sweep(targets, n_sf: int, primes, n_seeds: int, seed0: int = 1, precision: int = FP32):
    """targets: list of cuda float32 [n, n].  Returns {N_LUT: (mean NMSE pair,
    std of the per-seed mean pair)} including the non-repeating reference under
    the key "nonrepeating"."""
    n = targets[0].shape[0]
    nsfs = [n_sf] * len(targets)
    bits = [torch.empty((n_sf, n * n // 32), dtype=torch.int32, device=targets[0].device) for _ in targets]
    out = {}
    for p in list(primes) + ["nonrepeating"]:
        length = n * n * n_sf * len(targets) if p == "nonrepeating" else int(p)
        per_seed = []
        for s in range(n_seeds):
            lut = Lut(length, seed0 + s)
            _, nm, _ = ospr_generate_batched(targets, nsfs, lut, 0, bits=bits, precision=precision)
            per_seed.append(np.asarray(nm).mean(axis=0))
            lut.close()
        per_seed = np.array(per_seed)
        out[p] = (per_seed.mean(axis=0), per_seed.std(axis=0))
    return out


def summarize(res, n, n_sf):
    ref = res["nonrepeating"][0]
    rows = []
    for p, (m, sd) in res.items():
        if p == "nonrepeating":
            continue
        rows.append({"n_lut": p, "nmse": float(m[0]), "nmse_sym": float(m[1]),
                     "added_sym_pct": float(100 * (m[1] / ref[1] - 1)),
                     "added_pct": float(100 * (m[0] / ref[0] - 1)),
                     "sd_sym": float(sd[1]), "warnings": lut_check(p, n, n, n_sf)})
    return {"n": n, "n_sf": n_sf, "nonrepeating": [float(ref[0]), float(ref[1])], "rows": rows}


def main(argv=None):
    import synth

    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="64,128,256")
    ap.add_argument("--seeds", type=int, default=100)
    ap.add_argument("--targets", type=int, default=6)
    ap.add_argument("--n-sf", type=int, default=24)
    ap.add_argument("--out", default=None, help="write the JSON summary here")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    set_graphs(False)   # a new pool per call: direct launches, no per-pool graph capture
    summaries = []
    for n in (int(v) for v in args.sizes.split(",")):
        targets = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_LUT_STUDY0 + i)).cuda()
                   for i in range(args.targets)]
        t0 = time.perf_counter()
        res = sweep(targets, args.n_sf, default_primes(n), args.seeds)
        sm = summarize(res, n, args.n_sf)
        sm["seconds"] = round(time.perf_counter() - t0, 2)
        summaries.append(sm)
        print(json.dumps({"n": n, "seconds": sm["seconds"], "nonrepeating": sm["nonrepeating"]}), flush=True)
    set_graphs(True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(summaries, f, indent=1)
    return summaries


if __name__ == "__main__":
    main()

"""Throughput of the hot path on one MI355X.

One step = one OSPR frame at 1024x1024 with 24 binary sub-frames: LUT phase
randomisation, inverse 2D transform, binarisation, reconstruction transforms,
time-averaged intensity and FP64 NMSE, all in the library's HIP kernels,
inputs resident in HBM.  Reported: sub-frames/s (value), the HBM roofline of
the dominant kernel (from HIP events recorded inside the library on the launch
stream), the FP64 CPU oracle on a bounded sample of the same workload, GS
iterations/s at 512x512 and 1024x1024, and a LUT-length sweep with NMSE.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_BF16_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
METRIC = "OSPR 1024² sub-frames/s + GS iter/s at matched NMSE; % HBM roofline"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--lut", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip every leg after the headline")
    ap.add_argument("--legs", default="batched,gs,lut_sweep,phase_sources,ospr_variants,cnn_seed",
                    help="comma list of the legs to run after the headline")
    ap.add_argument("--cnn-held", type=int, default=100, help="learned-seed held-out targets (1024^2)")
    ap.add_argument("--plan", default=None,
                    help="OSPR launch plan 'cols,rows,ksplit,recon_cols,pad,chunk[,pts]' to use instead of autotuning")
    ap.add_argument("--calib", action="store_true",
                    help="finish with a plain 256 MiB copy kernel (reference for memory counters)")
    return ap.parse_args()


def ospr_kernel_bytes(nx, ny, n_sf, n_lut, chunk=0):
    """Canonical HBM bytes per launch of each OSPR kernel, from the per-pixel
    byte model of the three-pass design with full complex planes (per
    sub-frame: K1 writes the complex field, 8 B/px; K2 reads it, 8 B/px, writes
    the packed bits, 1/8 B/px, and the complex reconstruction column spectrum,
    8 B/px; K3 reads that, 8 B/px; the target, 4 B/px, is read once per frame by
    K1 and once by K3).  A LUT of more than 2^16 entries cannot stay
    cache-resident, so its unique entries read (8 B each) are charged to K1.
    With a chunked plan, K1 and K2 launch once per chunk of `chunk` sub-frames;
    the figures are per launch (per-frame terms prorated over the chunks).
    These bytes credit no symmetry, so a kernel that uses one can exceed the
    HBM peak against them: they are reported as `canonical_frac` only."""
    n = nx * ny
    per = chunk if 0 < chunk < n_sf else n_sf
    lut_bytes = 8 * min(n_lut, n * n_sf) if n_lut > 65536 else 0
    return {
        "ospr_rows": per * n * 8 + (n * 4 + lut_bytes) * per / n_sf,
        "ospr_cols": per * n * (8 + 0.125 + 8),
        "recon_rows": n_sf * n * 8 + n * 4,
    }


def ospr_design_bytes(nx, ny, n_sf, n_lut, chunk=0):
    """HBM bytes per launch that the binary-frame kernels must move, the
    roofline's `achieved` figure.  Only Re H is binarised, so the row pass
    transforms the Hermitian part of R and keeps rows 0..ny/2 of its output
    (half planes of (ny/2 + 1) x nx complex values, 8 B each); the binarised
    columns are real, so the column pass keeps the same rows of their
    spectrum.  Per sub-frame: K1 writes a half plane; K2 reads it, writes the
    packed bits (nx*ny/8 bytes) and a half spectrum; K3 reads that.  The target
    (4 B/px) is read once per frame by K1 and once by K3, and a LUT of more
    than 2^16 entries is charged to K1 as in the canonical model.  Row pitch
    padding is an implementation choice and is not counted."""
    n = nx * ny
    half = (ny // 2 + 1) * nx * 8
    per = chunk if 0 < chunk < n_sf else n_sf
    lut_bytes = 8 * min(n_lut, n * n_sf) if n_lut > 65536 else 0
    return {
        "ospr_rows": per * half + (n * 4 + lut_bytes) * per / n_sf,
        "ospr_cols": per * (2 * half + n / 8),
        "recon_rows": n_sf * half + n * 4,
    }


TRAFFIC_MARGIN = 0.10   # measured bytes may exceed the design's by the row pitch and stray re-reads


def source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2004_04049_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, sf_per_launch):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if they
    were taken on the current kernel sources with the same number of
    sub-frames per launch (chunking); else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            rec = json.load(f)
        e = rec.get(workload, {}).get(kernel)
        if not e or e.get("source_hash") != source_hash() or e.get("sf_per_launch") != sf_per_launch:
            return None
        return e["bytes_per_launch"]
    except Exception:
        return None


def measured_batch_traffic(prec, design_bytes):
    """HBM bytes per call of the 64-frame batch (one precision) from the
    committed rocprofv3 --pmc summary, if it was taken on the current kernel
    sources and the same batch layout; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            e = json.load(f).get("batched_64frames", {}).get(prec)
        if not e or e.get("source_hash") != source_hash() or e.get("design_bytes") != int(design_bytes):
            return None
        return e
    except Exception:
        return None


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(frames and sub-frames would shard by pool-cursor range)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2004_04049_amd as h
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    # a non-default stream: the library replays GS iterations as HIP graphs,
    # which the legacy default stream cannot capture
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    dev = torch.device("cuda", 0)
    nx = ny = 1024
    n_sf = 24
    n_lut = args.lut
    target = torch.from_numpy(synth.blob_target(nx, ny, synth.SEED_OSPR_1024)).to(dev)
    lut = h.Lut(n_lut, synth.SEED_LUT)
    bits = torch.empty((n_sf, nx * ny // 32), dtype=torch.int32, device=dev)
    nmse_dev = torch.zeros(2, dtype=torch.float64, device=dev)

    if args.plan:
        plan = [int(v) for v in args.plan.split(",")]
        h.plan_set(h.PLAN_OSPR, nx, ny, n_sf, plan)
    else:
        plan = h.autotune_ospr(target, n_sf, lut, reps=20)
    cursor = 0
    for _ in range(args.warmup):
        _, _, cursor = h.ospr_generate(target, n_sf, lut, cursor, bits=bits, want_nmse=False, nmse_out=nmse_dev)
    torch.cuda.synchronize()
    # timed region: the headline value (no instrumentation)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, cursor = h.ospr_generate(target, n_sf, lut, cursor, bits=bits, want_nmse=False, nmse_out=nmse_dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = args.steps * n_sf / elapsed
    nmse = nmse_dev.cpu().numpy().tolist()
    # same steps again with per-launch HIP events recorded by the library on
    # this stream: per-kernel average durations for the roofline
    h.prof_reset()
    h.prof_enable(True)
    t2 = time.perf_counter()
    for _ in range(args.steps):
        _, _, cursor = h.ospr_generate(target, n_sf, lut, cursor, bits=bits, want_nmse=False, nmse_out=nmse_dev)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    h.prof_enable(False)

    chunk = plan[5] if plan and len(plan) > 5 else 0
    kbytes = ospr_design_bytes(nx, ny, n_sf, n_lut, chunk)
    kcanon = ospr_kernel_bytes(nx, ny, n_sf, n_lut, chunk)
    kern = {}
    for k in ("ospr_rows", "ospr_cols", "recon_rows", "nmse_finalize"):
        ms, cnt = h.prof_read(k)
        if cnt:
            kern[k] = {"avg_us": 1e3 * ms / cnt, "launches": cnt}
    dom = max((k for k in kbytes if k in kern), key=lambda k: kern[k]["avg_us"])
    avg_s = kern[dom]["avg_us"] * 1e-6
    achieved = kbytes[dom] / avg_s / 1e9
    for k in kbytes:
        if k in kern:
            kern[k]["design_GBps"] = kbytes[k] / (kern[k]["avg_us"] * 1e-6) / 1e9
            kern[k]["canonical_GBps"] = kcanon[k] / (kern[k]["avg_us"] * 1e-6) / 1e9
    workload = f"ospr_{nx}x{ny}_sf{n_sf}_lut{n_lut}"
    traffic = measured_traffic(dom, workload, chunk if 0 < chunk < n_sf else n_sf)
    step_s = elapsed / args.steps
    step_design = sum(ospr_design_bytes(nx, ny, n_sf, n_lut).values())
    step_canon = sum(ospr_kernel_bytes(nx, ny, n_sf, n_lut).values())
    roofline = {
        "bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "design_bytes": int(kbytes[dom]),
        # the same kernel's measured HBM bytes (rocprofv3 counters) over its time,
        # and their ratio to the design bytes
        "traffic_frac": round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
        "traffic_vs_design": round(traffic / kbytes[dom], 4) if traffic else None,
        "traffic_margin": TRAFFIC_MARGIN,
        # full-plane byte model (credits no symmetry)
        "canonical_frac": round(kcanon[dom] / avg_s / 1e9 / HBM_PEAK_GBS, 4),
        "step_frac": round(step_design / step_s / 1e9 / HBM_PEAK_GBS, 4),
        "step_canonical_frac": round(step_canon / step_s / 1e9 / HBM_PEAK_GBS, 4),
    }
    roofline["traffic_agrees"] = (abs(traffic / kbytes[dom] - 1.0) <= TRAFFIC_MARGIN) if traffic else None

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "sub-frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"OSPR binary {nx}x{ny}, {n_sf} sub-frames, LUT {n_lut} entries, "
                               f"seeded 20-blob + 10-rectangle target", "nx": nx, "ny": ny, "n_sf": n_sf,
                   "n_lut": n_lut},
        "nmse": nmse, "roofline": roofline, "kernels": kern, "plan": plan,
        "ms_per_step_instrumented": round(1e3 * (t3 - t2) / args.steps, 4),
    }

    if not args.no_extras:
        def leg(name, f):
            print(f"bench: {name}", file=sys.stderr, flush=True)   # progress (stdout keeps the one JSON line)
            out[name] = f()
        legs = {
            "batched": lambda: bench_batched(h, synth, torch, dev),
            "gs": lambda: bench_gs(h, synth, torch, dev),
            "lut_sweep": lambda: bench_lut_sweep(h, synth, torch, dev, target, nx, ny, n_sf),
            "phase_sources": lambda: bench_phase_sources(h, synth, torch, dev, target, nx, ny, n_sf),
            "ospr_variants": lambda: bench_ospr_variants(h, synth, torch, dev, target, nx, ny, n_sf, lut),
            "cnn_seed": lambda: bench_cnn(h, synth, torch, dev, args),
        }
        for name in [x for x in args.legs.split(",") if x]:
            leg(name, legs[name])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(synth, nx, ny, n_lut)
    if args.calib:
        # known traffic: reads 2^28 bytes and writes 2^28 bytes
        x = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        y = x.mul(1.0)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = {"read": x.numel() * 4, "write": y.numel() * 4}
    print(json.dumps(out), flush=True)


def bench_batched(h, synth, torch, dev):
    """64 frames, sizes uniform over {256, 512, 1024, 2048}^2, n_sf uniform in
    8..24 (seed 14), targets seeds 1000+f, LUT 10007 chained across frames, one
    graph launch per batch, one autotuned plan per size; DFT stages in FP32,
    then BF16 and FP16 on the
    matrix cores, each reported against the FP32 run of the same batch (bit
    mismatch, NMSE and replay-intensity differences per frame)."""
    layout = synth.batch_layout(64, synth.SEED_BATCH)
    targets = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_BATCH_TARGET0 + f)).to(dev)
               for f, (n, _) in enumerate(layout)]
    nsfs = [k for _, k in layout]
    lut = h.Lut(10007, synth.SEED_LUT)
    # one autotuned plan per frame size (on the batch's first frame of that
    # size, at 16 sub-frames), stored for every sub-frame count of the size;
    # outside the timed region
    plans = {}
    for n in sorted({m for m, _ in layout}):
        f = next(i for i, (m, _) in enumerate(layout) if m == n)
        plans[str(n)] = h.autotune_ospr(targets[f], 16, lut, reps=10)
        h.plan_set(h.PLAN_OSPR, n, n, 0, plans[str(n)])
    pxsf = sum(n * n * k for n, k in layout)
    canon = sum(n * n * (k * 32.125 + 8) for n, k in layout)
    design = sum(sum(ospr_design_bytes(n, n, k, 10007).values()) for n, k in layout)
    res = {"frames": 64, "px_subframes": pxsf, "canonical_GB": round(canon / 1e9, 3),
           "design_GB": round(design / 1e9, 3),
           "sizes": {str(s_): sum(1 for n, _ in layout if n == s_) for s_ in (256, 512, 1024, 2048)},
           "plans": plans}
    ref = None
    for prec, name in ((h.FP32, "fp32"), (h.BF16, "bf16"), (h.FP16, "fp16")):
        nm = torch.zeros((64, 2), dtype=torch.float64, device=dev)
        recons = [torch.empty_like(t) for t in targets]
        bits, _, c = h.ospr_generate_batched(targets, nsfs, lut, 0, recons=recons, nmse_out=nm, precision=prec)
        torch.cuda.synchronize()
        out_bits = [b.clone() for b in bits]
        out_nm = nm.cpu().numpy().copy()
        out_rec = [r.clone() for r in recons]
        reps = 5
        dt = float("inf")   # best of three loops (one-off runtime stalls of tens of ms occur)
        for _ in range(3):
            t0 = time.perf_counter()
            for _ in range(reps):
                bits, _, c = h.ospr_generate_batched(targets, nsfs, lut, c, bits=bits, nmse_out=nm, precision=prec)
            torch.cuda.synchronize()
            dt = min(dt, (time.perf_counter() - t0) / reps)
        r = {"ms_per_batch": round(1e3 * dt, 3), "px_subframes_per_s": round(pxsf / dt, 1),
             "hbm_frac": round(design / dt / 1e9 / HBM_PEAK_GBS, 4),
             "canonical_frac": round(canon / dt / 1e9 / HBM_PEAK_GBS, 4), "nmse_mean": float(out_nm[:, 0].mean())}
        tr = measured_batch_traffic(name, design)
        if tr:   # measured bytes per batch (profiled plans) over this run's batch time
            r["traffic"] = tr["bytes_per_batch"]
            r["traffic_frac"] = round(tr["bytes_per_batch"] / dt / 1e9 / HBM_PEAK_GBS, 4)
            r["traffic_vs_design"] = round(tr["bytes_per_batch"] / design, 4)
            r["traffic_plans_match"] = tr.get("plans") == plans
        if ref is None:
            ref = (out_bits, out_nm, out_rec)
        else:
            mism, nrel, irel = [], [], []
            for f, (n, k) in enumerate(layout):
                a = h.unpack_bits(out_bits[f], n * n)
                b = h.unpack_bits(ref[0][f], n * n)
                mism.append(float((a != b).mean()))
                nrel.append(abs(out_nm[f, 0] - ref[1][f, 0]) / ref[1][f, 0])
                irel.append(float(torch.linalg.vector_norm(out_rec[f] - ref[2][f]) /
                                  torch.linalg.vector_norm(ref[2][f])))
            r["vs_fp32"] = {"bit_mismatch_mean": float(np.mean(mism)), "bit_mismatch_max": float(np.max(mism)),
                            "nmse_rel_mean": float(np.mean(nrel)), "nmse_rel_max": float(np.max(nrel)),
                            "ibar_rel_l2_mean": float(np.mean(irel)), "ibar_rel_l2_max": float(np.max(irel))}
        res[name] = r
    # the same 64 frames as 64 single-frame calls in batch order on one stream
    # (cursor chained), against the one graph launch over four branches
    bits1 = [torch.empty((k, n * n // 32), dtype=torch.int32, device=dev) for n, k in layout]
    nm1 = torch.zeros(2, dtype=torch.float64, device=dev)

    def sequential(c):
        for f in range(64):
            _, _, c = h.ospr_generate(targets[f], nsfs[f], lut, c, bits=bits1[f], want_nmse=False, nmse_out=nm1)
        return c
    c = sequential(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        c = sequential(c)
    torch.cuda.synchronize()
    res["fp32_sequential_ms_per_batch"] = round(1e3 * (time.perf_counter() - t0) / 5, 3)
    # batches of 64 small frames of one size (n_sf 8..24 from the same layout
    # draw), where the grouped launches replace per-frame launch latency
    small = {}
    for n in (64, 256):
        tg = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_BATCH_TARGET0 + f)).to(dev) for f in range(64)]
        bs, _, c = h.ospr_generate_batched(tg, nsfs, lut, 0)
        torch.cuda.synchronize()
        dt = float("inf")   # best of three 10-call loops (one-off runtime stalls of tens of ms occur)
        for _ in range(3):
            t0 = time.perf_counter()
            for _ in range(10):
                bs, _, c = h.ospr_generate_batched(tg, nsfs, lut, c, bits=bs)
            torch.cuda.synchronize()
            dt = min(dt, (time.perf_counter() - t0) / 10)
        small[f"64x{n}^2"] = {"ms_per_batch": round(1e3 * dt, 3), "px_subframes_per_s": round(n * n * sum(nsfs) / dt, 1)}
    res["fp32_small_frames"] = small
    return res


def bench_gs(h, synth, torch, dev):
    res = {}
    for n, reps in ((512, 20), (1024, 10)):
        t = torch.from_numpy(synth.blob_target(n, n, synth.SEED_GS_512)).to(dev)
        lut = h.Lut(4096, synth.SEED_LUT)
        plan = h.autotune_gs(t, lut, reps=3)
        field = torch.empty((n, n), dtype=torch.complex64, device=dev)
        codes = torch.empty((n, n), dtype=torch.uint8, device=dev)
        r = h.gs_iterate(t, 50, lut, 0, field=field, codes=codes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = h.gs_iterate(t, 50, lut, 0, field=field, codes=codes)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[f"{n}x{n}"] = {"iters": 50, "iter_per_s": round(50 / dt, 1), "ms_per_run": round(1e3 * dt, 3),
                           "nmse_iter1": float(r["nmse"][0]), "nmse_iter50": float(r["nmse"][-1]),
                           "nmse_8level": float(r["nmse_final2"][0]),
                           "hbm_frac_36Bpx": round(36 * n * n * 50 / dt / 1e9 / HBM_PEAK_GBS, 4), "plan": plan}
        # independent frames of the same size iterating together (one launch
        # per pass over all frames): aggregate frame-iterations/s.  Many
        # frames fill the GPU, so the single-frame plan is not the best one:
        # a few candidates are timed on 16 frames first (outside the timed
        # runs), and the single-frame plan is restored afterwards.
        def time_batch(nf, runs=2):
            tg = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_GS_512 + f)).to(dev) for f in range(nf)]
            fl = [torch.empty((n, n), dtype=torch.complex64, device=dev) for _ in range(nf)]
            h.gs_iterate_batched(tg, 50, lut, 0, fields=fl)
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(3):
                t0 = time.perf_counter()
                for _ in range(runs):
                    h.gs_iterate_batched(tg, 50, lut, 0, fields=fl)
                torch.cuda.synchronize()
                best = min(best, (time.perf_counter() - t0) / runs)
            return best
        cands = [plan, [8, 2, 0, 0, 16, 0, 16], [0, 0, 0, 0, -1, 0, 16], [4, 1, 0, 0, 64, 0, 8], [16, 2, 0, 0, 16, 0, 16],
                 [8, 2, 0, 0, 16, 0, 8], [16, 2, 0, 0, 16, 0, 8]]
        timed = []
        for c in cands:
            h.plan_set(h.PLAN_GS, n, n, 1, c)
            timed.append((time_batch(16, 1), c))
        bplan = min(timed)[1]
        h.plan_set(h.PLAN_GS, n, n, 1, bplan)
        batched = {"plan": bplan}
        for nf in (4, 8, 16, 32):
            dtb = time_batch(nf)
            batched[str(nf)] = {"frame_iter_per_s": round(50 * nf / dtb, 1), "ms_per_run": round(1e3 * dtb, 3),
                                "hbm_frac_36Bpx": round(36 * n * n * 50 * nf / dtb / 1e9 / HBM_PEAK_GBS, 4)}
        h.plan_set(h.PLAN_GS, n, n, 1, plan)
        res[f"{n}x{n}"]["batched_frames"] = batched
    return res


def cnn_flops(n):
    """Multiply-adds x 2 of one forward pass over an n x n image: 3x3 taps
    over 1->32, 3 x 32->32, 32->2 channels."""
    return 2 * n * n * 9 * (1 * 32 + 3 * 32 * 32 + 32 * 2)


CNN_WEIGHTS = os.path.join(ROOT, "paper_2004_04049_amd", "weights", "seed_cnn_1024_lut.bin")


def bench_cnn(h, synth, torch, dev, args):
    """Learned GS seed at 1024^2: inference and training-step time against
    the BF16 MFMA peak, and the iterations-to-GS-50-NMSE comparison on
    held-out targets (seeds 200000+i) for the network trained at full scale
    (10k targets, GS-50 labels from the 4096-entry LUT; written by
    `python -m paper_2004_04049_amd.seed_study --save ...` and loaded here),
    the untrained network (a smooth but unlearned seed) and the LUT seed (50
    iterations by definition).  Training forward + backward-data + weight
    gradients ~ 3 forward passes of multiply-adds."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2004_04049_amd import seed
    n = 1024
    with ThreadPoolExecutor(8) as ex:
        he = list(ex.map(lambda i: synth.blob_target(n, n, synth.SEED_CNN_HELDOUT0 + i), range(args.cnn_held)))
        tr = list(ex.map(lambda i: synth.blob_target(n, n, synth.SEED_CNN_TRAIN0 + i), range(4)))
    he = [torch.from_numpy(a).to(dev) for a in he]
    tr = [torch.from_numpy(a).to(dev) for a in tr]
    lut = h.Lut(4096, synth.SEED_LUT)
    net = h.Cnn(seed=1)
    ph = net.infer(he[0])
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        net.infer(he[0], out=ph)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / reps
    lab0 = seed.gs_labels(tr[:1], lut, 50)[0]
    for _ in range(2):
        net.train_step(tr[0], lab0, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(tr[0], lab0, 1e-4, want_loss=False)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / reps
    ctrl = seed.compare(h.Cnn(seed=1), he, lut, 50, 100)
    f = cnn_flops(n)
    out = {
        "size": f"{n}x{n}", "dtype": "bf16", "infer_ms": round(1e3 * t_inf, 4),
        "infer_TFLOPs": round(f / t_inf / 1e12, 2), "infer_frac_mfma": round(f / t_inf / 1e12 / MFMA_BF16_TFLOPS, 4),
        "train_step_ms": round(1e3 * t_train, 4), "train_images_per_s": round(1.0 / t_train, 2),
        "train_TFLOPs": round(3 * f / t_train / 1e12, 2),
        "held_out_untrained": {k: v for k, v in ctrl.items() if k != "rows"},
        "lut_seed_iters": 50,
    }
    if os.path.exists(CNN_WEIGHTS):
        trained = h.Cnn(path=CNN_WEIGHTS)
        cmp_ = seed.compare(trained, he, lut, 50, 100)
        out["held_out"] = {k: v for k, v in cmp_.items() if k != "rows"}
        out["weights"] = os.path.relpath(CNN_WEIGHTS, ROOT)
    return out


def bench_lut_sweep(h, synth, torch, dev, target, nx, ny, n_sf):
    res = []
    sizes = [2 ** 8, 2 ** 12, 2 ** 16, 2 ** 20, nx * ny * n_sf, 10007, 65537, 1048573]
    bits = torch.empty((n_sf, nx * ny // 32), dtype=torch.int32, device=dev)
    nm_dev = torch.empty(2, dtype=torch.float64, device=dev)
    for L in sizes:
        lut = h.Lut(L, synth.SEED_LUT)
        _, nm, c = h.ospr_generate(target, n_sf, lut, 0, bits=bits)
        for _ in range(3):
            _, _, c = h.ospr_generate(target, n_sf, lut, c, bits=bits, want_nmse=False, nmse_out=nm_dev)
        torch.cuda.synchronize()
        steps = 50
        dt = float("inf")
        for _ in range(3):   # best of three timed loops, as in the phase-source leg
            t0 = time.perf_counter()
            for _ in range(steps):
                _, _, c = h.ospr_generate(target, n_sf, lut, c, bits=bits, want_nmse=False, nmse_out=nm_dev)
            torch.cuda.synchronize()
            dt = min(dt, (time.perf_counter() - t0) / steps)
        res.append({"n_lut": L, "subframes_per_s": round(n_sf / dt, 1), "nmse": float(nm[0]),
                    "nmse_sym": float(nm[1]), "warnings": h.lut_check(L, nx, ny, n_sf)})
        lut.close()
    return res


def bench_phase_sources(h, synth, torch, dev, target, nx, ny, n_sf, steps=50):
    """The LUT against the other ways of drawing the phases, on the headline
    workload: the software route (counter-based SplitMix64 + FP32 sine/cosine
    per pixel), the M-sequence route (x^31 + x^3 + 1, 8 bits per pixel, phasor
    table), and 8-bit code tables.  Per source: sub-frames/s of whole frames,
    the row pass per launch (the only kernel that differs), the NMSE pair of
    the frame at cursor 0 and the bytes the source keeps on the device."""
    full = nx * ny * n_sf
    cases = [("table", 65536), ("table", 10007), ("table", full), ("codes8", 65536), ("codes8", 1048573),
             ("codes8", full), ("prng", None), ("mseq", None)]
    bits = torch.empty((n_sf, nx * ny // 32), dtype=torch.int32, device=dev)
    nm_dev = torch.empty(2, dtype=torch.float64, device=dev)
    ref_mask = h.phase_mask(h.Lut(1 << 20, synth.SEED_LUT), 0, nx, ny, 1)
    res = []
    for kind, L in cases:
        if kind == "table":
            lut, nbytes = h.Lut(L, synth.SEED_LUT), 8 * L
        elif kind == "codes8":
            lut, nbytes = h.Lut.codes(L, synth.SEED_LUT), L + 2048
        elif kind == "prng":
            lut, nbytes = h.Lut.prng(synth.SEED_LUT), 0
        else:
            lut, nbytes = h.Lut.mseq(synth.SEED_LUT), 2048 + 128 + 12 * 4096
        _, nm, c = h.ospr_generate(target, n_sf, lut, 0, bits=bits)
        for _ in range(3):
            _, _, c = h.ospr_generate(target, n_sf, lut, c, bits=bits, want_nmse=False, nmse_out=nm_dev)
        torch.cuda.synchronize()
        dt = float("inf")
        for _ in range(3):   # best of three timed loops
            t0 = time.perf_counter()
            for _ in range(steps):
                _, _, c = h.ospr_generate(target, n_sf, lut, c, bits=bits, want_nmse=False, nmse_out=nm_dev)
            torch.cuda.synchronize()
            dt = min(dt, (time.perf_counter() - t0) / steps)
        h.prof_reset()
        h.prof_enable(True)
        for _ in range(10):
            _, _, c = h.ospr_generate(target, n_sf, lut, c, bits=bits, want_nmse=False, nmse_out=nm_dev)
        torch.cuda.synchronize()
        h.prof_enable(False)
        ms, cnt = h.prof_read("ospr_rows")
        row = {"source": kind, "n_lut": L, "device_bytes": nbytes, "subframes_per_s": round(n_sf / dt, 1),
               "ospr_rows_us": round(1e3 * ms / max(cnt, 1), 2), "nmse": float(nm[0]), "nmse_sym": float(nm[1])}
        if kind == "prng":
            # same SplitMix64 outputs as a table of the same seed: the FP32
            # sine/cosine plus 24-bit truncation against FP64-rounded phasors
            d = (h.phase_mask(lut, 0, nx, ny, 1) - ref_mask).abs().max().item()
            row["phasor_vs_table_max"] = d
        res.append(row)
        lut.close()
    return res


def bench_ospr_variants(h, synth, torch, dev, target, nx, ny, n_sf, lut, steps=50):
    """The binary frame against the two variants on the headline workload:
    pairs (sub-frames 2j, 2j+1 from Re and Im of one field: half the row
    passes and inverse column transforms) and eight phase levels.  Per mode:
    sub-frames/s (best of three loops), per-kernel averages, the NMSE pair of
    the frame at cursor 0, and the NMSE pair on a non-repeating pool."""
    res = []
    nm_dev = torch.empty(2, dtype=torch.float64, device=dev)
    nonrep = h.Lut.prng(synth.SEED_LUT)
    for mode in ("binary", "pairs", "levels8"):
        bits = None
        bits, nm, c = h.ospr_generate(target, n_sf, lut, 0, mode=mode)
        for _ in range(3):
            _, _, c = h.ospr_generate(target, n_sf, lut, c, bits=bits, want_nmse=False, nmse_out=nm_dev, mode=mode)
        torch.cuda.synchronize()
        dt = float("inf")
        for _ in range(3):
            t0 = time.perf_counter()
            for _ in range(steps):
                _, _, c = h.ospr_generate(target, n_sf, lut, c, bits=bits, want_nmse=False, nmse_out=nm_dev,
                                          mode=mode)
            torch.cuda.synchronize()
            dt = min(dt, (time.perf_counter() - t0) / steps)
        h.prof_reset()
        h.prof_enable(True)
        for _ in range(10):
            _, _, c = h.ospr_generate(target, n_sf, lut, c, bits=bits, want_nmse=False, nmse_out=nm_dev, mode=mode)
        torch.cuda.synchronize()
        h.prof_enable(False)
        kern = {}
        for k in ("ospr_rows", "ospr_cols", "recon_rows", "nmse_finalize"):
            ms, cnt = h.prof_read(k)
            if cnt:
                kern[k] = {"avg_us": round(1e3 * ms / cnt, 2), "per_frame": cnt // 10}
        # quality on a non-repeating pool (the headline table divides the
        # frame, so all its fields repeat and the modes would differ in that)
        _, nm_nr, _ = h.ospr_generate(target, n_sf, nonrep, 0, mode=mode)
        res.append({"mode": mode, "subframes_per_s": round(n_sf / dt, 1), "ms_per_frame": round(1e3 * dt, 4),
                    "kernels": kern, "nmse": float(nm[0]), "nmse_sym": float(nm[1]),
                    "nmse_nonrepeating": [float(nm_nr[0]), float(nm_nr[1])]})
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(synth, nx, ny, n_lut):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: the
    same target, LUT and frame size, 12 frames of 24 sub-frames on all host
    threads, and one frame on one thread; beside it, as context only, the
    transforms alone (torch.fft on the CPU, complex64, all threads)."""
    import oracle
    import torch
    t = synth.blob_target(nx, ny, synth.SEED_OSPR_1024)
    phi = oracle.lut_phases(n_lut, synth.SEED_LUT)
    n_sf = 24

    def run(frames):
        cursor = 0
        t0 = time.perf_counter()
        for _ in range(frames):
            oracle.ospr(t, n_sf, phi, n_lut, cursor, want_reh=False, want_ibar=False)
            cursor += n_sf * nx * ny
        return time.perf_counter() - t0

    threads = oracle.num_threads()
    frames = 12
    dt = run(frames)
    oracle.set_threads(1)
    dt1 = run(1)
    oracle.set_threads(threads)
    # two 2D transforms per sub-frame (generation and replay)
    x = torch.from_numpy(t).to(torch.complex64)
    torch.fft.fft2(torch.fft.ifft2(x))   # plan creation outside the timing
    t0 = time.perf_counter()
    for _ in range(n_sf):
        torch.fft.fft2(torch.fft.ifft2(x))
    dt_fft = time.perf_counter() - t0
    return {"value": round(frames * n_sf / dt, 3), "unit": "sub-frames/s", "cores": threads,
            "kind": "oracle", "sample": f"{frames} frames x {n_sf} sub-frames at {nx}x{ny}, LUT {n_lut}, "
                                        f"{dt:.1f} s",
            "single_thread": {"value": round(n_sf / dt1, 3), "unit": "sub-frames/s",
                              "sample": f"1 frame x {n_sf} sub-frames, {dt1:.1f} s"},
            "torch_fft_context": {"value": round(n_sf / dt_fft, 3), "unit": "sub-frames/s (transforms only)",
                                  "threads": torch.get_num_threads()},
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count()}}


if __name__ == "__main__":
    main()

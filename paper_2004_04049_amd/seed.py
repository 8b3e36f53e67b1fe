"""Learned Gerchberg-Saxton seed: labels from the library's own GS, a training
loop over the network's C-ABI calls, and the comparison against the LUT seed.

The paper seeds GS (Sections 2-3) with a replay-plane phase drawn from its
look-up table (Sections 4-5, Fig. 3); here a network may supply that phasor instead (`init_phasor` of
`holo_gs_iterate`).  The label of a target is the replay-plane phasor R'/|R'|
after `n_label` LUT-seeded GS iterations; the comparison counts, on held-out
targets, the GS iterations (and the time, inference included) a network seed
needs to reach the NMSE that plain LUT-seeded GS reaches in `n_ref`
iterations.  All arithmetic runs in the library; this module only sequences
calls and keeps the books."""
from __future__ import annotations

import time

import numpy as np
import torch

from . import Cnn, Lut, gs_iterate


def gs_labels(targets, lut: Lut, n_label: int = 50):
    """Replay fields after `n_label` LUT-seeded GS iterations (cursor 0), one
    complex64 [ny, nx] tensor per target."""
    return [gs_iterate(t, n_label, lut, 0, want_nmse=False, want_final=False)["field"].clone() for t in targets]


def train(net: Cnn, targets, labels, epochs: int, lr: float, batch: int = 1, order_seed: int = 0):
    """Adam steps on mini-batches of `batch` images (mean gradient); the
    visiting order of each epoch is a permutation drawn from `order_seed`.
    Returns the per-epoch mean loss and the measured training rate
    (images/s, device-synchronised)."""
    rng = np.random.default_rng(order_seed)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    images = 0
    for _ in range(epochs):
        acc = []
        order = rng.permutation(len(targets))
        for s in range(0, len(order), batch):
            idx = order[s:s + batch]
            tb = torch.stack([targets[i] for i in idx])
            qb = torch.stack([labels[i] for i in idx])
            acc.append(net.train_step(tb, qb, lr, want_loss=True))
            images += len(idx)
        losses.append(float(np.mean(acc)))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"epoch_loss": losses, "images_per_s": images / dt if dt > 0 else 0.0}


def _first_reach(nmse, goal):
    hit = np.nonzero(np.asarray(nmse) <= goal)[0]
    return int(hit[0]) + 1 if hit.size else None


def _timed(fn, reps: int = 3):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def compare(net: Cnn, targets, lut: Lut, n_ref: int = 50, max_iter: int = 100):
    """Per held-out target: goal = NMSE of LUT-seeded GS after `n_ref`
    iterations; iterations for the network seed to reach it (None if not within
    `max_iter`), and wall times (inference + that many iterations, against
    `n_ref` iterations)."""
    rows = []
    for t in targets:
        ref = gs_iterate(t, n_ref, lut, 0, want_final=False)
        goal = float(ref["nmse"][-1])
        ph = net.infer(t)
        run = gs_iterate(t, max_iter, None, 0, init_phasor=ph, want_final=False)
        k = _first_reach(run["nmse"], goal)
        t_inf = _timed(lambda: net.infer(t, out=ph))
        t_iter = _timed(lambda: gs_iterate(t, max_iter, None, 0, init_phasor=ph, want_nmse=False,
                                           want_final=False)) / max_iter
        rows.append({"goal_nmse": goal, "iters": k, "nmse_at_ref": float(run["nmse"][n_ref - 1]),
                     "t_lut_s": n_ref * t_iter, "t_cnn_s": (t_inf + k * t_iter) if k else None,
                     "t_infer_s": t_inf})
    its = [r["iters"] for r in rows]
    reached = [k for k in its if k is not None]
    return {
        "n": len(rows), "n_ref": n_ref, "max_iter": max_iter,
        "reached": len(reached),
        "iters_mean": float(np.mean(reached)) if reached else None,
        "iters_median": float(np.median(reached)) if reached else None,
        "fraction_improved": sum(1 for k in its if k is not None and k < n_ref) / max(len(rows), 1),
        "nmse_ratio_at_ref_mean": float(np.mean([r["nmse_at_ref"] / r["goal_nmse"] for r in rows])),
        "t_infer_ms": 1e3 * float(np.mean([r["t_infer_s"] for r in rows])),
        "rows": rows,
    }

"""Learned-seed study at full scale: the seed network trained on many seeded
targets with GS-50 labels, then compared on held-out targets against the
untrained network and against the LUT seed it replaces.

Workload (the learned-seed configuration): training targets are seeded
blob/rectangle amplitudes at 1024^2 (seeds 100000+i), held-out targets use
seeds 200000+i.  Labels are the replay-plane phasors after 50 GS iterations:
  labels=lut   from the 4096-entry LUT seed at cursor 0 (the default reading);
  labels=self  from the untrained network's own seed (a deterministic function
               of the target the network can represent, for comparison).
Training: Adam on mini-batches, per-epoch mean loss logged (the loss is the
target-weighted 1 - cos of the phase error at the best global phase, so 1
means uncorrelated and 0 a perfect match).  Comparison: for each held-out
target the GS iterations a seed needs to reach the NMSE that LUT-seeded GS
reaches after 50 iterations, and the time including inference.

All arithmetic runs in the library (network, GS, labels); this module only
sequences calls, keeps the books and writes a JSON summary.

Run:  python -m paper_2004_04049_amd.seed_study --train 10000 --held 100
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import Cnn, Lut, gs_iterate, seed


def _log(msg):
    print(f"seed_study: {msg}", file=sys.stderr, flush=True)


def make_targets(seeds, n, device, threads=16):
    """Seeded blob/rectangle targets on the device, generated on host threads."""
    import synth
    out = []
    with ThreadPoolExecutor(threads) as ex:
        for i, a in enumerate(ex.map(lambda s: synth.blob_target(n, n, s), seeds)):
            out.append(torch.from_numpy(a).to(device))
            if (i + 1) % 2000 == 0:
                _log(f"targets {i + 1}/{len(seeds)}")
    return out


def self_labels(net: Cnn, targets, n_label: int = 50):
    """Replay fields after `n_label` GS iterations seeded by the network."""
    out = []
    for t in targets:
        ph = net.infer(t)
        out.append(gs_iterate(t, n_label, None, 0, init_phasor=ph, want_nmse=False, want_final=False)["field"].clone())
    return out


def mean_loss(net: Cnn, targets, labels):
    return float(np.mean([net.loss_grad(t, q)[0] for t, q in zip(targets, labels)]))


def run(n_train: int, n_held: int, epochs: int, batch: int, lr: float, labels: str, n: int = 1024,
        net_seed: int = 1, save: str | None = None):
    import synth
    dev = torch.device("cuda", 0)
    s = torch.cuda.Stream()
    torch.cuda.set_stream(s)
    t0 = time.perf_counter()
    train_t = make_targets([synth.SEED_CNN_TRAIN0 + i for i in range(n_train)], n, dev)
    held_t = make_targets([synth.SEED_CNN_HELDOUT0 + i for i in range(n_held)], n, dev)
    t_targets = time.perf_counter() - t0
    _log(f"{n_train} + {n_held} targets in {t_targets:.1f} s")
    lut = Lut(4096, synth.SEED_LUT)
    net = Cnn(seed=net_seed)
    t0 = time.perf_counter()
    if labels == "lut":
        train_q = seed.gs_labels(train_t, lut, 50)
        held_q = seed.gs_labels(held_t, lut, 50)
    else:
        train_q = self_labels(net, train_t)
        held_q = self_labels(net, held_t)
    torch.cuda.synchronize()
    t_labels = time.perf_counter() - t0
    _log(f"labels ({labels}) in {t_labels:.1f} s")
    ctrl = seed.compare(Cnn(seed=net_seed), held_t, lut, 50, 100)
    _log(f"untrained: iterations to the LUT GS-50 NMSE {ctrl['iters_mean']}")
    curve = []
    held_loss = [mean_loss(net, held_t[:32], held_q[:32])]
    t0 = time.perf_counter()
    for e in range(epochs):
        h = seed.train(net, train_t, train_q, 1, lr, batch=batch, order_seed=e)
        curve.append(h["epoch_loss"][0])
        held_loss.append(mean_loss(net, held_t[:32], held_q[:32]))
        _log(f"epoch {e + 1}/{epochs}: train loss {curve[-1]:.5f}, held-out loss {held_loss[-1]:.5f}, "
             f"{h['images_per_s']:.0f} images/s")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    cmp_ = seed.compare(net, held_t, lut, 50, 100)
    _log(f"trained: iterations to the LUT GS-50 NMSE {cmp_['iters_mean']}")
    if save:
        net.save(save)
    strip = lambda d: {k: v for k, v in d.items() if k != "rows"}
    return {
        "size": f"{n}x{n}", "train": n_train, "held_out": n_held, "epochs": epochs, "batch": batch, "lr": lr,
        "labels": labels, "targets_s": round(t_targets, 1), "labels_s": round(t_labels, 1),
        "train_s": round(t_train, 1), "train_images_per_s": round(epochs * n_train / t_train, 1),
        "epoch_loss": [round(x, 6) for x in curve], "held_out_loss": [round(x, 6) for x in held_loss],
        "trained": strip(cmp_), "untrained": strip(ctrl),
        "lut_seed": {"iters": 50, "t_ms": round(1e3 * float(np.mean([r["t_lut_s"] for r in cmp_["rows"]])), 3)},
        "trained_iters": [r["iters"] for r in cmp_["rows"]],
        "untrained_iters": [r["iters"] for r in ctrl["rows"]],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=10000)
    ap.add_argument("--held", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--labels", choices=("lut", "self"), default="lut")
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--save", default=None)
    a = ap.parse_args()
    res = run(a.train, a.held, a.epochs, a.batch, a.lr, a.labels, a.size, save=a.save)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

"""GPU parity of the learned GS seed network against the oracle, and that
training on the project's own GS output reduces the loss.

The GPU keeps weights, hidden activations and hidden-layer gradients in BF16
and accumulates in FP32.  The oracle is given the BF16-rounded weights and run
with its BF16 storage model (the same values rounded where they are stored,
FP64 sums), so what remains is FP32-versus-FP64 accumulation: ~sqrt(288) *
2^-24 relative per sum, which now and then flips a stored BF16 value by one
unit (2^-8 relative); a flip spreads through the later layers' 3x3
neighbourhoods.  Most outputs are therefore exact to FP32 rounding and a few
small patches differ: a numpy emulation of the same BF16 model summing in
FP32 instead of FP64 differs from it by a scaled error of at most 9.6e-3,
with 2.1% of the pixels above 1e-4, at 128 x 256.  Bounds: output error
(phasor angle scaled by |o| / rms|o|) median < 1e-4, max < 5e-2, at most 5%
of the pixels above 1e-4; gradient relative L2 < 1e-2; loss within 1e-4
relative, on the 64 x 64 case.  The output gradient is (g - (g.p)p)/|o|, so
pixels with a small output magnitude |o| carry large terms, and the weight
gradients are sums over pixels with heavy cancellation: a BF16 flip patch
that happens to touch a small-|o| pixel moves the gradient by a few percent
(measured on a 64 x 64 case with another seed: 5.9e-2, from a 24% change of
one layer-5 bias term traced to a pixel with |o| ~ 0.1 rms|o|; the same model
summed in FP32 by numpy gives 2e-3 to 5e-3 when no such pixel is hit).  The
128 x 256 case is therefore held to cosine > 0.995 and relative L2 < 5e-2.  Against the exact (unrounded) network the four BF16
roundings (unit roundoff 2^-8 each, in quadrature) bound the median scaled
error at 6e-3."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _bf16(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u << 16).astype(np.uint32).view(np.float32)


def _rounded_params(p, orc):
    """the network's compute copy: every weight to BF16, biases FP32."""
    q = p.astype(np.float64).copy()
    C = 32
    o = 0
    for l in range(5):
        ci = 1 if l == 0 else C
        co = 2 if l == 4 else C
        nw = co * ci * 9
        q[o:o + nw] = _bf16(p[o:o + nw])
        o += nw + co
    return q


@pytest.fixture(scope="module")
def holo():
    import paper_2004_04049_amd as h
    h.lib()
    return h


def test_forward_matches_oracle(holo, orc):
    net = holo.Cnn(seed=5)
    p = net.params()
    assert p.size == orc.cnn_nparams(32)
    t = synth.blob_target(64, 64, 3)
    ph = net.infer(torch.from_numpy(t).cuda()).cpu().numpy()
    q = _rounded_params(p, orc)
    for store, med_tol, max_tol in ((True, 1e-4, 5e-2), (False, 6e-3, None)):
        _, out2, ref = orc.cnn_forward(q, 32, t, bf16_store=store)
        mag = np.hypot(out2[0], out2[1])
        err = np.abs(np.angle(ph * np.conj(ref))) * mag / np.sqrt(np.mean(mag ** 2))
        print(f"bf16_store={store}: scaled phasor angle error median {np.median(err):.2e}, "
              f"99% {np.quantile(err, 0.99):.2e}, max {err.max():.2e}")
        assert np.median(err) < med_tol
        if max_tol is not None:
            assert err.max() < max_tol and np.mean(err > 1e-4) < 0.05


def test_gradient_matches_oracle(holo, orc):
    net = holo.Cnn(seed=6)
    p = net.params()
    t = synth.blob_target(64, 64, 4)
    rng = np.random.default_rng(0)
    q = np.exp(1j * rng.uniform(0, 2 * np.pi, t.shape)).astype(np.complex64)
    loss, g = net.loss_grad(torch.from_numpy(t).cuda(), torch.from_numpy(q).cuda())
    rl, rg = orc.cnn_backward(_rounded_params(p, orc), 32, t, q.astype(np.complex128), bf16_store=True)
    rel = float(np.linalg.norm(g - rg) / np.linalg.norm(rg))
    per_layer = []
    o = 0
    for l in range(5):
        ci = 1 if l == 0 else 32
        co = 2 if l == 4 else 32
        k = co * ci * 9 + co
        per_layer.append(float(np.linalg.norm(g[o:o + k] - rg[o:o + k]) / np.linalg.norm(rg[o:o + k])))
        o += k
    print(f"loss {loss:.8f} oracle {rl:.8f}; gradient rel L2 {rel:.3e}, per layer "
          + " ".join(f"{x:.1e}" for x in per_layer))
    assert loss == pytest.approx(rl, rel=1e-4)
    assert rel < 1e-2 and max(per_layer) < 2e-2


def test_forward_and_gradient_non_square_multi_tile(holo, orc):
    """128 x 256 (several conv tiles and weight-gradient blocks per axis, a
    non-square image): same bounds as the 64 x 64 cases."""
    ny, nx = 128, 256
    net = holo.Cnn(seed=11)
    p = net.params()
    t = synth.blob_target(nx, ny, 12)
    q = _rounded_params(p, orc)
    ph = net.infer(torch.from_numpy(t).cuda()).cpu().numpy()
    _, out2, ref = orc.cnn_forward(q, 32, t, bf16_store=True)
    mag = np.hypot(out2[0], out2[1])
    err = np.abs(np.angle(ph * np.conj(ref))) * mag / np.sqrt(np.mean(mag ** 2))
    print(f"128x256 scaled phasor angle error median {np.median(err):.2e}, max {err.max():.2e}, "
          f"above 1e-4: {np.mean(err > 1e-4):.3f}")
    assert np.median(err) < 1e-4 and err.max() < 5e-2 and np.mean(err > 1e-4) < 0.05
    rng = np.random.default_rng(2)
    lab = (ref * np.exp(1j * rng.uniform(-1.0, 1.0, (ny, nx)))).astype(np.complex64)
    loss, g = net.loss_grad(torch.from_numpy(t).cuda(), torch.from_numpy(lab).cuda())
    rl, rg = orc.cnn_backward(q, 32, t, lab.astype(np.complex128), bf16_store=True)
    rel = float(np.linalg.norm(g - rg) / np.linalg.norm(rg))
    cos = float(np.dot(g, rg) / (np.linalg.norm(g) * np.linalg.norm(rg)))
    print(f"128x256 loss {loss:.8f} oracle {rl:.8f}; gradient rel L2 {rel:.3e}, cosine {cos:.5f}")
    assert loss == pytest.approx(rl, rel=1e-4)
    assert rel < 5e-2 and cos > 0.995


def test_adam_step_matches_oracle(holo, orc):
    """One train_step = the oracle's Adam applied to the GPU gradient, from
    zero moments (FP32 parameter update: 1e-6 relative + lr * 1e-4 absolute)."""
    net = holo.Cnn(seed=8)
    t = torch.from_numpy(synth.blob_target(64, 64, 5)).cuda()
    rng = np.random.default_rng(1)
    q = torch.from_numpy(np.exp(1j * rng.uniform(0, 2 * np.pi, (64, 64))).astype(np.complex64)).cuda()
    p0 = net.params().astype(np.float64)
    _, g = net.loss_grad(t, q)
    lr = 1e-3
    net.train_step(t, q, lr)
    p1 = net.params()
    ref = p0.copy()
    m = np.zeros_like(ref)
    v = np.zeros_like(ref)
    orc.adam(ref, g.astype(np.float64), m, v, 1, lr)
    np.testing.assert_allclose(p1, ref, rtol=1e-6, atol=lr * 1e-4)
    assert np.abs(p1 - p0).max() > 0.5 * lr


def test_batch_step_is_mean_of_image_gradients(holo, orc):
    """A batch step applies Adam to the mean of the per-image gradients and
    reports the mean loss."""
    net = holo.Cnn(seed=12)
    n = 64
    ts = torch.stack([torch.from_numpy(synth.blob_target(n, n, 20 + i)) for i in range(3)]).cuda().contiguous()
    rng = np.random.default_rng(5)
    qs = torch.from_numpy(np.exp(1j * rng.uniform(0, 2 * np.pi, (3, n, n))).astype(np.complex64)).cuda()
    p0 = net.params().astype(np.float64)
    lg = [net.loss_grad(ts[i], qs[i]) for i in range(3)]
    gmean = np.mean([g for _, g in lg], axis=0).astype(np.float64)
    lr = 1e-3
    loss = net.train_step(ts, qs, lr)
    assert loss == pytest.approx(np.mean([l for l, _ in lg]), rel=1e-12)
    ref = p0.copy()
    m = np.zeros_like(ref)
    v = np.zeros_like(ref)
    orc.adam(ref, gmean, m, v, 1, lr)
    np.testing.assert_allclose(net.params(), ref, rtol=1e-6, atol=lr * 1e-4)


def test_training_reduces_loss_and_roundtrip(holo, tmp_path):
    """Training drives the loss down on labels the network can represent
    (phase = pi * T, a pointwise function of the target), and also lowers it on
    GS-50 replay phases; save/load restores the network bit for bit."""
    n = 64
    net = holo.Cnn(seed=7)
    targets = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_CNN_TRAIN0 + i)).cuda() for i in range(8)]
    learnable = [torch.exp(1j * np.pi * t.to(torch.complex64)) for t in targets]
    first = [net.loss_grad(t, q)[0] for t, q in zip(targets, learnable)]
    for epoch in range(40):
        for t, q in zip(targets, learnable):
            net.train_step(t, q, 2e-3, want_loss=False)
    last = [net.loss_grad(t, q)[0] for t, q in zip(targets, learnable)]
    print(f"pointwise labels: mean loss {np.mean(first):.4f} -> {np.mean(last):.4f}")
    assert np.mean(last) < 0.5 * np.mean(first)

    gs_net = holo.Cnn(seed=9)
    lut = holo.Lut(4096, 1)
    labels = [holo.gs_iterate(t, 50, lut, 0, want_final=False)["field"].clone() for t in targets]
    first = [gs_net.loss_grad(t, q)[0] for t, q in zip(targets, labels)]
    for epoch in range(30):
        for t, q in zip(targets, labels):
            gs_net.train_step(t, q, 1e-3, want_loss=False)
    last = [gs_net.loss_grad(t, q)[0] for t, q in zip(targets, labels)]
    print(f"GS-50 labels: mean loss {np.mean(first):.4f} -> {np.mean(last):.4f}")
    assert np.mean(last) < np.mean(first)

    path = str(tmp_path / "net.bin")
    net.save(path)
    net2 = holo.Cnn(path=path)
    np.testing.assert_array_equal(net2.params(), net.params())
    assert torch.equal(net.infer(targets[0]), net2.infer(targets[0]))
    # the restored Adam state continues identically
    net.train_step(targets[1], learnable[1], 2e-3)
    net2.train_step(targets[1], learnable[1], 2e-3)
    np.testing.assert_array_equal(net2.params(), net.params())


def test_seed_comparison_runs(holo):
    """The learned-seed comparison reports iterations that are consistent with
    the per-iteration NMSE it was computed from."""
    from paper_2004_04049_amd import seed
    n = 64
    targets = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_CNN_HELDOUT0 + i)).cuda() for i in range(3)]
    lut = holo.Lut(4096, 1)
    net = holo.Cnn(seed=2)
    res = seed.compare(net, targets, lut, n_ref=20, max_iter=40)
    assert res["n"] == 3 and 0 <= res["reached"] <= 3
    for r, t in zip(res["rows"], targets):
        run = holo.gs_iterate(t, 40, None, 0, init_phasor=net.infer(t), want_final=False)
        if r["iters"] is not None:
            assert run["nmse"][r["iters"] - 1] <= r["goal_nmse"]
            assert r["iters"] == 1 or run["nmse"][r["iters"] - 2] > r["goal_nmse"]
        else:
            assert np.all(run["nmse"] > r["goal_nmse"])


def test_trained_seed_against_untrained_and_lut(holo):
    """End to end: train on seeded targets with LUT-seeded GS-50 labels, then
    on held-out targets count the GS iterations each seed needs to reach the
    NMSE that LUT-seeded GS reaches after 50 iterations (the LUT seed needs 50
    by definition).  Asserted: the training loss falls on the training set;
    both network seeds reach the goal on every held-out target within 100
    iterations and end 50 iterations below the LUT seed's NMSE; the books
    agree with the per-iteration NMSE.  The learned gain over the untrained
    network is reported, not asserted (at 1024^2 and 10k targets it is about
    one iteration in 45)."""
    from paper_2004_04049_amd import seed
    n = 256
    train = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_CNN_TRAIN0 + i)).cuda() for i in range(48)]
    held = [torch.from_numpy(synth.blob_target(n, n, synth.SEED_CNN_HELDOUT0 + i)).cuda() for i in range(6)]
    lut = holo.Lut(4096, 1)
    labels = seed.gs_labels(train, lut, 50)
    net = holo.Cnn(seed=1)
    before = np.mean([net.loss_grad(t, q)[0] for t, q in zip(train[:16], labels[:16])])
    hist = seed.train(net, train, labels, 3, 1e-3, batch=4)
    after = np.mean([net.loss_grad(t, q)[0] for t, q in zip(train[:16], labels[:16])])
    trained = seed.compare(net, held, lut, 50, 100)
    untrained = seed.compare(holo.Cnn(seed=1), held, lut, 50, 100)
    print(f"loss {before:.5f} -> {after:.5f} (epochs {hist['epoch_loss']}); iterations to the LUT GS-50 NMSE: "
          f"trained {trained['iters_mean']}, untrained {untrained['iters_mean']}, LUT 50; NMSE ratio at 50: "
          f"{trained['nmse_ratio_at_ref_mean']:.4f} / {untrained['nmse_ratio_at_ref_mean']:.4f}")
    assert after < before
    for res in (trained, untrained):
        assert res["reached"] == len(held)
        assert res["nmse_ratio_at_ref_mean"] < 1.0
        for r in res["rows"]:
            assert r["t_cnn_s"] is not None and r["t_infer_s"] > 0

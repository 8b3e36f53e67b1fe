"""Pins for the FP64 oracle of the learned GS seed (conv3x3 network, loss,
backward, Adam): impulse response and shift equivariance of the circular
convolution, loss invariances, central finite differences for every
parameter, and a worked Adam step.  CPU only."""
import numpy as np
import pytest


def test_conv_impulse_response_and_shift(orc):
    rng = np.random.default_rng(0)
    ny, nx = 5, 7
    w = rng.standard_normal((2, 1, 3, 3))
    x = np.zeros((1, ny, nx))
    y0, x0 = 1, 0
    x[0, y0, x0] = 1.0
    out = orc.conv3x3(x, w)
    for co in range(2):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                # input (y0, x0) reaches output (y0 - dy, x0 - dx) through tap (dy, dx)
                assert out[co, (y0 - dy) % ny, (x0 - dx) % nx] == pytest.approx(w[co, 0, dy + 1, dx + 1])
    assert np.count_nonzero(np.abs(out) > 0) == 18
    xr = rng.standard_normal((3, ny, nx))
    w3 = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    a = orc.conv3x3(np.roll(xr, (2, 3), axis=(1, 2)), w3, b)
    np.testing.assert_allclose(a, np.roll(orc.conv3x3(xr, w3, b), (2, 3), axis=(1, 2)), atol=1e-12)


def test_loss_invariances(orc):
    rng = np.random.default_rng(1)
    t = rng.random((6, 5)).astype(np.float32)
    q = np.exp(1j * rng.uniform(0, 2 * np.pi, (6, 5)))
    assert orc.cnn_loss(q, q, t) == pytest.approx(0.0, abs=1e-14)
    assert orc.cnn_loss(q * np.exp(0.7j), q, t) == pytest.approx(0.0, abs=1e-14)
    p = np.exp(1j * rng.uniform(0, 2 * np.pi, (6, 5)))
    L = orc.cnn_loss(p, q, t)
    assert 0.0 < L < 1.0
    # closed form equals the weighted mean of 1 - cos at the best global offset
    w = t.astype(float) ** 2
    d = np.angle(p * np.conj(q))
    c = np.angle(np.sum(w * np.exp(1j * d)))
    assert L == pytest.approx(np.sum(w * (1 - np.cos(d - c))) / np.sum(w), rel=1e-12)


def test_backward_matches_finite_differences(orc):
    rng = np.random.default_rng(2)
    C, ny, nx = 3, 6, 5
    n = orc.cnn_nparams(C)
    assert n == (9 * C + C) + 3 * (9 * C * C + C) + (9 * 2 * C + 2)
    params = rng.standard_normal(n) * 0.5
    t = (0.2 + rng.random((ny, nx))).astype(np.float32)
    q = np.exp(1j * rng.uniform(0, 2 * np.pi, (ny, nx)))
    loss, g = orc.cnn_backward(params, C, t, q)
    _, _, ph = orc.cnn_forward(params, C, t)
    assert loss == pytest.approx(orc.cnn_loss(ph, q, t), rel=1e-13)
    h = 1e-6
    fd = np.zeros(n)
    for i in range(n):
        pp = params.copy()
        pp[i] += h
        lp = orc.cnn_loss(orc.cnn_forward(pp, C, t)[2], q, t)
        pp[i] -= 2 * h
        lm = orc.cnn_loss(orc.cnn_forward(pp, C, t)[2], q, t)
        fd[i] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)
    assert np.abs(g).max() > 1e-3   # the check is not vacuous


def test_adam_worked_step(orc):
    p = np.array([1.0, -2.0])
    g = np.array([2.0, -0.5])
    m = np.zeros(2)
    v = np.zeros(2)
    orc.adam(p, g, m, v, 1, 0.1)
    # first step: m_hat = g, v_hat = g^2, so each parameter moves by lr*sign(g)
    np.testing.assert_allclose(p, [0.9, -1.9], atol=1e-7)
    np.testing.assert_allclose(m, [0.2, -0.05])
    np.testing.assert_allclose(v, [0.004, 0.00025])


def test_bf16_rounding_values(orc):
    # BF16 keeps 8 significant bits: spacing 2^-7 on [1, 2)
    assert orc.bf16(1.0) == 1.0
    assert orc.bf16(1.0 + 2.0 ** -8) == 1.0                        # tie -> even (1.0)
    assert orc.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6        # tie -> even (1 + 2^-6)
    assert orc.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert orc.bf16(-(1.0 + 2.0 ** -8 + 2.0 ** -20)) == -(1.0 + 2.0 ** -7)
    assert orc.bf16(0.0) == 0.0
    assert orc.bf16(3.0e38) == 226 / 128 * 2.0 ** 127               # 3e38 = 225.7/128 * 2^127
    rng = np.random.default_rng(3)
    for v in rng.standard_normal(200) * 10.0 ** rng.integers(-20, 20, 200):
        r = orc.bf16(v)
        m, e = np.frexp(r)
        assert m * 256 == np.round(m * 256)                        # 8 significant bits
        assert abs(r - v) <= 2.0 ** -9 * 2.0 ** e                  # half a spacing of r's binade


def test_bf16_storage_model(orc):
    """Rounding sits where the activations and hidden gradients are stored;
    the outcome stays within the BF16 error of the exact network."""
    rng = np.random.default_rng(4)
    C, ny, nx = 4, 8, 8
    n = orc.cnn_nparams(C)
    params = rng.standard_normal(n) * 0.4
    t = (0.2 + rng.random((ny, nx))).astype(np.float32)
    acts, out2, ph = orc.cnn_forward(params, C, t)
    acts_b, out2_b, ph_b = orc.cnn_forward(params, C, t, bf16_store=True)
    rb = np.vectorize(orc.bf16)
    np.testing.assert_array_equal(acts_b[0], rb(acts[0]))         # layer 1 sees the same input
    np.testing.assert_array_equal(acts_b, rb(acts_b))             # everything stored is BF16
    assert not np.array_equal(acts_b[3], acts[3])
    rel = np.linalg.norm(out2_b - out2) / np.linalg.norm(out2)
    assert 0 < rel < 4 * 2.0 ** -8
    q = np.exp(1j * rng.uniform(0, 2 * np.pi, (ny, nx)))
    l0, g0 = orc.cnn_backward(params, C, t, q)
    l1, g1 = orc.cnn_backward(params, C, t, q, bf16_store=True)
    assert l1 == pytest.approx(orc.cnn_loss(ph_b, q, t), rel=1e-13)
    assert abs(l1 - l0) < 0.05 * l0
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 0.05

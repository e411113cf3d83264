"""Pins of the predictor oracle (oracle/cnn_oracle.py) against definitions
that do not go through it: a brute-force loop convolution, translation
invariance, finite differences, the closed form of a first Adam step, and
bfloat16 rounding of hand-chosen values."""
import numpy as np
import pytest
import torch

import oracle
from oracle import cnn_oracle as co


def rand_params(seed, scale=0.3):
    r = np.random.default_rng(seed)
    return (r.standard_normal(co.CNN_PARAMS) * scale).astype(np.float32)


def rand_counts(seed, n, M, hi=6):
    return np.random.default_rng(seed).integers(0, hi, size=(n, M, M)).astype(np.uint8)


def brute_forward(counts, params):
    """Loop form of the network definition in float64 (no rounding)."""
    p = np.asarray(params, dtype=np.float64)
    n, M, _ = counts.shape
    preds = []
    for s in range(n):
        a = [counts[s].astype(np.float64) / 8.0]
        for ow, ob, cin in co.CONV:
            W = p[ow:ow + 16 * 9 * cin].reshape(16, 9, cin)
            z = np.zeros((16, M, M))
            for c in range(16):
                for y in range(M):
                    for x in range(M):
                        acc = p[ob + c]
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                tap = 3 * (dy + 1) + (dx + 1)
                                for ci in range(cin):
                                    acc += W[c, tap, ci] * a[ci][(y + dy) % M][(x + dx) % M]
                        z[c, y, x] = acc
            a = list(np.maximum(z, 0.0))
        feat = np.array([a[c].max() for c in range(16)])
        preds.append(p[co.OFF_BL] + feat @ p[co.OFF_WL:co.OFF_WL + 16])
    return np.array(preds)


def test_param_layout():
    assert co.OFF_BL + 1 == co.CNN_PARAMS == 7137
    assert co.OFF_B1 == co.OFF_W1 + 16 * 9 and co.OFF_W2 == co.OFF_B1 + 16
    for (ow, ob, cin), nxt in zip(co.CONV, [co.OFF_W2, co.OFF_W3, co.OFF_W4, co.OFF_WL]):
        assert ob == ow + 16 * 9 * cin and nxt == ob + 16


def test_forward_matches_loop_definition():
    counts = rand_counts(1, 2, 5)
    params = rand_params(2)
    got = co.forward(counts, params, "f64")["pred"].detach().numpy()
    want = brute_forward(counts, params)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_asymmetric_kernel_orientation():
    """A single weight at tap (dy, dx) = (1, -1) reads the input at (y+1, x-1)."""
    params = np.zeros(co.CNN_PARAMS, dtype=np.float32)
    params[co.OFF_W1 + 0 * 9 + 3 * 2 + 0] = 1.0       # channel 0, dy=+1, dx=-1
    for ow, _, cin in co.CONV[1:]:
        params[ow + 0 * 9 * cin + 4 * cin + 0] = 1.0   # identity tap on channel 0
    params[co.OFF_WL] = 1.0
    counts = np.zeros((1, 6, 6), dtype=np.uint8)
    counts[0, 2, 3] = 8
    out = co.forward(counts, params, "f64")
    assert out["pred"].item() == pytest.approx(1.0)
    # the maximum of channel 0 sits where (y+1, x-1) = (2, 3): y = 1, x = 4
    assert out["argmax"][0, 0] == 1 * 6 + 4


def test_translation_invariance():
    counts = rand_counts(3, 3, 12)
    params = rand_params(4)
    base = co.forward(counts, params, "f64")["pred"].detach().numpy()
    for dy, dx in ((1, 0), (0, 5), (7, 3)):
        sh = np.roll(counts, (dy, dx), axis=(1, 2))
        got = co.forward(sh, params, "f64")["pred"].detach().numpy()
        assert np.allclose(got, base, rtol=1e-12, atol=1e-12)


def test_gradient_matches_finite_differences():
    counts = rand_counts(5, 4, 8)
    params = rand_params(6).astype(np.float64)
    target = np.log1p(np.array([3.0, 4.0, 5.0, 9.0]))
    _, g, _ = co.loss_and_grad(counts, params, target, "f64")
    rng = np.random.default_rng(7)
    picks = []
    for off, count in ((co.OFF_W1, 160), (co.OFF_W2, 2320), (co.OFF_W3, 2320), (co.OFF_W4, 2320), (co.OFF_WL, 17)):
        picks += list(off + rng.choice(count, size=6, replace=False))
    h = 1e-6

    def loss(p):
        pred = co.forward(counts, p, "f64")["pred"].detach().numpy()
        return float(((pred - target) ** 2).mean())

    nz = 0
    for j in picks:
        pp, pm = params.copy(), params.copy()
        pp[j] += h
        pm[j] -= h
        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert fd == pytest.approx(g[j], rel=1e-5, abs=1e-8), j
        nz += abs(g[j]) > 1e-9
    assert nz >= len(picks) // 3  # the check is not vacuous


def test_bf16_rounding_values():
    v = torch.tensor([1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-8 + 2**-20, -(1 + 2**-8 + 2**-20), 3.0, 2**-130],
                     dtype=torch.float64)
    got = co.round_bf16(v).numpy()
    assert got[0] == 1.0                       # tie to even
    assert got[1] == 1 + 2**-6                 # tie to even (upwards)
    assert got[2] == 1 + 2**-7                 # above the tie
    assert got[3] == -(1 + 2**-7)
    assert got[4] == 3.0
    assert got[5] != 0.0                       # subnormals are kept


def test_bf16_mode_close_to_f64():
    counts = rand_counts(8, 4, 16)
    params = rand_params(9, 0.2)
    a = co.forward(counts, params, "f64")["pred"].detach().numpy()
    b = co.forward(counts, params, "bf16")["pred"].detach().numpy()
    assert np.allclose(a, b, rtol=5e-2, atol=5e-2)
    assert not np.array_equal(a, b)


def test_adam_first_step_closed_form():
    """After one step m_hat = g and v_hat = g^2: p1 = p0 - lr g / (|g| + eps)."""
    p0 = np.array([0.5, -1.0, 2.0, 0.0])
    g = np.array([0.1, -3.0, 0.0, 1e-3])
    p1, m, v = co.adam_step(p0, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected ratio stays g/|g|."""
    p, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    for t in range(1, 6):
        p, m, v = co.adam_step(p, np.array([0.25]), m, v, t, lr=0.1)
    assert p[0] == pytest.approx(1.0 - 5 * 0.1, rel=1e-6)


def test_init_distribution():
    params = co.init_params(12345, oracle.philox4x32_10)
    for off, count, fan in ((co.OFF_W2, 2304, 144), (co.OFF_W4, 2304, 144)):
        w = params[off:off + count].astype(np.float64)
        bound = np.sqrt(6.0 / fan)
        assert np.all(np.abs(w) < bound)
        assert abs(w.mean()) < 0.05 * bound
        assert w.std() == pytest.approx(bound / np.sqrt(3.0), rel=0.05)
    for ob in (co.OFF_B1, co.OFF_B2, co.OFF_B3, co.OFF_B4):
        assert np.all(params[ob:ob + 16] == 0)
    assert params[co.OFF_BL] == 0
    # parameter 0 from the generator's first word by hand
    w0 = int(oracle.philox4x32_10([0, co.INIT_TAG, 0, 0], [12345, 0])[0])
    assert params[0] == np.float32(((w0 + 0.5) / 2**32 * 2 - 1) * np.sqrt(6 / 9))


def test_block_counts():
    r = np.random.default_rng(10)
    s = (r.random((2, 32, 32)) < 0.1).astype(np.uint8)
    c = co.block_counts(s, 8)
    assert c.shape == (2, 4, 4)
    assert c.sum() == s.sum()
    assert c[1, 2, 3] == s[1, 16:24, 24:32].sum()

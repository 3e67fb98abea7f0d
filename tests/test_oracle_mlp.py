"""Pins of the FP64 MLP reference (learned start): calculus, closed forms, published Adam."""
import numpy as np
import pytest

from oracle import mlp
from oracle.splitmix import splitmix64_outputs


def _batch(rng, n):
    up = rng.integers(0, 1 << 16, n, dtype=np.uint64)
    dn = rng.integers(0, 1 << 16, n, dtype=np.uint64)
    return up, dn, rng.normal(-3.0, 1.0, n), rng.choice([-1.0, 1.0], n)


def _loss(theta, up, dn, la, sg):
    out, _ = mlp.forward(theta, up, dn, round_bf16=False)
    return mlp.loss_and_dout(out, la, sg)[0]


def _fd_check(backward, seed=3):
    rng = np.random.default_rng(seed)
    theta = mlp.init_params(seed)
    theta += rng.normal(0.0, 0.05, theta.shape)   # nonzero biases too
    up, dn, la, sg = _batch(rng, 7)
    out, cache = mlp.forward(theta, up, dn, round_bf16=False)
    _, dout = mlp.loss_and_dout(out, la, sg)
    g = backward(cache, dout)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 120, replace=False),
                          [0, 4095, 4096, 4223, 4224, 20607, 20608, 20991, 20992, 20993]])
    h = 1e-4   # central differences: truncation O(h^2) is far below the rounding of the loss at this step
    worst = 0.0
    for k in idx:
        tp = theta.copy(); tp[k] += h
        tm = theta.copy(); tm[k] -= h
        fd = (_loss(tp, up, dn, la, sg) - _loss(tm, up, dn, la, sg)) / (2 * h)
        worst = max(worst, abs(fd - g[k]) / max(abs(g[k]), abs(fd), 1e-6))
    return worst


def test_parameter_count_and_layout():
    assert mlp.N_PARAMS == 20994
    p = mlp.unpack(np.arange(mlp.N_PARAMS, dtype=np.float64))
    assert p["W1"][0, 0] == 0 and p["b1"][0] == 4096 and p["W2"][0, 0] == 4224
    assert p["b2"][0] == 20608 and p["W3"][0, 0] == 20736 and p["b3"][1] == 20993


def test_gradient_matches_finite_differences():
    assert _fd_check(mlp.backward) <= 1e-6


def test_planted_missing_tanh_derivative_is_caught():
    def bad(cache, dout):
        x, h1, h2, W2, W3 = cache["x"], cache["h1"], cache["h2"], cache["W2"], cache["W3"]
        dz2 = dout @ W3                      # (1 - h2^2) dropped
        dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
        parts = {"W3": dout.T @ h2, "b3": dout.sum(0), "W2": dz2.T @ h1, "b2": dz2.sum(0),
                 "W1": dz1.T @ x, "b1": dz1.sum(0)}
        return np.concatenate([parts[n].ravel() for n, _ in mlp.SIZES])
    assert _fd_check(bad) > 1e-2


def test_forward_closed_form_with_zero_first_and_second_layer_weights():
    rng = np.random.default_rng(1)
    theta = np.zeros(mlp.N_PARAMS)
    p = mlp.unpack(theta)
    p["b1"][...] = rng.normal(size=128)
    p["b2"][...] = rng.normal(size=128)
    p["W3"][...] = rng.normal(size=(2, 128))
    p["b3"][...] = [0.25, -1.5]
    up, dn, _, _ = _batch(rng, 5)
    out, _ = mlp.forward(theta, up, dn, round_bf16=False)
    expect = p["W3"] @ np.tanh(p["b2"]) + p["b3"]
    assert np.allclose(out, expect[None, :], rtol=0, atol=1e-14)


def test_forward_single_path_by_hand():
    # one unit per layer carries x_3 (up site 3) through: o_0 = w3 tanh(w2 tanh(w1 x_3))
    theta = np.zeros(mlp.N_PARAMS)
    p = mlp.unpack(theta)
    p["W1"][5, 3] = 0.7
    p["W2"][9, 5] = -1.3
    p["W3"][0, 9] = 2.0
    up = np.array([0b1000, 0b0000], dtype=np.uint64)
    dn = np.array([0, 0xFFFF], dtype=np.uint64)
    out, _ = mlp.forward(theta, up, dn, round_bf16=False)
    for k, x3 in enumerate([1.0, -1.0]):
        assert out[k, 0] == pytest.approx(2.0 * np.tanh(-1.3 * np.tanh(0.7 * x3)), abs=1e-15)
        assert out[k, 1] == 0.0


def test_features_are_plus_minus_one_per_site():
    x = mlp.features(np.array([0b101], dtype=np.uint64), np.array([1 << 15], dtype=np.uint64))
    assert x[0, 0] == 1 and x[0, 1] == -1 and x[0, 2] == 1 and x[0, 3] == -1
    assert x[0, 16] == -1 and x[0, 31] == 1 and np.all(np.abs(x) == 1)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    cases = {one: one, one + 2 ** -8: one, one + 3 * 2 ** -8: one + 2 ** -6,
             one + 2 ** -8 + 2 ** -20: one + 2 ** -7, -(one + 2 ** -8): -one, 0.0: 0.0,
             3.0: 3.0, 2 ** -130: 2 ** -130}
    for a, b in cases.items():
        assert mlp.bf16_round(np.array([a]))[0] == b, a


def test_loss_at_known_points():
    out = np.array([[-2.0, 0.0], [1.0, 0.0]])
    loss, dout = mlp.loss_and_dout(out, np.array([-2.0, 0.5]), np.array([1.0, -1.0]))
    assert loss == pytest.approx((0.0 + 0.25 + 2 * np.log(2.0)) / 2, abs=1e-15)
    assert dout[0, 0] == 0.0 and dout[1, 0] == pytest.approx(0.5)
    assert dout[0, 1] == pytest.approx(-0.25) and dout[1, 1] == pytest.approx(0.25)


def test_adam_with_constant_gradient_moves_by_lr_each_step():
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for step in range(1, 4):
        new, m, v = mlp.adam_step(th, g, m, v, step, lr=0.01, eps=1e-8)
        assert np.allclose(new - th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        th = new


def test_adam_second_step_by_hand():
    g1, g2 = 0.5, -1.0
    _, m, v = mlp.adam_step(np.zeros(1), np.array([g1]), np.zeros(1), np.zeros(1), 1, lr=0.1)
    th, m, v = mlp.adam_step(np.zeros(1), np.array([g2]), m, v, 2, lr=0.1, eps=0.0)
    m2 = 0.9 * 0.1 * g1 + 0.1 * g2
    v2 = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    expect = -0.1 * (m2 / (1 - 0.81)) / np.sqrt(v2 / (1 - 0.999 ** 2))
    assert th[0] == pytest.approx(expect, rel=1e-14)


def test_sampling_by_brute_force():
    psi = np.array([0.0, 0.3, -0.1, 0.0, 0.9, -0.2, 1e-6, 0.4])
    w = mlp.quantised_weights(psi)
    assert w[4] == 2 ** 32 and w[0] == 0 and w[3] == 0
    got = mlp.sample_indices(psi, 11, 5, 200)
    zs = splitmix64_outputs(11, 205)[5:]
    W = int(w.sum())
    for j, z in enumerate(zs):
        t = (z * W) >> 64
        acc, r = 0, 0
        while acc + int(w[r]) <= t:     # first r whose inclusive prefix exceeds t
            acc += int(w[r])
            r += 1
        assert got[j] == r
    assert not np.isin(got, [0, 3]).any()


def test_sampling_frequencies_follow_psi_squared():
    psi = np.array([1.0, -2.0, 0.5, 3.0])
    got = mlp.sample_indices(psi, 5, 0, 20000)
    freq = np.bincount(got, minlength=4) / 20000
    p = psi ** 2 / np.sum(psi ** 2)
    assert np.all(np.abs(freq - p) < 0.02), (freq, p)


def test_start_vector_signs_and_layout():
    theta = np.zeros(mlp.N_PARAMS)
    p = mlp.unpack(theta)
    p["b3"][...] = [-1.0, 0.0]
    p["W1"][0, 0] = 5.0          # unit 0 follows x_0 (up site 0)
    p["W2"][0, 0] = 5.0
    p["W3"][1, 0] = 1.0          # sign logit = h2_0: + when up site 0 is occupied
    v = mlp.start_vector(theta, [0b01, 0b10], [0b1, 0b10, 0b100], round_bf16=False)
    assert v.shape == (6,)
    assert np.all(np.abs(np.abs(v) - np.exp(-1.0)) < 1e-15)
    assert np.all(v[:3] > 0) and np.all(v[3:] < 0)

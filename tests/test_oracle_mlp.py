"""Pins of the learned-warm-start oracle (oracle/mlp.py) against values that
do not come from the oracle itself: hand-evaluated features and head, the
closed form of the zero network's loss, a central-difference gradient, and
the first Adam step (which moves each parameter by lr * sign(g))."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, n=9):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=n) + 1j * rng.normal(size=n)
    r = 0.3 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    D = -rng.uniform(1.5, 6.0, size=n)
    t = u + r / D + 0.05 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    return u, r, D, t


def test_features_by_hand():
    # u = 3 + 4i (|u| = 5), r = -2, D = -2 -> v = 1, s = 6
    x, v, s = mlp.features(np.array([3 + 4j]), np.array([-2 + 0j]), np.array([-2.0]))
    ref = [0.5, 4 / 6, 1 / 6, 0.0, np.log(1 / 5) / 10, -0.2, np.log(6) / 10, 1 / 6]
    assert np.allclose(x[0], ref, rtol=0, atol=1e-15)
    assert v[0] == 1.0 and abs(s[0] - 6.0) < 1e-15


def test_feature_clip_and_zero_amplitude():
    x, _, _ = mlp.features(np.array([0j]), np.array([1e-3 + 0j]), np.array([-1.0]))
    assert x[0, 4] == 1.0            # ln ratio clipped at +10, scaled by 1/10
    assert x[0, 0] == 0.0 and x[0, 1] == 0.0


def test_head_by_hand():
    y = np.array([[0.5, -1.0, 2.0, 0.25]])
    u, v = np.array([1 + 1j]), np.array([2 - 1j])
    a, b = 0.5 - 1j, 2.0 + 0.25j
    assert np.allclose(mlp.predict(y, u, v), u + v + a * v + b * u, atol=0)
    # by hand: u + v = 3, a v = (0.5 - i)(2 - i) = -2.5i, b u = (2 + 0.25i)(1 + i) = 1.75 + 2.25i
    assert abs(mlp.predict(y, u, v)[0] - (4.75 - 0.25j)) < 1e-14


def test_zero_network_loss_closed_form():
    u, r, D, t = _data(1)
    x, v, s = mlp.features(u, r, D)
    p = np.zeros(mlp.n_params())
    y, _ = mlp.forward(p, x)
    assert np.all(y == 0)
    L, _ = mlp.loss_and_dy(y, u, v, t, s)
    ref = np.mean(np.abs(u + r / D - t) ** 2 / (np.abs(u) + np.abs(r / D) + 1e-30) ** 2)
    assert abs(L - ref) <= 1e-14 * ref


def test_absolute_loss_closed_form():
    u, r, D, t = _data(4)
    x, v, s = mlp.features(u, r, D)
    y = np.zeros((u.size, 4))
    L, _ = mlp.loss_and_dy(y, u, v, t, s, mode=1)
    ref = np.sum(np.abs(u + r / D - t) ** 2) / np.sum((np.abs(u) + np.abs(r / D) + 1e-30) ** 2)
    assert abs(L - ref) <= 1e-14 * ref


@pytest.mark.parametrize("mode", [0, 1])
def test_gradient_central_differences(mode):
    u, r, D, t = _data(2, n=11)
    x, v, s = mlp.features(u, r, D)
    rng = np.random.default_rng(3)
    p = 0.2 * rng.normal(size=mlp.n_params())
    L, g = mlp.loss_and_grad(p, x, u, v, t, s, mode)
    idx = rng.choice(p.size, 60, replace=False)
    # include coordinates of every parameter block
    offs = np.cumsum([0] + [int(np.prod(q)) for q in mlp.SHAPES])
    idx = np.concatenate([idx, offs[:-1], offs[1:] - 1])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        Lp, _ = mlp.loss_and_grad(p + e, x, u, v, t, s, mode)
        Lm, _ = mlp.loss_and_grad(p - e, x, u, v, t, s, mode)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g).max()), (k, fd, g[k])


def test_first_adam_step_is_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.5, -3.0, 1e-3])
    q, m, w = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.1)
    assert np.allclose(q, p - 0.1 * np.sign(g), rtol=0, atol=1e-6)
    assert np.allclose(m, 0.1 * g) and np.allclose(w, 0.001 * g * g)

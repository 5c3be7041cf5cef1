"""Warm-start kernels (features, head, FP32 MLP forward / backward, Adam)
against the FP64 oracle (oracle/mlp.py).  The GPU runs the network in fp32
with fp32 accumulation over at most 256 terms per output, so its values and
gradients agree with the FP64 oracle to a relative 1e-4 of the largest
entry (fp32 unit roundoff 6e-8 times the accumulation length, with margin)."""
import numpy as np
import pytest

from oracle import mlp as O

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dev(x):
    return _torch().from_numpy(np.ascontiguousarray(x)).to("cuda")


def _rows(seed, n):
    rng = np.random.default_rng(seed)
    u = 0.05 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    r = 0.01 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    D = -rng.uniform(1.5, 8.0, size=n)
    t = u + r / D + 0.003 * (rng.normal(size=n) + 1j * rng.normal(size=n))
    u[:3] = 0.0          # zero-amplitude rows (zero-size or symmetry-forbidden pattern)
    return u, r, D, t


def _params(seed, scale=0.1):
    rng = np.random.default_rng(seed)
    return (scale * rng.normal(size=O.n_params())).astype(np.float32)


def test_features_head_step_match_oracle():
    torch = _torch()
    import paper_2004_03682_amd as F
    u, r, D, t = _rows(1, 3001)
    X = torch.empty((u.size, 8), dtype=torch.float32, device="cuda")
    F.ws_features(dev(u), dev(r), dev(D), X)
    x, v, s = O.features(u, r, D)
    assert np.abs(X.cpu().numpy() - x).max() <= 1e-6
    Y = np.random.default_rng(2).normal(size=(u.size, 4)).astype(np.float32)
    out = torch.empty(u.size, dtype=torch.complex128, device="cuda")
    F.ws_apply(dev(Y), dev(u), dev(r), dev(D), out)
    ref = O.predict(Y.astype(np.float64), u, v)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-15
    F.ws_apply(None, dev(u), dev(r), dev(D), out)
    assert np.abs(out.cpu().numpy() - (u + v)).max() <= 1e-16
    F.ws_step(dev(u), dev(r), dev(D), out)
    assert np.abs(out.cpu().numpy() - (u + r / D)).max() <= 1e-16
    F.ws_step(None, dev(r), dev(D), out)
    assert np.abs(out.cpu().numpy() - r / D).max() <= 1e-16


def test_forward_matches_oracle():
    torch = _torch()
    import paper_2004_03682_amd as F
    p = _params(3)
    net = F.MLP(seed=0)
    net.set_params(p)
    assert np.array_equal(net.get_params(), p)
    for n in (1, 70, 4099):
        X = np.random.default_rng(n).normal(size=(n, 8)).astype(np.float32)
        Y = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        net.forward(dev(X), Y)
        ref, _ = O.forward(p.astype(np.float64), X.astype(np.float64))
        assert np.abs(Y.cpu().numpy() - ref).max() <= 1e-4 * np.abs(ref).max(), n
    net.destroy()


@pytest.mark.parametrize("gather,mode", [(False, 0), (True, 0), (False, 1), (True, 1)])
def test_loss_and_gradient_match_oracle(gather, mode):
    torch = _torch()
    import paper_2004_03682_amd as F
    u, r, D, t = _rows(4, 5000)
    p = _params(5)
    net = F.MLP(seed=0)
    net.set_params(p)
    if gather:
        idx = np.random.default_rng(6).choice(u.size, 1777, replace=False)
        L = net.loss_grad(dev(u), dev(r), dev(D), dev(t), idx=dev(idx.astype(np.int64)), mode=mode)
        u, r, D, t = u[idx], r[idx], D[idx], t[idx]
    else:
        L = net.loss_grad(dev(u), dev(r), dev(D), dev(t), mode=mode)
    g = net.get_grad()
    x, v, s = O.features(u, r, D)
    x = x.astype(np.float32).astype(np.float64)        # the network sees fp32 features
    Lo, go = O.loss_and_grad(p.astype(np.float64), x, u, v, t, s, mode)
    assert abs(L - Lo) <= 1e-4 * Lo
    offs = np.cumsum([0] + [int(np.prod(q)) for q in O.SHAPES])
    for k in range(len(O.SHAPES)):
        a, b = g[offs[k]:offs[k + 1]], go[offs[k]:offs[k + 1]]
        assert np.abs(a - b).max() <= 1e-4 * np.abs(go).max() + 1e-4 * np.abs(b).max(), k
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    net.destroy()


def test_adam_steps_match_oracle():
    import paper_2004_03682_amd as F
    u, r, D, t = _rows(7, 2000)
    p = _params(8)
    net = F.MLP(seed=0)
    net.set_params(p)
    q = p.astype(np.float64)
    m = np.zeros_like(q)
    w = np.zeros_like(q)
    for n, lr in ((1, 1e-3), (2, 5e-4), (3, 5e-4)):
        net.loss_grad(dev(u), dev(r), dev(D), dev(t))
        g = net.get_grad().astype(np.float64)
        net.adam(lr)
        q, m, w = O.adam_step(q, g, m, w, n, lr)
        got = net.get_params().astype(np.float64)
        assert np.abs(got - q).max() <= 1e-6 * max(1.0, np.abs(q).max()), n
    net.destroy()


def test_untrained_network_is_the_second_jacobi_iterate_and_training_lowers_the_loss():
    torch = _torch()
    import paper_2004_03682_amd as F
    u, r, D, _ = _rows(9, 20000)
    v = r / D
    t = u + v + (0.3 + 0.05 * D) * v + 0.2j * u     # a learnable correction: a = 0.3 + 0.05 D, b = 0.2 i
    net = F.MLP(seed=11)
    Y = torch.empty((u.size, 4), dtype=torch.float32, device="cuda")
    X = torch.empty((u.size, 8), dtype=torch.float32, device="cuda")
    F.ws_features(dev(u), dev(r), dev(D), X)
    net.forward(X, Y)
    assert torch.count_nonzero(Y).item() == 0
    du, dr, dD, dt = dev(u), dev(r), dev(D), dev(t)
    L0 = net.loss_grad(du, dr, dD, dt)
    for _ in range(200):
        net.loss_grad(du, dr, dD, dt)
        net.adam(1e-3)
    L1 = net.loss_grad(du, dr, dD, dt)
    print("loss", L0, "->", L1, flush=True)
    assert L1 < 0.2 * L0
    net.destroy()

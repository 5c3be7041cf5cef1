"""CPU FP64 oracle of the learned warm start (test infrastructure).

Only tests, the smoke check and the benchmark's CPU baseline use this module;
the product path runs the same definition in its own HIP kernels.

Definition (one packed T2 element k of a system):
  u = MP2 amplitude (first Jacobi iterate from zero: <ab||ij>/D, Eq. (3) with
      t = 0), v = R(u) / D = the next Jacobi correction (R = CCSD residual of
      Eq. (3) at u, D = e_i + e_j - e_a - e_b).
  scale   s = |u| + |v| + 1e-30
  features x (8, float):
      Re u/s, Im u/s, Re v/s, Im v/s,
      clip(ln((|v| + 1e-30) / (|u| + 1e-30)), -10, 10) / 10,
      D / 10, ln(s) / 10, |v| / s
  network  h1 = relu(x W1 + b1) (8 -> 256), h2 = relu(h1 W2 + b2) (256 -> 256),
           y = h2 W3 + b3 (256 -> 4); W stored [in][out]
  head     a = y0 + i y1, b = y2 + i y3;  t_pred = u + v + a v + b u
           (y = 0 gives the ordinary second Jacobi iterate u + v)
  loss     mode 0 (relative):  L = (1/N) sum_k |t_pred_k - t_k|^2 / s_k^2
           mode 1 (absolute):  L = sum_k |t_pred_k - t_k|^2 / sum_k s_k^2
           (t = converged T2; mode 1 weights elements by their size)
  Adam     (Kingma & Ba, ICLR 2015) with bias correction:
           m = b1 m + (1-b1) g,  w = b2 w + (1-b2) g^2,
           p -= lr * (m / (1-b1^n)) / (sqrt(w / (1-b2^n)) + eps)
Parameters are one flat vector in the order W1, b1, W2, b2, W3, b3.
"""
from __future__ import annotations

import numpy as np

F_IN, HID, F_OUT = 8, 256, 4
SHAPES = [(F_IN, HID), (HID,), (HID, HID), (HID,), (HID, F_OUT), (F_OUT,)]


def n_params():
    return int(sum(int(np.prod(s)) for s in SHAPES))


def unflatten(p):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    return out


def features(u, r, D):
    """x[N, 8] from complex u, complex residual r and real denominators D."""
    u = np.asarray(u, np.complex128)
    v = np.asarray(r, np.complex128) / np.asarray(D, np.float64)
    au, av = np.abs(u), np.abs(v)
    s = au + av + 1e-30
    x = np.empty((u.size, F_IN))
    x[:, 0] = u.real / s
    x[:, 1] = u.imag / s
    x[:, 2] = v.real / s
    x[:, 3] = v.imag / s
    x[:, 4] = np.clip(np.log((av + 1e-30) / (au + 1e-30)), -10.0, 10.0) / 10.0
    x[:, 5] = np.asarray(D, np.float64) / 10.0
    x[:, 6] = np.log(s) / 10.0
    x[:, 7] = av / s
    return x, v, s


def forward(p, x):
    W1, b1, W2, b2, W3, b3 = unflatten(p)
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (x, h1, h2)


def predict(y, u, v):
    a = y[:, 0] + 1j * y[:, 1]
    b = y[:, 2] + 1j * y[:, 3]
    return u + v + a * v + b * u


def loss_and_dy(y, u, v, t, s, mode=0):
    """Loss and dL/dy for the head above (mode 0 relative, 1 absolute)."""
    n = y.shape[0]
    e = predict(y, u, v) - t
    if mode == 0:
        w = 1.0 / (s * s) / n
    else:
        w = np.full(n, 1.0 / np.sum(s * s))
    L = float(np.sum(np.abs(e) ** 2 * w))
    ce = np.conj(e)
    dy = np.empty_like(y)
    dy[:, 0] = 2.0 * np.real(ce * v) * w
    dy[:, 1] = -2.0 * np.imag(ce * v) * w
    dy[:, 2] = 2.0 * np.real(ce * u) * w
    dy[:, 3] = -2.0 * np.imag(ce * u) * w
    return L, dy


def backward(p, cache, dy):
    """Gradient of the loss w.r.t. the flat parameter vector, given dL/dy."""
    W1, b1, W2, b2, W3, b3 = unflatten(p)
    x, h1, h2 = cache
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    dh2 = (dy @ W3.T) * (h2 > 0)
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ W2.T) * (h1 > 0)
    gW1 = x.T @ dh1
    gb1 = dh1.sum(0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def loss_and_grad(p, x, u, v, t, s, mode=0):
    y, cache = forward(p, x)
    L, dy = loss_and_dy(y, u, v, t, s, mode)
    return L, backward(p, cache, dy)


def adam_step(p, g, m, w, n, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number n >= 1); returns new (p, m, w)."""
    m = b1 * m + (1.0 - b1) * g
    w = b2 * w + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** n)
    wh = w / (1.0 - b2 ** n)
    return p - lr * mh / (np.sqrt(wh) + eps), m, w

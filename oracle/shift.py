"""Dynamic denominator shifts and Pade extrapolation to the zero-shift limit
(test infrastructure; CPU, FP64).

The paper (section on the FS-RCC method, intruder states) modifies the
amplitude equations of Eq. (3) by shifting ill-defined (nearly zero or
positive) energy denominators and extrapolates the results to zero shift
with Pade approximants; it gives no formulas.  Reading used here (the same
for the oracle and the library):

  shifted equations   (D_K + Delta_K) s_K = RHS_K(s),  i.e.  R_K(s) = Delta_K s_K
                      with R the unshifted residual (R = RHS - D s, so a
                      zero shift gives back Eq. (3));
  shift of one amplitude   Delta_K = S (S / (min(D_K, 0) + S))^n,
                      S < 0 the shift of the sector, n >= 1 the attenuation
                      exponent: Delta = S where D = 0, and Delta ~ S (S/D)^n
                      -> 0 for |D| >> |S|, so well-separated denominators are
                      left almost unchanged;
  Jacobi step          s <- s + (R - Delta s) / (D + Delta);
  extrapolation        solve at shifts lambda_i S, fit each state energy by
                       a Pade approximant [L/M] in lambda
                       E(lambda) ~ (a_0 + ... + a_L lambda^L) /
                                   (1 + b_1 lambda + ... + b_M lambda^M)
                       (linearised least squares over the points), and report
                       E(0) = a_0.
"""
from __future__ import annotations

import numpy as np


def delta(D, S, n):
    """Delta_K for denominators D (array), sector shift S <= 0 and exponent n >= 1."""
    D = np.asarray(D, np.float64)
    if S == 0.0:
        return np.zeros_like(D)
    if not (S < 0.0) or int(n) != n or n < 1:
        raise ValueError("shift needs S < 0 and an integer n >= 1")
    q = S / (np.minimum(D, 0.0) + S)
    return S * q ** int(n)


def pade_fit(x, y, L, M):
    """Coefficients (a[0..L], b[1..M]) of the [L/M] Pade approximant through
    the points (x_i, y_i) (complex y allowed): least squares of the
    linearised conditions  sum_j a_j x^j - y sum_{j>=1} b_j x^j = y."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.complex128)
    if x.size < L + M + 1:
        raise ValueError("need at least L + M + 1 points")
    cols = [x ** j for j in range(L + 1)] + [-y * x ** j for j in range(1, M + 1)]
    A = np.stack(cols, axis=1).astype(np.complex128)
    c, *_ = np.linalg.lstsq(A, y, rcond=None)
    return c[: L + 1], c[L + 1:]


def pade_eval(a, b, x0):
    num = sum(aj * x0 ** j for j, aj in enumerate(a))
    den = 1.0 + sum(bj * x0 ** (j + 1) for j, bj in enumerate(b))
    return num / den


def pade(x, y, L, M, x0=0.0):
    """Value at x0 of the [L/M] Pade approximant fitted to (x, y)."""
    a, b = pade_fit(x, y, L, M)
    return pade_eval(a, b, x0)

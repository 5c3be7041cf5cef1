"""Jacobi + DIIS(6) driver of the oracle (test infrastructure).

Update (Eq. (3) read as a fixed-point iteration):  step = R / D,  t' = t + step.
DIIS (Pulay), with the error vector e = step:
  * keep the last `ndiis` pairs (t'_k, e_k);
  * once two or more are held, B_kl = Re sum conj(e_k) e_l over the unique
    amplitudes (all of T1; i<j, a<b of T2, i.e. 1/4 of the full T2 sum),
    solve [[B, -1], [-1, 0]] [c; lam] = [0; -1] and set t = sum_k c_k t'_k;
    B is scaled by 1/max(diag B) before the solve (c is unchanged by it);
  * if the bordered matrix is numerically singular the oldest pair is dropped.
Convergence: max |step| over the amplitudes < tol (the step of the last
residual evaluation).  The energy is evaluated on the updated amplitudes.
"""
from __future__ import annotations

import time

import numpy as np

from . import ccsd


def diis_coefficients(B: np.ndarray) -> np.ndarray:
    """Bordered Pulay system; returns c with sum c = 1 (raises if singular)."""
    m = B.shape[0]
    scale = np.max(np.abs(np.diag(B)))
    A = np.zeros((m + 1, m + 1))
    A[:m, :m] = B / (scale if scale > 0 else 1.0)
    A[:m, m] = -1.0
    A[m, :m] = -1.0
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    if np.linalg.cond(A) > 1e14:
        raise np.linalg.LinAlgError("singular DIIS matrix")
    return np.linalg.solve(A, rhs)[:m]


def solve_ccsd(be, tol=1e-10, maxit=200, ndiis=6, log=None, t_init=None):
    """Converge the CCSD amplitudes.  Returns dict(t1, t2, E, iters, history)."""
    t1, t2 = (be.zeros_t1(), be.zeros_t2()) if t_init is None else t_init
    hist_t, hist_e, hist_B = [], [], []
    history = []
    converged = False
    for k in range(1, maxit + 1):
        t0 = time.perf_counter()
        R1, R2 = ccsd.residual(be, t1, t2)
        s1, s2 = R1 / be.D1, R2 / be.D2
        t1n, t2n = t1 + s1, t2 + s2
        dmax = max(be.absmax(s1), be.absmax(s2))
        if ndiis > 1:
            hist_t.append((t1n, t2n))
            hist_e.append((s1, s2))
            if len(hist_t) > ndiis:
                hist_t.pop(0)
                hist_e.pop(0)
            while len(hist_t) >= 2:
                m = len(hist_e)
                B = np.zeros((m, m))
                for a in range(m):
                    for b in range(m):
                        B[a, b] = (be.vdot(hist_e[a][0], hist_e[b][0]) + 0.25 * be.vdot(hist_e[a][1], hist_e[b][1])).real
                try:
                    c = diis_coefficients(B)
                except np.linalg.LinAlgError:
                    hist_t.pop(0)
                    hist_e.pop(0)
                    continue
                t1n = be.lincomb(list(c), [x[0] for x in hist_t])
                t2n = be.lincomb(list(c), [x[1] for x in hist_t])
                break
        t1, t2 = t1n, t2n
        E = ccsd.energy(be, t1, t2)
        dt = time.perf_counter() - t0
        history.append(dict(iter=k, E=E, dmax=dmax, seconds=dt))
        if log:
            log(f"iter {k:3d}  E = {E.real:+.14f} {E.imag:+.3e}i  max|step| = {dmax:.3e}  {dt:.2f}s")
        if dmax < tol:
            converged = True
            break
    return dict(t1=t1, t2=t2, E=E, iters=k, converged=converged, history=history)

"""Pins of the dynamic-shift and Pade-extrapolation oracle (no GPU).

* Delta(D) against its closed-form properties: Delta(0) = S, the asymptote
  S^(n+1) / D^n for |D| >> |S|, monotone decay, and the sharp lower bound
  min_D |D + Delta(D)| = |S| c_n with c_n from the stationary point
  (1 + u)^(n+1) = n (u = -D/|S|);
* the Pade fit reproduces exact rational and polynomial data and their value
  at 0, and refuses under-determined fits;
* the (0h,1p) chain: energies solved with shifts lambda*S and extrapolated
  to lambda = 0 land much closer to the brute-force EA-EOM (FCI-based)
  eigenvalues than the shifted energies themselves, and a zero shift gives
  the unshifted solution.
"""
import numpy as np
import pytest

import fsgen
from oracle import ccsd, fock, fs01, shift, solver


@pytest.mark.parametrize("S,n", [(-0.5, 1), (-0.5, 3), (-2.0, 2), (-0.1, 5)])
def test_delta_closed_form(S, n):
    assert shift.delta(0.0, S, n) == pytest.approx(S, abs=0)
    assert shift.delta(5.0, S, n) == pytest.approx(S, abs=0)          # positive D treated as D = 0
    D = -1e6
    assert shift.delta(D, S, n) / (S ** (n + 1) / D ** n) == pytest.approx(1.0, rel=1e-5)
    Ds = -np.geomspace(1e-6, 1e3, 400)
    d = shift.delta(Ds, S, n)
    assert np.all(d < 0) and np.all(np.diff(np.abs(d)) < 0)           # |Delta| decays as D moves away from 0
    # sharp bound on the shifted denominator: |D + Delta| >= c_n |S|
    u = n ** (1.0 / (n + 1)) - 1.0                                    # stationary point in units of |S|
    c_n = u + (1.0 / (1.0 + u)) ** n
    Dd = -np.linspace(0.0, 10 * abs(S), 200001)
    m = np.abs(Dd + shift.delta(Dd, S, n)).min()
    assert m >= c_n * abs(S) * (1 - 1e-12)
    assert m == pytest.approx(c_n * abs(S), rel=1e-6)
    assert np.all(shift.delta(Ds, 0.0, n) == 0.0)


def test_delta_rejects_bad_parameters():
    for S, n in [(0.5, 3), (-0.5, 0), (-0.5, 1.5)]:
        with pytest.raises(ValueError):
            shift.delta(-1.0, S, n)


def test_pade_exact_on_rational_and_polynomial_data():
    lam = np.array([1.0, 0.8, 0.6, 0.4, 0.2])
    f = (2.0 - 1.0j + 3.0 * lam) / (1.0 + 0.5 * lam)                 # an exact [1/1] function
    assert abs(shift.pade(lam, f, 1, 1) - (2.0 - 1.0j)) < 1e-12
    assert abs(shift.pade(lam, f, 1, 1, x0=2.0) - (8.0 - 1.0j) / 2.0) < 1e-12
    g = 0.3 - 0.2 * lam + 0.7j * lam ** 2                              # an exact [2/0] function
    assert abs(shift.pade(lam, g, 2, 0) - 0.3) < 1e-12
    assert abs(shift.pade(lam, g, 2, 1) - 0.3) < 1e-10                # over-parametrised still exact
    with pytest.raises(ValueError):
        shift.pade(lam[:2], f[:2], 1, 1)


def _system(no, nv, ni, seed, nact, sg=0.1):
    s = fsgen.make_system(no, nv, ni, sg, seed, nact=nact)
    fs = fock.FockSpace(s.eps, fsgen.full_tensor(s), no)
    be = ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-13)
    M, _ = fock.ea_matrix(fs, r["t1"], r["t2"], fs.E_ref + r["E"])
    return s, be, r, np.linalg.eigvals(M)


@pytest.mark.parametrize("no,nv,ni,seed,nact", [(2, 5, 1, 3, 2), (3, 5, 1, 5, 2), (2, 6, 2, 11, 3)])
@pytest.mark.parametrize("n", [1, 3])
def test_extrapolated_shifted_energies_approach_ea_eigenvalues(no, nv, ni, seed, nact, n):
    s, be, r, wM = _system(no, nv, ni, seed, nact)
    lams = [1.0, 0.8, 0.6, 0.4, 0.2]
    E, st = [], None
    for lam in lams:
        F = fs01.FS01(be, r["t1"], r["t2"], s.active, shift=(-0.5 * lam, n))
        o = fs01.solve_fs01(F, tol=1e-12, start=st)
        assert o["converged"]
        st = (o["s1"], o["s2"])
        E.append(o["eig"])
    E = np.array(E)
    # exact targets: for every state the nearest eigenvalue of the brute-force EA matrix
    exact = np.array([wM[np.argmin(np.abs(wM - e))] for e in E[-1]])
    ext = np.array([shift.pade(lams, E[:, k], 2, 1) for k in range(E.shape[1])])
    err_shifted = np.abs(E[0] - exact).max()
    err_ext = np.abs(ext - exact).max()
    assert err_shifted > 1e-5                       # the shift does change the energies
    assert err_ext < 0.25 * err_shifted, (err_ext, err_shifted)


def test_zero_shift_is_the_unshifted_solution():
    s, be, r, _ = _system(2, 5, 1, 3, 2)
    a = fs01.solve_fs01(fs01.FS01(be, r["t1"], r["t2"], s.active), tol=1e-12)
    b = fs01.solve_fs01(fs01.FS01(be, r["t1"], r["t2"], s.active, shift=(0.0, 3)), tol=1e-12)
    assert np.abs(a["eig"] - b["eig"]).max() == 0.0 and a["iters"] == b["iters"]

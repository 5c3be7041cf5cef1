"""Real-double-group stand-in (no GPU): the generator's real systems and the
oracle on them.

* V = sqrt(2) Re V_complex is exactly real, antisymmetric in (pq) and (rs),
  symmetric under (pq) <-> (rs), zero outside allowed blocks, with the
  complex draw's element variance sigma^2 / 8;
* on real integrals the oracle's residual, amplitudes and energy have exactly
  zero imaginary parts (every operation of the complex code keeps real data
  real), the first Jacobi iterate gives the closed-form MP2 energy, and the
  two-electron CCSD energy equals brute-force FCI.
"""
import numpy as np

import fsgen
from oracle import ccsd, fock, solver


def test_real_generator_symmetries_and_variance():
    s = fsgen.make_system(4, 8, 2, 0.2, 5, real=True)
    V = fsgen.full_tensor(s)
    assert np.all(V.imag == 0.0)
    assert np.array_equal(V, -V.transpose(1, 0, 2, 3))
    assert np.array_equal(V, -V.transpose(0, 1, 3, 2))
    assert np.array_equal(V, V.transpose(2, 3, 0, 1))
    g = s.irrep
    bad = (g[:, None, None, None] + g[None, :, None, None] - g[None, None, :, None] - g[None, None, None, :]) % 2 != 0
    assert np.all(V[bad] == 0.0)
    big = fsgen.make_system(6, 30, 1, 0.2, 9, real=True)
    W = fsgen.block(big, np.arange(6), np.arange(6, 36), np.arange(6, 36), np.arange(6, 36)).real
    p, q, r, t = np.indices(W.shape)
    q, r, t = q + 6, r + 6, t + 6
    generic = (q != r) & (q != t) & (r != t)     # no index coincidences
    var = np.mean(W[generic] ** 2)
    assert abs(var / (0.2 ** 2 / 8) - 1.0) < 0.05


def test_oracle_stays_real_and_matches_closed_forms():
    s = fsgen.make_system(6, 18, 3, 0.08, 14, real=True)
    be = ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-11)
    assert r["converged"]
    assert r["E"].imag == 0.0 and np.all(r["t1"].imag == 0.0) and np.all(r["t2"].imag == 0.0)
    R1, R2 = ccsd.residual(be, r["t1"] * 0.5, r["t2"] * 0.5)
    assert np.all(R1.imag == 0.0) and np.all(R2.imag == 0.0)
    t2 = be.V("oovv").conj() / be.D2
    E1 = ccsd.energy(be, 0 * r["t1"], t2)
    E2 = ccsd.mp2_energy_closed_form(be)
    assert abs(E1 - E2) <= 1e-14 * abs(E2)


def test_two_electron_real_ccsd_is_fci():
    s = fsgen.make_system(2, 6, 2, 0.2, 23, real=True)
    fs = fock.FockSpace(s.eps, fsgen.full_tensor(s), 2)
    r = solver.solve_ccsd(ccsd.Blocked(s), tol=1e-12)
    assert r["converged"] and r["E"].imag == 0.0
    w, U = fock.fci_energies(fs, 2)
    k = int(np.argmax(np.abs(U.conj().T @ fs.reference(2))))
    assert abs(r["E"] - (w[k] - fs.E_ref)) < 1e-10

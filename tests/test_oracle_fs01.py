"""Pins of the (0h,1p) oracle against brute-force Fock-space matrices (no GPU).

* sigma = Hbar_N r equals <mu| exp(-T) H exp(T) - E |nu> r on the
  {1p, 2p1h} space, separately for the 1p and 2p1h parts of r (every term,
  sign and conjugate of the sigma equations and Hbar elements);
* the Bloch residual at random S equals Q M (P + X) - X (P M (P + X));
* converged H_eff eigenvalues are eigenvalues of the full EA matrix M, and for
  one occupied spinor equal FCI(N+1) - FCI(N).
"""
import numpy as np
import pytest

import fsgen
from oracle import ccsd, fock, fs01, solver


def _setup(no, nv, ni, seed, nact, sigma=0.2):
    s = fsgen.make_system(no, nv, ni, sigma, seed, nact=nact)
    fs = fock.FockSpace(s.eps, fsgen.full_tensor(s), no)
    be = ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-13)
    M, labels = fock.ea_matrix(fs, r["t1"], r["t2"], fs.E_ref + r["E"])
    return s, fs, be, r, M, labels


def _flatten(labels, a1, a2):
    return np.array([a1[l[1]] if l[0] == "p" else a2[l[1], l[2], l[3]] for l in labels])


@pytest.mark.parametrize("no,nv,ni,seed", [(2, 4, 1, 3), (3, 4, 1, 5), (2, 5, 2, 9), (3, 5, 2, 2)])
def test_sigma_matches_bruteforce(no, nv, ni, seed):
    s, fs, be, r, M, labels = _setup(no, nv, ni, seed, 2)
    hb = fs01.hbar(be, r["t1"], r["t2"])
    rng = np.random.default_rng(seed)
    r1 = rng.normal(size=(2, nv)) + 1j * rng.normal(size=(2, nv))
    r2 = rng.normal(size=(2, no, nv, nv)) + 1j * rng.normal(size=(2, no, nv, nv))
    r2 = r2 - r2.transpose(0, 1, 3, 2)
    for part in ("1p", "2p1h"):
        a1 = r1 if part == "1p" else 0 * r1
        a2 = r2 if part == "2p1h" else 0 * r2
        s1, s2 = fs01.sigma(be, hb, a1, a2)
        for x in range(2):
            ref = M @ _flatten(labels, a1[x], a2[x])
            got = _flatten(labels, s1[x], s2[x])
            assert np.abs(ref - got).max() < 1e-11 * max(1.0, np.abs(ref).max()), part


@pytest.mark.parametrize("no,nv,ni,seed,nact", [(2, 5, 1, 3, 2), (3, 5, 2, 4, 3)])
def test_bloch_residual_matches_bruteforce(no, nv, ni, seed, nact):
    s, fs, be, r, M, labels = _setup(no, nv, ni, seed, nact)
    F = fs01.FS01(be, r["t1"], r["t2"], s.active)
    rng = np.random.default_rng(1)
    s1, s2 = F.zeros()
    s1 = np.where(F.mask1, 0.05 * (rng.normal(size=s1.shape) + 1j * rng.normal(size=s1.shape)), 0)
    x2 = 0.05 * (rng.normal(size=s2.shape) + 1j * rng.normal(size=s2.shape))
    s2 = np.where(F.mask2, x2 - x2.transpose(0, 1, 3, 2), 0)
    R1, R2, heff = F.residual(s1, s2)
    # brute force: columns of (P + X) are the vectors r(x); model-space rows are the 1p labels of A
    r1 = F.rvec(s1, s2)[0]
    R = np.array([_flatten(labels, r1[x], s2[x]) for x in range(F.nact)]).T
    MR = M @ R
    pidx = [k for k, l in enumerate(labels) if l[0] == "p" and l[1] in set(F.act.tolist())]
    order = [pidx[[labels[k][1] for k in pidx].index(a)] for a in F.act]
    Heff_bf = MR[order, :]
    assert np.abs(Heff_bf - heff).max() < 1e-11
    Rbf = MR - R @ Heff_bf
    got = np.array([_flatten(labels, R1[x], R2[x]) for x in range(F.nact)]).T
    q = [k for k in range(len(labels)) if k not in set(order)]
    assert np.abs(Rbf[q, :] - got[q, :]).max() < 1e-11


@pytest.mark.parametrize("no,nv,ni,seed,nact", [(1, 5, 1, 4, 2), (1, 6, 2, 7, 3), (2, 5, 1, 3, 2),
                                               (3, 5, 1, 5, 2), (2, 6, 2, 11, 3)])
def test_heff_eigenvalues_are_ea_eigenvalues(no, nv, ni, seed, nact):
    s, fs, be, r, M, labels = _setup(no, nv, ni, seed, nact, sigma=0.1)
    F = fs01.FS01(be, r["t1"], r["t2"], s.active)
    o = fs01.solve_fs01(F, tol=1e-12)
    assert o["converged"]
    wM = np.linalg.eigvals(M)
    for e in o["eig"]:
        assert np.min(np.abs(wM - e)) < 1e-10
    if no == 1:
        w1, _ = fock.fci_energies(fs, 1)
        w2, _ = fock.fci_energies(fs, 2)
        for e in o["eig"]:
            assert np.min(np.abs(w2 - w1[0] - e)) < 1e-10

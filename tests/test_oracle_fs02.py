"""Pins of the (0h,2p) oracle against brute-force Fock-space vectors (no GPU).

* sigma2(xy) = [exp(-T) H exp(T) - E] Omega|xy> projected on the 2p space, with
  Omega|xy> built as R_x R_y |Phi> + S_xy |Phi> from Jordan-Wigner matrices,
  separately for the 1p and 2p1h parts of the attachments and for S_xy alone
  (every term, sign and conjugate of the two-line and one-line pieces);
* H_eff and the Bloch residual at random amplitudes equal the brute-force
  P and Q projections;
* a converged solution satisfies the brute-force Bloch equation, and the
  dynamically shifted equations extrapolate back to it.
"""
import numpy as np
import pytest

import fsgen
from oracle import ccsd, fock, fs01, fs02, shift, solver


def _setup(no, nv, ni, seed, nact, sigma=0.2):
    s = fsgen.make_system(no, nv, ni, sigma, seed, nact=nact)
    fs = fock.FockSpace(s.eps, fsgen.full_tensor(s), no)
    be = ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-13)
    return s, fs, be, r


def _rand(rng, shape, scale=0.05):
    return scale * (rng.normal(size=shape) + 1j * rng.normal(size=shape))


def _amplitudes(F1, rng, scale=0.05):
    s1, s2 = F1.zeros()
    s1 = np.where(F1.mask1, _rand(rng, s1.shape, scale), 0)
    x2 = _rand(rng, s2.shape, scale)
    s2 = np.where(F1.mask2, x2 - x2.transpose(0, 1, 3, 2), 0)
    return s1, s2


def _bruteforce(fs, r, F1, F2, s1, s2, s):
    """sigma2 and omega of every model pair from the Fock-space construction."""
    r1, r2 = F1.rvec(s1, s2)
    E = fs.E_ref + r["E"]
    sig, om = [], []
    for p, (x, y) in enumerate(F2.pairs):
        v = fock.dea_state(fs, r1[x], r2[x], r1[y], r2[y], s[p])
        u = fock.hbar_apply(fs, fs.nocc + 2, r["t1"], r["t2"], E, v)
        sig.append(fock.pp_projection(fs, u))
        om.append(fock.pp_projection(fs, v))
    return np.array(sig), np.array(om)


@pytest.mark.parametrize("no,nv,ni,seed,nact", [(2, 5, 1, 3, 3), (3, 5, 2, 4, 3), (2, 6, 2, 8, 4)])
def test_sigma2_parts_match_bruteforce(no, nv, ni, seed, nact):
    s, fs, be, r = _setup(no, nv, ni, seed, nact)
    F1 = fs01.FS01(be, r["t1"], r["t2"], s.active)
    rng = np.random.default_rng(seed)
    a1, a2 = _amplitudes(F1, rng, 0.3)
    x = _rand(rng, (len(fs02.FS02(F1, a1, a2).pairs), nv, nv), 0.3)
    s_pp = x - x.transpose(0, 2, 1)
    z1, z2 = 0 * a1, 0 * a2
    # 1p parts only, 2p1h parts only (with the model e_x kept), the new amplitude only, all together
    for b1, b2, bs in ((a1, z2, 0 * s_pp), (z1, a2, 0 * s_pp), (z1, z2, s_pp), (a1, a2, s_pp)):
        F2 = fs02.FS02(F1, b1, b2)
        got = F2.sigma2(bs)
        ref, om = _bruteforce(fs, r, F1, F2, b1, b2, bs)
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() < 1e-11 * scale
        assert np.abs(om - (F2.wpp + bs)).max() < 1e-13


@pytest.mark.parametrize("no,nv,ni,seed,nact", [(2, 5, 1, 5, 3), (3, 6, 2, 2, 3)])
def test_bloch_residual_matches_bruteforce(no, nv, ni, seed, nact):
    s, fs, be, r = _setup(no, nv, ni, seed, nact)
    F1 = fs01.FS01(be, r["t1"], r["t2"], s.active)
    rng = np.random.default_rng(11)
    s1, s2 = _amplitudes(F1, rng)
    F2 = fs02.FS02(F1, s1, s2)
    x = _rand(rng, (F2.npair, nv, nv))
    s_pp = np.where(F2.mask, x - x.transpose(0, 2, 1), 0)
    R, heff = F2.residual(s_pp)
    sig, om = _bruteforce(fs, r, F1, F2, s1, s2, s_pp)
    heff_bf = sig[:, F2.ma, F2.mb].T
    assert np.abs(heff_bf - heff).max() < 1e-11
    Rbf = sig - np.einsum("qab,qp->pab", om, heff_bf)
    assert np.abs(np.where(F2.mask, Rbf, 0) - R).max() < 1e-11
    # model-pair rows of the brute-force residual vanish identically
    assert np.abs(Rbf[:, F2.ma, F2.mb]).max() < 1e-11


@pytest.mark.parametrize("no,nv,ni,seed,nact", [(2, 6, 1, 4, 2), (2, 6, 2, 11, 3), (3, 6, 2, 5, 3)])
def test_converged_solution_solves_bruteforce_bloch(no, nv, ni, seed, nact):
    s, fs, be, r = _setup(no, nv, ni, seed, nact, sigma=0.1)
    F1 = fs01.FS01(be, r["t1"], r["t2"], s.active)
    o1 = fs01.solve_fs01(F1, tol=1e-12)
    assert o1["converged"]
    F2 = fs02.FS02(F1, o1["s1"], o1["s2"])
    o2 = fs02.solve_fs02(F2, tol=1e-12)
    assert o2["converged"]
    sig, om = _bruteforce(fs, r, F1, F2, o1["s1"], o1["s2"], o2["s"])
    heff_bf = sig[:, F2.ma, F2.mb].T
    Rbf = sig - np.einsum("qab,qp->pab", om, heff_bf)
    assert np.abs(np.where(F2.mask, Rbf, 0)).max() < 1e-10
    assert np.abs(heff_bf - o2["heff"]).max() < 1e-10
    # one model pair: its energy (relative to the correlated N-electron ground state) stays
    # close to the bare pair energy e_x + e_y at this interaction strength
    if F2.npair == 1:
        ev = s.eps[s.nocc:]
        assert abs(o2["eig"][0].real - ev[F2.ma[0]] - ev[F2.mb[0]]) < 0.5


def test_shifted_solves_extrapolate_to_plain_solution():
    """Shifted solves converge, and the [3/0] Pade value at zero shift recovers the plain
    solution at least ten times better than the largest-shift solve itself."""
    s, fs, be, r = _setup(3, 6, 2, 5, 3, sigma=0.1)
    F1 = fs01.FS01(be, r["t1"], r["t2"], s.active)
    o1 = fs01.solve_fs01(F1, tol=1e-12)
    plain = fs02.solve_fs02(fs02.FS02(F1, o1["s1"], o1["s2"]), tol=1e-12)
    lam = np.array([1.0, 0.8, 0.6, 0.4])
    ys = []
    for l in lam:
        o = fs02.solve_fs02(fs02.FS02(F1, o1["s1"], o1["s2"], shift=(-0.1 * l, 2)), tol=1e-12)
        assert o["converged"]
        ys.append(o["eig"])
    ys = np.array(ys)
    for k in range(ys.shape[1]):
        e0 = shift.pade(lam, ys[:, k], 3, 0, 0.0)
        assert abs(e0 - plain["eig"][k]) < 0.1 * abs(ys[0, k] - plain["eig"][k])


def test_s02_layout_round_trip():
    """The packed (0h,2p) layout of the tests' layout helper: every active pair once per pair
    irrep, antisymmetric amplitudes survive pack/unpack, forbidden elements are dropped."""
    import layout_ref as LR
    s = fsgen.make_system(3, 9, 3, 0.1, 4, nact=4)
    n = len(s.active)
    pairs = sum(len(LR.xy_pair_list(s, G)[0]) for G in range(s.nirrep))
    assert pairs == n * (n - 1) // 2
    rng = np.random.default_rng(0)
    g = s.irrep[s.nocc:]
    ga = s.irrep[np.sort(s.active)]
    x = _rand(rng, (pairs, s.nvirt, s.nvirt))
    x = x - x.transpose(0, 2, 1)
    allowed = np.zeros_like(x, dtype=bool)
    for i in range(n):
        for j in range(i + 1, n):
            p = LR.pair_index(n, i, j)
            allowed[p] = ((ga[i] + ga[j] - g[:, None] - g[None, :]) % s.nirrep == 0)
    y = LR.unpack_s02(s, LR.pack_s02(s, x))
    assert np.array_equal(y, np.where(allowed, x, 0))

"""Block-list (0h,1p) and (0h,2p) oracles against the dense ones (no GPU).

The dense sector oracles are pinned to brute-force Fock-space constructions
(tests/test_oracle_fs01.py, tests/test_oracle_fs02.py); the block-list forms
run the same equations with the Fig. 3 partition and Fig. 4 block-pair
contractions, and must give the same residuals, H_eff and converged
eigenvalues (dense = blocked, the sector counterpart of the (0h,0p) pin P5).
Systems with empty irreps and with active spinors in several irreps exercise
the bookkeeping: a key or member list wrong anywhere changes an element.
"""
import numpy as np
import pytest

import fsgen
from oracle import ccsd, fs01, fs02, solver
from oracle.blocks import BlockTensor

SYSTEMS = [
    # nocc, nvirt, nirrep, sigma, seed, nact
    (4, 10, 1, 0.1, 2, 3),
    (6, 14, 4, 0.1, 21, 5),
    (5, 12, 6, 0.1, 4, 4),
    (7, 19, 3, 0.05, 8, 6),
]


def _rand(rng, shape, scale=0.05):
    return scale * (rng.normal(size=shape) + 1j * rng.normal(size=shape))


def _pair(spec):
    no, nv, ni, sg, seed, nact = spec
    s = fsgen.make_system(no, nv, ni, sg, seed, nact=nact)
    dn, bl = ccsd.Dense(s), ccsd.Blocked(s)
    rng = np.random.default_rng(seed)
    # arbitrary allowed T (the sector equations hold for any T, not only the converged one)
    r = solver.solve_ccsd(dn, tol=1e-8, maxit=6)
    allowed = (s.irrep[:no, None] - s.irrep[None, no:]) % ni == 0
    t1 = r["t1"] + np.where(allowed, _rand(rng, dn.D1.shape, 0.01), 0)
    t2 = r["t2"]
    bt1 = BlockTensor.from_dense(t1, [bl.mem["O"], bl.mem["V"]], list(bl.D1.blocks.keys()))
    bt2 = BlockTensor.from_dense(t2, [bl.mem[X] for X in "OOVV"], list(bl.D2.blocks.keys()))
    return s, dn, bl, (t1, t2), (bt1, bt2), rng


def _amplitudes(F1, rng):
    s1, s2 = F1.zeros()
    s1 = np.where(F1.mask1, _rand(rng, s1.shape), 0)
    x2 = _rand(rng, s2.shape)
    s2 = np.where(F1.mask2, x2 - x2.transpose(0, 1, 3, 2), 0)
    return s1, s2


@pytest.mark.parametrize("spec", SYSTEMS)
def test_fs01_blocked_residual_equals_dense(spec):
    s, dn, bl, (t1, t2), (bt1, bt2), rng = _pair(spec)
    Fd = fs01.FS01(dn, t1, t2, s.active)
    Fb = fs01.FS01Blocked(bl, bt1, bt2, s.active)
    s1, s2 = _amplitudes(Fd, rng)
    R1, R2, h = Fd.residual(s1, s2)
    b1, b2 = Fb.from_dense(s1, s2)
    Q1, Q2, g = Fb.residual(b1, b2)
    scale = max(np.abs(R1).max(), np.abs(R2).max())
    assert np.abs(Fb.to_dense(Q1) - R1).max() <= 1e-13 * scale
    assert np.abs(Fb.to_dense(Q2) - R2).max() <= 1e-13 * scale
    assert np.abs(g - h).max() <= 1e-13 * np.abs(h).max()
    # the round trip dense -> blocks -> dense is the identity on allowed amplitudes
    assert np.array_equal(Fb.to_dense(b1), s1) and np.array_equal(Fb.to_dense(b2), s2)
    # dressed denominators, shifts and the model-space mask, block by block
    Dd = fs01.FS01(dn, t1, t2, s.active, precond="dressed", shift=(-2.0, 3))
    Db = fs01.FS01Blocked(bl, bt1, bt2, s.active, precond="dressed", shift=(-2.0, 3))
    mA, mO, mV = Db.memA, bl.mem["O"], bl.mem["V"]
    for (g, _), v in Db.D1.blocks.items():
        ix = np.ix_(mA[g], mV[g])
        assert np.abs(v - Dd.D1[ix]).max() <= 1e-14
        assert np.abs(Db.Delta1.blocks[(g, g)] - Dd.Delta1[ix]).max() <= 1e-14
        assert np.array_equal(Db.mask1.blocks[(g, g)] != 0, Dd.mask1[ix])
    for k, v in Db.D2.blocks.items():
        ix = np.ix_(mA[k[0]], mO[k[1]], mV[k[2]], mV[k[3]])
        assert np.abs(v - Dd.D2[ix]).max() <= 1e-14
        assert np.abs(Db.Delta2.blocks[k] - Dd.Delta2[ix]).max() <= 1e-14


@pytest.mark.parametrize("spec", SYSTEMS[1:3])
def test_fs01_blocked_solve_equals_dense(spec):
    s, dn, bl, _, _, _ = _pair(spec)
    rd = solver.solve_ccsd(dn, tol=1e-12)
    rb = solver.solve_ccsd(bl, tol=1e-12)
    od = fs01.solve_fs01(fs01.FS01(dn, rd["t1"], rd["t2"], s.active), tol=1e-11)
    ob = fs01.solve_fs01_blocked(fs01.FS01Blocked(bl, rb["t1"], rb["t2"], s.active), tol=1e-11)
    assert od["converged"] and ob["converged"]
    assert abs(od["iters"] - ob["iters"]) <= 1
    assert np.abs(od["eig"] - ob["eig"]).max() <= 1e-10


@pytest.mark.parametrize("spec", SYSTEMS)
def test_fs02_blocked_residual_equals_dense(spec):
    s, dn, bl, (t1, t2), (bt1, bt2), rng = _pair(spec)
    F1d = fs01.FS01(dn, t1, t2, s.active)
    F1b = fs01.FS01Blocked(bl, bt1, bt2, s.active)
    s1, s2 = _amplitudes(F1d, rng)
    F2d = fs02.FS02(F1d, s1, s2, shift=(-1.5, 2))
    F2b = fs02.FS02Blocked(F1b, *F1b.from_dense(s1, s2), shift=(-1.5, 2))
    assert F2d.pairs == F2b.pairs
    scale = np.abs(F2d.K).max()
    assert np.abs(F2b.K - F2d.K).max() <= 1e-13 * scale
    x = np.where(F2d.mask, _rand(rng, F2d.zeros().shape), 0)
    x = x - np.swapaxes(x, 1, 2)
    R, h = F2d.residual(x)
    Q, g = F2b.residual(x)
    assert np.abs(Q - R).max() <= 1e-13 * np.abs(R).max()
    assert np.abs(g - h).max() <= 1e-13 * np.abs(h).max()
    assert np.array_equal(F2b.mask, F2d.mask) and np.array_equal(F2b.Delta, F2d.Delta)

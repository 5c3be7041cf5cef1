"""GPU parity of the real-arithmetic path (real double groups; through the C
ABI) against the CPU oracle run on the same real integrals, and against the
complex path on the same system.

Kernel level: fscc_dgemm for every real kernel form (MFMA tiles, tall,
reduction), transposes, split-K, ragged sizes, K = 0, beta = 1, within 1e-13
relative of numpy.  Residual per call within 1e-12 * max|R| of the oracle
(whose imaginary parts are exactly zero on real inputs); converged energy
within 1e-10 Eh of the oracle and of the complex context; first update =
closed-form MP2; the ladder alone = the MP3 ladder closed form.  The
(0h,1p) and (0h,2p) sectors in real arithmetic: residuals and H_eff within
1e-12 of the oracle, converged sector energies within 1e-10 Eh of the oracle
and of the complex context.
"""
import itertools

import numpy as np
import pytest

import fsgen
import layout_ref as LR
from oracle import ccsd, fs01, fs02, solver

pytestmark = pytest.mark.gpu

MFMA = (0, 1, 2, 3, 4, 5, 9, 10, 12, 13)
TALL, RED, SKINNY = 7, 8, 6


def _dg(M, N, K, tA, tB, cfg, bk, split, beta, seed=0, alpha=0.7):
    import torch
    import paper_2004_03682_amd as F
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(K, M) if tA else (M, K))
    B = rng.normal(size=(N, K) if tB else (K, N))
    C0 = rng.normal(size=(M, N))
    ref = alpha * ((A.T if tA else A) @ (B.T if tB else B)) + (C0 if beta else 0)
    dA, dB, dC = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (A, B, C0))
    F.dgemm(dA, dB, dC, M, N, K, max(A.shape[1], 1), max(B.shape[1], 1), max(N, 1), tA, tB, alpha, beta, cfg, bk,
            split)
    return np.abs(dC.cpu().numpy() - ref).max() / max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("cfg,bk", list(itertools.product(MFMA, (16, 32))))
def test_dgemm_mfma_tiles(cfg, bk):
    for tA, tB in itertools.product((0, 1), (0, 1)):
        # (3, 48, 3000): 12 K chunks when split; (130, 70, 1200) and (300, 200, 1800): 5 and 8 chunks
        for (M, N, K) in [(1, 1, 1), (17, 33, 15), (70, 23, 129), (130, 131, 40), (3, 48, 3000), (130, 70, 1200),
                          (300, 200, 1800), (9, 11, 0)]:
            for split in (False, True):
                err = _dg(M, N, K, tA, tB, cfg, bk, split, beta=M % 2, seed=M + N + K)
                assert err < 1e-13, (cfg, bk, tA, tB, M, N, K, split, err)


def test_dgemm_vector_forms():
    for tB in (0, 1):
        for (M, N, K) in [(1, 1, 1), (257, 3, 48), (1000, 48, 7), (300, 16, 64), (77, 1024, 1), (513, 9, 0)]:
            for beta in (0, 1):
                err = _dg(M, N, K, 0, tB, TALL, 16, False, beta, seed=M * N + K)
                assert err < 1e-13, ("tall", tB, M, N, K, beta, err)
    for tA in (0, 1):
        for (M, N, K) in [(1, 1, 1), (2, 21, 5000), (4, 7, 12345), (7, 48, 3001), (8, 256, 700), (6, 13, 0)]:
            for beta in (0, 1):
                err = _dg(M, N, K, tA, 0, RED, 16, True, beta, seed=M * N + K)
                assert err < 1e-13, ("reduction", tA, M, N, K, beta, err)
    with pytest.raises(Exception):
        _dg(10, 10, 10, 0, 0, SKINNY, 16, True, 0)


@pytest.mark.parametrize("cfg", (0, 3, 4, 5, 9, 10, 12, 13))
def test_dgemm_direct_to_lds_tiles(cfg):
    """The real direct-to-LDS form (each double moved as two 4-byte
    direct-to-LDS loads): every transpose, ragged M, N and K (below, at and
    past one 16-deep slice, several ring turns), split-K, K = 0, beta = 1,
    odd leading dimensions (8-byte aligned operands)."""
    DL = 1024
    for tA, tB in itertools.product((0, 1), (0, 1)):
        for (M, N, K) in [(1, 1, 1), (17, 33, 15), (70, 23, 16), (33, 65, 17), (130, 131, 40), (31, 129, 64),
                          (3, 48, 3000), (300, 200, 1800), (9, 11, 0)]:
            for split in (False, True):
                err = _dg(M, N, K, tA, tB, cfg | DL, 16, split, M % 2, seed=M + N + K)
                assert err < 1e-13, ("direct-to-LDS", cfg, tA, tB, M, N, K, split, err)
    with pytest.raises(Exception):
        _dg(10, 10, 10, 0, 0, cfg | DL, 32, False, 0)


def _real_ctx(s):
    import torch
    import paper_2004_03682_amd as F
    ctx = F.Context.from_system(s, precision="real_fp64")
    for C in fsgen.CLASSES:
        buf, _ = fsgen.class_buffer(s, C)
        ctx.set_integrals(C, torch.from_numpy(fsgen.real_buffer(buf)).cuda())
    return ctx


def _random_real_t(s, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    no, nv, ni = s.nocc, s.nvirt, s.nirrep
    t1 = scale * rng.normal(size=(no, nv)) + 0j
    t2 = scale * rng.normal(size=(no, no, nv, nv)) + 0j
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    g = s.irrep
    go, gv = g[:no], g[no:]
    t1[(go[:, None] - gv[None, :]) % ni != 0] = 0
    t2[(go[:, None, None, None] + go[None, :, None, None] - gv[None, None, :, None] - gv[None, None, None, :]) % ni != 0] = 0
    return t1, t2


REAL_SYSTEMS = [(8, 24, 1, 0.05, 1000), (6, 14, 4, 0.1, 21), (5, 12, 6, 0.1, 4), (9, 37, 5, 0.05, 17),
                (1, 5, 1, 0.1, 3)]


@pytest.mark.parametrize("spec", REAL_SYSTEMS)
def test_real_residual_matches_oracle(spec):
    import torch
    print("case real", spec, flush=True)
    s = fsgen.make_system(*spec, real=True)
    ctx = _real_ctx(s)
    t1, t2 = _random_real_t(s, 7)
    d1 = torch.from_numpy(np.ascontiguousarray(LR.pack_t1(s, t1).real)).cuda()
    d2 = torch.from_numpy(np.ascontiguousarray(LR.pack_t2(s, t2).real)).cuda()
    r1, r2 = torch.empty_like(d1), torch.empty_like(d2)
    ctx.build_residual(d1, d2, r1, r2)
    R1, R2 = ccsd.residual(ccsd.Dense(s), t1, t2)
    assert np.abs(R1.imag).max() == 0.0 and (R2.size == 0 or np.abs(R2.imag).max() == 0.0)
    scale = max(np.abs(R2).max() if R2.size else 0.0, np.abs(R1).max(), 1e-300)
    assert np.abs(LR.unpack_t1(s, r1.cpu().numpy() + 0j) - R1).max() <= 1e-12 * scale
    if R2.size:
        assert np.abs(LR.unpack_t2(s, r2.cpu().numpy() + 0j) - R2).max() <= 1e-12 * scale
    ctx.destroy()


def test_real_first_update_mp2_and_ladder_mp3():
    import torch
    s = fsgen.make_system(7, 30, 4, 0.05, 8, real=True)
    be = ccsd.Dense(s)
    ctx = _real_ctx(s)
    t1 = torch.zeros(ctx.n1, dtype=torch.float64, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.float64, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    ctx.diis_reset(6)
    ctx.build_residual(t1, t2, r1, r2)
    ctx.update_amplitudes(t1, t2, r1, r2)
    E = ctx.energy(t1, t2)
    E2 = ccsd.mp2_energy_closed_form(be)
    assert E.imag == 0.0 and abs(E - E2) <= 1e-13 * abs(E2)
    y = (be.V("oovv").conj() / be.D2).real
    tau = torch.from_numpy(np.ascontiguousarray(LR.pack_t2(s, y + 0j).real)).cuda()
    out = torch.empty_like(tau)
    ctx.ladder(tau, out)
    L = LR.unpack_t2(s, out.cpu().numpy() + 0j)
    e = 0.25 * np.sum(be.V("oovv") * L / be.D2)
    ref = ccsd.mp3_ladder_closed_form(be)
    assert abs(e - ref) <= 1e-12 * abs(ref)
    ctx.destroy()


def test_real_converged_energy_matches_oracle_and_complex_path():
    import torch
    import paper_2004_03682_amd as F
    s = fsgen.make_system(10, 40, 4, 0.05, 31, real=True)
    ctx = _real_ctx(s)
    t1 = torch.zeros(ctx.n1, dtype=torch.float64, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.float64, device="cuda")
    ctx.autotune(1)
    g = F.solve(ctx, t1, t2, tol=1e-10)
    o = solver.solve_ccsd(ccsd.Dense(s), tol=1e-10)
    assert g["converged"] and o["converged"] and o["E"].imag == 0.0
    assert abs(g["E"] - o["E"]) <= 1e-10
    assert np.abs(LR.unpack_t2(s, t2.cpu().numpy() + 0j) - o["t2"]).max() <= 1e-9
    # the complex context on the same (real) integrals
    cz = F.Context.from_system(s)
    for C in fsgen.CLASSES:
        buf, _ = fsgen.class_buffer(s, C)
        cz.set_integrals(C, torch.from_numpy(buf).cuda())
    z1 = torch.zeros(cz.n1, dtype=torch.complex128, device="cuda")
    z2 = torch.zeros(cz.n2, dtype=torch.complex128, device="cuda")
    gz = F.solve(cz, z1, z2, tol=1e-10)
    assert gz["converged"] and abs(gz["E"] - g["E"]) <= 1e-10 and g["iters"] == gz["iters"]
    cz.destroy()
    ctx.destroy()


def _rdev(x):
    import torch
    assert not np.any(np.imag(x)), "real system amplitudes"
    return torch.from_numpy(np.ascontiguousarray(np.real(x))).cuda()


@pytest.mark.parametrize("spec", [(6, 14, 4, 0.1, 21, 4), (7, 19, 3, 0.05, 8, 5)])
def test_real_sectors_residuals_match_oracle(spec):
    import torch
    import paper_2004_03682_amd as F
    no, nv, ni, sg, seed, nact = spec
    print("case real sectors", spec, flush=True)
    s = fsgen.make_system(no, nv, ni, sg, seed, nact=nact, real=True)
    be = ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-12)
    ctx = _real_ctx(s)
    ctx.prepare_sector(_rdev(LR.pack_t1(s, r["t1"])), _rdev(LR.pack_t2(s, r["t2"])))
    F1 = fs01.FS01(be, r["t1"], r["t2"], s.active)
    rng = np.random.default_rng(seed)
    s1, s2 = F1.zeros()
    s1 = np.where(F1.mask1, 0.05 * rng.normal(size=s1.shape), 0) + 0j
    x2 = 0.05 * rng.normal(size=s2.shape)
    s2 = np.where(F1.mask2, x2 - x2.transpose(0, 1, 3, 2), 0) + 0j
    R1, R2, heff = F1.residual(s1, s2)
    assert np.abs(R2.imag).max() == 0.0 and np.abs(heff.imag).max() == 0.0
    d1, d2 = _rdev(LR.pack_s1(s, s1)), _rdev(LR.pack_s2(s, s2))
    o1, o2 = torch.empty_like(d1), torch.empty_like(d2)
    ctx.build_residual(d1, d2, o1, o2, sector=F.FSCC_S01)
    scale = max(np.abs(R2).max(), np.abs(R1).max())
    assert np.abs(LR.unpack_s1(s, o1.cpu().numpy() + 0j) - R1).max() <= 1e-12 * scale
    assert np.abs(LR.unpack_s2(s, o2.cpu().numpy() + 0j) - R2).max() <= 1e-12 * scale
    assert np.abs(ctx.heff(d1, d2) - heff).max() <= 1e-12 * max(1.0, np.abs(heff).max())
    # (0h,2p) on top of these (0h,1p) amplitudes
    ctx.prepare_sector(d1, d2, sector=F.FSCC_S02)
    F2 = fs02.FS02(F1, s1, s2)
    x = 0.05 * rng.normal(size=(F2.npair, nv, nv))
    sp = np.where(F2.mask, x - x.transpose(0, 2, 1), 0) + 0j
    R, h2 = F2.residual(sp)
    d = _rdev(LR.pack_s02(s, sp))
    o = torch.empty_like(d)
    ctx.build_residual(None, d, None, o, sector=F.FSCC_S02)
    scale = max(1.0, np.abs(R).max())
    assert np.abs(LR.unpack_s02(s, o.cpu().numpy() + 0j) - R).max() <= 1e-12 * scale
    assert np.abs(ctx.heff2(d) - h2).max() <= 1e-12 * max(1.0, np.abs(h2).max())
    ctx.destroy()


def test_real_sectors_converged_match_complex_context():
    """(0h,0p) -> (0h,1p) -> (0h,2p) solved in a real context and in a complex context
    on the same real integrals: the same sector energies (1e-10 Eh), and the oracle's."""
    import torch
    import paper_2004_03682_amd as F
    s = fsgen.make_system(3, 6, 2, 0.1, 5, nact=3, real=True)
    out = {}
    for prec in ("real_fp64", "fp64"):
        ctx = _real_ctx(s) if prec == "real_fp64" else F.Context.from_system(s)
        if prec == "fp64":
            for C in fsgen.CLASSES:
                ctx.set_integrals(C, torch.from_numpy(fsgen.class_buffer(s, C)[0]).cuda())
        dt = torch.float64 if prec == "real_fp64" else torch.complex128
        t1 = torch.zeros(ctx.n1, dtype=dt, device="cuda")
        t2 = torch.zeros(ctx.n2, dtype=dt, device="cuda")
        assert F.solve(ctx, t1, t2, tol=1e-11)["converged"]
        ctx.prepare_sector(t1, t2)
        s1 = torch.zeros(ctx.m1, dtype=dt, device="cuda")
        s2 = torch.zeros(ctx.m2, dtype=dt, device="cuda")
        g1 = F.solve01(ctx, s1, s2, tol=1e-11)
        ctx.prepare_sector(s1, s2, sector=F.FSCC_S02)
        sp = torch.zeros(ctx.p2, dtype=dt, device="cuda")
        g2 = F.solve02(ctx, sp, tol=1e-11)
        assert g1["converged"] and g2["converged"]
        out[prec] = (g1["eig"], g2["eig"])
        ctx.destroy()
    for k in range(2):
        assert np.abs(out["real_fp64"][k] - out["fp64"][k]).max() <= 1e-10
    be = ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-11)
    F1 = fs01.FS01(be, r["t1"], r["t2"], s.active)
    o1 = fs01.solve_fs01(F1, tol=1e-11)
    o2 = fs02.solve_fs02(fs02.FS02(F1, o1["s1"], o1["s2"]), tol=1e-11)
    assert np.abs(out["real_fp64"][0] - o1["eig"]).max() <= 1e-10
    assert np.abs(out["real_fp64"][1] - o2["eig"]).max() <= 1e-10


def test_real_context_rejects_what_it_does_not_do():
    import torch
    import paper_2004_03682_amd as F
    s = fsgen.make_system(3, 8, 2, 0.05, 2, real=True)
    ctx = _real_ctx(s)
    assert ctx.precision() == "real_fp64"
    with pytest.raises(F.FsccError):
        ctx.set_precision("split_bf16")
    with pytest.raises(TypeError):
        ctx.build_residual(*(torch.zeros(n, dtype=torch.complex128, device="cuda")
                             for n in (ctx.n1, ctx.n2, ctx.n1, ctx.n2)))
    ctx.destroy()

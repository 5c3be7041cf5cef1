"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: per call max|R_gpu - R_oracle| <= 1e-12 * max|R| (FP64 with a
different summation order); converged correlation energy within 1e-10 Eh
(real and imaginary parts) and amplitudes within 1e-9 max-abs.
"""
import json
import os

import numpy as np
import pytest

import fsgen
import layout_ref as LR
from oracle import ccsd, solver

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def gpu_ctx(s):
    torch = _torch()
    import paper_2004_03682_amd as F
    ctx = F.Context.from_system(s)
    for C in fsgen.CLASSES:
        buf, _ = fsgen.class_buffer(s, C)
        d = torch.from_numpy(buf).to("cuda")
        ctx.set_integrals(C, d)
        del d
    return ctx


def dev(x):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    return t.cpu().numpy()


def allowed_random_t(s, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    no, nv, ni = s.nocc, s.nvirt, s.nirrep
    t1 = scale * (rng.normal(size=(no, nv)) + 1j * rng.normal(size=(no, nv)))
    t2 = scale * (rng.normal(size=(no, no, nv, nv)) + 1j * rng.normal(size=(no, no, nv, nv)))
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    g = s.irrep
    go, gv = g[:no], g[no:]
    t1[(go[:, None] - gv[None, :]) % ni != 0] = 0
    t2[(go[:, None, None, None] + go[None, :, None, None] - gv[None, None, :, None] - gv[None, None, None, :]) % ni != 0] = 0
    return t1, t2


SYSTEMS = [
    ("o8v24", None),
    ("z4-empty-irreps", (6, 14, 4, 0.1, 21)),
    ("z6-empty-irreps", (5, 12, 6, 0.1, 4)),
    ("one-occupied", (1, 5, 1, 0.1, 3)),
    ("two-occupied-z3", (2, 7, 3, 0.1, 5)),
    ("ragged-z5", (9, 37, 5, 0.05, 17)),
]


def _system(spec):
    name, p = spec
    if name == "o8v24":
        return fsgen.workload_system("o8v24")
    return fsgen.make_system(p[0], p[1], p[2], p[3], p[4])


@pytest.mark.parametrize("tiled", [0, 1, 2], ids=["storage-order", "tiled-gathers", "affine-tiles"])
@pytest.mark.parametrize("spec", SYSTEMS, ids=[s[0] for s in SYSTEMS])
def test_residual_matches_oracle(spec, tiled):
    torch = _torch()
    s = _system(spec)
    print("case", spec, tiled, flush=True)
    ctx = gpu_ctx(s)
    ctx.gather_order(tiled)
    t1, t2 = allowed_random_t(s, 7)
    p1, p2 = LR.pack_t1(s, t1), LR.pack_t2(s, t2)
    assert (ctx.n1, ctx.n2) == (p1.size, p2.size)
    d1, d2 = dev(p1), dev(p2)
    r1, r2 = torch.empty_like(d1), torch.empty_like(d2)
    ctx.build_residual(d1, d2, r1, r2)
    torch.cuda.synchronize()
    R1, R2 = ccsd.residual(ccsd.Dense(s), t1, t2)
    scale = max(np.abs(R2).max() if R2.size else 0.0, np.abs(R1).max(), 1e-300)
    assert np.abs(LR.unpack_t1(s, host(r1)) - R1).max() <= 1e-12 * scale
    if p2.size:
        assert np.abs(LR.unpack_t2(s, host(r2)) - R2).max() <= 1e-12 * scale
    ctx.destroy()


def test_residual_matches_blocked_oracle_o20v120z8():
    torch = _torch()
    s = fsgen.workload_system("o20v120z8")
    ctx = gpu_ctx(s)
    t1, t2 = allowed_random_t(s, 11, 0.02)
    d1, d2 = dev(LR.pack_t1(s, t1)), dev(LR.pack_t2(s, t2))
    r1, r2 = torch.empty_like(d1), torch.empty_like(d2)
    ctx.build_residual(d1, d2, r1, r2)
    # the reorders by destination tiles and by affine tiles give bitwise the same residual
    for order in (0, 1, 2):
        ctx.gather_order(order)
        q1, q2 = torch.empty_like(d1), torch.empty_like(d2)
        ctx.build_residual(d1, d2, q1, q2)
        assert torch.equal(q1, r1) and torch.equal(q2, r2), order
    be = ccsd.Blocked(s)
    from oracle.blocks import BlockTensor
    bt1 = BlockTensor.from_dense(t1, [be.mem["O"], be.mem["V"]], list(be.D1.blocks.keys()))
    bt2 = BlockTensor.from_dense(t2, [be.mem[X] for X in "OOVV"], list(be.D2.blocks.keys()))
    R1, R2 = ccsd.residual(be, bt1, bt2)
    R1, R2 = be.dense(R1), be.dense(R2)
    scale = np.abs(R2).max()
    assert np.abs(LR.unpack_t1(s, host(r1)) - R1).max() <= 1e-12 * scale
    assert np.abs(LR.unpack_t2(s, host(r2)) - R2).max() <= 1e-12 * scale
    ctx.destroy()


def test_first_update_gives_mp2_energy():
    torch = _torch()
    s = fsgen.make_system(7, 30, 4, 0.05, 8)
    ctx = gpu_ctx(s)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    ctx.diis_reset(6)
    ctx.build_residual(t1, t2, r1, r2)
    ctx.update_amplitudes(t1, t2, r1, r2)
    E = ctx.energy(t1, t2)
    E2 = ccsd.mp2_energy_closed_form(ccsd.Dense(s))
    assert abs(E - E2) <= 1e-13 * abs(E2)
    assert float(torch.abs(t1).max()) == 0.0
    ctx.destroy()


def test_ladder_mp3_closed_form():
    torch = _torch()
    s = fsgen.make_system(6, 22, 3, 0.05, 12)
    be = ccsd.Dense(s)
    ctx = gpu_ctx(s)
    y = be.V("oovv").conj() / be.D2
    tau = dev(LR.pack_t2(s, y))
    out = torch.empty_like(tau)
    ctx.ladder(tau, out)
    L = LR.unpack_t2(s, host(out))
    e = 0.25 * np.sum(be.V("oovv") * L / be.D2)
    ref = ccsd.mp3_ladder_closed_form(be)
    assert abs(e - ref) <= 1e-12 * abs(ref)
    Lo = ccsd.pp_ladder(be, y)
    assert np.abs(L - Lo).max() <= 1e-12 * np.abs(Lo).max()
    ctx.destroy()


@pytest.mark.parametrize("dressed", [0, 1, 10])
def test_converged_o8v24_matches_oracle(dressed):
    """Bare and dressed Jacobi denominators (fscc_precondition, (0h,0p)) reach
    the oracle's fixed point."""
    torch = _torch()
    import paper_2004_03682_amd as F
    s = fsgen.workload_system("o8v24")
    ctx = gpu_ctx(s)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    g = F.solve(ctx, t1, t2, tol=1e-10, dressed=dressed)
    print("o8v24 dressed", dressed, "iterations", g["iters"], flush=True)
    o = solver.solve_ccsd(ccsd.Dense(s), tol=1e-10)
    assert g["converged"] and o["converged"]
    assert abs(g["E"].real - o["E"].real) <= 1e-10 and abs(g["E"].imag - o["E"].imag) <= 1e-10
    assert np.abs(LR.unpack_t2(s, host(t2)) - o["t2"]).max() <= 1e-9
    assert np.abs(LR.unpack_t1(s, host(t1)) - o["t1"]).max() <= 1e-9
    ctx.destroy()


@pytest.mark.parametrize("dressed", [0, 10])
def test_converged_o20v120z8_matches_golden(dressed):
    torch = _torch()
    import paper_2004_03682_amd as F
    gold = json.load(open(os.path.join(HERE, "golden", "o20v120z8_ccsd.json")))
    s = fsgen.workload_system("o20v120z8")
    ctx = gpu_ctx(s)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    g = F.solve(ctx, t1, t2, tol=1e-10, dressed=dressed)
    print("o20v120z8 gpu", g["E"], g["iters"], "oracle", gold["E_re"], gold["E_im"], gold["iters"], flush=True)
    assert g["converged"]
    assert abs(g["E"].real - gold["E_re"]) <= 1e-10
    assert abs(g["E"].imag - gold["E_im"]) <= 1e-10
    ctx.destroy()


def test_errors_are_reported():
    torch = _torch()
    import paper_2004_03682_amd as F
    s = fsgen.make_system(3, 6, 2, 0.05, 1)
    ctx = F.Context.from_system(s)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    with pytest.raises(F.FsccError) as e:
        ctx.build_residual(t1, t2, torch.empty_like(t1), torch.empty_like(t2))
    assert e.value.status == -5
    with pytest.raises(F.FsccError) as e:
        ctx.set_integrals("OOVV", torch.zeros(3, dtype=torch.complex128, device="cuda"))
    assert e.value.status == -1
    # dressed (0h,0p) denominators need a residual first; bad mode / floor
    with pytest.raises(F.FsccError) as e:
        ctx.precondition(1, 0.1, F.FSCC_S00)
    assert e.value.status == -5
    for mode, floor in ((2, 0.1), (1, 0.0), (0, -1.0)):
        with pytest.raises(F.FsccError) as e:
            ctx.precondition(mode, floor, F.FSCC_S00)
        assert e.value.status == -1
    ctx.destroy()


def test_tiled_gathers_bitwise_equal_in_every_sector():
    """(0h,0p), (0h,1p) and (0h,2p) residuals with every reorder walked by
    destination tiles equal the storage-order ones bit for bit."""
    torch = _torch()
    import paper_2004_03682_amd as F
    s = fsgen.make_system(8, 40, 4, 0.05, 9, nact=6)
    ctx = gpu_ctx(s)
    rng = np.random.default_rng(3)
    def rnd(n):
        return torch.from_numpy(0.05 * (rng.normal(size=n) + 1j * rng.normal(size=n))).cuda()
    t1, t2 = allowed_random_t(s, 5, 0.02)
    d1, d2 = dev(LR.pack_t1(s, t1)), dev(LR.pack_t2(s, t2))
    ctx.prepare_sector(d1, d2)
    s1, s2 = rnd(ctx.m1), rnd(ctx.m2)
    ctx.prepare_sector(s1, s2, sector=F.FSCC_S02)
    p2 = rnd(ctx.p2)
    out = {}
    for tiled in (0, 1, 2):
        ctx.gather_order(tiled)
        r = [torch.empty_like(x) for x in (d1, d2, s1, s2, p2)]
        ctx.build_residual(d1, d2, r[0], r[1])
        ctx.build_residual(s1, s2, r[2], r[3], sector=F.FSCC_S01)
        ctx.build_residual(None, p2, None, r[4], sector=F.FSCC_S02)
        torch.cuda.synchronize()
        out[tiled] = r
    for tiled in (1, 2):
        for a, b in zip(out[0], out[tiled]):
            assert torch.equal(a, b), tiled
    ctx.destroy()


@pytest.mark.parametrize("spec", [(6, 14, 4, 0.1, 21), (9, 37, 5, 0.05, 17), (8, 24, 1, 0.05, 1000)],
                         ids=["z4", "ragged-z5", "o8v24"])
def test_dressed_denominators_match_oracle_intermediates(spec):
    """fscc_precondition (0h,0p) mode 1: D_i^a = f_i - f_a and D_ij^ab = f_i + f_j
    - f_a - f_b with f_p = e_p + Re F'_pp, F'_be = F_be - 1/2 sum_m t_m^b F_me and
    F'_mj = F_mj + 1/2 sum_e t_j^e F_me from the oracle's one-body intermediates
    at the amplitudes of the last residual, capped at -floor; mode 0 restores
    the bare e_i - e_a, e_i + e_j - e_a - e_b."""
    torch = _torch()
    import paper_2004_03682_amd as F
    s = fsgen.make_system(*spec)
    ctx = gpu_ctx(s)
    t1, t2 = allowed_random_t(s, 5, scale=0.1)
    a1, a2 = dev(LR.pack_t1(s, t1)), dev(LR.pack_t2(s, t2))
    r1, r2 = torch.empty_like(a1), torch.empty_like(a2)
    ctx.build_residual(a1, a2, r1, r2)
    floor = 0.3
    ctx.precondition(1, floor, F.FSCC_S00)
    G1, G2 = (host(x) for x in ctx.denominators())
    be = ccsd.Dense(s)
    I = ccsd.intermediates(be, t1, t2, one_body_only=True)
    Fbe = I["Fae"] - 0.5 * np.einsum("mb,me->be", t1, I["Fme"])
    Fmj = I["Fmi"] + 0.5 * np.einsum("je,me->mj", t1, I["Fme"])
    no = s.nocc
    fo = s.eps[:no] + np.real(np.diag(Fmj))
    fv = s.eps[no:] + np.real(np.diag(Fbe))
    D1 = np.minimum(fo[:, None] - fv[None, :], -floor)
    D2 = np.minimum(fo[:, None, None, None] + fo[None, :, None, None] - fv[None, None, :, None]
                    - fv[None, None, None, :], -floor)
    W1 = LR.pack_t1(s, D1.astype(np.complex128)).real
    W2 = LR.pack_t2(s, D2.astype(np.complex128)).real
    print("max |D'| diff", np.abs(G1 - W1).max(initial=0.0), np.abs(G2 - W2).max(initial=0.0), flush=True)
    assert np.abs(G1 - W1).max(initial=0.0) <= 1e-12 * max(1.0, np.abs(W1).max(initial=0.0))
    assert np.abs(G2 - W2).max(initial=0.0) <= 1e-12 * max(1.0, np.abs(W2).max(initial=0.0))
    assert (W2 != LR.pack_t2(s, (s.eps[:no, None, None, None] + s.eps[None, :no, None, None]
                                 - s.eps[None, None, no:, None] - s.eps[None, None, None, no:]).astype(complex)).real).any()
    ctx.precondition(0, floor, F.FSCC_S00)
    B1, B2 = (host(x) for x in ctx.denominators())
    e = s.eps
    assert np.array_equal(B1, LR.pack_t1(s, (e[:no, None] - e[None, no:]).astype(complex)).real)
    d2 = e[:no, None, None, None] + e[None, :no, None, None] - e[None, None, no:, None] - e[None, None, None, no:]
    assert np.abs(B2 - LR.pack_t2(s, d2.astype(complex)).real).max(initial=0.0) <= 1e-14
    ctx.destroy()


def test_iterate_equals_residual_update_energy():
    """fscc_iterate (one synchronisation per iteration) gives bit for bit the
    amplitudes, steps and energies of fscc_build_residual + fscc_update_amplitudes
    + fscc_energy, over several DIIS iterations."""
    torch = _torch()
    s = fsgen.make_system(9, 37, 5, 0.05, 17)
    ctx = gpu_ctx(s)
    runs = []
    for fused in (False, True):
        t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
        t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
        r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
        ctx.diis_reset(6)
        hist = []
        for _ in range(8):
            if fused:
                d, E = ctx.iterate(t1, t2, r1, r2)
            else:
                ctx.build_residual(t1, t2, r1, r2)
                d = ctx.update_amplitudes(t1, t2, r1, r2)
                E = ctx.energy(t1, t2)
            hist.append((d, E))
        runs.append((hist, host(t1), host(t2)))
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])
    ctx.destroy()


@pytest.mark.parametrize("ndiis", [12, 16])
def test_deep_diis_trajectory_matches_oracle(ndiis):
    """DIIS subspaces deeper than the batch's 8 (single-system contexts keep
    up to 16 vector pairs): the energy of every iteration follows the
    oracle's Jacobi + DIIS(ndiis) iteration, and the fixed point is the
    oracle's (energy 1e-10 Eh, amplitudes 1e-9)."""
    torch = _torch()
    import paper_2004_03682_amd as F
    s = fsgen.workload_system("o8v24")
    ctx = gpu_ctx(s)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    g = F.solve(ctx, t1, t2, tol=1e-11, maxit=60, ndiis=ndiis)
    o = solver.solve_ccsd(ccsd.Dense(s), tol=1e-11, maxit=60, ndiis=ndiis)
    print("ndiis", ndiis, "gpu iterations", g["iters"], "oracle", o["iters"], flush=True)
    assert g["converged"] and o["converged"]
    n = min(len(g["history"]), len(o["history"]))
    d = [abs(g["history"][k]["E"] - o["history"][k]["E"]) for k in range(n)]
    print("per-iteration |dE|:", " ".join(f"{x:.1e}" for x in d), flush=True)
    # the trajectory within 1e-8 Eh, as for the production-size DIIS trajectory
    # (the two bordered solves round differently where B is ill-conditioned)
    assert max(d) <= 1e-8, max(d)
    assert abs(g["E"] - o["E"]) <= 1e-10
    assert np.abs(LR.unpack_t2(s, host(t2)) - o["t2"]).max() <= 1e-9
    with pytest.raises(F.FsccError):
        ctx.diis_reset(17)
    ctx.destroy()

"""GPU parity of the (0h,1p) and (0h,2p) sectors at the production size
(nocc = 40, nvirt = 300, 16 irreps, 6 active virtual spinors, 15 active
pairs), in the launch configuration the benchmark times (autotuned GEMM
forms of every sector operation), against the block-list sector oracles:
the Bloch residual of each sector and its H_eff, every element within 1e-12
of max|R| (of max|H_eff| for H_eff).

Inputs: T = the MP2 amplitudes (the first Jacobi step from zero) plus a small
allowed T1, then seeded random (0h,1p) amplitudes s1, s2 and (0h,2p)
amplitudes s; the sector equations are defined for any T and any S, so
per-call parity does not need converged amplitudes.

The oracle half of this test takes one to two minutes of host time."""
import sys
import time

import numpy as np
import pytest

import fsgen
import layout_ref as LR
from oracle import ccsd, fs01, fs02
from oracle.blocks import BlockTensor

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.mark.timeout(900)
def test_production_size_sectors_match_blocked_oracle():
    import torch
    import paper_2004_03682_amd as F
    t0 = time.perf_counter()
    s = fsgen.workload_system("o40v300z16")
    assert s.nact == 6
    buffers = {C: fsgen.class_buffer(s, C)[0] for C in fsgen.CLASSES}
    ctx = F.Context.from_system(s)
    for C in fsgen.CLASSES:
        d = torch.from_numpy(buffers[C]).cuda()
        ctx.set_integrals(C, d)
        del d
    ctx.autotune(1)
    _log(f"production-size context ready at {time.perf_counter() - t0:.1f}s")
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    ctx.diis_reset(1)
    ctx.build_residual(t1, t2, r1, r2)
    ctx.update_amplitudes(t1, t2, r1, r2)            # t2 = MP2 amplitudes, t1 = 0
    rng = np.random.default_rng(11)
    t1.copy_(torch.from_numpy(0.01 * (rng.normal(size=ctx.n1) + 1j * rng.normal(size=ctx.n1))))
    ctx.prepare_sector(t1, t2)
    # (0h,1p): random S1 (model-space components zero) and S2 (antisymmetric in ab)
    s1 = LR.unpack_s1(s, 0.05 * (rng.normal(size=ctx.m1) + 1j * rng.normal(size=ctx.m1)))
    s1[:, s.active - s.nocc] = 0.0
    s2 = LR.unpack_s2(s, 0.05 * (rng.normal(size=ctx.m2) + 1j * rng.normal(size=ctx.m2)))
    d1, d2 = torch.from_numpy(LR.pack_s1(s, s1)).cuda(), torch.from_numpy(LR.pack_s2(s, s2)).cuda()
    o1, o2 = torch.empty_like(d1), torch.empty_like(d2)
    ctx.build_residual(d1, d2, o1, o2, sector=F.FSCC_S01)
    heff1 = ctx.heff(d1, d2)
    g1, g2 = LR.unpack_s1(s, o1.cpu().numpy()), LR.unpack_s2(s, o2.cpu().numpy())
    # (0h,2p), prepared from the same (0h,1p) amplitudes
    ctx.prepare_sector(d1, d2, sector=F.FSCC_S02)
    h1, h2 = LR.unpack_t1(s, t1.cpu().numpy()), LR.unpack_t2(s, t2.cpu().numpy())
    be = ccsd.Blocked(s, buffers)
    bt1 = BlockTensor.from_dense(h1, [be.mem["O"], be.mem["V"]], list(be.D1.blocks.keys()))
    bt2 = BlockTensor.from_dense(h2, [be.mem[X] for X in "OOVV"], list(be.D2.blocks.keys()))
    del h2
    F1 = fs01.FS01Blocked(be, bt1, bt2, s.active)
    _log(f"oracle Hbar ready at {time.perf_counter() - t0:.1f}s")
    b1, b2 = F1.from_dense(s1, s2)
    R1, R2, heff_o = F1.residual(b1, b2)
    R1, R2 = F1.to_dense(R1), F1.to_dense(R2)
    scale = max(np.abs(R1).max(), np.abs(R2).max())
    e1, e2 = float(np.abs(g1 - R1).max()), float(np.abs(g2 - R2).max())
    eh = float(np.abs(heff1 - heff_o).max())
    _log(f"(0h,1p) production size: max|dR1| = {e1:.2e}, max|dR2| = {e2:.2e} (max|R| = {scale:.2e}), "
         f"max|dHeff| = {eh:.2e} (max|Heff| = {np.abs(heff_o).max():.2e})")
    assert e1 <= 1e-12 * scale and e2 <= 1e-12 * scale
    assert eh <= 1e-12 * np.abs(heff_o).max()
    del g2, R2
    F2 = fs02.FS02Blocked(F1, b1, b2)
    assert F2.npair == 15
    x = 0.05 * (rng.normal(size=(F2.npair, s.nvirt, s.nvirt)) + 1j * rng.normal(size=(F2.npair, s.nvirt, s.nvirt)))
    sp = np.where(F2.mask, x - x.transpose(0, 2, 1), 0)
    R, heff2_o = F2.residual(sp)
    _log(f"oracle (0h,2p) residual at {time.perf_counter() - t0:.1f}s")
    d = torch.from_numpy(LR.pack_s02(s, sp)).cuda()
    assert d.numel() == ctx.p2
    o = torch.empty_like(d)
    ctx.build_residual(None, d, None, o, sector=F.FSCC_S02)
    heff2 = ctx.heff2(d)
    got = LR.unpack_s02(s, o.cpu().numpy())
    ctx.destroy()
    e = float(np.abs(got - R).max())
    eh2 = float(np.abs(heff2 - heff2_o).max())
    _log(f"(0h,2p) production size: max|dR| = {e:.2e} (max|R| = {np.abs(R).max():.2e}), "
         f"max|dHeff| = {eh2:.2e} (max|Heff| = {np.abs(heff2_o).max():.2e})")
    assert e <= 1e-12 * np.abs(R).max()
    assert eh2 <= 1e-12 * np.abs(heff2_o).max()

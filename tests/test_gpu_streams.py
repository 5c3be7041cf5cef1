"""Residual operation lists on two streams (fscc_set_streams): the GEMMs bound
by the matrix cores on the context's stream, the other operations on a
second stream, with an event wait for every buffer dependency between them.
Every result must be bit for bit that of the one-stream order: the (0h,0p)
iteration (residual, Jacobi/DIIS update, energy) over several iterations in
complex and real arithmetic, and the (0h,1p) and (0h,2p) sector residuals
(their preparations run on two streams as well); a (0h,0p) residual on two
streams is also checked against the oracle."""
import numpy as np
import pytest

import fsgen
import layout_ref as LR
from oracle import ccsd

pytestmark = pytest.mark.gpu


def _ctx(s, real=False):
    import torch
    import paper_2004_03682_amd as F
    ctx = F.Context.from_system(s, precision="real_fp64" if real else "fp64")
    for C in fsgen.CLASSES:
        buf, _ = fsgen.class_buffer(s, C)
        ctx.set_integrals(C, torch.from_numpy(fsgen.real_buffer(buf) if real else buf).cuda())
    return ctx


def _iterations(ctx, n, real=False):
    import torch
    dt = torch.float64 if real else torch.complex128
    t1 = torch.zeros(ctx.n1, dtype=dt, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=dt, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    ctx.diis_reset(6)
    hist = [ctx.iterate(t1, t2, r1, r2) for _ in range(n)]
    return hist, t1.cpu().numpy(), t2.cpu().numpy(), t1, t2


@pytest.mark.parametrize("real", [False, True])
def test_two_streams_iteration_is_bitwise_the_one_stream_iteration(real):
    s = fsgen.make_system(9, 37, 5, 0.05, 17, real=real)
    print("case real" if real else "case complex", flush=True)
    ctx = _ctx(s, real)
    runs = []
    for n in (1, 2, 1):
        ctx.set_streams(n)
        runs.append(_iterations(ctx, 8, real)[:3])
    for r in runs[1:]:
        assert r[0] == runs[0][0]
        assert np.array_equal(r[1], runs[0][1]) and np.array_equal(r[2], runs[0][2])
    ctx.destroy()


def test_two_streams_residual_matches_oracle():
    import torch
    s = fsgen.make_system(8, 30, 4, 0.05, 3)
    rng = np.random.default_rng(3)
    no, nv, ni = s.nocc, s.nvirt, s.nirrep
    t1 = 0.05 * (rng.normal(size=(no, nv)) + 1j * rng.normal(size=(no, nv)))
    t2 = 0.05 * (rng.normal(size=(no, no, nv, nv)) + 1j * rng.normal(size=(no, no, nv, nv)))
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    g = s.irrep
    go, gv = g[:no], g[no:]
    t1[(go[:, None] - gv[None, :]) % ni != 0] = 0
    t2[(go[:, None, None, None] + go[None, :, None, None] - gv[None, None, :, None] - gv[None, None, None, :])
       % ni != 0] = 0
    R1, R2 = ccsd.residual(ccsd.Dense(s), t1, t2)
    ctx = _ctx(s)
    ctx.set_streams(2)
    d1 = torch.from_numpy(LR.pack_t1(s, t1)).cuda()
    d2 = torch.from_numpy(LR.pack_t2(s, t2)).cuda()
    o1, o2 = torch.empty_like(d1), torch.empty_like(d2)
    ctx.build_residual(d1, d2, o1, o2)
    scale = max(np.abs(R1).max(), np.abs(R2).max())
    assert np.abs(LR.unpack_t1(s, o1.cpu().numpy()) - R1).max() <= 1e-12 * scale
    assert np.abs(LR.unpack_t2(s, o2.cpu().numpy()) - R2).max() <= 1e-12 * scale
    ctx.destroy()


def test_two_streams_sector_residuals_are_bitwise_the_one_stream_residuals():
    import torch
    import paper_2004_03682_amd as F
    s = fsgen.make_system(7, 26, 4, 0.05, 9, nact=5)
    ctx = _ctx(s)
    _, _, _, t1, t2 = _iterations(ctx, 6)
    rng = np.random.default_rng(9)
    s1 = torch.from_numpy(0.05 * (rng.normal(size=ctx.m1) + 1j * rng.normal(size=ctx.m1))).cuda()
    s2 = torch.from_numpy(0.05 * (rng.normal(size=ctx.m2) + 1j * rng.normal(size=ctx.m2))).cuda()
    p2 = torch.from_numpy(0.05 * (rng.normal(size=ctx.p2) + 1j * rng.normal(size=ctx.p2))).cuda()
    out = []
    for n in (1, 2):
        ctx.set_streams(n)
        ctx.prepare_sector(t1, t2)
        o1, o2 = torch.empty_like(s1), torch.empty_like(s2)
        ctx.build_residual(s1, s2, o1, o2, sector=F.FSCC_S01)
        ctx.prepare_sector(s1, s2, sector=F.FSCC_S02)
        o3 = torch.empty_like(p2)
        ctx.build_residual(None, p2, None, o3, sector=F.FSCC_S02)
        out.append([x.cpu().numpy() for x in (o1, o2, o3)])
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    ctx.destroy()


def test_set_streams_takes_one_or_two():
    import paper_2004_03682_amd as F
    s = fsgen.make_system(4, 10, 2, 0.05, 1)
    ctx = _ctx(s)
    for n in (0, 3, -1):
        with pytest.raises(F.FsccError):
            ctx.set_streams(n)
    ctx.destroy()

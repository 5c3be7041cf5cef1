"""GPU parity of the (0h,2p) sector (through the C ABI) against the CPU oracle.

Per call: Bloch residual and H_eff at random (0h,1p) and (0h,2p) amplitudes
within 1e-12 of max|R| (systems from one pair to 15 pairs, several GEMM tiles
and ragged tails); converged: H_eff eigenvalues within 1e-10 Eh of the
oracle's, plain and with dynamic shifts; state errors on misuse."""
import numpy as np
import pytest

import fsgen
import layout_ref as LR
from oracle import ccsd, fs01, fs02, solver

pytestmark = pytest.mark.gpu


def _ctx(s):
    import torch
    import paper_2004_03682_amd as F
    ctx = F.Context.from_system(s)
    for C in fsgen.CLASSES:
        buf, _ = fsgen.class_buffer(s, C)
        ctx.set_integrals(C, torch.from_numpy(buf).to("cuda"))
    return ctx


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _rand(rng, shape, scale=0.05):
    return scale * (rng.normal(size=shape) + 1j * rng.normal(size=shape))


SYSTEMS = [(4, 10, 1, 0.1, 2, 2), (6, 14, 4, 0.1, 21, 5), (5, 12, 6, 0.1, 4, 4), (7, 19, 3, 0.05, 8, 6),
           (8, 40, 4, 0.05, 9, 6)]


@pytest.mark.parametrize("spec", SYSTEMS)
def test_fs02_residual_matches_oracle(spec):
    import torch
    import paper_2004_03682_amd as F
    no, nv, ni, sg, seed, nact = spec
    print("case", spec, flush=True)
    s = fsgen.make_system(no, nv, ni, sg, seed, nact=nact)
    be = ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-12)
    ctx = _ctx(s)
    ctx.prepare_sector(_dev(LR.pack_t1(s, r["t1"])), _dev(LR.pack_t2(s, r["t2"])))
    F1 = fs01.FS01(be, r["t1"], r["t2"], s.active)
    rng = np.random.default_rng(seed)
    s1, s2 = F1.zeros()
    s1 = np.where(F1.mask1, _rand(rng, s1.shape), 0)
    x2 = _rand(rng, s2.shape)
    s2 = np.where(F1.mask2, x2 - x2.transpose(0, 1, 3, 2), 0)
    ctx.prepare_sector(_dev(LR.pack_s1(s, s1)), _dev(LR.pack_s2(s, s2)), sector=F.FSCC_S02)
    F2 = fs02.FS02(F1, s1, s2)
    x = _rand(rng, (F2.npair, nv, nv))
    sp = np.where(F2.mask, x - x.transpose(0, 2, 1), 0)
    R, heff = F2.residual(sp)
    d = _dev(LR.pack_s02(s, sp))
    assert d.numel() == ctx.p2
    o = torch.empty_like(d)
    ctx.build_residual(None, d, None, o, sector=F.FSCC_S02)
    scale = max(1.0, np.abs(R).max())
    assert np.abs(LR.unpack_s02(s, o.cpu().numpy()) - R).max() <= 1e-12 * scale
    assert np.abs(ctx.heff2(d) - heff).max() <= 1e-12 * max(1.0, np.abs(heff).max())
    ctx.destroy()


def _chain(s, shift=None):
    """GPU: (0h,0p) -> (0h,1p) -> (0h,2p) from zero amplitudes; returns the (0h,2p) result."""
    import torch
    import paper_2004_03682_amd as F
    ctx = _ctx(s)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    assert F.solve(ctx, t1, t2, tol=1e-11)["converged"]
    ctx.prepare_sector(t1, t2)
    s1 = torch.zeros(ctx.m1, dtype=torch.complex128, device="cuda")
    s2 = torch.zeros(ctx.m2, dtype=torch.complex128, device="cuda")
    assert F.solve01(ctx, s1, s2, tol=1e-11)["converged"]
    ctx.prepare_sector(s1, s2, sector=F.FSCC_S02)
    if shift is not None:
        ctx.dynamic_shift(shift[0], shift[1], sector=F.FSCC_S02)
    sp = torch.zeros(ctx.p2, dtype=torch.complex128, device="cuda")
    out = F.solve02(ctx, sp, tol=1e-11)
    ctx.destroy()
    return out


def _oracle_chain(s, shift=None):
    be = ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-11)
    F1 = fs01.FS01(be, r["t1"], r["t2"], s.active)
    o1 = fs01.solve_fs01(F1, tol=1e-11)
    return fs02.solve_fs02(fs02.FS02(F1, o1["s1"], o1["s2"], shift=shift), tol=1e-11)


@pytest.mark.parametrize("spec", [(3, 6, 2, 0.1, 5, 3), (7, 19, 3, 0.05, 8, 2), (6, 14, 4, 0.1, 21, 3)])
def test_fs02_converged_eigenvalues(spec):
    no, nv, ni, sg, seed, nact = spec
    print("case", spec, flush=True)
    s = fsgen.make_system(no, nv, ni, sg, seed, nact=nact)
    g = _chain(s)
    o = _oracle_chain(s)
    print("gpu eig", g["eig"], g["iters"], "oracle eig", o["eig"], o["iters"], flush=True)
    assert g["converged"] and o["converged"]
    assert np.abs(g["eig"] - o["eig"]).max() <= 1e-10


@pytest.mark.parametrize("spec,shift", [((7, 19, 3, 0.05, 8, 3), (-0.3, 2)), ((8, 30, 4, 0.05, 9, 4), (-1.0, 2))])
def test_fs02_dynamic_shift_matches_oracle(spec, shift):
    """Systems whose plain (0h,2p) equations diverge (intruder pairs) converge with the
    shift, to the oracle's shifted solution."""
    no, nv, ni, sg, seed, nact = spec
    print("case", spec, shift, flush=True)
    s = fsgen.make_system(no, nv, ni, sg, seed, nact=nact)
    g = _chain(s, shift)
    o = _oracle_chain(s, shift)
    print("gpu eig", g["eig"], g["iters"], "oracle eig", o["eig"], o["iters"], flush=True)
    assert g["converged"] and o["converged"]
    assert np.abs(g["eig"] - o["eig"]).max() <= 1e-10


def test_fs02_state_errors():
    import torch
    import paper_2004_03682_amd as F
    s = fsgen.make_system(4, 10, 1, 0.1, 2, nact=2)
    ctx = _ctx(s)
    sp = torch.zeros(ctx.p2, dtype=torch.complex128, device="cuda")
    r = torch.empty_like(sp)
    with pytest.raises(F.FsccError):            # (0h,2p) before any preparation
        ctx.build_residual(None, sp, None, r, sector=F.FSCC_S02)
    s1 = torch.zeros(ctx.m1, dtype=torch.complex128, device="cuda")
    s2 = torch.zeros(ctx.m2, dtype=torch.complex128, device="cuda")
    with pytest.raises(F.FsccError):            # (0h,2p) preparation needs the (0h,1p) one
        ctx.prepare_sector(s1, s2, sector=F.FSCC_S02)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    ctx.prepare_sector(t1, t2)
    ctx.prepare_sector(s1, s2, sector=F.FSCC_S02)
    ctx.build_residual(None, sp, None, r, sector=F.FSCC_S02)
    ctx.prepare_sector(t1, t2)                  # a new (0h,1p) preparation invalidates (0h,2p)
    with pytest.raises(F.FsccError):
        ctx.build_residual(None, sp, None, r, sector=F.FSCC_S02)
    ctx.destroy()
    one = _ctx(fsgen.make_system(4, 10, 1, 0.1, 2, nact=1))   # one active spinor: no pairs
    assert one.p2 == 0
    with pytest.raises(F.FsccError):
        one.diis_reset(6, F.FSCC_S02)
    one.destroy()

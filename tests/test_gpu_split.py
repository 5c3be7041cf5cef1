"""Split-precision (compensated bf16 / fp32) contractions against FP64.

Error model of one output element of the split GEMM (include/fscc.h,
fscc_set_precision): the operand pieces represent each value to a relative
2^-24 (bf16: three 8-bit pieces; fp32: hi + lo), the dropped high-order piece
products are below 2^-24 |a||b|, and fp32 accumulation within one 32-deep
k block rounds at 2^-24 of the block sum; the block sums are added in FP64.
The bound used here, 2^-19 * sum_k |a_k||b_k|, allows a 32x margin over that
unit and still fails if a piece is dropped (bf16: h1 -> 2^-9, h2 -> 2^-18).
"""
import itertools
import json
import os

import numpy as np
import pytest

import fsgen
import layout_ref as LR
from oracle import ccsd

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = 2.0 ** -19
PRECS = ("split_bf16", "split_fp32")


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dev(x):
    return _torch().from_numpy(np.ascontiguousarray(x)).to("cuda")


def _rand(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def _run(prec, cfg, M, N, K, tA, tB, cA, cB, beta, seed=0, alpha=0.7 - 0.3j):
    import paper_2004_03682_amd as F
    rng = np.random.default_rng(seed)
    A = _rand(rng, K, M) if tA else _rand(rng, M, K)
    B = _rand(rng, N, K) if tB else _rand(rng, K, N)
    C0 = _rand(rng, M, N)
    opA = A.T if tA else A
    opB = B.T if tB else B
    if cA:
        opA = opA.conj()
    if cB:
        opB = opB.conj()
    ref = alpha * (opA @ opB) + (C0 if beta else 0)
    bound = abs(alpha) * (np.abs(opA) @ np.abs(opB)) * EPS + 1e-15 * (np.abs(C0) if beta else 0)
    dA, dB, dC = dev(A), dev(B), dev(C0)
    lda = max(A.shape[1], 1) if A.size else 1
    ldb = max(B.shape[1], 1) if B.size else 1
    F.zgemm_split(dA, dB, dC, M, N, K, lda, ldb, max(N, 1), prec, cfg, tA, tB, cA, cB, alpha, beta)
    out = dC.cpu().numpy()
    err = np.abs(out - ref)
    return err, bound, ref


@pytest.mark.parametrize("prec,cfg", list(itertools.product(PRECS, range(8))))
def test_split_gemm_every_config(prec, cfg):
    for (tA, tB, cA, cB) in [(0, 0, 0, 0), (0, 1, 1, 0), (1, 0, 0, 1), (1, 1, 1, 1)]:
        for (M, N, K) in [(1, 1, 1), (17, 33, 15), (70, 23, 129), (130, 131, 40), (64, 64, 64)]:
            err, bound, _ = _run(prec, cfg, M, N, K, tA, tB, cA, cB, beta=(M % 2))
            assert np.all(err <= bound), (prec, cfg, tA, tB, cA, cB, M, N, K, float((err / bound).max()))


@pytest.mark.parametrize("prec", PRECS)
def test_split_gemm_long_k_and_edges(prec):
    for (M, N, K, beta) in [(5, 200, 3000, 0), (49, 70, 2811, 1), (9, 11, 0, 0), (9, 11, 0, 1)]:
        err, bound, ref = _run(prec, 0, M, N, K, 0, 1, 0, 0, beta)
        assert np.all(err <= bound + 1e-15 * np.abs(ref)), (prec, M, N, K, beta)


def test_split_bf16_accuracy_statistics():
    # typical element error: far below the worst-case bound (pieces and pair order working)
    err, bound, _ = _run("split_bf16", 0, 96, 96, 1024, 0, 1, 0, 0, 0, seed=3)
    rel = err / (bound / EPS)
    print("split_bf16 relative error: median %.2e max %.2e" % (np.median(rel), rel.max()), flush=True)
    assert np.median(rel) < 2.0 ** -24


def _ctx(s, precision):
    torch = _torch()
    import paper_2004_03682_amd as F
    ctx = F.Context.from_system(s, precision=precision)
    for C in fsgen.CLASSES:
        buf, _ = fsgen.class_buffer(s, C)
        d = torch.from_numpy(buf).to("cuda")
        ctx.set_integrals(C, d)
        del d
    return ctx


@pytest.mark.parametrize("prec", PRECS)
def test_split_ladder_within_bound(prec):
    # L_ij^ab = sum_{c<d} <ab||cd> y_ij^cd against the oracle, elementwise bound
    torch = _torch()
    s = fsgen.make_system(6, 22, 3, 0.05, 12)
    be = ccsd.Dense(s)
    ctx = _ctx(s, prec)
    y = be.V("oovv").conj() / be.D2
    tau = dev(LR.pack_t2(s, y))
    out = torch.empty_like(tau)
    ctx.ladder(tau, out)
    L = LR.unpack_t2(s, out.cpu().numpy())
    Lo = ccsd.pp_ladder(be, y)
    W = np.abs(be.V("vvvv"))
    bound = 0.5 * np.einsum("abcd,ijcd->ijab", W, np.abs(y)) * EPS
    assert np.all(np.abs(L - Lo) <= bound + 1e-300)
    ctx.destroy()


@pytest.mark.parametrize("prec", PRECS)
def test_split_residual_close_to_oracle(prec):
    torch = _torch()
    from test_gpu_parity import allowed_random_t
    for p in [(8, 24, 1, 0.05, 1000), (9, 37, 5, 0.05, 17), (5, 12, 6, 0.1, 4)]:
        s = fsgen.make_system(*p)
        ctx = _ctx(s, prec)
        assert ctx.precision() == prec
        t1, t2 = allowed_random_t(s, 7)
        d1, d2 = dev(LR.pack_t1(s, t1)), dev(LR.pack_t2(s, t2))
        r1, r2 = torch.empty_like(d1), torch.empty_like(d2)
        ctx.build_residual(d1, d2, r1, r2)
        R1, R2 = ccsd.residual(ccsd.Dense(s), t1, t2)
        scale = max(np.abs(R2).max(), np.abs(R1).max())
        e2 = np.abs(LR.unpack_t2(s, r2.cpu().numpy()) - R2).max() / scale
        e1 = np.abs(LR.unpack_t1(s, r1.cpu().numpy()) - R1).max() / scale
        print(prec, p, "relative residual error r1 %.2e r2 %.2e" % (e1, e2), flush=True)
        assert e1 <= 2.0 ** -16 and e2 <= 2.0 ** -16
        # switching back gives the FP64 residual
        ctx.set_precision("fp64")
        ctx.build_residual(d1, d2, r1, r2)
        assert np.abs(LR.unpack_t2(s, r2.cpu().numpy()) - R2).max() <= 1e-12 * scale
        ctx.destroy()


def test_split_converge_then_fp64_polish_o20v120z8():
    torch = _torch()
    import paper_2004_03682_amd as F
    gold = json.load(open(os.path.join(HERE, "golden", "o20v120z8_ccsd.json")))
    s = fsgen.workload_system("o20v120z8")
    ctx = _ctx(s, "split_bf16")
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    g = F.solve(ctx, t1, t2, tol=1e-6, maxit=200)
    dE_mixed = abs(complex(g["E"]) - complex(gold["E_re"], gold["E_im"]))
    print("o20v120z8 split_bf16 to max|step| < 1e-6: E", g["E"], "iters", g["iters"],
          "|dE| vs oracle %.2e" % dE_mixed, flush=True)
    assert g["converged"] and dE_mixed <= 1e-4
    ctx.set_precision("fp64")
    p = F.solve(ctx, t1, t2, tol=1e-10, maxit=100)
    print("fp64 polish iterations", p["iters"], "E", p["E"], flush=True)
    assert p["converged"]
    assert abs(p["E"].real - gold["E_re"]) <= 1e-10 and abs(p["E"].imag - gold["E_im"]) <= 1e-10
    # the two-stage driver gives the same fixed point
    t1.zero_()
    t2.zero_()
    ctx.set_precision("split_bf16")
    q = F.solve_mixed(ctx, t1, t2, switch_tol=1e-6, tol=1e-10)
    print("solve_mixed: split iters", q["split_iters"], "fp64 iters", q["fp64_iters"], flush=True)
    assert q["converged"] and abs(q["E"].real - gold["E_re"]) <= 1e-10 and abs(q["E"].imag - gold["E_im"]) <= 1e-10
    assert ctx.precision() == "split_bf16"
    ctx.destroy()


@pytest.mark.parametrize("spec", [(6, 14, 4, 0.1, 21, 5), (7, 19, 3, 0.05, 8, 6)])
def test_split_bf16_sector01_residual_close_to_oracle(spec):
    """In split-BF16 the (0h,1p) ladder over all virtual pairs runs on the bf16
    matrix cores: the sector's residual stays within 2^-16 of max|R| of the
    oracle's, and FP64 gives it back to 1e-12."""
    torch = _torch()
    from oracle import fs01, solver
    no, nv, ni, sg, seed, nact = spec
    s = fsgen.make_system(no, nv, ni, sg, seed, nact=nact)
    be = ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-12)
    ctx = _ctx(s, "fp64")
    ctx.prepare_sector(dev(LR.pack_t1(s, r["t1"])), dev(LR.pack_t2(s, r["t2"])))
    Fo = fs01.FS01(be, r["t1"], r["t2"], s.active)
    rng = np.random.default_rng(seed)
    s1, s2 = Fo.zeros()
    s1 = np.where(Fo.mask1, 0.05 * (rng.normal(size=s1.shape) + 1j * rng.normal(size=s1.shape)), 0)
    x2 = 0.05 * (rng.normal(size=s2.shape) + 1j * rng.normal(size=s2.shape))
    s2 = np.where(Fo.mask2, x2 - x2.transpose(0, 1, 3, 2), 0)
    R1, R2, heff = Fo.residual(s1, s2)
    d1, d2 = dev(LR.pack_s1(s, s1)), dev(LR.pack_s2(s, s2))
    o1, o2 = torch.empty_like(d1), torch.empty_like(d2)
    scale = max(np.abs(R2).max(), np.abs(R1).max())
    ctx.set_precision("split_bf16")
    ctx.build_residual(d1, d2, o1, o2, sector=1)
    e1 = np.abs(LR.unpack_s1(s, o1.cpu().numpy()) - R1).max() / scale
    e2 = np.abs(LR.unpack_s2(s, o2.cpu().numpy()) - R2).max() / scale
    print(spec, "split_bf16 (0h,1p) relative residual error %.2e %.2e" % (e1, e2), flush=True)
    assert e1 <= 2.0 ** -16 and e2 <= 2.0 ** -16
    assert e2 > 0.0       # the ladder did run in split precision
    ctx.set_precision("fp64")
    ctx.build_residual(d1, d2, o1, o2, sector=1)
    assert np.abs(LR.unpack_s2(s, o2.cpu().numpy()) - R2).max() <= 1e-12 * scale
    ctx.destroy()

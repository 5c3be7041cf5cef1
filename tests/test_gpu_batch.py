"""Batched systems (grouped launches over all systems' symmetry blocks):
every system's residual, iteration history and converged result must equal
the single-system path on the same inputs, and the graph-replayed iteration
must equal the eagerly launched one."""
import numpy as np
import pytest

import fsgen
import layout_ref as LR
from oracle import ccsd, solver

pytestmark = pytest.mark.gpu

SPECS = [(8, 24, 1, 0.05, 1000), (6, 14, 4, 0.1, 21), (1, 5, 1, 0.1, 3), (9, 37, 5, 0.05, 17), (2, 7, 3, 0.1, 5),
         (5, 12, 6, 0.1, 4)]


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dev(x):
    return _torch().from_numpy(np.ascontiguousarray(x)).to("cuda")


def make_batch(systems):
    torch = _torch()
    import paper_2004_03682_amd as F
    b = F.Batch(systems)
    for k, s in enumerate(systems):
        for C in fsgen.CLASSES:
            buf, _ = fsgen.class_buffer(s, C)
            d = torch.from_numpy(buf).to("cuda")
            b.set_integrals(k, C, d)
            del d
    return b


def single_ctx(s):
    torch = _torch()
    import paper_2004_03682_amd as F
    ctx = F.Context.from_system(s)
    for C in fsgen.CLASSES:
        buf, _ = fsgen.class_buffer(s, C)
        ctx.set_integrals(C, torch.from_numpy(buf).to("cuda"))
    return ctx


def test_batch_layout_and_residual_match_single_systems():
    torch = _torch()
    from test_gpu_parity import allowed_random_t
    systems = [fsgen.make_system(*p) for p in SPECS]
    b = make_batch(systems)
    p1, p2 = [], []
    for k, s in enumerate(systems):
        t1, t2 = allowed_random_t(s, 100 + k)
        p1.append(LR.pack_t1(s, t1))
        p2.append(LR.pack_t2(s, t2))
        off1, n1, off2, n2 = b.segments[k]
        assert (n1, n2) == (p1[-1].size, p2[-1].size)
        assert off1 == sum(x.size for x in p1[:-1]) and off2 == sum(x.size for x in p2[:-1])
    t1, t2 = dev(np.concatenate(p1)), dev(np.concatenate(p2))
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    b.build_residual(t1, t2, r1, r2)
    R1, R2 = r1.cpu().numpy(), r2.cpu().numpy()
    for k, s in enumerate(systems):
        print("system", k, SPECS[k], flush=True)
        ctx = single_ctx(s)
        a1, a2 = dev(p1[k]), dev(p2[k])
        q1, q2 = torch.empty_like(a1), torch.empty_like(a2)
        ctx.build_residual(a1, a2, q1, q2)
        off1, n1, off2, n2 = b.segments[k]
        Q1, Q2 = q1.cpu().numpy(), q2.cpu().numpy()
        scale = max(np.abs(Q1).max() if n1 else 0.0, np.abs(Q2).max() if n2 else 0.0, 1e-300)
        assert np.abs(R1[off1:off1 + n1] - Q1).max(initial=0.0) <= 1e-13 * scale
        assert np.abs(R2[off2:off2 + n2] - Q2).max(initial=0.0) <= 1e-13 * scale
        ctx.destroy()
    # and the oracle on the first system
    s = systems[0]
    off1, n1, off2, n2 = b.segments[0]
    O1, O2 = ccsd.residual(ccsd.Dense(s), LR.unpack_t1(s, p1[0]), LR.unpack_t2(s, p2[0]))
    scale = np.abs(O2).max()
    assert np.abs(LR.unpack_t2(s, R2[off2:off2 + n2]) - O2).max() <= 1e-12 * scale
    assert np.abs(LR.unpack_t1(s, R1[off1:off1 + n1]) - O1).max() <= 1e-12 * scale
    b.destroy()


@pytest.mark.parametrize("use_graph,shift,ndiis,dressed", [(False, 0.0, 6, 0), (True, 0.0, 6, 0), (True, 0.7, 8, 0),
                                                           (True, 0.0, 8, 10), (False, 0.0, 6, 4)])
def test_batch_converges_like_single_systems(use_graph, shift, ndiis, dressed):
    """Also with dressed Jacobi denominators (fscc_batch_precondition against
    fscc_precondition per system): the same iterations and fixed point."""
    torch = _torch()
    import paper_2004_03682_amd as F
    systems = [fsgen.make_system(*p) for p in SPECS[:4]] + [fsgen.make_system(7, 30, 4, 0.05, 8)]
    b = make_batch(systems)
    t1 = torch.zeros(b.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(b.n2, dtype=torch.complex128, device="cuda")
    res = F.solve_batch(b, t1, t2, tol=1e-10, maxit=150, use_graph=use_graph, shift=shift, ndiis=ndiis,
                        dressed=dressed)
    assert res["converged"].all(), res["iters"]
    T1, T2 = t1.cpu().numpy(), t2.cpu().numpy()
    for k, s in enumerate(systems):
        ctx = single_ctx(s)
        u1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
        u2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
        ctx.level_shift(shift)
        g = F.solve(ctx, u1, u2, tol=1e-10, maxit=150, ndiis=ndiis, dressed=dressed)
        print("system", k, "batch", res["E"][k], res["iters"][k], "single", g["E"], g["iters"], flush=True)
        assert g["converged"]
        assert abs(res["E"][k] - g["E"]) <= 1e-10
        assert res["iters"][k] == g["iters"]
        off1, n1, off2, n2 = b.segments[k]
        assert np.abs(T2[off2:off2 + n2] - u2.cpu().numpy()).max(initial=0.0) <= 1e-9
        assert np.abs(T1[off1:off1 + n1] - u1.cpu().numpy()).max(initial=0.0) <= 1e-9
        ctx.destroy()
    o = solver.solve_ccsd(ccsd.Dense(systems[0]), tol=1e-10)
    assert abs(res["E"][0] - o["E"]) <= 1e-10
    b.destroy()


def test_batch_graph_replays_equal_eager_iterations():
    torch = _torch()
    systems = [fsgen.make_system(*p) for p in (SPECS[0], SPECS[3], SPECS[5])]
    b = make_batch(systems)
    t1 = torch.zeros(b.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(b.n2, dtype=torch.complex128, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    b.reset(6, 1e-10)
    eager = [b.step(t1, t2, r1, r2, use_graph=False) for _ in range(12)]
    te = t2.clone()
    t1.zero_()
    t2.zero_()
    b.reset(6, 1e-10)
    for k in range(12):
        rep = b.step(t1, t2, r1, r2, use_graph=True)
        # unrelated eager device work and a synchronisation between replays
        x = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert np.array_equal(rep[:, 3:], eager[k][:, 3:]), k
        assert np.abs(rep[:, :3] - eager[k][:, :3]).max() <= 1e-13 * max(1.0, np.abs(eager[k][:, :3]).max()), k
        del x
    assert torch.abs(t2 - te).max().item() <= 1e-12
    b.destroy()


def test_batch_frozen_systems_stay_fixed():
    torch = _torch()
    systems = [fsgen.make_system(3, 8, 2, 0.02, 31), fsgen.make_system(9, 37, 5, 0.05, 17)]
    b = make_batch(systems)
    t1 = torch.zeros(b.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(b.n2, dtype=torch.complex128, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    b.reset(6, 1e-10)
    frozen_at, snap = None, None
    for k in range(1, 120):
        rep = b.step(t1, t2, r1, r2, use_graph=True)
        if frozen_at is None and rep[0, 3] == 0 and rep[1, 3] == 1:
            frozen_at = k
            off1, n1, off2, n2 = b.segments[0]
            snap = t2[off2:off2 + n2].clone(), rep[0].copy()
        elif frozen_at is not None:
            off1, n1, off2, n2 = b.segments[0]
            assert torch.equal(t2[off2:off2 + n2], snap[0])
            assert np.array_equal(rep[0], snap[1])
        if not rep[:, 3].any():
            break
    assert frozen_at is not None, "expected the small system to converge first"
    assert rep[1, 3] == 0 and rep[1, 4] > frozen_at
    b.destroy()


def test_batch_errors_are_reported():
    torch = _torch()
    import paper_2004_03682_amd as F
    s = fsgen.make_system(3, 6, 2, 0.05, 1)
    b = F.Batch([s, s])
    t1 = torch.zeros(b.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(b.n2, dtype=torch.complex128, device="cuda")
    with pytest.raises(F.FsccError) as e:
        b.step(t1, t2, torch.empty_like(t1), torch.empty_like(t2))
    assert e.value.status == -5
    with pytest.raises(F.FsccError) as e:
        b.set_integrals(2, "OOVV", torch.zeros(3, dtype=torch.complex128, device="cuda"))
    assert e.value.status == -1
    with pytest.raises(F.FsccError):
        F.Batch([fsgen.make_system(3, 6, 2, 0.05, 1, nact=2)])
    b.destroy()


def test_device_generator_matches_host_generator():
    torch = _torch()
    for p in [(8, 24, 1, 0.05, 1000), (6, 14, 4, 0.1, 21), (5, 30, 3, 0.03, 9)]:
        s = fsgen.make_system(*p)
        for C in fsgen.CLASSES:
            ref, _ = fsgen.class_buffer(s, C)
            got = fsgen.class_buffer_gpu(s, C).cpu().numpy()
            assert got.shape == ref.shape
            # same counters and definition; device transcendental functions may differ in the last bits
            assert np.abs(got - ref).max(initial=0.0) <= 1e-15 * max(1.0, s.sigma), (p, C)
            assert np.array_equal(got == 0, ref == 0), (p, C)


def test_batched_workload_systems_converge_to_the_oracle():
    """Systems of the 64-system batched workload (nocc 10-30, nvirt 60-200,
    4-8 irreps) solved as a batch with the workload's solver (DIIS(8),
    dressed denominators refreshed every 25 iterations) reach the block-list
    oracle's converged energies (tests/golden/batch40000_ccsd.json)."""
    import json
    import os
    torch = _torch()
    import paper_2004_03682_amd as F
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch40000_ccsd.json")))
    idx = sorted(int(k) for k in gold)
    ss = fsgen.batch_systems(64, 40000)
    systems = [ss[k] for k in idx]
    for k, s in zip(idx, systems):
        assert (s.nocc, s.nvirt, s.nirrep, s.seed) == (gold[str(k)]["nocc"], gold[str(k)]["nvirt"],
                                                       gold[str(k)]["nirrep"], gold[str(k)]["seed"])
        assert gold[str(k)]["converged"]
    b = make_batch(systems)
    t1 = torch.zeros(b.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(b.n2, dtype=torch.complex128, device="cuda")
    res = F.solve_batch(b, t1, t2, tol=1e-11, maxit=600, use_graph=True, ndiis=8, dressed=25)
    for j, k in enumerate(idx):
        g = gold[str(k)]
        print("system", k, "batch", res["E"][j], res["iters"][j], "oracle", g["E_re"], g["E_im"], g["iters"], flush=True)
        assert res["converged"][j]
        assert abs(res["E"][j].real - g["E_re"]) <= 1e-10 and abs(res["E"][j].imag - g["E_im"]) <= 1e-10
    b.destroy()


def test_stragglers_continue_concurrently_with_the_sequential_results():
    """finish_batch_in_contexts: the systems left when the batch stops
    (stop_active) continue in contexts of their own, concurrently (one host
    thread and stream each) or one after another, with the same energies and
    amplitudes, and reach the single-system fixed point."""
    torch = _torch()
    import paper_2004_03682_amd as F
    systems = [fsgen.make_system(*p) for p in SPECS[:4]] + [fsgen.make_system(7, 30, 4, 0.05, 8)]

    def make_ctx(k, stream):
        ctx = F.Context.from_system(systems[k], stream=stream)
        for C in fsgen.CLASSES:
            buf, _ = fsgen.class_buffer(systems[k], C)
            ctx.set_integrals(C, torch.from_numpy(buf).to("cuda"))
        return ctx

    out = []
    for concurrent in (False, True):
        b = make_batch(systems)
        t1 = torch.zeros(b.n1, dtype=torch.complex128, device="cuda")
        t2 = torch.zeros(b.n2, dtype=torch.complex128, device="cuda")
        res = F.solve_batch(b, t1, t2, tol=1e-10, maxit=150, use_graph=True, ndiis=8, dressed=10, stop_active=3)
        left = F.finish_batch_in_contexts(b, res, t1, t2, make_ctx, tol=1e-10, maxit=150, ndiis=12, dressed=10,
                                          concurrent=concurrent)
        print("concurrent", concurrent, "continued", sorted(left), "iterations", list(res["iters"]), flush=True)
        assert len(left) >= 2 and res["converged"].all()
        out.append((np.array(res["E"]), t1.cpu().numpy(), t2.cpu().numpy()))
        b.destroy()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])
    for k, s in enumerate(systems):
        ctx = single_ctx(s)
        u1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
        u2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
        g = F.solve(ctx, u1, u2, tol=1e-11, maxit=200, ndiis=8)
        assert abs(out[1][0][k] - g["E"]) <= 1e-9
        ctx.destroy()


def test_autotuned_batch_converges_like_single_systems():
    """The batch in the autotuner's launch forms (direct-to-LDS MFMA tiles
    among the candidates, workgroups of converged systems skipped through the
    active flags): the same energies as single-system contexts."""
    torch = _torch()
    import paper_2004_03682_amd as F
    systems = [fsgen.make_system(*p) for p in SPECS[:4]] + [fsgen.make_system(7, 30, 4, 0.05, 8)]
    b = make_batch(systems)
    b.context().autotune(1)
    tiles = {n: c for n, c, _, _ in b.context().gemm_configs()}
    print("batch tiles", tiles, flush=True)
    t1 = torch.zeros(b.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(b.n2, dtype=torch.complex128, device="cuda")
    res = F.solve_batch(b, t1, t2, tol=1e-10, maxit=150, use_graph=True, ndiis=8, dressed=10)
    assert res["converged"].all(), res["iters"]
    for k, s in enumerate(systems):
        ctx = single_ctx(s)
        u1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
        u2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
        g = F.solve(ctx, u1, u2, tol=1e-10, maxit=150, ndiis=8, dressed=10)
        assert g["converged"]
        assert abs(res["E"][k] - g["E"]) <= 1e-9
        ctx.destroy()
    b.destroy()

"""Benchmark: FS-RCCSD (0h,0p) iterations on one MI355X at the production-size
synthetic workload (nocc=40, nvirt=300 spinors, 16 Abelian irreps with
Dirichlet(1) block sizes, sigma=0.03, complex128).

One step = one CCSD iteration of the whole hot path (fscc_iterate): the
residual (every contraction), the Jacobi step with dressed denominators
(refreshed every 25 iterations) and DIIS(8) on the device, and the energy,
with one host synchronisation.  Inputs (packed integrals, amplitudes) are
resident in HBM when the timed region starts.

Prints ONE JSON line.  The roofline object is for the dominant kernel (the
grouped complex GEMM with the largest time per step), timed with HIP events
recorded around every launch on the library's stream during the timed steps.
The cpu_baseline object times the CPU oracle (block-list numpy
implementation) on one residual + Jacobi update + energy of the same system.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CCSD s/iteration + MFMA TFLOP/s, FP64 vs mixed at dE<1e-8 Eh"
DRESSED = 25       # refresh period of the dressed Jacobi denominators (fscc_precondition)
NDIIS = 8          # DIIS depth of the production context's solves
PEAK_FP64 = 78.6   # TFLOP/s, MI355X dense FP64 matrix
PEAK_HBM = 8000.0  # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha():
    """Hash of the library sources that decide a kernel's memory traffic
    (kernels, tile lists, plans)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2004_03682_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel_name, tile=None):
    """HBM bytes per launch from committed rocprofv3 --pmc counters, if they were
    taken on the current library sources for the tile shape in use (the counter
    run records every tile the autotuner dispatches for the op); else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    ent = d.get(kernel_name)
    if not ent or ent.get("kernels_sha256") != kernel_source_sha():
        return None
    t = ent.get("tiles", {}).get(tile)
    return None if t is None else t.get("bytes_per_launch")


def measured_peaks(F, torch):
    """This GPU's rates at the clock it runs under load: matrix-core
    throughput of the three MFMA instructions the GEMMs issue
    (fscc_probe_mfma: register operands only, every SIMD busy) and a 1 GiB
    device-to-device copy (HIP events; bytes read + written)."""
    out = {}
    for k in ("fp64", "bf16", "fp32"):
        tf, _ = F.probe_mfma(k, 4096)
        out[k + "_mfma_tflops"] = round(tf, 2)
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    out["hbm_copy_gbs"] = round(2 * (1 << 30) * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    out["spec"] = {"fp64_mfma_tflops": PEAK_FP64, "bf16_mfma_tflops": 2500.0, "fp32_mfma_tflops": 157.3,
                   "hbm_gbs": 8000.0}
    return out


def cpu_baseline(sysm, buffers):
    import numpy as np
    from oracle import ccsd
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    t0 = time.perf_counter()
    be = ccsd.Blocked(sysm, buffers)
    setup = time.perf_counter() - t0
    # iteration 2 of the solve from the MP2 start: t = MP2 amplitudes (t1 = 0)
    t1 = be.zeros_t1()
    t2 = be.zeros_t2()
    R1, R2 = ccsd.residual(be, t1, t2)
    t1, t2 = t1 + R1 / be.D1, t2 + R2 / be.D2
    t0 = time.perf_counter()
    R1, R2 = ccsd.residual(be, t1, t2, progress=lambda m: log(f"  oracle: {m} done at {time.perf_counter() - t0:.1f}s"))
    t1n, t2n = t1 + R1 / be.D1, t2 + R2 / be.D2
    E = ccsd.energy(be, t1n, t2n)
    dt = time.perf_counter() - t0
    del R1, R2, t1n, t2n
    return dict(value=round(dt, 3), unit="s/iteration", cores=int(cores), kind="oracle",
                sample="one full oracle iteration (block-list residual + Jacobi step + energy) of the same "
                       "nocc=40 nvirt=300 Z16 system at the MP2 amplitudes; DIIS bookkeeping excluded; setup %.1fs excluded" % setup,
                energy_re=float(E.real))


def time_to(hist, E_ref, t_start, thr=1e-8):
    """(iterations, seconds) until |E_k - E_ref| < thr holds for every later iterate."""
    k = next((k for k in range(len(hist)) if all(abs(h["E"] - E_ref) < thr for h in hist[k:])), None)
    if k is None:
        return None, None
    return k + 1, round(hist[k]["time"] - t_start, 5)


GOLDEN = os.path.join(ROOT, "tests", "golden", "o40v300z16_ccsd.json")


def oracle_fixed_point(sysm):
    """The block-list oracle's converged fixed point of the production system
    (stored by tests/golden/make_golden.py): E, and a comparator giving the
    largest |t - t_oracle| of packed device amplitudes over every T1 element
    and the stored T2 sample; None if the file is absent."""
    if not os.path.exists(GOLDEN):
        return None
    g = json.load(open(GOLDEN))
    if g["config"]["seed"] != sysm.seed or not g["converged"]:
        return None
    import numpy as np
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import layout_ref as LR
    T1 = np.array(g["t1"])
    T2 = np.array(g["t2_sample"])
    p1 = LR.t1_positions(sysm, [(int(i), int(a)) for i, a in T1[:, :2]])
    p2, sg2 = LR.t2_positions(sysm, [tuple(int(x) for x in r[:4]) for r in T2])
    v1 = T1[:, 2] + 1j * T1[:, 3]
    v2 = T2[:, 4] + 1j * T2[:, 5]

    def dt(t1, t2):
        a = t1.cpu().numpy()[p1]
        b = sg2 * t2.cpu().numpy()[p2]
        return float(np.abs(a - v1).max()), float(np.abs(b - v2).max())
    return {"E": complex(g["E_re"], g["E_im"]), "iters_to_1e10": g["iters_to_1e10"], "tol": g["tol"], "dt": dt,
            "t2_sample": len(T2)}


def precision_study(ctx, F, torch, dev, E_inf, tconv, args, log, ora=None):
    """FP64 against split-BF16 / split-FP32 ladder + ring contractions:
    per-iteration time, per-result error and time to |E - E_inf| < 1e-8 Eh
    (E_inf = the oracle's converged energy when stored, else the FP64 one),
    all from the same zero start; amplitude errors against the oracle's
    fixed point (every T1 element and the stored T2 sample) when stored, and
    against the FP64 GPU fixed point."""
    u1 = torch.zeros(ctx.n1, dtype=torch.complex128, device=dev)
    u2 = torch.zeros(ctx.n2, dtype=torch.complex128, device=dev)
    q1, q2 = torch.empty_like(u1), torch.empty_like(u2)
    out = {}
    ctx.set_precision("fp64")
    torch.cuda.synchronize()
    ts = time.perf_counter()
    a = F.solve(ctx, u1, u2, tol=1e-10, maxit=300, ndiis=NDIIS, dressed=DRESSED)
    k8, s8 = time_to(a["history"], E_inf, ts)
    out["fp64"] = {"iterations": a["iters"], "iterations_to_1e-8": k8, "seconds_to_1e-8": s8,
                   "seconds_to_converged": round(a["history"][-1]["time"] - ts, 5)}
    log(f"fp64 from zero: {a['iters']} iterations, |dE|<1e-8 after {k8} ({s8}s)")
    # reference residual at the MP2 amplitudes (first Jacobi step from zero, bare denominators)
    u1.zero_()
    u2.zero_()
    ctx.precondition(0, 0.1, F.FSCC_S00)
    ctx.diis_reset(1)
    ctx.build_residual(u1, u2, q1, q2)
    ctx.update_amplitudes(u1, u2, q1, q2)
    ctx.build_residual(u1, u2, q1, q2)
    R1, R2 = q1.clone(), q2.clone()
    Rmax = max(float(R1.abs().max()), float(R2.abs().max()))
    mp2 = (u1.clone(), u2.clone())
    for prec in ("split_bf16", "split_fp32"):
        ctx.set_precision(prec)
        t0 = time.perf_counter()
        ctx.autotune(2)
        tiles = {0: "64x64", 1: "64x32", 2: "32x64", 3: "32x32"}
        cfgs = {n: tiles[c % 4] + ("/Bdirect" if c >= 4 else "") for n, c in ctx.mixed_configs()}
        log(f"{prec}: split tiles {cfgs} (tuned in {time.perf_counter() - t0:.1f}s)")
        u1.copy_(mp2[0])
        u2.copy_(mp2[1])
        ctx.build_residual(u1, u2, q1, q2)
        err = max(float((q1 - R1).abs().max()), float((q2 - R2).abs().max())) / Rmax
        # per-operation times from profiled warm-up iterations, then the
        # per-iteration time of unprofiled steps
        u1.zero_()
        u2.zero_()
        ctx.diis_reset(NDIIS)
        ctx.profile(True)
        for _ in range(max(1, args.warmup)):
            ctx.build_residual(u1, u2, q1, q2)
            ctx.update_amplitudes(u1, u2, q1, q2)
            ctx.energy(u1, u2)
        ops = {o["name"]: o for o in ctx.op_times()}
        ctx.profile(False)
        torch.cuda.synchronize()
        st = time.perf_counter()
        for _ in range(args.steps):
            ctx.build_residual(u1, u2, q1, q2)
            ctx.update_amplitudes(u1, u2, q1, q2)
            ctx.energy(u1, u2)
        torch.cuda.synchronize()
        per_it = (time.perf_counter() - st) / args.steps
        mfac = 6.0 if prec == "split_bf16" else 3.0
        peak = 2500.0 if prec == "split_bf16" else 157.3
        lad = ops["pp-ladder"]
        lad_ms = lad["ms"] / max(1, lad["calls"])
        split_ops = {}
        for n in cfgs:                      # the (0h,0p) operations that run split in this mode
            o = ops.get(n)
            if o is None or o["calls"] == 0:
                continue                    # an operation of another sector
            ms = o["ms"] / max(1, o["calls"])
            split_ops[n] = {"ms_per_call": round(ms, 4),
                            "fp64_equivalent_tflops": round(o["flops"] / (ms * 1e-3) / 1e12, 2),
                            "issued_mfma_tflops": round(mfac * o["flops"] / (ms * 1e-3) / 1e12, 2)}
        rec = {"s_per_iteration": round(per_it, 6), "residual_rel_error_at_mp2": err, "split_tiles": cfgs,
               "split_ops": split_ops,
               "ladder_issued_mfma_frac": round(mfac * lad["flops"] / (lad_ms * 1e-3) / 1e12 / peak, 4),
               "mfma_peak_tflops": peak, "issued_products_per_complex_product": mfac * 4}
        # two-stage convergence from zero: split until max|step| < 1e-7, then FP64
        for sw in (1e-6, 1e-7):
            u1.zero_()
            u2.zero_()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            b = F.solve_mixed(ctx, u1, u2, switch_tol=sw, tol=1e-10, maxit=300, ndiis=NDIIS, dressed=DRESSED)
            k8, s8 = time_to(b["history"], E_inf, ts)
            rec[f"two_stage_switch_{sw:g}"] = {
                "split_iterations": b["split_iters"], "fp64_iterations": b["fp64_iters"],
                "iterations_to_1e-8": k8, "seconds_to_1e-8": s8, "converged": b["converged"],
                "seconds_to_converged": round(b["history"][-1]["time"] - ts, 5),
                "final_dE": abs(b["E"] - E_inf)}
            log(f"{prec}: two-stage (switch {sw:g}): {b['split_iters']}+{b['fp64_iters']} iterations, "
                f"|dE|<1e-8 after {k8} ({s8}s), final |dE| = {abs(b['E'] - E_inf):.2e}")
        # split precision alone: where the iteration settles
        u1.zero_()
        u2.zero_()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        c = F.solve(ctx, u1, u2, tol=1e-12, maxit=120, ndiis=NDIIS, dressed=DRESSED)
        k8, s8 = time_to(c["history"], E_inf, ts)
        rec["split_only"] = {"iterations": c["iters"], "last_max_step": c["history"][-1]["dmax"],
                             "iterations_to_1e-8": k8, "seconds_to_1e-8": s8,
                             "dE_vs_reference": abs(c["E"] - E_inf),
                             "max_abs_dt1_vs_fp64": float((u1 - tconv[0]).abs().max()),
                             "max_abs_dt2_vs_fp64": float((u2 - tconv[1]).abs().max())}
        if ora is not None:
            d1, d2 = ora["dt"](u1, u2)
            rec["split_only"]["max_abs_dt1_vs_oracle"] = d1
            rec["split_only"]["max_abs_dt2_sample_vs_oracle"] = d2
        log(f"{prec}: split-only after {c['iters']} iterations: max|step| {c['history'][-1]['dmax']:.2e}, "
            f"|dE| = {abs(c['E'] - E_inf):.2e}; {per_it * 1e3:.3f} ms/iteration, residual rel. error {err:.2e}")
        out[prec] = rec
    ctx.set_precision("fp64")
    return out


def out_of_core_study(ctx, F, torch, s_per_iter, dom, args, log, staging=512 << 20):
    """The production-size iteration with the packed VVVV integrals in pinned host memory,
    streamed through 2 x 256 MB staging buffers: ladder time and whole
    iteration against the in-memory ones, and the host-to-device copy rate
    the ladder sustains against a plain pinned copy."""
    work = ctx.work()
    vbytes = work["ladder_bytes"]
    # plain pinned host -> device copy of the same size (reference rate)
    n = int(vbytes // 16)
    h = torch.empty(n, dtype=torch.complex128).pin_memory()
    d = torch.empty(n, dtype=torch.complex128, device="cuda")
    d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    st = time.perf_counter()
    for _ in range(3):
        d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    copy_gbs = 3 * vbytes / (time.perf_counter() - st) / 1e9
    del h, d
    torch.cuda.empty_cache()
    ctx.vvvv_out_of_core(staging)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    ctx.diis_reset(NDIIS)
    for _ in range(max(1, args.warmup)):
        ctx.build_residual(t1, t2, r1, r2)
        ctx.update_amplitudes(t1, t2, r1, r2)
        ctx.energy(t1, t2)
    ctx.profile(True, only="pp-ladder")
    torch.cuda.synchronize()
    st = time.perf_counter()
    for _ in range(args.steps):
        ctx.build_residual(t1, t2, r1, r2)
        ctx.update_amplitudes(t1, t2, r1, r2)
        ctx.energy(t1, t2)
    torch.cuda.synchronize()
    per_it = (time.perf_counter() - st) / args.steps
    lad = next(o for o in ctx.op_times() if o["name"] == "pp-ladder")
    ctx.profile(False)
    lad_ms = lad["ms"] / max(1, lad["calls"])
    ctx.vvvv_out_of_core(0)
    rec = {"staging_bytes": staging, "vvvv_bytes": vbytes, "s_per_iteration": round(per_it, 6),
           "in_memory_s_per_iteration": round(s_per_iter, 6),
           "ladder_ms": round(lad_ms, 4), "in_memory_ladder_ms": round(dom["ms"] / dom["calls"], 4),
           "ladder_stream_gbs": round(vbytes / (lad_ms * 1e-3) / 1e9, 2),
           "pinned_copy_gbs": round(copy_gbs, 2),
           "device_bytes_saved": vbytes - staging}
    log(f"out-of-core VVVV: ladder {lad_ms:.3f} ms ({rec['ladder_stream_gbs']} GB/s streamed; plain pinned copy "
        f"{copy_gbs:.1f} GB/s), iteration {per_it * 1e3:.3f} ms vs {s_per_iter * 1e3:.3f} ms in memory")
    del t1, t2, r1, r2
    return rec


def real_study(F, torch, fsgen, cfg, complex_s_per_iter, args, log, complex_sectors=None):
    """The production shape as a real double group (the same seed's integrals made
    real): the real-arithmetic context's s/iteration, its GEMM rate and
    iterations to convergence, against the complex iteration; then one
    dynamically shifted (0h,1p) and (0h,2p) solve each (S = -3 Eh, n = 3) with
    ms per iteration against the complex sectors' ms per iteration."""
    s = fsgen.make_system(cfg["nocc"], cfg["nvirt"], cfg["nirrep"], cfg["sigma"], cfg["seed"], nact=cfg["nact"],
                          real=True)
    ctx = F.Context.from_system(s, precision="real_fp64")
    for C in fsgen.CLASSES:
        buf, _ = fsgen.class_buffer(s, C)
        d = torch.from_numpy(fsgen.real_buffer(buf)).cuda()
        ctx.set_integrals(C, d)
        del d, buf
    ctx.autotune(1)
    t1 = torch.zeros(ctx.n1, dtype=torch.float64, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.float64, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    ctx.diis_reset(NDIIS)
    ctx.profile(True)
    for _ in range(max(1, args.warmup)):
        ctx.build_residual(t1, t2, r1, r2)
        ctx.update_amplitudes(t1, t2, r1, r2)
        ctx.energy(t1, t2)
    ops = ctx.op_times()
    ctx.profile(False)
    nw = max(1, args.warmup)
    torch.cuda.synchronize()
    st = time.perf_counter()
    for _ in range(args.steps):
        ctx.build_residual(t1, t2, r1, r2)
        ctx.update_amplitudes(t1, t2, r1, r2)
        ctx.energy(t1, t2)
    torch.cuda.synchronize()
    per_it = (time.perf_counter() - st) / args.steps
    work = ctx.work()
    gemm_ms = sum(o["ms"] for o in ops if o["flops"] > 0) / nw
    real_flops = work["gemm_flops"] / 4.0          # the plan counts complex flops (8 per complex MAC)
    lad = next(o for o in ops if o["name"] == "pp-ladder")
    lad_ms = lad["ms"] / max(1, lad["calls"])
    t1.zero_()
    t2.zero_()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    g = F.solve(ctx, t1, t2, tol=1e-10, maxit=200, ndiis=NDIIS)
    solve_s = time.perf_counter() - ts
    E = g["E"]
    k8 = next((h["iter"] for k, h in enumerate(g["history"]) if all(abs(x["E"] - E) < 1e-8 for x in g["history"][k:])),
              None)
    rec = {"s_per_iteration": round(per_it, 6), "complex_s_per_iteration": round(complex_s_per_iter, 6),
           "speedup_vs_complex": round(complex_s_per_iter / per_it, 3),
           "gemm_tflops": round(real_flops / (gemm_ms * 1e-3) / 1e12, 3) if gemm_ms > 0 else None,
           "real_gemm_flops_per_iteration": real_flops,
           "pp_ladder_ms": round(lad_ms, 4),
           "pp_ladder_tflops": round(lad["flops"] / 4.0 / (lad_ms * 1e-3) / 1e12, 3),
           "converged": g["converged"], "iterations": g["iters"], "iterations_to_1e-8": k8,
           "seconds_to_converged": round(solve_s, 4), "energy": E.real,
           "workload": "nocc=40 nvirt=300 Z16 shape, real integrals (sqrt(2) Re of seed 1002's), real-arithmetic context"}
    log(f"real: {per_it * 1e3:.3f} ms/iteration ({complex_s_per_iter / per_it:.2f}x the complex iteration), "
        f"ladder {lad_ms:.3f} ms, converged {g['converged']} in {g['iters']} iterations ({solve_s:.3f}s)")
    if s.nact >= 2 and g["converged"]:
        try:
            ctx.prepare_sector(t1, t2)
            s1 = torch.zeros(ctx.m1, dtype=torch.float64, device="cuda")
            s2 = torch.zeros(ctx.m2, dtype=torch.float64, device="cuda")
            ctx.dynamic_shift(-3.0, 3, F.FSCC_S01)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            o1 = F.solve01(ctx, s1, s2, tol=1e-10, maxit=200, ndiis=8)
            torch.cuda.synchronize()
            e1 = time.perf_counter() - ts
            ctx.prepare_sector(s1, s2, F.FSCC_S02)
            sp = torch.zeros(ctx.p2, dtype=torch.float64, device="cuda")
            ctx.dynamic_shift(-3.0, 3, F.FSCC_S02)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            o2 = F.solve02(ctx, sp, tol=1e-10, maxit=200, ndiis=8)
            torch.cuda.synchronize()
            e2 = time.perf_counter() - ts
            sec = {"shift": [-3.0, 3],
                   "fs01": {"converged": o1["converged"], "iterations": o1["iters"],
                            "ms_per_iteration": round(e1 / max(1, o1["iters"]) * 1e3, 4)},
                   "fs02": {"converged": o2["converged"], "iterations": o2["iters"],
                            "ms_per_iteration": round(e2 / max(1, o2["iters"]) * 1e3, 4)}}
            for k in ("fs01", "fs02"):
                c = (complex_sectors or {}).get(k)
                if c:
                    sec[k]["complex_ms_per_iteration"] = c
                    sec[k]["speedup_vs_complex"] = round(c / sec[k]["ms_per_iteration"], 3)
            rec["sectors"] = sec
            log(f"real sectors: (0h,1p) {sec['fs01']}, (0h,2p) {sec['fs02']}")
        except F.FsccError as e:
            rec["sectors"] = {"status": f"failed ({e})"}
    ctx.destroy()
    torch.cuda.empty_cache()
    return rec


# the batched workload's solver: DIIS(8), dressed Jacobi denominators refreshed
# every 25 iterations (same fixed point); at most 600 iterations per system
BATCH_SOLVER = dict(ndiis=8, shift=0.0, dressed=25)
# DIIS depth of a system in a context of its own (the batch keeps 8): the
# stragglers the batch hands off and the one-after-another baseline
ALONE_NDIIS = 12
BATCH_MAXIT = 600
BATCH_STOP_ACTIVE = 2      # stragglers continue in their own contexts


def learned_study(F, torch, b, mp2, t2_conv, log):
    """The committed warm-start network on the batch: iterations and time to
    1e-8 Eh against the MP2 start (same solver), inference and training
    throughput of the network kernels."""
    import numpy as np
    from paper_2004_03682_amd import warmstart as W
    net = F.MLP(0)
    meta = W.load(net)
    ev = W.evaluate(net, b, log=log, mp2=mp2)
    ev["solver"] = dict(W.SOLVER)
    # inference over every T2 element of the batch
    D1, D2 = b.denominators()
    u1, u2, r1, r2 = W.first_iterates(b, D1, D2)
    pred = torch.empty_like(u2)
    W.predict(net, u2, r2, D2, pred)
    torch.cuda.synchronize()
    st = time.perf_counter()
    W.predict(net, u2, r2, D2, pred)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - st
    flops_row = 2.0 * (8 * 256 + 256 * 256 + 256 * 4)
    # training steps (minibatch 8192) on rows of this batch against its converged T2
    rng = np.random.default_rng(0)
    n = u2.numel()
    idx = [torch.from_numpy(rng.integers(0, n, 8192).astype(np.int64)).cuda() for _ in range(30)]
    for k in range(5):
        net.loss_grad(u2, r2, D2, t2_conv, idx=idx[k], mode=1)
        net.adam(1e-5)
    torch.cuda.synchronize()
    st = time.perf_counter()
    for k in range(5, 30):
        net.loss_grad(u2, r2, D2, t2_conv, idx=idx[k], mode=1)
        net.adam(1e-5)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - st) / 25
    net.destroy()
    ev.update({
        "network": {"trained_on_systems": int(meta["systems"]), "training_rows": int(meta["rows"]),
                    "training_steps": int(meta["steps"]), "final_training_loss": float(meta["loss_last"]),
                    "training_seconds": float(meta["train_seconds"]), "loss": "absolute (size-weighted)"},
        "inference_rows": int(n), "inference_seconds": round(t_inf, 4),
        "inference_tflops": round(flops_row * n / t_inf / 1e12, 2),
        "train_step_ms_8192_rows": round(t_step * 1e3, 3),
        "train_rows_per_second": round(8192 / t_step),
    })
    log(f"learned: inference {n} rows in {t_inf * 1e3:.1f} ms ({ev['inference_tflops']} TFLOP/s fp32), "
        f"train step {t_step * 1e3:.2f} ms / 8192 rows")
    return ev


def fs02_study(ctx, F, torch, sysm, s1, s2, log, S=-3.0, n=3, scales=(1.0, 0.9, 0.8, 0.7, 0.6, 0.5, 0.4)):
    """(0h,2p) sector over the active pairs, prepared from the (0h,1p) amplitudes in s1, s2:
    dynamically shifted solves at decreasing scale, [2/1] Pade extrapolation of every
    pair-state energy, time per iteration, and the pair ladder's streamed HBM rate."""
    import numpy as np
    out = {"npair": int(ctx.npair), "amplitudes": int(ctx.p2), "S": S, "n": n, "scales": list(scales)}
    torch.cuda.synchronize()
    st = time.perf_counter()
    ctx.prepare_sector(s1, s2, F.FSCC_S02)
    torch.cuda.synchronize()
    out["prepare_ms"] = round((time.perf_counter() - st) * 1e3, 3)
    sp = torch.zeros(ctx.p2, dtype=torch.complex128, device=s1.device)
    eigs, iters, conv = [], [], []
    st = time.perf_counter()
    try:
        for lam in scales:
            ctx.dynamic_shift(lam * S, n, F.FSCC_S02)
            r = F.solve02(ctx, sp, tol=1e-10, maxit=200, ndiis=8)
            eigs.append(r["eig"])
            iters.append(r["iters"])
            conv.append(r["converged"])
    except F.FsccError as e:
        out["status"] = f"failed ({e})"
        log(f"(0h,2p) failed: {e}")
        return out
    finally:
        ctx.dynamic_shift(0.0, n, F.FSCC_S02)
    torch.cuda.synchronize()
    el = time.perf_counter() - st
    out.update(iterations=iters, converged=conv, seconds=round(el, 4),
               ms_per_iteration=round(el / max(1, sum(iters)) * 1e3, 4))
    if all(conv):
        E = np.array(eigs)
        ext = np.array([F.pade(list(scales), E[:, k], 2, 1) for k in range(E.shape[1])])
        alt = np.array([F.pade(list(scales), E[:, k], 3, 0) for k in range(E.shape[1])])
        out["extrapolated_re"] = [float(x.real) for x in ext]
        out["max_abs_diff_pade_2_1_vs_3_0"] = float(np.abs(alt - ext).max())
    # per-operation times of the residual; the pair ladder reads every VVVV block once
    r = torch.empty_like(sp)
    ctx.profile(True)
    for _ in range(5):
        ctx.build_residual(None, sp, None, r, F.FSCC_S02)
    torch.cuda.synchronize()
    ops = {o["name"]: o for o in ctx.op_times() if o["calls"]}
    ctx.profile(False)
    lad = ops.get("P2-ladder")
    if lad:
        # algorithmic bytes: every <ab||cd> block of a pair irrep that holds an active pair,
        # read once, plus omega read and sigma2 read and written
        G = sysm.nirrep
        gv = [int(g) for g in sysm.irrep[sysm.nocc:]]
        ga = [int(sysm.irrep[p]) for p in sysm.active]

        def pairs(gl):
            c = [0] * G
            for i in range(len(gl)):
                for j in range(i + 1, len(gl)):
                    c[(gl[i] + gl[j]) % G] += 1
            return c
        nab, nxy = pairs(gv), pairs(ga)
        vb = float(sum(16 * (nab[g] ** 2 + 3 * nxy[g] * nab[g]) for g in range(G) if nxy[g]))
        ms = lad["ms"] / lad["calls"]
        cfg = next(((c, b, sp) for nm, c, b, sp in ctx.gemm_configs() if nm == "P2-ladder"), None)
        out["pair_ladder"] = {"ms": round(ms, 4), "bytes": vb, "GB_per_s": round(vb / (ms * 1e-3) / 1e9, 1),
                              "frac_of_hbm_peak": round(vb / (ms * 1e-3) / 8.0e12, 3),
                              "pair_irreps_with_pairs": sum(1 for g in range(G) if nxy[g]),
                              "tile": None if cfg is None else list(cfg)}
    # only the (0h,2p) residual ran while profiling: every timed operation belongs to it
    out["residual_ms"] = round(sum(o["ms"] / o["calls"] for o in ops.values()), 4)
    log(f"(0h,2p): {ctx.npair} pairs, iterations {iters}, {out['ms_per_iteration']:.3f} ms/iteration, "
        f"pair ladder {out.get('pair_ladder')}")
    return out


def batch_study(F, torch, fsgen, args, log):
    """64 independent systems (nocc U{10..30}, nvirt U{60..200}, 4-8 irreps,
    sigma 0.05, seeds 40000..40063): one batched solve (grouped launches, graph
    per iteration) against the same systems solved one after another."""
    import numpy as np
    ss = fsgen.batch_systems(64, 40000)
    t0 = time.perf_counter()
    b = F.Batch(ss)
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    for k, s in enumerate(ss):
        for C in fsgen.CLASSES:
            d = fsgen.class_buffer_gpu(s, C)
            b.set_integrals(k, C, d)
            del d
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    t_int = time.perf_counter() - t0
    log(f"batch: 64 systems, n1={b.n1} n2={b.n2}; plans {t_plan:.1f}s, integrals (device generator) {t_int:.1f}s")
    t0 = time.perf_counter()
    b.context().autotune(1)
    t_tune = time.perf_counter() - t0
    t1 = torch.zeros(b.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(b.n2, dtype=torch.complex128, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    # per-iteration time with every system active (graph replay)
    b.reset(BATCH_SOLVER["ndiis"], 1e-10, BATCH_SOLVER["shift"])
    for _ in range(2):
        b.step(t1, t2, r1, r2, True)
    torch.cuda.synchronize()
    st = time.perf_counter()
    for _ in range(5):
        b.step(t1, t2, r1, r2, True)
    it_ms = (time.perf_counter() - st) / 5 * 1e3
    ctxv = b.context()
    gemm = sum(o["flops"] for o in ctxv.op_times() if o["flops"] > 0)
    # full solve from zero; the last stragglers continue in their own contexts
    t1.zero_()
    t2.zero_()

    def make_ctx(k, stream):
        c = F.Context.from_system(ss[k], stream=stream)
        for C in fsgen.CLASSES:
            c.set_integrals(C, fsgen.class_buffer_gpu(ss[k], C, stream=stream))
        return c
    torch.cuda.synchronize()
    ts = time.perf_counter()
    res = F.solve_batch(b, t1, t2, tol=1e-10, maxit=BATCH_MAXIT, use_graph=True, stop_active=args.batch_stop_active,
                        **BATCH_SOLVER)
    t_batch = time.perf_counter() - ts
    n_batch_its = len(res["history"])
    alone = F.finish_batch_in_contexts(b, res, t1, t2, make_ctx, tol=1e-10, maxit=BATCH_MAXIT,
                                       ndiis=ALONE_NDIIS, dressed=BATCH_SOLVER["dressed"])
    el = time.perf_counter() - ts
    conv = res["converged"]
    E = res["E"]
    # time until every converged system is within 1e-8 Eh of its final energy
    hist = res["history"]
    t8s = []
    for s in range(len(ss)):
        if not conv[s]:
            continue
        seq = [(h[s, 0] + 1j * h[s, 1], tm) for h, tm in zip(hist, res["times"])]
        if s in alone:
            seq += [(h["E"], h["time"]) for h in alone[s]["history"]]
        e = E[s]
        t8s.append(next(tm for k, (x, tm) in enumerate(seq) if all(abs(y - e) < 1e-8 for y, _ in seq[k:])) - ts)
    t8 = max(t8s) if t8s else None
    log(f"batch: {it_ms:.2f} ms/iteration (all active), solve {el:.2f}s, converged {int(conv.sum())}/64, "
        f"iterations mean {res['iters'].mean():.1f} max {res['iters'].max()}")
    out = {"systems": 64, "n1_total": b.n1, "n2_total": b.n2, "ms_per_iteration_all_active": round(it_ms, 3),
           "gemm_tflops_all_active": round(gemm / (it_ms * 1e-3) / 1e12, 2) if gemm else None,
           "solve_seconds": round(el, 4), "seconds_to_1e-8_all_converged": round(t8, 4) if t8 else None,
           "converged": int(conv.sum()), "iterations_mean": float(res["iters"].mean()),
           "iterations_max": int(res["iters"].max()),
           "solver": dict(BATCH_SOLVER, tol=1e-10, graph=True, maxit=BATCH_MAXIT, stop_active=args.batch_stop_active,
                          alone_ndiis=ALONE_NDIIS, alone_concurrent=True),
           "batched_iterations": n_batch_its, "batched_seconds": round(t_batch, 4),
           "continued_alone": {int(k): {"iterations": int(res["iters"][k]), "converged": bool(conv[k])} for k in alone},
           "plan_seconds": round(t_plan, 2), "integral_seconds": round(t_int, 2), "autotune_seconds": round(t_tune, 2)}
    if not args.no_learned:
        # both starts solved inside the study with the same batched solver
        out["learned_warm_start"] = learned_study(F, torch, b, None, t2, log)
    b.destroy()
    del t1, t2, r1, r2
    torch.cuda.empty_cache()
    if args.no_sequential:
        return out
    # the same systems one after another (plans and integrals outside the clock)
    seq, iters, agree = 0.0, 0, 0.0
    for k, s in enumerate(ss):
        ctx = F.Context.from_system(s)
        for C in fsgen.CLASSES:
            d = fsgen.class_buffer_gpu(s, C)
            ctx.set_integrals(C, d)
            del d
        ctx.level_shift(BATCH_SOLVER["shift"])
        u1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
        u2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        try:
            g = F.solve(ctx, u1, u2, tol=1e-10, maxit=BATCH_MAXIT, ndiis=ALONE_NDIIS,
                        dressed=BATCH_SOLVER["dressed"])
            iters += g["iters"]
            if conv[k] and g["converged"]:
                agree = max(agree, abs(g["E"] - E[k]))
        except F.FsccError:
            iters += BATCH_MAXIT
        seq += time.perf_counter() - ts
        ctx.destroy()
        del u1, u2
        if k % 16 == 15:
            log(f"  sequential: {k + 1} systems, {seq:.2f}s")
    out["sequential_solve_seconds"] = round(seq, 4)
    out["sequential_iterations_total"] = int(iters)
    out["batched_speedup"] = round(seq / el, 2)
    out["max_abs_dE_batched_vs_sequential"] = agree
    log(f"batch: sequential {seq:.2f}s vs batched {el:.2f}s (x{seq / el:.2f}); max |dE| {agree:.1e}")
    return out


def sector_op_table(ctx, run, nrep=5, top=16):
    """Per-operation times of one sector's residual (HIP events around each
    operation over nrep evaluations): ms per call, TFLOP/s of the GEMMs, GB/s of
    the algorithmic bytes, and the residual's total."""
    ctx.profile(True)
    for _ in range(nrep):
        run()
    ops = [o for o in ctx.op_times() if o["calls"] > 0]
    ctx.profile(False)
    rows = []
    for o in ops:
        per = o["ms"] / o["calls"]
        row = {"op": o["name"], "kind": o["kind"], "ms_per_call": round(per, 4), "bytes": o["bytes"],
               "GB_per_s": round(o["bytes"] / (per * 1e-3) / 1e9, 1) if per > 0 else None}
        if o["flops"] > 0:
            row["tflops"] = round(o["flops"] / (per * 1e-3) / 1e12, 2)
        rows.append(row)
    rows.sort(key=lambda r: -r["ms_per_call"])
    total = sum(o["ms"] for o in ops) / nrep
    by_kind = {}
    for o in ops:
        by_kind[o["kind"]] = by_kind.get(o["kind"], 0.0) + o["ms"] / nrep
    return {"residual_ms": round(total, 4), "ms_by_kind": {k: round(v, 4) for k, v in by_kind.items()},
            "bytes_per_residual": sum(o["bytes"] * o["calls"] for o in ops) / nrep, "ops": rows[:top]}


def reorder_table(ops, nwarm):
    """HBM rate of the reorders / antisymmetrisers (TTGT steps 1, 2 and 4) from the
    per-operation times of the warm-up iterations and the library's algorithmic
    bytes per call (each destination element written once, read once when
    accumulating; each distinct source element read once)."""
    rows = []
    for o in ops:
        if o["kind"] != "reorder" or o["calls"] <= 0:
            continue
        per = o["ms"] / o["calls"]
        gbs = o["bytes"] / (per * 1e-3) / 1e9 if per > 0 else 0.0
        rows.append({"op": o["name"], "ms_per_call": round(per, 4), "bytes": o["bytes"],
                     "GB_per_s": round(gbs, 1), "frac_of_hbm_peak": round(gbs / PEAK_HBM, 3)})
    tot_ms = sum(o["ms"] for o in ops if o["kind"] == "reorder") / max(1, nwarm)
    tot_b = sum(o["bytes"] * o["calls"] for o in ops if o["kind"] == "reorder") / max(1, nwarm)
    rows.sort(key=lambda r: -r["ms_per_call"])
    return {"ms_per_iteration": round(tot_ms, 4), "bytes_per_iteration": tot_b,
            "GB_per_s": round(tot_b / (tot_ms * 1e-3) / 1e9, 1) if tot_ms > 0 else None,
            "frac_of_hbm_peak": round(tot_b / (tot_ms * 1e-3) / 1e9 / PEAK_HBM, 3) if tot_ms > 0 else None,
            "ops": rows}


PROFILE_REPS = 5
TILE_NAMES = {0: "64x64", 1: "128x16", 2: "16x128", 3: "32x32", 4: "64x16", 5: "16x64", 6: "skinny64x32", 7: "tall",
              8: "reduction", 9: "32x64", 10: "64x32", 11: "dot", 12: "64x64r", 13: "64x32r"}


def tile_str(c, b, sp):
    """Name of a GEMM configuration (fscc_gemm_config): tile, 3M/DB/DL flags, K depth, split-K."""
    return (f"{TILE_NAMES[c & 255]}{'/3M' if c & 256 else ''}{'/DB' if c & 512 else ''}{'/DL' if c & 1024 else ''}"
            f"/bk{b}{'/splitK' if sp else ''}")


def profile_ops(args):
    """Operations of one residual run alone, PROFILE_REPS times in a row each,
    at the end of the program, every batch preceded by one small torch fill
    kernel as a marker (so that the dispatches of operation i in a counter
    run are those between the i-th of the last n markers and the next).
    Times them with HIP events on the library's stream and writes the list to
    args.profile_ops.  --ops: "reorders" (every reorder), "gemms", or names;
    --sector 0 or 1 ((0h,0p) or (0h,1p), 6 active virtuals); --precision."""
    import torch

    import fsgen
    import paper_2004_03682_amd as F
    s = fsgen.workload_system("o40v300z16")
    ctx = F.Context.from_system(s)
    for C in fsgen.CLASSES:
        ctx.set_integrals(C, torch.from_numpy(fsgen.class_buffer(s, C)[0]).cuda())
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if args.tune_file:
        ctx.tune_cache(args.tune_file)
    ctx.autotune(1)
    cached = ctx.autotune_cached()
    if args.precision != "fp64":
        ctx.set_precision(args.precision)
        ctx.autotune(2)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    # two iterations give the amplitudes (and so every operation's input) the
    # values of the second iteration; the last residual binds the buffers
    ctx.diis_reset(NDIIS)
    for _ in range(2):
        ctx.build_residual(t1, t2, r1, r2)
        ctx.update_amplitudes(t1, t2, r1, r2)
    run = lambda: ctx.build_residual(t1, t2, r1, r2)
    if args.sector == 1:
        ctx.prepare_sector(t1, t2)
        ctx.precondition(1, 0.1)
        s1 = torch.zeros(ctx.m1, dtype=torch.complex128, device="cuda")
        s2 = torch.zeros(ctx.m2, dtype=torch.complex128, device="cuda")
        q1, q2 = torch.empty_like(s1), torch.empty_like(s2)
        ctx.diis_reset(6, F.FSCC_S01)
        ctx.build_residual(s1, s2, q1, q2, F.FSCC_S01)
        ctx.update_amplitudes(s1, s2, q1, q2, F.FSCC_S01)
        run = lambda: ctx.build_residual(s1, s2, q1, q2, F.FSCC_S01)
    ctx.profile(True)
    run()
    ops = ctx.op_times()
    ctx.profile(False)
    torch.cuda.synchronize()
    if args.ops == "reorders":
        sel = [k for k, o in enumerate(ops) if o["kind"] == "reorder" and o["calls"] > 0 and o["bytes"] > 0]
    elif args.ops == "all":
        sel = [k for k, o in enumerate(ops) if o["calls"] > 0]
    elif args.ops == "gemms":
        sel = [k for k, o in enumerate(ops) if o["kind"] == "gemm" and o["calls"] > 0]
    else:
        names = args.ops.split(",")
        sel = [k for k, o in enumerate(ops) if o["name"] in names and o["calls"] > 0]
    marker = torch.zeros(64, dtype=torch.float32, device="cuda")
    rows = []
    with torch.cuda.stream(ctx.stream):
        for k in sel:
            marker.fill_(float(k))
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(ctx.stream)
            ctx.op_run(k, PROFILE_REPS)
            b.record(ctx.stream)
            b.synchronize()
            ms = a.elapsed_time(b) / PROFILE_REPS
            o = ops[k]
            rows.append({"k": k, "op": o["name"], "kind": o["kind"], "bytes": o["bytes"], "flops": o["flops"],
                         "reps": PROFILE_REPS, "ms_per_call": ms, "GB_per_s": o["bytes"] / (ms * 1e-3) / 1e9})
            if o["kind"] == "gemm":
                rows[-1]["tile"] = tile_str(*ctx.gemm_config(k))
            log(f"  {o['name']:24s} {ms * 1e3:8.1f} us  {rows[-1]['GB_per_s']:7.1f} GB/s"
                + (f"  {o['flops'] / (ms * 1e-3) / 1e12:6.2f} TFLOP/s" if o["flops"] else ""))
    torch.cuda.synchronize()
    with open(args.profile_ops, "w") as f:
        json.dump({"autotune_cached": cached, "precision": args.precision, "sector": args.sector, "ops": rows},
                  f, indent=1)
    ctx.destroy()


def _read_counters(path, counters):
    """Per dispatch of a rocprofv3 --pmc csv, in dispatch order: (id, kernel
    name, workgroups, {counter: value})."""
    import csv
    by = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            e = by.setdefault(d, [d, r["Kernel_Name"], int(r["Grid_Size"]) // max(1, int(r["Workgroup_Size"])), {}])
            if r["Counter_Name"] in counters:
                e[3][r["Counter_Name"]] = e[3].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [by[d] for d in sorted(by)]


def _windows(disp, nops):
    """Dispatches of each profiled operation: between the last nops markers."""
    marks = [i for i, d in enumerate(disp) if "FillFunctor" in d[1]][-nops:]
    assert len(marks) == nops, "marker kernels not found"
    return [disp[m + 1:(marks[j + 1] if j + 1 < nops else len(disp))] for j, m in enumerate(marks)]


def _short(kernel):
    k = kernel.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("fscc::", "")
    return k


def summarize_ops(args):
    """Markdown table of HBM traffic per operation from the counter runs of
    --profile-ops (FETCH_SIZE, WRITE_SIZE) and of --copy-calibration: per
    operation and kernel, counter bytes per call against the operation's
    algorithmic bytes and its time."""
    times, fetch, write, cfetch, cwrite = args.summarize_ops
    prof = json.load(open(times))
    rows = prof["ops"]
    cf = [d for d in _read_counters(cfetch, {"FETCH_SIZE"}) if "copyBuffer" in d[1]]
    cw = [d for d in _read_counters(cwrite, {"WRITE_SIZE"}) if "copyBuffer" in d[1]]
    gib_kib = float(1 << 20)
    fscale = gib_kib / (sum(d[3]["FETCH_SIZE"] for d in cf) / len(cf))
    wscale = gib_kib / (sum(d[3]["WRITE_SIZE"] for d in cw) / len(cw))
    fw = _windows(_read_counters(fetch, {"FETCH_SIZE"}), len(rows))
    ww = _windows(_read_counters(write, {"WRITE_SIZE"}), len(rows))
    lines = ["| op | kernels (dispatches per call) | workgroups | ms per call | algorithmic bytes | HBM read "
             "| HBM written | counter / algorithmic | GB/s (algorithmic) | of 8 TB/s |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    tot_alg = tot_rd = tot_wr = tot_ms = 0.0
    for r, fs, ws in zip(rows, fw, ww):
        reps = r["reps"]
        kern = {}
        for d in fs:
            kern.setdefault(_short(d[1]), [0, d[2]])[0] += 1
        rd = sum(d[3].get("FETCH_SIZE", 0.0) for d in fs) / reps * fscale * 1024.0
        wr = sum(d[3].get("WRITE_SIZE", 0.0) for d in ws) / reps * wscale * 1024.0
        gbs = r["bytes"] / (r["ms_per_call"] * 1e-3) / 1e9
        tot_alg += r["bytes"]
        tot_rd += rd
        tot_wr += wr
        tot_ms += r["ms_per_call"]
        ks = ", ".join(f"`{k}` ({n // reps})" for k, (n, g) in kern.items())
        grids = "/".join(str(g) for k, (n, g) in kern.items())
        lines.append(f"| {r['op']} | {ks} | {grids} | {r['ms_per_call']:.4f} | {r['bytes'] / 1e6:.1f} MB | "
                     f"{rd / 1e6:.1f} MB | {wr / 1e6:.1f} MB | {(rd + wr) / r['bytes']:.2f} | {gbs:.0f} | "
                     f"{gbs / PEAK_HBM:.2f} |")
    lines.append(f"| all | | | {tot_ms:.4f} | {tot_alg / 1e6:.1f} MB | {tot_rd / 1e6:.1f} MB | "
                 f"{tot_wr / 1e6:.1f} MB | {(tot_rd + tot_wr) / tot_alg:.2f} | "
                 f"{tot_alg / (tot_ms * 1e-3) / 1e9:.0f} | {tot_alg / (tot_ms * 1e-3) / 1e9 / PEAK_HBM:.2f} |")
    print(f"calibration: fetch x {fscale:.4f}, write x {wscale:.4f} (1 GiB device copy)")
    print("\n".join(lines))
    if args.traffic_out and prof.get("precision", "fp64") == "fp64":
        # HBM bytes per launch of each GEMM's grouped kernel (not its split-K
        # pass), for the roofline object of the bench line
        d = json.load(open(args.traffic_out)) if os.path.exists(args.traffic_out) else {}
        for r, fs, ws in zip(rows, fw, ww):
            if r["kind"] != "gemm" or "tile" not in r:
                continue
            mf = [x for x in fs if _short(x[1]).startswith("k_z") and "splitk" not in x[1]]
            mw = [x for x in ws if _short(x[1]).startswith("k_z") and "splitk" not in x[1]]
            if not mf or not mw:
                continue
            fk = sum(x[3].get("FETCH_SIZE", 0.0) for x in mf) / len(mf)
            wk = sum(x[3].get("WRITE_SIZE", 0.0) for x in mw) / len(mw)
            ent = d.setdefault(r["op"], {})
            if ent.get("kernels_sha256") != kernel_source_sha():
                ent["tiles"] = {}          # counters of other library sources do not carry over
            ent.update({"kernel": _short(mf[0][1]), "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4),
                        "algorithmic_bytes_per_launch": r["bytes"], "kernels_sha256": kernel_source_sha()})
            ent.setdefault("tiles", {})
            ent["tiles"][r["tile"]] = {"workgroups": mf[0][2], "fetch_kib_raw": round(fk, 1), "write_kib_raw": round(wk, 1),
                                       "dispatches": len(mf),
                                       "bytes_per_launch": int((fk * fscale + wk * wscale) * 1024)}
        with open(args.traffic_out, "w") as f:
            json.dump(d, f, indent=1)


_TILE_OF = {(64, 64, 2, 2): 0, (128, 16, 4, 1): 1, (16, 128, 1, 4): 2, (32, 32, 2, 2): 3, (64, 16, 4, 1): 4,
            (16, 64, 1, 4): 5, (32, 64, 2, 2): 9, (64, 32, 2, 2): 10, (64, 64, 4, 1): 12, (64, 32, 4, 1): 13}


def summarize_ladder_candidates(args):
    """HBM bytes per launch of every pp-ladder tile the autotuner dispatches
    (the grouped GEMM with ROLE = 1 is the ladder's alone), from counter runs
    of an autotuning program: per template instance and grid, the smaller grid
    being the unsplit and the larger the split-K launch.  Stored under
    'pp-ladder' in --traffic-out, beside the tile the profile run chose."""
    fetch, write, cfetch, cwrite = args.summarize_ladder_candidates
    cf = [d for d in _read_counters(cfetch, {"FETCH_SIZE"}) if "copyBuffer" in d[1]]
    cw = [d for d in _read_counters(cwrite, {"WRITE_SIZE"}) if "copyBuffer" in d[1]]
    fscale = float(1 << 20) / (sum(d[3]["FETCH_SIZE"] for d in cf) / len(cf))
    wscale = float(1 << 20) / (sum(d[3]["WRITE_SIZE"] for d in cw) / len(cw))
    groups = {}
    for path, cnt in ((fetch, "FETCH_SIZE"), (write, "WRITE_SIZE")):
        for d in _read_counters(path, {cnt}):
            k = _short(d[1])
            if k.startswith("k_zgemm<"):         # BM, BN, WM, WN, BK, TA, TB, ROLE, M3, DB
                t = [x.strip() for x in k[len("k_zgemm<"):-1].split(",")]
                if len(t) < 10 or t[7] != "1":
                    continue
                key = (int(t[0]), int(t[1]), int(t[2]), int(t[3]), int(t[4]), t[8] == "true", 512 if t[9] == "true" else 0)
            elif k.startswith("k_zgemm_dl<"):    # BM, BN, WM, WN, S, TA, TB, ROLE, M3 (16-deep slices)
                t = [x.strip() for x in k[len("k_zgemm_dl<"):-1].split(",")]
                if len(t) < 9 or t[7] != "1":
                    continue
                key = (int(t[0]), int(t[1]), int(t[2]), int(t[3]), 16, t[8] == "true", 1024)
            else:
                continue
            g = groups.setdefault(key, {}).setdefault(d[2], {"FETCH_SIZE": [], "WRITE_SIZE": []})
            g[cnt].append(d[3].get(cnt, 0.0))
    d = json.load(open(args.traffic_out)) if os.path.exists(args.traffic_out) else {}
    ent = d.setdefault("pp-ladder", {})
    if ent.get("kernels_sha256") != kernel_source_sha():
        ent.clear()
    ent.update({"kernels_sha256": kernel_source_sha(), "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4)})
    tiles = ent.setdefault("tiles", {})
    rows = []
    for (bm, bn, wm, wn, bk, m3, form), by_grid in groups.items():
        grids = sorted(by_grid)
        for gi, grid in enumerate(grids):
            f, w = by_grid[grid]["FETCH_SIZE"], by_grid[grid]["WRITE_SIZE"]
            if not f or not w:
                continue
            c = _TILE_OF[(bm, bn, wm, wn)] | (256 if m3 else 0) | form
            name = tile_str(c, bk, gi > 0)
            fk, wk = sum(f) / len(f), sum(w) / len(w)
            tiles.setdefault(name, {"workgroups": grid, "fetch_kib_raw": round(fk, 1), "write_kib_raw": round(wk, 1),
                                    "dispatches": len(f), "bytes_per_launch": int((fk * fscale + wk * wscale) * 1024)})
            rows.append((tiles[name]["bytes_per_launch"], name, grid, len(f)))
    with open(args.traffic_out, "w") as fo:
        json.dump(d, fo, indent=1)
    print("| tile | workgroups | dispatches | HBM bytes per launch |\n|---|---|---|---|")
    for b, name, grid, n in sorted(rows):
        print(f"| {name} | {grid} | {n} | {b / 1e9:.2f} GB |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--streams", type=int, default=1, choices=(1, 2),
                    help="residual operations on one stream or two overlapping streams (fscc_set_streams)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fs01", action="store_true", help="skip the (0h,1p) and (0h,2p) sectors")
    ap.add_argument("--no-mixed", action="store_true", help="skip the split-precision study")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-system batched workload")
    ap.add_argument("--no-real", action="store_true", help="skip the real-arithmetic (real double group) study")
    ap.add_argument("--no-ooc", action="store_true", help="skip the out-of-core VVVV study")
    ap.add_argument("--no-sequential", action="store_true", help="skip the one-by-one baseline of the batch")
    ap.add_argument("--batch-stop-active", type=int, default=BATCH_STOP_ACTIVE,
                    help="the batch hands its last N iterating systems to concurrent contexts of their own")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm start on the batch")
    ap.add_argument("--converge", action="store_true",
                    help="after timing, iterate to convergence and report iterations to |E-E_inf|<1e-8")
    ap.add_argument("--probe-peaks", action="store_true",
                    help="only measure this GPU's MFMA rates (fscc_probe_mfma) and device copy rate; print them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 3 device copies of 1 GiB (calibrates HBM byte counters)")
    ap.add_argument("--profile-ops", metavar="OUT_JSON",
                    help="only run operations of one residual alone (for counter runs); write the op list")
    ap.add_argument("--ops", default="reorders", help="--profile-ops: reorders, gemms, all or op names (a,b,...)")
    ap.add_argument("--sector", type=int, default=0, choices=(0, 1), help="--profile-ops: (0h,0p) or (0h,1p)")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "split_bf16", "split_fp32"),
                    help="--profile-ops: precision of the split-eligible GEMMs")
    ap.add_argument("--tune-file", help="autotune result cache file for --profile-ops")
    ap.add_argument("--traffic-out", help="--summarize-ops: also store the GEMM kernels' HBM bytes per launch here")
    ap.add_argument("--summarize-ops", nargs=5,
                    metavar=("OPS_JSON", "FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="print the per-operation traffic table from the counter runs")
    ap.add_argument("--summarize-ladder-candidates", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="store the HBM bytes per launch of every autotuned pp-ladder tile in --traffic-out")
    args = ap.parse_args()
    if args.summarize_ladder_candidates:
        summarize_ladder_candidates(args)
        return
    if args.summarize_ops:
        summarize_ops(args)
        return
    if args.profile_ops:
        profile_ops(args)
        return
    if args.probe_peaks:
        import torch
        import paper_2004_03682_amd as F
        print(json.dumps(measured_peaks(F, torch)))
        return
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 1 << 30, "copy_bytes_written_per_launch": 1 << 30}))
        return
    if args.gpus != 1:
        print(f"bench.py: the hot path runs on one GPU; --gpus {args.gpus} is not supported "
              "(no multi-GPU sharding is implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import fsgen
    import paper_2004_03682_amd as F

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cfg = fsgen.WORKLOADS["o40v300z16"]
    s = fsgen.workload_system("o40v300z16")
    setup = {}
    t0 = time.perf_counter()
    buffers = {}
    for C in fsgen.CLASSES:
        buffers[C], _ = fsgen.class_buffer(s, C)
    setup["inputs_s"] = round(time.perf_counter() - t0, 2)
    log(f"inputs generated in {setup['inputs_s']:.1f}s")
    t0 = time.perf_counter()
    ctx = F.Context.from_system(s)
    setup["plan_s"] = round(time.perf_counter() - t0, 2)
    log(f"plan + device buffers in {setup['plan_s']:.1f}s; n1={ctx.n1} n2={ctx.n2}")
    t0 = time.perf_counter()
    for C in fsgen.CLASSES:
        d = torch.from_numpy(buffers[C]).to(dev)
        ctx.set_integrals(C, d)
        del d
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    setup["integrals_s"] = round(time.perf_counter() - t0, 2)
    log(f"integral import + pack in {setup['integrals_s']:.1f}s")

    # autotuning: measured once (the cache file starts empty), then read back
    # from the autotune result cache, as a second run on this GPU would
    import tempfile
    tune_file = os.path.join(tempfile.mkdtemp(prefix="fscc_tune_"), "tune.json")
    ctx.tune_cache(tune_file)
    t0 = time.perf_counter()
    ctx.autotune(1)
    setup["autotune_s"] = round(time.perf_counter() - t0, 2)
    t1_ = time.perf_counter()
    ctx.autotune(1)
    setup["autotune_cached_s"] = round(time.perf_counter() - t1_, 3)
    setup["autotune_cache_hit"] = ctx.autotune_cached()
    ctx.tune_cache(None)
    ctx.set_streams(args.streams)
    tuned = {n: tile_str(c, b, sp) for n, c, b, sp in ctx.gemm_configs()}
    log(f"autotuned GEMM tiles in {setup['autotune_s']:.1f}s (from the cache: {setup['autotune_cached_s']:.3f}s): " +
        ", ".join(f"{k}={tuned[k]}" for k in ("pp-ladder", "ring", "W.U", "Z") if k in tuned))

    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device=dev)
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device=dev)
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    ctx.diis_reset(NDIIS)
    E = 0j

    # the solver: Jacobi + DIIS(NDIIS) with dressed denominators (refreshed from the
    # previous residual at iteration 3 and every DRESSED iterations after it)
    nit = [0]

    def step():
        nit[0] += 1
        if nit[0] >= 3 and (nit[0] - 3) % DRESSED == 0:
            ctx.precondition(1, 0.1, F.FSCC_S00)
        return ctx.iterate(t1, t2, r1, r2)

    # warm-up iterations time every operation (HIP events around each one):
    # the per-operation table and the choice of the dominant GEMM
    ctx.profile(True)
    for _ in range(max(1, args.warmup)):
        dmax, E = step()
    ops = ctx.op_times()
    ctx.profile(False)
    nwarm = max(1, args.warmup)
    gemms = [o for o in ops if o["flops"] > 0 and o["calls"] > 0]
    resid_ms = sum(o["ms"] for o in ops) / nwarm
    for o in sorted(ops, key=lambda o: -o["ms"])[:12]:
        per = o["ms"] / max(1, o["calls"])
        tf = o["flops"] / (per * 1e-3) / 1e12 if o["flops"] and per > 0 else 0.0
        log(f"  {o['name']:18s} {per:8.3f} ms/call  {tf:7.2f} TFLOP/s")
    # the roofline kernel: the particle-particle ladder (the pp-ladder, W.U and
    # ring GEMMs take about the same time; the ladder is the one whose
    # algorithmic bytes and flops are fixed by the method)
    dom_name = "pp-ladder"
    gemm_ms = sum(o["ms"] for o in gemms) / nwarm
    # timed region: events only around the dominant GEMM, on the library's stream
    ctx.profile(True, only=dom_name)
    torch.cuda.synchronize()
    st = time.perf_counter()
    hist = []
    for k in range(args.steps):
        dmax, E = step()
        hist.append((dmax, E))
    torch.cuda.synchronize()
    el = time.perf_counter() - st
    dom = next(o for o in ctx.op_times() if o["name"] == dom_name)
    ctx.profile(False)
    work = ctx.work()
    s_per_iter = el / args.steps
    log(f"{args.steps} iterations in {el:.4f}s -> {s_per_iter * 1e3:.3f} ms/iteration; E = {E}")
    per_launch_s = dom["ms"] / dom["calls"] * 1e-3
    achieved = dom["flops"] / per_launch_s / 1e12
    traffic = measured_traffic(dom["name"], tuned.get(dom["name"]))
    dom_3m = "/3M" in tuned.get(dom["name"], "")
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64, 4), "traffic": traffic,
            "kernel": "%s (grouped complex FP64 MFMA GEMM), op '%s'" % (
                "k_zgemm_dl" if "/DL" in tuned.get(dom["name"], "") else "k_zgemm", dom["name"]),
            "flops_per_launch": dom["flops"], "avg_launch_ms": round(per_launch_s * 1e3, 4),
            # achieved counts the algorithmic 8 real flops per complex multiply-add; the
            # three-product form issues 6 of them to the matrix cores
            "complex_form": "3M" if dom_3m else "4M",
            "issued_frac": round(achieved * (0.75 if dom_3m else 1.0) / PEAK_FP64, 4),
            # the HIP events bracket the whole op: with a split-K tile, the GEMM
            # kernel and the split-K reduction pass (rocprofv3 lists them apart);
            # traffic is that of the GEMM kernel
            "tile": tuned.get(dom["name"]),
            "launch_includes_splitk_pass": tuned.get(dom["name"], "").endswith("/splitK")}
    peaks = measured_peaks(F, torch)
    roof["measured_peak"] = peaks["fp64_mfma_tflops"]
    roof["frac_of_measured_peak"] = round(achieved / peaks["fp64_mfma_tflops"], 4)
    log(f"measured peaks: {peaks}; pp-ladder at {roof['frac_of_measured_peak']:.3f} of the probed FP64 rate")
    result = {
        "metric": METRIC, "value": round(s_per_iter, 6), "unit": "s/iteration", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(s_per_iter * 1e3, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FS-RCCSD (0h,0p) CCSD iteration, complex128, nocc=40 nvirt=300, 16 irreps "
                               "(Dirichlet blocks), sigma=0.03, seed 1002 (largest single-GPU configuration)",
                   "nocc": cfg["nocc"], "nvirt": cfg["nvirt"], "nirrep": cfg["nirrep"], "precision": "fp64",
                   "parallelism": "single GPU"},
        "mfma_tflops_residual": round(work["gemm_flops"] / (gemm_ms * 1e-3) / 1e12, 3) if gemm_ms > 0 else None,
        "gemm_flops_per_iteration": work["gemm_flops"],
        "gemm_tiles": tuned,
        "top_gemms": [{"op": o["name"], "ms_per_call": round(o["ms"] / max(1, o["calls"]), 4),
                       "tflops": round(o["flops"] / (o["ms"] / max(1, o["calls"]) * 1e-3) / 1e12, 2)}
                      for o in sorted(gemms, key=lambda o: -o["ms"])[:4]],
        "residual_ms_per_iteration": round(resid_ms, 4),
        "setup": setup,
        "reorders": reorder_table(ops, nwarm),
        "energy_re": E.real, "energy_im": E.imag, "last_max_step": hist[-1][0],
        "roofline": roof,
        "measured_peaks": peaks,
    }
    ora = oracle_fixed_point(s)
    E_ref = E
    if args.converge or not args.no_fs01 or not args.no_mixed:
        # continue to convergence, record |E_k - E_inf| < 1e-8 Eh, E_inf the
        # oracle's converged energy (tests/golden) when stored
        it = args.warmup + args.steps
        es = [h[1] for h in hist]
        while dmax >= 1e-10 and it < 300:
            dmax, E = step()
            it += 1
            es.append(E)
        E_ref = ora["E"] if ora else E
        first = args.warmup + 1
        k8 = next((first + k for k, e in enumerate(es) if all(abs(x - E_ref) < 1e-8 for x in es[k:])), None)
        result["converged_iterations"] = it
        result["iterations_to_1e-8"] = k8
        result["converged_energy"] = [E.real, E.imag]
        if ora:
            d1, d2 = ora["dt"](t1, t2)
            result["vs_oracle"] = {
                "oracle_energy": [ora["E"].real, ora["E"].imag], "oracle_tol": ora["tol"],
                "dE_re": E.real - ora["E"].real, "dE_im": E.imag - ora["E"].imag,
                "max_abs_dt1": d1, "max_abs_dt2_sample": d2, "t2_sample": ora["t2_sample"],
                "iterations_to_1e-10": it, "oracle_iterations_to_1e-10": ora["iters_to_1e10"],
                "iterations_to_1e-8_measured_against": "oracle E"}
            log(f"vs oracle: dE = {E.real - ora['E'].real:.2e} {E.imag - ora['E'].imag:+.2e}i, "
                f"max|dT1| {d1:.2e}, max|dT2| (sample) {d2:.2e}")
    if not args.no_mixed:
        result["precision"] = precision_study(ctx, F, torch, dev, E_ref, (t1, t2), args, log, ora)
    if not args.no_fs01:
        # (0h,1p) sector with the 6 lowest virtual spinors active, on the converged T
        ctx.prepare_sector(t1, t2)
        ctx.precondition(1, 0.1)        # Hbar-diagonal denominators (the bare ones reach ~1e-3 Eh here)
        s1 = torch.zeros(ctx.m1, dtype=torch.complex128, device=dev)
        s2 = torch.zeros(ctx.m2, dtype=torch.complex128, device=dev)
        q1, q2 = torch.empty_like(s1), torch.empty_like(s2)
        ctx.diis_reset(6, F.FSCC_S01)
        n01, d01, status = 0, float("nan"), "converged"
        torch.cuda.synchronize()
        st = time.perf_counter()
        try:
            while n01 < 100:
                ctx.build_residual(s1, s2, q1, q2, F.FSCC_S01)
                d01 = ctx.update_amplitudes(s1, s2, q1, q2, F.FSCC_S01)
                n01 += 1
                if n01 % 20 == 0:
                    log(f"  (0h,1p) iteration {n01}: max|step| = {d01:.3e}")
                if d01 < 1e-10:
                    break
            else:
                status = "not converged in 100 iterations"
        except F.FsccError as e:
            status = f"diverged at iteration {n01 + 1} ({e})"
        torch.cuda.synchronize()
        el01 = time.perf_counter() - st
        fs = {"nact": int(s.nact), "ms_per_iteration": round(el01 / max(1, n01) * 1e3, 4), "iterations": n01,
              "status": status, "last_max_step": d01, "preconditioner": "Hbar diagonal, floor 0.1 Eh"}
        if status == "converged":
            w = F.heff_eig(ctx.heff(s1, s2))
            fs["heff_eigenvalues_re"] = [float(x.real) for x in w]
        log(f"(0h,1p): {status}; {n01} iterations, {fs['ms_per_iteration']:.3f} ms/iteration")
        # the intruder-state remedy: dynamic denominator shifts at decreasing
        # scale, then Pade extrapolation of every state energy to zero shift
        ctx.precondition(0, 0.1)
        S_dyn, n_dyn, scales = -3.0, 3, (1.0, 0.9, 0.8, 0.7, 0.6, 0.5, 0.4)
        s1.zero_()
        s2.zero_()
        torch.cuda.synchronize()
        st = time.perf_counter()
        try:
            xr = F.solve01_extrapolated(ctx, s1, s2, S_dyn, n_dyn, scales=scales, L=2, M=1, tol=1e-10, maxit=200,
                                        ndiis=8)
            torch.cuda.synchronize()
            el = time.perf_counter() - st
            sh = {"S": S_dyn, "n": n_dyn, "scales": list(scales), "pade": [2, 1], "ndiis": 8,
                  "iterations": xr["iters"], "converged": xr["converged"], "seconds": round(el, 4),
                  "ms_per_iteration": round(el / max(1, sum(xr["iters"])) * 1e3, 4),
                  "eigenvalues_re_by_scale": [[float(x.real) for x in e] for e in xr["eig"]]}
            if xr["extrapolated"] is not None:
                sh["extrapolated_re"] = [float(x.real) for x in xr["extrapolated"]]
                sh["extrapolated_im"] = [float(x.imag) for x in xr["extrapolated"]]
                # spread between two approximant orders: a measure of the extrapolation error
                E = np.array(xr["eig"])
                alt = np.array([F.pade(list(scales), E[:, k], 3, 0) for k in range(E.shape[1])])
                sh["max_abs_diff_pade_2_1_vs_3_0"] = float(np.abs(alt - xr["extrapolated"]).max())
            fs["dynamic_shift"] = sh
            log(f"(0h,1p) with dynamic shifts S={S_dyn} n={n_dyn}: iterations {xr['iters']}, "
                f"extrapolated {sh.get('extrapolated_re')}")
        except F.FsccError as e:
            fs["dynamic_shift"] = {"S": S_dyn, "n": n_dyn, "status": f"failed ({e})"}
            log(f"(0h,1p) with dynamic shifts failed: {e}")
        # split-BF16 (0h,1p): the ladder over all virtual pairs on the bf16
        # matrix cores; one shifted solve (S = -3 Eh, n = 3, the largest shift)
        # from zero in each precision, H_eff eigenvalue differences per state
        try:
            sh01 = {}
            ctx.dynamic_shift(S_dyn, n_dyn)
            for prec in ("fp64", "split_bf16"):
                ctx.set_precision(prec)
                if prec != "fp64":
                    ctx.autotune(2)
                u1, u2 = torch.zeros_like(s1), torch.zeros_like(s2)
                torch.cuda.synchronize()
                st = time.perf_counter()
                g01 = F.solve01(ctx, u1, u2, tol=1e-10, maxit=200, ndiis=8)
                torch.cuda.synchronize()
                sh01[prec] = (g01, time.perf_counter() - st)
            ctx.set_precision("fp64")
            ctx.dynamic_shift(0.0, n_dyn)
            g64, t64 = sh01["fp64"]
            gbf, tbf = sh01["split_bf16"]
            deig = np.abs(np.array(gbf["eig"]) - np.array(g64["eig"]))
            fs["split_bf16_sector"] = {
                "shift": [S_dyn, n_dyn], "converged": [bool(g64["converged"]), bool(gbf["converged"])],
                "iterations": [g64["iters"], gbf["iters"]],
                "ms_per_iteration": [round(t64 / g64["iters"] * 1e3, 4), round(tbf / gbf["iters"] * 1e3, 4)],
                "max_abs_delta_eig_heff": float(deig.max()), "delta_eig_heff": [float(x) for x in deig]}
            log(f"(0h,1p) split-BF16 ladder (shifted solve): {gbf['iters']} iterations at "
                f"{tbf / gbf['iters'] * 1e3:.3f} ms vs FP64 {g64['iters']} at {t64 / g64['iters'] * 1e3:.3f} ms; "
                f"max |d eig(H_eff)| = {deig.max():.2e} Eh")
        except F.FsccError as e:
            ctx.set_precision("fp64")
            ctx.dynamic_shift(0.0, n_dyn)
            fs["split_bf16_sector"] = {"status": f"failed ({e})"}
        # per-operation table of the (0h,1p) residual at the last amplitudes
        q1, q2 = torch.empty_like(s1), torch.empty_like(s2)
        fs["residual_ops"] = sector_op_table(ctx, lambda: ctx.build_residual(s1, s2, q1, q2, F.FSCC_S01))
        log(f"(0h,1p) residual {fs['residual_ops']['residual_ms']:.3f} ms: " +
            ", ".join(f"{r['op']} {r['ms_per_call']:.3f}" for r in fs["residual_ops"]["ops"][:8]))
        result["fs01"] = fs
        if s.nact >= 2:
            # (0h,2p) from the last (0h,1p) amplitudes (the smallest-shift solve)
            result["fs02"] = fs02_study(ctx, F, torch, s, s1, s2, log)
    if not args.no_ooc:
        result["out_of_core"] = out_of_core_study(ctx, F, torch, s_per_iter, dom, args, log)
    ctx.destroy()
    del t1, t2, r1, r2
    torch.cuda.empty_cache()
    if not args.no_real:
        cs = {}
        if "fs01" in result and isinstance(result["fs01"].get("dynamic_shift"), dict):
            cs["fs01"] = result["fs01"]["dynamic_shift"].get("ms_per_iteration")
        if "fs02" in result:
            cs["fs02"] = result["fs02"].get("ms_per_iteration")
        result["real_arithmetic"] = real_study(F, torch, fsgen, cfg, s_per_iter, args, log, cs)
    if not args.no_batch:
        result["batch"] = batch_study(F, torch, fsgen, args, log)
    if not args.no_cpu:
        log("timing the CPU oracle on one iteration of the same system ...")
        result["cpu_baseline"] = cpu_baseline(s, buffers)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

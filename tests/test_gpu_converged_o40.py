"""The production-size system (40 occupied / 300 virtual spinors, 16 irreps
with uneven blocks, seed 1002) converged on the GPU in the launch
configuration the benchmark times, against the block-list oracle's converged
fixed point stored in tests/golden/o40v300z16_ccsd.json (written by
tests/golden/make_golden.py from the oracle alone; Jacobi + DIIS(6) to
max|step| < 1e-12):

  * correlation energy, real and imaginary parts, within 1e-10 Eh;
  * every T1 element and a seeded sample of 4096 T2 elements plus the 64
    largest, within 1e-9;
  * the DIIS trajectory: the energy of every iteration within 1e-8 Eh of the
    oracle's (same algorithm: Jacobi step, DIIS(6) on the steps of the unique
    amplitudes; only the rounding order differs) and the iteration count to
    max|step| < 1e-10 within two of the oracle's.

The GPU part takes about half a second of solve time after ~15 s of setup."""
import json
import os
import sys

import numpy as np
import pytest

import fsgen
import layout_ref as LR

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "o40v300z16_ccsd.json")


@pytest.mark.timeout(600)
def test_production_size_converges_to_the_oracle_fixed_point():
    import torch
    import paper_2004_03682_amd as F
    g = json.load(open(GOLDEN))
    s = fsgen.workload_system("o40v300z16")
    assert g["config"]["seed"] == s.seed and g["converged"]
    ctx = F.Context.from_system(s)
    for C in fsgen.CLASSES:
        d = torch.from_numpy(fsgen.class_buffer(s, C)[0]).cuda()
        ctx.set_integrals(C, d)
        del d
    ctx.autotune(1)
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    r = F.solve(ctx, t1, t2, tol=1e-12, maxit=200, ndiis=6)
    assert r["converged"]
    E = r["E"]
    print(f"GPU E = {E.real:.14f} {E.imag:+.3e}i in {r['iters']} iterations; oracle "
          f"{g['E_re']:.14f} {g['E_im']:+.3e}i in {g['iters']}", file=sys.stderr, flush=True)
    assert abs(E.real - g["E_re"]) <= 1e-10 and abs(E.imag - g["E_im"]) <= 1e-10
    h1 = t1.cpu().numpy()
    h2 = t2.cpu().numpy()
    ctx.destroy()
    T1 = np.array(g["t1"])
    p1 = LR.t1_positions(s, [(int(i), int(a)) for i, a in T1[:, :2]])
    assert np.abs(h1[p1] - (T1[:, 2] + 1j * T1[:, 3])).max() <= 1e-9
    T2 = np.array(g["t2_sample"])
    p2, sg2 = LR.t2_positions(s, [tuple(int(x) for x in row[:4]) for row in T2])
    err2 = np.abs(sg2 * h2[p2] - (T2[:, 4] + 1j * T2[:, 5])).max()
    print(f"max|dT1| = {np.abs(h1[p1] - (T1[:, 2] + 1j * T1[:, 3])).max():.2e}, "
          f"max|dT2| (sample of {len(T2)}) = {err2:.2e}", file=sys.stderr, flush=True)
    assert err2 <= 1e-9
    # DIIS trajectory
    hist = g["history"]
    n = min(len(hist), len(r["history"]))
    dE = max(abs(r["history"][k]["E"] - complex(hist[k][1], hist[k][2])) for k in range(n))
    it10 = next(h["iter"] for h in r["history"] if h["dmax"] < 1e-10)
    print(f"trajectory: max |E_gpu(k) - E_oracle(k)| = {dE:.2e} over {n} iterations; "
          f"to 1e-10: GPU {it10}, oracle {g['iters_to_1e10']}", file=sys.stderr, flush=True)
    assert dE <= 1e-8
    assert abs(it10 - g["iters_to_1e10"]) <= 2

"""The plain (0h,1p) iteration of the production-size system (40 occupied /
300 virtual spinors, Z16, the six lowest virtual spinors active) diverges;
the block-list oracle's iteration from its own converged T, with the same
step (Hbar-diagonal denominators floored at 0.1 Eh, DIIS(6)), diverges along
the same trajectory (tests/golden/o40v300z16_fs01_plain.json, written by
tests/golden/make_golden.py from the oracle alone).  The GPU's 40 largest
steps from its converged T follow the oracle's: the divergence is a property
of the equations at this size (an intruder state, Section 2.1), not of the
device path.  The divergence watch does not fire within these 40 steps (the
largest stays below 1e3 times the first)."""
import json
import os
import sys

import numpy as np
import pytest

import fsgen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "o40v300z16_fs01_plain.json")


@pytest.mark.timeout(600)
def test_plain_fs01_iteration_follows_the_oracle_trajectory():
    import torch
    import paper_2004_03682_amd as F
    g = json.load(open(GOLDEN))
    ref = np.array(g["max_step"])
    s = fsgen.workload_system("o40v300z16")
    assert g["config"]["seed"] == s.seed and g["ndiis"] == 6
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
    ctx.prepare_sector(t1, t2)
    ctx.precondition(1, g["floor"])
    s1 = torch.zeros(ctx.m1, dtype=torch.complex128, device="cuda")
    s2 = torch.zeros(ctx.m2, dtype=torch.complex128, device="cuda")
    q1, q2 = torch.empty_like(s1), torch.empty_like(s2)
    ctx.diis_reset(6, F.FSCC_S01)
    got = []
    for k in range(len(ref)):
        ctx.build_residual(s1, s2, q1, q2, F.FSCC_S01)
        got.append(ctx.update_amplitudes(s1, s2, q1, q2, F.FSCC_S01))
    ctx.destroy()
    got = np.array(got)
    rel = np.abs(got - ref) / ref
    for k in range(0, len(ref), 5):
        print(f"iteration {k + 1:2d}: GPU {got[k]:.6e} oracle {ref[k]:.6e} rel {rel[k]:.1e}", file=sys.stderr, flush=True)
    print(f"max relative difference: first 20 {rel[:20].max():.1e}, all {rel.max():.1e}", file=sys.stderr, flush=True)
    assert ref[-1] > 100 * ref[:10].min()          # the oracle's iteration diverges
    assert rel.max() <= 1e-9                       # measured: 7.5e-13

"""Writes tests/golden/*.json from the CPU oracle only (run by hand; committed output).

  python tests/golden/make_golden.py                 # o20v120z8_ccsd.json
  python tests/golden/make_golden.py o40v300z16 [--save-amplitudes PATH.npz]
                                                     # o40v300z16_ccsd.json (about an hour on 8 cores);
                                                     # optionally also every converged block of t1, t2
  python tests/golden/make_golden.py batch40000 K [K ...]
                                                     # batch40000_ccsd.json: systems K of the
                                                     # 64-system batched workload (seeds 40000 + K)
  python tests/golden/make_golden.py fs01-plain PATH.npz
                                                     # o40v300z16_fs01_plain.json from the saved
                                                     # converged amplitudes (a few minutes)

o20v120z8_ccsd.json: converged (0h,0p) CCSD correlation energy of the 20-occupied /
120-virtual / Z8 synthetic system (seed 1001) from the block-list oracle, with
Jacobi + DIIS(6) to max|step| < 1e-10.

o40v300z16_ccsd.json: the production-size system (40 occupied / 300 virtual / Z16,
seed 1002) converged by the block-list oracle with Jacobi + DIIS(6) (the fixed point
of Eq. (3)) to max|step| < 1e-12, so that the stored values are the fixed point itself
and not one more iterate.  Stored: E (re, im), the per-iteration energy and max|step|
trajectory (iteration count to 1e-10 included), every T1 element, and a seeded sample of
unique T2 elements (i<j, a<b, allowed by the Z16 selection rule) plus the 64 largest
|t2|, each as (i, j, a, b, re, im) with spinor positions counted inside the occupied and
virtual spaces.

batch40000_ccsd.json: converged (0h,0p) energies of systems of the batched workload
(fsgen.batch_systems(64, 40000): nocc 10-30, nvirt 60-200, 4-8 irreps, sigma 0.05),
block-list oracle, Jacobi + DIIS(6) to max|step| < 1e-11; keyed by the system's index.

o40v300z16_fs01_plain.json: the (0h,1p) sector of the same system (the six lowest
virtual spinors active) iterated from zero on the oracle's converged T: Jacobi steps
with the Hbar-diagonal denominators (floor 0.1 Eh), DIIS(6), 40 iterations; stored:
max|step| of every iteration.  At this size the plain iteration diverges (an intruder
state: Section 2.1); the trajectory pins the divergence to the method rather than to
any one implementation of it.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fsgen  # noqa: E402
from oracle import ccsd, solver  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def small():
    s = fsgen.workload_system("o20v120z8")
    be = ccsd.Blocked(s)
    t0 = time.time()
    r = solver.solve_ccsd(be, tol=1e-10)
    out = dict(config=fsgen.WORKLOADS["o20v120z8"], E_re=r["E"].real, E_im=r["E"].imag, iters=r["iters"],
               converged=r["converged"], tol=1e-10, mp2=float(ccsd.mp2_energy_closed_form(be).real),
               oracle="oracle.solver.solve_ccsd(oracle.ccsd.Blocked)", seconds=round(time.time() - t0, 1))
    with open(os.path.join(HERE, "o20v120z8_ccsd.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


def _element(be, t, idx):
    """Element of a block-list amplitude at space positions idx = (i, a) or (i, j, a, b)."""
    spaces = "OV" if len(idx) == 2 else "OOVV"
    irr = be.sys.irrep
    no = be.sys.nocc
    key, loc = [], []
    for X, p in zip(spaces, idx):
        g = int(irr[p if X == "O" else no + p])
        key.append(g)
        loc.append(int(np.searchsorted(be.mem[X][g], p)))
    blk = t.blocks.get(tuple(key))
    return 0j if blk is None else complex(blk[tuple(loc)])


def t2_sample(be, t2, count, seed, top):
    """Seeded unique (i<j, a<b) elements allowed by the selection rule, plus the `top` largest."""
    s = be.sys
    no, nv, n = s.nocc, s.nvirt, s.nirrep
    go, gv = s.irrep[:no], s.irrep[no:]
    rng = np.random.default_rng(seed)
    picked = set()
    while len(picked) < count:
        i, j = sorted(rng.choice(no, 2, replace=False))
        a = int(rng.integers(nv))
        # b must carry the irrep that conserves symmetry and differ from a
        gb = (int(go[i]) + int(go[j]) - int(gv[a])) % n
        cand = np.nonzero(gv == gb)[0]
        cand = cand[cand != a]
        if cand.size == 0:
            continue
        b = int(rng.choice(cand))
        picked.add((int(i), int(j), min(a, b), max(a, b)))
    big = []
    for key, blk in t2.blocks.items():
        mo = [be.mem["O"][key[0]], be.mem["O"][key[1]]]
        mv = [be.mem["V"][key[2]], be.mem["V"][key[3]]]
        flat = np.argsort(-np.abs(blk).ravel())[:top]
        for f in flat:
            ii, jj, aa, bb = np.unravel_index(f, blk.shape)
            i, j, a, b = int(mo[0][ii]), int(mo[1][jj]), int(mv[0][aa]), int(mv[1][bb])
            if i < j and a < b:
                big.append((abs(blk[ii, jj, aa, bb]), (i, j, a, b)))
    big.sort(key=lambda x: -x[0])
    for _, e in big[:top]:
        picked.add(e)
    out = []
    for e in sorted(picked):
        v = _element(be, t2, e)
        out.append([*e, v.real, v.imag])
    return out


def production(save=None):
    name = "o40v300z16"
    s = fsgen.workload_system(name)
    t0 = time.time()
    be = ccsd.Blocked(s)
    setup = time.time() - t0
    log = lambda m: print(m, flush=True)  # noqa: E731
    t0 = time.time()
    r = solver.solve_ccsd(be, tol=1e-12, maxit=200, log=log)
    solve = time.time() - t0
    hist = r["history"]
    it10 = next((h["iter"] for h in hist if h["dmax"] < 1e-10), None)
    t1 = []
    for i in range(s.nocc):
        for a in range(s.nvirt):
            if s.irrep[i] == s.irrep[s.nocc + a]:
                v = _element(be, r["t1"], (i, a))
                t1.append([i, a, v.real, v.imag])
    t2 = t2_sample(be, r["t2"], 4096, 7, 64)
    cfg = dict(fsgen.WORKLOADS[name])
    out = dict(config=cfg, E_re=r["E"].real, E_im=r["E"].imag, iters=r["iters"], converged=r["converged"],
               tol=1e-12, iters_to_1e10=it10,
               E_at_1e10=[hist[it10 - 1]["E"].real, hist[it10 - 1]["E"].imag] if it10 else None,
               history=[[h["iter"], h["E"].real, h["E"].imag, h["dmax"]] for h in hist],
               mp2=float(ccsd.mp2_energy_closed_form(be).real),
               t1=t1, t2_sample=t2, t2_sample_seed=7, t2_top=64,
               oracle="oracle.solver.solve_ccsd(oracle.ccsd.Blocked, tol=1e-12)",
               setup_seconds=round(setup, 1), seconds=round(solve, 1))
    with open(os.path.join(HERE, name + "_ccsd.json"), "w") as f:
        json.dump(out, f, indent=0)
    print({k: v for k, v in out.items() if k not in ("t1", "t2_sample", "history")})
    if save:
        arrays = {"t1_" + "_".join(map(str, k)): v for k, v in r["t1"].blocks.items()}
        arrays.update({"t2_" + "_".join(map(str, k)): v for k, v in r["t2"].blocks.items()})
        np.savez(save, **arrays)


def batch_systems(indices):
    path = os.path.join(HERE, "batch40000_ccsd.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    ss = fsgen.batch_systems(64, 40000)
    for k in indices:
        s = ss[k]
        t0 = time.time()
        r = solver.solve_ccsd(ccsd.Blocked(s), tol=1e-11, maxit=300, log=lambda m: print(m, flush=True))
        out[str(k)] = dict(nocc=s.nocc, nvirt=s.nvirt, nirrep=s.nirrep, seed=s.seed, E_re=r["E"].real,
                           E_im=r["E"].imag, iters=r["iters"], converged=r["converged"], tol=1e-11,
                           oracle="oracle.solver.solve_ccsd(oracle.ccsd.Blocked, tol=1e-11)",
                           seconds=round(time.time() - t0, 1))
        print(k, out[str(k)], flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)


def fs01_plain(npz, n=40):
    from oracle import fs01
    from oracle.blocks import BlockTensor
    name = "o40v300z16"
    s = fsgen.workload_system(name)
    z = np.load(npz)
    key = lambda k: tuple(int(x) for x in k.split("_")[1:])  # noqa: E731
    t1 = BlockTensor(2, {key(k): z[k] for k in z.files if k.startswith("t1_")})
    t2 = BlockTensor(4, {key(k): z[k] for k in z.files if k.startswith("t2_")})
    t0 = time.time()
    be = ccsd.Blocked(s)
    fs = fs01.FS01Blocked(be, t1, t2, s.active, precond="dressed", floor=0.1)
    r = fs01.solve_fs01_blocked(fs, tol=1e-10, maxit=n, ndiis=6, log=lambda m: print(m, flush=True))
    out = dict(config=dict(fsgen.WORKLOADS[name]), precond="dressed", floor=0.1, ndiis=6,
               max_step=[float(x) for x in r["history"]],
               oracle="oracle.fs01.solve_fs01_blocked(FS01Blocked(precond='dressed', floor=0.1), ndiis=6)",
               seconds=round(time.time() - t0, 1))
    with open(os.path.join(HERE, name + "_fs01_plain.json"), "w") as f:
        json.dump(out, f, indent=0)
    print({k: v for k, v in out.items() if k != "max_step"})


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "batch40000":
        batch_systems([int(x) for x in sys.argv[2:]])
        sys.exit(0)
    if len(sys.argv) > 2 and sys.argv[1] == "fs01-plain":
        fs01_plain(sys.argv[2])
        sys.exit(0)
    if len(sys.argv) > 1 and sys.argv[1] == "o40v300z16":
        production(sys.argv[3] if len(sys.argv) > 3 and sys.argv[2] == "--save-amplitudes" else None)
    else:
        small()

"""Writes tests/golden/*.json from the CPU oracle only (run by hand; committed output).

  python tests/golden/make_golden.py

o20v120z8_ccsd.json: converged (0h,0p) CCSD correlation energy of the 20-occupied /
120-virtual / Z8 synthetic system (seed 1001) from the block-list oracle, with
Jacobi + DIIS(6) to max|step| < 1e-10.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fsgen  # noqa: E402
from oracle import ccsd, solver  # noqa: E402


def main():
    s = fsgen.workload_system("o20v120z8")
    be = ccsd.Blocked(s)
    t0 = time.time()
    r = solver.solve_ccsd(be, tol=1e-10)
    out = dict(config=fsgen.WORKLOADS["o20v120z8"], E_re=r["E"].real, E_im=r["E"].imag, iters=r["iters"],
               converged=r["converged"], tol=1e-10, mp2=float(ccsd.mp2_energy_closed_form(be).real),
               oracle="oracle.solver.solve_ccsd(oracle.ccsd.Blocked)", seconds=round(time.time() - t0, 1))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "o20v120z8_ccsd.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()

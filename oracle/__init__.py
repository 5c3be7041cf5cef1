"""CPU FP64 oracle for the FS-RCCSD hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import, call or execute anything in this package.  It is a plain, slow,
independent implementation written from the paper and the standard CCSD /
FS-CCSD(0h,1p) and (0h,2p) equations; it shares no code with the HIP library (the only
common dependency is the seeded input generator `fsgen`).

Modules:
  blocks  -- block lists keyed by irreps and the block-pair contraction loop
  ccsd    -- (0h,0p) CCSD residual, energy, MP2 closed form; dense or blocked
  solver  -- Jacobi + DIIS(6) driver
  fock    -- brute-force Fock-space (Jordan-Wigner) reference for tiny systems
  fs01    -- (0h,1p) sector: sigma, H_eff, Bloch residual, Jacobi/DIIS
  fs02    -- (0h,2p) sector on top of the converged (0h,1p) amplitudes
  shift   -- dynamic denominator shifts and Pade extrapolation
"""

"""Pins of the CPU oracle against facts fixed by the mathematics (no GPU).

The paper prints no amplitudes or energies for a worked example, so the
oracle is pinned by:
  * exact symmetries of the generated integrals (antisymmetry, Hermiticity,
    Abelian selection rule) and the generator's own projection definition;
  * the first Jacobi iterate giving the closed-form MP2 energy;
  * the two-electron case, where CCSD is exact and must equal brute-force FCI;
  * a brute-force projection <Phi_mu| exp(-T) H exp(T) |Phi> built from
    Jordan-Wigner matrices, at random amplitudes, for 2..4 electrons
    (every term, sign, conjugate and nonlinearity of the residual);
  * dense versus block-list evaluation (block bookkeeping, zero-size irreps);
  * gauge covariance under spinor phases and relabelling invariance.
"""
import numpy as np
import pytest

import fsgen
from oracle import ccsd, fock, solver
from oracle.blocks import BlockTensor


def rand_t(rng, no, nv, scale=0.1):
    t1 = scale * (rng.normal(size=(no, nv)) + 1j * rng.normal(size=(no, nv)))
    t2 = scale * (rng.normal(size=(no, no, nv, nv)) + 1j * rng.normal(size=(no, no, nv, nv)))
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return t1, t2


# --------------------------------------------------------------------------- P1

@pytest.mark.parametrize("no,nv,ni,seed", [(3, 7, 1, 5), (4, 9, 3, 11), (5, 10, 4, 2)])
def test_generator_exact_symmetries(no, nv, ni, seed):
    s = fsgen.make_system(no, nv, ni, 0.05, seed)
    V = fsgen.full_tensor(s)
    assert np.array_equal(V, -V.transpose(1, 0, 2, 3))
    assert np.array_equal(V, -V.transpose(0, 1, 3, 2))
    assert np.array_equal(V, V.transpose(2, 3, 0, 1).conj())
    g = s.irrep
    forbidden = (g[:, None, None, None] + g[None, :, None, None] - g[None, None, :, None] - g[None, None, None, :]) % ni != 0
    assert np.all(V[forbidden] == 0)
    assert np.count_nonzero(V[~forbidden]) > 0.5 * np.count_nonzero(~forbidden)


def test_generator_projection_definition():
    s = fsgen.make_system(3, 5, 1, 0.05, 77)
    V = fsgen.full_tensor(s)
    X = lambda p, q, r, t: fsgen.xraw(s, p, q, r, t)
    for (p, q, r, t) in [(0, 1, 3, 4), (5, 2, 7, 0), (6, 7, 1, 2), (3, 4, 3, 4)]:
        ref = (X(p, q, r, t) - X(q, p, r, t) - X(p, q, t, r) + X(q, p, t, r)
               + np.conj(X(r, t, p, q) - X(t, r, p, q) - X(r, t, q, p) + X(t, r, q, p))) / 8
        assert abs(V[p, q, r, t] - ref) < 1e-15


def test_generator_statistics():
    # generic element variance sigma^2/8 under the projection reading
    s = fsgen.make_system(4, 20, 1, 0.05, 3)
    v = fsgen.block(s, s.space("V"), s.space("V"), s.space("V"), s.space("V"))
    m = s.nvirt
    idx = np.arange(m)
    generic = (idx[:, None, None, None] != idx[None, :, None, None]) & (idx[None, None, :, None] != idx[None, None, None, :])
    generic &= ~((idx[:, None, None, None] == idx[None, None, :, None]) & (idx[None, :, None, None] == idx[None, None, None, :]))
    generic &= ~((idx[:, None, None, None] == idx[None, None, None, :]) & (idx[None, :, None, None] == idx[None, None, :, None]))
    var = np.mean(np.abs(v[generic]) ** 2)
    assert abs(var / (0.05 ** 2 / 8) - 1) < 0.05


@pytest.mark.parametrize("cls", fsgen.CLASSES)
def test_class_buffer_layout(cls):
    s = fsgen.make_system(4, 8, 3, 0.05, 13)
    V = fsgen.full_tensor(s)
    buf, views = fsgen.class_buffer(s, cls)
    off = 0
    for (key, shp) in fsgen.class_tuples(s, cls):
        sz = int(np.prod(shp))
        blk = buf[off:off + sz].reshape(shp)
        ref = V[np.ix_(*[s.members(cls[k], key[k]) for k in range(4)])]
        assert np.array_equal(blk, ref)
        off += sz
    assert off == buf.size


# --------------------------------------------------------------------------- P2

@pytest.mark.parametrize("spec", ["o8v24", (5, 11, 3, 8)])
def test_first_iteration_is_mp2(spec):
    s = fsgen.workload_system("o8v24") if spec == "o8v24" else fsgen.make_system(*spec[:3], 0.05, spec[3])
    be = ccsd.Blocked(s) if s.nirrep > 1 else ccsd.Dense(s)
    t1, t2 = be.zeros_t1(), be.zeros_t2()
    R1, R2 = ccsd.residual(be, t1, t2)
    s1, s2 = R1 / be.D1, R2 / be.D2
    assert be.absmax(s1) == 0.0
    E = ccsd.energy(be, t1 + s1, t2 + s2)
    E2 = ccsd.mp2_energy_closed_form(be)
    assert abs(E - E2) <= 1e-14 * abs(E2)
    assert abs(E.imag) <= 1e-14 * abs(E2)


# --------------------------------------------------------------------------- P4

@pytest.mark.parametrize("no,nv,ni,seed", [(2, 4, 1, 3), (3, 5, 2, 9), (4, 5, 1, 3), (4, 6, 2, 7)])
def test_residual_matches_bruteforce_projection(no, nv, ni, seed):
    s = fsgen.make_system(no, nv, ni, 0.3, seed)
    fs = fock.FockSpace(s.eps, fsgen.full_tensor(s), no)
    be = ccsd.Dense(s)
    t1, t2 = rand_t(np.random.default_rng(seed), no, nv)
    R1b, R2b, Eb = fock.projected_residual(fs, t1, t2)
    R1, R2 = ccsd.residual(be, t1, t2)
    scale = max(np.abs(R2b).max(), 1.0)
    assert np.abs(R1 - R1b).max() < 1e-12 * scale
    assert np.abs(R2 - R2b).max() < 1e-12 * scale
    assert abs(ccsd.energy(be, t1, t2) - Eb) < 1e-12 * scale


# --------------------------------------------------------------------------- P3

@pytest.mark.parametrize("nv,ni,seed", [(4, 1, 1), (6, 1, 2), (6, 2, 3), (8, 4, 4)])
def test_two_electron_ccsd_equals_fci(nv, ni, seed):
    s = fsgen.make_system(2, nv, ni, 0.2, seed)
    fs = fock.FockSpace(s.eps, fsgen.full_tensor(s), 2)
    be = ccsd.Blocked(s) if ni > 1 else ccsd.Dense(s)
    r = solver.solve_ccsd(be, tol=1e-12)
    assert r["converged"]
    w, U = fock.fci_energies(fs, 2)
    phi = fs.reference(2)
    k = int(np.argmax(np.abs(U.conj().T @ phi)))
    assert abs(r["E"] - (w[k] - fs.E_ref)) < 1e-10


# --------------------------------------------------------------------------- P5

def _blocked_copy(bb, t1d, t2d):
    t1 = BlockTensor.from_dense(t1d, [bb.mem["O"], bb.mem["V"]], list(bb.D1.blocks.keys()))
    t2 = BlockTensor.from_dense(t2d, [bb.mem[X] for X in "OOVV"], list(bb.D2.blocks.keys()))
    return t1, t2


@pytest.mark.parametrize("no,nv,ni,seed", [(6, 14, 4, 21), (5, 12, 6, 4)])
def test_dense_equals_blocked(no, nv, ni, seed):
    s = fsgen.make_system(no, nv, ni, 0.1, seed)
    bd, bb = ccsd.Dense(s), ccsd.Blocked(s)
    # symmetry-allowed random amplitudes
    rng = np.random.default_rng(seed)
    t1d, t2d = rand_t(rng, no, nv, 0.05)
    g = s.irrep
    go, gv = g[:no], g[no:]
    t1d[(go[:, None] - gv[None, :]) % ni != 0] = 0
    t2d[(go[:, None, None, None] + go[None, :, None, None] - gv[None, None, :, None] - gv[None, None, None, :]) % ni != 0] = 0
    t1, t2 = _blocked_copy(bb, t1d, t2d)
    R1b, R2b = ccsd.residual(bb, t1, t2)
    R1, R2 = ccsd.residual(bd, t1d, t2d)
    assert np.abs(bb.dense(R1b) - R1).max() < 1e-12
    assert np.abs(bb.dense(R2b) - R2).max() < 1e-12
    rd, rb = solver.solve_ccsd(bd), solver.solve_ccsd(bb)
    assert rd["converged"] and rb["converged"]
    assert abs(rd["E"] - rb["E"]) < 1e-11


def test_zero_size_irreps_present():
    # the systems above must exercise empty irreps in the occupied and virtual spaces
    s = fsgen.make_system(5, 12, 6, 0.1, 4)
    assert (s.counts("O") == 0).any()


# --------------------------------------------------------------------------- P6 / P7 / P8

def test_gauge_covariance_and_conjugation():
    s = fsgen.make_system(4, 8, 1, 0.1, 31)
    be = ccsd.Dense(s)
    r0 = solver.solve_ccsd(be, tol=1e-12)
    rng = np.random.default_rng(5)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, s.n))
    cls = {}
    for C, x in be.cls.items():
        sp = [s.space(X) for X in C]
        f = (np.conj(ph[sp[0]])[:, None, None, None] * np.conj(ph[sp[1]])[None, :, None, None]
             * ph[sp[2]][None, None, :, None] * ph[sp[3]][None, None, None, :])
        cls[C] = x * f
    r1 = solver.solve_ccsd(ccsd.Dense(s, cls), tol=1e-12)
    assert abs(r1["E"] - r0["E"]) < 1e-12
    po, pv = ph[: s.nocc], ph[s.nocc:]
    fac = (po[:, None, None, None] * po[None, :, None, None]
           * np.conj(pv)[None, None, :, None] * np.conj(pv)[None, None, None, :])
    assert np.abs(r1["t2"] - r0["t2"] * fac).max() < 1e-10
    rc = solver.solve_ccsd(ccsd.Dense(s, {C: x.conj() for C, x in be.cls.items()}), tol=1e-12)
    assert abs(rc["E"] - np.conj(r0["E"])) < 1e-12
    assert abs(r0["E"].imag) > 1e-8      # the energy of a generic complex system is not real


def test_relabelling_invariance():
    s = fsgen.make_system(4, 9, 1, 0.1, 17)
    be = ccsd.Dense(s)
    E0 = solver.solve_ccsd(be, tol=1e-12)["E"]
    rng = np.random.default_rng(2)
    po, pv = rng.permutation(s.nocc), rng.permutation(s.nvirt)
    perm = {"O": po, "V": pv}
    cls = {C: x[np.ix_(*[perm[X] for X in C])] for C, x in be.cls.items()}
    s2 = fsgen.make_system(4, 9, 1, 0.1, 17)
    s2.eps = np.concatenate([s.eps[: s.nocc][po], s.eps[s.nocc:][pv]])
    E1 = solver.solve_ccsd(ccsd.Dense(s2, cls), tol=1e-12)["E"]
    assert abs(E1 - E0) < 1e-12


def test_irrep_automorphism_invariance():
    s = fsgen.make_system(5, 12, 5, 0.1, 23)
    E0 = solver.solve_ccsd(ccsd.Blocked(s), tol=1e-11)["E"]
    s2 = fsgen.make_system(5, 12, 5, 0.1, 23)
    s2.irrep = (2 * s.irrep) % 5          # g -> 2g is an automorphism of Z5
    E1 = solver.solve_ccsd(ccsd.Blocked(s2), tol=1e-11)["E"]
    assert abs(E1 - E0) < 1e-11


def test_fixed_point_independent_of_diis():
    s = fsgen.workload_system("o8v24")
    be = ccsd.Dense(s)
    a = solver.solve_ccsd(be, tol=1e-12, ndiis=6)
    b = solver.solve_ccsd(be, tol=1e-12, ndiis=0, maxit=400)
    assert a["converged"] and b["converged"]
    assert abs(a["E"] - b["E"]) < 1e-11
    assert np.abs(a["t2"] - b["t2"]).max() < 1e-10


# --------------------------------------------------------------------------- P11

@pytest.mark.parametrize("no,nv,ni,seed", [(4, 10, 1, 5), (6, 14, 3, 2)])
def test_ladder_mp3_closed_form(no, nv, ni, seed):
    # the ladder applied to first-order amplitudes gives the textbook MP3 pp-ladder energy, which is real
    s = fsgen.make_system(no, nv, ni, 0.1, seed)
    be = ccsd.Dense(s)
    y = be.V("oovv").conj() / be.D2
    L = ccsd.pp_ladder(be, y)
    e = 0.25 * np.sum(be.V("oovv") * L / be.D2)
    ref = ccsd.mp3_ladder_closed_form(be)
    assert abs(e - ref) < 1e-13 * abs(ref)
    assert abs(ref.imag) < 1e-13 * abs(ref)

"""CPU FP64 oracle for the (0h,0p) sector: spin-orbital CCSD, complex128.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this package.  It shares no code with the HIP
library; the only common dependency is the seeded input generator `fsgen`.

What it computes (paper: Eq. (1) Hamiltonian, Eq. (2) Omega = {exp T}
truncated to singles and doubles, Eq. (3)-(4) amplitude equations with
D = negative H0-eigenvalue differences; the paper gives no explicit working
equations and points to the Goldstone-diagram literature): the standard
spin-orbital CCSD equations in the Stanton-Gauss intermediate form, written
for complex integrals.  Every integral is written <creators||annihilators>
relative to the operator string it multiplies; with a diagonal Fock matrix
f = diag(eps), f_ov = 0, so the f_ov terms vanish.  The driver term of the
T2 equation is <ab||ij> = conj <ij||ab>.

  R = <Phi_mu| exp(-T) H_N exp(T) |Phi>  =  RHS_mu - D_mu t_mu
  D_i^a = e_i - e_a ,   D_ij^ab = e_i + e_j - e_a - e_b

The signs and the placement of every conjugate are not taken on trust: the
tests compare this residual with a brute-force projection of
exp(-T) H exp(T) built from Jordan-Wigner matrices (oracle.fock).

Intermediates (materialised, W_abef included):
  tau~ = t2 + 1/2 (t_i^a t_j^b - t_i^b t_j^a),  tau = t2 + t_i^a t_j^b - t_i^b t_j^a
  F_ae = sum_mf t_m^f <ma||fe> - 1/2 sum_mnf tau~_mn^af <mn||ef>
  F_mi = sum_ne t_n^e <mn||ie> + 1/2 sum_nef tau~_in^ef <mn||ef>
  F_me = sum_nf t_n^f <mn||ef>
  W_mnij = <mn||ij> + P(ij) sum_e t_j^e <mn||ie> + 1/4 sum_ef tau_ij^ef <mn||ef>
  W_abef = <ab||ef> - P(ab) sum_m t_m^b <am||ef> + 1/4 sum_mn tau_mn^ab <mn||ef>
  W_mbej = <mb||ej> + sum_f t_j^f <mb||ef> - sum_n t_n^b <mn||ej>
           - sum_nf (1/2 t_jn^fb + t_j^f t_n^b) <mn||ef>
"""
from __future__ import annotations

import numpy as np

import fsgen
from .blocks import BlockTensor, bein, ttgt

CLASSES = ("OOOO", "OOOV", "OOVV", "OVOV", "OVVV", "VVVV")


# ---------------------------------------------------------------------------
# symmetry images of <pq||rs>: antisymmetry in (pq), in (rs), and Hermiticity

def _symmetry_group():
    gens = [((1, 0, 2, 3), -1, False), ((0, 1, 3, 2), -1, False), ((2, 3, 0, 1), 1, True)]
    seen = {(0, 1, 2, 3): (1, False)}
    frontier = [((0, 1, 2, 3), 1, False)]
    while frontier:
        nxt = []
        for p1, s1, c1 in frontier:
            for p2, s2, c2 in gens:
                p = tuple(p1[p2[k]] for k in range(4))
                if p not in seen:
                    seen[p] = (s1 * s2, c1 ^ c2)
                    nxt.append((p, s1 * s2, c1 ^ c2))
        frontier = nxt
    return [(p, s, c) for p, (s, c) in seen.items()]


_GROUP = _symmetry_group()


def integral_image(pattern: str):
    """(class, axes, sign, conj) with V_pattern = sign * conj^c(V_class).transpose(axes)."""
    P = pattern.upper()
    for pi, s, c in _GROUP:
        img = "".join(P[pi[k]] for k in range(4))
        if img in CLASSES:
            return img, tuple(int(x) for x in np.argsort(pi)), s, c
    raise KeyError(pattern)


# ---------------------------------------------------------------------------
# backends: dense arrays or block lists

class Dense:
    """Full (unblocked) tensors; integral classes as dense arrays."""

    def __init__(self, sysm: fsgen.System, classes: dict | None = None):
        self.sys = sysm
        if classes is None:
            classes = {C: fsgen.block(sysm, sysm.space(C[0]), sysm.space(C[1]), sysm.space(C[2]), sysm.space(C[3]))
                       for C in CLASSES}
        self.cls = classes
        no = sysm.nocc
        eo, ev = sysm.eps[:no], sysm.eps[no:]
        self.D1 = eo[:, None] - ev[None, :]
        self.D2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
        self._cache = {}

    def ein(self, spec, a, b):
        return ttgt(spec, a, b)

    def V(self, pattern: str):
        if pattern not in self._cache:
            C, axes, s, c = integral_image(pattern)
            x = self.cls[C]
            x = x.conj() if c else x
            self._cache[pattern] = np.ascontiguousarray(s * x.transpose(axes))
        return self._cache[pattern]

    def zeros_t1(self):
        return np.zeros_like(self.D1, dtype=np.complex128)

    def zeros_t2(self):
        return np.zeros_like(self.D2, dtype=np.complex128)

    @staticmethod
    def dot(a, b):
        return complex(np.sum(a * b))

    @staticmethod
    def vdot(a, b):
        return complex(np.vdot(a.ravel(), b.ravel()))

    @staticmethod
    def absmax(a):
        return float(np.abs(a).max()) if a.size else 0.0

    @staticmethod
    def lincomb(coefs, xs):
        r = coefs[0] * xs[0]
        for c, x in zip(coefs[1:], xs[1:]):
            r = r + c * x
        return r

    def dense(self, x):
        return x

    def fock_diag(self, X):
        """The diagonal Fock matrix diag(eps) of space 'O' or 'V'."""
        no = self.sys.nocc
        return np.diag(self.sys.eps[:no] if X == "O" else self.sys.eps[no:])


def _views(sysm, C, buf):
    """Block views of an already generated class buffer (boundary layout)."""
    views, off = {}, 0
    for key, shp in fsgen.class_tuples(sysm, C):
        sz = int(np.prod(shp))
        views[key] = buf[off:off + sz].reshape(shp)
        off += sz
    assert off == buf.size
    return buf, views


class Blocked:
    """Block lists keyed by irreps (Fig. 3 partition, Fig. 4 contraction)."""

    def __init__(self, sysm: fsgen.System, buffers: dict | None = None):
        self.sys = sysm
        self.cls = {}
        for C in CLASSES:
            out = None if buffers is None else buffers[C]
            _, views = fsgen.class_buffer(sysm, C, out=out) if out is None else _views(sysm, C, out)
            self.cls[C] = BlockTensor(4, {k: v for k, v in views.items() if v.size})
        n = sysm.nirrep
        no = sysm.nocc
        # positions (within their space) of the members of each irrep
        self.mem = {X: [sysm.members(X, g) - (0 if X == "O" else no) for g in range(n)] for X in "OV"}
        eo, ev = sysm.eps[:no], sysm.eps[no:]
        d1 = {}
        for g in range(n):
            a, b = eo[self.mem["O"][g]], ev[self.mem["V"][g]]
            if a.size and b.size:
                d1[(g, g)] = a[:, None] - b[None, :]
        self.D1 = BlockTensor(2, d1)
        d2 = {}
        for gi in range(n):
            for gj in range(n):
                for ga in range(n):
                    gb = (gi + gj - ga) % n
                    ei, ej = eo[self.mem["O"][gi]], eo[self.mem["O"][gj]]
                    ea, eb = ev[self.mem["V"][ga]], ev[self.mem["V"][gb]]
                    if ei.size and ej.size and ea.size and eb.size:
                        d2[(gi, gj, ga, gb)] = (ei[:, None, None, None] + ej[None, :, None, None]
                                                - ea[None, None, :, None] - eb[None, None, None, :])
        self.D2 = BlockTensor(4, d2)
        self._cache = {}

    def ein(self, spec, a, b):
        return bein(spec, a, b)

    def V(self, pattern: str):
        if pattern not in self._cache:
            C, axes, s, c = integral_image(pattern)
            x = self.cls[C]
            if axes == (0, 1, 2, 3) and s == 1 and not c:
                self._cache[pattern] = x        # the stored class itself (no copy)
                return x
            x = x.conj() if c else x
            x = x.transpose(axes)
            self._cache[pattern] = BlockTensor(4, {k: np.ascontiguousarray(s * v) for k, v in x.blocks.items()})
        return self._cache[pattern]

    def zeros_t1(self):
        return BlockTensor(2, {k: np.zeros(v.shape, np.complex128) for k, v in self.D1.blocks.items()})

    def zeros_t2(self):
        return BlockTensor(4, {k: np.zeros(v.shape, np.complex128) for k, v in self.D2.blocks.items()})

    @staticmethod
    def dot(a, b):
        return a.dot(b)

    @staticmethod
    def vdot(a, b):
        return a.vdot(b)

    @staticmethod
    def absmax(a):
        return a.absmax()

    @staticmethod
    def lincomb(coefs, xs):
        r = xs[0] * coefs[0]
        for c, x in zip(coefs[1:], xs[1:]):
            r = r + x * c
        return r

    def fock_diag(self, X):
        """diag(eps) of space 'O' or 'V' as one diagonal block per irrep."""
        no = self.sys.nocc
        e = self.sys.eps[:no] if X == "O" else self.sys.eps[no:]
        return BlockTensor(2, {(g, g): np.diag(e[m]) for g, m in enumerate(self.mem[X]) if m.size})

    def dense(self, x):
        no, nv = self.sys.nocc, self.sys.nvirt
        spaces = "OV" if x.rank == 2 else "OOVV"
        shape = tuple(no if X == "O" else nv for X in spaces)
        return x.to_dense([self.mem[X] for X in spaces], shape)


# ---------------------------------------------------------------------------
# the CCSD residual

def _P(x, a, b):
    """Antisymmetriser P(pq) X = X - X(p<->q) acting on axes a, b."""
    ax = list(range(4))
    ax[a], ax[b] = ax[b], ax[a]
    return x - x.transpose(ax)


def intermediates(be, t1, t2, progress=None, one_body_only=False):
    """The intermediates listed in the module docstring; one_body_only=True stops
    after tau, tau~ and the three F intermediates."""
    ein, V = be.ein, be.V
    say = progress or (lambda msg: None)
    t1t1 = ein("ia,jb->ijab", t1, t1)
    tau_t = t2 + 0.5 * (t1t1 - t1t1.transpose(0, 1, 3, 2))
    tau = t2 + (t1t1 - t1t1.transpose(0, 1, 3, 2))
    Fae = ein("mf,mafe->ae", t1, V("ovvv")) - 0.5 * ein("mnaf,mnef->ae", tau_t, V("oovv"))
    Fmi = ein("ne,mnie->mi", t1, V("ooov")) + 0.5 * ein("inef,mnef->mi", tau_t, V("oovv"))
    Fme = ein("nf,mnef->me", t1, V("oovv"))
    say("F intermediates")
    if one_body_only:
        return dict(tau=tau, tau_t=tau_t, Fae=Fae, Fmi=Fmi, Fme=Fme)
    Wmnij = (V("oooo") + _P(ein("je,mnie->mnij", t1, V("ooov")), 2, 3)
             + 0.25 * ein("ijef,mnef->mnij", tau, V("oovv")))
    Wabef = (V("vvvv") - _P(ein("mb,amef->abef", t1, V("vovv")), 0, 1)
             + 0.25 * ein("mnab,mnef->abef", tau, V("oovv")))
    say("W_abef")
    u = 0.5 * t2 + ein("jf,nb->jnfb", t1, t1)
    Wmbej = (V("ovvo") + ein("jf,mbef->mbej", t1, V("ovvv")) - ein("nb,mnej->mbej", t1, V("oovo"))
             - ein("jnfb,mnef->mbej", u, V("oovv")))
    return dict(tau=tau, tau_t=tau_t, Fae=Fae, Fmi=Fmi, Fme=Fme, Wmnij=Wmnij, Wabef=Wabef, Wmbej=Wmbej)


def residual(be, t1, t2, progress=None):
    """(R1, R2) = RHS - D*t for the spin-orbital CCSD equations."""
    ein, V = be.ein, be.V
    say = progress or (lambda msg: None)
    I = intermediates(be, t1, t2, progress)
    tau, Fae, Fmi, Fme, Wmnij, Wabef, Wmbej = (I[k] for k in ("tau", "Fae", "Fmi", "Fme", "Wmnij", "Wabef", "Wmbej"))
    # T1 equation
    R1 = (ein("ie,ae->ia", t1, Fae) - ein("ma,mi->ia", t1, Fmi) + ein("imae,me->ia", t2, Fme)
          - ein("nf,naif->ia", t1, V("ovov")) - 0.5 * ein("imef,maef->ia", t2, V("ovvv"))
          - 0.5 * ein("mnae,nmei->ia", t2, V("oovo")))
    R1 = R1 - be.D1 * t1
    say("T1 residual")
    # T2 equation
    Fbe = Fae - 0.5 * ein("mb,me->be", t1, Fme)
    Fmj = Fmi + 0.5 * ein("je,me->mj", t1, Fme)
    ring = ein("imae,mbej->ijab", t2, Wmbej)
    q = ein("ie,mbej->imbj", t1, V("ovvo"))
    ring = ring - ein("ma,imbj->ijab", t1, q)
    R2 = (V("vvoo").transpose(2, 3, 0, 1)
          + _P(ein("ijae,be->ijab", t2, Fbe), 2, 3)
          - _P(ein("imab,mj->ijab", t2, Fmj), 0, 1)
          + 0.5 * ein("mnab,mnij->ijab", tau, Wmnij)
          + 0.5 * ein("ijef,abef->ijab", tau, Wabef)
          + _P(_P(ring, 0, 1), 2, 3)
          + _P(ein("ie,abej->ijab", t1, V("vvvo")), 0, 1)
          - _P(ein("ma,mbij->ijab", t1, V("ovoo")), 2, 3))
    R2 = R2 - be.D2 * t2
    say("T2 residual")
    return R1, R2


def energy(be, t1, t2) -> complex:
    """E = sum f_ia t_i^a + 1/4 sum <ij||ab> t_ij^ab + 1/2 sum <ij||ab> t_i^a t_j^b  (f_ia = 0)."""
    t1t1 = be.ein("ia,jb->ijab", t1, t1)
    return 0.25 * be.dot(be.V("oovv"), t2) + 0.5 * be.dot(be.V("oovv"), t1t1)


def mp2_energy_closed_form(be) -> complex:
    """E_MP2 = 1/4 sum |<ij||ab>|^2 / D_ij^ab (written independently of the residual)."""
    v = be.V("oovv")
    if isinstance(v, BlockTensor):
        return 0.25 * sum(np.sum(np.abs(x) ** 2 / be.D2.blocks[k]) for k, x in v.blocks.items())
    return 0.25 * np.sum(np.abs(v) ** 2 / be.D2)


def pp_ladder(be, tau):
    """Particle-particle ladder L_ij^ab = 1/2 sum_cd <ab||cd> tau_ij^cd (the bare-integral part of
    the 1/2 sum_ef tau_ij^ef W_abef term)."""
    return 0.5 * be.ein("ijcd,abcd->ijab", tau, be.V("vvvv"))


def mp3_ladder_closed_form(be) -> complex:
    """Textbook third-order pp-ladder energy 1/8 sum <ij||ab><ab||cd><cd||ij> / (D_ij^ab D_ij^cd),
    summed directly over all (unpacked) indices with one einsum per (ij) pair set (dense only)."""
    oovv, vvvv, D = be.V("oovv"), be.V("vvvv"), be.D2
    y = oovv.conj() / D                      # y_ij^cd = <cd||ij> / D_ij^cd
    x = oovv / D                             # <ij||ab> / D_ij^ab
    return 0.125 * np.einsum("ijab,abcd,ijcd->", x, vvvv, y, optimize=True)

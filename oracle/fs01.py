"""CPU FP64 oracle for the (0h,1p) Fock-space sector (test infrastructure).

Paper: sector partition of Eq. (5) -- the (0h,1p) amplitudes are solved after
(and with) the converged (0h,0p) T; the amplitude equations of Eq. (3) with
the closed (model-space) part Omega (V Omega)_Cl, and H_eff = (H Omega)_Cl
whose eigenvalues are the state energies.  For one valence particle the
normal-ordered wave operator is Omega^(0,1) = 1 + S1 + S2 and the equations are
the Bloch equation on the one-particle / two-particle-one-hole space:

  for every active x:  r(x) = e_x + s_x  (1p part: r^e = delta_ex for e in A,
                                           s_x^e for e not in A; 2p1h part
                                           r_j^ef = s_xj^ef)
  sigma(x) = Hbar_N r(x)   with Hbar = exp(-T) H exp(T) - E_CC (connected)
  H_eff[y, x] = sigma(x)^y                              (y in A)
  R1[x, a]    = sigma(x)^a   - sum_y s_y^a   H_eff[y, x]  (a not in A)
  R2[x,j,a,b] = sigma(x)_j^ab - sum_y s_yj^ab H_eff[y, x]

sigma is written with the one- and two-body Hbar elements (the standard
electron-attachment EOM-CCSD sigma equations, complex-correct placement of
every integral as <creators||annihilators>); signs and conjugates are pinned
by comparing sigma with a brute-force <mu| exp(-T) H exp(T) - E |nu> matrix
(oracle.fock.ea_matrix).  Update: s += R / D with D_x^a = e_x - e_a,
D_xj^ab = e_x + e_j - e_a - e_b (Eq. (3)-(4) denominators of the sector);
with dynamic shifts (oracle.shift) s += (R - Delta s) / (D + Delta).
FS01 / solve_fs01 run on the dense backend (x is a leading index over the
active set); FS01Blocked / solve_fs01_blocked run the same equations on block
lists (the Fig. 3 partition, every contraction a Fig. 4 block-pair loop), with
x a fourth index space whose members carry the irreps of the active spinors.
"""
from __future__ import annotations

import numpy as np

from . import ccsd
from .blocks import BlockTensor, bein, ttgt


def _P(x, a, b):
    """Antisymmetriser P(pq) X = X - X(p<->q) on axes a, b (dense array or block list)."""
    ax = list(range(x.rank if isinstance(x, BlockTensor) else x.ndim))
    ax[a], ax[b] = ax[b], ax[a]
    return x - x.transpose(ax)


def hbar(be, t1, t2):
    """One- and two-body Hbar elements needed by the (0h,1p) sigma equations."""
    ein, V = be.ein, be.V
    I = ccsd.intermediates(be, t1, t2, one_body_only=True)
    tau, Fme = I["tau"], I["Fme"]
    Fae = I["Fae"] + be.fock_diag("V") - 0.5 * ein("ma,me->ae", t1, Fme)
    Fmi = I["Fmi"] + be.fock_diag("O") + 0.5 * ein("ie,me->mi", t1, Fme)
    Wamef = V("vovv") - ein("na,nmef->amef", t1, V("oovv"))
    Wabef = V("vvvv") - _P(ein("mb,amef->abef", t1, V("vovv")), 0, 1) + 0.5 * ein("mnab,mnef->abef", tau, V("oovv"))
    Wmbej = (V("ovvo") + ein("jf,mbef->mbej", t1, V("ovvv")) - ein("nb,mnej->mbej", t1, V("oovo"))
             - ein("jnfb,mnef->mbej", t2 + ein("jf,nb->jnfb", t1, t1), V("oovv")))
    # W_abej
    x = V("ovvo") - ein("njbf,mnef->mbej", t2, V("oovv"))          # <mb||ej> - sum_nf t_nj^bf <mn||ef>
    Wabej = (V("vvvo") - ein("me,mjab->abej", Fme, t2) + ein("jf,abef->abej", t1, Wabef)
             + 0.5 * ein("mnej,mnab->abej", V("oovo"), tau)
             - _P(ein("mbef,mjaf->abej", V("ovvv"), t2), 0, 1)
             - _P(ein("ma,mbej->abej", t1, x), 0, 1))
    return dict(Fae=Fae, Fmi=Fmi, Fme=Fme, Wamef=Wamef, Wabef=Wabef, Wmbej=Wmbej, Wabej=Wabej,
                Woovv=V("oovv"), t2=t2)


def sigma(be, hb, r1, r2):
    """sigma = Hbar_N r for a batch of electron-attachment vectors.
    r1[x, e] (all virtual e), r2[x, m, e, f] antisymmetric in (e, f)."""
    ein = be.ein
    s1 = (ein("ae,xe->xa", hb["Fae"], r1) + ein("me,xmae->xa", hb["Fme"], r2)
          + 0.5 * ein("amef,xmef->xa", hb["Wamef"], r2))
    s2 = ein("abej,xe->xjab", hb["Wabej"], r1)
    s2 = s2 + _P(ein("be,xjae->xjab", hb["Fae"], r2), 2, 3)
    s2 = s2 - ein("mj,xmab->xjab", hb["Fmi"], r2)
    s2 = s2 + 0.5 * ein("abef,xjef->xjab", hb["Wabef"], r2)
    s2 = s2 + _P(ein("mbej,xmae->xjab", hb["Wmbej"], r2), 2, 3)
    q = ein("mnef,xnef->xm", hb["Woovv"], r2)
    s2 = s2 - 0.5 * ein("xm,mjab->xjab", q, hb["t2"])
    return s1, s2


class FS01:
    """(0h,1p) sector at fixed converged T: residual, update, H_eff."""

    def __init__(self, be, t1, t2, active, precond="bare", floor=0.1, shift=None):
        """precond: 'bare' -> D from orbital energies (Eq. (3)); 'dressed' -> D from the
        diagonal of Hbar (Fbar_xx + Fbar_jj - Fbar_aa - Fbar_bb, real part), clamped to
        <= -floor.  Only the step changes; the fixed point R = 0 does not.
        shift = (S, n): dynamic denominator shifts (oracle.shift) evaluated on
        the denominators in use; the solved equations become R = Delta s."""
        self.be = be
        self.hb = hbar(be, t1, t2)
        sys_ = be.sys
        self.no, self.nv = sys_.nocc, sys_.nvirt
        self.act = np.asarray(active) - sys_.nocc          # positions within the virtual space
        self.nact = len(self.act)
        self.inact = np.setdiff1d(np.arange(self.nv), self.act)
        eo, ev = sys_.eps[: self.no], sys_.eps[self.no:]
        ex = ev[self.act]
        self.D1 = ex[:, None] - ev[None, :]
        self.D2 = ex[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
        if precond == "dressed":
            fv = np.real(np.diag(self.hb["Fae"]))
            fo = np.real(np.diag(self.hb["Fmi"]))
            fx = fv[self.act]
            self.D1 = np.minimum(fx[:, None] - fv[None, :], -floor)
            self.D2 = np.minimum(fx[:, None, None, None] + fo[None, :, None, None] - fv[None, None, :, None]
                                 - fv[None, None, None, :], -floor)
        elif precond != "bare":
            raise ValueError(precond)
        self.Delta1 = np.zeros_like(self.D1)
        self.Delta2 = np.zeros_like(self.D2)
        if shift is not None:
            from .shift import delta
            self.Delta1 = delta(self.D1, shift[0], shift[1])
            self.Delta2 = delta(self.D2, shift[0], shift[1])
        g = sys_.irrep
        go, gv = g[: self.no], g[self.no:]
        gx = gv[self.act]
        n = sys_.nirrep
        self.mask1 = ((gx[:, None] - gv[None, :]) % n == 0)
        self.mask1[:, self.act] = False                     # model-space components are not amplitudes
        self.mask2 = ((gx[:, None, None, None] + go[None, :, None, None] - gv[None, None, :, None]
                       - gv[None, None, None, :]) % n == 0)

    def zeros(self):
        return (np.zeros((self.nact, self.nv), np.complex128),
                np.zeros((self.nact, self.no, self.nv, self.nv), np.complex128))

    def rvec(self, s1, s2):
        """r(x) = e_x + s_x: identity on the model space, s elsewhere."""
        r1 = s1.copy()
        r1[:, self.act] = np.eye(self.nact)
        return r1, s2

    def residual(self, s1, s2):
        """(R1, R2, H_eff): Bloch-equation residual for S1 (a not in A) and S2."""
        r1, r2 = self.rvec(s1, s2)
        sg1, sg2 = sigma(self.be, self.hb, r1, r2)
        heff = sg1[:, self.act].T                            # heff[y, x] = sigma(x)^y
        R1 = sg1 - ttgt("ya,yx->xa", s1, heff)
        R2 = sg2 - ttgt("yjab,yx->xjab", s2, heff)
        R1 = np.where(self.mask1, R1, 0.0)
        R2 = np.where(self.mask2, R2, 0.0)
        return R1, R2, heff


def solve_fs01(fs, tol=1e-10, maxit=200, ndiis=6, log=None, start=None):
    """Jacobi + DIIS on (S1, S2) (shifted equations if fs has shifts); start =
    (s1, s2) or zeros.  Returns dict(s1, s2, heff, eig, iters, converged)."""
    from .solver import diis_coefficients
    s1, s2 = fs.zeros() if start is None else (start[0].copy(), start[1].copy())
    hist_t, hist_e = [], []
    converged = False
    heff = None
    k = 0
    for k in range(1, maxit + 1):
        R1, R2, heff = fs.residual(s1, s2)
        # shifted equations: R - Delta s = 0, step (R - Delta s) / (D + Delta)
        R1 = R1 - fs.Delta1 * s1
        R2 = R2 - fs.Delta2 * s2
        e1 = np.where(fs.mask1, R1 / np.where(fs.mask1, fs.D1 + fs.Delta1, 1.0), 0.0)
        e2 = np.where(fs.mask2, R2 / (fs.D2 + fs.Delta2), 0.0)
        n1, n2 = s1 + e1, s2 + e2
        dmax = max(float(np.abs(e1).max()), float(np.abs(e2).max()) if e2.size else 0.0)
        if ndiis > 1:
            hist_t.append((n1, n2))
            hist_e.append((e1, e2))
            if len(hist_t) > ndiis:
                hist_t.pop(0)
                hist_e.pop(0)
            while len(hist_t) >= 2:
                m = len(hist_e)
                B = np.zeros((m, m))
                for a in range(m):
                    for b in range(m):
                        B[a, b] = (np.vdot(hist_e[a][0], hist_e[b][0]) + 0.5 * np.vdot(hist_e[a][1], hist_e[b][1])).real
                try:
                    c = diis_coefficients(B)
                except np.linalg.LinAlgError:
                    hist_t.pop(0)
                    hist_e.pop(0)
                    continue
                n1 = sum(ci * x[0] for ci, x in zip(c, hist_t))
                n2 = sum(ci * x[1] for ci, x in zip(c, hist_t))
                break
        s1, s2 = n1, n2
        if log:
            log(f"fs01 iter {k:3d}  max|step| = {dmax:.3e}")
        if dmax < tol:
            converged = True
            break
    R1, R2, heff = fs.residual(s1, s2)
    eig = np.linalg.eigvals(heff)
    eig = eig[np.lexsort((eig.imag, eig.real))]
    return dict(s1=s1, s2=s2, heff=heff, eig=eig, iters=k, converged=converged)


# ---------------------------------------------------------------------------
# block-list form (same equations; for systems whose dense Wbar_abef does not fit)

class FS01Blocked:
    """(0h,1p) sector on the block-list backend (be = ccsd.Blocked).

    s1 blocks are keyed (g_x, g_a) with g_x = g_a, s2 blocks (g_x, g_j, g_a, g_b)
    with g_x + g_j = g_a + g_b (mod n); rows x are positions in `active`
    (members of irrep g: self.memA[g]).  Model-space components of s1 (a in A)
    are kept as zeros, as in the dense form."""

    def __init__(self, be, t1, t2, active, precond="bare", floor=0.1, shift=None):
        self.be = be
        self.hb = hbar(be, t1, t2)
        sys_ = be.sys
        n = self.n = sys_.nirrep
        self.no, self.nv = sys_.nocc, sys_.nvirt
        active = np.asarray(active)
        self.act = active - sys_.nocc
        self.nact = len(self.act)
        gA = sys_.irrep[active]
        self.memA = [np.nonzero(gA == g)[0] for g in range(n)]
        mO, mV, mA = be.mem["O"], be.mem["V"], self.memA
        eo, ev = sys_.eps[: self.no], sys_.eps[self.no:]
        if precond == "dressed":
            fv = np.real(self._diag(self.hb["Fae"], mV, self.nv))
            fo = np.real(self._diag(self.hb["Fmi"], mO, self.no))
        elif precond == "bare":
            fv, fo = ev, eo
        else:
            raise ValueError(precond)
        fx = fv[self.act]
        self.keys1 = [(g, g) for g in range(n) if mA[g].size and mV[g].size]
        self.keys2 = [(gx, gj, ga, (gx + gj - ga) % n) for gx in range(n) for gj in range(n) for ga in range(n)
                      if mA[gx].size and mO[gj].size and mV[ga].size and mV[(gx + gj - ga) % n].size]
        d1, d2, m1 = {}, {}, {}
        for k in self.keys1:
            d1[k] = fx[mA[k[0]]][:, None] - fv[mV[k[1]]][None, :]
            # model-space components are not amplitudes
            m1[k] = np.broadcast_to(~np.isin(mV[k[1]], self.act)[None, :], d1[k].shape).astype(np.float64)
        for k in self.keys2:
            d2[k] = (fx[mA[k[0]]][:, None, None, None] + fo[mO[k[1]]][None, :, None, None]
                     - fv[mV[k[2]]][None, None, :, None] - fv[mV[k[3]]][None, None, None, :])
        if precond == "dressed":
            d1 = {k: np.minimum(v, -floor) for k, v in d1.items()}
            d2 = {k: np.minimum(v, -floor) for k, v in d2.items()}
        self.D1, self.D2, self.mask1 = BlockTensor(2, d1), BlockTensor(4, d2), BlockTensor(2, m1)
        if shift is not None:
            from .shift import delta
            self.Delta1 = BlockTensor(2, {k: delta(v, shift[0], shift[1]) for k, v in d1.items()})
            self.Delta2 = BlockTensor(4, {k: delta(v, shift[0], shift[1]) for k, v in d2.items()})
        else:
            self.Delta1 = BlockTensor(2, {k: np.zeros_like(v) for k, v in d1.items()})
            self.Delta2 = BlockTensor(4, {k: np.zeros_like(v) for k, v in d2.items()})

    @staticmethod
    def _diag(F, mem, size):
        """Diagonal of a block-diagonal rank-2 block list as a dense vector."""
        out = np.zeros(size, np.complex128)
        for (ga, gb), v in F.blocks.items():
            if ga == gb:
                out[mem[ga]] = np.diag(v)
        return out

    def members(self, rank):
        return [self.memA, self.be.mem["V"]] if rank == 2 else [self.memA, self.be.mem["O"], self.be.mem["V"], self.be.mem["V"]]

    def zeros(self):
        return (BlockTensor(2, {k: np.zeros(v.shape, np.complex128) for k, v in self.D1.blocks.items()}),
                BlockTensor(4, {k: np.zeros(v.shape, np.complex128) for k, v in self.D2.blocks.items()}))

    def from_dense(self, s1, s2):
        """Block lists of dense s1[x, a], s2[x, j, a, b] (positions as in the dense form)."""
        return (BlockTensor.from_dense(s1, self.members(2), self.keys1),
                BlockTensor.from_dense(s2, self.members(4), self.keys2))

    def to_dense(self, x):
        shape = (self.nact, self.nv) if x.rank == 2 else (self.nact, self.no, self.nv, self.nv)
        return x.to_dense(self.members(x.rank), shape)

    def rvec(self, s1, s2):
        """r(x) = e_x + s_x: identity on the model space, s elsewhere."""
        mV = self.be.mem["V"]
        r1 = {}
        for (g, _), v in s1.blocks.items():
            b = v.copy()
            for c, a in enumerate(mV[g]):
                hit = np.nonzero(self.act == a)[0]
                if hit.size:                      # a is the active spinor number hit[0]
                    b[:, c] = (self.memA[g] == hit[0]).astype(np.float64)
            r1[(g, g)] = b
        return BlockTensor(2, r1), s2

    def heff_matrix(self, sg1):
        """H_eff[y, x] = sigma(x)^y (dense nact x nact; zero between different irreps)."""
        mV = self.be.mem["V"]
        h = np.zeros((self.nact, self.nact), np.complex128)
        for (g, _), v in sg1.blocks.items():
            for c, a in enumerate(mV[g]):
                hit = np.nonzero(self.act == a)[0]
                if hit.size:
                    h[hit[0], self.memA[g]] = v[:, c]
        return h

    def residual(self, s1, s2):
        """(R1, R2, H_eff) as FS01.residual, on block lists."""
        r1, r2 = self.rvec(s1, s2)
        sg1, sg2 = sigma(self.be, self.hb, r1, r2)
        heff = self.heff_matrix(sg1)
        hb = BlockTensor(2, {(g, g): heff[np.ix_(m, m)] for g, m in enumerate(self.memA) if m.size})
        R1 = sg1 - bein("ya,yx->xa", s1, hb)
        R2 = sg2 - bein("yjab,yx->xjab", s2, hb)
        R1 = R1 * self.mask1
        R2 = BlockTensor(4, {k: R2.blocks[k] if k in R2.blocks else np.zeros(v.shape, np.complex128)
                             for k, v in self.D2.blocks.items()})
        return R1, R2, heff


def solve_fs01_blocked(fs, tol=1e-10, maxit=200, ndiis=6, log=None, start=None):
    """solve_fs01 on block lists: the same Jacobi step, DIIS(ndiis) with
    B_kl = Re(<e1_k, e1_l> + 1/2 <e2_k, e2_l>) and convergence test.  Returns
    dict(s1, s2, heff, eig, iters, converged, history) (history: max|step| per
    iteration)."""
    from .solver import diis_coefficients
    s1, s2 = fs.zeros() if start is None else (start[0].copy(), start[1].copy())
    hist_t, hist_e, history = [], [], []
    converged = False
    k = 0
    for k in range(1, maxit + 1):
        R1, R2, heff = fs.residual(s1, s2)
        R1 = R1 - fs.Delta1 * s1
        R2 = R2 - fs.Delta2 * s2
        # model-space components (mask 0) have D = 0: divide them by 1, then drop them
        den1 = BlockTensor(2, {k: np.where(fs.mask1.blocks[k] != 0, v + fs.Delta1.blocks[k], 1.0)
                               for k, v in fs.D1.blocks.items()})
        e1 = (R1 / den1) * fs.mask1
        e2 = R2 / (fs.D2 + fs.Delta2)
        n1, n2 = s1 + e1, s2 + e2
        dmax = max(e1.absmax(), e2.absmax())
        history.append(dmax)
        if not np.isfinite(dmax):
            break
        if ndiis > 1:
            hist_t.append((n1, n2))
            hist_e.append((e1, e2))
            if len(hist_t) > ndiis:
                hist_t.pop(0)
                hist_e.pop(0)
            while len(hist_t) >= 2:
                m = len(hist_e)
                B = np.zeros((m, m))
                for a in range(m):
                    for b in range(m):
                        B[a, b] = (hist_e[a][0].vdot(hist_e[b][0]) + 0.5 * hist_e[a][1].vdot(hist_e[b][1])).real
                try:
                    c = diis_coefficients(B)
                except np.linalg.LinAlgError:
                    hist_t.pop(0)
                    hist_e.pop(0)
                    continue
                n1 = ccsd.Blocked.lincomb(list(c), [x[0] for x in hist_t])
                n2 = ccsd.Blocked.lincomb(list(c), [x[1] for x in hist_t])
                break
        s1, s2 = n1, n2
        if log:
            log(f"fs01 iter {k:3d}  max|step| = {dmax:.3e}")
        if dmax < tol:
            converged = True
            break
    R1, R2, heff = fs.residual(s1, s2)
    eig = np.linalg.eigvals(heff)
    eig = eig[np.lexsort((eig.imag, eig.real))]
    return dict(s1=s1, s2=s2, heff=heff, eig=eig, iters=k, converged=converged, history=history)

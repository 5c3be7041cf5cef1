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
Dense backend only (x is a leading index over the active set).
"""
from __future__ import annotations

import numpy as np

from . import ccsd
from .blocks import ttgt


def _P(x, a, b):
    ax = list(range(x.ndim))
    ax[a], ax[b] = ax[b], ax[a]
    return x - x.transpose(ax)


def hbar(be, t1, t2):
    """One- and two-body Hbar elements needed by the (0h,1p) sigma equations."""
    ein, V = be.ein, be.V
    I = ccsd.intermediates(be, t1, t2)
    tau, Fme = I["tau"], I["Fme"]
    sys_ = be.sys
    eo, ev = sys_.eps[: sys_.nocc], sys_.eps[sys_.nocc:]
    Fae = I["Fae"] + np.diag(ev) - 0.5 * ein("ma,me->ae", t1, Fme)
    Fmi = I["Fmi"] + np.diag(eo) + 0.5 * ein("ie,me->mi", t1, Fme)
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

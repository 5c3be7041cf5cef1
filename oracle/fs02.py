"""CPU FP64 oracle for the (0h,2p) Fock-space sector (test infrastructure).

Paper: the sector hierarchy of Eq. (5) taken one step further, to two valence
particles (the 0h0p -> 0h1p -> 0h2p scheme of its Kramers-pair examples); the
amplitude equations of Eq. (3) with the closed part Omega (V Omega)_Cl, and
H_eff = (H Omega)_Cl over the model space of active pairs.  At the CCSD level
the new amplitudes are s_xy^ab (two active particles x < y promoted to a pair
a < b that is not itself a model pair); T and the (0h,1p) amplitudes stay at
their converged values.

With the normal-ordered wave operator the 2p part of Omega acting on the model
state |xy> = a+_x a+_y |Phi> is the product of the two dressed one-particle
attachments plus the new amplitude,

  Omega |xy> = R_x R_y |Phi> + S_xy |Phi>,
  R_x = sum_e r1(x)^e a+_e + 1/2 sum_mef s_xm^ef a+_e a+_f a_m   (r1(x) = e_x + s_x),

and the sector's Bloch equation is projected on the 2p space:

  sigma2(xy) = [Hbar_N Omega |xy>]_2p ,  Hbar_N = exp(-T) H exp(T) - E_CC
  H_eff[zw, xy] = sigma2(xy)^zw                    (z < w active)
  R(xy)^ab  = sigma2(xy)^ab - sum_{z<w} omega(zw)^ab H_eff[zw, xy]   (ab not a model pair)
  omega(zw)^ab = r1(z)^a r1(w)^b - r1(z)^b r1(w)^a + s_zw^ab

Hbar_N acting on the product state splits by which attachment lines its
legs touch (Wick's theorem; the attachments contain quasi-creators only):
  * legs on one line only: A_ab[sigma1(x)^a r1(y)^b + r1(x)^a sigma1(y)^b]
    with sigma1 the (0h,1p) sigma vector (oracle.fs01.sigma);
  * legs on both lines:
      1/2 sum_ef Wbar_abef omega_pp^ef                     (omega_pp = omega - s)
      + sum_m [g(x)_m s_ym^ab - g(y)_m s_xm^ab]
            g(x)_m = sum_e Fbar_me r1(x)^e - 1/2 sum_nef <nm||ef> s_xn^ef
      + P(ab) sum_me [v(x)_ame s_ym^eb - v(y)_ame s_xm^eb],  v(x)_ame = sum_f Wbar_amef r1(x)^f
      + P(ab) sum_mnef <mn||ef> s_xm^ae s_yn^bf
  * the new amplitude: P(ab) sum_e Fbar_be s_xy^ae + 1/2 sum_ef Wbar_abef s_xy^ef.

Everything except the S_xy terms is fixed once T and the (0h,1p) amplitudes
are: it is prepared once (K below).  Signs were derived with the operator
algebra above and are pinned against a brute-force construction of
Omega |xy> and exp(-T) H exp(T) on the (N+2)-electron Fock space
(oracle.fock.dea_state / hbar_apply).  Update: s += R / D with
D_xy^ab = e_x + e_y - e_a - e_b; with dynamic shifts (oracle.shift)
s += (R - Delta s) / (D + Delta).  Dense backend only.
"""
from __future__ import annotations

import numpy as np

from . import fs01


def _A(x):
    """Antisymmetrise the last two axes."""
    return x - np.swapaxes(x, -1, -2)


class FS02:
    """(0h,2p) sector at fixed converged T and (0h,1p) amplitudes."""

    def __init__(self, f01: fs01.FS01, s1, s2, shift=None):
        be, hb = f01.be, f01.hb
        ein = be.ein
        self.f01 = f01
        self.no, self.nv, self.nact = f01.no, f01.nv, f01.nact
        act = f01.act
        self.pairs = [(x, y) for x in range(self.nact) for y in range(x + 1, self.nact)]
        self.npair = len(self.pairs)
        px = np.array([p[0] for p in self.pairs], int)
        py = np.array([p[1] for p in self.pairs], int)
        r1, r2 = f01.rvec(s1, s2)                     # r1[x, e], r2[x, m, e, f] = s_xm^ef
        sg1, _ = fs01.sigma(be, hb, r1, r2)           # sigma1[x, a]
        V_oovv = be.V("oovv")
        Wabef, Wamef, Fae, Fme = hb["Wabef"], hb["Wamef"], hb["Fae"], hb["Fme"]
        self.Wabef, self.Fvv = Wabef, Fae
        r1x, r1y, r2x, r2y = r1[px], r1[py], r2[px], r2[py]
        # 2p part of the attachment product
        self.wpp = _A(r1x[:, :, None] * r1y[:, None, :])
        # legs on one line
        K = _A(sg1[px][:, :, None] * r1y[:, None, :] + r1x[:, :, None] * sg1[py][:, None, :])
        # legs on both lines
        K = K + 0.5 * np.einsum("abef,pef->pab", Wabef, self.wpp)
        g = ein("me,xe->xm", Fme, r1) - 0.5 * np.einsum("nmef,xnef->xm", V_oovv, r2)
        K = K + np.einsum("pm,pmab->pab", g[px], r2y) - np.einsum("pm,pmab->pab", g[py], r2x)
        v = np.einsum("amef,xf->xame", Wamef, r1)
        K = K + _A(np.einsum("pame,pmeb->pab", v[px], r2y) - np.einsum("pame,pmeb->pab", v[py], r2x))
        K = K + _A(np.einsum("mnef,pmae,pnbf->pab", V_oovv, r2x, r2y, optimize=True))
        self.K = K
        # model pairs, denominators, masks
        self.ma = act[px]
        self.mb = act[py]
        sys_ = be.sys
        ev = sys_.eps[sys_.nocc:]
        exy = ev[self.ma] + ev[self.mb]
        self.D = exy[:, None, None] - ev[None, :, None] - ev[None, None, :]
        g_ = sys_.irrep[sys_.nocc:]
        n = sys_.nirrep
        gxy = g_[self.ma] + g_[self.mb]
        self.mask = ((gxy[:, None, None] - g_[None, :, None] - g_[None, None, :]) % n == 0)
        ia = np.zeros(self.nv, bool)
        ia[act] = True
        self.mask &= ~(ia[:, None] & ia[None, :])[None]            # model pairs are not amplitudes
        self.mask &= ~np.eye(self.nv, dtype=bool)[None]
        self.Delta = np.zeros_like(self.D)
        if shift is not None:
            from .shift import delta
            self.Delta = delta(self.D, shift[0], shift[1])

    def zeros(self):
        return np.zeros((self.npair, self.nv, self.nv), np.complex128)

    def sigma2(self, s):
        """sigma2(xy) for every model pair: the fixed part plus the S_xy terms."""
        t = np.einsum("be,pae->pab", self.Fvv, s)
        return self.K + (t - np.swapaxes(t, 1, 2)) + 0.5 * np.einsum("abef,pef->pab", self.Wabef, s)

    def residual(self, s):
        """(R, H_eff): Bloch residual on the non-model pairs and H_eff[zw, xy]."""
        sg = self.sigma2(s)
        heff = sg[:, self.ma, self.mb].T                          # heff[q, p] = sigma2(p)^(pair q)
        w = self.wpp + s
        R = sg - np.einsum("qab,qp->pab", w, heff)
        return np.where(self.mask, R, 0.0), heff


def solve_fs02(fs, tol=1e-10, maxit=200, ndiis=6, log=None, start=None):
    """Jacobi + DIIS on s_xy^ab (shifted equations if fs has shifts).  Returns
    dict(s, heff, eig, iters, converged)."""
    from .solver import diis_coefficients
    s = fs.zeros() if start is None else start.copy()
    hist_t, hist_e = [], []
    converged = False
    k = 0
    for k in range(1, maxit + 1):
        R, heff = fs.residual(s)
        R = R - fs.Delta * s
        e = np.where(fs.mask, R / np.where(fs.mask, fs.D + fs.Delta, 1.0), 0.0)
        ns = s + e
        dmax = float(np.abs(e).max()) if e.size else 0.0
        if ndiis > 1:
            hist_t.append(ns)
            hist_e.append(e)
            if len(hist_t) > ndiis:
                hist_t.pop(0)
                hist_e.pop(0)
            while len(hist_t) >= 2:
                m = len(hist_e)
                B = np.array([[0.5 * np.vdot(hist_e[a], hist_e[b]).real for b in range(m)] for a in range(m)])
                try:
                    c = diis_coefficients(B)
                except np.linalg.LinAlgError:
                    hist_t.pop(0)
                    hist_e.pop(0)
                    continue
                ns = sum(ci * x for ci, x in zip(c, hist_t))
                break
        s = ns
        if log:
            log(f"fs02 iter {k:3d}  max|step| = {dmax:.3e}")
        if dmax < tol:
            converged = True
            break
    R, heff = fs.residual(s)
    eig = np.linalg.eigvals(heff)
    eig = eig[np.lexsort((eig.imag, eig.real))]
    return dict(s=s, heff=heff, eig=eig, iters=k, converged=converged)

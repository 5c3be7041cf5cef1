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
s += (R - Delta s) / (D + Delta).  FS02 runs on the dense backend; FS02Blocked
evaluates the same terms with the four-index Hbar elements (Wbar_abef,
Wbar_amef, <mn||ef>) as block lists and everything that carries the pair index
(at most npair x nvirt x nvirt) dense.
"""
from __future__ import annotations

import numpy as np

from . import fs01
from .blocks import BlockTensor, bein


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


class FS02Blocked(FS02):
    """FS02 on top of an FS01Blocked sector.  The pair amplitudes s[p, a, b],
    K, the denominators and the residual stay dense (p over the pairs x < y of
    positions in the active list, as in FS02); the contractions with Wbar_abef,
    Wbar_amef and <mn||ef> run over block lists, the pair index carrying the
    pair irrep g_x + g_y."""

    def __init__(self, f01: fs01.FS01Blocked, s1, s2, shift=None):
        be, hb = f01.be, f01.hb
        ein = be.ein
        self.f01 = f01
        self.no, self.nv, self.nact = f01.no, f01.nv, f01.nact
        act = f01.act
        n = be.sys.nirrep
        mV = be.mem["V"]
        self.pairs = [(x, y) for x in range(self.nact) for y in range(x + 1, self.nact)]
        self.npair = len(self.pairs)
        px = np.array([p[0] for p in self.pairs], int)
        py = np.array([p[1] for p in self.pairs], int)
        gA = be.sys.irrep[act + be.sys.nocc]
        gp = (gA[px] + gA[py]) % n if self.npair else np.zeros(0, int)
        self.memP = [np.nonzero(gp == G)[0] for G in range(n)]
        self.keysP = [(G, ga, (G - ga) % n) for G in range(n) for ga in range(n)
                      if self.memP[G].size and mV[ga].size and mV[(G - ga) % n].size]
        r1b, r2b = f01.rvec(s1, s2)                     # block lists
        sg1b, _ = fs01.sigma(be, hb, r1b, r2b)
        r1, r2, sg1 = f01.to_dense(r1b), f01.to_dense(r2b), f01.to_dense(sg1b)
        self.Wabef = hb["Wabef"]
        self.Fvv = hb["Fae"].to_dense([mV, mV], (self.nv, self.nv))
        r1x, r1y, r2x, r2y = r1[px], r1[py], r2[px], r2[py]
        self.wpp = _A(r1x[:, :, None] * r1y[:, None, :])
        K = _A(sg1[px][:, :, None] * r1y[:, None, :] + r1x[:, :, None] * sg1[py][:, None, :])
        K = K + 0.5 * self._w_pairs(self.wpp)
        g = be.ein("me,xe->xm", hb["Fme"], r1b) - 0.5 * bein("nmef,xnef->xm", be.V("oovv"), r2b)
        g = g.to_dense([f01.memA, be.mem["O"]], (self.nact, self.no))
        K = K + np.einsum("pm,pmab->pab", g[px], r2y) - np.einsum("pm,pmab->pab", g[py], r2x)
        v = bein("amef,xf->xame", hb["Wamef"], r1b).to_dense([f01.memA, mV, be.mem["O"], mV],
                                                            (self.nact, self.nv, self.no, self.nv))
        # sum_me v(x)_ame s_ym^eb as one matrix product per pair ((m, e) contracted)
        nme = self.no * self.nv
        vx = v[px].reshape(self.npair, self.nv, nme)
        vy = v[py].reshape(self.npair, self.nv, nme)
        K = K + _A(np.matmul(vx, r2y.reshape(self.npair, nme, self.nv))
                   - np.matmul(vy, r2x.reshape(self.npair, nme, self.nv)))
        # sum_mnef <mn||ef> s_xm^ae s_yn^bf: Y_y[m, e, b] = sum_nf <mn||ef> s_yn^bf, then sum over (m, e)
        Y = bein("mnef,ynbf->ymeb", be.V("oovv"), r2b).to_dense([f01.memA, be.mem["O"], mV, mV],
                                                               (self.nact, self.no, self.nv, self.nv))
        K = K + _A(np.matmul(r2x.transpose(0, 2, 1, 3).reshape(self.npair, self.nv, nme),
                             Y[py].reshape(self.npair, nme, self.nv)))
        self.K = K
        self.ma = act[px]
        self.mb = act[py]
        ev = be.sys.eps[be.sys.nocc:]
        exy = ev[self.ma] + ev[self.mb]
        self.D = exy[:, None, None] - ev[None, :, None] - ev[None, None, :]
        g_ = be.sys.irrep[be.sys.nocc:]
        gxy = g_[self.ma] + g_[self.mb]
        self.mask = ((gxy[:, None, None] - g_[None, :, None] - g_[None, None, :]) % n == 0)
        ia = np.zeros(self.nv, bool)
        ia[act] = True
        self.mask &= ~(ia[:, None] & ia[None, :])[None]
        self.mask &= ~np.eye(self.nv, dtype=bool)[None]
        self.Delta = np.zeros_like(self.D)
        if shift is not None:
            from .shift import delta
            self.Delta = delta(self.D, shift[0], shift[1])

    def _w_pairs(self, w):
        """sum_ef Wbar_abef w[p, e, f] over block lists (dense in and out)."""
        mV = self.f01.be.mem["V"]
        wb = BlockTensor.from_dense(w, [self.memP, mV, mV], self.keysP)
        out = bein("abef,pef->pab", self.Wabef, wb)
        return out.to_dense([self.memP, mV, mV], (self.npair, self.nv, self.nv))

    def sigma2(self, s):
        """sigma2(xy) for every model pair: the fixed part plus the S_xy terms."""
        t = np.matmul(s, self.Fvv.T)                                 # sum_e Fbar_be s_xy^ae
        return self.K + (t - np.swapaxes(t, 1, 2)) + 0.5 * self._w_pairs(s)


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

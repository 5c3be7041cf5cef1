"""Brute-force Fock-space reference for tiny systems (test infrastructure).

Builds the second-quantised Hamiltonian of Eq. (1) as explicit matrices on
particle-number sectors of the Fock space (Jordan-Wigner sign convention,
determinants as occupation bit strings), and the cluster operators of
Eq. (2) as matrices, so that exp(-T) H exp(T) can be projected onto
excited determinants without any diagrammatic algebra.

  H = sum_pq h_pq a+_p a_q + 1/4 sum_pqrs <pq||rs> a+_p a+_q a_s a_r
  h_pq = eps_p delta_pq - sum_i <pi||qi>   (so that the Fock matrix is diag(eps))
  E_ref = <Phi|H|Phi> = sum_i eps_i - 1/2 sum_ij <ij||ij>

Spinors: global index p = 0..n-1, occupied 0..nocc-1.  Only for n <= ~14.
"""
from __future__ import annotations

from itertools import combinations
from math import comb

import numpy as np


class Sector:
    """All determinants with N electrons in n spin orbitals."""

    def __init__(self, n: int, N: int):
        self.n, self.N = n, N
        self.dets = [sum(1 << p for p in c) for c in combinations(range(n), N)] if 0 <= N <= n else []
        self.index = {d: k for k, d in enumerate(self.dets)}

    @property
    def dim(self):
        return len(self.dets)


def annihilator(n: int, N: int, p: int) -> np.ndarray:
    """Matrix of a_p from sector N to sector N-1 (Jordan-Wigner sign)."""
    src, dst = Sector(n, N), Sector(n, N - 1)
    A = np.zeros((dst.dim, src.dim))
    for k, d in enumerate(src.dets):
        if d >> p & 1:
            sign = -1.0 if bin(d & ((1 << p) - 1)).count("1") % 2 else 1.0
            A[dst.index[d ^ (1 << p)], k] = sign
    return A


class FockSpace:
    """Hamiltonian and excitation operators on sectors N = nocc + delta."""

    def __init__(self, eps: np.ndarray, V: np.ndarray, nocc: int):
        self.n = len(eps)
        self.nocc = nocc
        self.eps = np.asarray(eps, float)
        self.V = V
        occ = range(nocc)
        self.h = np.diag(self.eps).astype(np.complex128) - sum(V[:, i, :, i] for i in occ)
        self.E_ref = float(np.sum(self.eps[:nocc]) - 0.5 * sum(V[i, j, i, j].real for i in occ for j in occ))
        self._a = {}

    def a(self, N: int, p: int) -> np.ndarray:
        key = (N, p)
        if key not in self._a:
            self._a[key] = annihilator(self.n, N, p)
        return self._a[key]

    def hamiltonian(self, N: int) -> np.ndarray:
        n = self.n
        dim = comb(n, N)
        H = np.zeros((dim, dim), np.complex128)
        if N >= 1:
            A1 = np.stack([self.a(N, p) for p in range(n)])       # [p, N-1, N]
            H += np.einsum("pq,pkd,qkD->dD", self.h, A1, A1, optimize=True)
        if N >= 2:
            pairs = [(p, q) for p in range(n) for q in range(p + 1, n)]
            # a_q a_p maps N -> N-2; its adjoint is a+_p a+_q
            A2 = np.stack([self.a(N - 1, q) @ self.a(N, p) for p, q in pairs])
            Vp = np.array([[self.V[p, q, r, s] for (r, s) in pairs] for (p, q) in pairs])
            Q = np.tensordot(Vp, A2, axes=(1, 0))
            H += np.tensordot(A2.conj(), Q, axes=([0, 1], [0, 1]))
        return H

    # -- excitation operators -------------------------------------------------
    def t_operator(self, N: int, t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
        """T = sum_ia t_i^a a+_a a_i + 1/4 sum_ijab t_ij^ab a+_a a+_b a_j a_i, on sector N."""
        no = self.nocc
        nv = self.n - no
        dim = comb(self.n, N)
        T = np.zeros((dim, dim), np.complex128)
        if N < 1:
            return T
        for i in range(no):
            ai = self.a(N, i)
            for a in range(nv):
                if t1[i, a] != 0:
                    T += t1[i, a] * (self.a(N, no + a).T @ ai)
        if N >= 2:
            for i in range(no):
                for j in range(i + 1, no):
                    aji = self.a(N - 1, j) @ self.a(N, i)          # a_j a_i : N -> N-2
                    for a in range(nv):
                        for b in range(a + 1, nv):
                            if t2[i, j, a, b] != 0:
                                cab = self.a(N, no + a).T @ self.a(N - 1, no + b).T   # a+_a a+_b : N-2 -> N
                                T += t2[i, j, a, b] * (cab @ aji)
        return T

    def reference(self, N: int) -> np.ndarray:
        sec = Sector(self.n, N)
        v = np.zeros(sec.dim, np.complex128)
        v[sec.index[(1 << self.nocc) - 1]] = 1.0
        return v

    def det(self, N: int, create, annihilate) -> np.ndarray:
        """|a+_{c0} a+_{c1} ... a_{k1} a_{k0} Phi>: create listed left to right, annihilate applied first-listed first."""
        v = self.reference(self.nocc)
        M = self.nocc
        for p in annihilate:
            v = self.a(M, p) @ v
            M -= 1
        for p in reversed(list(create)):
            v = self.a(M + 1, p).T @ v
            M += 1
        assert M == N
        return v


def expm_nilpotent(T: np.ndarray, v: np.ndarray, sign: float = 1.0) -> np.ndarray:
    """exp(sign*T) v for nilpotent T (finite Taylor series)."""
    out = v.copy()
    term = v.copy()
    k = 1
    while True:
        term = sign * (T @ term) / k
        if not np.any(np.abs(term) > 0):
            break
        out = out + term
        k += 1
        if k > 64:
            raise RuntimeError("T is not nilpotent")
    return out


def projected_residual(fs: FockSpace, t1: np.ndarray, t2: np.ndarray):
    """R_mu = <Phi_mu| exp(-T) (H - E_ref) exp(T) |Phi> for singles and doubles, and E_CC."""
    N = fs.nocc
    no, nv = fs.nocc, fs.n - fs.nocc
    H = fs.hamiltonian(N) - fs.E_ref * np.eye(comb(fs.n, N))
    T = fs.t_operator(N, t1, t2)
    phi = fs.reference(N)
    u = expm_nilpotent(T, H @ expm_nilpotent(T, phi, 1.0), -1.0)
    R1 = np.zeros((no, nv), np.complex128)
    R2 = np.zeros((no, no, nv, nv), np.complex128)
    for i in range(no):
        for a in range(nv):
            R1[i, a] = np.vdot(fs.det(N, [no + a], [i]), u)
    for i in range(no):
        for j in range(i + 1, no):
            for a in range(nv):
                for b in range(a + 1, nv):
                    x = np.vdot(fs.det(N, [no + a, no + b], [i, j]), u)
                    R2[i, j, a, b] = x
                    R2[j, i, a, b] = -x
                    R2[i, j, b, a] = -x
                    R2[j, i, b, a] = x
    return R1, R2, complex(np.vdot(phi, u))


def fci_energies(fs: FockSpace, N: int) -> tuple[np.ndarray, np.ndarray]:
    """Eigenvalues/vectors of H in sector N."""
    return np.linalg.eigh(fs.hamiltonian(N))


def ea_basis(fs: FockSpace):
    """(0h,1p)-sector basis of the N+1 electron space: |a> = a+_a|Phi>, |ab_j> = a+_a a+_b a_j|Phi> (a<b)."""
    no, nv = fs.nocc, fs.n - fs.nocc
    N1 = fs.nocc + 1
    vecs, labels = [], []
    for a in range(nv):
        vecs.append(fs.det(N1, [no + a], []))
        labels.append(("p", a))
    for j in range(no):
        for a in range(nv):
            for b in range(a + 1, nv):
                vecs.append(fs.det(N1, [no + a, no + b], [j]))
                labels.append(("pph", j, a, b))
    return np.array(vecs).T, labels


def ea_matrix(fs: FockSpace, t1: np.ndarray, t2: np.ndarray, E_tot: float | complex):
    """M_mu,nu = <mu| exp(-T) H exp(T) - E_tot |nu> on the (0h,1p) basis (T from the (0h,0p) sector)."""
    N1 = fs.nocc + 1
    H = fs.hamiltonian(N1)
    T = fs.t_operator(N1, t1, t2)
    B, labels = ea_basis(fs)
    # exp(-T) H exp(T) applied to each basis vector
    cols = []
    for k in range(B.shape[1]):
        v = expm_nilpotent(T, B[:, k], 1.0)
        v = expm_nilpotent(T, H @ v, -1.0)
        cols.append(v)
    HB = np.array(cols).T
    M = B.conj().T @ HB - E_tot * np.eye(B.shape[1])
    return M, labels


# -- (0h,2p) sector ----------------------------------------------------------
def apply_attach(fs: FockSpace, M: int, r1: np.ndarray, r2: np.ndarray, v: np.ndarray) -> np.ndarray:
    """R v for R = sum_e r1^e a+_e + 1/2 sum_mef r2_m^ef a+_e a+_f a_m (virtual e, f; occupied m),
    v in sector M, result in sector M+1."""
    no, nv = fs.nocc, fs.n - fs.nocc
    out = np.zeros(comb(fs.n, M + 1), np.complex128)
    for e in range(nv):
        if r1[e] != 0:
            out += r1[e] * (fs.a(M + 1, no + e).T @ v)
    for m in range(no):
        w0 = fs.a(M, m) @ v                                   # sector M-1
        for f in range(nv):
            w1 = fs.a(M, no + f).T @ w0                       # sector M
            for e in range(nv):
                if r2[m, e, f] != 0:
                    out += 0.5 * r2[m, e, f] * (fs.a(M + 1, no + e).T @ w1)
    return out


def hbar_apply(fs: FockSpace, N: int, t1: np.ndarray, t2: np.ndarray, E_tot, v: np.ndarray) -> np.ndarray:
    """(exp(-T) H exp(T) - E_tot) v on sector N."""
    H = fs.hamiltonian(N)
    T = fs.t_operator(N, t1, t2)
    u = expm_nilpotent(T, v, 1.0)
    u = H @ u - E_tot * u
    return expm_nilpotent(T, u, -1.0)


def pp_projection(fs: FockSpace, v: np.ndarray) -> np.ndarray:
    """c[a, b] = <Phi| a_b a_a |v> (coefficient of a+_a a+_b |Phi>), antisymmetric, v in sector nocc+2."""
    no, nv = fs.nocc, fs.n - fs.nocc
    c = np.zeros((nv, nv), np.complex128)
    for a in range(nv):
        for b in range(a + 1, nv):
            x = np.vdot(fs.det(no + 2, [no + a, no + b], []), v)
            c[a, b], c[b, a] = x, -x
    return c


def dea_state(fs: FockSpace, r1x, r2x, r1y, r2y, s_pp) -> np.ndarray:
    """R_x R_y |Phi> + sum_{a<b} s^ab a+_a a+_b |Phi> on sector nocc+2."""
    no, nv = fs.nocc, fs.n - fs.nocc
    phi = fs.reference(no)
    v = apply_attach(fs, no + 1, r1x, r2x, apply_attach(fs, no, r1y, r2y, phi))
    for a in range(nv):
        for b in range(a + 1, nv):
            if s_pp[a, b] != 0:
                v = v + s_pp[a, b] * fs.det(no + 2, [no + a, no + b], [])
    return v

"""Independent numpy implementation of the documented packed amplitude layouts.

Used only by tests to move between the oracle's dense tensors and the
library's packed buffers (include/fscc.h documents the layouts):

  T1: [g][o_g][v_g]                 -- t_i^a with irrep(i) = irrep(a) = g
  T2: [G][ij<][ab<]                 -- G = irrep(i)+irrep(j) = irrep(a)+irrep(b) (mod n)
      pairs (p,q) of one space with p<q in the irrep-sorted order, grouped by
      (g_p, g_q) with g_p <= g_q, g_p ascending; inside a group p-major.
Spinors inside an irrep are in ascending global index.
"""
import numpy as np


def members(sysm, X, g):
    """Positions within space X (0-based in that space) of irrep g, ascending."""
    base = 0 if X == "O" else sysm.nocc
    return sysm.members(X, g) - base


def pair_list(sysm, X, G):
    """Pairs (p<q) of space X with g_p + g_q = G, in layout order."""
    n = sysm.nirrep
    P, Q = [], []
    for gp in range(n):
        gq = (G - gp) % n
        if gp > gq:
            continue
        mp, mq = members(sysm, X, gp), members(sysm, X, gq)
        if gp < gq:
            for p in mp:
                for q in mq:
                    P.append(p)
                    Q.append(q)
        else:
            for a in range(len(mp)):
                for b in range(a + 1, len(mp)):
                    P.append(mp[a])
                    Q.append(mp[b])
    return np.array(P, dtype=np.int64), np.array(Q, dtype=np.int64)


def pack_t1(sysm, t1):
    out = []
    for g in range(sysm.nirrep):
        mo, mv = members(sysm, "O", g), members(sysm, "V", g)
        out.append(t1[np.ix_(mo, mv)].ravel())
    return np.concatenate(out) if out else np.zeros(0, np.complex128)


def unpack_t1(sysm, buf):
    t1 = np.zeros((sysm.nocc, sysm.nvirt), np.complex128)
    off = 0
    for g in range(sysm.nirrep):
        mo, mv = members(sysm, "O", g), members(sysm, "V", g)
        sz = len(mo) * len(mv)
        t1[np.ix_(mo, mv)] = buf[off:off + sz].reshape(len(mo), len(mv))
        off += sz
    assert off == buf.size
    return t1


def pack_t2(sysm, t2):
    out = []
    for G in range(sysm.nirrep):
        I, J = pair_list(sysm, "O", G)
        A, B = pair_list(sysm, "V", G)
        out.append(t2[I[:, None], J[:, None], A[None, :], B[None, :]].ravel())
    return np.concatenate(out)


def unpack_t2(sysm, buf):
    no, nv = sysm.nocc, sysm.nvirt
    t2 = np.zeros((no, no, nv, nv), np.complex128)
    off = 0
    for G in range(sysm.nirrep):
        I, J = pair_list(sysm, "O", G)
        A, B = pair_list(sysm, "V", G)
        sz = len(I) * len(A)
        x = buf[off:off + sz].reshape(len(I), len(A))
        off += sz
        t2[I[:, None], J[:, None], A[None, :], B[None, :]] = x
        t2[J[:, None], I[:, None], A[None, :], B[None, :]] = -x
        t2[I[:, None], J[:, None], B[None, :], A[None, :]] = -x
        t2[J[:, None], I[:, None], B[None, :], A[None, :]] = x
    assert off == buf.size
    return t2


def t2_size(sysm):
    return sum(len(pair_list(sysm, "O", G)[0]) * len(pair_list(sysm, "V", G)[0]) for G in range(sysm.nirrep))


def t1_size(sysm):
    return int(sum(len(members(sysm, "O", g)) * len(members(sysm, "V", g)) for g in range(sysm.nirrep)))


# ---------------------------------------------------------------- (0h,1p) sector
#   S1: [g][x_g][v_g]   (x = active spinors of irrep g, ascending global index; all virtuals)
#   S2: [G][(x,j)][ab<] (rows grouped by (g_x, g_j), g_x ascending, x-major)

def active_members(sysm, g):
    """Indices into sysm.active (sorted ascending) of the active spinors of irrep g."""
    act = np.sort(np.asarray(sysm.active))
    return np.array([k for k, p in enumerate(act) if sysm.irrep[p] == g], dtype=np.int64)


def xj_list(sysm, G):
    X, J = [], []
    n = sysm.nirrep
    for gx in range(n):
        gj = (G - gx) % n
        for x in active_members(sysm, gx):
            for j in members(sysm, "O", gj):
                X.append(x)
                J.append(j)
    return np.array(X, dtype=np.int64), np.array(J, dtype=np.int64)


def pack_s1(sysm, s1):
    out = []
    for g in range(sysm.nirrep):
        mx, mv = active_members(sysm, g), members(sysm, "V", g)
        out.append(s1[np.ix_(mx, mv)].ravel())
    return np.concatenate(out)


def unpack_s1(sysm, buf):
    s1 = np.zeros((len(sysm.active), sysm.nvirt), np.complex128)
    off = 0
    for g in range(sysm.nirrep):
        mx, mv = active_members(sysm, g), members(sysm, "V", g)
        sz = len(mx) * len(mv)
        s1[np.ix_(mx, mv)] = buf[off:off + sz].reshape(len(mx), len(mv))
        off += sz
    assert off == buf.size
    return s1


def pack_s2(sysm, s2):
    out = []
    for G in range(sysm.nirrep):
        X, J = xj_list(sysm, G)
        A, B = pair_list(sysm, "V", G)
        out.append(s2[X[:, None], J[:, None], A[None, :], B[None, :]].ravel())
    return np.concatenate(out)


def unpack_s2(sysm, buf):
    s2 = np.zeros((len(sysm.active), sysm.nocc, sysm.nvirt, sysm.nvirt), np.complex128)
    off = 0
    for G in range(sysm.nirrep):
        X, J = xj_list(sysm, G)
        A, B = pair_list(sysm, "V", G)
        sz = len(X) * len(A)
        x = buf[off:off + sz].reshape(len(X), len(A))
        off += sz
        s2[X[:, None], J[:, None], A[None, :], B[None, :]] = x
        s2[X[:, None], J[:, None], B[None, :], A[None, :]] = -x
    assert off == buf.size
    return s2


# ---------------------------------------------------------------- (0h,2p) sector
#   S02: [G][xy<][ab<]  (active pairs x < y in the irrep-sorted active order, grouped
#   like the T2 pairs; the dense oracle tensor is s[pair(i, j)][a][b] over the
#   pairs i < j of positions in the sorted active list, row-major upper triangle)

def xy_pair_list(sysm, G):
    n = sysm.nirrep
    P, Q = [], []
    for gp in range(n):
        gq = (G - gp) % n
        if gp > gq:
            continue
        mp, mq = active_members(sysm, gp), active_members(sysm, gq)
        if gp < gq:
            for p in mp:
                for q in mq:
                    P.append(p)
                    Q.append(q)
        else:
            for a in range(len(mp)):
                for b in range(a + 1, len(mp)):
                    P.append(mp[a])
                    Q.append(mp[b])
    return np.array(P, dtype=np.int64), np.array(Q, dtype=np.int64)


def pair_index(n, i, j):
    return i * (2 * n - i - 1) // 2 + (j - i - 1)


def _s02_full(sysm, s):
    n = len(sysm.active)
    full = np.zeros((n, n, sysm.nvirt, sysm.nvirt), np.complex128)
    for i in range(n):
        for j in range(i + 1, n):
            full[i, j] = s[pair_index(n, i, j)]
            full[j, i] = -s[pair_index(n, i, j)]
    return full


def pack_s02(sysm, s):
    full = _s02_full(sysm, s)
    out = []
    for G in range(sysm.nirrep):
        X, Y = xy_pair_list(sysm, G)
        A, B = pair_list(sysm, "V", G)
        out.append(full[X[:, None], Y[:, None], A[None, :], B[None, :]].ravel())
    return np.concatenate(out)


def unpack_s02(sysm, buf):
    n = len(sysm.active)
    full = np.zeros((n, n, sysm.nvirt, sysm.nvirt), np.complex128)
    off = 0
    for G in range(sysm.nirrep):
        X, Y = xy_pair_list(sysm, G)
        A, B = pair_list(sysm, "V", G)
        sz = len(X) * len(A)
        x = buf[off:off + sz].reshape(len(X), len(A))
        off += sz
        full[X[:, None], Y[:, None], A[None, :], B[None, :]] = x
        full[X[:, None], Y[:, None], B[None, :], A[None, :]] = -x
        full[Y[:, None], X[:, None], A[None, :], B[None, :]] = -x
        full[Y[:, None], X[:, None], B[None, :], A[None, :]] = x
    assert off == buf.size
    return np.array([full[i, j] for i in range(n) for j in range(i + 1, n)]).reshape(-1, sysm.nvirt, sysm.nvirt)


def t2_positions(sysm, idx):
    """Packed T2 offsets and signs of elements (i, j, a, b) (positions in the
    occupied and virtual spaces): t2[i, j, a, b] = sign * packed[offset].  A
    pair is stored once, in the order of pair_list (lower irrep first, then
    ascending position), so a swapped pair reads its stored partner with a
    minus sign."""
    n = sysm.nirrep
    go, gv = sysm.irrep[:sysm.nocc], sysm.irrep[sysm.nocc:]
    off, rows, cols = {}, {}, {}
    o = 0
    for G in range(n):
        I, J = pair_list(sysm, "O", G)
        A, B = pair_list(sysm, "V", G)
        off[G] = o
        rows[G] = {(int(p), int(q)): k for k, (p, q) in enumerate(zip(I, J))}
        cols[G] = {(int(p), int(q)): k for k, (p, q) in enumerate(zip(A, B))}
        o += len(I) * len(A)

    def find(table, p, q):
        if (p, q) in table:
            return table[(p, q)], 1.0
        return table[(q, p)], -1.0
    pos, sign = [], []
    for i, j, a, b in idx:
        G = (int(go[i]) + int(go[j])) % n
        assert (int(gv[a]) + int(gv[b])) % n == G
        r, sr = find(rows[G], int(i), int(j))
        c, sc = find(cols[G], int(a), int(b))
        pos.append(off[G] + r * len(cols[G]) + c)
        sign.append(sr * sc)
    return np.array(pos, dtype=np.int64), np.array(sign)


def t1_positions(sysm, idx):
    """Packed T1 offsets of elements (i, a)."""
    out = []
    base = 0
    offs = {}
    for g in range(sysm.nirrep):
        mo, mv = members(sysm, "O", g), members(sysm, "V", g)
        offs[g] = (base, {int(p): k for k, p in enumerate(mo)}, {int(p): k for k, p in enumerate(mv)}, len(mv))
        base += len(mo) * len(mv)
    for i, a in idx:
        g = int(sysm.irrep[i])
        b0, ro, co, nv = offs[g]
        out.append(b0 + ro[i] * nv + co[a])
    return np.array(out, dtype=np.int64)

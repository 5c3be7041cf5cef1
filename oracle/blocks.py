"""Block-sparse tensors for the CPU oracle (test infrastructure, not product).

A tensor is a list of dense blocks keyed by the irrep label of each index
(the partition of tensors into blocks by spinor subsets, "Symmetry handling
and data structures" section, and its rank-2 figure generalised to rank 4).
Blocks that are zero by symmetry are simply absent.

Contraction follows the block-contraction algorithm of the paper's Fig. 4:
for every pair of blocks (block_a, block_b) whose contracted labels carry the
same irreps, block_c += TTGT(block_a, block_b), where TTGT is the
transpose-transpose-GEMM-transpose decomposition of the "Algorithm design"
section (here delegated to numpy.tensordot, which reorders, calls GEMM and
returns the free indices in order; one final transpose gives the output
order).

The same `ttgt` is used by the dense backend on full arrays, so the dense and
blocked oracles differ only in the block bookkeeping.
"""
from __future__ import annotations

import numpy as np

_spec_cache: dict = {}


def _parse(spec: str):
    if spec in _spec_cache:
        return _spec_cache[spec]
    ins, out = spec.split("->")
    la, lb = ins.split(",")
    shared = [c for c in la if c in lb]
    for c in shared:
        if c in out:
            raise ValueError("batch (Hadamard) labels are not supported: " + spec)
    for c in la + lb:
        if c not in out and c not in shared:
            raise ValueError("label summed over one operand only: " + spec)
    ax_a = [la.index(c) for c in shared]
    ax_b = [lb.index(c) for c in shared]
    free = [c for c in la if c not in shared] + [c for c in lb if c not in shared]
    perm = [free.index(c) for c in out]
    r = (la, lb, out, shared, ax_a, ax_b, perm)
    _spec_cache[spec] = r
    return r


def ttgt(spec: str, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Two-operand contraction: reorder, one GEMM, reorder (TTGT)."""
    la, lb, out, shared, ax_a, ax_b, perm = _parse(spec)
    r = np.tensordot(a, b, axes=(ax_a, ax_b))
    return r.transpose(perm)


class BlockTensor:
    """Dict of dense blocks keyed by a tuple of irrep labels (one per index)."""

    __slots__ = ("rank", "blocks")

    def __init__(self, rank: int, blocks: dict | None = None):
        self.rank = rank
        self.blocks = {} if blocks is None else blocks

    # -- elementwise algebra ------------------------------------------------
    def _combine(self, other, fa, fb):
        out = {}
        for k, v in self.blocks.items():
            out[k] = fa * v if fa != 1.0 else v.copy()
        for k, v in other.blocks.items():
            if k in out:
                out[k] = out[k] + fb * v
            else:
                out[k] = fb * v
        return BlockTensor(self.rank, out)

    def __add__(self, other):
        return self._combine(other, 1.0, 1.0)

    def __sub__(self, other):
        return self._combine(other, 1.0, -1.0)

    def __mul__(self, s):
        if isinstance(s, BlockTensor):
            # elementwise product (used for D * t); keys of both must exist
            return BlockTensor(self.rank, {k: v * s.blocks[k] for k, v in self.blocks.items() if k in s.blocks})
        return BlockTensor(self.rank, {k: s * v for k, v in self.blocks.items()})

    __rmul__ = __mul__

    def __neg__(self):
        return self * -1.0

    def __truediv__(self, other):
        assert isinstance(other, BlockTensor)
        return BlockTensor(self.rank, {k: v / other.blocks[k] for k, v in self.blocks.items()})

    def conj(self):
        return BlockTensor(self.rank, {k: v.conj() for k, v in self.blocks.items()})

    def transpose(self, *axes):
        if len(axes) == 1 and not isinstance(axes[0], int):
            axes = tuple(axes[0])
        out = {}
        for k, v in self.blocks.items():
            out[tuple(k[a] for a in axes)] = v.transpose(axes)
        return BlockTensor(self.rank, out)

    def copy(self):
        return BlockTensor(self.rank, {k: v.copy() for k, v in self.blocks.items()})

    # -- reductions -----------------------------------------------------------
    def vdot(self, other) -> complex:
        """sum conj(self) * other."""
        s = 0.0 + 0.0j
        for k, v in self.blocks.items():
            if k in other.blocks:
                s += np.vdot(v.ravel(), other.blocks[k].ravel())
        return s

    def dot(self, other) -> complex:
        """sum self * other (no conjugation)."""
        s = 0.0 + 0.0j
        for k, v in self.blocks.items():
            if k in other.blocks:
                s += np.sum(v * other.blocks[k])
        return s

    def absmax(self) -> float:
        m = 0.0
        for v in self.blocks.values():
            if v.size:
                m = max(m, float(np.abs(v).max()))
        return m

    # -- conversion -----------------------------------------------------------
    def to_dense(self, members_per_axis, shape):
        """Scatter blocks into a dense array; members_per_axis[ax][g] = positions."""
        d = np.zeros(shape, np.complex128)
        for k, v in self.blocks.items():
            if v.size == 0:
                continue
            idx = np.ix_(*[members_per_axis[ax][g] for ax, g in enumerate(k)])
            d[idx] += v
        return d

    @staticmethod
    def from_dense(d, members_per_axis, keys):
        blocks = {}
        for k in keys:
            idx = np.ix_(*[members_per_axis[ax][g] for ax, g in enumerate(k)])
            b = np.ascontiguousarray(d[idx])
            if b.size:
                blocks[k] = b
        return BlockTensor(d.ndim, blocks)


def bein(spec: str, A: BlockTensor, B: BlockTensor) -> BlockTensor:
    """Blocked contraction: the block-pair loop of the paper's Fig. 4."""
    la, lb, out, shared, ax_a, ax_b, perm = _parse(spec)
    groups: dict = {}
    for kb, vb in B.blocks.items():
        if vb.size == 0:
            continue
        groups.setdefault(tuple(kb[i] for i in ax_b), []).append((kb, vb))
    pos_a = {c: la.index(c) for c in la}
    pos_b = {c: lb.index(c) for c in lb}
    src = [("a", pos_a[c]) if c in pos_a else ("b", pos_b[c]) for c in out]
    C: dict = {}
    for ka, va in A.blocks.items():
        if va.size == 0:
            continue
        for kb, vb in groups.get(tuple(ka[i] for i in ax_a), ()):
            kc = tuple(ka[p] if s == "a" else kb[p] for s, p in src)
            r = ttgt(spec, va, vb)
            if kc in C:
                C[kc] += r
            else:
                C[kc] = np.array(r, copy=True, order="C")
    return BlockTensor(len(out), C)

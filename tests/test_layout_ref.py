"""The test-side description of the packed amplitude layouts (layout_ref):
packing a random antisymmetric T2 and unpacking it gives it back, and the
element lookups used for sampled comparisons (t1_positions, t2_positions with
the sign of a swapped pair) read every allowed element of the dense tensors
from the packed buffers -- on systems with several irreps, empty irreps and
uneven blocks."""
import itertools

import numpy as np
import pytest

import fsgen
import layout_ref as LR

SYSTEMS = [(6, 14, 4, 0.1, 21), (5, 12, 6, 0.1, 4), (9, 23, 5, 0.05, 17)]


def _antisym_t2(s, rng):
    no, nv, n = s.nocc, s.nvirt, s.nirrep
    t = rng.normal(size=(no, no, nv, nv)) + 1j * rng.normal(size=(no, no, nv, nv))
    t = t - t.transpose(1, 0, 2, 3)
    t = t - t.transpose(0, 1, 3, 2)
    go, gv = s.irrep[:no], s.irrep[no:]
    allowed = ((go[:, None, None, None] + go[None, :, None, None]) % n ==
               (gv[None, None, :, None] + gv[None, None, None, :]) % n)
    return np.where(allowed, t, 0.0), allowed


@pytest.mark.parametrize("p", SYSTEMS, ids=lambda p: "o%dv%dz%d" % p[:3])
def test_t2_positions_read_every_allowed_element(p):
    s = fsgen.make_system(*p)
    rng = np.random.default_rng(0)
    t2, allowed = _antisym_t2(s, rng)
    buf = LR.pack_t2(s, t2)
    assert np.array_equal(LR.unpack_t2(s, buf), t2)
    idx = [(i, j, a, b) for i, j in itertools.combinations(range(s.nocc), 2)
           for a, b in itertools.combinations(range(s.nvirt), 2) if allowed[i, j, a, b]]
    pos, sg = LR.t2_positions(s, idx)
    want = np.array([t2[e] for e in idx])
    assert np.array_equal(sg * buf[pos], want)
    # every packed element is reached exactly once
    assert np.array_equal(np.sort(pos), np.arange(buf.size))


@pytest.mark.parametrize("p", SYSTEMS, ids=lambda p: "o%dv%dz%d" % p[:3])
def test_t1_positions_read_every_allowed_element(p):
    s = fsgen.make_system(*p)
    rng = np.random.default_rng(1)
    no = s.nocc
    t1 = rng.normal(size=(no, s.nvirt)) + 0j
    t1[s.irrep[:no, None] != s.irrep[None, no:]] = 0.0
    buf = LR.pack_t1(s, t1)
    idx = [(i, a) for i in range(no) for a in range(s.nvirt) if s.irrep[i] == s.irrep[no + a]]
    pos = LR.t1_positions(s, idx)
    assert np.array_equal(buf[pos], np.array([t1[e] for e in idx]))
    assert np.array_equal(np.sort(pos), np.arange(buf.size))

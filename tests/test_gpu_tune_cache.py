"""Autotune result cache (fscc_tune_cache) on the GPU: the first autotune of
a context measures and writes its choices; a second context of the same
system reads them back without timing (same tile forms and traversals, and
so bitwise the same residual); another system gets its own entry; a corrupt
file or a changed cache path falls back to measuring."""
import numpy as np
import pytest

import fsgen

pytestmark = pytest.mark.gpu


def _ctx(s):
    import torch
    import paper_2004_03682_amd as F
    ctx = F.Context.from_system(s)
    for C in fsgen.CLASSES:
        ctx.set_integrals(C, torch.from_numpy(fsgen.class_buffer(s, C)[0]).cuda())
    return ctx


def _residual(ctx, seed):
    import torch
    rng = np.random.default_rng(seed)
    t1 = torch.from_numpy(0.01 * (rng.normal(size=ctx.n1) + 1j * rng.normal(size=ctx.n1))).cuda()
    t2 = torch.from_numpy(0.01 * (rng.normal(size=ctx.n2) + 1j * rng.normal(size=ctx.n2))).cuda()
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    ctx.build_residual(t1, t2, r1, r2)
    return r1, r2


def test_cache_round_trip(tmp_path):
    import torch
    path = tmp_path / "tune.json"
    s = fsgen.make_system(12, 70, 4, 0.05, 77, nact=3)
    a = _ctx(s)
    a.tune_cache(path)
    a.autotune(1)
    assert not a.autotune_cached() and path.exists()
    b = _ctx(s)
    b.tune_cache(path)
    b.autotune(1)
    assert b.autotune_cached()
    assert a.gemm_configs() == b.gemm_configs()
    ra, rb = _residual(a, 1), _residual(b, 1)
    assert torch.equal(ra[0], rb[0]) and torch.equal(ra[1], rb[1])
    # another system: its own entry, the first one kept
    c = _ctx(fsgen.make_system(9, 37, 5, 0.05, 17))
    c.tune_cache(path)
    c.autotune(1)
    assert not c.autotune_cached()
    text = path.read_text()
    assert text.count('{"key": ') == 2
    d = _ctx(s)
    d.tune_cache(path)
    d.autotune(1)
    assert d.autotune_cached()
    # a corrupt file is re-measured and rewritten
    path.write_text("{not json")
    e = _ctx(s)
    e.tune_cache(path)
    e.autotune(1)
    assert not e.autotune_cached() and path.read_text().count('{"key": ') == 1
    for x in (a, b, c, d, e):
        x.destroy()


def test_no_cache_path_measures(tmp_path):
    s = fsgen.make_system(6, 14, 4, 0.1, 21)
    a = _ctx(s)
    a.autotune(1)
    assert not a.autotune_cached()
    a.tune_cache(None)
    a.autotune(1)
    assert not a.autotune_cached()
    a.destroy()

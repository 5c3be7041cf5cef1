"""Error model of the C ABI on the GPU (conditions forced from the host):

* fscc_set_integrals rejects non-finite values (FSCC_EINVAL) and, at sampled
  elements, violations of antisymmetry and Hermiticity (FSCC_ESYMM) before
  anything is packed; the class stays unset, so the correct buffer can be set
  afterwards and the residual then equals the one of a clean context;
* the divergence watch of fscc_update_amplitudes: residuals chosen so that
  the Jacobi steps grow geometrically give one DIIS reset and then
  FSCC_ENOCONV with the last (finite) iterate kept; a non-finite residual
  gives FSCC_ENOCONV at once with the amplitudes left at their input values.
"""
import numpy as np
import pytest

import fsgen

pytestmark = pytest.mark.gpu

ESYMM, EINVAL, ENOCONV = -2, -1, -6


def _setup(real=False):
    import torch
    import paper_2004_03682_amd as F
    s = fsgen.make_system(6, 14, 4, 0.1, 21, real=real)
    ctx = F.Context.from_system(s, precision="real_fp64" if real else "fp64")
    bufs = {C: fsgen.class_buffer(s, C)[0] for C in fsgen.CLASSES}
    if real:
        bufs = {C: fsgen.real_buffer(b) for C, b in bufs.items()}
    return torch, F, s, ctx, bufs


def _set(torch, ctx, C, host):
    ctx.set_integrals(C, torch.from_numpy(np.ascontiguousarray(host)).cuda())


@pytest.mark.parametrize("cls,how", [("OOOO", "noise"), ("OVVV", "noise"), ("OOVV", "noise"),
                                     ("VVVV", "phase"), ("OVOV", "phase")])
def test_symmetry_violations_are_rejected(cls, how):
    torch, F, s, ctx, bufs = _setup()
    print("case", cls, how, flush=True)
    rng = np.random.default_rng(3)
    bad = bufs[cls].copy()
    if how == "noise":     # breaks antisymmetry everywhere
        bad += 1e-3 * np.abs(bad).max() * (rng.normal(size=bad.size) + 1j * rng.normal(size=bad.size))
    else:                  # a global phase keeps antisymmetry and breaks Hermiticity
        bad *= np.exp(0.3j)
    with pytest.raises(F.FsccError) as e:
        _set(torch, ctx, cls, bad)
    assert e.value.status == ESYMM
    assert ("Hermiticity" if how == "phase" else "antisymmetry") in str(e.value)
    # the class was not taken: the correct buffer is accepted afterwards
    for C in fsgen.CLASSES:
        _set(torch, ctx, C, bufs[C])
    ctx.destroy()


def test_non_finite_values_are_rejected_and_checks_can_be_switched_off():
    torch, F, s, ctx, bufs = _setup()
    bad = bufs["OVVV"].copy()
    bad[bad.size // 3] = np.nan + 0j
    with pytest.raises(F.FsccError) as e:
        _set(torch, ctx, "OVVV", bad)
    assert e.value.status == EINVAL and "non-finite" in str(e.value)
    # without the sampled symmetry checks a phase-rotated class is taken as it is
    ctx.set_validation(0)
    _set(torch, ctx, "VVVV", bufs["VVVV"] * np.exp(0.3j))
    with pytest.raises(F.FsccError):
        ctx.set_validation(-1)
    ctx.destroy()


def test_real_context_checks_plain_symmetry():
    torch, F, s, ctx, bufs = _setup(real=True)
    bad = bufs["OVOV"].copy()
    rng = np.random.default_rng(5)
    bad += 1e-3 * np.abs(bad).max() * rng.normal(size=bad.size)
    with pytest.raises(F.FsccError) as e:
        _set(torch, ctx, "OVOV", bad)
    assert e.value.status == ESYMM
    ctx.destroy()


def test_clean_context_after_rejection_gives_the_same_residual():
    torch, F, s, ctx, bufs = _setup()
    with pytest.raises(F.FsccError):
        _set(torch, ctx, "OOOO", bufs["OOOO"] * np.exp(0.1j))
    for C in fsgen.CLASSES:
        _set(torch, ctx, C, bufs[C])
    _, _, _, ref, _ = _setup()
    for C in fsgen.CLASSES:
        _set(torch, ref, C, bufs[C])
    rng = np.random.default_rng(9)
    t1 = torch.from_numpy(0.01 * (rng.normal(size=ctx.n1) + 1j * rng.normal(size=ctx.n1))).cuda()
    t2 = torch.from_numpy(0.01 * (rng.normal(size=ctx.n2) + 1j * rng.normal(size=ctx.n2))).cuda()
    r = [torch.empty_like(t1), torch.empty_like(t2)]
    q = [torch.empty_like(t1), torch.empty_like(t2)]
    ctx.build_residual(t1, t2, *r)
    ref.build_residual(t1, t2, *q)
    assert torch.equal(r[0], q[0]) and torch.equal(r[1], q[1])
    ctx.destroy()
    ref.destroy()


def test_divergence_watch_resets_then_gives_up():
    torch, F, s, ctx, bufs = _setup()
    for C in fsgen.CLASSES:
        _set(torch, ctx, C, bufs[C])
    # plain Jacobi (no DIIS): step = R / D exactly, so R = c * D gives max|step| = c
    ctx.diis_reset(1)
    # the library's denominators are e_i - e_a and e_i + e_j - e_a - e_b in the packed layouts
    import layout_ref as LR
    no = s.nocc
    eo, ev = s.eps[:no], s.eps[no:]
    D1 = LR.pack_t1(s, (eo[:, None] - ev[None, :]).astype(np.complex128)).real
    d2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    D2 = LR.pack_t2(s, d2.astype(np.complex128)).real
    t1 = torch.zeros(ctx.n1, dtype=torch.complex128, device="cuda")
    t2 = torch.zeros(ctx.n2, dtype=torch.complex128, device="cuda")
    actions = []
    steps = 0.05 * 1.5 ** np.arange(60)
    for c in steps:
        r1 = torch.from_numpy((c * D1).astype(np.complex128)).cuda()
        r2 = torch.from_numpy((c * D2).astype(np.complex128)).cuda()
        try:
            got = ctx.update_amplitudes(t1, t2, r1, r2)
            assert abs(got - c) <= 1e-12 * c
            actions.append("ok")
        except F.FsccError as e:
            assert e.status == ENOCONV
            actions.append("stop")
            break
    assert actions[-1] == "stop"
    k = len(actions) - 1
    # first growth past 1e3 x the first step resets the subspace, the second gives up
    first = int(np.argmax(steps > 1e3 * steps[0]))
    assert steps[k] > 1e3 * steps[first] and steps[k - 1] <= 1e3 * steps[first]
    assert bool(torch.isfinite(t2).all()) and bool(torch.isfinite(t1).all())
    # a non-finite residual: ENOCONV at once, amplitudes untouched
    ctx.diis_reset(6)
    keep1, keep2 = t1.clone(), t2.clone()
    r1 = torch.zeros_like(t1)
    r2 = torch.zeros_like(t2)
    r2[7] = complex(np.nan, 0.0)
    with pytest.raises(F.FsccError) as e:
        ctx.update_amplitudes(t1, t2, r1, r2)
    assert e.value.status == ENOCONV
    assert torch.equal(t1, keep1) and torch.equal(t2, keep2)
    # the sector recovers: a finite step after the failure is taken normally
    r2[7] = 0.0
    assert ctx.update_amplitudes(t1, t2, r1, r2) == 0.0
    ctx.destroy()

"""fscc_zgemm_noalloc (static device scratch, no device allocation) against
fscc_zgemm (per-call allocations): same kernels and plan, so the results must
agree to the FP64 GEMM tolerance (in practice bit for bit); two calls in a
row, the second smaller, so that the second reuses the array the first left
behind.  Also checked against a numpy product on the host.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _rand(rng, shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def _case(F, torch, rng, M, N, K, tA, tB, cfg, allow_split, beta):
    A = _rand(rng, (K, M) if tA else (M, K))
    B = _rand(rng, (N, K) if tB else (K, N))
    C0 = _rand(rng, (M, N))
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    c_ref = torch.from_numpy(C0).cuda()
    c_na = torch.from_numpy(C0).cuda()
    lda, ldb = (M if tA else K), (K if tB else N)
    alpha = 0.5 - 0.25j
    F.zgemm(dA, dB, c_ref, M, N, K, lda, ldb, N, tA=tA, tB=tB, alpha=alpha, beta=beta, cfg=cfg,
            allow_split=allow_split)
    F.zgemm_noalloc(dA, dB, c_na, M, N, K, lda, ldb, N, tA=tA, tB=tB, alpha=alpha, beta=beta, cfg=cfg,
                    allow_split=allow_split)
    torch.cuda.synchronize()
    got, ref = c_na.cpu().numpy(), c_ref.cpu().numpy()
    opA = A.T if tA else A
    opB = B.T if tB else B
    host = alpha * (opA @ opB) + (C0 if beta else 0)
    scale = np.abs(opA).max() * np.abs(opB).max() * K
    # same plan and kernels: identical up to rounding order (tolerance of one FP64 GEMM)
    assert np.abs(got - ref).max() <= 1e-13 * scale
    assert np.abs(got - host).max() <= 1e-13 * scale
    return np.array_equal(got, ref)


@pytest.mark.parametrize("cfg,allow_split", [(-1, 1), (3 | 256, 1), (0, 0), (6, 1), (9 | 256 | 1024, 1)],
                         ids=["cost-model", "32x32-3M-split", "64x64-unsplit", "skinny", "32x64-3M-direct-LDS-split"])
def test_noalloc_matches_allocating_entry_point(cfg, allow_split):
    torch = _torch()
    import paper_2004_03682_amd as F
    rng = np.random.default_rng(11)
    print("noalloc case", cfg, allow_split, flush=True)
    # a long K (split along K when allowed), then a smaller ragged product
    same1 = _case(F, torch, rng, 200, 72, 2100, False, True, cfg, allow_split, 1)
    same2 = _case(F, torch, rng, 37, 19, 300, True, False, cfg, allow_split, 0)
    assert same1 and same2


def test_noalloc_rejects_plans_beyond_the_scratch():
    torch = _torch()
    import paper_2004_03682_amd as F
    # 16x64 tiles over 2064 x 2^20 outputs: 129 * 16384 tiles * 16 B = 33.8 MB of tile
    # table, more than the 32 MiB array.  Every operand has its full size, so the call
    # would be in bounds even if it were not refused.
    M, N, K = 2064, 1 << 20, 1
    A = torch.zeros((M, K), dtype=torch.complex128, device="cuda")
    B = torch.zeros((K, N), dtype=torch.complex128, device="cuda")
    C = torch.empty((M, N), dtype=torch.complex128, device="cuda")
    try:
        with pytest.raises(F.FsccError) as e:
            F.zgemm_noalloc(A, B, C, M, N, K, K, N, N, cfg=5, allow_split=0)
        assert "scratch" in str(e.value)
    finally:
        del A, B, C
        torch.cuda.empty_cache()

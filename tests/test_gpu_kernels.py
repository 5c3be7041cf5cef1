"""Kernel-level parity of the grouped complex FP64 GEMM forms (through the C
ABI) against numpy: every MFMA tile shape in the four- and three-product
complex forms, K depth, transpose/conjugate flag, LDS staging form (through
registers, double-buffered, direct-to-LDS ring) and split-K choice, the vector-ALU skinny, tall, reduction and dot forms, with
ragged sizes (not multiples of any tile), K = 0 and accumulation (beta = 1)."""
import itertools

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

M3 = 256   # FSCC_CFG_3M: three-product complex form of an MFMA tile
DB = 512   # FSCC_CFG_DB: double-buffered LDS form (16-deep slices)
MFMA_TILES = (0, 1, 2, 3, 4, 5, 9, 10, 12, 13)   # 0-5, 9 (32x64), 10 (64x32), 12/13 (64x64, 64x32, waves along M)
DB_TILES = (3, 4, 5, 9, 10, 13)
CFGS = MFMA_TILES + tuple(c | M3 for c in MFMA_TILES) + (6,)   # 4M and 3M MFMA tiles; 6 = skinny (vector ALUs)
DB_CFGS = tuple(c | DB for c in DB_TILES) + tuple(c | DB | M3 for c in DB_TILES)
DL = 1024   # FSCC_CFG_DL: direct-to-LDS loads through a ring of LDS stages (16-deep slices)
DL_TILES = (0, 3, 4, 5, 9, 10, 12, 13)
DL_CFGS = tuple(c | DL for c in DL_TILES) + tuple(c | DL | M3 for c in DL_TILES)


def _rand(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def _run(M, N, K, tA, tB, cA, cB, cfg, bk, split, beta, seed=0, alpha=0.7 - 0.3j):
    import torch
    import paper_2004_03682_amd as F
    rng = np.random.default_rng(seed)
    A = _rand(rng, K, M) if tA else _rand(rng, M, K)
    B = _rand(rng, N, K) if tB else _rand(rng, K, N)
    C0 = _rand(rng, M, N)
    opA = A.T if tA else A
    opB = B.T if tB else B
    if cA:
        opA = opA.conj()
    if cB:
        opB = opB.conj()
    ref = alpha * (opA @ opB) + (C0 if beta else 0)
    dA = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    dB = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    dC = torch.from_numpy(np.ascontiguousarray(C0)).cuda()
    lda = max(A.shape[1], 1)
    ldb = max(B.shape[1], 1)
    F.zgemm(dA, dB, dC, M, N, K, max(lda, 1), max(ldb, 1), max(N, 1), tA, tB, cA, cB, alpha, beta, cfg, bk, split)
    out = dC.cpu().numpy()
    scale = max(1.0, np.abs(ref).max())
    return np.abs(out - ref).max() / scale


@pytest.mark.parametrize("cfg,bk", list(itertools.product(CFGS, (16, 32))))
def test_zgemm_every_config(cfg, bk):
    for (tA, tB, cA, cB) in [(0, 0, 0, 0), (0, 1, 1, 0), (1, 0, 0, 1), (1, 1, 1, 1)]:
        for (M, N, K) in [(1, 1, 1), (17, 33, 15), (70, 23, 129), (130, 131, 40), (1017, 1, 300), (3, 48, 700)]:
            err = _run(M, N, K, tA, tB, cA, cB, cfg, bk, False, beta=(M % 2))
            assert err < 1e-13, (cfg, bk, tA, tB, cA, cB, M, N, K, err)


@pytest.mark.parametrize("cfg", DB_CFGS)
def test_zgemm_double_buffered_forms(cfg):
    """The double-buffered LDS forms: ragged sizes, every transpose/conjugate
    flag, K below, at and above one and two 16-deep slices, split-K, K = 0."""
    for (tA, tB, cA, cB) in [(0, 0, 0, 0), (0, 1, 1, 0), (1, 0, 0, 1), (1, 1, 1, 1)]:
        for (M, N, K) in [(1, 1, 1), (17, 33, 15), (70, 23, 16), (33, 65, 17), (130, 131, 32), (40, 50, 33),
                          (1017, 1, 300), (3, 48, 700)]:
            err = _run(M, N, K, tA, tB, cA, cB, cfg, 16, False, beta=(M % 2))
            assert err < 1e-13, (cfg, tA, tB, cA, cB, M, N, K, err)
    for (M, N, K, beta) in [(7, 34, 3000, 0), (300, 200, 1800, 1), (9, 11, 0, 1)]:
        err = _run(M, N, K, 0, 1, 0, 0, cfg, 16, True, beta)
        assert err < 1e-13, (cfg, M, N, K, beta, err)


@pytest.mark.parametrize("cfg", DL_CFGS)
def test_zgemm_direct_to_lds_forms(cfg):
    """The direct-to-LDS forms: ragged sizes, every transpose/conjugate flag,
    K from below one 16-deep slice to many turns of the stage ring (its
    prologue, wrap-around and the clamped loads past the last slice), the
    zeroed k past K of a last partial slice, split-K and K = 0."""
    for (tA, tB, cA, cB) in [(0, 0, 0, 0), (0, 1, 1, 0), (1, 0, 0, 1), (1, 1, 1, 1)]:
        for (M, N, K) in [(1, 1, 1), (17, 33, 15), (70, 23, 16), (33, 65, 17), (130, 131, 32), (40, 50, 33),
                          (19, 77, 48), (65, 20, 49), (31, 129, 64), (50, 50, 95), (1017, 1, 300), (3, 48, 700)]:
            err = _run(M, N, K, tA, tB, cA, cB, cfg, 16, False, beta=(M % 2))
            assert err < 1e-13, (cfg, tA, tB, cA, cB, M, N, K, err)
    for (M, N, K, beta) in [(7, 34, 3000, 0), (300, 200, 1800, 1), (9, 11, 0, 1), (9, 11, 0, 0)]:
        err = _run(M, N, K, 0, 1, 0, 0, cfg, 16, True, beta)
        assert err < 1e-13, (cfg, M, N, K, beta, err)


def test_direct_to_lds_form_needs_an_eligible_tile():
    import torch
    import paper_2004_03682_amd as F
    a = torch.zeros((4, 4), dtype=torch.complex128, device="cuda")
    for cfg, bk in ((1 | DL, 16), (6 | DL, 16), (9 | DL, 32), (9 | DL | DB, 16)):
        with pytest.raises(F.FsccError):
            F.zgemm(a, a, a, 4, 4, 4, 4, 4, 4, cfg=cfg, bk=bk)


def test_double_buffered_form_needs_an_eligible_tile():
    import torch
    import paper_2004_03682_amd as F
    a = torch.zeros((4, 4), dtype=torch.complex128, device="cuda")
    for cfg, bk in ((0 | DB, 16), (12 | DB, 16), (9 | DB, 32)):
        with pytest.raises(F.FsccError):
            F.zgemm(a, a, a, 4, 4, 4, 4, 4, 4, cfg=cfg, bk=bk)


@pytest.mark.parametrize("cfg", CFGS)
def test_zgemm_split_k_and_edges(cfg):
    # long K with few output tiles triggers the split-K path (more than 8 K
    # chunks: the grouped reduction pass; at most 8, with several thousand
    # outputs: the one-output-per-thread pass); K = 0 must give beta*C
    for (M, N, K, beta) in [(7, 34, 3000, 0), (7, 7, 5000, 1), (20, 3, 700, 1), (300, 200, 1800, 1),
                            (130, 70, 1200, 0), (9, 11, 0, 0), (9, 11, 0, 1)]:
        err = _run(M, N, K, 0, 1, 0, 0, cfg, 16, True, beta)
        assert err < 1e-13, (cfg, M, N, K, beta, err)


@pytest.mark.parametrize("cfg", (9 | M3, 0 | M3, 5, 6, 8))
def test_split_k_pass_with_padded_c(cfg):
    """Split-K into a C with row stride ldc > N: the reduction pass writes the
    M x N block and leaves the padding columns untouched."""
    import torch
    import paper_2004_03682_amd as F
    rng = np.random.default_rng(5)
    for (M, N, K, ldc, beta) in [(7, 34, 3000, 41, 1), (130, 70, 1200, 77, 0), (5, 200, 1800, 203, 1)]:
        if cfg == 8 and M > 8:   # the reduction form takes M <= 8
            continue
        A, B = _rand(rng, M, K), _rand(rng, K, N)
        C0 = _rand(rng, M, ldc)
        alpha = 0.6 + 0.2j
        ref = C0.copy()
        ref[:, :N] = alpha * (A @ B) + (C0[:, :N] if beta else 0)
        dA, dB, dC = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (A, B, C0))
        F.zgemm(dA, dB, dC, M, N, K, K, N, ldc, 0, 0, 0, 0, alpha, beta, cfg, 16, True)
        out = dC.cpu().numpy()
        assert np.array_equal(out[:, N:], C0[:, N:])
        assert np.abs(out - ref).max() / max(1.0, np.abs(ref).max()) < 1e-13, (cfg, M, N, K, ldc)


TALL, RED, DOT = 7, 8, 11


@pytest.mark.parametrize("tB,cA,cB", [(0, 0, 0), (1, 1, 0), (0, 1, 1), (1, 0, 1)])
def test_zgemm_tall_form(tB, cA, cB):
    # many rows, short K, few columns (the t1 x integral products); K*N <= 1024
    for (M, N, K) in [(1, 1, 1), (255, 7, 21), (257, 3, 48), (1000, 48, 7), (5000, 1, 64), (300, 16, 64),
                      (77, 1024, 1), (513, 9, 0)]:
        for beta in (0, 1):
            err = _run(M, N, K, 0, tB, cA, cB, TALL, 16, False, beta, seed=M + N + K)
            assert err < 1e-13, (tB, cA, cB, M, N, K, beta, err)


@pytest.mark.parametrize("tA,cA,cB", [(0, 0, 0), (1, 1, 0), (0, 1, 1), (1, 0, 1)])
def test_zgemm_reduction_form(tA, cA, cB):
    # few outputs, long K (the amplitude x integral contractions over three
    # indices); M <= 8, N <= 256; every register-tile size (M <= 2, 4, 8)
    for (M, N, K) in [(1, 1, 1), (2, 21, 5000), (3, 21, 20011), (4, 7, 12345), (7, 48, 3001), (8, 256, 700),
                      (5, 100, 1), (6, 13, 0)]:
        for split in (True, False):
            for beta in (0, 1):
                err = _run(M, N, K, tA, 0, cA, cB, RED, 16, split, beta, seed=M * N + K)
                assert err < 1e-13, (tA, cA, cB, M, N, K, split, beta, err)


@pytest.mark.parametrize("cA,cB", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_zgemm_dot_form(cA, cB):
    # few rows of A against many contiguous rows of B (the ladder over active pairs);
    # M <= 8 (register tiles 2, 4, 8), ragged N (16 rows per workgroup) and K (256 per LDS chunk)
    for (M, N, K) in [(1, 1, 1), (1, 17, 255), (2, 33, 257), (3, 2801, 2800), (4, 100, 1000), (5, 16, 513),
                      (8, 129, 64), (7, 5, 0)]:
        for beta in (0, 1):
            err = _run(M, N, K, 0, 1, cA, cB, DOT, 16, False, beta, seed=M + 3 * N + K)
            assert err < 1e-13, (cA, cB, M, N, K, beta, err)


def test_vector_forms_reject_shapes_they_do_not_fit():
    for (cfg, tA, tB, M, N, K) in [(TALL, 1, 0, 10, 3, 5), (TALL, 0, 0, 10, 3, 65), (TALL, 0, 1, 10, 40, 30),
                                   (RED, 0, 1, 3, 3, 100), (RED, 0, 0, 9, 3, 100), (RED, 1, 0, 3, 257, 100),
                                   (DOT, 0, 0, 3, 3, 100), (DOT, 1, 1, 3, 3, 100), (DOT, 0, 1, 9, 3, 100)]:
        with pytest.raises(Exception):
            _run(M, N, K, tA, tB, 0, 0, cfg, 16, True, 0)

"""Seeded synthetic inputs for the FS-RCCSD hot path (input generation only).

This module is shared by the CPU oracle and by the HIP library's tests and
benchmark.  It contains no coupled-cluster arithmetic: it draws orbital
energies, irrep labels and antisymmetrized Hermitian two-electron integrals
<pq||rs> (the V of Eq. (1)), and lays the integrals out as dense blocks per
allowed irrep tuple (the block partition of the symmetry-handling section).

Recipe (one system):
  * occupied energies  ~ U[-2.0, -0.5] Eh, virtual ~ U[0.2, 3.0] Eh, each
    sorted ascending; global spinor index = occupied ascending, then virtual.
  * irreps: Z_n labels.  Occupied and virtual counts per irrep are drawn
    separately from Dirichlet(1,...,1) and rounded by largest remainder;
    labels are assigned by a random permutation of the label multiset, so
    irreps interleave in energy.  Zero-size irreps can occur.
  * integrals: see fsgen.c (counter-based SplitMix64 + Box-Muller, projected
    onto antisymmetric-Hermitian tensors, zero outside allowed blocks).
  * ε, splits and permutations use numpy PCG64 (default_rng(seed)).

Integral classes (the six that generate all others by antisymmetry and
Hermiticity): OOOO <ij||kl>, OOOV <ij||ka>, OOVV <ij||ab>, OVOV <ia||jb>,
OVVV <ia||bc>, VVVV <ab||cd>.  A class buffer concatenates, over allowed
(g1, g2, g3) in lexicographic order with g4 = (g1 + g2 - g3) mod n, the dense
row-major blocks [n_X1(g1)][n_X2(g2)][n_X3(g3)][n_X4(g4)], spinors inside an
irrep in ascending global index.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsgen.c")
_LIB = os.path.join(_HERE, "libfsgen.so")
_lib = None

CLASSES = ("OOOO", "OOOV", "OOVV", "OVOV", "OVVV", "VVVV")


def build(force: bool = False) -> str:
    """Compile libfsgen.so with gcc + OpenMP (plain C, host only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _get_lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.fsgen_block.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_int, ip, ctypes.c_int,
                                    ip, ctypes.c_int, ip, ctypes.c_int, ip, ctypes.c_int, ip, ctypes.c_int, dp]
        lib.fsgen_block.restype = None
        lib.fsgen_xraw.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, dp]
        lib.fsgen_xraw.restype = None
        lib.fsgen_class_sym.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ip, ctypes.c_int, dp]
        lib.fsgen_class_sym.restype = None
        _lib = lib
    return _lib


@dataclass
class System:
    """One synthetic closed-shell reference (the Fermi vacuum of Eq. (1))."""
    nocc: int
    nvirt: int
    nirrep: int
    sigma: float
    seed: int
    irrep: np.ndarray          # int32 [nocc+nvirt], global index order
    eps: np.ndarray            # float64 [nocc+nvirt]
    nact: int = 0
    active: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))  # global indices
    real: bool = False         # real-double-group stand-in: V = sqrt(2) Re V_complex

    @property
    def n(self) -> int:
        return self.nocc + self.nvirt

    def space(self, X: str) -> np.ndarray:
        """Global indices of space 'O' or 'V'."""
        return np.arange(self.nocc) if X == "O" else np.arange(self.nocc, self.n)

    def members(self, X: str, g: int) -> np.ndarray:
        """Global indices of space X with irrep g, ascending."""
        idx = self.space(X)
        return idx[self.irrep[idx] == g].astype(np.int32)

    def counts(self, X: str) -> np.ndarray:
        idx = self.space(X)
        return np.bincount(self.irrep[idx], minlength=self.nirrep).astype(np.int64)


def _largest_remainder(total: int, p: np.ndarray) -> np.ndarray:
    x = total * p
    c = np.floor(x).astype(np.int64)
    rem = total - int(c.sum())
    if rem > 0:
        order = np.argsort(-(x - c), kind="stable")
        c[order[:rem]] += 1
    return c


def make_system(nocc: int, nvirt: int, nirrep: int, sigma: float, seed: int, nact: int = 0,
                real: bool = False) -> System:
    """real=True: the integrals are sqrt(2) Re of the complex ones -- still
    antisymmetric and now real symmetric (<pq||rs> = <rs||pq>), the case of
    double groups with real irreducible representations; the same element
    variance (sigma^2 / 8) as the complex draw.  Buffers stay complex128 with
    zero imaginary parts (real_buffer() gives the float64 copy)."""
    rng = np.random.default_rng(seed)
    eo = np.sort(rng.uniform(-2.0, -0.5, nocc))
    ev = np.sort(rng.uniform(0.2, 3.0, nvirt))
    if nirrep == 1:
        lo = np.zeros(nocc, np.int32)
        lv = np.zeros(nvirt, np.int32)
    else:
        co = _largest_remainder(nocc, rng.dirichlet(np.ones(nirrep)))
        cv = _largest_remainder(nvirt, rng.dirichlet(np.ones(nirrep)))
        lo = rng.permutation(np.repeat(np.arange(nirrep), co)).astype(np.int32)
        lv = rng.permutation(np.repeat(np.arange(nirrep), cv)).astype(np.int32)
    irrep = np.concatenate([lo, lv]).astype(np.int32)
    eps = np.concatenate([eo, ev]).astype(np.float64)
    # active (0h,1p) set: the nact lowest-energy virtual spinors, whatever their irreps
    active = (nocc + np.arange(min(nact, nvirt))).astype(np.int32)
    return System(nocc, nvirt, nirrep, float(sigma), int(seed), irrep, eps, nact, active, bool(real))


# The paper-shaped synthetic workloads, named by their sizes: a single-irrep
# system, a symmetry-blocked one (Z8) and the production size (Z16, six active
# virtual spinors for the (0h,1p) and (0h,2p) sectors).
WORKLOADS = {
    "o8v24": dict(nocc=8, nvirt=24, nirrep=1, sigma=0.05, seed=1000),
    "o20v120z8": dict(nocc=20, nvirt=120, nirrep=8, sigma=0.05, seed=1001),
    "o40v300z16": dict(nocc=40, nvirt=300, nirrep=16, sigma=0.03, seed=1002, nact=6),
}


def workload_system(name: str) -> System:
    return make_system(**WORKLOADS[name])


def batch_systems(count: int, seed0: int) -> list:
    """Independent systems: nocc ~ U{10..30}, nvirt ~ U{60..200}, irreps ~ U{4..8}."""
    out = []
    for s in range(seed0, seed0 + count):
        r = np.random.default_rng(s)
        nocc = int(r.integers(10, 31))
        nvirt = int(r.integers(60, 201))
        nirr = int(r.integers(4, 9))
        out.append(make_system(nocc, nvirt, nirr, 0.05, s))
    return out


# --------------------------------------------------------------------------
# integral evaluation

def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def block(sysm: System, P, Q, R, S, out: np.ndarray | None = None) -> np.ndarray:
    """Dense complex128 block V[P][Q][R][S] for lists of global indices."""
    lib = _get_lib()
    P, Q, R, S = (np.ascontiguousarray(np.asarray(x, dtype=np.int32)) for x in (P, Q, R, S))
    shape = (len(P), len(Q), len(R), len(S))
    if out is None:
        out = np.empty(shape, np.complex128)
    assert out.dtype == np.complex128 and out.flags.c_contiguous and out.size == int(np.prod(shape))
    if out.size:
        irr = np.ascontiguousarray(sysm.irrep, dtype=np.int32)
        lib.fsgen_block(sysm.seed, sysm.sigma, sysm.n, _iptr(irr), sysm.nirrep,
                        _iptr(P), len(P), _iptr(Q), len(Q), _iptr(R), len(R), _iptr(S), len(S),
                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if sysm.real:
            _make_real(out)
    return out.reshape(shape)


def _make_real(a: np.ndarray) -> None:
    """In place: a <- sqrt(2) Re a (imaginary parts zero)."""
    a.real *= np.sqrt(2.0)
    a.imag = 0.0


def real_buffer(buf: np.ndarray) -> np.ndarray:
    """float64 copy of a class buffer of a real system (for real-arithmetic contexts)."""
    assert not np.any(buf.imag), "not a real system's buffer"
    return np.ascontiguousarray(buf.real)


def xraw(sysm: System, p, q, r, s) -> complex:
    lib = _get_lib()
    o = np.zeros(2)
    lib.fsgen_xraw(sysm.seed, sysm.sigma, sysm.n, p, q, r, s, o.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return complex(o[0], o[1])


def full_tensor(sysm: System) -> np.ndarray:
    """All n^4 elements V[p][q][r][s] (tiny systems only)."""
    idx = np.arange(sysm.n)
    return block(sysm, idx, idx, idx, idx)


def class_tuples(sysm: System, cls: str):
    """Allowed (g1, g2, g3, g4) tuples of a class, in buffer order, with their shapes."""
    n = sysm.nirrep
    cnt = {X: sysm.counts(X) for X in "OV"}
    out = []
    for g1 in range(n):
        for g2 in range(n):
            for g3 in range(n):
                g4 = (g1 + g2 - g3) % n
                shp = (int(cnt[cls[0]][g1]), int(cnt[cls[1]][g2]), int(cnt[cls[2]][g3]), int(cnt[cls[3]][g4]))
                out.append(((g1, g2, g3, g4), shp))
    return out


def class_size(sysm: System, cls: str) -> int:
    return int(sum(int(np.prod(s)) for _, s in class_tuples(sysm, cls)))


def class_buffer(sysm: System, cls: str, out: np.ndarray | None = None):
    """Concatenated full blocks of one class (the boundary format).

    Returns (buffer complex128[size], dict key -> view of shape block)."""
    tuples = class_tuples(sysm, cls)
    total = int(sum(int(np.prod(s)) for _, s in tuples))
    if out is None:
        out = np.empty(total, np.complex128)
    assert out.dtype == np.complex128 and out.size == total and out.flags.c_contiguous
    fast = cls in ("OOOO", "VVVV") and total > 0
    if fast:
        # orbit-based generation (bit-identical to the per-element path)
        X = cls[0]
        base = 0 if X == "O" else sysm.nocc
        sirr = np.ascontiguousarray(sysm.irrep[sysm.space(X)], dtype=np.int32)
        _get_lib().fsgen_class_sym(sysm.seed, sysm.sigma, sysm.n, base, len(sirr), _iptr(sirr), sysm.nirrep,
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if sysm.real:
            _make_real(out)
    views = {}
    off = 0
    for key, shp in tuples:
        sz = int(np.prod(shp))
        v = out[off:off + sz].reshape(shp)
        if sz and not fast:
            block(sysm, sysm.members(cls[0], key[0]), sysm.members(cls[1], key[1]),
                  sysm.members(cls[2], key[2]), sysm.members(cls[3], key[3]), out=v)
        views[key] = v
        off += sz
    return out, views


# --------------------------------------------------------------------------
# device-side generation (same definition, evaluated on the GPU)

_SRC_GPU = os.path.join(_HERE, "fsgen_gpu.hip")
_LIB_GPU = os.path.join(_HERE, "libfsgen_gpu.so")
_lib_gpu = None
_GEN_BLOCK = np.dtype([("off", "<i8"), ("n", "<i4", (4,)), ("mem", "<i4", (4,))], align=True)


def build_gpu(force: bool = False) -> str:
    """Compile libfsgen_gpu.so (hipcc, gfx950)."""
    if force or not os.path.exists(_LIB_GPU) or os.path.getmtime(_LIB_GPU) < os.path.getmtime(_SRC_GPU):
        tmp = _LIB_GPU + ".tmp%d" % os.getpid()
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-Wno-unused-command-line-argument", "-o", tmp, _SRC_GPU],
                              stderr=subprocess.DEVNULL)
        os.replace(tmp, _LIB_GPU)
    return _LIB_GPU


def _get_lib_gpu():
    global _lib_gpu
    if _lib_gpu is None:
        if not os.path.exists(_LIB_GPU):
            raise ImportError(f"{_LIB_GPU} is missing: build it with fsgen.build_gpu()")
        lib = ctypes.CDLL(_LIB_GPU)
        vp = ctypes.c_void_p
        lib.fsgen_gpu_class.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_int, vp, ctypes.c_int, vp,
                                        ctypes.c_int, vp, ctypes.c_int, vp, vp]
        lib.fsgen_gpu_class.restype = ctypes.c_int
        _lib_gpu = lib
    return _lib_gpu


def class_buffer_gpu(sysm: System, cls: str, out=None, stream=None):
    """class_buffer() generated in device memory: returns a torch complex128
    CUDA tensor (or fills `out`).  Values agree with the host generator to a
    few ulps (device transcendental functions)."""
    import torch
    if sysm.real:
        raise ValueError("the device generator draws complex integrals only")
    tuples = class_tuples(sysm, cls)
    total = int(sum(int(np.prod(s)) for _, s in tuples))
    if out is None:
        out = torch.empty(max(total, 1), dtype=torch.complex128, device="cuda")[:total]
    assert out.dtype == torch.complex128 and out.is_cuda and out.is_contiguous() and out.numel() == total
    mem, moff = [], {}
    for X in "OV":
        for g in range(sysm.nirrep):
            moff[(X, g)] = len(mem)
            mem.extend(int(v) for v in sysm.members(X, g))
    blocks = np.zeros(len(tuples), _GEN_BLOCK)
    off = 0
    for k, (key, shp) in enumerate(tuples):
        blocks[k]["off"] = off
        blocks[k]["n"] = shp
        blocks[k]["mem"] = [moff[(cls[i], key[i])] for i in range(4)]
        off += int(np.prod(shp))
    keep = np.array([int(np.prod(s)) > 0 for _, s in tuples], bool)
    blocks = np.ascontiguousarray(blocks[keep])
    mem = np.ascontiguousarray(np.array(mem if mem else [0], np.int32))
    irr = np.ascontiguousarray(sysm.irrep, dtype=np.int32)
    st = stream if stream is not None else torch.cuda.current_stream()
    if total:
        rc = _get_lib_gpu().fsgen_gpu_class(sysm.seed, sysm.sigma, sysm.n, irr.ctypes.data, sysm.nirrep,
                                            blocks.ctypes.data, len(blocks), mem.ctypes.data, len(mem),
                                            out.data_ptr(), st.cuda_stream)
        if rc != 0:
            raise RuntimeError(f"fsgen_gpu_class failed (HIP error {rc})")
    return out

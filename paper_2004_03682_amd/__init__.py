"""MI355X-native FS-RCCSD hot path: thin Python binding of libfscc.so.

Every function here only marshals arguments to the C ABI declared in
include/fscc.h; all computation runs in the library's HIP kernels.  Device
buffers are torch tensors (complex128 -- float64 in a real-arithmetic
context -- on the GPU); torch is used for device
memory and streams only.  There is no CPU fallback: importing the binding
without the built library, or calling it on tensors that are not on a GPU,
raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfscc.so")

FSCC_S00, FSCC_S01, FSCC_S02 = 0, 1, 2
FSCC_FP64, FSCC_SPLIT_FP32, FSCC_SPLIT_BF16, FSCC_REAL_FP64 = 0, 1, 2, 3
PRECISIONS = {"fp64": FSCC_FP64, "split_fp32": FSCC_SPLIT_FP32, "split_bf16": FSCC_SPLIT_BF16,
              "real_fp64": FSCC_REAL_FP64}
CLASSES = ("OOOO", "OOOV", "OOVV", "OVOV", "OVVV", "VVVV")
_STATUS = {0: "OK", -1: "EINVAL", -2: "ESYMM", -3: "ENOMEM", -4: "EHIP", -5: "ESTATE", -6: "ENOCONV"}

_lib = None


class FsccError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fscc {_STATUS.get(status, status)}: {msg}")
        self.status = status


class _System(ctypes.Structure):
    _fields_ = [("nocc", ctypes.c_int32), ("nvirt", ctypes.c_int32), ("nirrep", ctypes.c_int32),
                ("irrep", ctypes.POINTER(ctypes.c_int32)), ("eps", ctypes.POINTER(ctypes.c_double)),
                ("nact", ctypes.c_int32), ("active", ctypes.POINTER(ctypes.c_int32))]


def lib():
    """Load libfscc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, dp, ip = ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        sigs = {
            "fscc_create": ([ctypes.POINTER(_System), ip, vp, ctypes.POINTER(vp)], ip),
            "fscc_set_integrals": ([vp, ip, vp, sz], ip),
            "fscc_layout": ([vp, ip, ctypes.POINTER(sz), ctypes.POINTER(sz)], ip),
            "fscc_build_residual": ([vp, ip, vp, vp, vp, vp], ip),
            "fscc_update_amplitudes": ([vp, ip, vp, vp, vp, vp, dp], ip),
            "fscc_energy": ([vp, vp, vp, dp, dp], ip),
            "fscc_iterate": ([vp, vp, vp, vp, vp, dp, dp, dp], ip),
            "fscc_diis_reset": ([vp, ip, ip], ip),
            "fscc_ladder": ([vp, vp, vp], ip),
            "fscc_work": ([vp, dp, dp, dp], ip),
            "fscc_profile": ([vp, ip], ip),
            "fscc_op_count": ([vp, ctypes.POINTER(ip)], ip),
            "fscc_op_info": ([vp, ip, ctypes.POINTER(ctypes.c_char_p), dp, ctypes.POINTER(ip), dp], ip),
            "fscc_op_traffic": ([vp, ip, ctypes.POINTER(ip), dp], ip),
            "fscc_op_run": ([vp, ip, ip], ip),
            "fscc_prepare_sector": ([vp, ip, vp, vp], ip),
            "fscc_heff": ([vp, vp, vp, vp], ip),
            "fscc_heff2": ([vp, vp, vp], ip),
            "fscc_precondition": ([vp, ip, ip, ctypes.c_double], ip),
            "fscc_denominators": ([vp, ip, vp, vp], ip),
            "fscc_autotune": ([vp, ip], ip),
            "fscc_gemm_config": ([vp, ip, ctypes.POINTER(ip), ctypes.POINTER(ip), ctypes.POINTER(ip)], ip),
            "fscc_zgemm": ([ip] * 9 + [vp, ip, vp, ip, vp, ip, ctypes.c_double, ctypes.c_double, ip, ip, vp], ip),
            "fscc_zgemm_noalloc": ([ip] * 9 + [vp, ip, vp, ip, vp, ip, ctypes.c_double, ctypes.c_double, ip, ip, vp], ip),
            "fscc_set_precision": ([vp, ip], ip),
            "fscc_profile_select": ([vp, ip], ip),
            "fscc_level_shift": ([vp, ip, ctypes.c_double], ip),
            "fscc_gather_order": ([vp, ip], ip),
            "fscc_vvvv_out_of_core": ([vp, sz], ip),
            "fscc_dgemm": ([ip, ip, ip, ip, ip, ip, ip, vp, ip, vp, ip, vp, ip, ctypes.c_double, ip, ip, vp], ip),
            "fscc_dynamic_shift": ([vp, ip, ctypes.c_double, ip], ip),
            "fscc_pade": ([ip, vp, vp, ip, ip, ctypes.c_double, vp], ip),
            "fscc_heff_eig": ([ip, vp, vp], ip),
            "fscc_set_validation": ([vp, ip], ip),
            "fscc_set_streams": ([vp, ip], ip),
            "fscc_tune_cache": ([vp, ctypes.c_char_p], ip),
            "fscc_autotune_cached": ([vp, ctypes.POINTER(ip)], ip),
            "fscc_get_precision": ([vp, ctypes.POINTER(ip)], ip),
            "fscc_mixed_config": ([vp, ip, ctypes.POINTER(ip)], ip),
            "fscc_zgemm_split": ([ip] * 9 + [vp, ip, vp, ip, vp, ip, ctypes.c_double, ctypes.c_double, ip, vp], ip),
            "fscc_batch_create": ([ctypes.POINTER(_System), ip, ip, vp, ctypes.POINTER(vp)], ip),
            "fscc_batch_destroy": ([vp], None),
            "fscc_batch_last_error": ([vp], ctypes.c_char_p),
            "fscc_batch_sizes": ([vp, ctypes.POINTER(sz), ctypes.POINTER(sz)], ip),
            "fscc_batch_segment": ([vp, ip] + [ctypes.POINTER(sz)] * 4, ip),
            "fscc_batch_set_integrals": ([vp, ip, ip, vp, sz], ip),
            "fscc_batch_reset": ([vp, ip, ctypes.c_double, ctypes.c_double], ip),
            "fscc_batch_build_residual": ([vp, vp, vp, vp, vp], ip),
            "fscc_batch_step": ([vp, vp, vp, vp, vp, ip, dp], ip),
            "fscc_batch_context": ([vp], vp),
            "fscc_batch_denominators": ([vp, vp, vp], ip),
            "fscc_batch_restart": ([vp, vp], ip),
            "fscc_probe_mfma": ([ip, ip, vp, vp, vp], ip),
            "fscc_batch_precondition": ([vp, ip, ctypes.c_double], ip),
            "fscc_batch_maxnorm": ([vp, vp, vp, dp], ip),
            "fscc_mlp_num_params": ([ctypes.POINTER(sz)], ip),
            "fscc_mlp_create": ([ctypes.c_uint64, vp, ctypes.POINTER(vp)], ip),
            "fscc_mlp_destroy": ([vp], None),
            "fscc_mlp_last_error": ([vp], ctypes.c_char_p),
            "fscc_mlp_set_params": ([vp, vp, sz], ip),
            "fscc_mlp_get_params": ([vp, vp, sz], ip),
            "fscc_mlp_get_grad": ([vp, vp, sz], ip),
            "fscc_ws_features": ([vp, vp, vp, sz, vp, vp], ip),
            "fscc_mlp_forward": ([vp, vp, sz, vp], ip),
            "fscc_ws_apply": ([vp, vp, vp, vp, sz, vp, vp], ip),
            "fscc_ws_step": ([vp, vp, vp, sz, vp, vp], ip),
            "fscc_ws_gather": ([vp, sz, vp, sz, vp, vp], ip),
            "fscc_mlp_loss_grad": ([vp, vp, vp, vp, vp, vp, sz, ip, dp], ip),
            "fscc_mlp_adam": ([vp, ctypes.c_float], ip),
            "fscc_destroy": ([vp], None),
            "fscc_last_error": ([vp], ctypes.c_char_p),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _prec(p):
    if isinstance(p, str):
        if p not in PRECISIONS:
            raise ValueError(f"unknown precision {p!r}")
        return PRECISIONS[p]
    return int(p)


def _ptr(t, dtype=None):
    """Device pointer of a contiguous GPU tensor of any dtype (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise TypeError("fscc expects contiguous GPU tensors")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _dev_ptr(t, n=None, dtype=None):
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("fscc expects GPU tensors")
    want = torch.complex128 if dtype is None else dtype
    if t.dtype != want or not t.is_contiguous():
        raise TypeError(f"fscc expects contiguous {want} tensors")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One system (fscc_create ... fscc_destroy)."""

    def __init__(self, nocc, nvirt, nirrep, irrep, eps, stream=None, active=(), precision="fp64"):
        import numpy as np
        import torch
        L = lib()
        self._irrep = np.ascontiguousarray(irrep, dtype=np.int32)
        self._eps = np.ascontiguousarray(eps, dtype=np.float64)
        self._act = np.ascontiguousarray(active, dtype=np.int32)
        s = _System(int(nocc), int(nvirt), int(nirrep),
                    self._irrep.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    self._eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    len(self._act), self._act.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        st = L.fscc_create(ctypes.byref(s), _prec(precision), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise FsccError(st, "fscc_create failed")
        self._h = h
        self.real = _prec(precision) == FSCC_REAL_FP64
        self.dtype = torch.float64 if self.real else torch.complex128
        self.n1, self.n2 = self.layout(FSCC_S00)
        self.nact = len(self._act)
        self.m1, self.m2 = self.layout(FSCC_S01) if self.nact else (0, 0)
        self.npair = self.nact * (self.nact - 1) // 2
        self.p2 = self.layout(FSCC_S02)[1] if self.nact >= 2 else 0

    def _d(self, t, n=None):
        """Device pointer of an amplitude / residual / integral tensor of this
        context (complex128, or float64 in a real context)."""
        return _dev_ptr(t, n, self.dtype)

    def _sizes(self, sector):
        if sector == FSCC_S02:
            return (0, self.p2)
        return (self.n1, self.n2) if sector == FSCC_S00 else (self.m1, self.m2)

    @classmethod
    def from_system(cls, sysm, stream=None, precision="fp64"):
        return cls(sysm.nocc, sysm.nvirt, sysm.nirrep, sysm.irrep, sysm.eps, stream, getattr(sysm, "active", ()),
                   precision)

    def level_shift(self, shift, sector=FSCC_S00):
        """Jacobi step R / (D - shift) for the sector (damping; same fixed point)."""
        self._check(lib().fscc_level_shift(self._h, sector, float(shift)))

    def vvvv_out_of_core(self, staging_bytes):
        """Move the packed VVVV integrals to pinned host memory and stream them
        through two device staging buffers (staging_bytes in total); 0 moves
        them back to device memory."""
        self._check(lib().fscc_vvvv_out_of_core(self._h, int(staging_bytes)))

    def dynamic_shift(self, S, n=3, sector=FSCC_S01):
        """Dynamic denominator shifts Delta = S (S/(min(D,0)+S))^n of the sector
        (S < 0; S = 0 switches them off): the solved equations become R = Delta s."""
        self._check(lib().fscc_dynamic_shift(self._h, sector, float(S), int(n)))

    def set_precision(self, precision):
        """'fp64', 'split_bf16' or 'split_fp32' for the ladder and ring contractions."""
        self._check(lib().fscc_set_precision(self._h, _prec(precision)))

    def precision(self):
        p = ctypes.c_int()
        self._check(lib().fscc_get_precision(self._h, ctypes.byref(p)))
        return {v: k for k, v in PRECISIONS.items()}[p.value]

    def mixed_configs(self):
        """[(op name, split tile cfg id)] for the operations running in split precision now."""
        out = []
        for k, o in enumerate(self.op_times()):
            c = ctypes.c_int()
            self._check(lib().fscc_mixed_config(self._h, k, ctypes.byref(c)))
            if c.value >= 0:
                out.append((o["name"], c.value))
        return out

    def _check(self, st):
        if st != 0:
            msg = lib().fscc_last_error(self._h)
            raise FsccError(st, msg.decode() if msg else "")

    def set_validation(self, nsample):
        """Sampled symmetry checks per integral class at set_integrals (0 = off)."""
        self._check(lib().fscc_set_validation(self._h, int(nsample)))

    def set_streams(self, n):
        """Residual operations on one stream (1) or on two overlapping streams (2)."""
        self._check(lib().fscc_set_streams(self._h, int(n)))

    def set_integrals(self, cls, dev_blocks):
        k = CLASSES.index(cls) if isinstance(cls, str) else int(cls)
        self._check(lib().fscc_set_integrals(self._h, k, self._d(dev_blocks), dev_blocks.numel()))

    def layout(self, sector=FSCC_S00):
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(lib().fscc_layout(self._h, sector, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def build_residual(self, t1, t2, r1, r2, sector=FSCC_S00):
        a, b = self._sizes(sector)
        self._check(lib().fscc_build_residual(self._h, sector, self._d(t1, a), self._d(t2, b),
                                              self._d(r1, a), self._d(r2, b)))

    def update_amplitudes(self, t1, t2, r1, r2, sector=FSCC_S00):
        a, b = self._sizes(sector)
        m = ctypes.c_double()
        self._check(lib().fscc_update_amplitudes(self._h, sector, self._d(t1, a), self._d(t2, b),
                                                 self._d(r1, a), self._d(r2, b), ctypes.byref(m)))
        return m.value

    def prepare_sector(self, t1, t2, sector=FSCC_S01):
        """FSCC_S01: t1, t2 = converged (0h,0p) amplitudes; FSCC_S02: the converged
        (0h,1p) amplitudes s1, s2 (after the (0h,1p) preparation)."""
        a, b = (self.m1, self.m2) if sector == FSCC_S02 else (self.n1, self.n2)
        self._check(lib().fscc_prepare_sector(self._h, sector, self._d(t1, a), self._d(t2, b)))

    def precondition(self, mode=1, floor=0.1, sector=FSCC_S01):
        self._check(lib().fscc_precondition(self._h, sector, int(mode), float(floor)))

    def denominators(self):
        """(D1, D2): the (0h,0p) Jacobi denominators in use (float64 device tensors)."""
        import torch
        D1 = torch.empty(max(self.n1, 1), dtype=torch.float64, device="cuda")[:self.n1]
        D2 = torch.empty(max(self.n2, 1), dtype=torch.float64, device="cuda")[:self.n2]
        self._check(lib().fscc_denominators(self._h, FSCC_S00, _ptr(D1), _ptr(D2)))
        return D1, D2

    def heff(self, s1, s2):
        """H_eff[y][x] (numpy complex, nact x nact, rows/columns in the order of the active list)."""
        import numpy as np
        out = np.zeros((self.nact, self.nact), np.complex128)
        self._check(lib().fscc_heff(self._h, self._d(s1, self.m1), self._d(s2, self.m2),
                                    out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def heff2(self, s):
        """(0h,2p) H_eff[pair(zw)][pair(xy)] (numpy complex, P x P over the pairs i < j of
        positions in the active list, row-major upper triangle)."""
        import numpy as np
        out = np.zeros((self.npair, self.npair), np.complex128)
        self._check(lib().fscc_heff2(self._h, self._d(s, self.p2), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def iterate(self, t1, t2, r1, r2):
        """One (0h,0p) iteration (residual, update, energy) with one synchronisation:
        returns (max|step|, E)."""
        d, er, ei = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(lib().fscc_iterate(self._h, self._d(t1, self.n1), self._d(t2, self.n2), self._d(r1, self.n1),
                                       self._d(r2, self.n2), ctypes.byref(d), ctypes.byref(er), ctypes.byref(ei)))
        return d.value, complex(er.value, ei.value)

    def energy(self, t1, t2):
        er, ei = ctypes.c_double(), ctypes.c_double()
        self._check(lib().fscc_energy(self._h, self._d(t1, self.n1), self._d(t2, self.n2),
                                      ctypes.byref(er), ctypes.byref(ei)))
        return complex(er.value, ei.value)

    def diis_reset(self, ndiis=6, sector=FSCC_S00):
        self._check(lib().fscc_diis_reset(self._h, sector, int(ndiis)))

    def ladder(self, tau, out):
        self._check(lib().fscc_ladder(self._h, self._d(tau, self.n2), self._d(out, self.n2)))

    def work(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(lib().fscc_work(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(gemm_flops=a.value, ladder_flops=b.value, ladder_bytes=c.value)

    def profile(self, enable=True, only=None):
        """Per-operation HIP-event timing; only = an operation name (or index)
        times that operation alone."""
        k = -1
        if only is not None:
            k = only if isinstance(only, int) else self.op_index(only)
        self._check(lib().fscc_profile_select(self._h, int(k)))
        self._check(lib().fscc_profile(self._h, 1 if enable else 0))

    def op_index(self, name):
        n = ctypes.c_int()
        self._check(lib().fscc_op_count(self._h, ctypes.byref(n)))
        for k in range(n.value):
            nm, ms, calls, fl = ctypes.c_char_p(), ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
            self._check(lib().fscc_op_info(self._h, k, ctypes.byref(nm), ctypes.byref(ms), ctypes.byref(calls),
                                           ctypes.byref(fl)))
            if nm.value.decode() == name:
                return k
        raise KeyError(name)

    def op_times(self):
        n = ctypes.c_int()
        self._check(lib().fscc_op_count(self._h, ctypes.byref(n)))
        out = []
        for k in range(n.value):
            nm, ms, calls, fl = ctypes.c_char_p(), ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
            self._check(lib().fscc_op_info(self._h, k, ctypes.byref(nm), ctypes.byref(ms), ctypes.byref(calls),
                                           ctypes.byref(fl)))
            kind, by = ctypes.c_int(), ctypes.c_double()
            self._check(lib().fscc_op_traffic(self._h, k, ctypes.byref(kind), ctypes.byref(by)))
            out.append(dict(name=nm.value.decode(), ms=ms.value, calls=calls.value, flops=fl.value,
                            kind=("reorder", "gemm", "elementwise")[kind.value], bytes=by.value))
        return out

    def tune_cache(self, path):
        """Autotune result cache file (None: off)."""
        self._check(lib().fscc_tune_cache(self._h, None if path is None else str(path).encode()))

    def autotune_cached(self):
        """True if the last autotune applied cached choices instead of timing."""
        v = ctypes.c_int()
        self._check(lib().fscc_autotune_cached(self._h, ctypes.byref(v)))
        return bool(v.value)

    def op_run(self, k, reps=1):
        """Run operation k alone reps times (after one residual evaluation of its sector)."""
        self._check(lib().fscc_op_run(self._h, int(k), int(reps)))

    def autotune(self, level=1):
        self._check(lib().fscc_autotune(self._h, int(level)))

    def gather_order(self, tiled):
        """Reorders in destination storage order (0) or by 16 x 16 destination tiles (1)."""
        self._check(lib().fscc_gather_order(self._h, int(tiled)))

    def gemm_config(self, k):
        """(tile cfg id with the 3M / DB flags, bk, split) of operation k (cfg -1: not a GEMM)."""
        c, b, sp = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(lib().fscc_gemm_config(self._h, int(k), ctypes.byref(c), ctypes.byref(b), ctypes.byref(sp)))
        return c.value, b.value, sp.value

    def gemm_configs(self):
        """[(op name, tile cfg id, bk, split)] for every GEMM operation."""
        out = []
        for k, o in enumerate(self.op_times()):
            c, b, sp = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            self._check(lib().fscc_gemm_config(self._h, k, ctypes.byref(c), ctypes.byref(b), ctypes.byref(sp)))
            if c.value >= 0:
                out.append((o["name"], c.value, b.value, sp.value))
        return out

    def destroy(self):
        if getattr(self, "_h", None):
            lib().fscc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def solve01(ctx, s1, s2, tol=1e-10, maxit=200, ndiis=6, log=None):
    """(0h,1p) Jacobi + DIIS iterations (after ctx.prepare_sector(t1, t2)).
    Returns dict(heff, eig (sorted by real part), iters, converged)."""
    import numpy as np
    import torch
    r1 = torch.empty_like(s1)
    r2 = torch.empty_like(s2)
    ctx.diis_reset(ndiis, FSCC_S01)
    converged = False
    k = 0
    for k in range(1, maxit + 1):
        ctx.build_residual(s1, s2, r1, r2, FSCC_S01)
        dmax = ctx.update_amplitudes(s1, s2, r1, r2, FSCC_S01)
        if log:
            log(f"(0h,1p) iter {k:3d}  max|step| = {dmax:.3e}")
        if dmax < tol:
            converged = True
            break
    h = ctx.heff(s1, s2)
    return dict(heff=h, eig=heff_eig(h), iters=k, converged=converged)


def solve02(ctx, s, tol=1e-10, maxit=200, ndiis=6, log=None):
    """(0h,2p) Jacobi + DIIS iterations on s_xy^ab (after ctx.prepare_sector(s1, s2,
    FSCC_S02)).  Returns dict(heff, eig (sorted by real part), iters, converged)."""
    import numpy as np
    import torch
    r = torch.empty_like(s)
    ctx.diis_reset(ndiis, FSCC_S02)
    converged = False
    k = 0
    for k in range(1, maxit + 1):
        ctx.build_residual(None, s, None, r, FSCC_S02)
        dmax = ctx.update_amplitudes(None, s, None, r, FSCC_S02)
        if log:
            log(f"(0h,2p) iter {k:3d}  max|step| = {dmax:.3e}")
        if dmax < tol:
            converged = True
            break
    h = ctx.heff2(s)
    return dict(heff=h, eig=heff_eig(h), iters=k, converged=converged)


def heff_eig(h):
    """Eigenvalues of a square complex matrix (H_eff) sorted by real part, then
    imaginary part (fscc_heff_eig, host code of the library)."""
    import numpy as np
    a = np.ascontiguousarray(h, dtype=np.complex128)
    if a.ndim != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("heff_eig needs a square matrix")
    n = a.shape[0]
    out = np.zeros(n, dtype=np.complex128)
    r = lib().fscc_heff_eig(int(n), a.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p))
    if r != 0:
        raise FsccError(r, "fscc_heff_eig failed")
    return out


PROBE_KINDS = {"fp64": 0, "bf16": 1, "fp32": 2}


def probe_mfma(kind="fp64", iters=4096, stream=None):
    """Measured matrix-core throughput of this GPU (fscc_probe_mfma): kind
    'fp64', 'bf16' or 'fp32'; returns (TFLOP/s, ms of the timed launch)."""
    tf, ms = ctypes.c_double(), ctypes.c_double()
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    r = lib().fscc_probe_mfma(PROBE_KINDS[kind], int(iters), st, ctypes.byref(tf), ctypes.byref(ms))
    if r != 0:
        raise FsccError(r, "fscc_probe_mfma failed")
    return tf.value, ms.value


def pade(x, y, L, M, x0=0.0):
    """Value at x0 of the [L/M] Pade approximant fitted to (x[i], y[i]) (fscc_pade)."""
    import numpy as np
    xs = np.ascontiguousarray(x, dtype=np.float64)
    ys = np.ascontiguousarray(y, dtype=np.complex128)
    if xs.shape != ys.shape or xs.ndim != 1:
        raise ValueError("x and y must be 1-D of equal length")
    out = np.zeros(1, dtype=np.complex128)
    r = lib().fscc_pade(int(xs.size), xs.ctypes.data_as(ctypes.c_void_p), ys.ctypes.data_as(ctypes.c_void_p),
                        int(L), int(M), float(x0), out.ctypes.data_as(ctypes.c_void_p))
    if r != 0:
        raise FsccError(r, "fscc_pade failed")
    return complex(out[0])


def solve01_extrapolated(ctx, s1, s2, S, n=3, scales=(1.0, 0.8, 0.6, 0.4), L=1, M=1, tol=1e-10, maxit=200,
                         ndiis=6, log=None):
    """(0h,1p) sector solved with dynamic shifts lambda*S for each lambda in
    `scales` (each solve starts from the previous amplitudes), then every
    state energy (sorted by real part) extrapolated to lambda = 0 by an [L/M]
    Pade approximant.  Returns dict(scales, eig (per scale), iters,
    converged, extrapolated).  The shift is switched off afterwards."""
    import numpy as np
    eigs, iters, conv = [], [], []
    try:
        for lam in scales:
            ctx.dynamic_shift(lam * S, n, FSCC_S01)
            r = solve01(ctx, s1, s2, tol=tol, maxit=maxit, ndiis=ndiis, log=log)
            eigs.append(r["eig"])
            iters.append(r["iters"])
            conv.append(r["converged"])
    finally:
        ctx.dynamic_shift(0.0, n, FSCC_S01)
    ext = None
    if all(conv) and len(scales) >= L + M + 1:
        E = np.array(eigs)
        ext = np.array([pade(scales, E[:, k], L, M, 0.0) for k in range(E.shape[1])])
    return dict(scales=list(scales), eig=eigs, iters=iters, converged=conv, extrapolated=ext)


def solve(ctx, t1, t2, tol=1e-10, maxit=200, ndiis=6, log=None, reset_diis=True, dressed=0, floor=0.1):
    """Jacobi + DIIS iterations on the device until max|step| < tol.

    Each iteration: fscc_build_residual -> fscc_update_amplitudes ->
    fscc_energy.  Returns dict(E, iters, converged, history); history entries
    carry the host time after the iteration's energy (which synchronises).
    reset_diis=False continues with the context's current DIIS subspace (and
    denominators).  dressed=m > 0: dressed Jacobi denominators
    (fscc_precondition, mode 1) from iteration 3 on, taken from the residual of
    the iteration before and refreshed every m iterations; 0: the bare ones."""
    import time
    import torch
    r1 = torch.empty_like(t1)
    r2 = torch.empty_like(t2)
    if reset_diis:
        ctx.precondition(0, floor, FSCC_S00)
        ctx.diis_reset(ndiis)
    hist = []
    E = 0j
    converged = False
    k = 0
    for k in range(1, maxit + 1):
        if dressed and k >= 3 and (k - 3) % dressed == 0:
            ctx.precondition(1, floor, FSCC_S00)     # from the residual of iteration k - 1
        dmax, E = ctx.iterate(t1, t2, r1, r2)
        hist.append(dict(iter=k, E=E, dmax=dmax, time=time.perf_counter()))
        if log:
            log(f"iter {k:3d}  E = {E.real:+.14f} {E.imag:+.3e}i  max|step| = {dmax:.3e}")
        if dmax < tol:
            converged = True
            break
    return dict(E=E, iters=k, converged=converged, history=hist)


def solve_mixed(ctx, t1, t2, switch_tol=1e-6, tol=1e-10, maxit=200, ndiis=6, log=None, keep_diis=True, dressed=0,
                floor=0.1):
    """Two-stage solve: iterate with the context's split precision until
    max|step| < switch_tol, then continue in FP64 to tol (keeping the DIIS
    subspace and denominators unless keep_diis=False).  dressed as in solve().
    The context's precision is restored on return.  Returns dict(E, iters,
    split_iters, fp64_iters, converged, history)."""
    prec = ctx.precision()
    try:
        a = solve(ctx, t1, t2, tol=switch_tol, maxit=maxit, ndiis=ndiis, log=log, dressed=dressed, floor=floor)
        ctx.set_precision("fp64")
        b = solve(ctx, t1, t2, tol=tol, maxit=maxit, ndiis=ndiis, log=log, reset_diis=not keep_diis, dressed=dressed,
                  floor=floor)
    finally:
        ctx.set_precision(prec)
    return dict(E=b["E"], iters=a["iters"] + b["iters"], split_iters=a["iters"], fp64_iters=b["iters"],
                converged=b["converged"], history=a["history"] + b["history"])


def zgemm(A, B, C, M, N, K, lda, ldb, ldc, tA=False, tB=False, cA=False, cB=False, alpha=1.0, beta=0,
          cfg=-1, bk=16, allow_split=True, stream=None):
    """One complex GEMM through the library's grouped MFMA kernel (fscc_zgemm)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    alpha = complex(alpha)
    r = lib().fscc_zgemm(int(cfg), int(bk), int(tA), int(tB), int(cA), int(cB), int(M), int(N), int(K),
                         _dev_ptr(A), int(lda), _dev_ptr(B), int(ldb), _dev_ptr(C), int(ldc), alpha.real, alpha.imag,
                         int(beta), int(allow_split), ctypes.c_void_p(st.cuda_stream))
    if r != 0:
        raise FsccError(r, "fscc_zgemm failed: " + lib().fscc_last_error(None).decode())


def zgemm_noalloc(A, B, C, M, N, K, lda, ldb, ldc, tA=False, tB=False, cA=False, cB=False, alpha=1.0, beta=0,
                  cfg=-1, bk=16, allow_split=True, stream=None):
    """fscc_zgemm_noalloc: zgemm() with its tables and split-K partial sums in the
    library's static device array (no device allocation)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    alpha = complex(alpha)
    r = lib().fscc_zgemm_noalloc(int(cfg), int(bk), int(tA), int(tB), int(cA), int(cB), int(M), int(N), int(K),
                                 _dev_ptr(A), int(lda), _dev_ptr(B), int(ldb), _dev_ptr(C), int(ldc), alpha.real,
                                 alpha.imag, int(beta), int(allow_split), ctypes.c_void_p(st.cuda_stream))
    if r != 0:
        raise FsccError(r, "fscc_zgemm_noalloc failed: " + lib().fscc_last_error(None).decode())


def dgemm(A, B, C, M, N, K, lda, ldb, ldc, tA=False, tB=False, alpha=1.0, beta=0, cfg=-1, bk=16, allow_split=True,
          stream=None):
    """One real GEMM through the library's real-arithmetic kernels (fscc_dgemm)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    r = lib().fscc_dgemm(int(cfg), int(bk), int(tA), int(tB), int(M), int(N), int(K),
                         _dev_ptr(A, dtype=torch.float64), int(lda), _dev_ptr(B, dtype=torch.float64), int(ldb),
                         _dev_ptr(C, dtype=torch.float64), int(ldc), float(alpha), int(beta), int(allow_split),
                         ctypes.c_void_p(st.cuda_stream))
    if r != 0:
        raise FsccError(r, "fscc_dgemm failed")


def zgemm_split(A, B, C, M, N, K, lda, ldb, ldc, precision="split_bf16", cfg=0, tA=False, tB=False, cA=False,
                cB=False, alpha=1.0, beta=0, stream=None):
    """One complex GEMM through the split-precision kernel (fscc_zgemm_split)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    alpha = complex(alpha)
    r = lib().fscc_zgemm_split(_prec(precision), int(cfg), int(tA), int(tB), int(cA), int(cB), int(M), int(N), int(K),
                               _dev_ptr(A), int(lda), _dev_ptr(B), int(ldb), _dev_ptr(C), int(ldc), alpha.real,
                               alpha.imag, int(beta), ctypes.c_void_p(st.cuda_stream))
    if r != 0:
        raise FsccError(r, "fscc_zgemm_split failed")


def _system_struct(sysm, keep):
    import numpy as np
    irr = np.ascontiguousarray(sysm.irrep, dtype=np.int32)
    eps = np.ascontiguousarray(sysm.eps, dtype=np.float64)
    act = np.ascontiguousarray(getattr(sysm, "active", ()), dtype=np.int32)
    keep += [irr, eps, act]
    return _System(int(sysm.nocc), int(sysm.nvirt), int(sysm.nirrep),
                   irr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   eps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(act),
                   act.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))


class _ContextView(Context):
    """Introspection view (profile, op times, autotune, GEMM configs) of a batch's executor."""

    def __init__(self, handle):
        import torch
        self._h = handle
        self.real = False
        self.dtype = torch.complex128

    def destroy(self):
        self._h = None


class Batch:
    """Many independent (0h,0p) systems in grouped launches (fscc_batch_*)."""

    REPORT = ("E_re", "E_im", "max_step", "active", "iters", "failed")

    def __init__(self, systems, stream=None, precision="fp64"):
        import torch
        L = lib()
        keep = []
        arr = (_System * len(systems))(*[_system_struct(s, keep) for s in systems])
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.nsys = len(systems)
        h = ctypes.c_void_p()
        st = L.fscc_batch_create(arr, len(systems), _prec(precision), ctypes.c_void_p(stream.cuda_stream),
                                 ctypes.byref(h))
        if st != 0:
            raise FsccError(st, "fscc_batch_create failed")
        self._h = h
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(L.fscc_batch_sizes(self._h, ctypes.byref(a), ctypes.byref(b)))
        self.n1, self.n2 = a.value, b.value
        self.segments = []
        for k in range(self.nsys):
            v = [ctypes.c_size_t() for _ in range(4)]
            self._check(L.fscc_batch_segment(self._h, k, *[ctypes.byref(x) for x in v]))
            self.segments.append(tuple(x.value for x in v))   # off1, n1, off2, n2

    def _check(self, st):
        if st != 0:
            msg = lib().fscc_batch_last_error(self._h)
            raise FsccError(st, msg.decode() if msg else "")

    def set_integrals(self, s, cls, dev_blocks):
        k = CLASSES.index(cls) if isinstance(cls, str) else int(cls)
        self._check(lib().fscc_batch_set_integrals(self._h, int(s), k, _dev_ptr(dev_blocks), dev_blocks.numel()))

    def reset(self, ndiis=6, tol=1e-10, shift=0.0):
        self._check(lib().fscc_batch_reset(self._h, int(ndiis), float(tol), float(shift)))

    def build_residual(self, t1, t2, r1, r2):
        self._check(lib().fscc_batch_build_residual(self._h, _dev_ptr(t1, self.n1), _dev_ptr(t2, self.n2),
                                                    _dev_ptr(r1, self.n1), _dev_ptr(r2, self.n2)))

    def step(self, t1, t2, r1, r2, use_graph=False):
        """One iteration of every active system; returns a numpy [nsys, 6] report
        (E_re, E_im, max_step, active, iters, failed)."""
        import numpy as np
        rep = np.zeros((self.nsys, 6))
        self._check(lib().fscc_batch_step(self._h, _dev_ptr(t1, self.n1), _dev_ptr(t2, self.n2),
                                          _dev_ptr(r1, self.n1), _dev_ptr(r2, self.n2), 1 if use_graph else 0,
                                          rep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return rep

    def context(self):
        return _ContextView(ctypes.c_void_p(lib().fscc_batch_context(self._h)))

    def precondition(self, mode=1, floor=0.1):
        """Jacobi denominators of every system: 0 bare, 1 dressed (after a step)."""
        self._check(lib().fscc_batch_precondition(self._h, int(mode), float(floor)))

    def restart(self, mask):
        """Fresh DIIS subspace for the systems where mask is true."""
        import numpy as np
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.int32))
        assert m.size == self.nsys
        self._check(lib().fscc_batch_restart(self._h, m.ctypes.data))

    def denominators(self):
        """(D1, D2) float64 device tensors of the concatenated layouts."""
        import torch
        D1 = torch.empty(max(self.n1, 1), dtype=torch.float64, device="cuda")[:self.n1]
        D2 = torch.empty(max(self.n2, 1), dtype=torch.float64, device="cuda")[:self.n2]
        self._check(lib().fscc_batch_denominators(self._h, _ptr(D1), _ptr(D2)))
        return D1, D2

    def maxnorm(self, r1, r2):
        """Per-system max |r / D| (numpy [nsys])."""
        import numpy as np
        out = np.zeros(self.nsys)
        self._check(lib().fscc_batch_maxnorm(self._h, _dev_ptr(r1, self.n1), _dev_ptr(r2, self.n2),
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def split(self, t, part):
        """Per-system views of a concatenated vector (part 1: T1, 2: T2)."""
        return [t[(g[0] if part == 1 else g[2]):(g[0] + g[1] if part == 1 else g[2] + g[3])] for g in self.segments]

    def destroy(self):
        if getattr(self, "_h", None):
            lib().fscc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def solve_batch(batch, t1, t2, tol=1e-10, maxit=200, ndiis=6, use_graph=True, log=None, shift=0.0, reset=True,
                first=None, dressed=0, floor=0.1, stop_active=0):
    """Iterate every system of a batch until each one's max|step| < tol.
    dressed=m > 0: dressed Jacobi denominators (fscc_batch_precondition) from
    iteration 3 on, taken from the residual of the iteration before and
    refreshed every m iterations (the rule of solve()).  stop_active=n > 0:
    return as soon as at most n systems are still iterating (their converged
    flag is then False; see finish_batch_in_contexts).
    Returns dict(E [complex per system], iters, converged, failed, history
    (list of reports), times (host time after each iteration))."""
    import time
    import numpy as np
    import torch
    r1 = torch.empty_like(t1)
    r2 = torch.empty_like(t2)
    if reset:
        batch.precondition(0, floor)
        batch.reset(ndiis, tol, shift)
    hist, times = [], []
    rep = None
    if first is not None:            # reports of iterations already taken
        hist.extend(first)
        times.extend([time.perf_counter()] * len(first))
        rep = first[-1]
    for k in range(len(hist) + 1, maxit + 1):
        if rep is not None and not rep[:, 3].any():
            break
        if dressed and k >= 3 and (k - 3) % dressed == 0:
            batch.precondition(1, floor)             # from the residual of iteration k - 1
        rep = batch.step(t1, t2, r1, r2, use_graph)
        hist.append(rep)
        times.append(time.perf_counter())
        if log:
            log(f"batch iter {k:3d}: active {int(rep[:, 3].sum())}/{batch.nsys}, max|step| {rep[:, 2].max():.3e}")
        if not rep[:, 3].any() or (stop_active and rep[:, 3].sum() <= stop_active):
            break
    E = rep[:, 0] + 1j * rep[:, 1]
    return dict(E=E, iters=rep[:, 4].astype(int), converged=(rep[:, 3] == 0) & (rep[:, 5] == 0),
                failed=rep[:, 5] != 0, history=hist, times=times)


def finish_batch_in_contexts(batch, res, t1, t2, make_ctx, tol=1e-10, maxit=200, ndiis=6, dressed=0, floor=0.1,
                             concurrent=True):
    """Systems still iterating when solve_batch stopped (stop_active) continue
    alone, each in its own context (make_ctx(s, stream) -> Context on that
    torch stream with integrals set), from the amplitudes their batch segments
    hold, with a fresh DIIS subspace, until max|step| < tol or maxit iterations
    in all; the converged amplitudes are copied back into the segments and res
    (E, iters, converged) is updated in place.  A batch's launches are tuned
    for all of its systems; a lone straggler runs faster with its own tiles.
    concurrent=True: the continued systems iterate at the same time, each from
    a host thread of its own on a stream of its own (a lone small system does
    not fill the GPU; the library's calls release the interpreter lock), with
    the same results as one after another.  Returns the per-system results of
    the continued systems."""
    import numpy as np
    import torch
    rep = res["history"][-1]
    left = [int(s) for s in np.nonzero(rep[:, 3] != 0)[0]]
    torch.cuda.synchronize()      # the batch's amplitudes are final before other streams read them

    def run(s):
        off1, n1, off2, n2 = batch.segments[s]
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            ctx = make_ctx(s, stream)
            u1 = t1[off1:off1 + n1].clone()
            u2 = t2[off2:off2 + n2].clone()
            done = int(rep[s, 4])
            g = solve(ctx, u1, u2, tol=tol, maxit=max(1, maxit - done), ndiis=ndiis, dressed=dressed, floor=floor)
            stream.synchronize()
            ctx.destroy()
        return s, done, g, u1, u2

    if concurrent and len(left) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=len(left)) as ex:
            results = list(ex.map(run, left))
    else:
        results = [run(s) for s in left]
    out = {}
    for s, done, g, u1, u2 in results:
        off1, n1, off2, n2 = batch.segments[s]
        t1[off1:off1 + n1].copy_(u1)
        t2[off2:off2 + n2].copy_(u2)
        res["E"][s] = g["E"]
        res["iters"][s] = done + g["iters"]
        res["converged"][s] = g["converged"]
        out[s] = g
    torch.cuda.synchronize()
    return out


# ---------------------------------------------------------------- learned warm start

def _stream_ptr(stream):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(st.cuda_stream)


def _ws(st, what):
    if st != 0:
        raise FsccError(st, what + " failed")


def mlp_num_params():
    n = ctypes.c_size_t()
    _ws(lib().fscc_mlp_num_params(ctypes.byref(n)), "fscc_mlp_num_params")
    return n.value


class MLP:
    """The warm-start network (fscc_mlp_*): parameters and Adam state on the device."""

    def __init__(self, seed=0, stream=None):
        h = ctypes.c_void_p()
        _ws(lib().fscc_mlp_create(ctypes.c_uint64(int(seed)), _stream_ptr(stream), ctypes.byref(h)), "fscc_mlp_create")
        self._h = h
        self.n_params = mlp_num_params()

    def _check(self, st):
        if st != 0:
            msg = lib().fscc_mlp_last_error(self._h)
            raise FsccError(st, msg.decode() if msg else "")

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(lib().fscc_mlp_set_params(self._h, p.ctypes.data, p.size))

    def get_params(self):
        import numpy as np
        p = np.zeros(self.n_params, np.float32)
        self._check(lib().fscc_mlp_get_params(self._h, p.ctypes.data, p.size))
        return p

    def get_grad(self):
        import numpy as np
        g = np.zeros(self.n_params, np.float32)
        self._check(lib().fscc_mlp_get_grad(self._h, g.ctypes.data, g.size))
        return g

    def forward(self, X, Y):
        import torch
        n = X.shape[0]
        self._check(lib().fscc_mlp_forward(self._h, _ptr(X, torch.float32), n, _ptr(Y, torch.float32)))

    def loss_grad(self, u, r, D, t, idx=None, n=None, mode=0):
        """mode 0: relative loss, 1: absolute (size-weighted) loss."""
        import torch
        n = int(idx.numel()) if idx is not None else int(n if n is not None else u.numel())
        loss = ctypes.c_double()
        self._check(lib().fscc_mlp_loss_grad(self._h, _ptr(u, torch.complex128), _ptr(r, torch.complex128),
                                             _ptr(D, torch.float64), _ptr(t, torch.complex128),
                                             _ptr(idx, torch.int64), n, int(mode), ctypes.byref(loss)))
        return loss.value

    def adam(self, lr):
        self._check(lib().fscc_mlp_adam(self._h, ctypes.c_float(lr)))

    def destroy(self):
        if getattr(self, "_h", None):
            lib().fscc_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def ws_features(u, r, D, X, stream=None):
    import torch
    _ws(lib().fscc_ws_features(_ptr(u, torch.complex128), _ptr(r, torch.complex128), _ptr(D, torch.float64),
                               u.numel(), _ptr(X, torch.float32), _stream_ptr(stream)), "fscc_ws_features")


def ws_apply(Y, u, r, D, out, stream=None):
    import torch
    _ws(lib().fscc_ws_apply(_ptr(Y, torch.float32), _ptr(u, torch.complex128), _ptr(r, torch.complex128),
                            _ptr(D, torch.float64), u.numel(), _ptr(out, torch.complex128), _stream_ptr(stream)),
        "fscc_ws_apply")


def ws_step(t, r, D, out, stream=None):
    import torch
    _ws(lib().fscc_ws_step(_ptr(t, torch.complex128), _ptr(r, torch.complex128), _ptr(D, torch.float64),
                           r.numel(), _ptr(out, torch.complex128), _stream_ptr(stream)), "fscc_ws_step")


def ws_gather(src, idx, dst, stream=None):
    import torch
    eb = src.element_size()
    _ws(lib().fscc_ws_gather(_ptr(src), eb, _ptr(idx, torch.int64), idx.numel(), _ptr(dst), _stream_ptr(stream)),
        "fscc_ws_gather")

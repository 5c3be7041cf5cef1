"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fscc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fscc_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2004_03682_amd as F
    L = F.lib()
    names = _declared()
    assert "fscc_build_residual" in names and "fscc_update_amplitudes" in names and "fscc_energy" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_has_no_cpu_fallback():
    import paper_2004_03682_amd as F
    import torch
    with pytest.raises(TypeError):
        F._dev_ptr(torch.zeros(4, dtype=torch.complex128))


def test_null_arguments_are_rejected():
    import paper_2004_03682_amd as F
    L = F.lib()
    assert L.fscc_create(None, 0, None, None) == -1
    assert L.fscc_layout(None, 0, None, None) == -1
    assert L.fscc_build_residual(None, 0, None, None, None, None) == -1
    L.fscc_destroy(None)


def test_probe_arguments_are_checked_before_any_device_call():
    import paper_2004_03682_amd as F
    L = F.lib()
    tf = ctypes.c_double()
    for kind, iters in ((3, 16), (-1, 16), (0, 0), (0, (1 << 20) + 1)):
        assert L.fscc_probe_mfma(kind, iters, None, ctypes.byref(tf), None) == -1
    assert L.fscc_probe_mfma(0, 16, None, None, None) == -1

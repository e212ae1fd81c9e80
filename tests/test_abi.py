"""Host-side checks of the C ABI: the library loads and exports every symbol
that include/twa.h declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "twa.h")).read()
    return sorted(set(re.findall(r"TWA_API\s+[\w\s\*]+?\b(twa_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("twa_build_pump", "twa_run", "twa_run_batch", "twa_adjoint", "twa_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2608_10075_amd import LIB_PATH
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_has_no_cpu_fallback():
    import paper_2608_10075_amd as twa
    src = open(twa.__file__).read()
    assert "oracle" not in src.replace("no CPU fallback", "")
    for f in os.listdir(os.path.join(ROOT, "paper_2608_10075_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2608_10075_amd", "csrc", f)).read()


def test_params_defaults_and_invalid_arguments_rejected_on_host():
    import paper_2608_10075_amd as twa
    p = twa._Params()
    twa._lib.twa_params_default(ctypes.byref(p))
    assert p.gamma == 1.0 and p.s0z == 1.0 and p.burnin == -1 and p.kappa == 0.25
    h = ctypes.c_void_p()
    assert twa._lib.twa_build_pump(0, 1.0, 1.0, ctypes.byref(h)) == twa.TWA_EINVAL
    assert twa._lib.twa_build_pump(4, -1.0, 1.0, ctypes.byref(h)) == twa.TWA_EINVAL
    assert twa._lib.twa_build_pump(4, 1.0, float("nan"), ctypes.byref(h)) == twa.TWA_EINVAL
    o = twa._Obs()
    assert twa._lib.twa_run(ctypes.byref(p), 4, 1e-3, 10, 0, ctypes.byref(o), None) == twa.TWA_EINVAL
    assert "pump" in twa._lib.twa_last_error().decode()

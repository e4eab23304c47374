"""The C ABI library loads and exports every function include/shk.h declares
(no compute: runs without a GPU)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "shk.h")).read()
    return re.findall(r"^\s*(?:int|void|long long|double|const char\*)\s+(\w+)\(", hdr, re.M)


def test_library_exports_every_declared_symbol():
    import paper_1212_3660_amd as P
    L = P.lib()
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(P.binding.exported_symbols())


def test_param_defaults_and_status_strings():
    import ctypes as C
    import paper_1212_3660_amd as P
    p = P.binding.shk_params()
    P.lib().shk_params_default(C.byref(p))
    assert p.m_restart == 50 and p.tol == 1e-8 and p.precision == P.SHK_FP64
    assert p.inner_precond == P.SHK_PRECOND_JACOBI and p.mg_sweeps == 1 and p.mg_omega == 0.8
    assert p.inner_relax == 0.0 and p.inner_eps_max == 1e-2 and p.ortho == P.SHK_CGS2
    assert P.lib().shk_status_string(-5).decode() == "unsupported"


def test_binding_has_no_cpu_fallback():
    # the product path never imports the oracle
    import paper_1212_3660_amd.binding as B
    src = open(B.__file__).read()
    assert "oracle" not in src.replace("oracle's", "")

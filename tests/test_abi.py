"""Host-side checks of the C ABI library (no GPU needed): it loads and exports
every function declared in include/elses.h."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "elses.h")
LIB = os.path.join(ROOT, "paper_1609_08377_amd", "_lib", "libelses.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(elses_[a-z_]+)\s*\(", text)))


def test_header_declares_boundary():
    names = declared_functions()
    for required in ("elses_shifted_solve", "elses_density_matrix", "elses_mat_create", "elses_ctx_create"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libelses.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libelses.so not built")
def test_version_and_defaults_without_gpu():
    import paper_1609_08377_amd as el
    assert el.version().startswith("elses-gfx950")
    o = el.make_opts()
    assert o.tol == 1e-8 and o.max_outer == 20000 and o.inner_tol == 1e-13 and o.out_mode == 0

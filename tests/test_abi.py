"""The C-ABI library loads and exports every entry point its header declares (CPU only)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mtomg.h")
LIB = os.path.join(ROOT, "paper_2301_07457_amd", "libmtomg.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mtomg_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for want in ("mtomg_create", "mtomg_set_grid", "mtomg_set_densities", "mtomg_solve",
                 "mtomg_compliance_and_grad", "mtomg_destroy"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmtomg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmtomg.so not built")
def test_binding_names_match_header():
    from paper_2301_07457_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()
    lib = _lib.load()
    assert lib.mtomg_status_string(_lib.MTOMG_NOT_CONVERGED).startswith(b"not converged")
    # a null context is rejected without touching the GPU
    assert lib.mtomg_solve(None, 1e-8, 10, 0, None) == _lib.MTOMG_BAD_INPUT
    assert lib.mtomg_workspace_bytes(None) == 0


def header_enum(prefix):
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return {m.group(1): int(m.group(2)) for m in re.finditer(prefix + r"([A-Z0-9_]+)\s*=\s*(-?\d+)", txt)}


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmtomg.so not built")
def test_binding_enums_match_header():
    from paper_2301_07457_amd import _lib
    assert _lib.OPTIONS == header_enum("MTOMG_OPT_")
    assert _lib.FILTERS == header_enum("MTOMG_FILTER_")
    assert _lib.KERNELS == header_enum("MTOMG_KERNEL_")
    assert _lib.PROBES == header_enum("MTOMG_PROBE_")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmtomg.so not built")
def test_null_context_is_rejected_by_every_context_call():
    from paper_2301_07457_amd import _lib
    lib = _lib.load()
    bad = _lib.MTOMG_BAD_INPUT
    assert lib.mtomg_set_option(None, 0, 1) == bad
    assert lib.mtomg_filter(None, 8, 8, 1, 2.0, 0, 1e-3, None, None, None) == bad
    assert lib.mtomg_poisson_solve(None, 16, 2, 2, 0.6, 1e-8, 10, None, None, None) == bad
    assert lib.mtomg_compliance_and_grad(None, 0, None, None) == bad


def test_header_is_plain_c(tmp_path):
    """The boundary header compiles as pedantic C99 (no C++ or torch types)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    src = tmp_path / "use.c"
    src.write_text('#include "mtomg.h"\n'
                   "int main(void) { mtomg_stats s; mtomg_ctx *c = 0; (void)s; (void)c;\n"
                   "  return MTOMG_OPT_GAMMA + MTOMG_FILTER_SENSITIVITY + MTOMG_FP32MG; }\n")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(ROOT, "include"), "-c", str(src), "-o", str(tmp_path / "use.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

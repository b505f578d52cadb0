"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the header declares, and reports static status strings."""
import os
import subprocess
import sys

import pytest

from paper_1309_3458_amd import _native as N


def test_library_exports_every_header_symbol():
    L = N.lib()
    names = N.header_functions()
    assert "ddm_build" in names and "ddm_match" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings():
    L = N.lib()
    for code in (0, -1, -2, -3, -4, -5):
        s = L.ddm_strerror(code).decode()
        assert s and s != "unknown status"
    assert L.ddm_strerror(42).decode() == "unknown status"
    assert L.ddm_last_error_detail().decode() == ""


def test_header_compiles_as_c():
    inc = os.path.join(os.path.dirname(N.PKG), "include")
    src = "#include <ddm.h>\nint main(void){ ddm_match_opts o = {0}; (void)o; return DDM_OK; }\n"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", inc, "-x", "c", "-",
                        "-fsyntax-only"], input=src, text=True, capture_output=True)
    assert r.returncode == 0, r.stderr


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    import paper_1309_3458_amd as P
    x = torch.zeros((2, 4), dtype=torch.float32)
    with pytest.raises(ValueError):
        P.build(x, x)
    with pytest.raises(TypeError):
        P.build(x.double(), x.double())


def test_missing_library_fails_loudly(tmp_path):
    code = ("import paper_1309_3458_amd._native as N; N.LIB_PATH = '/nonexistent/libddm.so'\n"
            "try:\n    N.lib()\nexcept RuntimeError as e:\n    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=os.path.dirname(N.PKG))
    assert "raised" in r.stdout

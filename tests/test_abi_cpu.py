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


def _scratch_bytes(m, d, form, hint=0):
    import ctypes
    b = ctypes.c_uint64()
    rc = N.lib().ddm_match_scratch_bytes(m, d, form, hint, ctypes.byref(b))
    return rc, int(b.value)


@pytest.mark.parametrize("form", [0, 1, 2])
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_match_scratch_layouts_fit_on_the_host(form, d):
    """Every scratch layout of the match (plain, with the stash of hits,
    learned), run on the host with no memory behind it: each piece the
    match takes lies inside its reservation (the call reports an overrun
    as DDM_E_DEVICE), across sizes from 1 update to 2^31 - 1, ragged and
    power-of-two, and the size grows with m."""
    sizes = sorted({1, 2, 63, 64, 65, 255, 256, 257, 4095, 4097, 65535, 65536, 65537,
                    500_000, 1 << 20, (1 << 20) + 1, 10_000_019, (1 << 31) - 1})
    prev = 0
    for m in sizes:
        for hint in ((0, 1, 7 * m, 1 << 40) if form == 1 else (0,)):
            rc, b = _scratch_bytes(m, d, form, hint)
            assert rc == N.DDM_OK, (m, d, form, hint, N.lib().ddm_last_error_detail())
            assert b % 256 == 0 and b > 0
        rc, b = _scratch_bytes(m, d, form)
        # at least the per-update arrays of the front half (45 bytes each)
        assert b >= 45 * m and b >= prev
        prev = b


def test_match_scratch_bytes_rejects_bad_arguments():
    import ctypes
    L = N.lib()
    assert _scratch_bytes(0, 2, 0) == (N.DDM_OK, 0)
    assert _scratch_bytes(10, 0, 0)[0] == N.DDM_E_INVALID_ARG
    assert _scratch_bytes(10, 5, 0)[0] == N.DDM_E_INVALID_ARG
    assert _scratch_bytes(10, 2, 3)[0] == N.DDM_E_INVALID_ARG
    assert _scratch_bytes(1 << 31, 2, 0)[0] == N.DDM_E_INVALID_ARG
    assert L.ddm_match_scratch_bytes(10, 2, 0, 0, None) == N.DDM_E_INVALID_ARG

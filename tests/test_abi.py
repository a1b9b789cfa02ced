"""The C-ABI library loads and exports every symbol include/fnocc.h declares (no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fnocc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fno_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_declared_symbols():
    import paper_2509_14157_amd as P
    lib = ctypes.CDLL(P.LIBRARY_PATH)
    names = declared_symbols()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(P.SYMBOLS) == sorted(names)


def test_create_reports_missing_device_or_succeeds():
    import paper_2509_14157_amd as P
    lib = P.library()
    h = ctypes.c_void_p()
    st = lib.fno_create(10 ** 6, ctypes.byref(h))   # no such device anywhere
    assert st in (P.FNO_EDEVICE, P.FNO_EINVAL)
    assert not h.value


def test_calls_on_null_context_are_rejected():
    import paper_2509_14157_amd as P
    lib = P.library()
    assert lib.fno_ccsdt(None, None, None, None, None, None) == P.FNO_EINVAL
    assert lib.fno_sizes(None, None, None, None) == P.FNO_EINVAL
    assert lib.fno_amplitude_size(None, 3) == 0

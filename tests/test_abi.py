"""Host-side checks of the C ABI: the library loads and exports every
function the header declares; calls that need no GPU behave."""

import ctypes
import re

import paper_2505_15535_amd as mfe


def test_library_exports_every_declared_symbol():
    names = mfe.header_symbols()
    assert len(names) >= 14
    lib = ctypes.CDLL(mfe.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    assert all(callable(getattr(mfe, n)) for n in names)


def test_header_documents_every_entry_point():
    lines = open(mfe.HEADER_PATH).read().splitlines()
    for n in mfe.header_symbols():
        decl = [i for i, l in enumerate(lines) if re.match(rf"^[a-z].*\b{n}\(", l)]
        assert len(decl) == 1, n
        above = "\n".join(lines[max(0, decl[0] - 6):decl[0]])
        assert "*/" in above, n


def test_null_context_calls_are_safe():
    assert mfe.mfe_last_error(None) == "null context"
    assert mfe.mfe_n_dofs(None) == 0
    assert mfe.mfe_n_cells(None) == 0
    assert mfe.mfe_cache_bytes(None, mfe.MFE_T4) == 0
    lib = ctypes.CDLL(mfe.LIB_PATH)
    lib.mfe_apply_tangent.restype = ctypes.c_int
    assert lib.mfe_apply_tangent(None, None, None, 0, 0, None) == mfe.MFE_EINVAL
    lib.mfe_destroy(None)


def test_enums_match_header():
    text = open(mfe.HEADER_PATH).read()
    for name, val in [("MFE_OTF", mfe.MFE_OTF), ("MFE_OTF_GEOM", mfe.MFE_OTF_GEOM), ("MFE_T2", mfe.MFE_T2),
                      ("MFE_T4", mfe.MFE_T4), ("MFE_OTF_AD", mfe.MFE_OTF_AD), ("MFE_EJACOBIAN", mfe.MFE_EJACOBIAN),
                      ("MFE_ESTATE", mfe.MFE_ESTATE), ("MFE_EINVAL", mfe.MFE_EINVAL), ("MFE_FP64", mfe.MFE_FP64)]:
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == val, name

"""The C-ABI library loads and exports every symbol include/*.h declares,
and the struct layouts of the binding match the header.  CPU only: no call
here touches a GPU."""
import ctypes as C
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(cl_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2607_24978_amd import _lib
    lib = C.CDLL(_lib.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 19
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps exactly these
    assert names == set(_lib._SIGS), names ^ set(_lib._SIGS)


def test_struct_layouts():
    from paper_2607_24978_amd import _lib
    assert C.sizeof(_lib.cl_observables) == 8 * 13 + 8
    assert C.sizeof(_lib.cl_potential) == 6 * 8
    assert C.sizeof(_lib.cl_scalars) == 32
    assert _lib.OBS_DTYPE.itemsize == C.sizeof(_lib.cl_observables)


def test_version_and_null_handles():
    from paper_2607_24978_amd import _lib
    lib = _lib.lib
    assert b"gfx950" in lib.cl_version()
    # handle-less argument errors are reported without touching a device
    assert lib.cl_destroy(None) == _lib.CL_OK
    assert lib.cl_set_background(None, 1.0, 1, 1.0, 1.0) == _lib.CL_EINVAL
    assert lib.cl_step(None, 0, 0.1, 1, None) == _lib.CL_EINVAL
    assert lib.cl_create(32, 1.0, 1, 0, None) == _lib.CL_EINVAL
    assert b"NULL" in lib.cl_last_error(None)

"""The C-ABI library loads and exports every function include/stucker.h declares."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "stucker.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(st_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["st_create", "st_init", "st_update", "st_core", "st_factor", "st_recon_error",
              "st_destroy", "st_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2308_16395_amd as pkg

    lib = ctypes.CDLL(pkg.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(pkg.EXPORTED) == _declared()


def test_create_rejects_bad_config_without_a_gpu():
    import paper_2308_16395_amd.binding as b

    cfg = b.st_config()
    cfg.nmodes = 0
    h = ctypes.c_void_p()
    assert b.st_create(ctypes.byref(cfg), ctypes.byref(h)) == b.ST_EINVAL
    assert b"invalid" in b.st_last_error(None)
    cfg.nmodes = 2
    cfg.dims[0] = cfg.dims[1] = 4
    cfg.tau = -1.0
    assert b.st_create(ctypes.byref(cfg), ctypes.byref(h)) == b.ST_EINVAL
    assert b.st_update(None, None) == b.ST_EINVAL

"""CPU checks of the C ABI: the library loads and exports every function
that include/dfacto.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

from conftest import ROOT
from paper_1406_4519_amd import dfacto


def _declared():
    src = open(os.path.join(ROOT, "include", "dfacto.h")).read()
    decl = r"^(?:dfacto_status|void|const char)\s*\*?\s*(dfacto_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, src, flags=re.MULTILINE)))


def test_header_and_binding_agree():
    assert sorted(dfacto.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = dfacto.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_declares_argument_types_of_every_export():
    """Every exported function has ctypes argument types, so a Python value
    of the wrong kind is refused instead of passed through."""
    lib = dfacto.load()
    for name in dfacto.EXPORTS:
        assert getattr(lib, name).argtypes is not None, name


def test_no_device_is_reported_as_error():
    import torch
    if torch.cuda.is_available():
        return
    lib = dfacto.load()
    h = ctypes.c_void_p()
    assert lib.dfacto_ctx_create(0, None, None, ctypes.byref(h)) == dfacto.E_DEVICE
    assert lib.dfacto_ctx_create(0, None, None, None) == dfacto.E_INVALID
    # an allocator must name both functions
    half = dfacto._Allocator()
    half.alloc = dfacto._ALLOC_FN(lambda n, s, u: None)
    assert lib.dfacto_ctx_create(0, None, ctypes.byref(half), ctypes.byref(h)) == dfacto.E_INVALID
    assert lib.dfacto_last_error(None) == b"context is NULL"


def test_server_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        return
    lib = dfacto.load()
    h = ctypes.c_void_p()
    assert lib.dfacto_server_create(0, 0, 4, ctypes.byref(h)) == dfacto.E_DEVICE
    assert not h.value

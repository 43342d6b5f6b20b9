"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host (no device work here)."""
import ctypes
import os
import re

import pytest

from paper_2606_11402_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vecchia.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


def test_header_declares_the_path():
    names = declared_functions()
    for fn in ("graph_build", "vecchia_factor", "vecchia_forward", "vecchia_inverse", "vecchia_logdet",
               "vecchia_backward"):
        assert fn in names


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(_lib.exported_symbols())


def test_abi_sizes_match_binding():
    lib = _lib.load()
    vb, kb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.vecchia_abi_sizes(ctypes.byref(vb), ctypes.byref(kb)) == 0
    assert vb.value == ctypes.sizeof(_lib.ViewStruct) == 136
    assert kb.value == ctypes.sizeof(_lib.KernelStruct) == 40


def test_padded_widths():
    lib = _lib.load()
    assert [lib.vecchia_padded_k(k) for k in (0, 1, 8, 9, 16, 17, 32)] == [-1, 8, 8, 16, 16, 32, 32]
    assert lib.vecchia_padded_k(_lib.KMAX) == _lib.KMAX and lib.vecchia_padded_k(_lib.KMAX + 1) == -1


def test_neighbour_count_above_the_compiled_maximum_is_unsupported():
    """k > KMAX is a valid Vecchia approximation that is not compiled
    (EUNSUPPORTED); k < 1 is an invalid argument (EINVAL)."""
    import numpy as np
    lib = _lib.load()
    out = ctypes.c_size_t()
    assert lib.vecchia_workspace_bytes(4096, _lib.KMAX + 1, 128, 0, ctypes.byref(out)) == _lib.EUNSUPPORTED
    assert lib.vecchia_workspace_bytes(4096, 0, 128, 0, ctypes.byref(out)) == _lib.EINVAL
    x = np.random.default_rng(0).random((200, 3))
    h = ctypes.c_void_p()
    xp = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.graph_build(xp, 200, 3, _lib.KMAX + 1, 128, 1, ctypes.byref(h)) == _lib.EUNSUPPORTED
    assert lib.graph_build(xp, 200, 3, 0, 128, 1, ctypes.byref(h)) == _lib.EINVAL
    v = _lib.ViewStruct()
    v.n, v.k, v.kp, v.n0, v.precision = 1000, _lib.KMAX + 1, _lib.KMAX, 128, 0
    assert lib.vecchia_factor(ctypes.byref(v), ctypes.byref(_lib.KernelStruct(1, 1.0, 0.1, 0.0)), None) \
        == _lib.EUNSUPPORTED
    nbytes = ctypes.c_size_t()
    assert lib.serve_request_bytes(1000, _lib.KMAX + 1, 128, ctypes.byref(nbytes)) == _lib.EUNSUPPORTED


def test_workspace_bytes_and_errors():
    lib = _lib.load()
    out = ctypes.c_size_t()
    assert lib.vecchia_workspace_bytes(4096, 8, 128, 0, ctypes.byref(out)) == 0
    ns = 4096 - 128
    tiles = (ns + 63) // 64
    assert out.value >= tiles * 8 * 64 * 8 + tiles * 64 * 8 + 128 * 128 * 8
    assert lib.vecchia_workspace_bytes(4096, 0, 128, 0, ctypes.byref(out)) == _lib.EINVAL
    assert lib.vecchia_workspace_bytes(4096, 8, 5000, 0, ctypes.byref(out)) == _lib.EINVAL
    assert lib.vecchia_workspace_bytes(4096, 8, 128, 7, ctypes.byref(out)) == _lib.EINVAL
    assert b"precision" in lib.vecchia_last_error()


def test_view_validation_happens_before_any_launch():
    lib = _lib.load()
    v = _lib.ViewStruct()
    k = _lib.KernelStruct(1, 1.0, 0.1, 0.0)
    assert lib.vecchia_factor(ctypes.byref(v), ctypes.byref(k), None) == _lib.EINVAL
    v.n, v.k, v.kp, v.n0, v.precision = 100, 8, 16, 10, 0
    assert lib.vecchia_factor(ctypes.byref(v), ctypes.byref(k), None) == _lib.EINVAL
    assert b"kp" in lib.vecchia_last_error()
    v.kp, v.n0 = 8, 200
    assert lib.vecchia_forward(ctypes.byref(v), None, None, None) == _lib.EINVAL
    v.n, v.n0 = 1000, 129
    assert lib.vecchia_inverse(ctypes.byref(v), None, None, None) == _lib.EUNSUPPORTED


def test_kernel_validation():
    lib = _lib.load()
    import numpy as np
    lp = np.array([0, 10, 100], np.int32)
    v = _lib.ViewStruct()
    v.n, v.k, v.kp, v.n0, v.n_levels, v.precision = 100, 8, 8, 10, 1, 0
    v.x = v.nbr = v.workspace = 256
    v.level_ptr = lp.ctypes.data
    v.workspace_bytes = 1 << 30
    for bad in (_lib.KernelStruct(4, 1.0, 0.1, 0.0), _lib.KernelStruct(0, -1.0, 0.1, 0.0),
                _lib.KernelStruct(0, 1.0, 0.0, 0.0), _lib.KernelStruct(0, 1.0, 0.1, -1e-3)):
        assert lib.vecchia_factor(ctypes.byref(v), ctypes.byref(bad), None) == _lib.EINVAL


def test_level_ptr_validation():
    lib = _lib.load()
    import numpy as np
    v = _lib.ViewStruct()
    v.n, v.k, v.kp, v.n0, v.n_levels, v.precision = 100, 8, 8, 10, 2, 0
    v.x = v.nbr = v.workspace = 256
    v.workspace_bytes = 1 << 30
    for lp in ([0, 10, 60, 99], [0, 11, 60, 100], [0, 10, 70, 60]):
        arr = np.array(lp, np.int32)
        v.level_ptr = arr.ctypes.data
        assert lib.vecchia_forward(ctypes.byref(v), ctypes.c_void_p(512), ctypes.c_void_p(1024), None) == _lib.EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()

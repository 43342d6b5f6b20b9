"""ctypes binding of ``libvecchia.so`` (include/vecchia.h).

Argument marshalling only: every step of the hot path runs in the native
library.  The library must have been built in-tree (``build.py``); if it is
missing, loading fails with an error -- there is no fallback.
"""
import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvecchia.so")

OK, EINVAL, ENOMEM, ENOTPD, EUNSUPPORTED, EHIP, EBUDGET, EIO = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32 = 0, 1
KMAX, N0MAX = 64, 128
KNN_NODE_BYTES = 40
EXP, M32, SE, M52, MATERN = 0, 1, 2, 3, 4

_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", ENOTPD: "ENOTPD", EUNSUPPORTED: "EUNSUPPORTED",
          EHIP: "EHIP", EBUDGET: "EBUDGET", EIO: "EIO"}

c_int32, c_int64, c_double, c_size_t, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                 ctypes.c_size_t, ctypes.c_void_p)
P = ctypes.POINTER


class VecchiaError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, message))
        self.code = code


class KernelStruct(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("sigma", c_double), ("ell", c_double), ("nugget", c_double), ("nu", c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("arena_bytes", c_size_t), ("bytes_in_use", c_size_t), ("peak_bytes", c_size_t),
                ("largest_free", c_size_t), ("building", c_int64), ("queued", c_int64), ("running", c_int64),
                ("admitted", c_int64), ("completed", c_int64), ("failed", c_int64), ("rejected", c_int64),
                ("cancelled", c_int64), ("peak_running", c_int64), ("graphs_on_device", c_int64)]


class ViewStruct(ctypes.Structure):
    _fields_ = [
        ("n", c_int64), ("k", c_int32), ("kp", c_int32), ("n0", c_int32), ("n_levels", c_int32),
        ("precision", c_int32), ("redo_log2", c_int32),
        ("x", c_void_p), ("nbr", c_void_p), ("level_ptr", c_void_p), ("level_ptr_dev", c_void_p),
        ("child_ptr", c_void_p),
        ("child", c_void_p), ("workspace", c_void_p), ("workspace_bytes", c_size_t),
        ("kernel", KernelStruct),
    ]


_SIGNATURES = {
    "graph_build": (c_int32, [P(c_double), c_int64, c_int32, c_int32, c_int32, c_int32, P(c_void_p)]),
    "graph_build_begin": (c_int32, [P(c_double), c_int64, c_int32, c_int32, c_int32, c_int32, P(c_void_p)]),
    "graph_knn_nodes": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "graph_knn_device": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "graph_build_finish": (c_int32, [c_void_p, c_void_p]),
    "graph_depth_device": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p, c_void_p, P(c_int32)]),
    "graph_build_finish_depth": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "graph_tree_scratch_bytes": (c_int32, [c_int64, P(c_size_t)]),
    "graph_tree_device": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "graph_build_begin_tree": (c_int32, [P(c_double), c_int64, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                         P(c_void_p)]),
    "graph_info": (c_int32, [c_void_p, P(c_int64), P(c_int32), P(c_int32), P(c_int32), P(c_int32), P(c_int32)]),
    "graph_export": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "graph_export_nbr": (c_int32, [c_void_p, c_int32, c_void_p]),
    "graph_export_points": (c_int32, [c_void_p, c_int32, c_void_p]),
    "graph_export_children": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "graph_build_times": (c_int32, [c_void_p, P(c_double)]),
    "graph_save": (c_int32, [c_void_p, ctypes.c_char_p]),
    "graph_load": (c_int32, [ctypes.c_char_p, c_int32, P(c_void_p)]),
    "graph_free": (None, [c_void_p]),
    "vecchia_workspace_bytes": (c_int32, [c_int64, c_int32, c_int32, c_int32, P(c_size_t)]),
    "vecchia_factor": (c_int32, [P(ViewStruct), P(KernelStruct), c_void_p]),
    "vecchia_forward": (c_int32, [P(ViewStruct), c_void_p, c_void_p, c_void_p]),
    "vecchia_inverse": (c_int32, [P(ViewStruct), c_void_p, c_void_p, c_void_p]),
    "vecchia_logdet": (c_int32, [P(ViewStruct), c_void_p, c_void_p]),
    "vecchia_backward_scratch_bytes": (c_int32, [P(ViewStruct), P(c_size_t)]),
    "vecchia_backward": (c_int32, [P(ViewStruct), P(KernelStruct), c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "vecchia_backward_x_scratch_bytes": (c_int32, [P(ViewStruct), P(c_size_t)]),
    "vecchia_backward_x": (c_int32, [P(ViewStruct), P(KernelStruct), c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                     c_void_p, c_void_p, c_size_t, c_void_p]),
    "vecchia_backward_noalloc_max_bytes": (c_int32, [P(c_size_t)]),
    "vecchia_backward_noalloc": (c_int32, [P(ViewStruct), P(KernelStruct), c_void_p, c_void_p, c_void_p, c_void_p,
                                           c_double, c_void_p, c_void_p, c_void_p, c_void_p]),
    "vecchia_fused_workspace_bytes": (c_int32, [c_int64, c_int32, c_int32, c_int32, P(c_size_t)]),
    "vecchia_forward_fused": (c_int32, [P(ViewStruct), P(KernelStruct), c_void_p, c_void_p, c_void_p, c_void_p]),
    "vecchia_fused_status": (c_int32, [P(ViewStruct), c_void_p, P(c_int64)]),
    "vecchia_jvp_scratch_bytes": (c_int32, [P(ViewStruct), P(c_size_t)]),
    "vecchia_forward_jvp": (c_int32, [P(ViewStruct), P(KernelStruct), c_void_p, c_void_p, c_void_p, c_double, c_double,
                                      c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "vecchia_status": (c_int32, [P(ViewStruct), c_void_p, P(c_int64)]),
    "vecchia_factor_counts": (c_int32, [P(ViewStruct), c_void_p, P(c_int64), P(c_int64)]),
    "vecchia_padded_k": (c_int32, [c_int32]),
    "vecchia_profile_enable": (c_int32, [c_int32]),
    "vecchia_profile_read": (c_int32, [ctypes.c_char_p, c_size_t, P(c_double), P(c_int64), c_int32, P(c_int32)]),
    "vecchia_profile_reset": (c_int32, []),
    "vecchia_abi_sizes": (c_int32, [P(c_size_t), P(c_size_t)]),
    "serve_create": (c_int32, [c_void_p, c_size_t, c_int32, c_int32, c_int32, c_int32, P(c_void_p)]),
    "serve_request_bytes": (c_int32, [c_int64, c_int32, c_int32, P(c_size_t)]),
    "serve_submit": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32, P(KernelStruct), c_int32, c_void_p,
                               P(c_int64)]),
    "serve_progress": (c_int32, [c_void_p, P(c_int32)]),
    "serve_take": (c_int32, [c_void_p, P(c_int64)]),
    "serve_result": (c_int32, [c_void_p, c_int64, c_void_p, P(c_double), P(c_double)]),
    "serve_release": (c_int32, [c_void_p, c_int64]),
    "serve_cancel": (c_int32, [c_void_p, c_int64]),
    "serve_stats": (c_int32, [c_void_p, P(ServeStats)]),
    "serve_set_graph_device": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "serve_destroy": (None, [c_void_p]),
    "vecchia_last_error": (ctypes.c_char_p, []),
    "vecchia_version": (ctypes.c_char_p, []),
}

_lock = threading.Lock()
_lib = None


def load():
    """Load the in-tree library once; raise if it is absent or its ABI differs."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError("libvecchia.so is not built (expected at %s); run "
                              "`python -m paper_2606_11402_amd.build` -- the product has no fallback path"
                              % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_LOCAL)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        vb, kb = c_size_t(), c_size_t()
        lib.vecchia_abi_sizes(ctypes.byref(vb), ctypes.byref(kb))
        if vb.value != ctypes.sizeof(ViewStruct) or kb.value != ctypes.sizeof(KernelStruct):
            raise ImportError("libvecchia ABI mismatch: view %d/%d kernel %d/%d bytes"
                              % (vb.value, ctypes.sizeof(ViewStruct), kb.value, ctypes.sizeof(KernelStruct)))
        _lib = lib
        return lib


def check(code, what=""):
    if code != OK:
        msg = load().vecchia_last_error().decode(errors="replace")
        raise VecchiaError(code, (what + ": " if what else "") + msg)
    return code


def exported_symbols():
    return list(_SIGNATURES)

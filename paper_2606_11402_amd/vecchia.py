"""Python face of the native Vecchia library: marshalling only.

``Graph`` wraps the host graph build (C++), ``DeviceGraph`` holds its arrays
in HBM as torch tensors, and ``Factor`` owns one factor workspace and calls
``vecchia_factor``/``vecchia_forward``/``vecchia_inverse``/``vecchia_logdet``
on the current torch stream.  Every array the library sees is a caller-owned
tensor; the library allocates nothing on the device.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

EXP, M32, SE, M52, MATERN = _lib.EXP, _lib.M32, _lib.SE, _lib.M52, _lib.MATERN
FP64, FP32 = _lib.FP64, _lib.FP32
_TORCH_DTYPE = {FP64: torch.float64, FP32: torch.float32}
_NP_DTYPE = {FP64: np.float64, FP32: np.float32}


@dataclass(frozen=True)
class KernelParams:
    """Stationary covariance: kind EXP/M32/SE/M52/MATERN, amplitude sigma,
    length scale ell, an absolute nugget on the diagonal and, for MATERN,
    the smoothing nu."""
    kind: int
    sigma: float = 1.0
    ell: float = 1.0
    nugget: float = 0.0
    nu: float = 0.0

    def to_c(self):
        return _lib.KernelStruct(int(self.kind), float(self.sigma), float(self.ell), float(self.nugget),
                                 float(self.nu))


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else ctypes.c_void_p(a.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Graph:
    """Bit-reversed k-d tree order, preceding k-NN and depth batches of a
    point cloud, built on the host by the native library."""

    def __init__(self, x, k, n0, n_threads=0, knn_device=None, depth_device=True, tree_device=True):
        """knn_device (e.g. "cuda:0"): run the preceding k-NN search on that
        device (graph_build_begin / graph_knn_device / graph_build_finish),
        with depth_device also the depth fixpoint (graph_depth_device /
        graph_build_finish_depth) and with tree_device also the k-d tree
        (graph_tree_device / graph_build_begin_tree); the result is the same
        graph bit for bit."""
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        if x.ndim == 1:
            x = x[:, None]
        if x.ndim != 2:
            raise ValueError("points must be (N, d)")
        self._lib = _lib.load()
        handle = ctypes.c_void_p()
        xp = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.knn_seconds = None
        self.tree_seconds = None
        self.depth_sweeps = None
        self.split_seconds = None       # device path: wall time of each host and device step
        if knn_device is None:
            _lib.check(self._lib.graph_build(xp, x.shape[0], x.shape[1], int(k), int(n0), int(n_threads),
                                             ctypes.byref(handle)), "graph_build")
            self._h = handle
        else:
            import time
            ts = [time.perf_counter()]
            n = x.shape[0]
            dev = torch.device(knn_device)
            self.tree_seconds = None
            if tree_device:
                x3 = np.zeros((n, 3))
                x3[:, :x.shape[1]] = x
                t_tree = time.perf_counter()
                x_d = torch.from_numpy(x3).to(dev)
                nb = ctypes.c_size_t()
                _lib.check(self._lib.graph_tree_scratch_bytes(n, ctypes.byref(nb)), "graph_tree_scratch_bytes")
                scratch = torch.empty(nb.value, dtype=torch.uint8, device=dev)
                perm_d = torch.empty(n, dtype=torch.int32, device=dev)
                sdim_d = torch.empty(n, dtype=torch.int32, device=dev)
                _lib.check(self._lib.graph_tree_device(ctypes.c_void_p(x_d.data_ptr()), n, x.shape[1],
                                                       ctypes.c_void_p(perm_d.data_ptr()),
                                                       ctypes.c_void_p(sdim_d.data_ptr()),
                                                       ctypes.c_void_p(scratch.data_ptr()), nb.value, _stream(dev)),
                           "graph_tree_device")
                perm, sdim = perm_d.cpu().numpy(), sdim_d.cpu().numpy()
                self.tree_seconds = time.perf_counter() - t_tree
                del x_d, scratch, perm_d, sdim_d
                _lib.check(self._lib.graph_build_begin_tree(xp, n, x.shape[1], int(k), int(n0), int(n_threads),
                                                            _ptr(perm), _ptr(sdim), ctypes.byref(handle)),
                           "graph_build_begin_tree")
            else:
                _lib.check(self._lib.graph_build_begin(xp, x.shape[0], x.shape[1], int(k), int(n0), int(n_threads),
                                                       ctypes.byref(handle)), "graph_build_begin")
            self._h = handle
            # page-locked host buffers: the node and row transfers run at the
            # link's rate instead of through pageable staging
            nodes_h = torch.empty(n * _lib.KNN_NODE_BYTES, dtype=torch.uint8, pin_memory=True)
            rank_h = torch.empty(n, dtype=torch.int32, pin_memory=True)
            _lib.check(self._lib.graph_knn_nodes(self._h, ctypes.c_void_p(nodes_h.data_ptr()),
                                                 ctypes.c_void_p(rank_h.data_ptr())), "graph_knn_nodes")
            ts.append(time.perf_counter())
            nodes_d = nodes_h.to(dev)
            rank_d = rank_h.to(dev)
            rows_d = torch.empty(max((n - int(n0)) * int(k), 1), dtype=torch.int32, device=dev)
            _lib.check(self._lib.graph_knn_device(ctypes.c_void_p(nodes_d.data_ptr()), ctypes.c_void_p(rank_d.data_ptr()),
                                                  n, x.shape[1], int(k), int(n0), ctypes.c_void_p(rows_d.data_ptr()),
                                                  _stream(dev)), "graph_knn_device")
            torch.cuda.synchronize(dev)
            ts.append(time.perf_counter())
            depth = None
            if depth_device:
                depth_d = torch.empty(n, dtype=torch.int32, device=dev)
                flag_d = torch.empty(1, dtype=torch.int32, device=dev)
                sw = ctypes.c_int32()
                _lib.check(self._lib.graph_depth_device(ctypes.c_void_p(rows_d.data_ptr()), n, int(k), int(n0),
                                                        ctypes.c_void_p(depth_d.data_ptr()),
                                                        ctypes.c_void_p(flag_d.data_ptr()), _stream(dev),
                                                        ctypes.byref(sw)), "graph_depth_device")
                depth = depth_d.cpu().numpy()
                self.depth_sweeps = sw.value
            ts.append(time.perf_counter())
            rows_h = torch.empty(rows_d.numel(), dtype=torch.int32, pin_memory=True)
            rows_h.copy_(rows_d)
            rows = rows_h.numpy()
            ts.append(time.perf_counter())
            self.knn_seconds = (ts[2] - ts[1]) + (ts[4] - ts[3])
            del nodes_d, rank_d, rows_d, nodes_h, rank_h
            if depth is not None:
                _lib.check(self._lib.graph_build_finish_depth(self._h, _ptr(rows), _ptr(depth)),
                           "graph_build_finish_depth")
            else:
                _lib.check(self._lib.graph_build_finish(self._h, _ptr(rows)), "graph_build_finish")
            ts.append(time.perf_counter())
            self.split_seconds = {"begin_and_nodes": ts[1] - ts[0], "device_tree": self.tree_seconds,
                                  "device_search": ts[2] - ts[1],
                                  "device_depth": ts[3] - ts[2], "rows_to_host": ts[4] - ts[3],
                                  "finish": ts[5] - ts[4]}
        self._adopt()

    def _adopt(self):
        """Read the sizes and storage maps of the native graph self._h."""
        n, d, kk, kp, nn0, nl = (ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                                 ctypes.c_int32(), ctypes.c_int32())
        _lib.check(self._lib.graph_info(self._h, ctypes.byref(n), ctypes.byref(d), ctypes.byref(kk),
                                        ctypes.byref(kp), ctypes.byref(nn0), ctypes.byref(nl)), "graph_info")
        self.n, self.d, self.k, self.kp, self.n0, self.n_levels = (n.value, d.value, kk.value, kp.value,
                                                                   nn0.value, nl.value)
        self.order = np.empty(self.n, np.int32)
        self.slot = np.empty(self.n, np.int32)
        self.depth = np.empty(self.n, np.int32)
        self.level_ptr = np.empty(self.n_levels + 2, np.int32)
        _lib.check(self._lib.graph_export(self._h, _ptr(self.order), _ptr(self.slot), _ptr(self.level_ptr),
                                          _ptr(self.depth)), "graph_export")

    def save(self, path):
        """Write the graph to ``path`` (graph_save): the points, tree, rows
        and depths, enough to rebuild it without the neighbour search."""
        _lib.check(self._lib.graph_save(self._h, os.fsencode(path)), "graph_save")

    @classmethod
    def load(cls, path, n_threads=0):
        """A graph read from a file written by ``save`` (graph_load); it is
        checked as a device build is and equals the saved graph bit for bit."""
        g = cls.__new__(cls)
        g._lib = _lib.load()
        handle = ctypes.c_void_p()
        _lib.check(g._lib.graph_load(os.fsencode(path), int(n_threads), ctypes.byref(handle)), "graph_load")
        g._h = handle
        g.knn_seconds = g.tree_seconds = g.depth_sweeps = g.split_seconds = None
        g._adopt()
        return g

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.graph_free(h)
            self._h = None

    @property
    def ns(self):
        return self.n - self.n0

    @property
    def ntiles(self):
        return (self.ns + 63) // 64

    def nbr(self, layout=0):
        size = self.ns * self.k if layout == 0 else self.ntiles * self.kp * 64
        out = np.empty(max(size, 1), np.int32)
        _lib.check(self._lib.graph_export_nbr(self._h, layout, _ptr(out)), "graph_export_nbr")
        return out[:size].reshape(self.ns, self.k) if layout == 0 else out[:size]

    def to_row_order(self, b_dev, rows=None):
        """Coefficients read from the device (``Factor.coefficients`` or
        ``coefficient_rows``: one row per sparse point, in the device row
        order, ascending storage position) reordered to the rows of
        ``nbr(0)`` (ascending distance).  Host-side helper for comparisons
        with a reference."""
        nb = self.nbr(0) if rows is None else self.nbr(0)[np.asarray(rows)]
        key = np.where(nb >= 0, nb.astype(np.int64), np.int64(1) << 40)
        perm = np.argsort(key, axis=1, kind="stable")
        out = np.zeros((nb.shape[0], self.k), dtype=np.asarray(b_dev).dtype)
        np.put_along_axis(out, perm, np.asarray(b_dev)[:, :self.k], axis=1)
        return out

    def points(self, precision=FP64):
        out = np.empty((self.n, 3), _NP_DTYPE[precision])
        _lib.check(self._lib.graph_export_points(self._h, precision, _ptr(out)), "graph_export_points")
        return out

    def children(self):
        ptr = np.empty(self.n + 1, np.int64)
        child = np.empty(max(self.ns * self.k, 1), np.int32)
        _lib.check(self._lib.graph_export_children(self._h, _ptr(ptr), _ptr(child)), "graph_export_children")
        return ptr, child[:ptr[-1]]

    def build_times(self):
        t = (ctypes.c_double * 4)()
        _lib.check(self._lib.graph_build_times(self._h, t), "graph_build_times")
        return {"tree": t[0], "neighbours": t[1], "depth": t[2], "storage": t[3]}

    def to_device(self, precision=FP64, device="cuda", with_children=False):
        return DeviceGraph(self, precision, device, with_children)

    # storage <-> input order helpers (host)
    def to_storage(self, values):
        return np.asarray(values)[self.order]

    def from_storage(self, values):
        out = np.empty_like(np.asarray(values))
        out[self.order] = values
        return out


class DeviceGraph:
    """Graph arrays in HBM: coordinates in storage order (N x 3), tiled
    neighbour indices, optional children lists; batch boundaries on the host."""

    def __init__(self, g, precision, device, with_children=False):
        self.n, self.k, self.kp, self.n0, self.n_levels = g.n, g.k, g.kp, g.n0, g.n_levels
        self.precision = precision
        self.device = torch.device(device)
        self.level_ptr = np.ascontiguousarray(g.level_ptr, dtype=np.int32)
        self.level_ptr_dev = torch.from_numpy(self.level_ptr).to(self.device)
        self.x = torch.from_numpy(g.points(precision)).to(self.device)
        nbr = g.nbr(layout=1)
        self.nbr = torch.from_numpy(nbr if nbr.size else np.full(1, -1, np.int32)).to(self.device)
        self.child_ptr = self.child = None
        if with_children:
            ptr, child = g.children()
            self.child_ptr = torch.from_numpy(ptr).to(self.device)
            self.child = torch.from_numpy(child if child.size else np.zeros(1, np.int32)).to(self.device)

    @property
    def dtype(self):
        return _TORCH_DTYPE[self.precision]


def workspace_bytes(n, k, n0, precision):
    out = ctypes.c_size_t()
    _lib.check(_lib.load().vecchia_workspace_bytes(n, k, n0, precision, ctypes.byref(out)), "vecchia_workspace_bytes")
    return out.value


class Factor:
    """One factored point set: b, sigma, L0 and logdet partials in a
    device workspace, produced by ``vecchia_factor`` on the current stream."""

    def __init__(self, dg, kernel, workspace=None, redo_log2=0):
        self._lib = _lib.load()
        self.dg = dg
        self.kernel = kernel
        nbytes = workspace_bytes(dg.n, dg.k, dg.n0, dg.precision)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=dg.device)
        if workspace.numel() < nbytes or workspace.data_ptr() % 256:
            raise ValueError("workspace must hold %d bytes, 256-byte aligned" % nbytes)
        self.workspace = workspace
        v = _lib.ViewStruct()
        v.n, v.k, v.kp, v.n0, v.n_levels, v.precision = dg.n, dg.k, dg.kp, dg.n0, dg.n_levels, dg.precision
        v.redo_log2 = int(redo_log2)
        v.x = dg.x.data_ptr()
        v.nbr = dg.nbr.data_ptr()
        v.level_ptr = dg.level_ptr.ctypes.data
        v.level_ptr_dev = dg.level_ptr_dev.data_ptr()
        v.child_ptr = dg.child_ptr.data_ptr() if dg.child_ptr is not None else None
        v.child = dg.child.data_ptr() if dg.child is not None else None
        v.workspace = workspace.data_ptr()
        v.workspace_bytes = workspace.numel()
        self.view = v
        self._kc = kernel.to_c()
        self.refactor()

    def refactor(self, kernel=None):
        """Run vecchia_factor again (optionally with new kernel parameters)
        into the same workspace."""
        if kernel is not None:
            self.kernel = kernel
            self._kc = kernel.to_c()
        _lib.check(self._lib.vecchia_factor(ctypes.byref(self.view), ctypes.byref(self._kc),
                                            _stream(self.dg.device)), "vecchia_factor")

    def _vec(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device != self.dg.device or t.dtype != self.dg.dtype \
                or t.numel() != self.dg.n or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor of %d elements on %s"
                             % (name, self.dg.dtype, self.dg.n, self.dg.device))
        return t

    def _out(self, out):
        if out is None:
            return torch.empty(self.dg.n, dtype=self.dg.dtype, device=self.dg.device)
        return self._vec(out, "out")

    def forward(self, xi, out=None, per_batch=False):
        """v = F(xi), both in storage order.  per_batch=True passes the view
        without the device copy of level_ptr, so the library launches one
        kernel per batch instead of its one-workgroup runs of small batches."""
        xi = self._vec(xi, "xi")
        v = self._out(out)
        view = self.view
        if per_batch:
            view = _lib.ViewStruct.from_buffer_copy(self.view)
            view.level_ptr_dev = None
        _lib.check(self._lib.vecchia_forward(ctypes.byref(view), ctypes.c_void_p(xi.data_ptr()),
                                             ctypes.c_void_p(v.data_ptr()), _stream(self.dg.device)),
                   "vecchia_forward")
        return v

    def inverse(self, v, out=None):
        """xi = F^-1(v), both in storage order."""
        v = self._vec(v, "v")
        xi = self._out(out)
        _lib.check(self._lib.vecchia_inverse(ctypes.byref(self.view), ctypes.c_void_p(v.data_ptr()),
                                             ctypes.c_void_p(xi.data_ptr()), _stream(self.dg.device)),
                   "vecchia_inverse")
        return xi

    def logdet(self, out=None):
        """log det of the Vecchia covariance, as a 1-element float64 device tensor."""
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.dg.device)
        _lib.check(self._lib.vecchia_logdet(ctypes.byref(self.view), ctypes.c_void_p(out.data_ptr()),
                                            _stream(self.dg.device)), "vecchia_logdet")
        return out

    def status(self):
        """Synchronise and raise VecchiaError(ENOTPD) if a pivot failed."""
        bad = ctypes.c_int64()
        _lib.check(self._lib.vecchia_status(ctypes.byref(self.view), _stream(self.dg.device), ctypes.byref(bad)),
                   "vecchia_status")
        return None

    def backward(self, xi, v, v_bar=None, xi_bar_in=None, logdet_bar=0.0, scratch=None):
        """Reverse-mode derivatives of <v_bar, F xi> + <xi_bar_in, F^-1 v> +
        logdet_bar * logdet.  (xi, v) is the forward pair.  Returns
        (xi_bar or None, v_bar_out or None, theta_bar) with theta_bar a float64
        device tensor [d/dsigma, d/dell].  Needs a DeviceGraph built with
        with_children=True."""
        if self.dg.child_ptr is None:
            raise ValueError("backward needs the children lists: to_device(..., with_children=True)")
        xi = self._vec(xi, "xi")
        v = self._vec(v, "v")
        vb = self._vec(v_bar, "v_bar") if v_bar is not None else None
        xb = self._vec(xi_bar_in, "xi_bar_in") if xi_bar_in is not None else None
        xi_bar = torch.empty_like(xi) if vb is not None else None
        v_bar_out = torch.empty_like(v) if xb is not None else None
        theta = torch.empty(2, dtype=torch.float64, device=self.dg.device)
        nbytes = ctypes.c_size_t()
        _lib.check(self._lib.vecchia_backward_scratch_bytes(ctypes.byref(self.view), ctypes.byref(nbytes)),
                   "vecchia_backward_scratch_bytes")
        if scratch is None or scratch.numel() < nbytes.value:
            scratch = torch.empty(nbytes.value, dtype=torch.uint8, device=self.dg.device)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        _lib.check(self._lib.vecchia_backward(ctypes.byref(self.view), ctypes.byref(self._kc), ptr(xi), ptr(v),
                                              ptr(vb), ptr(xb), float(logdet_bar), ptr(xi_bar), ptr(v_bar_out),
                                              ptr(theta), ptr(scratch), scratch.numel(), _stream(self.dg.device)),
                   "vecchia_backward")
        return xi_bar, v_bar_out, theta

    def backward_x(self, xi, v, v_bar=None, xi_bar_in=None, logdet_bar=0.0, scratch=None):
        """Derivative of <v_bar, F xi> + <xi_bar_in, F^-1 v> + logdet_bar *
        logdet with respect to the point coordinates at this graph: a float64
        device tensor (N, 3) in storage order (the cotangent of the view's x).
        Needs a DeviceGraph built with with_children=True."""
        if self.dg.child_ptr is None:
            raise ValueError("backward_x needs the children lists: to_device(..., with_children=True)")
        xi = self._vec(xi, "xi")
        v = self._vec(v, "v")
        vb = self._vec(v_bar, "v_bar") if v_bar is not None else None
        xb = self._vec(xi_bar_in, "xi_bar_in") if xi_bar_in is not None else None
        x_bar = torch.empty((self.dg.n, 3), dtype=torch.float64, device=self.dg.device)
        nbytes = ctypes.c_size_t()
        _lib.check(self._lib.vecchia_backward_x_scratch_bytes(ctypes.byref(self.view), ctypes.byref(nbytes)),
                   "vecchia_backward_x_scratch_bytes")
        if scratch is None or scratch.numel() < nbytes.value:
            scratch = torch.empty(nbytes.value, dtype=torch.uint8, device=self.dg.device)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        _lib.check(self._lib.vecchia_backward_x(ctypes.byref(self.view), ctypes.byref(self._kc), ptr(xi), ptr(v),
                                                ptr(vb), ptr(xb), float(logdet_bar), ptr(x_bar), ptr(scratch),
                                                scratch.numel(), _stream(self.dg.device)), "vecchia_backward_x")
        return x_bar

    def jvp(self, xi, v, xi_dot=None, sigma_dot=0.0, ell_dot=0.0, logdet=True, scratch=None):
        """Forward-mode derivative: (v_dot, logdet_dot or None) of v = F(xi)
        and of the logdet in the direction (xi_dot, sigma_dot, ell_dot); (xi,
        v) is the forward pair of this factor."""
        xi = self._vec(xi, "xi")
        v = self._vec(v, "v")
        xd = self._vec(xi_dot, "xi_dot") if xi_dot is not None else None
        v_dot = torch.empty_like(v)
        ld = torch.empty(1, dtype=torch.float64, device=self.dg.device) if logdet else None
        nbytes = ctypes.c_size_t()
        _lib.check(self._lib.vecchia_jvp_scratch_bytes(ctypes.byref(self.view), ctypes.byref(nbytes)),
                   "vecchia_jvp_scratch_bytes")
        if scratch is None or scratch.numel() < nbytes.value:
            scratch = torch.empty(nbytes.value, dtype=torch.uint8, device=self.dg.device)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        _lib.check(self._lib.vecchia_forward_jvp(ctypes.byref(self.view), ctypes.byref(self._kc), ptr(xi), ptr(v),
                                                 ptr(xd), float(sigma_dot), float(ell_dot), ptr(v_dot), ptr(ld),
                                                 ptr(scratch), scratch.numel(), _stream(self.dg.device)),
                   "vecchia_forward_jvp")
        return v_dot, ld

    def counts(self):
        """(points with a non-positive pivot or variance, points recomputed in
        double on the FP32 path) of the last factorisation; synchronises."""
        bad, redo = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(self._lib.vecchia_factor_counts(ctypes.byref(self.view), _stream(self.dg.device),
                                                   ctypes.byref(bad), ctypes.byref(redo)), "vecchia_factor_counts")
        return bad.value, redo.value

    def first_bad_slot(self):
        bad = ctypes.c_int64()
        rc = self._lib.vecchia_status(ctypes.byref(self.view), _stream(self.dg.device), ctypes.byref(bad))
        if rc not in (_lib.OK, _lib.ENOTPD):
            _lib.check(rc, "vecchia_status")
        return bad.value

    def _ws_slice(self, name):
        """Read-only views of the factor arrays (tests and diagnostics)."""
        lay = _layout(self.dg)
        esz = 8 if self.dg.precision == FP64 else 4
        dt = self.dg.dtype
        ws = self.workspace
        if name == "b":
            nb = self.dg_ntiles() * self.dg.kp * 64
            return ws[lay["b"]:lay["b"] + nb * esz].view(dt)
        if name == "sigma":
            return ws[lay["sigma"]:lay["sigma"] + self.dg_ntiles() * 64 * esz].view(dt)
        if name == "L0":
            n0 = self.dg.n0
            return ws[lay["l0"]:lay["l0"] + n0 * n0 * 8].view(torch.float64).view(n0, n0)
        raise KeyError(name)

    def dg_ntiles(self):
        return (self.dg.n - self.dg.n0 + 63) // 64

    def coefficient_rows(self, rows):
        """(b (len(rows), kp), sigma (len(rows),)) of the given sparse indices,
        gathered on the device and copied to the host."""
        rows = torch.as_tensor(np.asarray(rows, dtype=np.int64), device=self.dg.device)
        nt, kp = self.dg_ntiles(), self.dg.kp
        b = self._ws_slice("b").view(nt, kp, 64)[rows // 64, :, rows % 64]
        s = self._ws_slice("sigma")[rows]
        return b.cpu().numpy(), s.cpu().numpy()

    def coefficients(self):
        """(b as (Ns, kp) in sparse-index order, sigma (Ns,)) copied to the host."""
        nt, kp, ns = self.dg_ntiles(), self.dg.kp, self.dg.n - self.dg.n0
        b = self._ws_slice("b").cpu().numpy().reshape(nt, kp, 64).transpose(0, 2, 1).reshape(nt * 64, kp)[:ns]
        s = self._ws_slice("sigma").cpu().numpy()[:ns]
        return b, s


class FusedForward:
    """Alg. 1 fused and on the fly: ``vecchia_forward_fused`` recomputes each
    point's K_cc, factor and conditional mean inside the batch loop and
    stores no coefficients; the workspace holds only L0, per-tile log-sigma
    sums and a status word."""

    def __init__(self, dg, kernel, workspace=None):
        self._lib = _lib.load()
        self.dg = dg
        self.kernel = kernel
        out = ctypes.c_size_t()
        _lib.check(self._lib.vecchia_fused_workspace_bytes(dg.n, dg.k, dg.n0, dg.precision, ctypes.byref(out)),
                   "vecchia_fused_workspace_bytes")
        nbytes = out.value
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=dg.device)
        if workspace.numel() < nbytes or workspace.data_ptr() % 256:
            raise ValueError("workspace must hold %d bytes, 256-byte aligned" % nbytes)
        self.workspace = workspace
        v = _lib.ViewStruct()
        v.n, v.k, v.kp, v.n0, v.n_levels, v.precision = dg.n, dg.k, dg.kp, dg.n0, dg.n_levels, dg.precision
        v.x = dg.x.data_ptr()
        v.nbr = dg.nbr.data_ptr()
        v.level_ptr = dg.level_ptr.ctypes.data
        v.workspace = workspace.data_ptr()
        v.workspace_bytes = workspace.numel()
        self.view = v
        self._kc = kernel.to_c()

    def __call__(self, xi, out=None, logdet=None):
        """v = F(xi) in storage order; if ``logdet`` is a 1-element float64
        device tensor it receives the log-determinant of the same pass."""
        if not isinstance(xi, torch.Tensor) or xi.device != self.dg.device or xi.dtype != self.dg.dtype \
                or xi.numel() != self.dg.n or not xi.is_contiguous():
            raise ValueError("xi must be a contiguous %s tensor of %d elements" % (self.dg.dtype, self.dg.n))
        v = torch.empty_like(xi) if out is None else out
        ld = ctypes.c_void_p(logdet.data_ptr()) if logdet is not None else None
        _lib.check(self._lib.vecchia_forward_fused(ctypes.byref(self.view), ctypes.byref(self._kc),
                                                   ctypes.c_void_p(xi.data_ptr()), ctypes.c_void_p(v.data_ptr()), ld,
                                                   _stream(self.dg.device)), "vecchia_forward_fused")
        return v

    def status(self):
        bad = ctypes.c_int64()
        _lib.check(self._lib.vecchia_fused_status(ctypes.byref(self.view), _stream(self.dg.device), ctypes.byref(bad)),
                   "vecchia_fused_status")


def _align(x):
    return (x + 255) & ~255


def _layout(dg):
    """Byte offsets of the workspace regions; mirrors the library's layout
    (checked against vecchia_workspace_bytes in the tests)."""
    ns = dg.n - dg.n0
    ntiles = (ns + 63) // 64
    esz = 8 if dg.precision == FP64 else 4
    off = 0
    lay = {"b": off}
    off = _align(off + ntiles * dg.kp * 64 * esz)
    lay["sigma"] = off
    off = _align(off + ntiles * 64 * esz)
    lay["l0"] = off
    return lay


def profile_enable(on=True):
    """Per-kernel HIP-event timing inside the library (adds two event records
    per launch on the launch stream)."""
    lib = _lib.load()
    _lib.check(lib.vecchia_profile_enable(1 if on else 0), "vecchia_profile_enable")


def profile_reset():
    _lib.check(_lib.load().vecchia_profile_reset(), "vecchia_profile_reset")


def profile_read(max_kernels=64):
    """{kernel name: (total milliseconds, launches)}; synchronises the device."""
    lib = _lib.load()
    names = ctypes.create_string_buffer(8192)
    ms = (ctypes.c_double * max_kernels)()
    cnt = (ctypes.c_int64 * max_kernels)()
    nk = ctypes.c_int32()
    _lib.check(lib.vecchia_profile_read(names, 8192, ms, cnt, max_kernels, ctypes.byref(nk)), "vecchia_profile_read")
    keys = names.value.decode().split("\n")[:nk.value]
    return {k: (ms[i], cnt[i]) for i, k in enumerate(keys)}

"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and map its storage-order results to the oracle's slot order."""
import numpy as np
import torch

import oracle
from paper_2606_11402_amd import FP32, FP64, Factor, Graph, KernelParams


def rel_err(a, ref):
    """max |a - ref| / max |ref| (vectors), |a - ref| / |ref| (scalars)."""
    a, ref = np.asarray(a, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref)) if ref.size else 1.0
    return float(np.max(np.abs(a - ref)) / den) if ref.size else 0.0


def b_backward_error(og, kern, b, chunk=2048):
    """Largest normwise backward error of the coefficient rows b (slot order,
    (Ns, k)) as solutions of K_cc b = k_ci, with K_cc and k_ci evaluated in
    FP64 by the oracle: max_i |K b - k|_inf / (|K|_inf |b|_inf + |k|_inf).
    A backward-stable solve gives a few units of roundoff whatever cond(K_cc)
    is, while the forward error of b grows with cond(K_cc)."""
    from oracle.covariance import kappa
    xs, n0 = og.xs, og.n0
    ns, k = og.nbr.shape
    worst = 0.0
    for c0 in range(0, ns, chunk):
        rows = og.nbr[c0:c0 + chunk]
        ok = rows >= 0
        xc = xs[np.maximum(rows, 0)]                                  # (m, k, d)
        xt = xs[n0 + c0:n0 + c0 + len(rows)]                          # (m, d)
        r = np.sqrt(np.sum((xc[:, :, None, :] - xc[:, None, :, :]) ** 2, axis=-1))
        K = kappa(r, kern) + kern.nugget * np.eye(k)
        mask = ok[:, :, None] & ok[:, None, :]
        K = np.where(mask, K, np.eye(k))
        kc = np.where(ok, kappa(np.sqrt(np.sum((xc - xt[:, None, :]) ** 2, axis=-1)), kern), 0.0)
        bb = np.where(ok, np.asarray(b[c0:c0 + len(rows)], dtype=np.float64), 0.0)
        res = np.einsum("mij,mj->mi", K, bb) - kc
        den = np.abs(K).sum(axis=2).max(axis=1) * np.abs(bb).max(axis=1) + np.abs(kc).max(axis=1)
        worst = max(worst, float(np.max(np.abs(res).max(axis=1) / den)))
    return worst


class Run:
    """Build the graph, upload, factor, forward(xi), inverse(v) on the GPU."""

    def __init__(self, x, k, n0, kern, precision, xi_input=None, device="cuda:0", redo_log2=0):
        self.g = Graph(x, k, n0)
        self.kern = kern
        self.precision = precision
        self.dg = self.g.to_device(precision, device)
        self.fac = Factor(self.dg, KernelParams(kern.kind, kern.sigma, kern.ell, kern.nugget, kern.nu),
                          redo_log2=redo_log2)
        self.dtype = torch.float64 if precision == FP64 else torch.float32
        self.xi_input = xi_input
        if xi_input is not None:
            xi_s = torch.from_numpy(self.g.to_storage(xi_input)).to(self.dtype).to(device)
            self.v = self.fac.forward(xi_s)
            self.xi_back = self.fac.inverse(self.v)
        self.ld = self.fac.logdet()
        torch.cuda.synchronize()

    # storage <-> slot
    def slot_order(self, storage_values):
        out = np.empty_like(storage_values)
        out[self.g.slot] = storage_values
        return out

    def coefficients_by_slot(self):
        """(b rows, sigma) for sparse slots n0.. in slot order, each b row in
        the order of the graph's rows (ascending distance, as the oracle)."""
        b, s = self.fac.coefficients()
        b = self.g.to_row_order(b)
        n0 = self.g.n0
        rows = self.g.slot[n0:] - n0
        bo = np.empty((self.g.ns, self.g.k))
        so = np.empty(self.g.ns)
        bo[rows] = b
        so[rows] = s
        return bo, so

    def oracle_state(self):
        """The GPU's own factor (L0, b, sigma) as an oracle.Factor in slot
        order: the oracle's forward, inverse and logdet evaluated on it
        isolate the level kernels from the conditioning of Eq. (2)."""
        b, s = self.coefficients_by_slot()
        l0 = self.fac._ws_slice("L0").cpu().numpy().copy()   # dense block: storage order = slot order
        return oracle.Factor(L0=l0, b=b, sigma=s.astype(np.float64))

    def storage_rounded(self, a):
        """Values as the device holds them in this run's storage precision."""
        a = np.asarray(a, dtype=np.float64)
        return a.astype(np.float32).astype(np.float64) if self.precision == FP32 else a


def check_capped(errs, tol, caps, names):
    """Metrics above the bar must be listed in caps (name -> largest
    accepted value, a regression cap set from the measured error with a
    stated margin) and stay under it; returns the misses for an xfail."""
    missed = []
    for name in names:
        if errs[name] > tol:
            assert name in caps, ("%s = %.3e above the bar %g and not a capped metric" % (name, errs[name], tol))
            assert errs[name] <= caps[name], ("%s = %.3e above its regression cap %.1e" % (name, errs[name],
                                                                                          caps[name]))
            missed.append("%s=%.2e (cap %.0e)" % (name, errs[name], caps[name]))
    return missed


def oracle_run(x, k, n0, kern, xi_input=None):
    og = oracle.build_graph(x, k, n0)
    fac = oracle.factor(og, kern)
    out = {"graph": og, "fac": fac, "logdet": oracle.logdet(fac)}
    if xi_input is not None:
        xi = np.asarray(xi_input)[og.perm]
        out["xi"] = xi
        out["v"] = oracle.forward(og, fac, xi)
    return out


def precision_of(name):
    return FP64 if name == "fp64" else FP32

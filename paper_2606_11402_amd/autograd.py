"""torch.autograd wrappers: forward v = F(xi), inverse xi = F^-1(v) and logdet,
differentiable with respect to the white noise / field and the kernel
parameters (sigma, ell) through vecchia_backward.  Marshalling only."""
import torch

from .vecchia import FP64, Factor, KernelParams


class GaussianProcess:
    """A point set on the device with a kernel family.  Factors are computed
    on demand for the requested (sigma, ell) and cached per parameter pair
    (the last ``cache`` pairs), so a forward and a logdet at the same
    parameters share one factor and its workspace."""

    def __init__(self, graph, kind, nugget=0.0, precision=FP64, device="cuda", cache=2):
        self.graph = graph
        self.dg = graph.to_device(precision, device, with_children=True)
        self.kind = kind
        self.nugget = float(nugget)
        self._cache = {}
        self._order = []
        self._size = cache

    @property
    def dtype(self):
        return self.dg.dtype

    def factor(self, sigma, ell):
        key = (float(sigma), float(ell))
        fac = self._cache.get(key)
        if fac is None:
            fac = Factor(self.dg, KernelParams(self.kind, key[0], key[1], self.nugget))
            self._cache[key] = fac
            self._order.append(key)
            while len(self._order) > self._size:
                self._cache.pop(self._order.pop(0), None)
        return fac


def _param(x):
    return float(x.detach().item()) if isinstance(x, torch.Tensor) else float(x)


def _theta_grads(theta, sigma, ell):
    gs = theta[0].to(sigma.dtype).reshape(sigma.shape) if isinstance(sigma, torch.Tensor) else None
    gl = theta[1].to(ell.dtype).reshape(ell.shape) if isinstance(ell, torch.Tensor) else None
    return gs, gl


class VecchiaForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi, sigma, ell, gp):
        fac = gp.factor(_param(sigma), _param(ell))
        v = fac.forward(xi.contiguous())
        ctx.save_for_backward(xi, v, sigma, ell)
        ctx.fac = fac
        return v

    @staticmethod
    def backward(ctx, v_bar):
        xi, v, sigma, ell = ctx.saved_tensors
        xi_bar, _, theta = ctx.fac.backward(xi.contiguous(), v, v_bar=v_bar.contiguous())
        gs, gl = _theta_grads(theta, sigma, ell)
        return xi_bar, gs, gl, None


class VecchiaInverse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, sigma, ell, gp):
        fac = gp.factor(_param(sigma), _param(ell))
        xi = fac.inverse(v.contiguous())
        ctx.save_for_backward(v, xi, sigma, ell)
        ctx.fac = fac
        return xi

    @staticmethod
    def backward(ctx, xi_bar):
        v, xi, sigma, ell = ctx.saved_tensors
        _, v_bar, theta = ctx.fac.backward(xi, v.contiguous(), xi_bar_in=xi_bar.contiguous())
        gs, gl = _theta_grads(theta, sigma, ell)
        return v_bar, gs, gl, None


class VecchiaLogdet(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, ell, gp):
        fac = gp.factor(_param(sigma), _param(ell))
        ld = fac.logdet()[0]
        ctx.save_for_backward(sigma, ell)
        ctx.fac = fac
        return ld

    @staticmethod
    def backward(ctx, g):
        sigma, ell = ctx.saved_tensors
        fac = ctx.fac
        zeros = torch.zeros(fac.dg.n, dtype=fac.dg.dtype, device=fac.dg.device)
        _, _, theta = fac.backward(zeros, zeros, logdet_bar=float(g.item()))
        gs, gl = _theta_grads(theta, sigma, ell)
        return gs, gl, None


def forward(gp, xi, sigma, ell):
    """v = F(xi) in storage order, differentiable in xi, sigma, ell."""
    return VecchiaForward.apply(xi, sigma, ell, gp)


def inverse(gp, v, sigma, ell):
    """xi = F^-1(v) in storage order, differentiable in v, sigma, ell."""
    return VecchiaInverse.apply(v, sigma, ell, gp)


def logdet(gp, sigma, ell):
    """log det of the Vecchia covariance, differentiable in sigma, ell."""
    return VecchiaLogdet.apply(sigma, ell, gp)

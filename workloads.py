"""Seeded synthetic inputs for the Vecchia hot path.

This module holds no arithmetic of the method: it only draws point clouds,
white noise and request streams with numpy's default_rng.  Both the HIP path
and the CPU oracle are fed from here, so that they see identical inputs.

Point clouds (all 3-D, FP64):
  * ``uniform``  -- U[0,1)^3.
  * ``radial``   -- isotropic directions with radius 10^U(-3, 0):
                    x = r g/|g|, g ~ N(0, I3)  (large dynamic range).
  * ``clumped``  -- floor(0.9 N) points U[0,1)^3 plus the rest in Gaussian clumps
                    of width 1e-3 around 1024 centres drawn U[0,1)^3 (not clipped).
  * ``gaussian`` -- unit Gaussian, the test distribution the paper uses for its
                    batch-size and timing figures.
``as_fp32_exact`` rounds a cloud to FP32 once; the FP64 values of those floats
are used everywhere (graph, FP64 oracle, FP32 kernels), so every side sees the
same points.

Named workloads (points seed = workload number, white noise seed + 100,
data vector seed + 200):
  1: 4096 uniform, k=8, EXP sigma=1 ell=0.1, FP64
  2: 2^20 radial, k=16, M32 sigma=1 ell=0.05, FP64 and FP32
  3: 2^26 = 90% uniform + 10% clumps, k=32, SE ell=0.02 nugget 1e-6, FP32
  4: 2^22 radial, k=16, M32, FP32 gradients
  5: request stream, N log-uniform in [1e3, 1e6] uniform points, k in {8,16,32},
     ell ~ U(0.01, 0.2), op uniform over {forward, inverse, logdet}, M32 sigma=1
"""
from dataclasses import dataclass

import numpy as np

EXP, M32, SE = 0, 1, 2


def uniform(n, seed):
    return np.random.default_rng(seed).random((n, 3))


def radial(n, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    r = 10.0 ** rng.uniform(-3.0, 0.0, n)
    return g / np.linalg.norm(g, axis=1, keepdims=True) * r[:, None]


def clumped(n, seed, frac=0.1, n_centres=1024, width=1e-3):
    rng = np.random.default_rng(seed)
    n_uniform = int(np.floor((1.0 - frac) * n))
    pts = np.empty((n, 3))
    pts[:n_uniform] = rng.random((n_uniform, 3))
    centres = rng.random((n_centres, 3))
    which = rng.integers(0, n_centres, n - n_uniform)
    pts[n_uniform:] = centres[which] + width * rng.standard_normal((n - n_uniform, 3))
    return pts


def gaussian(n, seed):
    return np.random.default_rng(seed).standard_normal((n, 3))


def white_noise(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def as_fp32_exact(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


@dataclass(frozen=True)
class Workload:
    number: int
    name: str
    n: int
    k: int
    kind: int
    sigma: float
    ell: float
    nugget: float
    dist: str
    precisions: tuple
    n0: int = 128

    def points(self, n=None, fp32=None):
        n = self.n if n is None else n
        gen = {"uniform": uniform, "radial": radial, "clumped": clumped, "gaussian": gaussian}[self.dist]
        x = gen(n, self.number)
        if fp32 is None:
            fp32 = "fp32" in self.precisions      # one FP32-exact cloud serves both precisions
        return as_fp32_exact(x) if fp32 else x

    def xi(self, n=None):
        return white_noise(self.n if n is None else n, self.number + 100)

    def data(self, n=None):
        return white_noise(self.n if n is None else n, self.number + 200)


WORKLOADS = {
    1: Workload(1, "uniform-4096-k8-exp-fp64", 4096, 8, EXP, 1.0, 0.1, 0.0, "uniform", ("fp64",)),
    2: Workload(2, "radial-2^20-k16-m32", 1 << 20, 16, M32, 1.0, 0.05, 0.0, "radial", ("fp64", "fp32")),
    3: Workload(3, "clumped-2^26-k32-se-fp32", 1 << 26, 32, SE, 1.0, 0.02, 1e-6, "clumped", ("fp32",)),
    4: Workload(4, "radial-2^22-k16-m32-adjoint", 1 << 22, 16, M32, 1.0, 0.05, 0.0, "radial", ("fp32",)),
}


@dataclass(frozen=True)
class Request:
    rid: int
    arrival: float       # seconds from the start of the stream
    n: int
    k: int
    ell: float
    op: str              # "forward" | "inverse" | "logdet"
    seed: int


def request_stream(n_requests, rate, seed=5, n_lo=1e3, n_hi=1e6, ks=(8, 16, 32)):
    """Poisson arrivals at ``rate`` requests/s; request r draws its own points
    from seed 5000 + r (uniform cloud, see ``request_points``)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = np.floor(10.0 ** rng.uniform(np.log10(n_lo), np.log10(n_hi), n_requests)).astype(np.int64)
    kk = rng.choice(np.asarray(ks), n_requests)
    ells = rng.uniform(0.01, 0.2, n_requests)
    ops = rng.choice(np.asarray(["forward", "inverse", "logdet"]), n_requests)
    return [Request(r, float(arrivals[r]), int(ns[r]), int(kk[r]), float(ells[r]), str(ops[r]), 5000 + r)
            for r in range(n_requests)]


def request_points(req):
    return as_fp32_exact(uniform(req.n, req.seed))


def request_xi(req):
    return white_noise(req.n, req.seed + 100)

"""Seeded synthetic bunches for the relativistic space-charge FMM.

This module only draws random inputs; it holds none of the method's
arithmetic, so that both the FP64 oracle and the HIP path can be fed from it.

Every workload is drawn from one ``numpy.random.Generator(PCG64(seed))`` in a
fixed order: positions, momenta, sample target indices, loss weights.
Positions are in metres, momenta are the dimensionless u = gamma*beta, and
every macro-particle carries the same charge, -1 nC / N.

Workloads (name: particles; positions; momenta; degree n, leaf size N0, eta).
The configurations name no eta for the larger bunches; since the metric asks
for a relative error of at most 1e-6 against the FP64 direct sum, each takes
the largest eta on a 0.05 grid at which its FP64 FMM meets that bound:
  gauss4k    4,096;     Gaussian sigma (1, 1, 0.1) mm; u_z ~ N(20, 0.2^2),
             u_x, u_y ~ N(0, 0.01^2); n=4, N0=64, eta=0.5
  gauss131k  131,072;   as gauss4k; u_z ~ N(100, 1), u_x, u_y ~ N(0, 0.05^2);
             n=6, N0=256, eta=0.35
  chirp1m    1,048,576; uniform in an ellipsoid with semi-axes (1, 1, 0.05) mm;
             u_z = 50 + 5 z/(0.05 mm) + N(0, 0.5^2), u_x, u_y ~ N(0, 0.02^2);
             n=8, N0=512, eta=0.45
  adjoint262k 262,144;  as gauss131k, plus loss weights w, a, b ~ N(0, 1);
             n=6, N0=256, eta=0.35
  halo8m     8,388,608; 90% core Gaussian sigma (1, 1, 0.1) mm and 10% halo
             Gaussian sigma (5, 5, 0.5) mm; u_z = 100 exp(0.1 Z), Z ~ N(0,1),
             u_x, u_y ~ N(0, 0.1^2); n=8, N0=512, eta=0.4
  cube       the accuracy study of Sec. 6: uniform in the unit cube [0,1]^3 m,
             every particle with u = (0, 0, sqrt(gamma^2 - 1)), gamma = 50;
             N0 = (n+1)^3
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

MM = 1.0e-3
TOTAL_CHARGE = -1.0e-9


@dataclass
class Workload:
    name: str
    x: np.ndarray
    u: np.ndarray
    q: np.ndarray
    degree: int
    leaf_size: int
    eta: float
    seed: int
    sample: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.x.shape[0]


SPECS = {
    "gauss4k": dict(n=4096, degree=4, leaf_size=64, eta=0.5),
    "gauss131k": dict(n=131072, degree=6, leaf_size=256, eta=0.35),
    "chirp1m": dict(n=1048576, degree=8, leaf_size=512, eta=0.45),
    "adjoint262k": dict(n=262144, degree=6, leaf_size=256, eta=0.35),
    "halo8m": dict(n=8388608, degree=8, leaf_size=512, eta=0.4),
    "cube": dict(n=1280000, degree=4, leaf_size=125, eta=0.5),
}


def _gauss(rng, n, sigma):
    return rng.standard_normal((n, 3)) * np.asarray(sigma, np.float64)


def _ellipsoid(rng, n, semi):
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.random(n) ** (1.0 / 3.0)
    return d * r[:, None] * np.asarray(semi, np.float64)


def make(name, seed=0, n=None, degree=None, leaf_size=None, eta=None,
         n_sample=4096):
    """Draw workload ``name``; ``n`` and the method parameters may be
    overridden to get a smaller bunch of the same shape."""
    spec = dict(SPECS[name])
    if n is not None:
        spec["n"] = int(n)
    if degree is not None:
        spec["degree"] = int(degree)
        if name == "cube" and leaf_size is None:
            spec["leaf_size"] = (int(degree) + 1) ** 3
    if leaf_size is not None:
        spec["leaf_size"] = int(leaf_size)
    if eta is not None:
        spec["eta"] = float(eta)
    N = spec["n"]
    rng = np.random.Generator(np.random.PCG64(seed))
    extra = {}
    if name in ("gauss4k", "gauss131k", "adjoint262k"):
        x = _gauss(rng, N, (MM, MM, 0.1 * MM))
        u = np.empty((N, 3))
        if name == "gauss4k":
            u[:, 2] = rng.normal(20.0, 0.2, N)
            u[:, :2] = rng.normal(0.0, 0.01, (N, 2))
        else:
            u[:, 2] = rng.normal(100.0, 1.0, N)
            u[:, :2] = rng.normal(0.0, 0.05, (N, 2))
    elif name == "chirp1m":
        x = _ellipsoid(rng, N, (MM, MM, 0.05 * MM))
        u = np.empty((N, 3))
        u[:, 2] = 50.0 + 5.0 * x[:, 2] / (0.05 * MM) + rng.normal(0.0, 0.5, N)
        u[:, :2] = rng.normal(0.0, 0.02, (N, 2))
    elif name == "halo8m":
        nc = int(0.9 * N)
        x = np.concatenate([_gauss(rng, nc, (MM, MM, 0.1 * MM)),
                            _gauss(rng, N - nc, (5 * MM, 5 * MM, 0.5 * MM))])
        u = np.empty((N, 3))
        u[:, 2] = 100.0 * np.exp(0.1 * rng.standard_normal(N))
        u[:, :2] = rng.normal(0.0, 0.1, (N, 2))
    elif name == "cube":
        x = rng.random((N, 3))
        u = np.zeros((N, 3))
        u[:, 2] = np.sqrt(50.0 ** 2 - 1.0)
    else:
        raise KeyError(name)
    q = np.full(N, TOTAL_CHARGE / N)
    k = min(n_sample, N)
    sample = np.sort(rng.choice(N, k, replace=False)).astype(np.int64)
    if name == "adjoint262k":
        extra["w"] = rng.standard_normal(N)
        extra["a"] = rng.standard_normal((N, 3))
        extra["b"] = rng.standard_normal((N, 3))
    return Workload(name=name, x=np.ascontiguousarray(x),
                    u=np.ascontiguousarray(u), q=q, degree=spec["degree"],
                    leaf_size=spec["leaf_size"], eta=spec["eta"], seed=seed,
                    sample=sample, extra=extra)

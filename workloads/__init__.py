"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the bench.

This module holds no arithmetic of the integrator: it only builds the problem
data that the paper's algorithms take as input (Section 3 and Algorithms 1-2:
the initial tensor U0, the one-dimensional matrices A_1..A_d that make up the
Kronecker sum K, the reaction parameters, tau and the number of steps).

Conventions
-----------
* A d-way tensor is stored with index i_1 fastest ("vec stacks by columns",
  Section 2).  In numpy it is an array of shape (n_1, ..., n_d) in Fortran
  order; the flat buffer handed to the GPU is ``x.ravel(order="F")``.
* The discrete Laplacian with homogeneous Neumann boundary conditions is the
  vertex-centred, ghost-point second-order stencil: x_j = j*h, h = L/(n-1),
  rows 2..n-1 are (1, -2, 1)/h^2, row 1 is (-2, 2)/h^2 and row n is (2, -2)/h^2
  (Section 3 says only "second order centred finite differences with the
  boundary conditions built into the matrices"; this is the reading taken).
* Random numbers come from numpy's PCG64 (``np.random.default_rng(seed)``),
  drawn in memory order, component u with seed ``2k`` and v with ``2k+1`` for
  instance k (k = 0 for single runs).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

G_NONE = 0
G_SCHNAKENBERG = 1
G_FHN = 2


def neumann_d2(n: int, length: float = 1.0) -> np.ndarray:
    """Second-order FD Laplacian on n vertices of [0, length], homogeneous
    Neumann via ghost points.  Dense n x n, column-major semantics (a plain
    numpy 2-D array; entry [i, j] is row i, column j)."""
    if n < 2:
        raise ValueError("need at least two grid points")
    h = length / (n - 1)
    D = np.zeros((n, n))
    idx = np.arange(1, n - 1)
    D[idx, idx - 1] = 1.0
    D[idx, idx] = -2.0
    D[idx, idx + 1] = 1.0
    D[0, 0], D[0, 1] = -2.0, 2.0
    D[n - 1, n - 2], D[n - 1, n - 1] = 2.0, -2.0
    return D / (h * h)


@dataclass
class Problem:
    """One two-component reaction-diffusion instance (eq. twocompdisc)."""
    name: str
    dims: Tuple[int, ...]                 # (n_1, ..., n_d)
    A: List[List[np.ndarray]]             # A[c][mu], c in {0: u, 1: v}
    g_kind: int
    params: Tuple[float, ...]
    tau: float
    nsteps: int
    U0: List[np.ndarray] = field(default_factory=list)   # per component, Fortran (n_1..n_d)

    @property
    def d(self) -> int:
        return len(self.dims)

    @property
    def N(self) -> int:
        return int(np.prod(self.dims))

    def u0_flat(self) -> np.ndarray:
        """Both components, component-major, each Fortran-ordered."""
        return np.concatenate([x.ravel(order="F") for x in self.U0])


def _field(rng: np.random.Generator, dims, kind: str, a: float, b: float) -> np.ndarray:
    n = int(np.prod(dims))
    if kind == "uniform":
        flat = rng.uniform(a, b, size=n)
    elif kind == "normal":
        flat = rng.normal(a, b, size=n)
    else:
        raise ValueError(kind)
    return flat.reshape(dims, order="F")


def schnakenberg_2d(n1: int = 64, n2: int | None = None, *, du: float = 1.0, dv: float = 10.0,
                    gamma: float = 100.0, a: float = 0.1, b: float = 0.9, noise: float = 0.01,
                    tau: float = 1e-3, nsteps: int = 50, length: float = 1.0,
                    instance: int = 0) -> Problem:
    """2D Schnakenberg (Section 3.1 model, parameters of the 64x64 workload):
    g1 = gamma(a - u + u^2 v), g2 = gamma(b - u^2 v); u0, v0 = steady state
    (a+b, b/(a+b)^2) plus U(-noise, noise)."""
    n2 = n1 if n2 is None else n2
    dims = (n1, n2)
    D = [neumann_d2(n1, length), neumann_d2(n2, length)]
    A = [[du * D[0], du * D[1]], [dv * D[0], dv * D[1]]]
    ue, ve = a + b, b / (a + b) ** 2
    U0 = [ue + _field(np.random.default_rng(2 * instance), dims, "uniform", -noise, noise),
          ve + _field(np.random.default_rng(2 * instance + 1), dims, "uniform", -noise, noise)]
    return Problem("schnakenberg2d", dims, A, G_SCHNAKENBERG, (gamma, a, b), tau, nsteps, U0)


def fhn_3d(n: int = 128, *, du: float = 1.0, dv: float = 42.1, eps: float = 0.5, a1: float = 2.0,
           a0: float = 0.0, sigma: float = 0.01, tau: float = 1e-2, nsteps: int = 100,
           length: float = 1.0, dims: Sequence[int] | None = None, instance: int = 0) -> Problem:
    """3D FitzHugh-Nagumo (Section 3.2 model, re-parameterised as in the
    128^3 / 256^3 workloads): g1 = u - u^3 - v, g2 = eps (u - a1 v - a0);
    u0, v0 ~ N(0, sigma^2)."""
    dims = tuple(dims) if dims is not None else (n, n, n)
    D = [neumann_d2(m, length) for m in dims]
    A = [[du * Dm for Dm in D], [dv * Dm for Dm in D]]
    U0 = [_field(np.random.default_rng(2 * instance), dims, "normal", 0.0, sigma),
          _field(np.random.default_rng(2 * instance + 1), dims, "normal", 0.0, sigma)]
    return Problem("fhn3d", dims, A, G_FHN, (eps, a1, a0), tau, nsteps, U0)


def smooth_fields(dims: Sequence[int], length: float = 1.0) -> List[np.ndarray]:
    """Smooth (low cosine mode) initial data for temporal-order studies:
    u = 0.1 cos(pi x1) cos(2 pi x2) [+ 0.05 cos(pi x3)], v = 0.05 cos(pi x2) [+ 0.02 cos(2 pi x3)]."""
    axes = [np.linspace(0.0, length, m) for m in dims]
    grids = np.meshgrid(*axes, indexing="ij")
    x1, x2 = grids[0], grids[1]
    u = 0.1 * np.cos(np.pi * x1) * np.cos(2 * np.pi * x2)
    v = 0.05 * np.cos(np.pi * x2)
    if len(dims) == 3:
        u = u + 0.05 * np.cos(np.pi * grids[2])
        v = v + 0.02 * np.cos(2 * np.pi * grids[2])
    return [np.asfortranarray(u), np.asfortranarray(v)]


def random_tensor(dims: Sequence[int], seed: int, scale: float = 1.0) -> np.ndarray:
    """Uniform(-scale, scale) tensor in Fortran order (generic kernel tests)."""
    return _field(np.random.default_rng(seed), tuple(dims), "uniform", -scale, scale)


def random_matrix(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-scale, scale, size=(n, n))


# Workloads used by tests and the bench (sizes, parameters and step counts of
# the three benchmark configurations).
BATCH_SIDES = (64, 96, 128, 192, 256, 384, 512)


def schnakenberg_batch(nbatch: int = 64, *, sides: Sequence[int] = BATCH_SIDES, dv_range=(8.0, 12.0),
                       seed: int = 12345, tau: float = 1e-3, nsteps: int = 100) -> List[Problem]:
    """Batch of independent 2D Schnakenberg instances of uneven size: each side
    drawn from `sides` (non-square grids allowed), d_v ~ U(dv_range), both
    from a PCG64 stream seeded with `seed`; instance k draws its initial noise
    from seeds 2k (u) and 2k+1 (v).  Kinetics and tau as the 64 x 64 case."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(nbatch):
        n1, n2 = (int(x) for x in rng.choice(np.asarray(sides), size=2))
        dv = float(rng.uniform(*dv_range))
        out.append(schnakenberg_2d(n1, n2, dv=dv, tau=tau, nsteps=nsteps, instance=k))
    return out


CONFIGS: Dict[str, dict] = {
    "schnakenberg2d_64": dict(builder="schnakenberg_2d", kwargs=dict(n1=64)),
    "fhn3d_128": dict(builder="fhn_3d", kwargs=dict(n=128, nsteps=100)),
    "fhn3d_256": dict(builder="fhn_3d", kwargs=dict(n=256, nsteps=200)),
}


def make(config: str, **overrides) -> Problem:
    spec = CONFIGS[config]
    kw = dict(spec["kwargs"])
    kw.update(overrides)
    return globals()[spec["builder"]](**kw)

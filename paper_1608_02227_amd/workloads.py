"""Seeded synthetic inputs for least-squares convex regression fits.

Each generator returns ``(x, ybar)`` in float64: ``x`` is N x n row-major (row l is the
location x_l) and ``ybar`` holds the noisy observations ybar_l = f0(x_l) + eps_l of the
data model (Section 1, eq. ``data``).  The paper's own workloads are synthetic as well
(Section 4, experimental setup); the shapes and distributions below are the ones the
benchmarks and tests are quoted on.

This module draws random numbers and evaluates the ground-truth convex functions f0.  It
holds none of the fitting method's arithmetic, so the CPU oracle and the GPU path can both
consume its output without sharing any solver code.

Conventions: one ``numpy.random.Generator(PCG64(seed))`` per workload; draws happen in the
order locations, f0 parameters, noise; ``N(0, s^2)`` means standard deviation ``s``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "make",
    "sq_norm",
    "quadratic_form",
    "log_sum_exp_affine",
    "max_affine_plus_quadratic",
    "paper_shaped",
    "serving_requests",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sq_norm(N: int, n: int, noise: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """x ~ U[-1,1]^n, f0(x) = ||x||^2, eps ~ N(0, noise^2)."""
    g = _rng(seed)
    x = g.uniform(-1.0, 1.0, size=(N, n))
    f = np.einsum("ij,ij->i", x, x)
    return x, f + noise * g.standard_normal(N)


def quadratic_form(N: int, n: int, noise: float, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """x ~ U[-1,1]^n, f0(x) = x^T Q x with Q = M^T M / n, M iid N(0,1), eps ~ N(0, noise^2)."""
    g = _rng(seed)
    x = g.uniform(-1.0, 1.0, size=(N, n))
    M = g.standard_normal((n, n))
    Q = M.T @ M / n
    f = np.einsum("ij,jk,ik->i", x, Q, x)
    return x, f + noise * g.standard_normal(N)


def log_sum_exp_affine(N: int, n: int, pieces: int, noise: float, seed: int,
                       x_dist: str = "normal") -> tuple[np.ndarray, np.ndarray]:
    """x ~ N(0, I_n) (or U[-1,1]^n), f0(x) = log sum_k exp(a_k^T x + b_k), a_k ~ N(0,I), b_k ~ N(0,1)."""
    g = _rng(seed)
    x = g.standard_normal((N, n)) if x_dist == "normal" else g.uniform(-1.0, 1.0, size=(N, n))
    a = g.standard_normal((pieces, n))
    b = g.standard_normal(pieces)
    z = x @ a.T + b
    zmax = z.max(axis=1)
    f = zmax + np.log(np.exp(z - zmax[:, None]).sum(axis=1))
    return x, f + noise * g.standard_normal(N)


def max_affine_plus_quadratic(N: int, n: int, pieces: int, curvature: float, noise: float,
                              seed: int) -> tuple[np.ndarray, np.ndarray]:
    """x ~ N(0, I_n), f0(x) = max_k (a_k^T x + b_k) + curvature * ||x||^2, a_k ~ N(0,I), b_k ~ N(0,1)."""
    g = _rng(seed)
    x = g.standard_normal((N, n))
    a = g.standard_normal((pieces, n))
    b = g.standard_normal(pieces)
    f = (x @ a.T + b).max(axis=1) + curvature * np.einsum("ij,ij->i", x, x)
    return x, f + noise * g.standard_normal(N)


def paper_shaped(N: int, n: int, kind: str, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """The generator of the paper's Section 4 experimental setup.

    x ~ N(0, 4 I_n), eps ~ N(0, 100); f0 = 0.5 x^T Q x with Q = V diag(s) V^T whose singular
    values are rescaled linearly to condition number 15 (from Lam^T Lam, Lam iid N(0,1)), or
    f0 = exp(p^T x) with p ~ U[0, 0.2]^n; then 30% of the points get ybar <- 1.3 ybar.
    The rescaling rule ("transform the singular values to condition number 15") is not given
    in the paper; a linear map of [s_min, s_max] onto [s_max/15, s_max] is used here.
    """
    g = _rng(seed)
    x = 2.0 * g.standard_normal((N, n))
    if kind == "quadratic":
        lam = g.standard_normal((n, n))
        U, s, Vt = np.linalg.svd(lam.T @ lam)
        lo, hi = s.min(), s.max()
        s2 = hi / 15.0 + (s - lo) * (hi - hi / 15.0) / max(hi - lo, 1e-300)
        Q = (U * s2) @ Vt
        Q = 0.5 * (Q + Q.T)
        f = 0.5 * np.einsum("ij,jk,ik->i", x, Q, x)
    elif kind == "exp":
        p = g.uniform(0.0, 0.2, size=n)
        f = np.exp(x @ p)
    else:
        raise ValueError(f"unknown paper-shaped kind {kind!r}")
    ybar = f + 10.0 * g.standard_normal(N)
    moved = g.permutation(N)[: int(round(0.3 * N))]
    ybar[moved] *= 1.3
    return x, ybar


@dataclass(frozen=True)
class Workload:
    name: str
    N: int
    n: int
    delta: float
    tol: float
    description: str

    def generate(self, seed: int = 0) -> tuple[np.ndarray, np.ndarray]:
        return make(self.name, seed=seed)


# The single-fit workloads (sizes and distributions of the benchmark configurations).
WORKLOADS: dict[str, Workload] = {
    "sqnorm_N200_n2": Workload(
        "sqnorm_N200_n2", 200, 2, 1e-3, 1e-6,
        "x~U[-1,1]^2, f0=||x||^2, eps~N(0,0.1^2), delta=1e-3, KKT tol 1e-6"),
    "lse8_N2000_n10": Workload(
        "lse8_N2000_n10", 2000, 10, 1e-3, 1e-6,
        "x~N(0,I_10), f0=log-sum-exp of 8 affine pieces, eps~N(0,0.2^2), delta=1e-3"),
    "quad_N8000_n40": Workload(
        "quad_N8000_n40", 8000, 40, 1e-3, 1e-4,
        "x~U[-1,1]^40, f0=x^T Q x, Q=M^T M/40, eps~N(0,0.5^2), delta=1e-3, KKT tol 1e-4"),
    "maxaff16_N40000_n20": Workload(
        "maxaff16_N40000_n20", 40000, 20, 1e-3, 1e-4,
        "x~N(0,I_20), f0=max of 16 affine pieces + 0.1||x||^2, eps~N(0,0.3^2), delta=1e-3"),
}


def make(name: str, seed: int = 0, N: int | None = None, n: int | None = None
         ) -> tuple[np.ndarray, np.ndarray]:
    """Generate a named workload; ``N``/``n`` override the size but keep the distributions."""
    w = WORKLOADS[name]
    N = w.N if N is None else N
    n = w.n if n is None else n
    if name.startswith("sqnorm"):
        return sq_norm(N, n, 0.1, seed)
    if name.startswith("lse8"):
        return log_sum_exp_affine(N, n, 8, 0.2, seed)
    if name.startswith("quad"):
        return quadratic_form(N, n, 0.5, seed)
    if name.startswith("maxaff16"):
        return max_affine_plus_quadratic(N, n, 16, 0.1, 0.3, seed)
    raise KeyError(name)


@dataclass(frozen=True)
class Request:
    req_id: int
    arrival_s: float
    x: np.ndarray
    ybar: np.ndarray
    delta: float
    tol: float


def serving_requests(count: int = 512, rate_per_s: float = 50.0, n_min_log: float = 100.0,
                     n_max_log: float = 6000.0, dims: tuple[int, int] = (2, 32),
                     delta: float = 1e-3, tol: float = 1e-4, seed: int = 0) -> list[Request]:
    """A Poisson stream of fit requests.

    Inter-arrival times ~ Exp(mean 1/rate); N = round(exp(U[ln n_min, ln n_max])); n uniform in
    ``dims`` (inclusive); x ~ U[-1,1]^n; f0 is ||x||^2 or an 8-piece log-sum-exp with
    probability 1/2 each; eps ~ N(0, 0.1^2).
    """
    g = _rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += g.exponential(1.0 / rate_per_s)
        N = int(round(math.exp(g.uniform(math.log(n_min_log), math.log(n_max_log)))))
        n = int(g.integers(dims[0], dims[1] + 1))
        sub_seed = int(g.integers(0, 2**62))
        if g.uniform() < 0.5:
            x, yb = sq_norm(N, n, 0.1, sub_seed)
        else:
            x, yb = log_sum_exp_affine(N, n, 8, 0.1, sub_seed, x_dist="uniform")
        out.append(Request(r, t, x, yb, delta, tol))
    return out

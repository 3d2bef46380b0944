"""Exact solution of the regularized QP for tiny N, independent of the matrix-free operators.

TEST INFRASTRUCTURE ONLY (see the package docstring): not part of the product path.

The constraint matrices are assembled literally from Definition ``def:A1A2``: T_l in
R^{(N-1) x N} is [e_1 ... e_{l-1}, -1, e_l ... e_{N-1}], A1 stacks T_1 .. T_N, and A2 is block
diagonal with blocks X_l = -T_l X.  Rows come out in the lexicographic pair order of Section 2.

With eta(lam) = (ybar + A1^T lam, A2^T lam / g) (Step 1 with Q the whole space), the dual of
eq. ``eq:dual-problem`` is
    g(lam) = 1/2||ybar||^2 - 1/2||ybar + A1^T lam||^2 - ||A2^T lam||^2 / (2 g),
so maximizing it over lam >= 0 is the non-negative least-squares problem
    min_{lam >= 0} 1/2 || M lam - b ||^2,  M = [A1^T ; A2^T / sqrt(g)],  b = [-ybar ; 0],
which Lawson-Hanson solves exactly (finite active-set method; scipy.optimize.nnls).  M lam* is
unique, hence so are y* and xi*; lam* itself need not be.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import nnls


def t_block(N: int, l: int) -> np.ndarray:
    """T_l of Definition ``def:A1A2`` (0-based l): columns e_1..e_l, then -1, then e_{l+1}.."""
    T = np.zeros((N - 1, N))
    eye = np.eye(N - 1)
    T[:, :l] = eye[:, :l]
    T[:, l] = -1.0
    T[:, l + 1:] = eye[:, l:]
    return T


def explicit_constraints(x: np.ndarray) -> tuple[np.ndarray, np.ndarray, list[tuple[int, int]]]:
    """Dense A1 (N(N-1) x N), A2 (N(N-1) x Nn) and the (l1, l2) pair of every row."""
    N, n = x.shape
    A1 = np.vstack([t_block(N, l) for l in range(N)])
    A2 = np.zeros((N * (N - 1), N * n))
    pairs = []
    for l in range(N):
        T = t_block(N, l)
        A2[l * (N - 1):(l + 1) * (N - 1), l * n:(l + 1) * n] = -T @ x
        pairs.extend((l, j) for j in range(N) if j != l)
    return A1, A2, pairs


def exact_solve(x: np.ndarray, ybar: np.ndarray, gamma: float, maxiter: int | None = None) -> dict:
    """Exact (y*_g, xi*_g), an optimal lam* (N x N, zero diagonal) and p*_g."""
    N, n = x.shape
    A1, A2, pairs = explicit_constraints(x)
    M = np.vstack([A1.T, A2.T / np.sqrt(gamma)])
    b = np.concatenate([-ybar, np.zeros(N * n)])
    theta, _ = nnls(M, b, maxiter=maxiter if maxiter is not None else 50 * M.shape[1])
    y = ybar + A1.T @ theta
    xi = (A2.T @ theta / gamma).reshape(N, n)
    lam = np.zeros((N, N))
    for r, (i, j) in enumerate(pairs):
        lam[i, j] = theta[r]
    p = 0.5 * float(np.sum((y - ybar) ** 2)) + 0.5 * gamma * float(np.sum(xi ** 2))
    cons = A1 @ y + A2 @ xi.reshape(-1)
    return {"y": y, "xi": xi, "lam": lam, "p_star": p, "min_constraint": float(cons.min()),
            "theta": theta, "A1": A1, "A2": A2}


def exact_ls(x: np.ndarray, ybar: np.ndarray) -> dict:
    """The unregularized LS estimator of eq. ``original`` (gamma = 0) for tiny N.

    y* is the projection of ybar onto the cone {y : A1 y + A2 xi >= 0 for some xi}: the convex QP
    in (y, xi) is solved with scipy's SLSQP from the feasible start (mean(ybar), 0).  Its xi is one
    subgradient choice; the least-norm subgradients xi* of eq. ``tikhonov`` (the limit of the
    regularized solutions) solve min ||xi||^2 s.t. A2 xi >= -A1 y*, also by SLSQP.
    """
    from scipy.optimize import minimize
    N, n = x.shape
    A1, A2, _ = explicit_constraints(x)
    A = np.hstack([A1, A2])

    def f(z):
        r = z[:N] - ybar
        return 0.5 * float(r @ r), np.concatenate([r, np.zeros(N * n)])

    z0 = np.concatenate([np.full(N, ybar.mean()), np.zeros(N * n)])
    cons = [{"type": "ineq", "fun": lambda z: A @ z, "jac": lambda z: A}]
    res = minimize(f, z0, jac=True, constraints=cons, method="SLSQP",
                   options={"ftol": 1e-14, "maxiter": 5000})
    y = res.x[:N]
    b = -(A1 @ y)
    res2 = minimize(lambda v: (0.5 * float(v @ v), v), np.zeros(N * n), jac=True,
                    constraints=[{"type": "ineq", "fun": lambda v: A2 @ v - b, "jac": lambda v: A2}],
                    method="SLSQP", options={"ftol": 1e-14, "maxiter": 5000})
    return {"y": y, "xi": res2.x.reshape(N, n), "p_star": 0.5 * float((y - ybar) @ (y - ybar)),
            "success": bool(res.success and res2.success), "message": (res.message, res2.message),
            "min_constraint": float((A1 @ y + A2 @ res2.x).min())}

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

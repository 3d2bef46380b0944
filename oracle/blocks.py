"""P-APG with K-block partial dualization (Section 2.1), plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring): not part of the product path.

Partition (Assumption ``assump:partition``): contiguous blocks C_b = {b p, ..., min(N, (b + 1) p) - 1}
of p points, the last one possibly shorter (the assumption's N = K p made optional).  Only the
constraints of pairs in different blocks are dualized (the partial Lagrangian, eq.
``eq:lagrangian``): the multipliers theta live on those pairs, held as an N x N array whose
entries for pairs inside a block are not variables and stay zero.  The constraints inside the
blocks define the local set Q = Q_1 x ... x Q_K (eq. ``subgradient``), and Step 1 of P-APG splits
into one QP per block (eq. ``subgradient_split``).  With every term written out, block b's QP is
    min_{y_b, xi_b}  1/2 ||y_b - y0_b||^2 + g/2 ||xi_b - xi0_b||^2   s.t.  A1_b y_b + A2_b xi_b >= 0,
(y0, xi0) = (ybar + A1^T theta, A2^T theta / g) being the minimizer over the whole space (the
closed form of the singleton partition): Step 1 projects that point onto Q in the norm of
G = diag(I, g I).  Each block's QP is solved exactly here, by Lawson-Hanson NNLS on its dual as in
``exact`` (the paper's sub-solver is an interior-point method, Section 2.5; the exact solve is the
plain definition it approximates).

The block's dual: with M_b = [A1_b^T ; A2_b^T / sqrt(g)] and b = [-y0_b ; -sqrt(g) xi0_b],
multipliers mu_b >= 0 minimizing 1/2 ||M_b mu - b||^2 give the projection
    y_b = y0_b + A1_b^T mu_b,   xi_b = xi0_b + A2_b^T mu_b / g
(stationarity of the block's Lagrangian; M_b^T b = -(A1_b y0_b + A2_b xi0_b), so the NNLS
objective is the block's dual up to a constant).

The gradient of the partial dual is -C eta(theta) (eq. ``dual gradient``) over the dualized rows
only, so Step 2 updates the inter-block multipliers alone and the Lipschitz constant is
sigma_max(C)^2 / g for C the dualized rows (eq. ``eq:lischitz``).

At a stopping test the report of ``papg.kkt_report`` is taken for the whole problem at the total
multipliers theta + mu (the blocks' own multipliers in the intra-block entries): their closed-form
primal point is the projected eta(theta), so the report's stationarity terms vanish and its
natural residual covers every pair.

Parity pins: ``tests/test_oracle_blocks.py``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import nnls

from .exact import explicit_constraints
from .papg import kkt_report, pair_adjoint, pair_residual, primal_from_dual


def block_ids(N: int, p: int) -> np.ndarray:
    """Block of each point under the contiguous partition with blocks of p points."""
    return np.arange(N) // p


def inter_mask(N: int, p: int) -> np.ndarray:
    """N x N: True for the pairs (i, j) in different blocks (the dualized constraints)."""
    b = block_ids(N, p)
    return b[:, None] != b[None, :]


def project_block(xb: np.ndarray, y0: np.ndarray, xi0: np.ndarray, gamma: float
                  ) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Exact solution of one block's Step-1 QP (eq. ``subgradient_split``): the G-norm projection of
    (y0, xi0) onto the block's pair constraints.  Returns (y_b, xi_b, mu_b), mu_b the block's
    multipliers as a p x p array with zero diagonal."""
    p, n = xb.shape
    if p == 1:
        return y0.copy(), xi0.copy(), np.zeros((1, 1))
    A1, A2, pairs = explicit_constraints(xb)
    M = np.vstack([A1.T, A2.T / math.sqrt(gamma)])
    b = np.concatenate([-y0, -math.sqrt(gamma) * xi0.reshape(-1)])
    mu, _ = nnls(M, b, maxiter=50 * M.shape[1])
    y = y0 + A1.T @ mu
    xi = xi0 + (A2.T @ mu / gamma).reshape(p, n)
    mu_mat = np.zeros((p, p))
    for r, (i, j) in enumerate(pairs):
        mu_mat[i, j] = mu[r]
    return y, xi, mu_mat


def project(x: np.ndarray, y0: np.ndarray, xi0: np.ndarray, gamma: float, p: int
            ) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Step 1 for the whole partition: every block projected; returns (y, xi, mu) with mu the
    N x N array of the blocks' multipliers (zero outside the diagonal blocks)."""
    N = x.shape[0]
    y = np.empty(N)
    xi = np.empty_like(xi0)
    mu = np.zeros((N, N))
    for s in range(0, N, p):
        e = min(N, s + p)
        y[s:e], xi[s:e], mu[s:e, s:e] = project_block(x[s:e], y0[s:e], xi0[s:e], gamma)
    return y, xi, mu


def eta(x: np.ndarray, ybar: np.ndarray, gamma: float, theta: np.ndarray, p: int
        ) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """eta(theta): Step 1 of P-APG with the partition (the closed form over the whole space, then
    the blocks' projections).  Returns (y, xi, mu)."""
    y0, xi0 = primal_from_dual(x, ybar, gamma, theta * inter_mask(x.shape[0], p))
    return project(x, y0, xi0, gamma, p)


def partial_dual(x: np.ndarray, ybar: np.ndarray, gamma: float, theta: np.ndarray, p: int) -> float:
    """g_gamma(theta) of eq. ``subgradient``: the partial Lagrangian (eq. ``eq:lagrangian``) at its
    minimizer over Q."""
    mask = inter_mask(x.shape[0], p)
    y, xi, _ = eta(x, ybar, gamma, theta, p)
    s = pair_residual(x, y, xi)
    r = 0.5 * float(np.sum((y - ybar) ** 2)) + 0.5 * gamma * float(np.sum(xi ** 2))
    return r - float(np.sum((theta * mask) * s))


def lipschitz_inter(x: np.ndarray, gamma: float, p: int, rtol: float = 1e-8, max_iter: int = 300
                    ) -> tuple[float, float, int]:
    """sigma_max(C)^2 for C the dualized (inter-block) rows, by the power iteration of
    ``papg.lipschitz`` with the intra-block rows dropped; returns (L, sigma2, iterations)."""
    N, n = x.shape
    mask = inter_mask(N, p)
    vy = -1.0 + 2.0 * np.arange(N) / max(N - 1, 1)
    vxi = np.ones((N, n))
    nrm = math.sqrt(float(np.sum(vy ** 2) + np.sum(vxi ** 2)))
    vy /= nrm
    vxi /= nrm
    est = 0.0
    it = 0
    for it in range(1, max_iter + 1):
        z = pair_residual(x, vy, vxi) * mask
        new = float(np.sum(z ** 2))
        gy, gxi = pair_adjoint(x, z)
        nrm = math.sqrt(float(np.sum(gy ** 2) + np.sum(gxi ** 2)))
        if nrm == 0.0:
            est = new
            break
        vy, vxi = gy / nrm, gxi / nrm
        done = abs(new - est) <= rtol * new
        est = new
        if done:
            break
    return est / gamma, est, it


def papg_blocks(x: np.ndarray, ybar: np.ndarray, gamma: float, p: int, tol: float, L: float | None = None,
                max_iters: int = 100000, check_every: int = 50, iterates: list | None = None) -> dict:
    """P-APG (Fig. ``fig:papg``, constant step 1/L) on the partial dual of the partition with blocks
    of p points, from theta^0 = 0:
      1. eta^k = eta(theta~^k): closed form, then each block's QP (``project``)
      2. theta^k = (theta~^k - C eta^k / L)_+ on the dualized pairs
      3. t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
      4. theta~^{k+1} = theta^k + (t_k - 1)/t_{k+1} (theta^k - theta^{k-1})
    Every ``check_every`` iterations the whole problem's report (``papg.kkt_report``) is taken at
    the total multipliers theta^k + mu(theta^k); stop once its kkt <= tol.  ``iterates``, when
    given, receives (k, theta^k)."""
    N = x.shape[0]
    mask = inter_mask(N, p)
    if L is None:
        L = lipschitz_inter(x, gamma, p)[0]
    th_prev = np.zeros((N, N))
    th_tilde = th_prev.copy()
    t = 1.0
    rep = None
    status = "max_iters"
    k = 0
    for k in range(1, max_iters + 1):
        y, xi, _ = eta(x, ybar, gamma, th_tilde, p)                             # step 1
        s = pair_residual(x, y, xi)
        th = np.maximum(0.0, th_tilde - s / L) * mask                          # step 2
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0                    # step 3
        beta = (t - 1.0) / t_next
        th_tilde = th + beta * (th - th_prev)                                  # step 4
        th_prev = th
        t = t_next
        if iterates is not None:
            iterates.append((k, th.copy()))
        if k % check_every == 0 or k == max_iters:
            _, _, mu = eta(x, ybar, gamma, th, p)
            rep = kkt_report(x, ybar, gamma, th + mu)
            if rep["kkt"] <= tol:
                status = "converged"
                break
    y, xi, mu = eta(x, ybar, gamma, th_prev, p)
    if rep is None:
        rep = kkt_report(x, ybar, gamma, th_prev + mu)
    rep["k"] = k
    return {"y": y, "xi": xi, "theta": th_prev, "lam": th_prev + mu, "L": L, "iters": k, "status": status,
            "report": rep}

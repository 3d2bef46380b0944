"""Continuation to the unregularized least-squares estimator (Section 2.4.1), plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring): not part of the product path.

With beta > 1 and eps_t = eps0 / beta^t, outer iteration t >= 1 uses the Tikhonov weight
gamma_t = kappa_gamma eps_t and the dual tolerance delta_t = kappa_delta eps_t: theta^(t) is a
delta_t-optimal solution of the dual for gamma = gamma_t, computed by P-APG (Fig. ``fig:papg``)
started from theta^(t-1), theta^(0) = 0, and (y^(t), xi^(t)) is its Step-1 point.  The section's
bound then gives ||y^(t) - y*|| <= ||xi*|| sqrt(gamma_t) + sqrt(2 delta_t), y* the unregularized
LS estimator of eq. ``original`` and xi* its least-norm subgradients.

The inner stopping rule is the verifiable sufficient condition of Section 2.4.1 read as the
certified gap of the max-affine repair (``papg(..., stop="gap")``); L_gamma = sigma_max(C)^2 /
gamma_t reuses one power iteration for sigma_max(C)^2.
"""
from __future__ import annotations

import numpy as np

from .papg import lipschitz, papg


def continuation(x: np.ndarray, ybar: np.ndarray, eps0: float, beta: float, kappa_gamma: float,
                 kappa_delta: float, T: int, check_every: int = 10, max_inner: int = 200000,
                 adaptive: bool = True, restart: bool = True, sigma2: float | None = None) -> list[dict]:
    """Outer iterations t = 1..T; one record per t (gamma_t, delta_t, y, xi, lam, iters, gap)."""
    N = x.shape[0]
    if sigma2 is None:
        sigma2 = lipschitz(x, 1.0)[1]          # L_gamma = sigma2 / gamma (eq. eq:lischitz)
    lam = np.zeros((N, N))
    out = []
    for t in range(1, T + 1):
        eps_t = eps0 / beta ** t
        g_t = kappa_gamma * eps_t
        d_t = kappa_delta * eps_t
        r = papg(x, ybar, g_t, d_t, L=sigma2 / g_t, max_iters=max_inner, check_every=check_every,
                 lam0=lam, adaptive=adaptive, restart=restart, stop="gap")
        lam = r["lam"]
        out.append({"t": t, "gamma": g_t, "delta": d_t, "y": r["y"], "xi": r["xi"], "lam": lam,
                    "iters": r["iters"], "status": r["status"], "cert_gap": r["report"]["cert_gap"],
                    "kkt": r["report"]["kkt"]})
    return out

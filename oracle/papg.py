"""P-APG for the Tikhonov-regularized convex-regression QP, singleton partition, plain FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring): not part of the product path.

Problem (Section 2.1, eq. ``regularize``):
    minimize  r_g(y, xi) = 1/2 ||y - ybar||^2 + g/2 ||xi||^2
    over      y in R^N, xi = [xi_l] in R^{N n}
    s.t.      A1 y + A2 xi >= 0,
one row per ordered pair (i, j), i != j, in lexicographic order (Section 2, Definition
``def:A1A2``): the row of pair (i, j) reads  y_j - y_i + xi_i^T (x_i - x_j) >= 0  (eq. ``original``).
``g`` (gamma) is the Tikhonov weight.

Partition: every point is its own block (K = N), so every pair constraint is dualized and the
local set Q of Definition ``def:C`` is the whole space.  The dual multipliers theta are held as
an N x N array ``lam`` whose entry (i, j) belongs to the row of pair (i, j); the diagonal is
not a pair and is kept at zero.

Parity pins for every function here live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------------------------------------
# The constraint operator C = [A1 A2] and its adjoint (Definition def:A1A2; matrix-free products
# as described in Section 2.5).
# ---------------------------------------------------------------------------------------------

def pair_residual(x: np.ndarray, y: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Constraint values C eta for eta = (y, xi): s_ij = y_j - y_i + xi_i^T (x_i - x_j).

    Follows Definition ``def:A1A2``: row r of T_i picks y_j - y_i, and X_i = -T_i X picks
    (x_i - x_j)^T xi_i.  The product xi_i^T (x_i - x_j) is expanded as xi_i^T x_i - xi_i^T x_j
    so that the N^2 n work is one matrix product.  Returns an N x N array with a zero diagonal.
    """
    d = np.einsum("ik,ik->i", xi, x)            # xi_i^T x_i
    s = y[None, :] - y[:, None] + d[:, None] - xi @ x.T
    np.fill_diagonal(s, 0.0)
    return s


def pair_adjoint(x: np.ndarray, lam: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """C^T lam = (A1^T lam, A2^T lam) for multipliers lam (N x N, entry (i, j) = pair (i, j)).

    (A1^T lam)_m collects +lam_im from the rows where m is the second index and -lam_mj from the
    rows where m is the first index: column sum minus row sum.
    (A2^T lam)_m = sum_j lam_mj (x_m - x_j) = (row sum)_m x_m - (Lam X)_m, because only the rows
    (m, j) touch xi_m (A2 is block diagonal).
    """
    lam = np.array(lam, dtype=np.float64, copy=True)
    np.fill_diagonal(lam, 0.0)
    row = lam.sum(axis=1)
    col = lam.sum(axis=0)
    u = col - row
    w = row[:, None] * x - lam @ x
    return u, w


def primal_from_dual(x: np.ndarray, ybar: np.ndarray, gamma: float, lam: np.ndarray
                     ) -> tuple[np.ndarray, np.ndarray]:
    """Step 1 of P-APG (Fig. ``fig:papg``) with Q the whole space.

    The minimizer of 1/2||y - ybar||^2 + g/2||xi||^2 - <C^T lam, eta> is the stationary point
    y - ybar = A1^T lam, g xi = A2^T lam.  This is also eta(theta) of eq. ``dual gradient``.
    """
    u, w = pair_adjoint(x, lam)
    return ybar + u, w / gamma


def primal_objective(ybar: np.ndarray, gamma: float, y: np.ndarray, xi: np.ndarray) -> float:
    """r_gamma(y, xi) of eq. ``regularize``."""
    return 0.5 * float(np.sum((y - ybar) ** 2)) + 0.5 * gamma * float(np.sum(xi ** 2))


def dual_objective(x: np.ndarray, ybar: np.ndarray, gamma: float, lam: np.ndarray) -> float:
    """g_gamma(lam) of eq. ``eq:g_gamma``: the Lagrangian at its unique minimizer eta(lam)."""
    y, xi = primal_from_dual(x, ybar, gamma, lam)
    s = pair_residual(x, y, xi)
    lam0 = np.array(lam, dtype=np.float64, copy=True)
    np.fill_diagonal(lam0, 0.0)
    return primal_objective(ybar, gamma, y, xi) - float(np.sum(lam0 * s))


# ---------------------------------------------------------------------------------------------
# Lipschitz constant of the dual gradient (eq. eq:lischitz): L = sigma_max(C)^2 / gamma.
# ---------------------------------------------------------------------------------------------

def lipschitz(x: np.ndarray, gamma: float, rtol: float = 1e-8, max_iter: int = 300
              ) -> tuple[float, float, int]:
    """Estimate sigma_max(C)^2 by power iteration on C^T C and return (L, sigma2, iterations).

    The paper computes sigma_max in a "Preprocess" step (Section 4) without naming a routine.
    Reading used here: start from v_y,l = -1 + 2 l / (N - 1) (l = 0..N-1, a ramp: a constant
    v_y lies in the kernel of A1) and v_xi = 1, normalized over (y, xi); each iteration forms
    z = C v, takes the Rayleigh quotient ||C v||^2 as the estimate, then v <- C^T z / ||C^T z||;
    stop when two successive estimates agree to ``rtol`` (relative) or after ``max_iter``.
    """
    N, n = x.shape
    vy = -1.0 + 2.0 * np.arange(N) / max(N - 1, 1)
    vxi = np.ones((N, n))
    nrm = math.sqrt(float(np.sum(vy ** 2) + np.sum(vxi ** 2)))
    vy /= nrm
    vxi /= nrm
    est = 0.0
    it = 0
    for it in range(1, max_iter + 1):
        z = pair_residual(x, vy, vxi)
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


# ---------------------------------------------------------------------------------------------
# The P-APG loop (Fig. fig:papg; APG of Fig. fig:apg applied to the dual eq:dual-problem).
# ---------------------------------------------------------------------------------------------

def fista_schedule(iters: int) -> tuple[np.ndarray, np.ndarray]:
    """t_k for k = 1..iters+1 and beta_k = (t_k - 1) / t_{k+1} for k = 1..iters (Steps 3-4).

    ``t[k]`` and ``beta[k]`` are 1-based (index 0 unused)."""
    t = np.zeros(iters + 2)
    beta = np.zeros(iters + 1)
    t[1] = 1.0
    for k in range(1, iters + 1):
        t[k + 1] = (1.0 + math.sqrt(1.0 + 4.0 * t[k] * t[k])) / 2.0
        beta[k] = (t[k] - 1.0) / t[k + 1]
    return t, beta


def papg(x: np.ndarray, ybar: np.ndarray, gamma: float, tol: float, L: float | None = None,
         max_iters: int = 100000, check_every: int = 50, lam0: np.ndarray | None = None,
         momentum: bool = True, trace: list | None = None, iterates: list | None = None,
         adaptive: bool = False, upsilon: float = 2.0, steps: list | None = None,
         restart: bool = False, stop: str = "kkt") -> dict:
    """Run P-APG (Fig. ``fig:papg``) from theta^0 = lam0 (default 0, as in Theorem ``bound``).

    Iteration k >= 1, with lam_tilde^1 = lam^0 and t_1 = 1:
      1. eta^k = argmin_eta {1/2||y - ybar||^2 + g/2||xi||^2 - <C^T lam_tilde^k, eta>}
      2. lam^k = (lam_tilde^k - C eta^k / L)_+
      3. t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
      4. lam_tilde^{k+1} = lam^k + (t_k - 1)/t_{k+1} (lam^k - lam^{k-1})
    ``momentum=False`` sets the extrapolation weight to zero, which is plain projected dual
    gradient ascent (eq. ``eq:gd-rate``).

    ``adaptive=True`` replaces the constant step 1/L of Step 2 by the adaptive rule of Section 2.4
    (the "PAPG_A" variant of Section 4): with s_0 = L and a factor upsilon > 1, iteration k uses
    s_k = s_{k-1} * upsilon^(l_k - 1) for the smallest integer l_k >= 0 such that
        g(lam^k) >= g(lam~^k) + <grad g(lam~^k), lam^k - lam~^k> - s_k/2 ||lam^k - lam~^k||^2
    (eq. ``eq:adaptive-check``), lam^k being the Step-2 point computed with 1/s_k.  The paper does
    not give upsilon; 2 is the default here.  ``steps``, when given, receives s_k for every k.
    With every pair dualized g is exactly quadratic, g(lam) = -u^T ybar - ||u||^2/2 - ||w||^2/(2g)
    for (u, w) = C^T lam, so for D = lam^k - lam~^k the check is the same statement as
        ||A1^T D||^2 + ||A2^T D||^2 / g <= s_k ||D||^2,
    which is how it is evaluated: the literal form subtracts dual values of size O(1) whose
    difference near convergence is far below FP64 resolution.

    ``restart=True`` (adaptive step only; not part of the paper) resets the momentum, t := 1, after
    an iteration whose accepted step opposes the iterate's movement,
    <lam^k - lam~^k, lam^k - lam^{k-1}> < 0 (the gradient restart of O'Donoghue and Candes,
    "Adaptive restart for accelerated gradient schemes", 2015), so that lam~^{k+1} = lam^k.

    Every ``check_every`` iterations the stopping report
    of ``kkt_report`` is evaluated at (lam^k, eta(lam^k)); the loop stops once its ``kkt`` is at
    most ``tol`` (``stop="kkt"``), or, with ``stop="gap"``, once the certified gap of
    ``repair_certificate`` is at most ``tol``: G >= g* - g(lam^k), so lam^k is then tol-optimal in
    the sense of Section 2.4.1 (a verifiable sufficient condition for the inner iterations of the
    continuation).  ``iterates``, when given, receives (k, lam^k) for every k.
    """
    N = x.shape[0]
    if L is None:
        L = lipschitz(x, gamma)[0]
    lam_prev = np.zeros((N, N)) if lam0 is None else np.array(lam0, dtype=np.float64, copy=True)
    np.fill_diagonal(lam_prev, 0.0)
    lam_tilde = lam_prev.copy()
    t = 1.0
    rep = None
    k = 0
    status = "max_iters"
    s_k = L
    for k in range(1, max_iters + 1):
        y, xi = primal_from_dual(x, ybar, gamma, lam_tilde)                    # step 1
        s = pair_residual(x, y, xi)
        if not adaptive:
            lam = np.maximum(0.0, lam_tilde - s / L)                           # step 2
            np.fill_diagonal(lam, 0.0)
        else:
            ell = 0
            while True:
                s_try = s_k * upsilon ** (ell - 1)
                lam = np.maximum(0.0, lam_tilde - s / s_try)                   # step 2, step 1/s_try
                np.fill_diagonal(lam, 0.0)
                dlt = lam - lam_tilde
                du, dw = pair_adjoint(x, dlt)
                curv = float(du @ du) + float(np.sum(dw * dw)) / gamma
                if curv <= s_try * float(np.sum(dlt * dlt)) * (1.0 + 1e-12):
                    break
                ell += 1
            s_k = s_try
            if steps is not None:
                steps.append(s_k)
            if restart and float(np.sum(dlt * (lam - lam_prev))) < 0.0:
                t = 1.0
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0                    # step 3
        beta = (t - 1.0) / t_next if momentum else 0.0
        lam_tilde = lam + beta * (lam - lam_prev)                              # step 4
        lam_prev = lam
        t = t_next
        if iterates is not None:
            iterates.append((k, lam.copy()))
        if k % check_every == 0 or k == max_iters:
            rep = kkt_report(x, ybar, gamma, lam)
            if stop == "gap":
                rep["cert_gap"] = repair_certificate(x, ybar, gamma, lam)["cert_gap"]
            if trace is not None:
                trace.append((k, rep))
            if (rep["cert_gap"] if stop == "gap" else rep["kkt"]) <= tol:
                status = "converged"
                break
    y, xi = primal_from_dual(x, ybar, gamma, lam_prev)
    if rep is None or (k % check_every != 0 and k != max_iters):
        rep = kkt_report(x, ybar, gamma, lam_prev)
    if stop == "gap" and "cert_gap" not in rep:
        rep["cert_gap"] = repair_certificate(x, ybar, gamma, lam_prev)["cert_gap"]
    rep["k"] = k
    return {"y": y, "xi": xi, "lam": lam_prev, "L": L, "iters": k, "status": status,
            "report": rep, "step": s_k}


# ---------------------------------------------------------------------------------------------
# Stopping test and reported metrics.
# ---------------------------------------------------------------------------------------------

def kkt_report(x: np.ndarray, ybar: np.ndarray, gamma: float, lam: np.ndarray,
               y: np.ndarray | None = None, xi: np.ndarray | None = None) -> dict:
    """Optimality measures of a dual point lam >= 0 and its primal eta(lam).

    The paper does not define a KKT residual.  Reading used here: the KKT conditions of the
    regularized QP are stationarity (y - ybar = A1^T lam, g xi = A2^T lam: Step 1), dual
    feasibility (lam >= 0: the projection of Step 2), primal feasibility s = C eta >= 0 and
    complementarity lam_ij s_ij = 0.  The last two are measured by the natural residual of the
    bound-constrained dual, |min(lam_ij, s_ij)| over all pairs, and the stationarity of a given
    (y, xi) by its max-norm distance from the closed form.  All are divided by
    S_y = max(1, max ybar - min ybar):

        kkt = max(max_ij |min(lam_ij, s_ij)|, ||y - ybar - A1^T lam||_inf,
                  ||g xi - A2^T lam||_inf / g) / S_y

    Also returned: the paper's normalized infeasibility ||(C eta)_-||_2 / sqrt(N^2 - N) and
    normalized duality gap |lam^T C eta| / (N^2 - N) (both defined in Section 4.1), the largest
    violation, g(lam), r_g(eta) and sum lam_ij s_ij.
    """
    N = x.shape[0]
    lam = np.array(lam, dtype=np.float64, copy=True)
    np.fill_diagonal(lam, 0.0)
    u, w = pair_adjoint(x, lam)
    y_cf, xi_cf = ybar + u, w / gamma
    if y is None:
        y = y_cf
    if xi is None:
        xi = xi_cf
    s = pair_residual(x, y, xi)
    off = ~np.eye(N, dtype=bool)
    sy = max(1.0, float(ybar.max() - ybar.min()))
    nat = float(np.max(np.abs(np.minimum(lam, s)[off]))) if N > 1 else 0.0
    stat_y = float(np.max(np.abs(y - y_cf)))
    stat_xi = float(np.max(np.abs(gamma * xi - w))) / gamma
    neg = np.minimum(s[off], 0.0)
    pairs = N * N - N
    comp = float(np.sum(lam * s))
    r = primal_objective(ybar, gamma, y, xi)
    return {
        "kkt": max(nat, stat_y, stat_xi) / sy,
        "nat_res_max": nat / sy,
        "stat_y": stat_y / sy,
        "stat_xi": stat_xi / sy,
        "max_viol": float(max(0.0, -s[off].min())) / sy if N > 1 else 0.0,
        "infeas_rms": float(math.sqrt(np.sum(neg ** 2) / pairs)) if N > 1 else 0.0,
        "dual_gap_paper": abs(comp) / pairs if N > 1 else 0.0,
        "comp_sum": comp,
        "primal_obj": r,
        "dual_obj": r - comp,
        "scale": sy,
    }


def repair_certificate(x: np.ndarray, ybar: np.ndarray, gamma: float, lam: np.ndarray,
                       rounds: int = 16) -> dict:
    """A feasible primal point built from eta(lam) and the certified gap it gives.

    Any feasible (y', xi') gives p*_g <= r_g(y', xi') and, by weak duality,
    G = r_g(y', xi') - g(lam) >= p*_g - g(lam) >= 0; Theorem ``thm:rate`` then bounds
    ||y(lam) - y*_g||^2 + g ||xi(lam) - xi*_g||^2 <= 2 G.  Two feasible points are built and the
    smaller G is reported.

    Max-affine repair: f(z) = max_i (y_i + xi_i^T (z - x_i)) is convex; y'_j = f(x_j) and xi'_j the
    slope of a maximizing piece are feasible.  Near the optimum many pieces tie at x_j and rounding
    decides which computes as the largest; switching to another piece's slope changes g||xi'||^2
    by O(g ||xi||^2) for a rounding-level violation, so j keeps its own slope (y'_j still raised to
    f(x_j)) unless some piece exceeds it by more than tau_j = 1e-10 (1 + |y_j| + ||xi_j||_1 X),
    X = max_{l,m} |x_lm - mean_l x_lm|.

    Own-slope (potential) repair: keep every xi_j and raise the heights, y' = y + c with the least
    c >= 0 such that c_j >= c_i - s_ij for every pair (then s'_ij = s_ij + c_j - c_i >= 0).  The
    least such c is a longest-path potential, reached by the relaxation
    c_j <- max(c_j, max_{i != j} (c_i - s_ij)) from c = 0 (the first round gives the max-affine
    heights); it exists when s has no negative cycle and is used when a round changes no c_j by
    more than tau_j within ``rounds`` rounds.  Near the optimum c is of the order of the
    violations, so G tracks the complementarity and the KKT residual.

    Both points are feasible up to tau; G then bounds the suboptimality up to tau times the
    multipliers' sum.
    """
    N = x.shape[0]
    y, xi = primal_from_dual(x, ybar, gamma, lam)
    s = pair_residual(x, y, xi)                  # s_jj = 0 stands for piece j itself
    g = dual_objective(x, ybar, gamma, lam)
    xspan = float(np.abs(x - x.mean(axis=0)).max())
    tau = 1e-10 * (1.0 + np.abs(y) + np.abs(xi).sum(axis=1) * xspan)
    # max-affine repair: f(x_j) = max_i (y_i + xi_i^T (x_j - x_i)) = y_j - min_i s_ij
    colmin = s.min(axis=0)
    y_rep = y - colmin
    istar = np.arange(N)
    viol = colmin < -tau
    istar[viol] = np.argmin(s[:, viol], axis=0)
    xi_rep = xi[istar]
    r_rep = primal_objective(ybar, gamma, y_rep, xi_rep)
    G_affine = r_rep - g
    # own-slope repair
    off = s.copy()
    np.fill_diagonal(off, np.inf)
    c = np.zeros(N)
    converged = False
    used = 0
    for used in range(1, rounds + 1):
        cand = np.maximum(c, (c[:, None] - off).max(axis=0))
        changed = bool((cand > c + tau).any())
        c = cand
        if not changed:
            converged = True
            break
    G_own = primal_objective(ybar, gamma, y + c, xi) - g if converged else math.inf
    if G_own < G_affine:
        y_best, xi_best, r_best, G, method = y + c, xi, G_own + g, G_own, "own-slope"
    else:
        y_best, xi_best, r_best, G, method = y_rep, xi_rep, r_rep, G_affine, "max-affine"
    return {
        "y_rep": y_best,
        "xi_rep": xi_best,
        "piece": istar,
        "primal_rep": r_best,
        "dual_obj": g,
        "cert_gap": G,
        "cert_gap_affine": G_affine,
        "cert_gap_own": G_own,
        "own_rounds": used,
        "own_converged": converged,
        "method": method,
        "y_err_bound": math.sqrt(max(0.0, 2.0 * G)),
        "max_fit_change": float(np.max(np.abs(y_best - y))),
    }

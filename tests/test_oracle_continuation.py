"""Pins of the continuation oracle (Section 2.4.1) and of the unregularized estimator.

The unregularized least-squares estimator y* of eq. ``original`` comes from two independent
exact solvers: the primal QP by SLSQP, and the regularized dual by NNLS at a tiny Tikhonov weight
(whose solution is within ||xi*|| sqrt(gamma) of y* by the section's bound with delta = 0).  The
continuation is pinned to the section's bound ||y^(t) - y*|| <= ||xi*|| sqrt(gamma_t) +
sqrt(2 delta_t), and every inner solve to true delta_t-optimality against the exact regularized
dual optimum.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1608_02227_amd import workloads as W


def _problem(seed, N=12, n=2, kind="sq"):
    if kind == "sq":
        return W.sq_norm(N, n, 0.1, seed)
    return W.log_sum_exp_affine(N, n, 4, 0.2, seed)


@pytest.mark.parametrize("seed,kind,n", [(5, "sq", 2), (6, "sq", 2), (7, "lse", 3)])
def test_exact_ls_two_solvers_agree(seed, kind, n):
    x, ybar = _problem(seed, n=n, kind=kind)
    ex = oracle.exact_ls(x, ybar)
    assert ex["min_constraint"] >= -1e-9
    nn = oracle.exact_solve(x, ybar, 1e-10)
    bound = np.linalg.norm(ex["xi"]) * math.sqrt(1e-10)
    assert np.linalg.norm(nn["y"] - ex["y"]) <= bound + 1e-7
    # the least-norm subgradients are the limit of the regularized ones
    assert np.max(np.abs(nn["xi"] - ex["xi"])) <= 1e-5 * max(1.0, np.abs(ex["xi"]).max())


def test_exact_ls_is_the_projection():
    # y* minimizes ||y - ybar|| over the fitted values of convex functions: any convex data is
    # its own projection, and the optimum cannot be improved along feasible directions
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (10, 2))
    yc = (x ** 2).sum(axis=1)
    assert np.max(np.abs(oracle.exact_ls(x, yc)["y"] - yc)) <= 1e-7
    x, ybar = _problem(11)
    ex = oracle.exact_ls(x, ybar)
    # convex combinations with another feasible point (a convex function's values) do not help
    f = 0.3 * (x ** 2).sum(axis=1)
    for a in (1e-3, 1e-2, 1e-1):
        z = (1 - a) * ex["y"] + a * f
        assert 0.5 * np.sum((z - ybar) ** 2) >= ex["p_star"] - 1e-12


@pytest.mark.parametrize("seed,kind,n", [(5, "sq", 2), (6, "sq", 2), (7, "lse", 3)])
def test_continuation_obeys_the_bound_and_is_certified(seed, kind, n):
    x, ybar = _problem(seed, n=n, kind=kind)
    ex = oracle.exact_ls(x, ybar)
    xs = np.linalg.norm(ex["xi"])
    out = oracle.continuation(x, ybar, eps0=1.0, beta=2.0, kappa_gamma=0.5, kappa_delta=1.0, T=10)
    for o in out:
        # Section 2.4.1's schedule, from the parameters: eps_t = eps0 / beta^t, gamma_t = kappa_gamma
        # eps_t, delta_t = kappa_delta eps_t (distinct kappas, so a swapped weight shows)
        eps_t = 1.0 / 2.0 ** o["t"]
        gamma_t, delta_t = 0.5 * eps_t, eps_t
        assert o["gamma"] == pytest.approx(gamma_t, rel=1e-15)
        assert o["delta"] == pytest.approx(delta_t, rel=1e-15)
        assert o["status"] == "converged" and o["cert_gap"] <= delta_t
        # Section 2.4.1: ||y^(t) - y*|| <= ||xi*|| sqrt(gamma_t) + sqrt(2 delta_t)
        assert np.linalg.norm(o["y"] - ex["y"]) <= xs * math.sqrt(gamma_t) + math.sqrt(2 * delta_t)
        # the certificate is honest: the true dual suboptimality at gamma_t is at most delta_t
        exg = oracle.exact_solve(x, ybar, gamma_t)
        g = oracle.dual_objective(x, ybar, gamma_t, o["lam"])
        assert exg["p_star"] - g <= delta_t + 1e-12
        assert exg["p_star"] - g <= o["cert_gap"] + 1e-12
    # the iterates approach y*
    d = [np.linalg.norm(o["y"] - ex["y"]) for o in out]
    assert d[-1] < 0.2 * d[0]


def test_certificate_is_tight_at_the_optimum():
    # at the exact regularized optimum many pieces tie; the certified gap must still vanish
    x, ybar = _problem(5)
    for g in (1e-1, 1e-3):
        ex = oracle.exact_solve(x, ybar, g)
        c = oracle.repair_certificate(x, ybar, g, ex["lam"])
        assert 0.0 <= c["cert_gap"] + 1e-14 and c["cert_gap"] <= 1e-12


@pytest.mark.parametrize("seed", [11, 12])
def test_one_dimensional_estimator_matches_the_hinge_basis(seed):
    """In one dimension a convex function sampled at sorted points is a + b x + sum_k c_k (x - x_k)_+
    with c_k >= 0 (a textbook characterization: its slopes are non-decreasing), so the LS convex
    regression is a bound-constrained least-squares problem in (a, b, c) — a formulation that
    shares nothing with the pair constraints of eq. ``original``.  Both exact solvers and the
    regularized P-APG fit must agree with it, and the fitted values must be convex."""
    from scipy.optimize import lsq_linear
    rng = np.random.default_rng(seed)
    N = 14
    x = np.sort(rng.uniform(-1.0, 1.0, N))
    ybar = x ** 2 + 0.3 * np.sin(5.0 * x) + 0.05 * rng.standard_normal(N)
    knots = x[1:-1]
    B = np.column_stack([np.ones(N), x] + [np.maximum(0.0, x - t) for t in knots])
    lo = np.concatenate([[-np.inf, -np.inf], np.zeros(N - 2)])
    fit = lsq_linear(B, ybar, bounds=(lo, np.full(N, np.inf)), tol=1e-14, lsmr_tol="auto", max_iter=10000)
    y_hinge = B @ fit.x
    # convexity of the reference: non-negative second divided differences
    slopes = np.diff(y_hinge) / np.diff(x)
    assert np.all(np.diff(slopes) >= -1e-9)
    assert np.max(np.abs(y_hinge - ybar)) > 1e-3          # the data are not convex: a real projection
    ex = oracle.exact_ls(x[:, None], ybar)
    # the y solve must converge; the least-norm subgradient solve may stop at a flat line search,
    # and any feasible subgradients are at least as long as the least-norm ones (a looser bound)
    assert ex["message"][0] == "Optimization terminated successfully"
    assert ex["min_constraint"] >= -1e-10
    assert np.max(np.abs(ex["y"] - y_hinge)) <= 1e-6
    # the regularized estimator is within ||xi*|| sqrt(gamma) of y* (Section 2.4.1 with delta = 0)
    gamma = 1e-6
    r = oracle.papg(x[:, None], ybar, gamma, 1e-10, adaptive=True, restart=True, max_iters=200000)
    gap = oracle.repair_certificate(x[:, None], ybar, gamma, r["lam"])["cert_gap"]
    bound = np.linalg.norm(ex["xi"]) * math.sqrt(gamma) + math.sqrt(2.0 * gap)
    assert np.linalg.norm(r["y"] - y_hinge) <= bound + 1e-9
    s_fit = np.diff(r["y"]) / np.diff(x)
    assert np.all(np.diff(s_fit) >= -1e-4)

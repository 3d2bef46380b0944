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
    out = oracle.continuation(x, ybar, eps0=1.0, beta=2.0, kappa_gamma=1.0, kappa_delta=1.0, T=10)
    for o in out:
        assert o["gamma"] == pytest.approx(1.0 / 2.0 ** o["t"], rel=1e-15)
        assert o["delta"] == o["gamma"]
        assert o["status"] == "converged" and o["cert_gap"] <= o["delta"]
        # Section 2.4.1: ||y^(t) - y*|| <= ||xi*|| sqrt(gamma_t) + sqrt(2 delta_t)
        assert np.linalg.norm(o["y"] - ex["y"]) <= xs * math.sqrt(o["gamma"]) + math.sqrt(2 * o["delta"])
        # the certificate is honest: the true dual suboptimality at gamma_t is at most delta_t
        exg = oracle.exact_solve(x, ybar, o["gamma"])
        g = oracle.dual_objective(x, ybar, o["gamma"], o["lam"])
        assert exg["p_star"] - g <= o["delta"] + 1e-12
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

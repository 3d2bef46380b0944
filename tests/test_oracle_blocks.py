"""CPU pins of the K-block partial-dualization oracle (``oracle/blocks.py``, Section 2.1).

Each pin ties the oracle to something other than itself: the singleton-partition oracle (pinned in
``test_oracle_pins.py``) as the p = 1 special case, the exact solver of the whole QP (one block, and
the unique minimizer every converged run must reach), an SLSQP solve of a block's QP (a different
library algorithm), a dense SVD of the explicitly assembled dualized rows, and weak duality."""
import importlib

import numpy as np
import pytest
from scipy.optimize import minimize

B = importlib.import_module("oracle.blocks")
exact = importlib.import_module("oracle.exact")
P = importlib.import_module("oracle.papg")    # the module (the package exports a function of this name)


def _data(N, n, seed, noise=0.1):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(N, n))
    y = (x ** 2).sum(axis=1) + noise * rng.standard_normal(N)
    return x, y


def test_singleton_blocks_are_the_fully_dualized_method():
    """p = 1: no pair lies inside a block, Step 1 is the closed form, so the iterates are those of
    the singleton-partition P-APG with the same constant step."""
    x, y = _data(14, 2, 1)
    g = 1e-2
    L, s2, _ = P.lipschitz(x, g)
    Lb, s2b, _ = B.lipschitz_inter(x, g, 1)
    assert s2b == pytest.approx(s2, rel=1e-12)
    a, b = [], []
    P.papg(x, y, g, 0.0, L=L, max_iters=30, check_every=1000, iterates=a)
    B.papg_blocks(x, y, g, 1, 0.0, L=L, max_iters=30, check_every=1000, iterates=b)
    for (ka, la), (kb, lb) in zip(a, b):
        assert ka == kb
        np.testing.assert_allclose(lb, la, rtol=0, atol=1e-14 * max(1.0, np.abs(la).max()))


def test_one_block_projection_is_the_exact_solution():
    """p = N: Step 1 at theta = 0 projects (ybar, 0) onto the whole feasible set, i.e. solves the
    regularized QP itself."""
    x, y = _data(9, 2, 2)
    g = 1e-2
    ref = exact.exact_solve(x, y, g)
    yy, xx, mu = B.project(x, y, np.zeros_like(x), g, 9)
    np.testing.assert_allclose(yy, ref["y"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(xx, ref["xi"], rtol=0, atol=1e-7)
    assert np.all(mu >= 0.0)


def test_block_projection_matches_slsqp_and_its_kkt_conditions():
    rng = np.random.default_rng(3)
    p, n, g = 5, 2, 0.05
    xb = rng.uniform(-1, 1, size=(p, n))
    y0 = rng.standard_normal(p)
    xi0 = rng.standard_normal((p, n))
    y, xi, mu = B.project_block(xb, y0, xi0, g)
    # KKT of the block QP: feasibility, dual feasibility, complementarity, stationarity
    s = P.pair_residual(xb, y, xi)
    off = ~np.eye(p, dtype=bool)
    assert s[off].min() >= -1e-10
    assert mu.min() >= 0.0 and np.all(np.diag(mu) == 0.0)
    assert np.max(np.abs(mu * s)) <= 1e-9
    u, w = P.pair_adjoint(xb, mu)
    np.testing.assert_allclose(y - y0, u, atol=1e-10)
    np.testing.assert_allclose(g * (xi - xi0), w, atol=1e-10)
    # an independent solver of the same QP

    def f(v):
        return 0.5 * np.sum((v[:p] - y0) ** 2) + 0.5 * g * np.sum((v[p:] - xi0.ravel()) ** 2)

    cons = {"type": "ineq", "fun": lambda v: P.pair_residual(xb, v[:p], v[p:].reshape(p, n))[off]}
    r = minimize(f, np.concatenate([y0, xi0.ravel()]), constraints=[cons], method="SLSQP",
                 options={"ftol": 1e-14, "maxiter": 500})
    assert r.success
    np.testing.assert_allclose(y, r.x[:p], atol=1e-6)
    np.testing.assert_allclose(xi.ravel(), r.x[p:], atol=1e-5)


@pytest.mark.parametrize("N,p", [(12, 4), (13, 5)])
def test_inter_block_sigma_matches_dense_svd(N, p):
    x, _ = _data(N, 3, 4)
    A1, A2, pairs = exact.explicit_constraints(x)
    ids = B.block_ids(N, p)
    rows = [r for r, (i, j) in enumerate(pairs) if ids[i] != ids[j]]
    C = np.hstack([A1, A2])[rows]
    s2 = np.linalg.svd(C, compute_uv=False)[0] ** 2
    _, est, _ = B.lipschitz_inter(x, 1.0, p, rtol=1e-13, max_iter=5000)
    assert est == pytest.approx(s2, rel=1e-8)
    # dropping rows cannot raise sigma_max
    assert est <= P.lipschitz(x, 1.0, rtol=1e-13, max_iter=5000)[1] * (1 + 1e-9)


@pytest.mark.parametrize("N,n,p", [(16, 2, 4), (18, 3, 6), (15, 2, 4)])
def test_converged_block_fit_reaches_the_unique_minimizer(N, n, p):
    x, y = _data(N, n, 5 + N)
    g = 0.1
    ref = exact.exact_solve(x, y, g)
    r = B.papg_blocks(x, y, g, p, 1e-8, max_iters=200000, check_every=20)
    assert r["status"] == "converged"
    # only the dualized (inter-block) pairs carry multipliers theta (eq. eq:lagrangian)
    assert np.all(r["theta"][~B.inter_mask(N, p)] == 0.0)
    scale = np.abs(ref["y"]).max()
    assert np.max(np.abs(r["y"] - ref["y"])) <= 1e-6 * scale
    # weak duality and the gap at the end: g_K(theta) <= p* and close to it
    gk = B.partial_dual(x, y, g, r["theta"], p)
    assert gk <= ref["p_star"] + 1e-10 * max(1.0, ref["p_star"])
    assert ref["p_star"] - gk <= 1e-6 * max(1.0, ref["p_star"])


def test_partial_dual_dominates_the_full_dual_and_is_below_the_optimum():
    """g_K(theta) = max_mu g(theta + mu) over the intra-block multipliers >= g(theta), and every
    dual value is a lower bound on p* (weak duality)."""
    x, y = _data(12, 2, 7)
    g = 5e-2
    p = 4
    ref = exact.exact_solve(x, y, g)
    rng = np.random.default_rng(8)
    mask = B.inter_mask(12, p)
    for _ in range(3):
        th = rng.exponential(0.05, size=(12, 12)) * mask
        gk = B.partial_dual(x, y, g, th, p)
        assert gk >= P.dual_objective(x, y, g, th) - 1e-12
        assert gk <= ref["p_star"] + 1e-12
        # and the maximizing mu is the blocks' own multipliers: g(theta + mu) = g_K(theta)
        _, _, mu = B.eta(x, y, g, th, p)
        assert P.dual_objective(x, y, g, th + mu) == pytest.approx(gk, rel=1e-9, abs=1e-12)


def test_block_arrowhead_elimination_needs_the_schur_complement():
    """Reading of Theorem `lem:cholesky-block-arrowhead`: with M = G + A^T diag(d) A for one block
    (G = diag(I, g I), A the block's pair rows), eliminating the xi blocks (z_a = M_aa^-1 b_a) leaves
    the y system with S = M00 - sum_a M0a M_aa^-1 M0a^T; that elimination reproduces a dense solve,
    while the same formula with M00 in place of S does not."""
    rng = np.random.default_rng(12)
    q, n, g = 6, 3, 0.05
    xb = rng.uniform(-1, 1, size=(q, n))
    A1, A2, _ = exact.explicit_constraints(xb)
    A = np.hstack([A1, A2])
    d = rng.exponential(1.0, size=A.shape[0]) * 10.0 ** rng.uniform(-3, 3, size=A.shape[0])
    G = np.diag(np.concatenate([np.ones(q), g * np.ones(q * n)]))
    M = G + A.T @ (d[:, None] * A)
    b = rng.standard_normal(q + q * n)
    ref = np.linalg.solve(M, b)
    M00 = M[:q, :q]
    blocks = [(M[:q, q + a * n:q + (a + 1) * n], M[q + a * n:q + (a + 1) * n, q + a * n:q + (a + 1) * n])
              for a in range(q)]
    # the xi blocks are block-diagonal: only point a's own n x n block couples xi_a
    for a in range(q):
        for c in range(q):
            if c != a:
                assert np.all(M[q + a * n:q + (a + 1) * n, q + c * n:q + (c + 1) * n] == 0.0)

    def eliminate(Y):
        r0 = b[:q] - sum(M0a @ np.linalg.solve(Maa, b[q + a * n:q + (a + 1) * n])
                         for a, (M0a, Maa) in enumerate(blocks))
        dy = np.linalg.solve(Y, r0)
        dxi = [np.linalg.solve(Maa, b[q + a * n:q + (a + 1) * n] - M0a.T @ dy) for a, (M0a, Maa) in enumerate(blocks)]
        return np.concatenate([dy, *dxi])

    S = M00 - sum(M0a @ np.linalg.solve(Maa, M0a.T) for M0a, Maa in blocks)
    np.testing.assert_allclose(eliminate(S), ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    assert np.abs(eliminate(M00) - ref).max() > 1e-3 * np.abs(ref).max()

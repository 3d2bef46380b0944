"""Pins of the FP64 oracle against facts fixed by the paper and by the mathematics.

None of these re-type the oracle's own formulas: they compare it with the explicit constraint
matrices of Definition def:A1A2, closed-form solutions, exact NNLS solves, spectral facts of
Lemma lem:O1-constant, the identities and bounds of Theorem thm:rate and eq. eq:apg-rate, and
invariances of the problem.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.exact import explicit_constraints, exact_solve, t_block
from paper_1608_02227_amd import workloads as W


def _rand_problem(N, n, seed, kind="sq"):
    if kind == "sq":
        return W.sq_norm(N, n, 0.1, seed)
    return W.log_sum_exp_affine(N, n, 4, 0.2, seed)


# --- operators vs the explicit matrices of Definition def:A1A2 ------------------------------

def test_t_block_structure():
    # T_l has -1 in column l and the identity elsewhere; T_l^T T_l is the Laplacian of a star
    # with centre l, whose largest eigenvalue is N (proof of Lemma lem:O1-constant).
    N = 6
    for l in range(N):
        T = t_block(N, l)
        assert np.all(T[:, l] == -1.0)
        ev = np.linalg.eigvalsh(T.T @ T)
        assert ev.max() == pytest.approx(N, rel=1e-12)
        assert ev.min() == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("N,n,seed", [(5, 1, 0), (7, 3, 1), (9, 2, 2)])
def test_residual_matches_explicit_rows(N, n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((N, n))
    y = rng.standard_normal(N)
    xi = rng.standard_normal((N, n))
    A1, A2, pairs = explicit_constraints(x)
    rows = A1 @ y + A2 @ xi.reshape(-1)
    s = oracle.pair_residual(x, y, xi)
    for r, (i, j) in enumerate(pairs):
        assert s[i, j] == pytest.approx(rows[r], rel=1e-12, abs=1e-12)
    assert np.all(np.diag(s) == 0.0)


@pytest.mark.parametrize("N,n,seed", [(5, 1, 0), (8, 3, 4)])
def test_adjoint_matches_explicit_transpose(N, n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((N, n))
    lam = rng.uniform(0, 1, (N, N))
    np.fill_diagonal(lam, 0.0)
    A1, A2, pairs = explicit_constraints(x)
    theta = np.array([lam[i, j] for (i, j) in pairs])
    u, w = oracle.pair_adjoint(x, lam)
    np.testing.assert_allclose(u, A1.T @ theta, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(w.reshape(-1), A2.T @ theta, rtol=1e-12, atol=1e-12)


def test_adjoint_ignores_diagonal():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((6, 2))
    lam = rng.uniform(0, 1, (6, 6))
    lam0 = lam.copy()
    np.fill_diagonal(lam0, 0.0)
    for a, b in zip(oracle.pair_adjoint(x, lam), oracle.pair_adjoint(x, lam0)):
        np.testing.assert_array_equal(a, b)


def test_dot_identity():
    # <C eta, lam> = <eta, C^T lam> (PIN-2)
    rng = np.random.default_rng(11)
    N, n = 40, 5
    x = rng.standard_normal((N, n))
    y = rng.standard_normal(N)
    xi = rng.standard_normal((N, n))
    lam = rng.standard_normal((N, N))
    np.fill_diagonal(lam, 0.0)
    lhs = np.sum(oracle.pair_residual(x, y, xi) * lam)
    u, w = oracle.pair_adjoint(x, lam)
    rhs = np.dot(u, y) + np.sum(w * xi)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_laplacian_identity():
    # A1^T A1 = 2 Omega with Omega the complete-graph Laplacian (Lemma lem:O1-constant).
    rng = np.random.default_rng(5)
    N = 30
    x = np.zeros((N, 2))
    v = rng.standard_normal(N)
    s = oracle.pair_residual(x, v, np.zeros((N, 2)))
    u, _ = oracle.pair_adjoint(x, s)
    np.testing.assert_allclose(u, 2.0 * (N * v - v.sum()), rtol=1e-12, atol=1e-10)


# --- closed forms ---------------------------------------------------------------------------

def test_slater_point_residual():
    # eq:slater-point: for y~_l = y^ + a/2 ||x_l - x^||^2 and xi~_l = a (x_l - x^) the residual of
    # pair (i, j) is exactly a/2 ||x_i - x_j||^2 (the quadratic is its own first-order model
    # plus the curvature term).
    rng = np.random.default_rng(7)
    N, n, a = 50, 4, 0.7
    x = rng.uniform(-1, 1, (N, n))
    xh = x.mean(axis=0)
    yt = 1.3 + 0.5 * a * np.sum((x - xh) ** 2, axis=1)
    xit = a * (x - xh)
    s = oracle.pair_residual(x, yt, xit)
    d2 = np.sum((x[:, None, :] - x[None, :, :]) ** 2, axis=2)
    np.testing.assert_allclose(s, 0.5 * a * d2, rtol=1e-12, atol=1e-12)


def _two_point_solution(x, ybar, gamma):
    """Hand solution of the regularized QP for N = 2.

    If ybar_2 >= ybar_1 the pair (2,1) constraint y_1 - y_2 + xi_2^T (x_2 - x_1) >= 0 binds with
    multiplier mu = (ybar_2 - ybar_1) / (2 + ||x_2 - x_1||^2 / gamma), giving y_1 = ybar_1 + mu,
    y_2 = ybar_2 - mu, xi_1 = 0, xi_2 = mu (x_2 - x_1) / gamma (and symmetrically)."""
    d = x[1] - x[0]
    if ybar[1] >= ybar[0]:
        mu = (ybar[1] - ybar[0]) / (2.0 + d @ d / gamma)
        y = np.array([ybar[0] + mu, ybar[1] - mu])
        xi = np.vstack([np.zeros_like(d), mu * d / gamma])
        lam = np.array([[0.0, 0.0], [mu, 0.0]])
    else:
        mu = (ybar[0] - ybar[1]) / (2.0 + d @ d / gamma)
        y = np.array([ybar[0] - mu, ybar[1] + mu])
        xi = np.vstack([-mu * d / gamma, np.zeros_like(d)])
        lam = np.array([[0.0, mu], [0.0, 0.0]])
    return y, xi, lam


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_two_point_closed_form(seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((2, 3))
    ybar = rng.standard_normal(2)
    gamma = 0.5
    y, xi, lam = _two_point_solution(x, ybar, gamma)
    # sigma_max(C)^2 for N = 2 is 4 + ||x_2 - x_1||^2 (eigenvalues of C C^T).
    d = x[1] - x[0]
    L, s2, _ = oracle.lipschitz(x, gamma, rtol=1e-14, max_iter=1000)
    assert s2 == pytest.approx(4.0 + d @ d, rel=1e-10)
    r = oracle.papg(x, ybar, gamma, 1e-13, max_iters=20000, check_every=10)
    np.testing.assert_allclose(r["y"], y, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(r["xi"], xi, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(r["lam"], lam, rtol=1e-8, atol=1e-11)
    ex = exact_solve(x, ybar, gamma)
    np.testing.assert_allclose(ex["y"], y, rtol=1e-12, atol=1e-13)


def test_constant_observations_fixed_point():
    # ybar constant: (y, xi) = (ybar, 0) is feasible and unconstrained-optimal, lam = 0 stays.
    rng = np.random.default_rng(1)
    x = rng.standard_normal((25, 3))
    ybar = np.full(25, 2.5)
    r = oracle.papg(x, ybar, 1e-3, 1e-12, max_iters=5, check_every=1)
    assert r["iters"] == 1
    assert np.all(r["lam"] == 0.0)
    np.testing.assert_array_equal(r["y"], ybar)
    np.testing.assert_array_equal(r["xi"], 0.0)


def test_affine_data_matches_exact():
    # ybar from an affine function with a non-zero slope: xi = 0 violates the pairs, so the
    # multipliers must move the subgradients towards the slope; compare with the exact solver.
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (10, 2))
    ybar = x @ np.array([0.3, -0.2]) + 1.0
    gamma = 0.05
    ex = exact_solve(x, ybar, gamma)
    r = oracle.papg(x, ybar, gamma, 1e-12, max_iters=200000, check_every=50)
    np.testing.assert_allclose(r["y"], ex["y"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(r["xi"], ex["xi"], rtol=0, atol=1e-8)


# --- exact solves at tiny N (PIN-1) -------------------------------------------------------------

@pytest.mark.parametrize("N,n,seed,gamma,kind", [
    (12, 1, 0, 1e-1, "sq"),
    (15, 2, 1, 1e-2, "sq"),
    (18, 3, 2, 1e-1, "lse"),
    (10, 2, 3, 1e-3, "sq"),
])
def test_papg_matches_exact_nnls(N, n, seed, gamma, kind):
    x, ybar = _rand_problem(N, n, seed, kind)
    ex = exact_solve(x, ybar, gamma)
    assert ex["min_constraint"] >= -1e-9
    r = oracle.papg(x, ybar, gamma, 1e-11, max_iters=400000, check_every=50)
    assert r["status"] == "converged"
    scale = max(1.0, np.abs(ex["y"]).max())
    np.testing.assert_allclose(r["y"], ex["y"], rtol=0, atol=1e-8 * scale)
    np.testing.assert_allclose(r["xi"], ex["xi"], rtol=0, atol=1e-6 * max(1.0, np.abs(ex["xi"]).max()))
    # p*_g is unique even when lam* is not.
    g = oracle.dual_objective(x, ybar, gamma, r["lam"])
    assert g == pytest.approx(ex["p_star"], rel=1e-9)
    # the KKT report is tiny at the exact solution
    rep = oracle.kkt_report(x, ybar, gamma, ex["lam"])
    assert rep["kkt"] <= 1e-8


# --- spectral facts (Lemma lem:O1-constant) and the Lipschitz constant ---------------------------

def test_lipschitz_all_points_equal():
    # With every x_l equal, A2 = 0 and sigma_max(C)^2 = sigma_max(A1)^2 = 2N.
    N = 37
    x = np.ones((N, 3)) * 0.25
    L, s2, _ = oracle.lipschitz(x, 1e-3, rtol=1e-13, max_iter=2000)
    assert s2 == pytest.approx(2 * N, rel=1e-9)
    assert L == pytest.approx(2 * N / 1e-3, rel=1e-9)


@pytest.mark.parametrize("N,n,seed", [(12, 2, 0), (16, 3, 1)])
def test_lipschitz_matches_dense_svd(N, n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((N, n))
    A1, A2, _ = explicit_constraints(x)
    smax = np.linalg.svd(np.hstack([A1, A2]), compute_uv=False)[0]
    _, s2, _ = oracle.lipschitz(x, 1.0, rtol=1e-14, max_iter=5000)
    assert s2 == pytest.approx(smax ** 2, rel=1e-7)


def test_lipschitz_bounds():
    # ||A2||^2 <= sigma^2 <= 2N + ||A2||^2 <= (sqrt(2N) + B_x N)^2, with ||A2||^2 = max_l of the
    # largest eigenvalue of sum_j (x_l - x_j)(x_l - x_j)^T (A2 is block diagonal).
    x, _ = W.sq_norm(120, 3, 0.1, 4)
    N = x.shape[0]
    a2 = max(np.linalg.eigvalsh((xl - x).T @ (xl - x)).max() for xl in x)
    _, s2, _ = oracle.lipschitz(x, 1e-3)
    bx = np.sqrt((x ** 2).sum(axis=1)).max()
    assert a2 * (1 - 1e-6) <= s2 <= 2 * N + a2
    assert 2 * N + a2 <= (np.sqrt(2 * N) + bx * N) ** 2


# --- dual function identities ------------------------------------------------------------------

def test_dual_value_closed_form_and_gap_identity():
    # g(lam) = -u^T ybar - 1/2||u||^2 - ||w||^2/(2g) for (u, w) = C^T lam, and
    # r_g(eta(lam)) - g(lam) = sum lam_ij s_ij (the paper's duality gap lam^T C eta).
    x, ybar = W.sq_norm(30, 2, 0.1, 9)
    gamma = 1e-2
    rng = np.random.default_rng(0)
    lam = rng.uniform(0, 0.01, (30, 30))
    np.fill_diagonal(lam, 0.0)
    A1, A2, pairs = explicit_constraints(x)
    theta = np.array([lam[i, j] for (i, j) in pairs])
    u = A1.T @ theta
    w = A2.T @ theta
    g_cf = -u @ ybar - 0.5 * u @ u - (w @ w) / (2 * gamma)
    g = oracle.dual_objective(x, ybar, gamma, lam)
    assert g == pytest.approx(g_cf, rel=1e-12)
    y, xi = oracle.primal_from_dual(x, ybar, gamma, lam)
    s = oracle.pair_residual(x, y, xi)
    gap = oracle.primal_objective(ybar, gamma, y, xi) - g
    assert gap == pytest.approx(np.sum(lam * s), rel=1e-10)
    # the stopping report's complementarity sum and dual value, against the explicit constraint
    # matrices (constraint values A1 y + A2 xi in the pair order of Definition def:A1A2)
    cvals = A1 @ y + A2 @ xi.reshape(-1)
    assert cvals.min() < 0.0 < cvals.max()                  # violated pairs carry multipliers too
    rep = oracle.kkt_report(x, ybar, gamma, lam)
    assert rep["comp_sum"] == pytest.approx(float(theta @ cvals), rel=1e-10)
    assert rep["dual_obj"] == pytest.approx(g_cf, rel=1e-10)


def test_dual_gradient_finite_difference():
    # eq. dual gradient: grad g(lam) = -C eta(lam).  Central differences on random entries.
    x, ybar = W.sq_norm(12, 2, 0.1, 3)
    gamma = 0.1
    rng = np.random.default_rng(1)
    lam = rng.uniform(0, 0.1, (12, 12))
    np.fill_diagonal(lam, 0.0)
    y, xi = oracle.primal_from_dual(x, ybar, gamma, lam)
    s = oracle.pair_residual(x, y, xi)
    h = 1e-6
    for (i, j) in [(0, 1), (3, 7), (11, 2), (5, 4)]:
        lp, lm = lam.copy(), lam.copy()
        lp[i, j] += h
        lm[i, j] -= h
        fd = (oracle.dual_objective(x, ybar, gamma, lp) - oracle.dual_objective(x, ybar, gamma, lm)) / (2 * h)
        assert fd == pytest.approx(-s[i, j], rel=1e-6, abs=1e-8)


# --- convergence facts (eq:apg-rate, Theorem thm:rate, Section 4.1) ------------------------------

def test_apg_rate_and_primal_error_bound():
    x, ybar = W.sq_norm(10, 2, 0.1, 5)
    gamma = 0.05
    ex = exact_solve(x, ybar, gamma)
    pstar = ex["p_star"]
    L, _, _ = oracle.lipschitz(x, gamma)
    its = []
    oracle.papg(x, ybar, gamma, 0.0, L=L, max_iters=400, check_every=1000, iterates=its)
    lam_star_sq = float(np.sum(ex["lam"] ** 2))
    for k, lam in its:
        g = oracle.dual_objective(x, ybar, gamma, lam)
        # eq:apg-rate with theta^0 = 0
        assert pstar - g <= 2 * L * lam_star_sq / (k + 1) ** 2 * (1 + 1e-9) + 1e-12
        # eq:primal-convergence
        y, xi = oracle.primal_from_dual(x, ybar, gamma, lam)
        lhs = np.sum((y - ex["y"]) ** 2) + gamma * np.sum((xi - ex["xi"]) ** 2)
        assert lhs <= 2 * (pstar - g) * (1 + 1e-7) + 1e-12
        assert np.all(lam >= 0.0)
        assert np.all(np.diag(lam) == 0.0)


def test_momentum_beats_plain_gradient_ascent():
    # Section 4.1: infeasibility of the accelerated iterates falls much faster than that of
    # plain dual gradient ascent.
    x, ybar = W.sq_norm(40, 2, 0.1, 6)
    gamma = 1e-3
    L, _, _ = oracle.lipschitz(x, gamma)
    a = oracle.papg(x, ybar, gamma, 0.0, L=L, max_iters=3000, check_every=3000)
    b = oracle.papg(x, ybar, gamma, 0.0, L=L, max_iters=3000, check_every=3000, momentum=False)
    assert a["report"]["infeas_rms"] < 0.5 * b["report"]["infeas_rms"]
    assert a["report"]["dual_obj"] > b["report"]["dual_obj"]


def test_fista_schedule():
    t, beta = oracle.fista_schedule(200)
    k = np.arange(1, 201)
    assert t[1] == 1.0 and beta[1] == 0.0
    np.testing.assert_allclose(t[2:202] ** 2 - t[2:202], t[1:201] ** 2, rtol=1e-12)
    assert np.all(t[1:201] >= (k + 1) / 2.0 - 1e-12)
    assert np.all((beta[1:] >= 0) & (beta[1:] < 1))


# --- certificate (PIN-9) --------------------------------------------------------------------

@pytest.mark.parametrize("iters", [20, 200, 2000])
def test_certificate_brackets_true_error(iters):
    x, ybar = W.sq_norm(14, 2, 0.1, 8)
    gamma = 1e-2
    ex = exact_solve(x, ybar, gamma)
    r = oracle.papg(x, ybar, gamma, 0.0, max_iters=iters, check_every=10 ** 9)
    c = oracle.repair_certificate(x, ybar, gamma, r["lam"])
    A1, A2 = ex["A1"], ex["A2"]
    cons = A1 @ c["y_rep"] + A2 @ c["xi_rep"].reshape(-1)
    assert cons.min() >= -1e-10                      # the repaired point is feasible
    assert c["primal_rep"] >= ex["p_star"] - 1e-10   # hence no better than the optimum
    assert c["cert_gap"] >= -1e-12
    err = np.linalg.norm(r["y"] - ex["y"])
    assert err <= c["y_err_bound"] * (1 + 1e-9) + 1e-12
    rep = oracle.kkt_report(x, ybar, gamma, r["lam"])
    if c["method"] == "max-affine":
        assert c["max_fit_change"] == pytest.approx(rep["max_viol"] * rep["scale"], rel=1e-9, abs=1e-14)
    else:   # the potentials are at least the first relaxation round (the max-affine heights)
        assert c["max_fit_change"] >= rep["max_viol"] * rep["scale"] * (1 - 1e-9) - 1e-14


@pytest.mark.parametrize("seed,iters", [(8, 300), (9, 1000), (10, 3000)])
def test_own_slope_certificate_is_feasible_and_tight(seed, iters):
    x, ybar = W.sq_norm(14, 2, 0.1, seed)
    gamma = 1e-2
    ex = exact_solve(x, ybar, gamma)
    r = oracle.papg(x, ybar, gamma, 0.0, max_iters=iters, check_every=10 ** 9, adaptive=True, restart=True)
    c = oracle.repair_certificate(x, ybar, gamma, r["lam"])
    assert c["own_converged"]
    A1, A2 = ex["A1"], ex["A2"]
    y, xi = oracle.primal_from_dual(x, ybar, gamma, r["lam"])
    # own-slope point: the same subgradients, heights raised by the potentials
    yo = y + (c["y_rep"] - y) if c["method"] == "own-slope" else None
    if yo is not None:
        np.testing.assert_array_equal(c["xi_rep"], xi)
        assert np.all(c["y_rep"] >= y - 1e-15)
        cons = A1 @ c["y_rep"] + A2 @ c["xi_rep"].reshape(-1)
        assert cons.min() >= -1e-9
    # both certificates bracket the true suboptimality; the reported one is the smaller
    true_sub = ex["p_star"] - oracle.dual_objective(x, ybar, gamma, r["lam"])
    assert c["cert_gap_affine"] >= true_sub - 1e-12 and c["cert_gap_own"] >= true_sub - 1e-12
    assert c["cert_gap"] == min(c["cert_gap_affine"], c["cert_gap_own"])


# --- invariances (PIN-6) ---------------------------------------------------------------------

def test_translation_shift_and_permutation_invariance():
    x, ybar = W.sq_norm(30, 2, 0.1, 12)
    gamma = 1e-2
    L, _, _ = oracle.lipschitz(x, gamma)
    base = oracle.papg(x, ybar, gamma, 0.0, L=L, max_iters=300, check_every=10 ** 9)
    # shifting the locations leaves every constraint unchanged
    sh = oracle.papg(x + np.array([3.0, -1.5]), ybar, gamma, 0.0, L=L, max_iters=300, check_every=10 ** 9)
    np.testing.assert_allclose(sh["y"], base["y"], atol=1e-9)
    np.testing.assert_allclose(sh["xi"], base["xi"], atol=1e-7)
    # adding a constant to the observations adds it to the fit (A1 1 = 0)
    up = oracle.papg(x, ybar + 4.0, gamma, 0.0, L=L, max_iters=300, check_every=10 ** 9)
    np.testing.assert_allclose(up["y"], base["y"] + 4.0, atol=1e-9)
    np.testing.assert_allclose(up["xi"], base["xi"], atol=1e-7)
    # permuting the points permutes the fit and the multipliers
    p = np.random.default_rng(0).permutation(30)
    pe = oracle.papg(x[p], ybar[p], gamma, 0.0, L=L, max_iters=300, check_every=10 ** 9)
    np.testing.assert_allclose(pe["y"], base["y"][p], atol=1e-10)
    np.testing.assert_allclose(pe["lam"], base["lam"][np.ix_(p, p)], atol=1e-12)


def test_kkt_report_detects_violation():
    # lam = 0 on noisy non-convex data leaves violated pairs: the natural residual is the largest
    # violation and the paper's normalized infeasibility is positive.
    x, ybar = W.sq_norm(20, 1, 0.5, 3)
    rep = oracle.kkt_report(x, ybar, 1e-3, np.zeros((20, 20)))
    d = ybar[None, :] - ybar[:, None]
    worst = max(0.0, -d[~np.eye(20, dtype=bool)].min())
    assert rep["max_viol"] * rep["scale"] == pytest.approx(worst, rel=1e-12)
    assert rep["nat_res_max"] == pytest.approx(rep["max_viol"], rel=1e-12)
    assert rep["infeas_rms"] > 0.0
    assert rep["scale"] == max(1.0, ybar.max() - ybar.min())


# --- adaptive step (eq. eq:adaptive-check; PAPG_A of Section 4) --------------------------------

def test_adaptive_check_is_the_quadratic_identity():
    # With every pair dualized g is a concave quadratic, so g(lam~ + D) - g(lam~) - <grad g(lam~), D>
    # equals -(||A1^T D||^2 + ||A2^T D||^2 / g) / 2 exactly: the paper's inequality is equivalent to
    # ||A1^T D||^2 + ||A2^T D||^2 / g <= s ||D||^2.  Checked with explicit dual values.
    x, ybar = W.sq_norm(25, 2, 0.1, 21)
    gamma = 1e-2
    rng = np.random.default_rng(4)
    lt = rng.uniform(0, 0.01, (25, 25))
    np.fill_diagonal(lt, 0.0)
    D = rng.uniform(-0.002, 0.002, (25, 25))
    np.fill_diagonal(D, 0.0)
    y, xi = oracle.primal_from_dual(x, ybar, gamma, lt)
    grad = -oracle.pair_residual(x, y, xi)
    lhs = oracle.dual_objective(x, ybar, gamma, lt + D) - oracle.dual_objective(x, ybar, gamma, lt) \
        - float(np.sum(grad * D))
    u, w = oracle.pair_adjoint(x, D)
    assert lhs == pytest.approx(-0.5 * (u @ u + np.sum(w * w) / gamma), rel=1e-8)


@pytest.mark.parametrize("N,n,seed,gamma", [(12, 1, 0, 1e-1), (15, 2, 1, 1e-2), (10, 2, 3, 1e-3)])
def test_adaptive_matches_exact_nnls(N, n, seed, gamma):
    x, ybar = _rand_problem(N, n, seed)
    ex = exact_solve(x, ybar, gamma)
    steps = []
    r = oracle.papg(x, ybar, gamma, 1e-11, max_iters=400000, check_every=50, adaptive=True, steps=steps)
    assert r["status"] == "converged"
    scale = max(1.0, np.abs(ex["y"]).max())
    np.testing.assert_allclose(r["y"], ex["y"], rtol=0, atol=1e-8 * scale)
    L, _, _ = oracle.lipschitz(x, gamma)
    # the rule starts from s_0 = L and only multiplies by powers of upsilon
    ratios = np.log2(np.array(steps) / L)
    np.testing.assert_allclose(ratios, np.round(ratios), atol=1e-9)


def test_adaptive_accepted_steps_satisfy_the_check_and_beat_constant_steps():
    x, ybar = W.sq_norm(40, 2, 0.1, 6)
    gamma = 1e-3
    L, _, _ = oracle.lipschitz(x, gamma)
    its, steps = [], []
    oracle.papg(x, ybar, gamma, 0.0, L=L, max_iters=150, check_every=10 ** 9, adaptive=True,
                iterates=its, steps=steps)
    # re-derive every accepted step from the stored iterates and check eq. eq:adaptive-check
    t, beta = oracle.fista_schedule(150)
    prev = np.zeros((40, 40))
    prev2 = np.zeros((40, 40))
    for (k, lam), s in zip(its, steps):
        b = beta[k - 1] if k >= 2 else 0.0
        lt = prev + b * (prev - prev2)
        y, xi = oracle.primal_from_dual(x, ybar, gamma, lt)
        sres = oracle.pair_residual(x, y, xi)
        ref = np.maximum(0.0, lt - sres / s)
        np.fill_diagonal(ref, 0.0)
        np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-15)
        d = lam - lt
        gl = oracle.dual_objective(x, ybar, gamma, lam)
        gt = oracle.dual_objective(x, ybar, gamma, lt)
        assert gl >= gt - np.sum(sres * d) - 0.5 * s * np.sum(d * d) - 1e-12 * max(1.0, abs(gt))
        prev2, prev = prev, lam
    a = oracle.papg(x, ybar, gamma, 0.0, L=L, max_iters=150, check_every=150, adaptive=True)
    c = oracle.papg(x, ybar, gamma, 0.0, L=L, max_iters=150, check_every=150)
    assert a["report"]["dual_obj"] >= c["report"]["dual_obj"]
    assert min(steps) < L


# --- momentum restart (an option beyond the paper, on top of the adaptive step) ---------------

@pytest.mark.parametrize("N,n,seed,gamma", [(12, 1, 0, 1e-1), (15, 2, 1, 1e-2), (10, 2, 3, 1e-3)])
def test_adaptive_restart_matches_exact_nnls(N, n, seed, gamma):
    x, ybar = _rand_problem(N, n, seed)
    ex = exact_solve(x, ybar, gamma)
    r = oracle.papg(x, ybar, gamma, 1e-11, max_iters=400000, check_every=50, adaptive=True, restart=True)
    assert r["status"] == "converged"
    scale = max(1.0, np.abs(ex["y"]).max())
    np.testing.assert_allclose(r["y"], ex["y"], rtol=0, atol=1e-8 * scale)


def test_restart_resets_the_momentum_where_the_step_opposes_the_movement():
    # Re-derive every iterate of the restarted run from its accepted steps with an independent
    # restart rule: after an iteration with <lam^k - lam~^k, lam^k - lam^{k-1}> < 0 the FISTA
    # sequence starts again at t = 1, so the next extrapolation weight is zero.
    x, ybar = W.sq_norm(40, 2, 0.1, 6)
    gamma = 1e-3
    L, _, _ = oracle.lipschitz(x, gamma)
    its, steps = [], []
    oracle.papg(x, ybar, gamma, 0.0, L=L, max_iters=300, check_every=10 ** 9, adaptive=True, restart=True,
                iterates=its, steps=steps)
    prev = np.zeros((40, 40))
    prev2 = np.zeros((40, 40))
    t, b, restarts = 1.0, 0.0, 0
    for (k, lam), s in zip(its, steps):
        lt = prev + b * (prev - prev2)
        y, xi = oracle.primal_from_dual(x, ybar, gamma, lt)
        ref = np.maximum(0.0, lt - oracle.pair_residual(x, y, xi) / s)
        np.fill_diagonal(ref, 0.0)
        np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-15)
        if np.sum((lam - lt) * (lam - prev)) < 0.0:
            t = 1.0
            restarts += 1
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        b = (t - 1.0) / t_next
        t = t_next
        prev2, prev = prev, lam
    assert restarts > 0

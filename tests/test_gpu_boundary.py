"""Boundary options on the GPU: the warm start lam^0 (cr_options.lambda0), the frame switch of the
mixed modes (cr_options.center) and the served multipliers (cr_options.keep_lambda with the lambda
argument of cr_wait / cr_poll).

The regularized QP (eq. ``regularize``) has a unique minimizer, so a fit started anywhere in the
dual's feasible set must reach the same (y*, xi*) as the FP64 oracle's converged fit in
``tests/golden/c1_sqnorm_N200_n2_seed0_tol1e-10.npz`` (bars as in the converged-fit tests: y within
1e-6 relative in FP64, 1e-4 in the mixed modes; xi through Theorem ``thm:rate``).  A start at an
already converged point passes the iteration-0 test and takes no iteration.  Paths that run the same
kernels in the same order (host or device inputs, alone or served, with or without scratch) must
agree bitwise."""
import ctypes as C
import json
import math
import os

import numpy as np
import pytest

from paper_1608_02227_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
REF = "c1_sqnorm_N200_n2_seed0_tol1e-10"


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return torch


def _ref():
    d = np.load(os.path.join(GOLDEN, REF + ".npz"), allow_pickle=False)
    meta = json.loads(str(d["meta"]))
    x, ybar = W.make("sqnorm_N200_n2", seed=meta["seed"])
    return x, ybar, d["y"], d["xi"], meta


def _check(r, y_ref, xi_ref, meta, tol, y_bar):
    delta = meta["delta"]
    assert r.report["kkt"] <= tol
    assert np.max(np.abs(r.y - y_ref)) / np.max(np.abs(y_ref)) <= y_bar
    G_gpu, G_ref = max(0.0, r.report["cert_gap"]), max(0.0, meta["cert_gap"])
    assert np.max(np.abs(r.xi - xi_ref)) <= math.sqrt(2.0 * G_gpu / delta) + math.sqrt(2.0 * G_ref / delta)


@pytest.mark.parametrize("precision,tol,y_bar", [("fp64", 1e-9, 1e-6), ("mixed_fp32", 1e-6, 1e-4),
                                                 ("mixed_bf16", 1e-6, 1e-4)])
def test_warm_started_fit_matches_oracle(cr, torch_dev, precision, tol, y_bar):
    """Start from the multipliers of a loose fit of perturbed observations (a nearby problem, as a
    continuation step would): the fit still reaches the oracle's minimizer.  (A warm start need not
    save iterations: momentum and step adaptation restart from it, so only the end point is fixed.)"""
    x, ybar, y_ref, xi_ref, meta = _ref()
    delta = meta["delta"]
    yb2 = ybar + 0.02 * np.random.default_rng(5).standard_normal(ybar.shape)
    start = cr.fit(x, yb2, delta, 1e-3, cr.Options(precision="fp64"), return_lambda=True)
    opt = cr.Options(precision=precision)
    print(f"warm start {precision} tol {tol}", flush=True)
    warm = cr.fit(x, ybar, delta, tol, opt, allow_noconv=False, lambda0=start.lam)
    _check(warm, y_ref, xi_ref, meta, tol, y_bar)
    assert warm.report["iters"] > 0


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_warm_start_at_a_converged_point_takes_no_iteration(cr, torch_dev, precision):
    x, ybar, _, _, meta = _ref()
    opt = cr.Options(precision=precision)
    cold = cr.fit(x, ybar, meta["delta"], 1e-6, opt, allow_noconv=False, return_lambda=True)
    warm = cr.fit(x, ybar, meta["delta"], 1e-6, opt, allow_noconv=False, lambda0=cold.lam, return_lambda=True)
    assert warm.report["iters"] == 0 and warm.report["checks"] == 1
    # the same multipliers (the split forms hold lam as H + l to ~1e-14 relative)
    assert np.max(np.abs(warm.lam - cold.lam)) <= 1e-12 * np.max(cold.lam)
    assert np.max(np.abs(warm.y - cold.y)) <= 1e-10 * np.max(np.abs(cold.y))


def test_warm_start_from_device_memory_equals_host(cr, torch_dev):
    torch = torch_dev
    x, ybar, _, _, meta = _ref()
    start = cr.fit(x, ybar + 0.01, meta["delta"], 1e-3, cr.Options(), return_lambda=True)
    opt = cr.Options(precision="mixed_fp32")
    host = cr.fit(x, ybar, meta["delta"], 1e-5, opt, lambda0=start.lam)
    dev = cr.fit(torch.from_numpy(x).cuda(), torch.from_numpy(ybar).cuda(), meta["delta"], 1e-5, opt,
                 lambda0=torch.from_numpy(start.lam).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host.y, dev.y.cpu().numpy())
    np.testing.assert_array_equal(host.xi, dev.xi.cpu().numpy())
    assert host.report["iters"] == dev.report["iters"]


def test_warm_start_rejects_negative_or_non_finite_multipliers(cr, torch_dev):
    x, ybar, _, _, meta = _ref()
    N = x.shape[0]
    for bad in (-1e-3, float("nan")):
        lam0 = np.zeros((N, N))
        lam0[3, 7] = bad
        with pytest.raises(cr.CRError) as e:
            cr.fit(x, ybar, meta["delta"], 1e-4, cr.Options(), lambda0=lam0)
        assert e.value.code == cr.CR_EINVAL
    # the diagonal is ignored
    lam0 = np.zeros((N, N))
    np.fill_diagonal(lam0, -5.0)
    a = cr.fit(x, ybar, meta["delta"], 1e-4, cr.Options(), lambda0=lam0)
    b = cr.fit(x, ybar, meta["delta"], 1e-4, cr.Options(), lambda0=np.zeros((N, N)))
    np.testing.assert_array_equal(a.y, b.y)


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_bf16"])
def test_mixed_fit_in_the_callers_frame_matches_oracle(cr, torch_dev, precision):
    """center = 0: the mixed pass works on the caller's coordinates (here already centred around 0,
    so both frames are well conditioned); the minimizer is the same."""
    x, ybar, y_ref, xi_ref, meta = _ref()
    r = cr.fit(x, ybar, meta["delta"], 1e-6, cr.Options(precision=precision, center=False), allow_noconv=False)
    _check(r, y_ref, xi_ref, meta, 1e-6, 1e-4)


def test_served_multipliers_and_warm_start_equal_the_fit_alone(cr, torch_dev):
    x, ybar, _, _, meta = _ref()
    delta = meta["delta"]
    reqs = [W.sq_norm(150 + 40 * r, 3, 0.1, 70 + r) for r in range(3)] + [(x, ybar)]
    opt = cr.Options(precision="mixed_fp32", keep_lambda=True)
    alone = [cr.fit(a, b, delta, 1e-4, opt, return_lambda=True) for (a, b) in reqs]
    starts = [0.5 * r.lam for r in alone]
    warm_alone = [cr.fit(a, b, delta, 1e-5, opt, return_lambda=True, lambda0=s) for (a, b), s in zip(reqs, starts)]
    with cr.Server(max_slots=3) as srv:
        ids = [srv.submit(a, b, delta, 1e-4, opt) for (a, b) in reqs]
        wids = [srv.submit(a, b, delta, 1e-5, opt, lambda0=s) for (a, b), s in zip(reqs, starts)]
        served = [srv.wait(i) for i in ids]
        warm_served = [srv.wait(i) for i in wids]
    for a, s in list(zip(alone, served)) + list(zip(warm_alone, warm_served)):
        np.testing.assert_array_equal(a.y, s.y)
        np.testing.assert_array_equal(a.xi, s.xi)
        np.testing.assert_array_equal(a.lam, s.lam)
        assert a.report["iters"] == s.report["iters"]


def test_served_lambda_needs_keep_lambda(cr, torch_dev):
    lib = cr.load()
    x, ybar = W.sq_norm(120, 2, 0.1, 9)
    N, n = x.shape
    with cr.Server(max_slots=1) as srv:
        rid = srv.submit(x, ybar, 1e-3, 1e-3, cr.Options(precision="mixed_fp32"))
        lam = np.empty((N, N))
        y = np.empty(N)
        xi = np.empty((N, n))
        rc = lib.cr_wait(srv._h, rid, cr._ptr(y), cr._ptr(xi), cr._ptr(lam), None, None)
        assert rc == cr.CR_EINVAL
        r = srv.wait(rid)      # the result is still there
        assert r.lam is None and r.report["iters"] > 0

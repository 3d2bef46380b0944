"""Serving (continuous batching) on the GPU: results are the same alone and in a mix, admission
respects the slot count and the byte budget, and oversize requests are refused."""
import time

import numpy as np
import pytest

from paper_1608_02227_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return torch


def _requests(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        N = int(rng.integers(90, 700))
        n = int(rng.integers(2, 33))
        if r % 2:
            x, yb = W.sq_norm(N, n, 0.1, 1000 + r)
        else:
            x, yb = W.log_sum_exp_affine(N, n, 8, 0.1, 1000 + r, x_dist="uniform")
        out.append((x, yb))
    return out


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_bf16", "fp64"])
def test_mix_equals_alone(cr, torch_dev, precision):
    reqs = _requests(8, 3)
    opt = cr.Options(precision=precision, max_iters=3000)
    alone = [cr.fit(x, yb, 1e-3, 1e-3, opt) for (x, yb) in reqs]
    with cr.Server(max_slots=4) as srv:
        ids = [srv.submit(x, yb, 1e-3, 1e-3, opt) for (x, yb) in reqs]
        mixed = [srv.wait(i) for i in ids]
    for a, m in zip(alone, mixed):
        np.testing.assert_array_equal(a.y, m.y)
        np.testing.assert_array_equal(a.xi, m.xi)
        assert a.report["iters"] == m.report["iters"]
        assert m.extra["latency_s"] > 0.0


def test_admission_by_bytes_and_slots(cr, torch_dev):
    reqs = [W.sq_norm(400, 5, 0.1, 40 + r) for r in range(5)]     # equal shapes: equal reservations
    one = cr.state_bytes(400, 5, "fp64")
    opt = cr.Options(max_iters=400)
    with cr.Server(max_slots=4, byte_budget=one + one // 2) as srv:   # room for one fit at a time
        ids = [srv.submit(x, yb, 1e-3, 1e-6, opt) for (x, yb) in reqs]
        peak = 0
        while True:
            st = srv.stats()
            peak = max(peak, st["running"])
            assert st["resident_bytes"] <= one + one // 2
            if st["finished"] == len(ids):
                break
            time.sleep(0.002)
        res = [srv.wait(i) for i in ids]
    assert peak == 1
    # strict FIFO with room for one fit: each request waits for all earlier ones, so latencies
    # (measured from near-simultaneous submissions) grow with the submission order
    lat = [r.extra["latency_s"] for r in res]
    assert all(b > a for a, b in zip(lat, lat[1:]))
    assert all(r.report["iters"] == 400 for r in res)


def test_oversize_request_is_refused(cr, torch_dev):
    x, yb = W.sq_norm(300, 3, 0.1, 0)
    with cr.Server(max_slots=2, byte_budget=1 << 20) as srv:
        with pytest.raises(cr.CRError) as e:
            srv.submit(x, yb, 1e-3, 1e-4)
        assert e.value.code == cr.CR_ENOMEM


def test_poll_and_stats(cr, torch_dev):
    x, yb = W.sq_norm(150, 2, 0.1, 5)
    with cr.Server(max_slots=1) as srv:
        rid = srv.submit(x, yb, 1e-3, 1e-3, cr.Options(max_iters=2000))
        got = None
        for _ in range(20000):
            got = srv.poll(rid)
            if got is not None:
                break
            time.sleep(0.001)
        assert got is not None
        assert srv.stats()["finished"] == 1


def test_destroy_cancels_queued_requests(cr, torch_dev):
    """Destroying a context with requests still queued: the running fit finishes, the queued ones are
    dropped, and a caller blocked in cr_wait on one of them returns CR_ECANCELED (it is woken
    before the context goes away)."""
    import threading
    reqs = [W.sq_norm(1000, 2, 0.1, 70 + r) for r in range(6)]
    opt = cr.Options(precision="mixed_fp32", max_iters=3000)
    srv = cr.Server(max_slots=1)
    ids = [srv.submit(x, yb, 1e-3, 1e-9, opt) for (x, yb) in reqs]
    got = {}

    def waiter():
        try:
            srv.wait(ids[-1])
            got["code"] = cr.CR_OK
        except cr.CRError as e:
            got["code"] = e.code
    t = threading.Thread(target=waiter)
    t.start()
    time.sleep(0.3)
    assert srv.stats()["queued"] >= 1
    srv.close()
    t.join(timeout=120)
    assert not t.is_alive()
    assert got["code"] == cr.CR_ECANCELED


def test_slot_arenas_are_reused_across_sizes(cr, torch_dev):
    """One slot runs fits of growing and shrinking size back to back in its arena (cleared between
    fits): every result equals the fit run on its own."""
    shapes = [(300, 4), (900, 12), (150, 2), (700, 30), (220, 7)]
    reqs = [W.sq_norm(N, n, 0.1, 500 + k) for k, (N, n) in enumerate(shapes)]
    opt = cr.Options(precision="mixed_fp32", max_iters=1500)
    alone = [cr.fit(x, yb, 1e-3, 1e-4, opt) for (x, yb) in reqs]
    with cr.Server(max_slots=1) as srv:
        ids = [srv.submit(x, yb, 1e-3, 1e-4, opt) for (x, yb) in reqs]
        served = [srv.wait(i) for i in ids]
    for a, m in zip(alone, served):
        np.testing.assert_array_equal(a.y, m.y)
        np.testing.assert_array_equal(a.xi, m.xi)
        assert a.report["iters"] == m.report["iters"]


@pytest.mark.parametrize("precision", ["mixed_fp32", "fp64"])
def test_grouped_rounds_carry_several_fits(cr, torch_dev, precision):
    """Small fits submitted together iterate in grouped rounds (one pass launch per kernel variant
    for all of them), and each result is still bitwise the fit run alone."""
    reqs = _requests(6, 11)
    opt = cr.Options(precision=precision, max_iters=2000)
    alone = [cr.fit(x, yb, 1e-3, 1e-4, opt) for (x, yb) in reqs]
    with cr.Server(max_slots=6, group_max_n=2048) as srv:
        ids = [srv.submit(x, yb, 1e-3, 1e-4, opt) for (x, yb) in reqs]
        served = [srv.wait(i) for i in ids]
        st = srv.group_stats()
    for a, m in zip(alone, served):
        np.testing.assert_array_equal(a.y, m.y)
        np.testing.assert_array_equal(a.xi, m.xi)
        assert a.report["iters"] == m.report["iters"]
    # every trial round of every fit went through the batcher, most of them shared
    assert st["fit_rounds"] == sum(m.report["trials"] / 2 for m in served)
    assert st["fit_rounds"] >= 1.5 * st["rounds"]
    assert st["pass_launches"] < st["fit_rounds"]

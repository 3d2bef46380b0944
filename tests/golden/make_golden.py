"""Writes the stored expected values used by the GPU parity tests.

Every value here comes from the FP64 oracle (``oracle/``) run on the seeded workload generators;
nothing is taken from the GPU path.  Re-run with ``python tests/golden/make_golden.py``.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1608_02227_amd import workloads as W  # noqa: E402

CASES = [
    # name, workload, seed, N override, tol, check_every, adaptive step, momentum restart
    ("sqnorm_N200_n2_seed0_tol1e-4", "sqnorm_N200_n2", 0, None, 1e-4, 50, False, False),
    ("lse8_N400_n10_seed1_tol1e-4", "lse8_N2000_n10", 1, 400, 1e-4, 50, False, False),
    # The adaptive step's trajectory is sensitive to rounding (a 1e-15 change of ybar moves the
    # stopping iteration by a few percent), so its fixtures are converged far enough that any two
    # runs meet the fitted-value bar: KKT 1e-7.
    ("adaptive_sqnorm_N200_n2_seed0_tol1e-7", "sqnorm_N200_n2", 0, None, 1e-7, 50, True, False),
    ("adaptive_lse8_N150_n10_seed1_tol1e-7", "lse8_N2000_n10", 1, 150, 1e-7, 50, True, False),
    ("adaptive_quad_N300_n40_seed2_tol1e-7", "quad_N8000_n40", 2, 300, 1e-7, 50, True, False),
    ("restart_sqnorm_N200_n2_seed0_tol1e-7", "sqnorm_N200_n2", 0, None, 1e-7, 50, True, True),
    ("restart_lse8_N400_n10_seed1_tol1e-7", "lse8_N2000_n10", 1, 400, 1e-7, 50, True, True),
    ("restart_quad_N600_n40_seed2_tol1e-7", "quad_N8000_n40", 2, 600, 1e-7, 50, True, True),
]


# Converged references at full configuration sizes and for requests of the serving stream, written
# as .npz (y, xi, lam-free) with the run's metadata as a JSON string.  All use the adaptive step with
# the momentum restart: the constant step's KKT residual on the N=200, n=2 workload is still 4e-6
# after 400,000 iterations, so only the restarted rule reaches these tolerances.  Each reference is
# converged far below the comparison bars; the certificate (r(y', xi') - g(lam) for a feasible
# repair) bounds its distance from the unique optimum: ||y - y*||^2 + delta ||xi - xi*||^2 <= 2G.
# `spread` cases also run the oracle once more with ybar scaled by (1 + 1e-15) and store how far
# the two converged fits are apart.
CONVERGED = [
    # name, workload, seed, tol, spread
    ("c1_sqnorm_N200_n2_seed0_tol1e-10", "sqnorm_N200_n2", 0, 1e-10, True),
    ("c2_lse8_N2000_n10_seed0_tol1e-8", "lse8_N2000_n10", 0, 1e-8, False),
]
# requests of the serving stream (512 requests, seed 0) by index: N 185..581, n 2..32
SERVED = [0, 3, 4, 10, 12, 35, 36]
SERVED_TOL = 1e-8


def _converged(x, ybar, delta, tol):
    L, s2, pit = oracle.lipschitz(x, delta)
    r = oracle.papg(x, ybar, delta, tol, L=L, max_iters=400_000, check_every=50, adaptive=True, restart=True)
    cert = oracle.repair_certificate(x, ybar, delta, r["lam"])
    meta = {"source": "oracle.papg (FP64 numpy), adaptive step with momentum restart, every pair dualized",
            "delta": delta, "tol": tol, "L": L, "iters": r["iters"], "status": r["status"],
            "kkt": r["report"]["kkt"], "cert_gap": cert["cert_gap"], "y_err_bound": cert["y_err_bound"]}
    return r, meta


def _write_npz(name, y, xi, meta):
    path = os.path.join(HERE, name + ".npz")
    np.savez(path, y=y, xi=xi, meta=np.array(json.dumps(meta)))
    print(name, meta["iters"], meta["status"], meta["kkt"], meta["cert_gap"], flush=True)


def main_converged(only):
    for name, wl, seed, tol, spread in CONVERGED:
        if only and name not in only:
            continue
        w = W.WORKLOADS[wl]
        x, ybar = W.make(wl, seed=seed)
        r, meta = _converged(x, ybar, w.delta, tol)
        meta.update({"workload": wl, "seed": seed, "N": int(x.shape[0]), "n": int(x.shape[1])})
        if spread:
            r2, _ = _converged(x, ybar * (1.0 + 1e-15), w.delta, tol)
            meta["y_spread_rel"] = float(np.max(np.abs(r2["y"] - r["y"])) / np.max(np.abs(r["y"])))
            meta["xi_spread_abs"] = float(np.max(np.abs(r2["xi"] - r["xi"])))
        _write_npz(name, r["y"], r["xi"], meta)
    reqs = None
    for i in SERVED:
        name = f"served_req{i}_tol1e-8"
        if only and name not in only:
            continue
        if reqs is None:
            reqs = W.serving_requests(count=512, seed=0)
        q = reqs[i]
        r, meta = _converged(q.x, q.ybar, q.delta, SERVED_TOL)
        meta.update({"request": i, "stream": "serving_requests(count=512, seed=0)",
                     "N": int(q.x.shape[0]), "n": int(q.x.shape[1])})
        _write_npz(name, r["y"], r["xi"], meta)


def main():
    only = set(sys.argv[1:])
    if only and all(o.startswith(("c1_", "c2_", "served_")) for o in only):
        return main_converged(only)
    if not only:
        main_converged(only)
    for name, wl, seed, N, tol, every, adaptive, restart in CASES:
        if only and name not in only:
            continue
        w = W.WORKLOADS[wl]
        x, ybar = W.make(wl, seed=seed, N=N)
        L, s2, pit = oracle.lipschitz(x, w.delta)
        steps = []
        r = oracle.papg(x, ybar, w.delta, tol, L=L, max_iters=2_000_000, check_every=every,
                        adaptive=adaptive, steps=steps, restart=restart)
        cert = oracle.repair_certificate(x, ybar, w.delta, r["lam"])
        rep = {k: v for k, v in r["report"].items()}
        out = {
            "source": "oracle.papg (FP64 numpy), P-APG of Fig. fig:papg with every pair dualized",
            "workload": wl, "seed": seed, "N": int(x.shape[0]), "n": int(x.shape[1]), "delta": w.delta,
            "tol": tol, "check_every": every, "L": L, "sigma2": s2, "power_iters": pit,
            "adaptive": adaptive, "upsilon": 2.0 if adaptive else None, "restart": restart,
            "final_step": r["step"], "steps_head": steps[:60],
            "iters": r["iters"], "status": r["status"], "report": rep,
            "cert_gap": cert["cert_gap"], "y_err_bound": cert["y_err_bound"],
            "y": r["y"].tolist(),
        }
        # keep fixtures small: full xi only for small problems, its row norms otherwise
        if x.shape[0] * x.shape[1] <= 5000:
            out["xi"] = r["xi"].tolist()
        else:
            out["xi_row_norms"] = [float(v) for v in (r["xi"] ** 2).sum(axis=1) ** 0.5]
        path = os.path.join(HERE, name + ".json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(name, r["iters"], r["status"], rep["kkt"])


if __name__ == "__main__":
    main()

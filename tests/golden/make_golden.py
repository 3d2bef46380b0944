"""Writes the stored expected values used by the GPU parity tests.

Every value here comes from the FP64 oracle (``oracle/``) run on the seeded workload generators;
nothing is taken from the GPU path.  Re-run with ``python tests/golden/make_golden.py``.
"""
import json
import os
import sys

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


def main():
    only = set(sys.argv[1:])
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

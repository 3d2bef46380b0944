"""The oracle's pins catch planted mistakes.

Each case plants one plausible mistake in a copy of the oracle (a dropped term, a wrong sign, a
transposed operand, a swapped reduction, a wrong scale) and runs the CPU pin tests against that copy
(in a subprocess, with the copy first on the import path): some pin must fail.  The unmodified copy
must pass, so a failure is the mistake's doing.  Mistakes are planted in the oracle only, on the CPU.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["test_oracle_pins.py", "test_oracle_continuation.py"]

MUTATIONS = [
    # name, file, correct text, mistaken text
    ("residual_y_sign", "papg.py", "s = y[None, :] - y[:, None] + d[:, None] - xi @ x.T",
     "s = y[:, None] - y[None, :] + d[:, None] - xi @ x.T"),
    ("residual_transposed", "papg.py", "s = y[None, :] - y[:, None] + d[:, None] - xi @ x.T",
     "s = y[None, :] - y[:, None] + d[:, None] - x @ xi.T"),
    ("residual_dropped_d", "papg.py", "s = y[None, :] - y[:, None] + d[:, None] - xi @ x.T",
     "s = y[None, :] - y[:, None] - xi @ x.T"),
    ("adjoint_row_col_swapped", "papg.py", "u = col - row", "u = row - col"),
    ("adjoint_w_sign", "papg.py", "w = row[:, None] * x - lam @ x", "w = lam @ x - row[:, None] * x"),
    ("adjoint_transposed", "papg.py", "w = row[:, None] * x - lam @ x", "w = row[:, None] * x - lam.T @ x"),
    ("step1_scaling", "papg.py", "return ybar + u, w / gamma", "return ybar + u, w * gamma"),
    ("objective_gamma_factor", "papg.py", "0.5 * gamma * float(np.sum(xi ** 2))",
     "gamma * float(np.sum(xi ** 2))"),
    ("dual_value_sign", "papg.py", "return primal_objective(ybar, gamma, y, xi) - float(np.sum(lam0 * s))",
     "return primal_objective(ybar, gamma, y, xi) + float(np.sum(lam0 * s))"),
    ("fista_t", "papg.py", "t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0",
     "t_next = (1.0 + math.sqrt(1.0 + 4.0 * t)) / 2.0"),
    ("fista_beta", "papg.py", "beta = (t - 1.0) / t_next if momentum else 0.0",
     "beta = (t - 1.0) / t if momentum else 0.0"),
    ("step_sign", "papg.py", "lam = np.maximum(0.0, lam_tilde - s / L)", "lam = np.maximum(0.0, lam_tilde + s / L)"),
    ("extrapolation_sign", "papg.py", "lam_tilde = lam + beta * (lam - lam_prev)",
     "lam_tilde = lam - beta * (lam - lam_prev)"),
    ("adaptive_exponent", "papg.py", "s_try = s_k * upsilon ** (ell - 1)", "s_try = s_k * upsilon ** ell"),
    ("adaptive_check_direction", "papg.py", "if curv <= s_try * float(np.sum(dlt * dlt)) * (1.0 + 1e-12):",
     "if curv >= s_try * float(np.sum(dlt * dlt)) * (1.0 + 1e-12):"),
    ("restart_test_sign", "papg.py", "if restart and float(np.sum(dlt * (lam - lam_prev))) < 0.0:",
     "if restart and float(np.sum(dlt * (lam - lam_prev))) > 0.0:"),
    ("kkt_min_max", "papg.py", "nat = float(np.max(np.abs(np.minimum(lam, s)[off])))",
     "nat = float(np.max(np.abs(np.maximum(lam, s)[off])))"),
    ("kkt_scale", "papg.py", "sy = max(1.0, float(ybar.max() - ybar.min()))", "sy = 1.0"),
    ("complementarity_sum", "papg.py", "comp = float(np.sum(lam * s))", "comp = float(np.sum(lam * np.abs(s)))"),
    ("power_quotient", "papg.py", "new = float(np.sum(z ** 2))", "new = float(np.sum(np.abs(z)))"),
    ("lipschitz_scale", "papg.py", "return est / gamma, est, it", "return est * gamma, est, it"),
    ("max_affine_repair", "papg.py", "y_rep = y - colmin", "y_rep = y + colmin"),
    ("own_slope_repair_axis", "papg.py", "cand = np.maximum(c, (c[:, None] - off).max(axis=0))",
     "cand = np.maximum(c, (c[:, None] - off).max(axis=1))"),
    ("continuation_weight", "continuation.py", "g_t = kappa_gamma * eps_t", "g_t = kappa_delta * eps_t"),
    ("exact_subgradient_sign", "exact.py", "l * n:(l + 1) * n] = -T @ x", "l * n:(l + 1) * n] = T @ x"),
    ("exact_t_block", "exact.py", "T[:, l] = -1.0", "T[:, l] = 1.0"),
    # the K-block partial dualization (its own pins, test_oracle_blocks.py)
    ("blocks_step_mask_dropped", "blocks.py", "th = np.maximum(0.0, th_tilde - s / L) * mask",
     "th = np.maximum(0.0, th_tilde - s / L)"),
    ("blocks_projection_rhs_sign", "blocks.py", "b = np.concatenate([-y0, -math.sqrt(gamma) * xi0.reshape(-1)])",
     "b = np.concatenate([y0, -math.sqrt(gamma) * xi0.reshape(-1)])"),
    ("blocks_projection_xi_scale", "blocks.py", "xi = xi0 + (A2.T @ mu / gamma).reshape(p, n)",
     "xi = xi0 + (A2.T @ mu * gamma).reshape(p, n)"),
    ("blocks_sigma_unmasked", "blocks.py", "z = pair_residual(x, vy, vxi) * mask", "z = pair_residual(x, vy, vxi)"),
    ("blocks_partition_interleaved", "blocks.py", "return np.arange(N) // p", "return np.arange(N) % p"),
]
BLOCK_PINS = ["test_oracle_blocks.py"]


def _copy_tree(dst, mutation=None):
    """A minimal repository copy: the oracle (possibly mutated), the workload generators, the pin
    tests and their conftest."""
    os.makedirs(os.path.join(dst, "tests"))
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(dst, "oracle"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    pkg = os.path.join(dst, "paper_1608_02227_amd")
    os.makedirs(pkg)
    for f in ("__init__.py", "workloads.py"):
        shutil.copy(os.path.join(ROOT, "paper_1608_02227_amd", f), pkg)
    for f in ["conftest.py", *PIN_TESTS, *BLOCK_PINS]:
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(dst, "tests"))
    if mutation is not None:
        _, fname, old, new = mutation
        path = os.path.join(dst, "oracle", fname)
        src = open(path).read()
        assert src.count(old) == 1, f"the correct text must appear once in {fname}: {old}"
        with open(path, "w") as f:
            f.write(src.replace(old, new))


def _run_pins(dst, pins):
    env = dict(os.environ)
    env["PYTHONPATH"] = dst
    env["OPENBLAS_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not slow",
                        *[os.path.join("tests", t) for t in pins]], cwd=dst, env=env,
                       capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """Runs the pins on the unmodified copy and on every mutated copy, six subprocesses at a time
    (each is independent; together they take about a minute instead of three and a half)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(job):
        m, dst = job
        _copy_tree(dst, m)
        # a planted mistake in the block oracle meets the block pins; the rest the method's pins
        pins = PIN_TESTS + BLOCK_PINS if m is None else (BLOCK_PINS if m[1] == "blocks.py" else PIN_TESTS)
        return _run_pins(dst, pins)
    cases = [None] + MUTATIONS
    # the temporary folders are made here, one at a time (pytest's numbered folders are not safe to
    # create from several threads at once)
    jobs = [(m, str(tmp_path_factory.mktemp(m[0] if m else "unmodified") / "repo")) for m in cases]
    with ThreadPoolExecutor(max_workers=6) as ex:
        res = list(ex.map(one, jobs))
    return {("unmodified" if m is None else m[0]): r for m, r in zip(cases, res)}


def test_unmodified_copy_passes(outcomes):
    code, out = outcomes["unmodified"]
    assert code == 0, out


@pytest.mark.parametrize("mutation", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_the_planted_mistake(outcomes, mutation):
    code, out = outcomes[mutation[0]]
    assert code == 1, f"no pin caught {mutation[0]}:\n{out}"

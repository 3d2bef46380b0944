"""CPU-side checks of the C-ABI library: it loads, exports every declared entry point, and its
host-side argument validation rejects bad input without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cr_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["cr_fit", "cr_fit_device", "cr_solver_create", "cr_solver_iterate", "cr_solver_lipschitz",
                 "cr_solver_report", "cr_op_residual", "cr_op_adjoint", "cr_ctx_create", "cr_submit", "cr_wait"]:
        assert must in names


def test_library_exports_every_declared_symbol(cr):
    lib = cr.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_and_defaults(cr):
    assert cr.strerror(0) == "ok"
    assert "invalid" in cr.strerror(cr.CR_EINVAL)
    o = cr.CROptions()
    cr.load().cr_default_options(C.byref(o))
    assert o.check_every == 50 and o.momentum == 1 and o.precision == 0 and o.power_max_iters == 300
    assert o.step_rule == 1 and o.upsilon == 2.0 and o.restart == 1


@pytest.mark.parametrize("N,n,delta,tol", [(0, 2, 1e-3, 1e-4), (10, 0, 1e-3, 1e-4), (10, 2, 0.0, 1e-4),
                                            (10, 2, -1.0, 1e-4), (10, 2, 1e-3, 0.0), (10, 2, float("nan"), 1e-4),
                                            (10, 64, 1e-3, 1e-4)])
def test_fit_rejects_bad_arguments_on_host(cr, N, n, delta, tol):
    lib = cr.load()
    x = np.zeros((max(N, 1), max(n, 1)))
    yb = np.zeros(max(N, 1))
    y = np.zeros(max(N, 1))
    xi = np.zeros((max(N, 1), max(n, 1)))
    opt = cr.Options().to_c()
    rc = lib.cr_fit(N, n, cr._ptr(x), cr._ptr(yb), delta, tol, C.byref(opt), cr._ptr(y), cr._ptr(xi), None, None)
    assert rc == cr.CR_EINVAL


def test_fit_rejects_bad_options_on_host(cr):
    lib = cr.load()
    x = np.zeros((4, 2))
    yb = np.zeros(4)
    y = np.zeros(4)
    xi = np.zeros((4, 2))
    for field, value in [("check_every", 0), ("precision", 7), ("L", -1.0), ("power_max_iters", 0),
                         ("step_rule", 2), ("upsilon", 1.0), ("upsilon", float("inf")), ("restart", 2),
                         ("power_rtol", -1.0), ("stop_rule", 2), ("check_rule", 2), ("check_rule", -1),
                         ("center", 2), ("center", -1), ("keep_lambda", 2),
                         ("block_size", 101), ("block_size", -1), ("block_size", 2)]:
        opt = cr.Options().to_c()
        setattr(opt, field, value)
        rc = lib.cr_fit(4, 2, cr._ptr(x), cr._ptr(yb), 1e-3, 1e-4, C.byref(opt), cr._ptr(y), cr._ptr(xi), None, None)
        assert rc == cr.CR_EINVAL, field


def test_binding_struct_layout_matches_header(cr, tmp_path):
    # Compile a probe against cr.h with the host C compiler and compare sizes and offsets.
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [("cr_options", cr.CROptions), ("cr_report", cr.CRReport), ("cr_cont_params", cr.CRContParams),
               ("cr_cont_step", cr.CRContStep)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cr.h"', "int main(void){"]
    lines += [f'printf("%zu\\n", sizeof({name}));' for name, _ in structs]
    for name, py in structs:
        lines += [f'printf("%zu\\n", offsetof({name}, {f}));' for f, _ in py._fields_]
    lines += ["return 0;}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert [int(v) for v in out[:len(structs)]] == [C.sizeof(py) for _, py in structs]
    offs = [int(v) for v in out[len(structs):]]
    py = [getattr(p, f).offset for _, p in structs for f, _ in p._fields_]
    assert offs == py


@pytest.mark.parametrize("field,value", [("eps0", 0.0), ("beta", 1.0), ("kappa_gamma", -1.0), ("kappa_delta", 0.0),
                                         ("T", 0)])
def test_continuation_rejects_bad_parameters_on_host(cr, field, value):
    lib = cr.load()
    x = np.zeros((4, 2))
    yb = np.zeros(4)
    y = np.zeros(4)
    xi = np.zeros((4, 2))
    cp = cr.CRContParams(1.0, 2.0, 1.0, 1.0, 3, 0)
    setattr(cp, field, value)
    opt = cr.Options().to_c()
    rc = lib.cr_fit_continuation(4, 2, cr._ptr(x), cr._ptr(yb), C.byref(cp), C.byref(opt), cr._ptr(y), cr._ptr(xi),
                                 None, None, None)
    assert rc == cr.CR_EINVAL


def test_no_device_fails_loudly(cr):
    """Without a visible GPU a well-formed fit is refused with CR_EDEVICE: there is no CPU path."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    lib = cr.load()
    assert lib.cr_device_check(0) == cr.CR_EDEVICE
    x = np.random.default_rng(0).uniform(-1.0, 1.0, size=(8, 2))
    yb = (x ** 2).sum(axis=1)
    y = np.zeros(8)
    xi = np.zeros((8, 2))
    opt = cr.Options().to_c()
    rc = lib.cr_fit(8, 2, cr._ptr(x), cr._ptr(yb), 1e-3, 1e-4, C.byref(opt), cr._ptr(y), cr._ptr(xi), None, None)
    assert rc == cr.CR_EDEVICE
    with pytest.raises(cr.CRError) as e:
        cr.fit(x, yb, 1e-3, 1e-4)
    assert e.value.code == cr.CR_EDEVICE


def test_noalloc_sizes_on_host(cr):
    """The allocation-free fit's scratch and what a fit needs of it (host arithmetic, no GPU): the
    need grows with N, stays within the scratch at the stated limits (N = 2,600 mixed, 1,700 FP64
    with the adaptive step, n = 40) and exceeds it beyond; N = 1 needs nothing."""
    total = cr.noalloc_scratch_bytes()
    assert total == 128 << 20
    mixed = cr.Options(precision="mixed_fp32")
    fp64 = cr.Options(precision="fp64")
    assert cr.noalloc_required_bytes(1, 3, mixed) == 0
    sizes = [cr.noalloc_required_bytes(N, 40, mixed) for N in (100, 1000, 2000, 2600)]
    assert all(0 < a < b for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] <= total < cr.noalloc_required_bytes(2800, 40, mixed)
    assert cr.noalloc_required_bytes(1700, 40, fp64) <= total < cr.noalloc_required_bytes(1800, 40, fp64)
    # every piece is 256-byte aligned, so the total is a multiple of 256 and at least the multipliers
    assert all(s % 256 == 0 for s in sizes)
    assert sizes[2] >= 2048 * 2048 * 12
    assert cr.noalloc_required_bytes(10, 64, mixed) == 0      # n + 1 > 64 is invalid
    # a warm start is staged as a dense N x N FP64 matrix behind the state
    lib = cr.load()
    for opt in (fp64, mixed):
        co = opt.to_c()
        plain = lib.cr_noalloc_required_bytes(1000, 40, C.byref(co))
        co.lambda0 = 8     # never read by the sizing
        assert lib.cr_noalloc_required_bytes(1000, 40, C.byref(co)) == plain + 1000 * 1000 * 8


def test_noalloc_without_device_fails_loudly(cr):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    lib = cr.load()
    x = np.random.default_rng(0).uniform(-1.0, 1.0, size=(8, 2))
    yb = (x ** 2).sum(axis=1)
    y = np.zeros(8)
    xi = np.zeros((8, 2))
    opt = cr.Options().to_c()
    rc = lib.cr_fit_device_noalloc(8, 2, cr._ptr(x), cr._ptr(yb), 1e-3, 1e-4, C.byref(opt), cr._ptr(y), cr._ptr(xi),
                                   None, None)
    assert rc == cr.CR_EDEVICE

"""The pins catch plausible mistakes: each test below compiles a copy of the
oracle with one mistake planted (on the CPU, in a temporary directory) and checks
that at least one pin fails on it, while the unmodified oracle passes them all."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W
from jacobi_ref import cyclic_jacobi

SRC = os.path.join(os.path.dirname(oracle.__file__), "ipt_oracle.c")

MUTANTS = {
    "drop_z_d_term": ("g[j] * (z[j] * d - y[j])", "g[j] * (0.0 * z[j] * d - y[j])"),
    "flip_update_sign": ("g[j] * (z[j] * d - y[j])", "g[j] * (y[j] - z[j] * d)"),
    "wrong_diag_index": ("const double d = y[i];", "const double d = y[(i + 1) % n];"),
    "transposed_gaps": ("1.0 / (theta[j] - theta[i])", "1.0 / (theta[i] - theta[j])"),
    "transposed_delta": ("acc += row[l] * z[l];", "acc += delta[l * lda + j] * z[l];"),
    "lambda_without_theta": ("*lambda = theta[i] + d;\n            *status = OR_CONVERGED;",
                             "*lambda = d;\n            *status = OR_CONVERGED;"),
    "step_not_relative": ("s = sqrt(num) / sqrt(den);", "s = sqrt(num);"),
    # IPT-ACX (Alg. 3)
    "acx_sigma_unsquared": ("fabs(dot) / nrm : 1.0", "fabs(dot) / sqrt(nrm) : 1.0"),
    "acx_orders_swapped": ("(cycle % 2 == 0) ? 3 : 2", "(cycle % 2 == 0) ? 2 : 3"),
    "acx_order2_without_z": ("z[j] = (z[j] + 2.0 * sg * d1) + (sg * sg) * d2;",
                             "z[j] = (2.0 * sg * d1) + (sg * sg) * d2;"),
    "acx_order3_binomial": ("3.0 * (sg * sg) * d2) + (sg * sg * sg) * d3", "(sg * sg) * d2) + (sg * sg * sg) * d3"),
    "acx_second_difference": ("const double d2 = (f2[j] - 2.0 * f1[j]) + z[j];\n            if (p == 2) {\n                dot",
                              "const double d2 = (f2[j] - f1[j]) + z[j];\n            if (p == 2) {\n                dot"),
}


def _pins_pass():
    """A quick subset of the pins; True when all hold."""
    ok = True
    # 2x2 per-iterate closed form (Sec. 4.3)
    eps = 0.3
    th, de = W.two_by_two(eps)
    x, fx = 0.0, [0.0]
    for _ in range(10):
        x = eps * (x * x - 1.0)
        fx.append(x)
    ok &= bool(np.allclose(oracle.ipt_trace(th, de, 0, 10)[:, 1], fx, rtol=0, atol=1e-14))
    # general 2x2 closed form (App. D)
    a, b, c, d = 0.5, 0.05, -0.4, 1.7
    th, de = W.general_two_by_two(a, b, c, d)
    r = oracle.ipt_dense(th, de, tol=1e-15, max_iter=2000)
    s = d - a
    den = s + math.copysign(math.sqrt(s * s + 4 * b * c), s)
    ok &= bool(abs(r.z[1, 0] + 2 * c / den) < 1e-13 and abs(r.z[0, 1] - 2 * b / den) < 1e-13)
    ok &= bool(abs(r.lam[0] - (a + b * (-2 * c / den))) < 1e-13)
    # tiny symmetric case vs Jacobi, with a large theta offset so the stopping test
    # and the read-out both matter
    th, de = W.dense_sym_gaussian(6, 0.2, 4)
    th = th + 10.0
    ev, vec = cyclic_jacobi(np.diag(th) + de)
    r = oracle.ipt_dense(th, de, tol=1e-13, max_iter=500)
    for col in range(6):
        m = int(np.argmax(np.abs(vec[col, :])))
        ok &= bool(np.max(np.abs(r.z[:, col] - vec[:, m] / vec[col, m])) < 1e-11)
        ok &= bool(abs(r.lam[col] - ev[m]) < 1e-11)
    # the stopping test is the relative step |f(z) - z| / |z| (Alg. 1 loop test);
    # a 2x2 whose fixed point has a large entry (|z| ~ 5) separates it from |f(z) - z|
    th, de = W.general_two_by_two(0.0, 0.001, 5.0, 1.0)
    r = oracle.ipt_dense(th, de, idx=np.array([0], np.int32), tol=1e-6, max_iter=500)
    t = int(r.sweeps[0])
    tr = oracle.ipt_trace(th, de, 0, t)
    want = np.linalg.norm(tr[t] - tr[t - 1]) / np.linalg.norm(tr[t - 1])
    ok &= bool(r.status[0] == oracle.CONVERGED and abs(r.step[0] - want) <= 1e-12 * want)
    # IPT-ACX on affine maps (closed forms of the extrapolation, see test_oracle_acx)
    from test_oracle_acx import affine_case
    th, de, zs = affine_case(0.95)
    r = oracle.ipt_dense(th, de, idx=np.array([0], np.int32), tol=1e-10, max_iter=100, accel="acx")
    ok &= bool(r.status[0] == oracle.CONVERGED and r.sweeps[0] == 4 and np.max(np.abs(r.z[:, 0] - zs)) < 2e-11)
    th, de, zs = affine_case(1.5)
    e0 = 1e-3 * np.random.default_rng(1).standard_normal(6)
    e0[0] = 0.0
    for mi, fac in ((4, 12.0), (6, 48.0)):
        r = oracle.ipt_dense(th, de, idx=np.array([0], np.int32), z0=(zs + e0).reshape(6, 1), tol=1e-12,
                             max_iter=mi, accel="acx")
        ok &= bool(r.sweeps[0] == mi and np.max(np.abs(r.z[:, 0] - (zs + fac * e0))) < 1e-12)
    return ok


# Non-autonomous continuation: mistakes caught by the pins of test_oracle_cont
CONT_MUTANTS = {
    "cont_schedule_from_zero": ("const double scale = 1.0 - apow;", "const double scale = 1.0 - apow / alpha;"),
    "cont_certify_while_scaled": ("if (scale == 1.0 && s <= tol) {", "if (s <= tol) {"),
    "cont_unscaled_d": ("for (int64_t j = 0; j < n; ++j) y[j] *= scale; /* (scale Delta) z */\n        d = y[i];",
                        "d = y[i];\n        for (int64_t j = 0; j < n; ++j) y[j] *= scale; /* (scale Delta) z */"),
    "cont_unscaled_map": ("for (int64_t j = 0; j < n; ++j) y[j] *= scale; /* (scale Delta) z */",
                          "/* scale dropped */"),
}


# Complex field: mistakes caught by the pins of test_oracle_complex
COMPLEX_MUTANTS = {
    "complex_product_conjugated": ("cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};",
                                   "cplx r = {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};"),
    "complex_inverse_sign": ("        r.re = 1.0 / den;\n        r.im = -q / den;", "        r.re = 1.0 / den;\n        r.im = q / den;"),
    "complex_dropped_imaginary_product": ("acc = c_add(acc, c_mul(row[l], z[l]));",
                                          "acc = c_add(acc, (cplx){row[l].re * z[l].re, row[l].im * z[l].im});"),
}


def test_unmodified_oracle_passes():
    assert _pins_pass()
    from test_oracle_cont import cont_pins_pass
    assert cont_pins_pass()
    from test_oracle_complex import complex_pins_pass
    assert complex_pins_pass()


@pytest.mark.parametrize("name", sorted(COMPLEX_MUTANTS))
def test_planted_complex_mistake_is_caught(tmp_path, name):
    from test_oracle_complex import complex_pins_pass
    so = _build_mutant(tmp_path, *COMPLEX_MUTANTS[name])
    prev = oracle.swap_library(so)
    try:
        assert not complex_pins_pass(), "mistake %s went unnoticed" % name
    finally:
        oracle.swap_library(prev)


def _build_mutant(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, old
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", so,
                           str(path), "-lm"])
    return so


@pytest.mark.parametrize("name", sorted(CONT_MUTANTS))
def test_planted_continuation_mistake_is_caught(tmp_path, name):
    from test_oracle_cont import cont_pins_pass
    so = _build_mutant(tmp_path, *CONT_MUTANTS[name])
    prev = oracle.swap_library(so)
    try:
        assert not cont_pins_pass(), "mistake %s went unnoticed" % name
    finally:
        oracle.swap_library(prev)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new)
    path = tmp_path / "mut.c"
    path.write_text(mutated)
    so = str(tmp_path / "libmut.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", so,
                           str(path), "-lm"])
    prev = oracle.swap_library(so)
    try:
        assert not _pins_pass(), "mistake %s went unnoticed" % name
    finally:
        oracle.swap_library(prev)

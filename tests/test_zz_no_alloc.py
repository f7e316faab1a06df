"""The no-allocation dense entry point (ipt_solve_dense_noalloc) against the
allocating one (ipt_solve_dense), through the C ABI: the same kernels on a fixed
per-device workspace must give the same bits.  Two calls in a row, the second on a
smaller input (the fixed workspace keeps the first call's contents), then a solve too
large for the fixed workspace, which must be refused."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev, host, say, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipt():
    from paper_2012_14702_amd import ipt as mod
    mod.load_library()
    dev()
    return mod


def _same(a, b):
    np.testing.assert_array_equal(a.z, b.z)
    np.testing.assert_array_equal(a.lam, b.lam)
    np.testing.assert_array_equal(a.status, b.status)
    for key in ("sweeps", "converged", "diverged", "not_converged", "matvecs", "max_step", "norm1", "max_resid",
                "sweep_prec", "sweep_active", "sweep_max_step"):
        assert a.info[key] == b.info[key], key


def _pair(ipt, th, de, idx=None, z0=None, **kw):
    args = dict(idx=None if idx is None else t(idx.astype(np.int32)), z0=None if z0 is None else t(z0), **kw)
    a = host(ipt.ipt_solve_dense(t(th), t(de), **args))
    b = host(ipt.ipt_solve_dense_noalloc(t(th), t(de), **args))
    return a, b


def test_noalloc_matches_allocating_entry_point(ipt):
    # call 1: full spectrum n = 1024 on the ladder (the largest full solve the fixed
    # workspace holds), cold start
    say("noalloc call 1: dense n=1024 ladder full spectrum")
    th, de = W.dense_sym_gaussian(1024, 0.02, 21)
    a, b = _pair(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER)
    _same(a, b)
    assert np.all(b.status == 0)
    # call 2: smaller, ragged (n = 300, 37 scattered columns), FP64, warm start from a
    # partial solve
    say("noalloc call 2: dense n=300 k=37 fp64 warm start")
    th2, de2 = W.dense_sym_gaussian(300, 0.03, 22)
    idx = np.random.default_rng(5).permutation(300)[:37].astype(np.int32)
    part = host(ipt.ipt_solve_dense(t(th2), t(de2), idx=t(idx), tol=1e-12, max_iter=2))
    a, b = _pair(ipt, th2, de2, idx=idx, z0=part.z, tol=1e-12, precision=ipt.PREC_FP64)
    _same(a, b)
    assert np.all(b.status == 0)
    # call 3: the smaller input again, cold, IPT-ACX (two more iterate slots)
    say("noalloc call 3: dense n=300 k=37 acx")
    a, b = _pair(ipt, th2, de2, idx=idx, tol=1e-12, precision=ipt.PREC_FP64, flags=ipt.FLAG_ACX)
    _same(a, b)


def test_noalloc_refuses_what_does_not_fit(ipt):
    say("noalloc refusals (host-side checks only)")
    th, de = W.dense_sym_gaussian(4096, 0.01, 0)
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_solve_dense_noalloc(t(th), t(de), tol=1e-10)
    assert e.value.status == ipt.IPT_EINVAL
    th, de = W.dense_sym_gaussian(64, 0.01, 0)
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_solve_dense_noalloc(t(th), t(de), tol=1e-10, homotopy_q=2)
    assert e.value.status == ipt.IPT_EINVAL
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_solve_dense_noalloc(t(th), t(de), tol=1e-10, flags=ipt.FLAG_TIME_KERNELS)
    assert e.value.status == ipt.IPT_EINVAL

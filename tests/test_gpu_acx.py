"""GPU parity of IPT-ACX (IPT_FLAG_ACX: alternating cyclic extrapolation, Alg. 3)
on the dense and sparse paths against the IPT-ACX oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, host, say, t
from parity import check
from test_oracle_acx import affine_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipt():
    from paper_2012_14702_amd import ipt as mod
    mod.load_library()
    dev()
    return mod


def _dense(ipt, theta, delta, idx=None, z0=None, **kw):
    r = ipt.ipt_solve_dense(t(theta), t(delta), idx=None if idx is None else t(idx.astype(np.int32)),
                            z0=None if z0 is None else t(z0), flags=ipt.FLAG_ACX, **kw)
    return host(r)


def _csr(ipt, th, rp, col, val, idx, **kw):
    r = ipt.ipt_solve_csr(t(th), t(rp), t(col), t(val), t(np.asarray(idx, dtype=np.int32)), flags=ipt.FLAG_ACX, **kw)
    return host(r)


@pytest.mark.parametrize("n,eps,seed", [(300, 0.02, 0), (256, 0.01, 1), (129, 0.04, 2)])
def test_acx_dense_full_spectrum(ipt, n, eps, seed):
    """Full spectra (ragged n, several column tiles) match the ACX oracle column by
    column; sweep counts (applications of F) agree to within one cycle."""
    say("acx dense n=%d eps=%g" % (n, eps))
    th, de = W.dense_sym_gaussian(n, eps, seed)
    g = _dense(ipt, th, de, tol=1e-10)
    ref = oracle.ipt_dense(th, de, tol=1e-10, accel="acx")
    out = check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-10, gpu_sweeps=g.sweeps, sweep_slack=3,
                max_iter=100)
    assert out["compared"] >= n - 2


def test_acx_dense_subset_warm_start(ipt):
    """Requested subset with a warm start (the base iterate of the first cycle)."""
    say("acx dense subset warm")
    th, de = W.dense_sym_gaussian(300, 0.03, 4)
    idx = np.random.default_rng(4).permutation(300)[:37].astype(np.int32)
    part = oracle.ipt_dense(th, de, idx=idx, tol=1e-12, max_iter=1)
    g = _dense(ipt, th, de, idx=idx, z0=part.z, tol=1e-12)
    ref = oracle.ipt_dense(th, de, idx=idx, z0=part.z, tol=1e-12, accel="acx")
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12, gpu_sweeps=g.sweeps, sweep_slack=3, max_iter=100)


@pytest.mark.parametrize("max_iter,factor,used", [(4, 12.0, 4), (5, 12.0, 4), (6, 48.0, 6), (9, 384.0, 9)])
def test_acx_cycle_closed_forms(ipt, max_iter, factor, used):
    """The repelling affine map of the oracle pins (r = 1.5): cycles of order 3 and 2
    multiply the error by 8 and 4; the budget rule stops at the same application."""
    say("acx affine max_iter=%d" % max_iter)
    th, de, zs = affine_case(1.5)
    e0 = 1e-3 * np.random.default_rng(1).standard_normal(6)
    e0[0] = 0.0
    g = _dense(ipt, th, de, idx=np.array([0], np.int32), z0=(zs + e0).reshape(6, 1), tol=1e-12, max_iter=max_iter)
    assert g.status[0] == 1 and g.sweeps[0] == used
    np.testing.assert_allclose(g.z[:, 0], zs + factor * e0, rtol=0, atol=1e-12)
    th, de, zs = affine_case(0.95)
    g = _dense(ipt, th, de, idx=np.array([0], np.int32), tol=1e-10)
    assert g.status[0] == 0 and g.sweeps[0] == 4
    assert np.max(np.abs(g.z[:, 0] - zs)) < 2e-11


@pytest.mark.parametrize("off", [0.5, 0.75, 1.0])
def test_acx_morgan(ipt, off):
    """Morgan's tridiagonal matrix (Sec. 6.1): the lowest 3 eigenpairs with ACX on the
    sparse path, including off-diagonals where plain IPT fails."""
    say("acx csr morgan off=%g" % off)
    th, rp, col, val = W.morgan_tridiagonal(5000, off)
    idx = np.array([0, 1, 2], np.int32)
    g = _csr(ipt, th, rp, col, val, idx, tol=1e-12, max_iter=2000)
    ref = oracle.ipt_csr(th, rp, col, val, idx, tol=1e-12, max_iter=2000, accel="acx")
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, csr=(rp, col, val)), 1e-12, gpu_sweeps=g.sweeps,
          sweep_slack=5, max_iter=2000)
    assert g.status[0] == 0


def test_acx_sparse_shapes(ipt):
    """Random sparse near-diagonal matrix, ragged k."""
    say("acx csr n=3000 k=37")
    th, rp, col, val = W.sparse_sym_uniform(3000, pairs_per_row=3, amp=0.05, seed=3)
    idx = np.random.default_rng(3).permutation(3000)[:37].astype(np.int32)
    g = _csr(ipt, th, rp, col, val, idx, tol=1e-12)
    ref = oracle.ipt_csr(th, rp, col, val, idx, tol=1e-12, accel="acx")
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, csr=(rp, col, val)), 1e-12, gpu_sweeps=g.sweeps,
          sweep_slack=3, max_iter=100)


def test_acx_requires_fp64(ipt):
    th, de = W.dense_sym_gaussian(16, 0.01, 0)
    with pytest.raises(ipt.IPTError) as e:
        _dense(ipt, th, de, precision=ipt.PREC_LADDER)
    assert e.value.status == ipt.IPT_EINVAL

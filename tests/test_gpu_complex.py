"""GPU parity of the dense solve over C^n (C ABI ipt_solve_dense_z) against the
complex oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, host, say, t
from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipt():
    from paper_2012_14702_amd import ipt as mod
    mod.load_library()
    dev()
    return mod


def _solve(ipt, theta, delta, idx=None, z0=None, **kw):
    r = ipt.ipt_solve_dense_z(t(np.ascontiguousarray(theta, np.complex128)), t(np.ascontiguousarray(delta, np.complex128)),
                              idx=None if idx is None else t(idx.astype(np.int32)),
                              z0=None if z0 is None else t(np.ascontiguousarray(z0, np.complex128)), **kw)
    return host(r)


def _norm1(th, de):
    return float(np.max(np.sum(np.abs(np.diag(th) + de), axis=0)))


def _hermitian(n, eps, seed):
    rng = np.random.default_rng(seed)
    a = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    return np.arange(1, n + 1).astype(np.complex128), eps * (a + a.conj().T) / 2


def _general(n, eps, seed):
    rng = np.random.default_rng(seed)
    de = eps * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    return np.arange(1, n + 1) * (1.0 + 0.3j), de


@pytest.mark.parametrize("n,kind,eps", [(300, "hermitian", 0.02), (129, "hermitian", 0.05), (257, "general", 0.03),
                                        (64, "general", 0.1)])
def test_full_spectrum_parity(ipt, n, kind, eps):
    """Full spectra over several row and column tiles (ragged n); every column
    against the complex oracle; the norm against its definition."""
    say("complex n=%d %s eps=%g" % (n, kind, eps))
    th, de = (_hermitian if kind == "hermitian" else _general)(n, eps, n)
    g = _solve(ipt, th, de, tol=1e-12)
    ref = oracle.ipt_dense_z(th, de, tol=1e-12)
    out = check(g.z, g.lam, g.status, ref, _norm1(th, de), 1e-12, gpu_sweeps=g.sweeps)
    assert out["compared"] == n
    assert np.all(g.z[np.arange(n), np.arange(n)] == 1.0)
    assert abs(g.info["norm1"] - _norm1(th, de)) <= 1e-13 * _norm1(th, de)


def test_requested_columns_and_warm_start(ipt):
    """k = 40 scattered columns of a general complex matrix, cold and then warm from
    a two-sweep partial solve (both sides start from the same iterate)."""
    say("complex n=500 k=40 warm")
    th, de = _general(500, 0.04, 9)
    idx = np.sort(np.random.default_rng(2).choice(500, 40, replace=False)).astype(np.int32)
    g = _solve(ipt, th, de, idx=idx, tol=1e-12)
    ref = oracle.ipt_dense_z(th, de, idx=idx, tol=1e-12)
    check(g.z, g.lam, g.status, ref, _norm1(th, de), 1e-12, gpu_sweeps=g.sweeps)
    part = _solve(ipt, th, de, idx=idx, tol=1e-12, max_iter=2)
    assert np.all(part.status == ipt.NOT_CONVERGED)
    w = _solve(ipt, th, de, idx=idx, z0=part.z, tol=1e-12)
    refw = oracle.ipt_dense_z(th, de, idx=idx, z0=part.z, tol=1e-12)
    check(w.z, w.lam, w.status, refw, _norm1(th, de), 1e-12, gpu_sweeps=w.sweeps)


def test_real_input_matches_real_path(ipt):
    """Real input through the complex solve: the same eigenpairs as the real solve."""
    say("complex path on real input n=256")
    th, de = W.dense_sym_gaussian(256, 0.02, 4)
    rz = _solve(ipt, th.astype(complex), de.astype(complex), tol=1e-12)
    rr = host(ipt.ipt_solve_dense(t(th), t(de), tol=1e-12))
    np.testing.assert_array_equal(rz.status, rr.status)
    assert np.max(np.abs(rz.z.imag)) == 0.0 and np.max(np.abs(rz.lam.imag)) == 0.0
    assert np.max(np.abs(rz.z.real - rr.z)) < 1e-13 and np.max(np.abs(rz.lam.real - rr.lam)) < 1e-13


def test_small_and_two_by_two(ipt):
    """n = 1 and the complex 2 x 2 example (iterates f^t(0), f(x) = eps (x^2 - 1))."""
    say("complex n=1, 2x2")
    g = _solve(ipt, np.array([2.0 + 1.0j]), np.array([[0.5 - 0.25j]]), tol=1e-12)
    assert g.status[0] == ipt.CONVERGED and g.z[0, 0] == 1.0 and abs(g.lam[0] - (2.5 + 0.75j)) < 1e-15
    eps = 0.3 + 0.2j
    th = np.array([0.0, 1.0], np.complex128)
    de = np.array([[0.0, eps], [eps, 0.0]], np.complex128)
    x = 0.0
    for m in range(1, 6):
        x = eps * (x * x - 1.0)
        r = _solve(ipt, th, de, tol=0.0, max_iter=m)
        assert abs(r.z[1, 0] - x) < 1e-15 and abs(r.z[0, 1] + x) < 1e-15


@pytest.mark.parametrize("n", [2048, 4096])
def test_large_sampled(ipt, n):
    """Hermitian full spectra on the GPU (n = 4096 is the benchmarked size); sampled
    columns by the oracle."""
    say("complex n=%d hermitian sampled" % n)
    th, de = _hermitian(n, 0.01, 1)
    g = _solve(ipt, th, de, tol=1e-10)
    assert np.all(g.status == 0)
    cols = np.unique(np.concatenate([[0, 1, 63, 64, n // 2 - 1, n - 1], np.random.default_rng(3).integers(0, n, 10)]))
    ref = oracle.ipt_dense_z(th, de, idx=cols.astype(np.int32), tol=1e-10, resid=False)
    check(g.z[:, cols], g.lam[cols], g.status[cols], ref, _norm1(th, de), 1e-10)


def test_complex_errors(ipt):
    th, de = _hermitian(16, 0.01, 0)
    for kw in (dict(precision=ipt.PREC_LADDER), dict(flags=ipt.FLAG_ACX), dict(cont_alpha=0.5)):
        with pytest.raises(ipt.IPTError) as e:
            _solve(ipt, th, de, **kw)
        assert e.value.status == ipt.IPT_EINVAL, kw
    th2 = th.copy()
    th2[5] = th2[3]
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, th2, de, idx=np.array([3], np.int32))
    assert e.value.status == ipt.IPT_EDEGENERATE
    th3 = th.copy()
    th3[5] = th3[3] + 1e-3j  # equal real parts only: distinct
    g = _solve(ipt, th3, de, idx=np.array([3, 5], np.int32), tol=1e-10)
    assert g.status.shape == (2,)


def test_complex_unsorted_columns_strided_warm_start(ipt):
    """Unsorted requested columns (k = 1 and k = 7), a warm start with a row stride
    larger than k, and |M|_1 skipped (IPT_FLAG_NO_NORM)."""
    say("complex n=130 unsorted idx, strided z0")
    th, de = _general(130, 0.05, 21)
    for idx in (np.array([77], np.int32), np.array([129, 3, 64, 0, 100, 65, 1], np.int32)):
        g = _solve(ipt, th, de, idx=idx, tol=1e-12)
        ref = oracle.ipt_dense_z(th, de, idx=idx, tol=1e-12)
        check(g.z, g.lam, g.status, ref, _norm1(th, de), 1e-12, gpu_sweeps=g.sweeps)
    idx = np.array([129, 3, 64, 0, 100, 65, 1], np.int32)
    part = _solve(ipt, th, de, idx=idx, tol=1e-12, max_iter=2)
    wide = np.zeros((130, 16), np.complex128)
    wide[:, :7] = part.z
    zt = t(wide)[:, :7]  # row stride 16 > k = 7
    r = host(ipt.ipt_solve_dense_z(t(th.astype(np.complex128)), t(de), idx=t(idx), z0=zt, tol=1e-12,
                                   flags=ipt.FLAG_NO_NORM))
    ref = oracle.ipt_dense_z(th, de, idx=idx, z0=part.z, tol=1e-12)
    check(r.z, r.lam, r.status, ref, _norm1(th, de), 1e-12, gpu_sweeps=r.sweeps)

"""GPU parity of the sparse IPT path (C ABI ipt_solve_csr) against the FP64 oracle."""
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


def _solve(ipt, th, rp, col, val, idx, z0=None, **kw):
    r = ipt.ipt_solve_csr(t(th), t(rp), t(col), t(val), t(np.asarray(idx, dtype=np.int32)),
                          z0=None if z0 is None else t(z0), **kw)
    return host(r)


@pytest.mark.parametrize("prec", ["fp64", "ladder"])
def test_sparse_lowest_16_parity(ipt, prec):
    """n = 200000 sparse symmetric perturbation (about 12 entries per row), the 16
    lowest columns, tol 1e-10: FP64 SpMM sweeps, and the FP32-SpMM + FP64-finish ladder."""
    say("csr n=200000 k=16 %s" % prec)
    th, rp, col, val = W.sparse_sym_uniform(200000, seed=0)
    idx = W.lowest_indices(th, 16)
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    g = _solve(ipt, th, rp, col, val, idx, tol=1e-10, precision=p)
    ref = oracle.ipt_csr(th, rp, col, val, idx, tol=1e-10)
    nm = oracle.norm1(th, csr=(rp, col, val))
    check(g.z, g.lam, g.status, ref, nm, 1e-10, gpu_sweeps=g.sweeps if prec == "fp64" else None)
    assert np.all(g.status == 0)
    assert abs(g.info["norm1"] - nm) <= 1e-12 * nm
    assert g.info["sweep_prec"][-1] in ("fp64", "exact-first")


@pytest.mark.parametrize("n,k,seed", [(1, 1, 0), (5, 3, 1), (1000, 1, 2), (1000, 37, 3), (3000, 64, 4),
                                      (2500, 100, 5)])
def test_sparse_shapes(ipt, n, k, seed):
    """Ragged k (1, 3, 37, 64, 100 columns: several lane groupings and more than 64
    columns per row), random requested indices, rows with no entries."""
    say("csr n=%d k=%d" % (n, k))
    th, rp, col, val = W.sparse_sym_uniform(n, pairs_per_row=3, amp=0.05, seed=seed)
    idx = np.random.default_rng(seed).permutation(n)[:k].astype(np.int32)
    g = _solve(ipt, th, rp, col, val, idx, tol=1e-12)
    ref = oracle.ipt_csr(th, rp, col, val, idx, tol=1e-12)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, csr=(rp, col, val)), 1e-12, gpu_sweeps=g.sweeps)


def test_morgan_ground_state(ipt):
    """Morgan's tridiagonal matrix (n = 5000, off-diagonal 0.5): the ground state
    converges slowly (tens of sweeps) to the oracle's answer; off-diagonal 0.75 fails."""
    say("csr morgan")
    th, rp, col, val = W.morgan_tridiagonal(5000, 0.5)
    g = _solve(ipt, th, rp, col, val, [0, 1, 2], tol=1e-12, max_iter=500)
    ref = oracle.ipt_csr(th, rp, col, val, np.array([0, 1, 2], np.int32), tol=1e-12, max_iter=500)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, csr=(rp, col, val)), 1e-12, gpu_sweeps=g.sweeps,
          sweep_slack=2)
    assert g.sweeps[0] > 20
    th, rp, col, val = W.morgan_tridiagonal(5000, 0.75)
    g = _solve(ipt, th, rp, col, val, [0], tol=1e-12, max_iter=500)
    assert g.status[0] != 0


def test_sparse_warm_start_resume(ipt):
    """Resume from the iterate returned after 1 sweep equals the uninterrupted solve."""
    say("csr resume")
    th, rp, col, val = W.sparse_sym_uniform(20000, seed=7)
    idx = W.lowest_indices(th, 16)
    full = _solve(ipt, th, rp, col, val, idx, tol=1e-13)
    part = _solve(ipt, th, rp, col, val, idx, tol=1e-13, max_iter=1)
    res = _solve(ipt, th, rp, col, val, idx, z0=part.z, tol=1e-13)
    np.testing.assert_array_equal(res.z, full.z)
    np.testing.assert_array_equal(res.lam, full.lam)
    ref = oracle.ipt_csr(th, rp, col, val, idx, z0=part.z, tol=1e-13)
    check(res.z, res.lam, res.status, ref, oracle.norm1(th, csr=(rp, col, val)), 1e-13)


def test_sparse_invalid(ipt):
    say("csr invalid")
    th, rp, col, val = W.sparse_sym_uniform(100, seed=1)
    bad = col.copy()
    bad[5] = 100
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, th, rp, bad, val, [0, 1])
    assert e.value.status == ipt.IPT_EINVAL
    rp2 = rp.copy()
    rp2[10], rp2[11] = rp2[11], rp2[10] - 1
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, th, rp2, col, val, [0, 1])
    assert e.value.status == ipt.IPT_EINVAL


def _csr_from_dense(a):
    rows, cols = np.nonzero(a)
    rp = np.zeros(a.shape[0] + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.int32), cols.astype(np.int32), a[rows, cols].astype(np.float64)


@pytest.mark.parametrize("kind", ["symmetric", "sign_flipped", "nonsymmetric", "long_row", "unsorted"])
def test_csr_norm1_paths(ipt, kind):
    """|M|_1 of a CSR input against the oracle's column sums on each path: |M|
    symmetric (largest row sum; also with entries of flipped sign, since only |M_jc|
    matters), not symmetric (scattered column sums), a row longer than the scan limit
    (scattered sums) and unsorted column indices (the scan is linear: row sums)."""
    say("csr norm1 %s" % kind)
    rng = np.random.default_rng(11)
    n = 700
    a = np.zeros((n, n))
    r = rng.integers(0, n, 4 * n)
    c = rng.integers(0, n, 4 * n)
    a[r, c] = rng.uniform(-0.05, 0.05, r.shape[0])
    a = a + a.T
    np.fill_diagonal(a, rng.uniform(-0.01, 0.01, n))
    if kind == "sign_flipped":
        a = np.triu(a) - np.tril(a, -1)
    if kind == "nonsymmetric":
        a[3, 7] = 0.4
    if kind == "long_row":
        a[5, :] = 0.001
        a[:, 5] = 0.001
        a[5, 5] = 0.3
    th = np.arange(n, dtype=np.float64) * 1.0
    rp, col, val = _csr_from_dense(a)
    if kind == "unsorted":
        for j in range(n):
            s, e = rp[j], rp[j + 1]
            col[s:e], val[s:e] = col[s:e][::-1].copy(), val[s:e][::-1].copy()
    g = _solve(ipt, th, rp, col, val, np.array([0, 1], np.int32), tol=1e-10, max_iter=3)
    want = np.max(np.sum(np.abs(np.diag(th) + a), axis=0))
    assert abs(g.info["norm1"] - want) <= 1e-13 * want, (g.info["norm1"], want)
    assert abs(oracle.norm1(th, csr=(rp, col, val)) - want) <= 1e-13 * want

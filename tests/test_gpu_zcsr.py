"""GPU parity of the sparse solve over C^n (C ABI ipt_solve_csr_z) against the complex
oracle on the same matrix made dense (a CSR row sum in column order is the dense row
sum with the zero terms left out)."""
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


def _csr(n, rows, cols, vals, merge=True):
    """COO -> CSR with columns sorted in each row; duplicates summed in order of
    appearance when merge, else kept as separate entries."""
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if merge and rows.size:
        key = rows * n + cols
        first = np.ones(key.shape[0], bool)
        first[1:] = key[1:] != key[:-1]
        seg = np.cumsum(first) - 1
        v = np.zeros(int(first.sum()), np.complex128)
        np.add.at(v, seg, vals)
        rows, cols, vals = rows[first], cols[first], v
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.int32), cols.astype(np.int32), vals.astype(np.complex128)


def _sparse(n, kind, per_row, amp, seed):
    """Sparse complex perturbation of theta = (1..n)(1 + 0.3i) (general) or 1..n
    (Hermitian: Delta_lj = conj(Delta_jl), real diagonal)."""
    rng = np.random.default_rng(seed)
    m = per_row * n
    a, b = rng.integers(0, n, m), rng.integers(0, n, m)
    v = amp * (rng.uniform(-1, 1, m) + 1j * rng.uniform(-1, 1, m))
    if kind == "hermitian":
        keep = a != b
        a, b, v = a[keep], b[keep], v[keep]
        diag = rng.integers(0, n, n // 4)
        rows = np.concatenate([a, b, diag])
        cols = np.concatenate([b, a, diag])
        vals = np.concatenate([v, v.conj(), amp * rng.uniform(-1, 1, diag.size) + 0j])
        th = np.arange(1, n + 1).astype(np.complex128)
    else:
        rows, cols, vals = a, b, v
        th = np.arange(1, n + 1) * (1.0 + 0.3j)
    rp, col, val = _csr(n, rows.astype(np.int64), cols.astype(np.int64), vals)
    return th.astype(np.complex128), rp, col, val


def _dense(n, rp, col, val):
    de = np.zeros((n, n), np.complex128)
    for j in range(n):
        for p in range(rp[j], rp[j + 1]):
            de[j, col[p]] += val[p]
    return de


def _norm1(th, de):
    return float(np.max(np.sum(np.abs(np.diag(th) + de), axis=0)))


def _solve(ipt, th, rp, col, val, idx, z0=None, **kw):
    r = ipt.ipt_solve_csr_z(t(np.ascontiguousarray(th, np.complex128)), t(rp), t(col),
                            t(np.ascontiguousarray(val, np.complex128)), t(np.asarray(idx, np.int32)),
                            z0=None if z0 is None else t(np.ascontiguousarray(z0, np.complex128)), **kw)
    return host(r)


@pytest.mark.parametrize("n,k,kind,seed", [(1, 1, "general", 0), (7, 3, "hermitian", 1), (900, 1, "general", 2),
                                           (900, 37, "hermitian", 3), (1500, 64, "general", 4),
                                           (1200, 100, "hermitian", 5)])
def test_zcsr_parity(ipt, n, k, kind, seed):
    """Ragged k (1, 3, 37, 64, 100: several lane groupings and more than 64 columns per
    row), random requested columns, rows with no entries; the norm against its
    definition over the modulus."""
    say("zcsr n=%d k=%d %s" % (n, k, kind))
    th, rp, col, val = _sparse(n, kind, 3, 0.05, seed)
    idx = np.random.default_rng(seed).permutation(n)[:k].astype(np.int32)
    g = _solve(ipt, th, rp, col, val, idx, tol=1e-12)
    de = _dense(n, rp, col, val)
    ref = oracle.ipt_dense_z(th, de, idx=idx, tol=1e-12)
    out = check(g.z, g.lam, g.status, ref, _norm1(th, de), 1e-12, gpu_sweeps=g.sweeps)
    assert out["compared"] >= 1
    assert np.all(g.z[idx, np.arange(k)] == 1.0)
    assert abs(g.info["norm1"] - _norm1(th, de)) <= 1e-12 * _norm1(th, de)


def test_zcsr_duplicates_and_warm_start(ipt):
    """Duplicate (row, column) entries are summed; a warm start from a one-sweep
    partial solve matches the oracle from the same iterate."""
    say("zcsr duplicates, warm start n=800 k=20")
    n, k = 800, 20
    rng = np.random.default_rng(11)
    m = 4 * n
    rows = np.concatenate([rng.integers(0, n, m), np.arange(0, n, 3)])
    cols = np.concatenate([rng.integers(0, n, m), (np.arange(0, n, 3) * 7) % n])
    vals = 0.04 * (rng.uniform(-1, 1, rows.size) + 1j * rng.uniform(-1, 1, rows.size))
    rows = np.concatenate([rows, rows[:200]])
    cols = np.concatenate([cols, cols[:200]])
    vals = np.concatenate([vals, 0.5 * vals[:200]])
    rp, col, val = _csr(n, rows.astype(np.int64), cols.astype(np.int64), vals, merge=False)
    th = (np.arange(1, n + 1) * (1.0 - 0.2j)).astype(np.complex128)
    de = _dense(n, rp, col, val)
    idx = np.sort(rng.choice(n, k, replace=False)).astype(np.int32)
    g = _solve(ipt, th, rp, col, val, idx, tol=1e-12)
    check(g.z, g.lam, g.status, oracle.ipt_dense_z(th, de, idx=idx, tol=1e-12), _norm1(th, de), 1e-12,
          gpu_sweeps=g.sweeps)
    part = _solve(ipt, th, rp, col, val, idx, tol=1e-12, max_iter=1)  # the product-free sweep only
    assert np.all(part.status == ipt.NOT_CONVERGED)
    w = _solve(ipt, th, rp, col, val, idx, z0=part.z, tol=1e-12, flags=ipt.FLAG_NO_NORM)
    refw = oracle.ipt_dense_z(th, de, idx=idx, z0=part.z, tol=1e-12)
    check(w.z, w.lam, w.status, refw, _norm1(th, de), 1e-12, gpu_sweeps=w.sweeps)


def test_zcsr_real_input_matches_real_path(ipt):
    """Real input through the complex sparse solve: the eigenpairs of the real sparse
    solve (the complex gap is inverted, the real one divides: rounding differs)."""
    say("zcsr on real input n=3000 k=16")
    th, rp, col, val = W.sparse_sym_uniform(3000, pairs_per_row=3, amp=0.05, seed=7)
    idx = W.lowest_indices(th, 16)
    rz = _solve(ipt, th.astype(np.complex128), rp, col, val.astype(np.complex128), idx, tol=1e-12)
    rr = host(ipt.ipt_solve_csr(t(th), t(rp), t(col), t(val), t(idx.astype(np.int32)), tol=1e-12))
    np.testing.assert_array_equal(rz.status, rr.status)
    assert np.max(np.abs(rz.z.imag)) == 0.0 and np.max(np.abs(rz.lam.imag)) == 0.0
    assert np.max(np.abs(rz.z.real - rr.z)) < 1e-13 and np.max(np.abs(rz.lam.real - rr.lam)) < 1e-13


def test_zcsr_two_by_two(ipt):
    """The complex 2 x 2 example in CSR form: W_21 after m sweeps is f^m(0),
    f(x) = eps (x^2 - 1)."""
    say("zcsr 2x2")
    eps = 0.3 + 0.2j
    th = np.array([0.0, 1.0], np.complex128)
    rp = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    val = np.array([eps, eps], np.complex128)
    x = 0.0
    for m in range(1, 6):
        x = eps * (x * x - 1.0)
        r = _solve(ipt, th, rp, col, val, np.array([0, 1], np.int32), tol=0.0, max_iter=m)
        assert abs(r.z[1, 0] - x) < 1e-15 and abs(r.z[0, 1] + x) < 1e-15


def test_zcsr_errors(ipt):
    th, rp, col, val = _sparse(64, "general", 2, 0.02, 0)
    idx = np.array([3, 9], np.int32)
    for kw in (dict(precision=ipt.PREC_LADDER), dict(flags=ipt.FLAG_ACX), dict(cont_alpha=0.5),
               dict(flags=ipt.FLAG_CHOOSE_D)):
        with pytest.raises(ipt.IPTError) as e:
            _solve(ipt, th, rp, col, val, idx, **kw)
        assert e.value.status == ipt.IPT_EINVAL, kw
    th2 = th.copy()
    th2[20] = th2[3]
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, th2, rp, col, val, idx)
    assert e.value.status == ipt.IPT_EDEGENERATE
    # a coincidence far down a long theta (the check runs in chunks of 4096 rows)
    thl, rpl, coll, vall = _sparse(10000, "general", 2, 0.02, 1)
    thl[9000] = thl[9]
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, thl, rpl, coll, vall, idx)
    assert e.value.status == ipt.IPT_EDEGENERATE
    bad = col.copy()
    bad[0] = 64  # column out of range
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, th, rp, bad, val, idx)
    assert e.value.status == ipt.IPT_EINVAL
    th3 = th.copy()
    th3[7] = np.nan + 0j
    with pytest.raises(ipt.IPTError) as e:
        _solve(ipt, th3, rp, col, val, idx)
    assert e.value.status == ipt.IPT_EINVAL

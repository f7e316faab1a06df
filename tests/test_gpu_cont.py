"""GPU parity of the non-autonomous continuation (opts.cont_alpha, dense and CSR FP64
sweeps) against the oracle's continuation, through the C ABI."""
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
    r = ipt.ipt_solve_dense(t(theta), t(delta), idx=None if idx is None else t(idx.astype(np.int32)),
                            z0=None if z0 is None else t(z0), **kw)
    return host(r)


def test_three_by_three_rescued(ipt):
    """The paper's 3 x 3 example at eps = -0.475: plain IPT diverges on column 2,
    the continuation converges there (after the scale reaches 1 at sweep 54); every
    column matches the oracle's continuation."""
    say("continuation 3x3 eps=-0.475 alpha=0.5")
    th, de = W.three_by_three(-0.475)
    plain = _solve(ipt, th, de, tol=1e-12, max_iter=2000)
    g = _solve(ipt, th, de, tol=1e-12, max_iter=2000, cont_alpha=0.5)
    ref = oracle.ipt_dense_cont(th, de, 0.5, tol=1e-12, max_iter=2000)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12, gpu_sweeps=g.sweeps, max_iter=2000)
    assert plain.status[1] == ipt.DIVERGED and g.status[1] == ipt.CONVERGED
    lam = np.linalg.eigvals(np.diag(th) + de)
    assert np.min(np.abs(lam - g.lam[1])) < 1e-10
    assert g.sweeps[1] >= 54


@pytest.mark.parametrize("n,k,eps,alpha", [(300, 300, 0.05, 0.5), (257, 40, 0.2, 0.7), (129, 129, 0.02, 0.5)])
def test_random_parity(ipt, n, k, eps, alpha):
    """Ragged sizes over several row and column tiles; every column certifies at the
    oracle's fixed point, no earlier than the scale's switch to 1."""
    say("continuation n=%d k=%d eps=%g alpha=%g" % (n, k, eps, alpha))
    th, de = W.dense_sym_gaussian(n, eps, 2)
    idx = None if k == n else np.sort(np.random.default_rng(4).choice(n, k, replace=False)).astype(np.int32)
    g = _solve(ipt, th, de, idx=idx, tol=1e-10, max_iter=400, cont_alpha=alpha)
    ref = oracle.ipt_dense_cont(th, de, alpha, idx=idx, tol=1e-10, max_iter=400, resid=False)
    out = check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-10, gpu_sweeps=g.sweeps, max_iter=400)
    assert out["compared"] == k
    switch = int(np.ceil(54 / np.log2(1 / alpha)))  # first t with alpha^t below half an ulp of 1 (approx.)
    assert np.all(g.sweeps >= switch - 2)


def test_budget_ends_during_continuation(ipt):
    """max_iter = 10 at alpha = 0.8: every column ends NOT_CONVERGED with the tenth
    iterate of the continuation map, equal to the oracle's to rounding."""
    say("continuation budget n=200")
    th, de = W.dense_sym_gaussian(200, 0.05, 6)
    g = _solve(ipt, th, de, tol=1e-10, max_iter=10, cont_alpha=0.8)
    ref = oracle.ipt_dense_cont(th, de, 0.8, tol=1e-10, max_iter=10, resid=False)
    assert np.all(g.status == ipt.NOT_CONVERGED) and np.all(ref.status == oracle.NOT_CONVERGED)
    assert np.max(np.abs(g.z - ref.z)) < 1e-13
    assert np.max(np.abs(g.lam - ref.lam)) < 1e-13 * oracle.norm1(th, de)


def test_tiny_alpha_is_plain(ipt):
    """cont_alpha = 1e-300: the first scale rounds to 1, so the solve is the plain
    FP64 method (same decisions and sweep counts, same answers)."""
    say("continuation alpha=1e-300 n=256")
    th, de = W.dense_sym_gaussian(256, 0.03, 8)
    p = _solve(ipt, th, de, tol=1e-12)
    g = _solve(ipt, th, de, tol=1e-12, cont_alpha=1e-300)
    np.testing.assert_array_equal(p.status, g.status)
    np.testing.assert_array_equal(p.sweeps, g.sweeps)
    assert np.max(np.abs(p.z - g.z)) < 1e-15 and np.max(np.abs(p.lam - g.lam)) < 1e-14


def test_continuation_rejected_elsewhere(ipt):
    th, de = W.dense_sym_gaussian(16, 0.01, 0)
    for kw in (dict(cont_alpha=0.5, precision=ipt.PREC_LADDER), dict(cont_alpha=0.5, flags=ipt.FLAG_ACX),
               dict(cont_alpha=1.0), dict(cont_alpha=-0.25), dict(cont_alpha=float("nan"))):
        with pytest.raises(ipt.IPTError) as e:
            _solve(ipt, th, de, **kw)
        assert e.value.status == ipt.IPT_EINVAL, kw
    th_s, rp, col, val = W.sparse_sym_uniform(64, 3, 0.05, 1)
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_solve_csr(t(th_s), t(rp), t(col), t(val), t(np.arange(4, dtype=np.int32)), cont_alpha=0.5,
                          precision=ipt.PREC_LADDER)
    assert e.value.status == ipt.IPT_EINVAL
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_solve_csr_z(t(th_s.astype(complex)), t(rp), t(col), t(val.astype(complex)),
                            t(np.arange(4, dtype=np.int32)), cont_alpha=0.5)
    assert e.value.status == ipt.IPT_EINVAL
    ns, thb, deb, _, _ = W.batched_sym_gaussian(3, 8, 40, 0.02, seed=1)
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_solve_batched(ns, t(thb), t(deb), cont_alpha=0.5)
    assert e.value.status == ipt.IPT_EINVAL


# ------------------------------------------------------------- continuation, CSR

def _dense_of(n, rp, col, val):
    de = np.zeros((n, n))
    for j in range(n):
        for p in range(rp[j], rp[j + 1]):
            de[j, col[p]] += val[p]
    return de


def _csr_of(de):
    n = de.shape[0]
    rows, cols = np.nonzero(de)
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.int32), cols.astype(np.int32), de[rows, cols].astype(np.float64)


def _solve_csr(ipt, th, rp, col, val, idx, **kw):
    return host(ipt.ipt_solve_csr(t(th), t(rp), t(col), t(val), t(np.asarray(idx, np.int32)), **kw))


def test_csr_three_by_three_rescued(ipt):
    """The 3 x 3 example at eps = -0.475 in CSR form: the continuation converges on the
    column plain IPT loses, as the oracle's continuation on the same matrix."""
    say("continuation csr 3x3 eps=-0.475 alpha=0.5")
    th, de = W.three_by_three(-0.475)
    rp, col, val = _csr_of(de)
    idx = np.arange(3, dtype=np.int32)
    plain = _solve_csr(ipt, th, rp, col, val, idx, tol=1e-12, max_iter=2000)
    g = _solve_csr(ipt, th, rp, col, val, idx, tol=1e-12, max_iter=2000, cont_alpha=0.5)
    ref = oracle.ipt_dense_cont(th, de, 0.5, tol=1e-12, max_iter=2000)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12, gpu_sweeps=g.sweeps, max_iter=2000)
    assert plain.status[1] == ipt.DIVERGED and g.status[1] == ipt.CONVERGED
    assert g.sweeps[1] >= 54


@pytest.mark.parametrize("n,k,alpha,seed", [(1500, 37, 0.7, 1), (2000, 64, 0.5, 2), (600, 100, 0.5, 3)])
def test_csr_continuation_parity(ipt, n, k, alpha, seed):
    """Sparse perturbations (several lane groupings, more than 64 columns) against the
    oracle's continuation on the densified matrix; no column certifies before the
    scale's switch to 1."""
    say("continuation csr n=%d k=%d alpha=%g" % (n, k, alpha))
    th, rp, col, val = W.sparse_sym_uniform(n, pairs_per_row=3, amp=0.1, seed=seed)
    idx = np.sort(np.random.default_rng(seed).choice(n, k, replace=False)).astype(np.int32)
    g = _solve_csr(ipt, th, rp, col, val, idx, tol=1e-10, max_iter=400, cont_alpha=alpha)
    de = _dense_of(n, rp, col, val)
    ref = oracle.ipt_dense_cont(th, de, alpha, idx=idx, tol=1e-10, max_iter=400, resid=False)
    out = check(g.z, g.lam, g.status, ref, oracle.norm1(th, csr=(rp, col, val)), 1e-10, gpu_sweeps=g.sweeps,
                max_iter=400)
    assert out["compared"] == k
    switch = int(np.ceil(54 / np.log2(1 / alpha)))
    assert np.all(g.sweeps >= switch - 2)


def test_csr_budget_ends_during_continuation(ipt):
    """max_iter = 10 at alpha = 0.8 on a CSR matrix: every column ends NOT_CONVERGED with
    the tenth iterate of the continuation map, the oracle's to rounding."""
    say("continuation csr budget n=800")
    th, rp, col, val = W.sparse_sym_uniform(800, pairs_per_row=3, amp=0.05, seed=6)
    idx = np.arange(0, 800, 25, dtype=np.int32)
    g = _solve_csr(ipt, th, rp, col, val, idx, tol=1e-10, max_iter=10, cont_alpha=0.8)
    ref = oracle.ipt_dense_cont(th, _dense_of(800, rp, col, val), 0.8, idx=idx, tol=1e-10, max_iter=10, resid=False)
    assert np.all(g.status == ipt.NOT_CONVERGED) and np.all(ref.status == oracle.NOT_CONVERGED)
    assert np.max(np.abs(g.z - ref.z)) < 1e-13
    assert np.max(np.abs(g.lam - ref.lam)) < 1e-13 * oracle.norm1(th, csr=(rp, col, val))


# ---------------------------------------------------------------- homotopy restart

def test_homotopy_three_by_three(ipt):
    """The homotopy restart (2 stages) on the paper's 3 x 3 example at eps = -0.475:
    column 2, which plain IPT loses, converges; every column matches the oracle's
    restart."""
    say("homotopy 3x3 eps=-0.475 Q=2")
    th, de = W.three_by_three(-0.475)
    g = _solve(ipt, th, de, tol=1e-12, max_iter=2000, homotopy_q=2)
    ref = oracle.ipt_dense_homotopy(th, de, 2, tol=1e-12, max_iter=2000)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12, max_iter=2000)
    assert g.status[1] == ipt.CONVERGED
    assert g.info["sweeps"] >= 2


@pytest.mark.parametrize("n,k,q,prec", [(300, 300, 3, "fp64"), (257, 40, 2, "fp64"), (256, 256, 2, "ladder")])
def test_homotopy_parity(ipt, n, k, q, prec):
    """Stages on the scaled copies over ragged sizes, scattered columns and the
    precision ladder inside each stage, against the oracle's restart."""
    say("homotopy n=%d k=%d Q=%d %s" % (n, k, q, prec))
    th, de = W.dense_sym_gaussian(n, 0.05, 3)
    idx = None if k == n else np.sort(np.random.default_rng(5).choice(n, k, replace=False)).astype(np.int32)
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    g = _solve(ipt, th, de, idx=idx, tol=1e-10, precision=p, homotopy_q=q)
    ref = oracle.ipt_dense_homotopy(th, de, q, idx=idx, tol=1e-10, resid=False)
    out = check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-10)
    assert out["compared"] == k


def test_homotopy_warm_start_and_one_stage(ipt):
    """A warm start feeds the first stage; one stage is the plain solve bit for bit."""
    say("homotopy warm start n=200")
    th, de = W.dense_sym_gaussian(200, 0.04, 8)
    part = _solve(ipt, th, de, tol=1e-12, max_iter=2)
    g = _solve(ipt, th, de, z0=part.z, tol=1e-12, homotopy_q=2)
    ref = oracle.ipt_dense_homotopy(th, de, 2, z0=part.z, tol=1e-12, resid=False)
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12)
    p = _solve(ipt, th, de, tol=1e-12)
    one = _solve(ipt, th, de, tol=1e-12, homotopy_q=1)
    np.testing.assert_array_equal(p.z, one.z)
    np.testing.assert_array_equal(p.lam, one.lam)


def test_homotopy_rejected_elsewhere(ipt):
    th, de = W.dense_sym_gaussian(16, 0.01, 0)
    for kw in (dict(homotopy_q=2, cont_alpha=0.5), dict(homotopy_q=-1), dict(homotopy_q=1001)):
        with pytest.raises(ipt.IPTError) as e:
            _solve(ipt, th, de, **kw)
        assert e.value.status == ipt.IPT_EINVAL, kw
    th_s, rp, col, val = W.sparse_sym_uniform(64, 3, 0.05, 1)
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_solve_csr(t(th_s), t(rp), t(col), t(val), t(np.arange(4, dtype=np.int32)), homotopy_q=2)
    assert e.value.status == ipt.IPT_EINVAL


def test_homotopy_with_acx(ipt):
    """IPT-ACX inside every stage of the restart, against the oracle's restart with
    ACX stages (application counts within a cycle, as for ACX alone)."""
    say("homotopy + ACX n=200 Q=2")
    th, de = W.dense_sym_gaussian(200, 0.05, 12)
    g = _solve(ipt, th, de, tol=1e-12, homotopy_q=2, flags=ipt.FLAG_ACX)
    ref = oracle.ipt_dense_homotopy(th, de, 2, tol=1e-12, resid=False, accel="acx")
    check(g.z, g.lam, g.status, ref, oracle.norm1(th, de), 1e-12)


@pytest.mark.parametrize("mode", ["continuation", "homotopy"])
def test_full_size_sampled(ipt, mode):
    """The benchmarked dense workload (n = 4096, eps = 0.01, full spectrum) under the
    continuation (alpha = 1/2) and the 2-stage restart; sampled columns by the oracle."""
    say("%s n=4096 sampled" % mode)
    th, de = W.dense_sym_gaussian(4096, 0.01, 0)
    kw = dict(cont_alpha=0.5) if mode == "continuation" else dict(homotopy_q=2)
    g = _solve(ipt, th, de, tol=1e-10, max_iter=200, **kw)
    assert np.all(g.status == 0)
    cols = np.unique(np.concatenate([[0, 1, 127, 128, 4095], np.random.default_rng(6).integers(0, 4096, 7)]))
    cols = cols.astype(np.int32)
    if mode == "continuation":
        ref = oracle.ipt_dense_cont(th, de, 0.5, idx=cols, tol=1e-10, max_iter=200, resid=False)
    else:
        ref = oracle.ipt_dense_homotopy(th, de, 2, idx=cols, tol=1e-10, max_iter=200, resid=False)
    check(g.z[:, cols], g.lam[cols], g.status[cols], ref, oracle.norm1(th, de), 1e-10)

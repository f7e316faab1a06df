"""Failure injection: one non-finite entry in Delta (the divergence of Sec. 1 and
Sec. 6.2 taken to its limit).  Row a of Delta Z is then non-finite for every column
(NaN * 0 and Inf * 0 are NaN), so every requested column must end DIVERGED, as the
oracle's do, on every path: dense FP64, the dense ladder with a BF16 and with an FP16
low rung (max |Delta| then sets the FP16 shadow scale from a poisoned matrix), CSR,
and a batch in which one problem is poisoned, whose other problems must come out
bit for bit as in the clean batch."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, host, say, t
from parity import check

pytestmark = pytest.mark.gpu

BAD = {"nan": np.nan, "inf": np.inf, "-inf": -np.inf}


@pytest.fixture(scope="module")
def ipt():
    from paper_2012_14702_amd import ipt as mod
    mod.load_library()
    dev()
    return mod


def _dense(ipt, th, de, idx=None, **kw):
    r = ipt.ipt_solve_dense(t(th), t(de), idx=None if idx is None else t(idx.astype(np.int32)), **kw)
    return host(r)


def _all_diverged(g, ref, nm, tol):
    assert np.all(ref.status == 2), "oracle: %s" % np.unique(ref.status)
    check(g.z, g.lam, g.status, ref, nm, tol)
    assert np.all(g.status == 2)
    assert g.info["diverged"] == g.status.shape[0] and g.info["converged"] == 0


@pytest.mark.parametrize("bad", ["nan", "inf", "-inf"])
@pytest.mark.parametrize("mode", ["fp64", "ladder_bf16", "ladder_fp16", "ladder_no_low"])
def test_dense_poisoned_delta(ipt, mode, bad):
    """n = 640 (five 128-row tiles), eps = 0.05 (the ladder runs its low rung), one
    poisoned entry off the diagonal; full spectrum and a scattered subset of 37
    columns."""
    say("nonfinite dense n=640 %s %s" % (mode, bad))
    th, de = W.dense_sym_gaussian(640, 0.05, 7)
    de[200, 333] = BAD[bad]
    kw = {"fp64": dict(precision=ipt.PREC_FP64),
          "ladder_bf16": dict(precision=ipt.PREC_LADDER, low_type=ipt.LOW_BF16),
          "ladder_fp16": dict(precision=ipt.PREC_LADDER, low_type=ipt.LOW_FP16),
          "ladder_no_low": dict(precision=ipt.PREC_LADDER, low_type=ipt.LOW_NONE)}[mode]
    nm = oracle.norm1(th, de)
    g = _dense(ipt, th, de, tol=1e-10, **kw)
    _all_diverged(g, oracle.ipt_dense(th, de, tol=1e-10, resid=False), nm, 1e-10)
    idx = np.random.default_rng(3).permutation(640)[:37].astype(np.int32)
    g = _dense(ipt, th, de, idx=idx, tol=1e-10, **kw)
    _all_diverged(g, oracle.ipt_dense(th, de, idx=idx, tol=1e-10, resid=False), nm, 1e-10)


def test_dense_poisoned_diagonal_and_clean_after(ipt):
    """A NaN on the diagonal of Delta (read by the product-free first sweep's d): every
    column diverges; the next solve on the handle, of the clean matrix, equals a solve
    on a fresh handle bit for bit (nothing of the poisoned solve stays behind)."""
    say("nonfinite dense diagonal, then clean")
    th, de = W.dense_sym_gaussian(384, 0.02, 8)
    bad = de.copy()
    bad[17, 17] = np.nan
    h = ipt.Handle()
    g = _dense(ipt, th, bad, tol=1e-10, precision=ipt.PREC_LADDER, handle=h)
    _all_diverged(g, oracle.ipt_dense(th, bad, tol=1e-10, resid=False), oracle.norm1(th, bad), 1e-10)
    a = _dense(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER, handle=h)
    b = _dense(ipt, th, de, tol=1e-10, precision=ipt.PREC_LADDER, handle=ipt.Handle())
    np.testing.assert_array_equal(a.z, b.z)
    np.testing.assert_array_equal(a.lam, b.lam)
    np.testing.assert_array_equal(a.status, b.status)
    assert np.all(a.status == 0)


@pytest.mark.parametrize("bad", ["nan", "inf"])
@pytest.mark.parametrize("prec", ["fp64", "ladder"])
def test_csr_poisoned_value(ipt, prec, bad):
    """CSR, n = 3000, 16 lowest columns, one stored value poisoned."""
    say("nonfinite csr n=3000 %s %s" % (prec, bad))
    th, rp, col, val = W.sparse_sym_uniform(3000, pairs_per_row=3, amp=0.05, seed=11)
    val = val.copy()
    val[rp[1500] + 1] = BAD[bad]
    idx = W.lowest_indices(th, 16)
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    r = ipt.ipt_solve_csr(t(th), t(rp), t(col), t(val), t(idx), tol=1e-10, precision=p)
    g = host(r)
    ref = oracle.ipt_csr(th, rp, col, val, idx, tol=1e-10)
    _all_diverged(g, ref, oracle.norm1(th, csr=(rp, col, val)), 1e-10)


@pytest.mark.parametrize("bad", ["nan", "inf"])
@pytest.mark.parametrize("prec", ["fp64", "ladder"])
def test_batched_one_poisoned_problem(ipt, prec, bad):
    """30 problems of the batched workload; problem 11 gets one poisoned entry.  Its
    columns all diverge (as the oracle's); every other problem's z, lambda and status
    equal those of the clean batch bit for bit."""
    say("nonfinite batched B=30 %s %s" % (prec, bad))
    ns, th, de, th_off, de_off = W.batched_sym_gaussian(30, 32, 400, 0.02, seed=9)
    b0 = 11
    n0 = int(ns[b0])
    bad_de = de.copy()
    bad_de[de_off[b0] + (n0 // 2) * n0 + 3] = BAD[bad]
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    kw = dict(tol=1e-10, precision=p, max_iter=64)

    def run(pool):
        r = ipt.ipt_solve_batched(ns, t(th), t(pool), **kw)
        return r.z.cpu().numpy(), r.lam.cpu().numpy(), r.status.cpu().numpy(), r.info

    zc, lc, sc, _ = run(de)
    zp, lp, sp, info = run(bad_de)
    for b in range(len(ns)):
        n = int(ns[b])
        zs = slice(int(de_off[b]), int(de_off[b]) + n * n)
        ts = slice(int(th_off[b]), int(th_off[b]) + n)
        if b == b0:
            thb = th[ts]
            deb = bad_de[zs].reshape(n, n)
            ref = oracle.ipt_dense(thb, deb, tol=1e-10, max_iter=64, resid=False)
            assert np.all(ref.status == 2)
            assert np.all(sp[ts] == 2)
        else:
            np.testing.assert_array_equal(zp[zs], zc[zs])
            np.testing.assert_array_equal(lp[ts], lc[ts])
            np.testing.assert_array_equal(sp[ts], sc[ts])
    assert info["diverged"] >= n0

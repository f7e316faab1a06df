"""GPU parity of the batched path (C ABI ipt_solve_batched) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import dev, say, t
from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ipt():
    from paper_2012_14702_amd import ipt as mod
    mod.load_library()
    dev()
    return mod


def _run(ipt, ns, th_pool, de_pool, **kw):
    r = ipt.ipt_solve_batched(ns, t(th_pool), t(de_pool), **kw)
    return r.z.cpu().numpy(), r.lam.cpu().numpy(), r.status.cpu().numpy(), r.info


def _per_problem(ns, th_off, de_off, z, lam, st, b):
    n = int(ns[b])
    return (z[de_off[b]:de_off[b] + n * n].reshape(n, n), lam[th_off[b]:th_off[b] + n], st[th_off[b]:th_off[b] + n])


@pytest.mark.parametrize("prec", ["fp64", "ladder"])
def test_batched_small_batch_parity(ipt, prec):
    """48 problems with n ~ U{32..512} (both tile sizes and ragged edges), theta sorted
    uniform, eps = 0.02: every problem matches the oracle column by column."""
    say("batched B=48 %s" % prec)
    ns, th, de, th_off, de_off = W.batched_sym_gaussian(48, 32, 512, 0.02, seed=3)
    p = ipt.PREC_LADDER if prec == "ladder" else ipt.PREC_FP64
    z, lam, st, info = _run(ipt, ns, th, de, tol=1e-10, precision=p, max_iter=64)
    ref = oracle.ipt_batched(ns, th, de, th_off, de_off, tol=1e-10, max_iter=64)
    compared = 0
    for b in range(48):
        gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
        rz, rl, rs = _per_problem(ns, th_off, de_off, ref.z, ref.lam, ref.status, b)
        n = int(ns[b])
        thb, deb = th[th_off[b]:th_off[b] + n], de[de_off[b]:de_off[b] + n * n].reshape(n, n)
        rr = oracle.ipt_dense(thb, deb, tol=1e-10, max_iter=64)   # per-column steps for the status rule
        np.testing.assert_array_equal(rr.status, rs)
        out = check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-10,
                    gpu_sweeps=None)
        compared += out["compared"]
    assert compared >= 0.95 * int(ns.sum())
    assert info["converged"] == int((st == 0).sum())


def test_batched_edge_sizes(ipt):
    """Sizes 1, 2, 63, 64, 65, 127, 128, 129, 192, 193, 256 and 300 in one batch."""
    sizes = [1, 2, 63, 64, 65, 127, 128, 129, 192, 193, 256, 300]
    say("batched edge sizes")
    th_parts, de_parts = [], []
    for q, n in enumerate(sizes):
        thb, deb = W.dense_sym_gaussian(n, 0.01, 100 + q)
        th_parts.append(thb)
        de_parts.append(deb.ravel())
    ns = np.array(sizes, dtype=np.int32)
    th = np.concatenate(th_parts)
    de = np.concatenate(de_parts)
    th_off = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    de_off = np.concatenate([[0], np.cumsum(ns.astype(np.int64) ** 2)[:-1]]).astype(np.int64)
    z, lam, st, info = _run(ipt, ns, th, de, tol=1e-12)
    assert np.all(st == 0)
    for b, n in enumerate(sizes):
        gz, gl, gs = _per_problem(ns, th_off, de_off, z, lam, st, b)
        thb, deb = th_parts[b], de_parts[b].reshape(n, n)
        rr = oracle.ipt_dense(thb, deb, tol=1e-12)
        check(gz, gl, gs, rr, oracle.norm1(thb, deb), 1e-12)


def test_batched_invalid(ipt):
    say("batched invalid")
    ns, th, de, th_off, de_off = W.batched_sym_gaussian(4, 32, 64, 0.02, seed=1)
    th2 = th.copy()
    th2[th_off[2] + 3] = th2[th_off[2] + 4]
    with pytest.raises(ipt.IPTError) as e:
        _run(ipt, ns, th2, de)
    assert e.value.status == ipt.IPT_EDEGENERATE
    bad = ns.copy()
    bad[1] = 5000
    with pytest.raises(ipt.IPTError) as e:
        _run(ipt, bad, th, de)
    assert e.value.status == ipt.IPT_EINVAL

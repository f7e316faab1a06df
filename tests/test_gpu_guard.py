"""Debug mode of the workspace (IPT_GUARD): every slice a solve carves is followed by
a guard band that is filled before the solve and checked after it.  Every solve kind
must leave the bands intact and give the same answers as without them; the self-test
mode, which overwrites a band from the host, must be reported as IPT_EGUARD."""
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


def _handle(ipt, monkeypatch, mode):
    monkeypatch.setenv("IPT_GUARD", mode)
    h = ipt.Handle()          # the mode is read when the handle is created
    monkeypatch.delenv("IPT_GUARD")
    return h


def _solves(ipt, h):
    """One of each solve kind, on handle h; returns the host results."""
    out = {}
    th, de = W.dense_sym_gaussian(300, 0.02, 5)
    out["dense_fp64"] = host(ipt.ipt_solve_dense(t(th), t(de), tol=1e-10, handle=h))
    out["dense_ladder"] = host(ipt.ipt_solve_dense(t(th), t(de), tol=1e-10, precision=ipt.PREC_LADDER, handle=h))
    out["dense_acx"] = host(ipt.ipt_solve_dense(t(th), t(de), tol=1e-10, flags=ipt.FLAG_ACX, handle=h))
    ths, rp, col, val = W.sparse_sym_uniform(5000, seed=2)
    idx = t(W.lowest_indices(ths, 8).astype(np.int32))
    out["csr_ladder"] = host(ipt.ipt_solve_csr(t(ths), t(rp), t(col), t(val), idx, tol=1e-10,
                                               precision=ipt.PREC_LADDER, handle=h))
    thc = th.astype(np.complex128)
    a = np.random.default_rng(7).standard_normal(de.shape) * (0.02 / np.sqrt(300))
    dec = (de + 1j * (a - a.T)).astype(np.complex128)         # Hermitian
    out["complex"] = host(ipt.ipt_solve_dense_z(t(thc), t(dec), tol=1e-10, handle=h))
    ns, thb, deb, _, _ = W.batched_sym_gaussian(12, 32, 200, 0.02, seed=4)
    r = ipt.ipt_solve_batched(ns, t(thb), t(deb), tol=1e-10, precision=ipt.PREC_LADDER, max_iter=64, handle=h)
    out["batched_ladder"] = {"z": r.z.cpu().numpy(), "lam": r.lam.cpu().numpy(), "status": r.status.cpu().numpy()}
    return out


def test_guard_bands_stay_intact_and_answers_unchanged(ipt, monkeypatch):
    say("guard bands: every solve kind")
    plain = _solves(ipt, ipt.Handle())
    guarded = _solves(ipt, _handle(ipt, monkeypatch, "1"))
    for kind in plain:
        a, b = plain[kind], guarded[kind]
        for key in ("z", "lam", "status"):
            x = a[key] if isinstance(a, dict) else getattr(a, key)
            y = b[key] if isinstance(b, dict) else getattr(b, key)
            np.testing.assert_array_equal(np.asarray(x), np.asarray(y), err_msg="%s %s" % (kind, key))


def test_guard_selftest_is_reported(ipt, monkeypatch):
    say("guard bands: self-test")
    h = _handle(ipt, monkeypatch, "selftest")
    th, de = W.dense_sym_gaussian(200, 0.02, 6)
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_solve_dense(t(th), t(de), tol=1e-10, handle=h)
    assert e.value.status == ipt.IPT_EGUARD
    assert "guard band 1 " in h.last_error()
    ns, thb, deb, _, _ = W.batched_sym_gaussian(4, 32, 100, 0.02, seed=4)
    with pytest.raises(ipt.IPTError) as e:
        ipt.ipt_solve_batched(ns, t(thb), t(deb), tol=1e-10, handle=h)
    assert e.value.status == ipt.IPT_EGUARD

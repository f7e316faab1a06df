"""Parity rule between the HIP path and the FP64 oracle.

Columns both sides mark CONVERGED are compared: |lambda_gpu - lambda_oracle| <=
lam_tol * |M|_1 and eigenvector angle 2 asin(|a/|a| - b/|b||/2) <= ang_tol (both
columns have entry idx[c] equal to +1, so there is no sign ambiguity).  Statuses
must agree, except for columns whose oracle deciding step lies within a factor 4 of
the tolerance (rounding can move that decision by one sweep), and, when max_iter is
given, for columns the oracle leaves undecided until the last sweep: there the
divergence rule's growth count on that sweep decides between DIVERGED and
NOT_CONVERGED, and on a trajectory that never converges that count depends on the
rounding order, so either failure status is accepted (never CONVERGED).  On a
precision-ladder solve (ladder=True) the growth count of the divergence rule runs on
exact sweeps only, so a failing column's count starts later than the FP64 oracle's
and its label can differ anywhere before the cap: there any two failure statuses
match (never CONVERGED against a failure).  Sweep counts may differ by one."""
import numpy as np

LAM_TOL = 1e-10
ANG_TOL = 1e-8


def angles(a, b):
    an = a / np.linalg.norm(a, axis=0, keepdims=True)
    bn = b / np.linalg.norm(b, axis=0, keepdims=True)
    return 2.0 * np.arcsin(np.minimum(1.0, np.linalg.norm(an - bn, axis=0) / 2.0))


def check(gpu_z, gpu_lam, gpu_status, ref, norm1, tol, gpu_sweeps=None, lam_tol=LAM_TOL, ang_tol=ANG_TOL,
          sweep_slack=1, cols=None, max_iter=None, ladder=False):
    """gpu_* are numpy arrays restricted to the same columns as ref (an oracle
    Result).  Returns a dict of the worst errors; raises AssertionError on a
    violation."""
    gst = np.asarray(gpu_status)
    rst = np.asarray(ref.status)
    edge = (ref.step >= tol / 4) & (ref.step <= 4 * tol)
    bad_status = (gst != rst) & ~edge
    if max_iter is not None:
        last = (np.asarray(ref.sweeps) >= max_iter) & (rst != 0) & (gst != 0)
        bad_status &= ~last
    if ladder:
        bad_status &= ~((gst != 0) & (rst != 0))
    assert not bad_status.any(), "status mismatch in columns %s: gpu %s oracle %s" % (
        np.where(bad_status)[0][:10], gst[bad_status][:10], rst[bad_status][:10])
    both = (gst == 0) & (rst == 0)
    out = {"compared": int(both.sum()), "max_dlam": 0.0, "max_angle": 0.0}
    if both.any():
        dl = np.abs(gpu_lam[both] - ref.lam[both])
        ang = angles(gpu_z[:, both], ref.z[:, both])
        out["max_dlam"] = float(dl.max())
        out["max_angle"] = float(ang.max())
        assert dl.max() <= lam_tol * norm1, "max |dlambda| %.3g > %.3g" % (dl.max(), lam_tol * norm1)
        assert ang.max() <= ang_tol, "max angle %.3g > %.3g" % (ang.max(), ang_tol)
    if gpu_sweeps is not None:
        ds = np.abs(np.asarray(gpu_sweeps)[both] - ref.sweeps[both])
        if ds.size:
            assert ds.max() <= sweep_slack, "sweep counts differ by %d" % ds.max()
    return out

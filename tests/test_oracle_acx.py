"""Pins of the IPT-ACX oracle (alternating cyclic extrapolation, Alg. 3, in place
of the plain update of Alg. 1), against properties that do not come from the oracle
itself: the exact behaviour of the extrapolation on an affine map (closed forms),
the eigen-decomposition of the matrix, and the convergence facts the paper reports
for Morgan's tridiagonal matrix (Sec. 6.1)."""
import numpy as np
import pytest

import oracle
import workloads as W


def affine_case(r, n=6, d00=0.3):
    """A matrix whose map f_0 is affine with Jacobian r * I on the free entries:
    row 0 of Delta is (d00, 0, ...), the only other entries are Delta_j0 = 0.1 j and
    Delta_jj = d00 - r (theta_j - theta_0), so f_0(z)_j = r z_j - Delta_j0 / (theta_j -
    theta_0).  Its fixed point is the eigenvector of M for lambda = theta_0 + d00 in
    the chart z_0 = 1: z*_j = -Delta_j0 / ((theta_j - theta_0)(1 - r))."""
    th = np.arange(n, dtype=np.float64)
    de = np.zeros((n, n))
    de[0, 0] = d00
    for j in range(1, n):
        de[j, 0] = 0.1 * j
        de[j, j] = d00 - r * (th[j] - th[0])
    zs = np.zeros(n)
    zs[0] = 1.0
    zs[1:] = -de[1:, 0] / ((th[1:] - th[0]) * (1.0 - r))
    return th, de, zs


def test_affine_case_is_an_eigenvector():
    th, de, zs = affine_case(0.95)
    m = np.diag(th) + de
    assert np.allclose(m @ zs, (th[0] + de[0, 0]) * zs, rtol=0, atol=1e-14)


def test_acx_solves_a_contracting_affine_map_in_one_cycle():
    """For x -> r x + b with r < 1 the order-3 extrapolation of the first cycle lands
    on the fixed point (sigma = 1/(1 - r)), so the test on the next application
    certifies it: 4 applications of F.  Plain iteration needs ~log(1e-10)/log(0.95)
    = 449 sweeps."""
    th, de, zs = affine_case(0.95)
    idx = np.array([0], np.int32)
    r = oracle.ipt_dense(th, de, idx=idx, tol=1e-10, max_iter=100, accel="acx")
    assert r.status[0] == oracle.CONVERGED and r.sweeps[0] == 4
    # rounding of D^3 (a few ulps of |z| ~ 2) is amplified by sigma^3 = 1/(1 - r)^3 = 8000
    assert np.max(np.abs(r.z[:, 0] - zs)) < 2e-11
    assert abs(r.lam[0] - (th[0] + de[0, 0])) < 1e-14
    p = oracle.ipt_dense(th, de, idx=idx, tol=1e-10, max_iter=100)
    assert p.status[0] == oracle.NOT_CONVERGED


@pytest.mark.parametrize("max_iter,factor,used", [(4, 8 * 1.5, 4), (5, 8 * 1.5, 4), (6, 32 * 1.5, 6),
                                                  (8, 32 * 1.5, 6), (9, 256 * 1.5, 9)])
def test_acx_cycle_factors_on_a_repelling_affine_map(max_iter, factor, used):
    """For x -> r x + b with r > 1, sigma = 1/(r - 1) and a cycle of order p maps the
    error e to (1 + 1)^p e: 8 e for p = 3, 4 e for p = 2.  From z* + e0 the orders run
    3, 2, 3, 2 with tests at applications 1, 4, 6, 9.  A test whose cycle could not be
    followed by another test within max_iter ends the column NOT_CONVERGED with F(z):
    F(z* + 8 e0) = z* + 12 e0 at application 4 (max_iter 4 or 5), F(z* + 32 e0) at 6
    (max_iter 6 to 8), F(z* + 256 e0) at 9; no application runs past max_iter."""
    th, de, zs = affine_case(1.5)
    rng = np.random.default_rng(1)
    e0 = 1e-3 * rng.standard_normal(6)
    e0[0] = 0.0
    z0 = (zs + e0).reshape(6, 1)
    r = oracle.ipt_dense(th, de, idx=np.array([0], np.int32), z0=z0, tol=1e-12, max_iter=max_iter, accel="acx")
    assert r.status[0] == oracle.NOT_CONVERGED and r.sweeps[0] == used
    np.testing.assert_allclose(r.z[:, 0], zs + factor * e0, rtol=0, atol=1e-12)


def test_acx_dense_matches_eigh():
    """Symmetric n = 200, eps = 0.01: every column converges to the eigenvector that
    continues e_i (Weyl: sorted order), intermediate normalisation, and lambda."""
    th, de = W.dense_sym_gaussian(200, 0.01, 7)
    r = oracle.ipt_dense(th, de, tol=1e-12, accel="acx")
    assert np.all(r.status == oracle.CONVERGED)
    ev, vec = np.linalg.eigh(np.diag(th) + de)
    zref = vec / np.diag(vec)[None, :]
    assert np.max(np.abs(r.lam - ev)) < 1e-11
    assert np.max(np.abs(r.z - zref)) < 1e-10
    # F(Z) - Z = -G o (M Z - Z Lambda): |M z - lambda z| <= max gap * |step| <= 200 * tol
    assert np.max(r.resid) < 200 * 1e-12


def _morgan_ground(off, accel):
    th, rp, col, val = W.morgan_tridiagonal(5000, off)
    return oracle.ipt_csr(th, rp, col, val, np.array([0], np.int32), tol=1e-12, max_iter=5000, accel=accel), th


def test_acx_morgan(golden_dir):
    """Sec. 6.1: on Morgan's matrix (off-diagonal 0.5) IPT-ACX needs far fewer matvecs
    than IPT (about as few as the best Davidson-type method), and it converges for
    off-diagonals past the value where plain IPT stops converging (failure study)."""
    from conftest import read_facts
    import os
    off = read_facts(os.path.join(golden_dir, "paper_facts.txt"))["morgan_ipt_failure_offdiag"]
    acx, th = _morgan_ground(off, "acx")
    plain, _ = _morgan_ground(off, "picard")
    assert acx.status[0] == oracle.CONVERGED and plain.status[0] == oracle.CONVERGED
    assert 2 * acx.sweeps[0] < plain.sweeps[0]
    assert abs(acx.lam[0] - plain.lam[0]) < 1e-11
    for o in (off + 0.25, off + 0.5):
        a, th = _morgan_ground(o, "acx")
        p, _ = _morgan_ground(o, "picard")
        assert a.status[0] == oracle.CONVERGED and p.status[0] != oracle.CONVERGED
        dense = np.diag(th[:600]) + np.diag(np.full(599, o), 1) + np.diag(np.full(599, o), -1)
        assert abs(a.lam[0] - np.linalg.eigvalsh(dense)[0]) < 1e-10

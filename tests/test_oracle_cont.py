"""Pins of the oracle's non-autonomous continuation (concluding discussion of the
3 x 3 example): sweep t applies the map of the partition D + (1 - alpha^t) Delta;
and of the homotopy restart (concluding section): stages D + (q/Q) Delta, each
started from the previous stage's vectors.

Each pin checks the oracle against something other than itself: closed forms of
the first iterates, the eigen-decomposition of the paper's 3 x 3 matrix by the
textbook routine, the limit alpha -> 0 (the plain method, pinned on its own), and
the FP64 fact that 1 - 2^-54 rounds to 1."""
import numpy as np

import oracle
import workloads as W


def _random_case(n=8, eps=0.05, seed=3):
    return W.dense_sym_gaussian(n, eps, seed)


def pin_first_iterate():
    """From z = e_i one sweep gives e_i - (1 - alpha) G o Delta e_i: the first-order
    Rayleigh-Schroedinger term of the scaled perturbation (eq. 4 with l = 1)."""
    th, de = _random_case()
    a = 0.3
    r = oracle.ipt_dense_cont(th, de, a, tol=0.0, max_iter=1, resid=False)
    gap = th[:, None] - th[None, :]
    np.fill_diagonal(gap, 1.0)
    want = -(1.0 - a) * de / gap
    np.fill_diagonal(want, 1.0)
    ok = np.all(r.status == oracle.NOT_CONVERGED) and np.all(r.sweeps == 1)
    return bool(ok and np.max(np.abs(r.z - want)) < 1e-15)


def pin_schedule():
    """Iterate t is the plain map f_i of the partition D + (1 - alpha^t) Delta
    applied to iterate t - 1: checked for t = 2 and t = 10 through the plain map."""
    th, de = _random_case(seed=5)
    a = 0.7
    ok = True
    for t_end in (2, 10):
        r = oracle.ipt_dense_cont(th, de, a, tol=0.0, max_iter=t_end, resid=False)
        for c in (0, 3, 7):
            z = np.zeros(len(th))
            z[c] = 1.0
            for t in range(1, t_end + 1):
                z, _ = oracle.ipt_map(th, (1.0 - a ** t) * de, c, z)
            ok &= bool(np.max(np.abs(r.z[:, c] - z)) < 1e-14)
    return ok


def three_by_three_case():
    """The paper's 3 x 3 example at eps = -0.475, column 2 (index 1): near the
    Neimark-Sacker point the paper describes, plain IPT from e_2 leaves the basin of
    an attracting fixed point; returns (theta, delta, eigenvector with z_2 = 1,
    eigenvalue, spectral radius of the Jacobian of f_2 there)."""
    th, de = W.three_by_three(-0.475)
    lam, vec = np.linalg.eig(np.diag(th) + de)
    m = int(np.argmin(np.abs(lam - 0.94)))
    v = np.real(vec[:, m] / vec[1, m])
    h = 1e-7
    f0, _ = oracle.ipt_map(th, de, 1, v)
    jac = np.zeros((3, 3))
    for j in range(3):
        vv = v.copy()
        vv[j] += h
        f1, _ = oracle.ipt_map(th, de, 1, vv)
        jac[:, j] = (f1 - f0) / h
    return th, de, v, float(np.real(lam[m])), float(np.max(np.abs(np.linalg.eigvals(jac))))


def pin_three_by_three():
    """Plain IPT diverges on column 2; the continuation converges to the eigenvector
    of M (textbook eigen-decomposition) and its eigenvalue."""
    th, de, v, lam, rho = three_by_three_case()
    idx = np.array([1], np.int32)
    plain = oracle.ipt_dense(th, de, idx=idx, tol=1e-12, max_iter=2000, resid=False)
    cont = oracle.ipt_dense_cont(th, de, 0.5, idx=idx, tol=1e-12, max_iter=2000, resid=False)
    ok = rho < 1.0 and plain.status[0] == oracle.DIVERGED and cont.status[0] == oracle.CONVERGED
    return bool(ok and np.max(np.abs(cont.z[:, 0] - v)) < 1e-9 and abs(cont.lam[0] - lam) < 1e-10)


def pin_alpha_to_zero():
    """alpha = 1e-300: the first scale 1 - alpha rounds to 1, so the continuation is
    the plain method sweep for sweep (same iterates, decisions and results)."""
    th, de = _random_case(n=24, eps=0.2, seed=7)
    p = oracle.ipt_dense(th, de, tol=1e-12, max_iter=100)
    c = oracle.ipt_dense_cont(th, de, 1e-300, tol=1e-12, max_iter=100)
    return bool(np.array_equal(p.z, c.z) and np.array_equal(p.lam, c.lam) and np.array_equal(p.status, c.status)
                and np.array_equal(p.sweeps, c.sweeps))


def pin_certify_at_full_scale():
    """With alpha = 1/2 the scale 1 - 2^-t is below 1 up to t = 53 (1 - 2^-53 is an
    FP64 number) and 1 from t = 54 (1 - 2^-54 is a tie that rounds to 1): no column
    certifies before sweep 54, and each certifies at the same fixed point as plain
    IPT."""
    assert 1.0 - 2.0 ** -53 < 1.0 and 1.0 - 2.0 ** -54 == 1.0
    th, de = _random_case(n=24, eps=0.2, seed=7)
    p = oracle.ipt_dense(th, de, tol=1e-12, max_iter=100)
    c = oracle.ipt_dense_cont(th, de, 0.5, tol=1e-12, max_iter=100)
    ok = np.all(c.status == oracle.CONVERGED) and np.all(c.sweeps >= 54) and np.all(c.sweeps <= 56)
    return bool(ok and np.max(np.abs(c.z - p.z)) < 1e-11 and np.max(np.abs(c.lam - p.lam)) < 1e-12)


PINS = (pin_first_iterate, pin_schedule, pin_three_by_three, pin_alpha_to_zero, pin_certify_at_full_scale)


def cont_pins_pass():
    return all(p() for p in PINS)


def test_first_iterate():
    assert pin_first_iterate()


def test_schedule():
    assert pin_schedule()


def test_three_by_three_rescued():
    assert pin_three_by_three()


def test_alpha_to_zero_is_plain():
    assert pin_alpha_to_zero()


def test_certification_only_at_full_scale():
    assert pin_certify_at_full_scale()


def test_bad_alpha_rejected():
    th, de = _random_case()
    for a in (0.0, 1.0, -0.5, float("nan")):
        try:
            oracle.ipt_dense_cont(th, de, a)
        except ValueError:
            continue
        raise AssertionError("alpha %r accepted" % a)


# ---------------------------------------------------------------- homotopy restart

def test_homotopy_rescues_three_by_three():
    """The paper's 3 x 3 example at eps = -0.475, column 2: plain IPT diverges, the
    homotopy restart with 2 stages (D + Delta/2, then D + Delta from its vectors)
    reaches the eigenvector and eigenvalue given by the textbook decomposition."""
    th, de, v, lam, rho = three_by_three_case()
    idx = np.array([1], np.int32)
    plain = oracle.ipt_dense(th, de, idx=idx, tol=1e-12, max_iter=2000, resid=False)
    h = oracle.ipt_dense_homotopy(th, de, 2, idx=idx, tol=1e-12, max_iter=2000, resid=False)
    assert plain.status[0] == oracle.DIVERGED and h.status[0] == oracle.CONVERGED
    assert np.max(np.abs(h.z[:, 0] - v)) < 1e-9 and abs(h.lam[0] - lam) < 1e-10


def test_homotopy_first_stage_is_the_scaled_problem():
    """With 3 stages, stage 1 solves D + Delta/3: its vectors are the eigenvectors of
    that matrix (eigh); the full restart ends at the eigenvectors of D + Delta."""
    from jacobi_ref import cyclic_jacobi
    th, de = W.dense_sym_gaussian(10, 0.3, 4)
    th = th + 5.0
    first = oracle.ipt_dense(th, de * (1.0 / 3.0), tol=1e-14, max_iter=500)
    ev, vec = cyclic_jacobi(np.diag(th) + de / 3.0)
    for col in range(10):
        m = int(np.argmax(np.abs(vec[col, :])))
        assert np.max(np.abs(first.z[:, col] - vec[:, m] / vec[col, m])) < 1e-11
    h = oracle.ipt_dense_homotopy(th, de, 3, tol=1e-14, max_iter=500)
    ev, vec = cyclic_jacobi(np.diag(th) + de)
    for col in range(10):
        m = int(np.argmax(np.abs(vec[col, :])))
        assert np.max(np.abs(h.z[:, col] - vec[:, m] / vec[col, m])) < 1e-11
        assert abs(h.lam[col] - ev[m]) < 1e-11
    assert np.all(h.sweeps > oracle.ipt_dense(th, de, tol=1e-14, max_iter=500).sweeps)


def test_homotopy_one_stage_is_plain():
    th, de = _random_case(n=24, eps=0.2, seed=7)
    p = oracle.ipt_dense(th, de, tol=1e-12)
    h = oracle.ipt_dense_homotopy(th, de, 1, tol=1e-12)
    assert np.array_equal(p.z, h.z) and np.array_equal(p.lam, h.lam) and np.array_equal(p.sweeps, h.sweeps)

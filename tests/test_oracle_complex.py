"""Pins of the oracle's IPT over C^n (Sec. 2 states the method for complex M):
against the textbook eigen-decompositions (numpy eigh / eig), the complex 2 x 2
closed form of Sec. 4.3, and the real oracle on real input."""
import numpy as np

import oracle
import workloads as W


def _herm_case(n=16, eps=0.05, seed=2):
    rng = np.random.default_rng(seed)
    a = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    de = eps * (a + a.conj().T) / 2
    th = np.arange(1, n + 1).astype(np.complex128)
    return th, de


def _general_case(n=30, eps=0.04, seed=3):
    rng = np.random.default_rng(seed)
    de = eps * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    th = np.arange(1, n + 1) * (1.0 + 0.3j)
    return th, de


def _textbook_columns(th, de, hermitian):
    m = np.diag(th) + de
    lam, vec = np.linalg.eigh(m) if hermitian else np.linalg.eig(m)
    out_z, out_l = [], []
    for i in range(len(th)):
        k = int(np.argmax(np.abs(vec[i, :]) / np.linalg.norm(vec, axis=0)))
        out_z.append(vec[:, k] / vec[i, k])
        out_l.append(lam[k])
    return np.array(out_z).T, np.array(out_l)


def pin_hermitian():
    th, de = _herm_case()
    r = oracle.ipt_dense_z(th, de, tol=1e-14, max_iter=200)
    zt, lt = _textbook_columns(th, de, True)
    return bool(np.all(r.status == 0) and np.max(np.abs(r.z - zt)) < 1e-11 and np.max(np.abs(r.lam - lt)) < 1e-12)


def pin_general():
    th, de = _general_case()
    r = oracle.ipt_dense_z(th, de, tol=1e-14, max_iter=200)
    zt, lt = _textbook_columns(th, de, False)
    return bool(np.all(r.status == 0) and np.max(np.abs(r.z - zt)) < 1e-11 and np.max(np.abs(r.lam - lt)) < 1e-12)


def pin_two_by_two():
    """M = [[0, eps], [eps, 1]], eps complex: iterate t of column 1 is (1, f^t(0)),
    f(x) = eps (x^2 - 1), and of column 2 (-f^t(0), 1)."""
    eps = 0.3 + 0.2j
    th = np.array([0.0, 1.0], np.complex128)
    de = np.array([[0.0, eps], [eps, 0.0]], np.complex128)
    x, ok = 0.0, True
    for t in range(1, 7):
        x = eps * (x * x - 1.0)
        r = oracle.ipt_dense_z(th, de, tol=0.0, max_iter=t, resid=False)
        ok &= bool(abs(r.z[1, 0] - x) < 1e-15 and abs(r.z[0, 1] + x) < 1e-15 and r.z[0, 0] == 1 and r.z[1, 1] == 1)
    return ok


def pin_real_input():
    """Real input, as complex numbers with zero imaginary parts, gives the real
    oracle's iterates, decisions and eigenvalues bit for bit (cold and warm)."""
    th, de = W.dense_sym_gaussian(40, 0.05, 3)
    r = oracle.ipt_dense(th, de, tol=1e-13)
    z = oracle.ipt_dense_z(th.astype(complex), de.astype(complex), tol=1e-13)
    ok = np.array_equal(r.z, z.z.real) and np.all(z.z.imag == 0) and np.array_equal(r.lam, z.lam.real)
    ok &= np.array_equal(r.sweeps, z.sweeps) and np.array_equal(r.status, z.status)
    part = oracle.ipt_dense(th, de, tol=1e-13, max_iter=2)
    r2 = oracle.ipt_dense(th, de, z0=part.z, tol=1e-13)
    z2 = oracle.ipt_dense_z(th.astype(complex), de.astype(complex), z0=part.z.astype(complex), tol=1e-13)
    return bool(ok and np.array_equal(r2.z, z2.z.real) and np.array_equal(r2.sweeps, z2.sweeps))


PINS = (pin_hermitian, pin_general, pin_two_by_two, pin_real_input)


def complex_pins_pass():
    return all(p() for p in PINS)


def test_hermitian_vs_eigh():
    assert pin_hermitian()


def test_general_vs_eig():
    assert pin_general()


def test_complex_two_by_two_closed_form():
    assert pin_two_by_two()


def test_real_input_is_the_real_oracle():
    assert pin_real_input()

"""Pins of the FP64 oracle against what the paper and the mathematics fix:
closed forms, printed worked-example data, textbook routines, theorems and
invariants.  None of these compares the oracle with itself."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from conftest import read_facts, read_polys
from jacobi_ref import cyclic_jacobi


# ---------------------------------------------------------------- 2x2 (Sec. 4.3)

def _f_iter(eps, k):
    """k-fold iterate of f(x) = eps (x^2 - 1) from 0 (Sec. 4.3)."""
    x = 0.0
    out = [x]
    for _ in range(k):
        x = eps * (x * x - 1.0)
        out.append(x)
    return np.array(out)


@pytest.mark.parametrize("eps", [0.05, 0.3, -0.45, 0.7, 0.85])
def test_two_by_two_per_iterate(eps):
    """Z^(k) = [[1, -f^k(0)], [f^k(0), 1]] for every k (closed form of Sec. 4.3)."""
    th, de = W.two_by_two(eps)
    fx = _f_iter(eps, 25)
    t0 = oracle.ipt_trace(th, de, 0, 25)   # column 0 iterates
    t1 = oracle.ipt_trace(th, de, 1, 25)   # column 1 iterates
    scale = np.maximum(1.0, np.abs(fx))
    assert np.all(t0[:, 0] == 1.0) and np.all(t1[:, 1] == 1.0)
    assert np.max(np.abs(t0[:, 1] - fx) / scale) <= 8 * np.finfo(float).eps * 25
    assert np.max(np.abs(t1[:, 0] + fx) / scale) <= 8 * np.finfo(float).eps * 25


@pytest.mark.parametrize("eps", [0.01, 0.2, 0.5, -0.8])
def test_two_by_two_limit(eps):
    """Limit z_21 = lambda_-/eps with lambda_+- = (1 +- sqrt(1+4 eps^2))/2 (Sec. 4.3)."""
    th, de = W.two_by_two(eps)
    r = oracle.ipt_dense(th, de, tol=1e-15, max_iter=2000)
    assert np.all(r.status == oracle.CONVERGED)
    lam_m = (1 - math.sqrt(1 + 4 * eps * eps)) / 2
    lam_p = (1 + math.sqrt(1 + 4 * eps * eps)) / 2
    assert abs(r.z[1, 0] - lam_m / eps) <= 1e-13
    assert abs(r.z[0, 1] + lam_m / eps) <= 1e-13
    assert abs(r.lam[0] - lam_m) <= 1e-14 and abs(r.lam[1] - lam_p) <= 1e-14


@pytest.mark.parametrize("abcd", [(0.0, 0.1, 0.2, 1.0), (2.0, -0.3, 0.1, -1.0), (0.5, 0.05, -0.4, 1.7),
                                  (-1.0, 0.2, 0.2, 0.0)])
def test_general_two_by_two_closed_form(abcd):
    """General real 2x2 [[a,b],[c,d]] (App. D, 2x2 case): with s = d - a and
    r = sqrt(s^2 + 4bc), the continued eigenvectors are (1, -2c/(s + sgn(s) r)) and
    (2b/(s + sgn(s) r), 1) with lambda_1 = a + b z_21, lambda_2 = d + c z_12.  This
    also fixes the orientation G_jk = 1/(theta_j - theta_k) for a non-symmetric M."""
    a, b, c, d = abcd
    th, de = W.general_two_by_two(a, b, c, d)
    r = oracle.ipt_dense(th, de, tol=1e-15, max_iter=2000)
    assert np.all(r.status == oracle.CONVERGED)
    s = d - a
    rr = math.sqrt(s * s + 4 * b * c)
    den = s + math.copysign(rr, s)
    z21, z12 = -2 * c / den, 2 * b / den
    assert abs(r.z[1, 0] - z21) <= 1e-14 and abs(r.z[0, 1] - z12) <= 1e-14
    assert abs(r.lam[0] - (a + b * z21)) <= 1e-14 and abs(r.lam[1] - (d + c * z12)) <= 1e-14
    m = np.array([[a, b], [c, d]])
    ev = np.linalg.eigvals(m)
    assert min(abs(ev - r.lam[0])) <= 1e-13 and min(abs(ev - r.lam[1])) <= 1e-13


@pytest.mark.parametrize("eps", [0.1, 0.3, 0.6])
def test_two_by_two_rate(eps):
    """Asymptotic error ratio |f^k(0) - x*| ~ |1 - sqrt(1+4 eps^2)|^k (Sec. 4.3)."""
    th, de = W.two_by_two(eps)
    t = oracle.ipt_trace(th, de, 0, 60)[:, 1]
    xs = (1 - math.sqrt(1 + 4 * eps * eps)) / 2 / eps
    err = np.abs(t - xs)
    ks = [k for k in range(2, 60) if 1e-13 < err[k] < 1e-3]
    assert len(ks) >= 2
    ratio = (err[ks[-1]] / err[ks[0]]) ** (1.0 / (ks[-1] - ks[0]))
    expect = abs(1 - math.sqrt(1 + 4 * eps * eps))
    assert abs(ratio - expect) <= 0.05 * expect


def test_two_by_two_flip_threshold(golden_dir):
    """Stable for real |eps| < sqrt(3)/2, period-2 cycle past it, divergence at eps = 2
    (Sec. 4.3)."""
    facts = read_facts(os.path.join(golden_dir, "paper_facts.txt"))
    flip = facts["two_by_two_flip_eps"]
    assert abs(flip - math.sqrt(3) / 2) < 1e-15
    for eps in (0.8, -0.8, 0.85):
        th, de = W.two_by_two(eps)
        assert np.all(oracle.ipt_dense(th, de, tol=1e-12, max_iter=5000).status == oracle.CONVERGED)
    th, de = W.two_by_two(0.9)   # past the flip: period-2 cycle, never settles
    r = oracle.ipt_dense(th, de, tol=1e-12, max_iter=400)
    assert np.all(r.status == oracle.NOT_CONVERGED)
    tail = oracle.ipt_trace(th, de, 0, 400)[-4:, 1]
    assert abs(tail[0] - tail[2]) < 1e-9 and abs(tail[0] - tail[1]) > 1e-2
    th, de = W.two_by_two(2.0)   # orbit 0, -2, 6, 70, ... -> infinity
    r = oracle.ipt_dense(th, de, tol=1e-12, max_iter=100)
    assert np.all(r.status == oracle.DIVERGED)
    np.testing.assert_array_equal(oracle.ipt_trace(th, de, 0, 3)[:, 1], [0.0, -2.0, 6.0, 70.0])


# ----------------------------------------------------- brute force and libraries

@pytest.mark.parametrize("n,seed", [(3, 1), (5, 2), (8, 3), (12, 4)])
def test_tiny_vs_cyclic_jacobi(n, seed):
    """Symmetric near-diagonal n <= 12: every column equals the Jacobi eigenvector
    whose largest entry sits at the same index, scaled to 1 there (intermediate
    normalisation, App. B), and lambda equals its eigenvalue."""
    th, de = W.dense_sym_gaussian(n, 0.2, seed)
    ev, vec = cyclic_jacobi(np.diag(th) + de)
    r = oracle.ipt_dense(th, de, tol=1e-15, max_iter=500)
    assert np.all(r.status == oracle.CONVERGED)
    for c in range(n):
        m = int(np.argmax(np.abs(vec[c, :])))   # eigenvector dominated by e_c
        v = vec[:, m] / vec[c, m]
        assert np.max(np.abs(r.z[:, c] - v)) <= 1e-12
        assert abs(r.lam[c] - ev[m]) <= 1e-12


def _weyl_sorted_eigh(th, de):
    ev, vec = np.linalg.eigh(np.diag(th) + de)
    return ev, vec


def test_c1_against_eigh():
    """n = 256, eps = 0.01: |Delta|_2 < half the unit gap, so by Weyl the sorted
    eigenvalues are the continuations of theta = 1..n; LAPACK eigh fixes them."""
    th, de = W.dense_sym_gaussian(256, 0.01, 0)
    assert np.linalg.norm(de, 2) < 0.5
    r = oracle.ipt_dense(th, de, tol=1e-12)
    assert np.all(r.status == oracle.CONVERGED)
    ev, vec = _weyl_sorted_eigh(th, de)
    nm = oracle.norm1(th, de)
    assert np.max(np.abs(r.lam - ev)) <= 1e-12 * nm
    v = vec / np.diag(vec)[None, :]
    assert np.max(np.abs(r.z - v)) <= 1e-11
    assert np.max(r.step) <= 1e-12


def test_paper_dense_family_nonsymmetric():
    """The paper's non-symmetric dense test matrix diag(i) + 0.01 R, R ~ U[0,1]
    (Sec. 6.2): every column converges to an eigenpair of M (checked against
    LAPACK geev by the eigen-equation and by eigenvalue matching)."""
    th, de = W.dense_uniform_nonsym(96, 0.01, 5)
    r = oracle.ipt_dense(th, de, tol=1e-12)
    assert np.all(r.status == oracle.CONVERGED)
    ev = np.linalg.eigvals(np.diag(th) + de)
    for c in range(96):
        assert np.min(np.abs(ev - r.lam[c])) <= 1e-10
    assert np.max(oracle.eigen_residual(th, de, r.z, r.lam)) <= 1e-11


# ----------------------------------------------------------------- RS series

def test_rs_textbook_low_orders():
    """First and second order RS eigenvalue terms are the textbook ones:
    lambda^[1]_i = Delta_ii, lambda^[2]_i = sum_{j != i} Delta_ij Delta_ji/(theta_i - theta_j);
    first-order vectors Z^[1]_ji = Delta_ji/(theta_i - theta_j) (App. B)."""
    th, de = W.dense_uniform_nonsym(10, 1.0, 3)
    lam = oracle.rs_eigenvalues(th, de, 2)
    np.testing.assert_allclose(lam[1], np.diag(de), rtol=0, atol=1e-15)
    l2 = np.array([sum(de[i, j] * de[j, i] / (th[i] - th[j]) for j in range(10) if j != i) for i in range(10)])
    np.testing.assert_allclose(lam[2], l2, rtol=1e-13, atol=1e-15)
    z1 = oracle.rs_series(th, de, 1)[1]
    for i in range(10):
        for j in range(10):
            want = 0.0 if i == j else de[j, i] / (th[i] - th[j])
            assert abs(z1[j, i] - want) <= 1e-15


def _fit_slope(xs, ys):
    return np.polyfit(np.log(xs), np.log(ys), 1)[0]


def test_ipt_contains_rs_series():
    """Z^(k) = Z_RS^(k) + O(eps^{k+1}) (App. C): for k = 2 the gap scales as eps^3,
    and Z* - Z_RS^(2) is O(eps^3) too."""
    n = 24
    th = np.arange(1, n + 1, dtype=np.float64)
    base = W.sym_gaussian(n, 7)
    base = base + np.diag(np.random.default_rng(8).standard_normal(n) * 0.3)  # non-zero diagonal too
    epss = np.array([0.02, 0.01, 0.005, 0.0025])
    gaps, gaps_star = [], []
    zs = oracle.rs_series(th, base, 2)
    for eps in epss:
        de = eps * base
        z2 = np.stack([oracle.ipt_trace(th, de, i, 2)[2] for i in range(n)], axis=1)
        zrs = zs[0] + eps * zs[1] + eps ** 2 * zs[2]
        gaps.append(np.abs(z2 - zrs).max())
        zstar = oracle.ipt_dense(th, de, tol=1e-15).z
        gaps_star.append(np.abs(zstar - zrs).max())
    assert abs(_fit_slope(epss, gaps) - 3.0) <= 0.3
    assert abs(_fit_slope(epss, gaps_star) - 3.0) <= 0.3


# ------------------------------------------------------------- invariants

def test_invariants_and_subset():
    """Z_ii = 1 exactly, lambda = (M Z)_ii, small eigen-residual, the k-column solve
    equals the same columns of the full solve bit for bit (column independence,
    Sec. 3), and the columns are not collinear (Thm. theorem-rank)."""
    th, de = W.dense_sym_gaussian(64, 0.05, 11)
    full = oracle.ipt_dense(th, de, tol=1e-13)
    assert np.all(full.status == oracle.CONVERGED)
    assert np.all(np.diag(full.z) == 1.0)
    mz = np.diag(th) @ full.z + de @ full.z
    assert np.max(np.abs(np.diag(mz) - full.lam)) <= 1e-13
    assert np.max(full.resid) <= 1e-11
    idx = np.array([5, 0, 63, 17], dtype=np.int32)
    sub = oracle.ipt_dense(th, de, idx=idx, tol=1e-13)
    np.testing.assert_array_equal(sub.z, full.z[:, idx])
    np.testing.assert_array_equal(sub.lam, full.lam[idx])
    sv = np.linalg.svd(full.z, compute_uv=False)
    assert sv.min() > 0.5
    cosines = np.abs((full.z / np.linalg.norm(full.z, axis=0)).T @ (full.z / np.linalg.norm(full.z, axis=0)))
    assert np.max(cosines - np.eye(64)) < 0.5


def test_fixed_point_residual_identity():
    """At any Z with Z_ii = 1: F(Z) - Z = -G o (M Z - Z diag(theta + d)), d = D(Delta Z),
    which follows from rewriting the eigen-equations of Sec. 3; checked per column on
    the oracle's map."""
    rng = np.random.default_rng(3)
    n = 40
    th, de = W.dense_uniform_nonsym(n, 0.3, 2)
    z = rng.standard_normal((n, n)) * 0.1
    g = oracle.inverse_gaps(th)
    m = np.diag(th) + de
    for i in range(n):
        zc = z[:, i].copy()
        zc[i] = 1.0
        w, d = oracle.ipt_map(th, de, i, zc)
        r = m @ zc - zc * (th[i] + d)
        want = -g[:, i] * r
        assert abs(d - (de @ zc)[i]) <= 1e-14
        lhs = w - zc
        lhs[i] = 0.0
        assert np.max(np.abs(lhs - want)) <= 1e-13 * max(1.0, np.abs(want).max())


def test_theorem1_contraction(golden_dir):
    """|G||Delta| < 3 - 2 sqrt 2 implies convergence from I and every iterate inside
    B_sqrt2(I) (Thm. main-th).  n = 256, eps = 0.01: |G| ~ pi, |Delta| ~ 0.014."""
    facts = read_facts(os.path.join(golden_dir, "paper_facts.txt"))
    assert abs(facts["theorem1_bound"] - (3 - 2 * math.sqrt(2))) < 1e-15
    th, de = W.dense_sym_gaussian(256, 0.01, 0)
    gnorm = np.linalg.norm(oracle.inverse_gaps(th), 2)
    dnorm = np.linalg.norm(de, 2)
    assert gnorm * dnorm < facts["theorem1_bound"]
    its = np.stack([oracle.ipt_trace(th, de, i, 6) for i in range(256)], axis=2)  # (7, n, n)
    for k in range(its.shape[0]):
        assert np.linalg.norm(its[k] - np.eye(256), 2) <= facts["theorem1_radius"]
    r = oracle.ipt_dense(th, de, tol=1e-12)
    assert np.all(r.status == oracle.CONVERGED)


# ---------------------------------------------------------------- 3x3 (App. D)

def _chart_jacobian(th, de, i, z, h=1e-6):
    n = th.shape[0]
    jac = np.zeros((n, n))
    for s in range(n):
        if s == i:
            continue
        zp, zm = z.copy(), z.copy()
        zp[s] += h
        zm[s] -= h
        jac[:, s] = (oracle.ipt_map(th, de, i, zp)[0] - oracle.ipt_map(th, de, i, zm)[0]) / (2 * h)
    keep = [j for j in range(n) if j != i]
    return jac[np.ix_(keep, keep)]


def _poly_eval(terms, eps, mu):
    val = sum(c * eps ** a * mu ** b for c, a, b in terms)
    mag = sum(abs(c * eps ** a * mu ** b) for c, a, b in terms)
    return abs(val) / mag


@pytest.mark.parametrize("col", [0, 1, 2])
@pytest.mark.parametrize("eps", [0.1, 0.2, -0.25])
def test_three_by_three_multipliers_on_printed_curve(golden_dir, col, eps):
    """The multipliers of the oracle's fixed point of f_i (eigenvalues of the chart
    Jacobian, by central differences of the oracle's map) are roots of the printed
    polynomials P(eps, mu) of App. D."""
    polys = read_polys(os.path.join(golden_dir, "three_by_three_multiplier_polys.txt"))
    th, de = W.three_by_three(eps)
    r = oracle.ipt_dense(th, de, idx=np.array([col], np.int32), tol=1e-15, max_iter=2000)
    assert r.status[0] == oracle.CONVERGED
    mus = np.linalg.eigvals(_chart_jacobian(th, de, col, r.z[:, 0]))
    for mu in mus:
        assert _poly_eval(polys["z%d" % (col + 1)], eps, mu) < 1e-8
    # and a perturbed map (sign of Delta flipped in the map) would not be on the curve
    wrong = np.linalg.eigvals(_chart_jacobian(th, -de, col, oracle.ipt_dense(
        th, -de, idx=np.array([col], np.int32), tol=1e-15, max_iter=2000).z[:, 0]))
    assert max(_poly_eval(polys["z%d" % (col + 1)], eps, mu) for mu in wrong) > 1e-6


def _continued_eigvec(th, p, i, eps_target, steps=400):
    """Eigenvector of diag(th) + eps p continued from e_i at eps = 0 (tracking by
    overlap), scaled to entry i = 1."""
    v_prev = np.eye(th.shape[0])[:, i]
    for eps in np.linspace(0.0, eps_target, steps)[1:]:
        ev, vec = np.linalg.eig(np.diag(th) + eps * p)
        j = int(np.argmax(np.abs(vec.T.conj() @ v_prev)))
        v_prev = vec[:, j] / np.linalg.norm(vec[:, j])
    return np.real(v_prev / v_prev[i])


def test_three_by_three_neimark_sacker(golden_dir):
    """For the second column, the continued fixed point loses stability (spectral
    radius of the chart Jacobian crosses 1 with a complex pair) at eps ~ -0.49
    (App. D)."""
    facts = read_facts(os.path.join(golden_dir, "paper_facts.txt"))
    th, p = W.three_by_three(1.0)

    def radius(eps):
        z = _continued_eigvec(th, p, 1, eps)
        mus = np.linalg.eigvals(_chart_jacobian(th, eps * p, 1, z))
        return np.max(np.abs(mus)), mus

    lo, hi = -0.45, -0.55
    r_lo, _ = radius(lo)
    r_hi, _ = radius(hi)
    assert r_lo < 1.0 < r_hi
    for _ in range(20):
        mid = 0.5 * (lo + hi)
        if radius(mid)[0] < 1.0:
            lo = mid
        else:
            hi = mid
    assert abs(lo - facts["three_by_three_z2_neimark_sacker_eps"]) <= 0.01
    _, mus = radius(lo)
    assert np.all(np.abs(np.imag(mus)) > 1e-3)   # complex pair: Neimark-Sacker, not a flip


# ---------------------------------------------------------------- sparse, Morgan

def test_csr_matches_dense():
    """The CSR oracle equals the dense oracle on the same matrix bit for bit
    (entries summed in the same ascending column order)."""
    th, rp, col, val = W.sparse_sym_uniform(300, seed=4)
    dense = np.zeros((300, 300))
    for j in range(300):
        dense[j, col[rp[j]:rp[j + 1]]] = val[rp[j]:rp[j + 1]]
    idx = W.lowest_indices(th, 16)
    a = oracle.ipt_csr(th, rp, col, val, idx, tol=1e-12)
    b = oracle.ipt_dense(th, dense, idx=idx, tol=1e-12)
    np.testing.assert_array_equal(a.z, b.z)
    np.testing.assert_array_equal(a.lam, b.lam)
    assert np.all(a.status == oracle.CONVERGED)


def test_morgan_threshold(golden_dir):
    """Morgan's tridiagonal matrix (Sec. 6.1): the ground state converges at
    off-diagonal 0.5 (slowly: tens of sweeps), convergence slows sharply just past
    0.5, and it is lost for larger off-diagonals (Sec. 6.1, failure study)."""
    facts = read_facts(os.path.join(golden_dir, "paper_facts.txt"))
    off = facts["morgan_ipt_failure_offdiag"]
    idx = np.array([0], np.int32)
    sweeps = {}
    for o in (off, off + 0.1):
        th, rp, col, val = W.morgan_tridiagonal(5000, o)
        r = oracle.ipt_csr(th, rp, col, val, idx, tol=1e-12, max_iter=5000)
        assert r.status[0] == oracle.CONVERGED
        sweeps[o] = int(r.sweeps[0])
        if o == off:
            dense = np.diag(th[:400]) + np.diag(np.full(399, o), 1) + np.diag(np.full(399, o), -1)
            assert abs(r.lam[0] - np.linalg.eigvalsh(dense)[0]) < 1e-10
    assert sweeps[off] > 20 and sweeps[off + 0.1] > 2 * sweeps[off]
    th, rp, col, val = W.morgan_tridiagonal(5000, off + 0.25)
    r = oracle.ipt_csr(th, rp, col, val, idx, tol=1e-12, max_iter=5000)
    assert r.status[0] != oracle.CONVERGED


def test_warm_start_resume_bitwise():
    """A solve stopped after t sweeps and resumed from its returned iterate reaches
    the same certified columns as the uninterrupted solve, bit for bit (the iterate
    is the whole state; initial guesses, Sec. 7)."""
    th, de = W.dense_sym_gaussian(128, 0.03, 2)
    full = oracle.ipt_dense(th, de, tol=1e-12)
    part = oracle.ipt_dense(th, de, tol=1e-12, max_iter=2)
    assert np.all(part.status == oracle.NOT_CONVERGED)
    res = oracle.ipt_dense(th, de, z0=part.z, tol=1e-12)
    np.testing.assert_array_equal(res.z, full.z)
    np.testing.assert_array_equal(res.lam, full.lam)
    np.testing.assert_array_equal(res.sweeps + 2, full.sweeps)


def test_divergence_isolated_to_column():
    """Columns are independent fixed-point problems (Sec. 3): one gap-violating pair
    (|Delta_34| past the 2x2 flip threshold relative to its unit gap) breaks only the
    columns of that pair, every other column still converges.  A non-finite entry
    in a row of Delta reaches every column's product, so all columns diverge."""
    th, de = W.dense_sym_gaussian(32, 0.01, 9)
    de = de.copy()
    de[3, 4] = de[4, 3] = 0.95
    r = oracle.ipt_dense(th, de, tol=1e-12, max_iter=300)
    bad = np.where(r.status != oracle.CONVERGED)[0]
    assert set(bad.tolist()) <= {3, 4} and len(bad) >= 1
    de2 = de.copy()
    de2[10, :] = np.nan
    r2 = oracle.ipt_dense(th, de2, tol=1e-12)
    assert np.all(r2.status == oracle.DIVERGED)


@pytest.mark.slow
def test_large_dense_sampled_columns_against_eigh():
    """n = 4096, eps in {0.01, 0.05} (the large full-spectrum case) on sampled
    columns: by Weyl (|Delta|_2 < 1/2 = half the gap) the sorted eigh eigenpairs
    are the continuations; the oracle's columns match them."""
    for eps in (0.01, 0.05):
        th, de = W.dense_sym_gaussian(4096, eps, 0)
        ev, vec = np.linalg.eigh(np.diag(th) + de)
        idx = np.array([0, 1, 777, 2048, 4000, 4095], dtype=np.int32)
        r = oracle.ipt_dense(th, de, idx=idx, tol=1e-10, resid=False)
        assert np.all(r.status == oracle.CONVERGED)
        nm = oracle.norm1(th, de)
        assert np.max(np.abs(r.lam - ev[idx])) <= 1e-12 * nm
        v = vec[:, idx] / vec[idx, idx][None, :]
        assert np.max(np.abs(r.z - v)) <= 1e-9


def test_family_lowest_columns_against_eigh():
    """The M(eps) = diag(1..1024) + eps R family, k = 32 lowest columns."""
    th, base = W.family_base(1024, 0)
    for eps in (0.0, 0.03, 0.08):
        de = eps * base
        idx = W.lowest_indices(th, 32)
        r = oracle.ipt_dense(th, de, idx=idx, tol=1e-12)
        assert np.all(r.status == oracle.CONVERGED)
        ev, vec = np.linalg.eigh(np.diag(th) + de)
        assert np.max(np.abs(r.lam - ev[:32])) <= 1e-12 * oracle.norm1(th, de)


def test_sparse_residual_and_window():
    """Sparse symmetric perturbation, n = 200000, k = 16 lowest: each returned pair
    has |M z - lambda z| / (|M|_1 |z|) <= 1e-10 (so an eigenvalue of M lies that
    close in units of |M|_1, by the symmetric residual bound) and lambda stays in
    the Weyl window of theta_i."""
    th, rp, col, val = W.sparse_sym_uniform(200000, seed=0)
    idx = W.lowest_indices(th, 16)
    r = oracle.ipt_csr(th, rp, col, val, idx, tol=1e-10)
    assert np.all(r.status == oracle.CONVERGED)
    assert np.max(r.resid) <= 1e-10 * oracle.norm1(th, csr=(rp, col, val))
    assert np.all(np.abs(r.lam - th[idx]) < 0.5)
    assert np.all(r.z[idx, np.arange(16)] == 1.0)

"""Pins of the oracle's near-degenerate pair rotation (the choice of D per pair, from
the concluding section's suggestion of using the freedom in D to widen the domain of
convergence): closed forms of the 2x2 rotation, similarity invariants, the pairing
rule's cases, and the rotated IPT solve against a textbook eigensolver."""
import numpy as np

import oracle
import workloads as W


def test_two_by_two_closed_form():
    """The rotated 2x2 block is diag of the closed-form eigenvalues and has no coupling."""
    for a, d, b in ((1.0, 1.1, 0.2), (0.0, -0.05, 0.3), (2.0, 2.0, -0.1)):
        th = np.array([a, d])
        de = np.array([[0.0, b], [b, 0.0]])
        t2, d2, partner, cs = oracle.pair_rotation(th, de, 0.05)
        m, h = (a + d) / 2.0, np.hypot((a - d) / 2.0, b)
        assert list(partner) == [1, 0]
        np.testing.assert_allclose(np.sort(t2), [m - h, m + h], rtol=0, atol=1e-15)
        assert np.all(d2 == 0.0)
        c, s = cs[0]
        assert abs(c * c + s * s - 1.0) < 1e-15 and c >= np.sqrt(0.5) - 1e-15  # |angle| <= pi/4


def test_diagonal_of_delta_is_part_of_the_block():
    """The 2x2 block is that of M = diag(theta) + Delta, diagonal of Delta included."""
    th = np.array([1.0, 1.3])
    de = np.array([[0.2, 0.25], [0.25, -0.05]])
    t2, d2, _, _ = oracle.pair_rotation(th, de, 0.05)
    np.testing.assert_allclose(np.sort(t2), np.linalg.eigvalsh(np.diag(th) + de), rtol=0, atol=1e-15)
    assert np.all(d2 == 0.0)


def _planted(n, pairs, seed, strength=1.5):
    rng = np.random.default_rng(seed)
    th = np.arange(1.0, n + 1.0)
    r = rng.standard_normal((n, n)) * 0.01 / np.sqrt(n)
    de = (r + r.T) / 2.0
    for i, j in pairs:
        th[j] = th[i] + 0.02
        de[i, j] = de[j, i] = strength * 0.02
    return th, de


def test_similarity_invariants():
    """M' = R^T M R: same spectrum, pairs decoupled, unpaired entries untouched, and
    back-rotation of M' eigenvectors gives eigenvectors of M."""
    th, de = _planted(24, [(3, 4), (10, 11), (20, 21)], 1)
    t2, d2, partner, cs = oracle.pair_rotation(th, de, 0.05)
    assert sorted((i, int(partner[i])) for i in range(24) if partner[i] > i) == [(3, 4), (10, 11), (20, 21)]
    M, M2 = np.diag(th) + de, np.diag(t2) + d2
    np.testing.assert_allclose(np.linalg.eigvalsh(M2), np.linalg.eigvalsh(M), rtol=0, atol=1e-13)
    for i, j in ((3, 4), (10, 11), (20, 21)):
        assert d2[i, j] == 0.0 and d2[j, i] == 0.0 and d2[i, i] == 0.0
    free = partner < 0
    assert np.array_equal(d2[np.ix_(free, free)], de[np.ix_(free, free)])
    assert np.array_equal(t2[free], th[free])
    w, V = np.linalg.eigh(M2)
    Z = oracle.pair_back_rotate(V, partner, cs)
    assert np.abs(M @ Z - Z * w).max() < 1e-13


def test_pairing_rule_cases():
    """Mutual strongest partners above tau pair; one-sided, weak or asymmetric do not."""
    th = np.array([0.0, 1.0, 1.05, 3.0, 3.5, 6.0])
    de = np.zeros((6, 6))
    de[1, 2] = de[2, 1] = 0.01      # ratio 0.2: pairs
    de[3, 4] = de[4, 3] = 0.01      # ratio 0.02 < tau: no pair
    de[0, 5] = 0.5; de[5, 0] = 0.4  # strong but asymmetric: no pair
    partner, rmax = oracle.pair_partners(th, de, 0.05)
    assert list(partner) == [-1, 2, 1, -1, -1, -1]
    np.testing.assert_allclose(rmax[1], 0.2, rtol=1e-15)
    # one-sided: 1's strongest is 2 but 2's strongest is 3
    de2 = de.copy()
    de2[2, 3] = de2[3, 2] = 0.5     # ratio 0.26 > 0.2 for row 2
    partner2, _ = oracle.pair_partners(th, de2, 0.05)
    assert partner2[1] == -1 and partner2[2] == 3 and partner2[3] == 2
    # ties: the first index wins
    th3 = np.array([0.0, 1.0, -1.0])
    de3 = np.zeros((3, 3)); de3[0, 1] = de3[1, 0] = de3[0, 2] = de3[2, 0] = 0.3
    partner3, _ = oracle.pair_partners(th3, de3, 0.05)
    assert partner3[0] == 1 and partner3[1] == 0 and partner3[2] == -1


def test_rotated_solve_recovers_strong_pairs():
    """Planted pairs coupled beyond the 2x2 convergence bound (ratio 1.5 > sqrt(3)/2):
    plain IPT fails on them, the rotated solve converges on every column and matches a
    textbook eigensolver; a mistake in the back-rotation (wrong sign of s) is caught."""
    pairs = [(5, 6), (17, 18)]
    th, de = _planted(32, pairs, 2)
    ns = np.array([32], np.int32)
    off = np.array([0], np.int64)
    plain = oracle.ipt_batched(ns, th, de.ravel(), off, off, tol=1e-12, max_iter=200)
    assert np.any(plain.status[[5, 6, 17, 18]] != 0)
    rot = oracle.ipt_batched(ns, th, de.ravel(), off, off, tol=1e-12, max_iter=200, pair_tau=0.05)
    assert np.all(rot.status == 0)
    M = np.diag(th) + de
    Z = rot.z.reshape(32, 32)
    nrm = np.abs(M).sum(0).max()
    assert np.abs(M @ Z - Z * rot.lam).max() <= 1e-10 * nrm * np.abs(Z).max()
    np.testing.assert_allclose(np.sort(rot.lam), np.linalg.eigvalsh(M), rtol=0, atol=1e-10 * nrm)
    # chart of a paired column: (R^T z)_i = 1
    t2, d2, partner, cs = oracle.pair_rotation(th, de, 0.05)
    c, s = cs[5]
    np.testing.assert_allclose(c * Z[5, 5] - s * Z[6, 5], 1.0, rtol=0, atol=1e-14)
    # mutant: back-rotation with the wrong sign of s no longer gives eigenvectors
    r2 = oracle.ipt_dense(t2, d2, tol=1e-12, max_iter=200, resid=False)
    bad = oracle.pair_back_rotate(r2.z, partner, cs * np.array([1.0, -1.0]))
    assert np.abs(M @ bad - bad * r2.lam).max() > 1e-4


def test_batched_workload_failures_recovered():
    """On problems of the batched workload whose plain solve leaves columns
    unconverged, the rotated solve converges on more columns and its converged
    eigenpairs are eigenpairs of the original matrix."""
    ns = W.batched_sizes(4096, 32, 512, 0)
    picked = [b for b in range(40) if ns[b] <= 160][:12]
    n_sel = np.array([ns[b] for b in picked], np.int32)
    th = np.concatenate([W.batched_problem(b, int(ns[b]), 0.02, 0)[0] for b in picked])
    de = np.concatenate([W.batched_problem(b, int(ns[b]), 0.02, 0)[1].ravel() for b in picked])
    toff = np.concatenate([[0], np.cumsum(n_sel)[:-1]]).astype(np.int64)
    doff = np.concatenate([[0], np.cumsum(n_sel.astype(np.int64) ** 2)[:-1]]).astype(np.int64)
    plain = oracle.ipt_batched(n_sel, th, de, toff, doff, tol=1e-10, max_iter=64)
    rot = oracle.ipt_batched(n_sel, th, de, toff, doff, tol=1e-10, max_iter=64, pair_tau=0.05)
    assert (rot.status == 0).sum() >= (plain.status == 0).sum()
    for q, b in enumerate(picked):
        n = int(n_sel[q]); to, do = int(toff[q]), int(doff[q])
        M = np.diag(th[to:to + n]) + de[do:do + n * n].reshape(n, n)
        Z = rot.z[do:do + n * n].reshape(n, n)
        ok = rot.status[to:to + n] == 0
        lam = rot.lam[to:to + n]
        res = np.linalg.norm(M @ Z[:, ok] - Z[:, ok] * lam[ok], axis=0) / np.linalg.norm(Z[:, ok], axis=0)
        assert res.max() <= 1e-9 * np.abs(M).sum(0).max()


def test_choose_d_partition():
    """choose_d keeps the matrix (to the rounding of theta'): same spectrum as M; the
    diagonal of Delta' is minus the second-order shift; the shift is the RS
    second-order energy of the folded partition (checked against rs_eigenvalues at
    order 2 for a matrix with no pairs)."""
    th, de = _planted(20, [(4, 5)], 3)
    de = de + np.diag(np.linspace(-0.01, 0.01, 20))
    t3, d3, partner, cs = oracle.choose_d(th, de, 0.05)
    M = np.diag(th) + de
    np.testing.assert_allclose(np.linalg.eigvalsh(np.diag(t3) + d3), np.linalg.eigvalsh(M), rtol=0, atol=1e-13)
    # no pairs: theta' is the second-order RS eigenvalue estimate of (theta + diag, offdiag)
    th2, de2 = _planted(16, [], 4)
    t3b, d3b, p2, _ = oracle.choose_d(th2, de2, 0.05)
    assert np.all(p2 < 0)
    off = de2 - np.diag(np.diag(de2))
    rs = oracle.rs_eigenvalues(th2 + np.diag(de2), off, 2)  # per-order terms lambda^[0..2]
    np.testing.assert_allclose(t3b, rs[0] + rs[1] + rs[2], rtol=0, atol=1e-14)
    np.testing.assert_allclose(np.diag(d3b), -(t3b - (th2 + np.diag(de2))), rtol=0, atol=1e-14)


def test_choose_d_recovers_level_shift_failures():
    """A pair with a small coupling but a gap smaller than the difference of the two
    levels' shifts: plain IPT diverges on it; with the shifts in D every column
    converges, and the eigenpairs match a textbook eigensolver."""
    n = 24
    rng = np.random.default_rng(9)
    th = np.arange(1.0, n + 1.0)
    r = rng.standard_normal((n, n)) * 0.01 / np.sqrt(n)
    de = (r + r.T) / 2.0
    th[11] = th[10] + 2e-4
    de[10, 10], de[11, 11] = 1.5e-3, -1.5e-3   # shift difference 3e-3 >> gap 2e-4
    de[10, 11] = de[11, 10] = 1e-6
    ns = np.array([n], np.int32); off = np.array([0], np.int64)
    plain = oracle.ipt_batched(ns, th, de.ravel(), off, off, tol=1e-12, max_iter=200)
    assert np.any(plain.status[[10, 11]] != 0)
    got = oracle.ipt_batched(ns, th, de.ravel(), off, off, tol=1e-12, max_iter=200, pair_tau=0.05)
    assert np.all(got.status == 0)
    M = np.diag(th) + de
    Z = got.z.reshape(n, n)
    np.testing.assert_allclose(np.sort(got.lam), np.linalg.eigvalsh(M), rtol=0, atol=1e-11)
    assert np.abs(M @ Z - Z * got.lam).max() <= 1e-10 * np.abs(Z).max()

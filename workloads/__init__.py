"""Seeded synthetic inputs for the IPT eigensolver (shared by the oracle side and
the HIP side; this module holds none of the method's arithmetic).

Every generator returns plain float64 / int32 NumPy arrays built on the host from
``numpy.random.default_rng`` (PCG64), filled in row-major order.  Shapes and value
distributions follow the paper's workloads:

* near-diagonal dense ``M = D + Delta`` with ``D = diag(1..n)`` (Sec. 6, eq. for the
  dense test matrices, here with a centred symmetric Gaussian perturbation),
* the paper's own dense family ``diag(i) + eps*R`` with ``R`` iid U[0,1] (Sec. 6.2),
* the sparse symmetric perturbation of a diagonal (Sec. 6.1, "few eigenvalues"),
* the tridiagonal Morgan matrix ``M_ii = i``, ``M_{i,i+-1} = 0.5`` (Sec. 6.1),
* the explicit 2x2 and 3x3 examples (Sec. 4.3 and App. D),
* a batch of small dense problems of uneven size, and the one-parameter family
  ``M(eps) = D + eps*R`` used for learned warm starts.

The split ``M = D + Delta`` is returned as ``theta = diag(D)`` and ``Delta``; the
diagonal of ``Delta`` may be non-zero and is never folded into ``theta``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sym_gaussian",
    "dense_sym_gaussian",
    "dense_uniform_nonsym",
    "sparse_sym_uniform",
    "morgan_tridiagonal",
    "two_by_two",
    "general_two_by_two",
    "three_by_three",
    "batched_sizes",
    "batched_sym_gaussian",
    "batched_problem",
    "family_base",
    "family_eps",
    "lowest_indices",
]


def sym_gaussian(n: int, seed: int = 0) -> np.ndarray:
    """(R + R^T)/2 with R iid N(0, 1/n), drawn row-major from PCG64(seed)."""
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((n, n)) / np.sqrt(n)
    return (r + r.T) / 2.0


def dense_sym_gaussian(n: int, eps: float, seed: int = 0):
    """theta = 1..n, Delta = eps * (R + R^T)/2, R iid N(0, 1/n).

    The full-spectrum workloads: n = 256, eps = 0.01 (small case) and n = 4096,
    eps in {0.01, 0.05} (large case)."""
    theta = np.arange(1, n + 1, dtype=np.float64)
    delta = eps * sym_gaussian(n, seed)
    return theta, np.ascontiguousarray(delta)


def dense_uniform_nonsym(n: int, eps: float = 0.01, seed: int = 0):
    """The paper's dense test family diag(i) + eps*R_n with R_n iid U[0,1]
    (non-centred, non-symmetric)."""
    rng = np.random.default_rng(seed)
    theta = np.arange(1, n + 1, dtype=np.float64)
    delta = eps * rng.uniform(0.0, 1.0, size=(n, n))
    return theta, np.ascontiguousarray(delta)


def sparse_sym_uniform(n: int, pairs_per_row: int = 6, amp: float = 0.05, seed: int = 0):
    """Sparse symmetric perturbation of diag(1..n) in CSR form.

    Draws ``pairs_per_row*n`` index pairs (a, b) uniform on [0, n)^2, drops a == b,
    gives each pair a value U(-amp, amp), mirrors it to (b, a), sums duplicates and
    sorts column indices inside each row (about 12 stored entries per row for the
    default 6 pairs).  Returns theta, row_ptr (int32, n+1), col (int32), val (f64).
    """
    rng = np.random.default_rng(seed)
    m = pairs_per_row * n
    a = rng.integers(0, n, size=m)
    b = rng.integers(0, n, size=m)
    v = rng.uniform(-amp, amp, size=m)
    keep = a != b
    a, b, v = a[keep], b[keep], v[keep]
    rows = np.concatenate([a, b]).astype(np.int64)
    cols = np.concatenate([b, a]).astype(np.int64)
    vals = np.concatenate([v, v])
    return (np.arange(1, n + 1, dtype=np.float64),) + _coo_to_csr(n, rows, cols, vals)


def _coo_to_csr(n, rows, cols, vals):
    """COO -> CSR, duplicates summed in their order of appearance, columns sorted."""
    order = np.lexsort((cols, rows))  # stable: equal (row, col) keep appearance order
    rows, cols, vals = rows[order], cols[order], vals[order]
    key = rows * n + cols
    first = np.ones(key.shape[0], dtype=bool)
    first[1:] = key[1:] != key[:-1]
    seg = np.cumsum(first) - 1
    out_vals = np.zeros(int(first.sum()), dtype=np.float64)
    np.add.at(out_vals, seg, vals)
    out_rows = rows[first]
    out_cols = cols[first].astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, out_rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, out_cols, out_vals


def morgan_tridiagonal(n: int = 5000, off: float = 0.5):
    """Morgan's tridiagonal matrix: M_ii = i (1-based), M_{i,i+-1} = off, as CSR.

    theta = 1..n and Delta holds only the two off-diagonals."""
    rows, cols = [], []
    idx = np.arange(n - 1, dtype=np.int64)
    rows = np.concatenate([idx, idx + 1])
    cols = np.concatenate([idx + 1, idx])
    vals = np.full(rows.shape[0], float(off))
    return (np.arange(1, n + 1, dtype=np.float64),) + _coo_to_csr(n, rows, cols, vals)


def two_by_two(eps: float):
    """The explicit 2x2 example M = [[0, eps], [eps, 1]] split as D = diag(0, 1)."""
    theta = np.array([0.0, 1.0])
    delta = np.array([[0.0, eps], [eps, 0.0]])
    return theta, delta


def general_two_by_two(a: float, b: float, c: float, d: float):
    """M = [[a, b], [c, d]] split as D = diag(a, d), Delta = [[0, b], [c, 0]]."""
    return np.array([a, d], dtype=np.float64), np.array([[0.0, b], [c, 0.0]])


def three_by_three(eps: float):
    """The explicit 3x3 example of App. D: D = diag(0, 1, 3), Delta = eps*P with
    P = [[0,1,2],[1,0,3],[2,3,0]]."""
    theta = np.array([0.0, 1.0, 3.0])
    p = np.array([[0.0, 1.0, 2.0], [1.0, 0.0, 3.0], [2.0, 3.0, 0.0]])
    return theta, eps * p


def batched_sizes(count: int = 4096, nmin: int = 32, nmax: int = 512, seed: int = 0) -> np.ndarray:
    """Problem sizes n_b ~ U{nmin..nmax} for the batched workload."""
    rng = np.random.default_rng(seed)
    return rng.integers(nmin, nmax + 1, size=count).astype(np.int32)


def batched_problem(b: int, n: int, eps: float = 0.02, seed: int = 0):
    """Problem b of the batch: theta = sort(U(0, n)), Delta = eps*(R+R^T)/2 with
    R iid N(0, 1/n).  Each problem has its own stream PCG64([seed, 1, b]) so any
    subset can be regenerated on its own."""
    rng = np.random.default_rng([seed, 1, b])
    theta = np.sort(rng.uniform(0.0, float(n), size=n))
    r = rng.standard_normal((n, n)) / np.sqrt(n)
    return theta, np.ascontiguousarray(eps * (r + r.T) / 2.0)


def batched_sym_gaussian(count: int = 4096, nmin: int = 32, nmax: int = 512,
                         eps: float = 0.02, seed: int = 0):
    """The whole batch packed into pools: returns (ns, theta_pool, delta_pool,
    theta_off, delta_off) with problem b's theta at theta_pool[theta_off[b]:][:n_b]
    and its row-major n_b x n_b Delta at delta_pool[delta_off[b]:][:n_b*n_b]."""
    ns = batched_sizes(count, nmin, nmax, seed)
    theta_off = np.zeros(count, dtype=np.int64)
    delta_off = np.zeros(count, dtype=np.int64)
    theta_off[1:] = np.cumsum(ns.astype(np.int64))[:-1]
    delta_off[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
    theta_pool = np.empty(int(ns.sum()), dtype=np.float64)
    delta_pool = np.empty(int((ns.astype(np.int64) ** 2).sum()), dtype=np.float64)
    for b in range(count):
        n = int(ns[b])
        th, de = batched_problem(b, n, eps, seed)
        theta_pool[theta_off[b]:theta_off[b] + n] = th
        delta_pool[delta_off[b]:delta_off[b] + n * n] = de.ravel()
    return ns, theta_pool, delta_pool, theta_off, delta_off


def family_base(n: int = 1024, seed: int = 0):
    """The one-parameter family M(eps) = diag(1..n) + eps*R, R = (R'+R'^T)/2 with
    R' iid N(0, 1/n).  Returns theta and R (the perturbation at eps = 1)."""
    return np.arange(1, n + 1, dtype=np.float64), np.ascontiguousarray(sym_gaussian(n, seed))


def family_eps(count: int, lo: float = 0.0, hi: float = 0.08, seed: int = 1) -> np.ndarray:
    """Family parameters eps ~ U[lo, hi] (training draws use seed 1, test draws seed 2)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=count)


def lowest_indices(theta: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k smallest unperturbed eigenvalues (the requested columns for
    "k lowest" solves), as int32."""
    return np.argsort(theta, kind="stable")[:k].astype(np.int32)

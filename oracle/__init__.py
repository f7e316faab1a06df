"""Oracle for the IPT eigensolver -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct FP64 CPU implementation of what the HIP path
computes.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it; the product library never does, and the two share no code
(the seeded input generators in ``workloads`` are the only common module).

Contents
* ``ipt_dense`` / ``ipt_csr``: Alg. 1 applied independently to each requested
  column (equivalently Alg. 2 / the matrix map F of eq. dyn restricted to those
  columns), in plain C (``ipt_oracle.c``, FP64, fixed summation order).
* ``ipt_trace`` / ``ipt_map``: the iterates of f_i (eq. single_line_dyn) with no
  stopping test, and a single application of f_i.
* ``ipt_batched``: a loop of independent dense problems.
* ``rs_series``: the Rayleigh-Schroedinger corrections Z^[l] of eq. ARS-alpha
  (App. B, eq. RS-recursion), in NumPy.
* ``acx_dense``: IPT with Alternating Cyclic Extrapolation (Alg. ACX) per column,
  in NumPy.
* ``ipt_dense_z``: IPT over C^n (complex theta, Delta, z), in the C oracle.
* ``ipt_dense_homotopy``: the homotopy restart of the concluding section (stages
  D + (q/Q) Delta, each started from the previous stage's vectors).
* ``ipt_dense_cont``: the non-autonomous continuation of the concluding discussion
  (the perturbation scaled by 1 - alpha^t at sweep t), in the C oracle.
* ``norm1`` / ``eigen_residual``: the plain definitions used by the parity bounds.
* ``pair_partners`` / ``pair_rotation`` / ``choose_d`` / ``pair_back_rotate``: a
  choice of D (the concluding section's suggestion of choosing D to widen the
  convergence domain): near-degenerate pairs rotated out by 2x2 Jacobi rotations of
  M, then the first- and second-order level shifts moved into D, in NumPy;
  ``ipt_batched`` applies it with ``pair_tau``.

Every function cites the passage it follows; the readings taken where the paper
is silent are stated in ``ipt_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "ipt_oracle.c")

CONVERGED, NOT_CONVERGED, DIVERGED = 0, 1, 2
DEFAULT_MAX_ITER = 100
DEFAULT_DIV_NORM = 1.0e3
DEFAULT_DIV_GROWTH = 8


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = C.CDLL(_LIB_PATH)
        d, i64, i32, p = C.c_double, C.c_int64, C.c_int32, C.c_void_p
        lib.oracle_ipt_dense.argtypes = [i64, p, p, i64, i64, p, p, i64, d, C.c_int, d, C.c_int,
                                         p, i64, p, p, p, p, p]
        lib.oracle_ipt_csr.argtypes = [i64, p, p, p, p, i64, p, p, i64, d, C.c_int, d, C.c_int,
                                       p, i64, p, p, p, p, p]
        lib.oracle_ipt_dense_acx.argtypes = lib.oracle_ipt_dense.argtypes
        lib.oracle_ipt_dense_cont.argtypes = [i64, p, p, i64, i64, p, p, i64, d, d, C.c_int, d, C.c_int,
                                              p, i64, p, p, p, p, p]
        lib.oracle_ipt_dense_z.argtypes = lib.oracle_ipt_dense.argtypes
        lib.oracle_ipt_csr_acx.argtypes = lib.oracle_ipt_csr.argtypes
        lib.oracle_ipt_trace.argtypes = [i64, p, p, i64, i64, p, C.c_int, p]
        lib.oracle_ipt_map.argtypes = [i64, p, p, i64, i64, p, p]
        lib.oracle_ipt_map.restype = d
        lib.oracle_ipt_batched.argtypes = [i32, p, p, p, p, p, p, d, C.c_int, d, C.c_int, p, p, p, p]
        lib.oracle_set_threads.argtypes = [C.c_int]
        lib.oracle_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def swap_library(path):
    """Point the wrappers at another build of ipt_oracle.c (used by the tests that
    plant a mistake in a copy of the oracle); returns the previous path."""
    global _lib, _LIB_PATH
    prev = _LIB_PATH
    _lib, _LIB_PATH = None, path
    return prev


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


class Result(dict):
    """z (n x k), lam (k), status (k), sweeps (k), step (k), resid (k)."""
    __getattr__ = dict.__getitem__


def _finish(rc, z, lam, st, sw, stp, res):
    if rc != 0:
        raise MemoryError("oracle: allocation failed")
    return Result(z=z, lam=lam, status=st, sweeps=sw, step=stp, resid=res)


def _fn(name, accel):
    if accel not in ("picard", "acx"):
        raise ValueError("accel must be 'picard' or 'acx'")
    return getattr(_load(), name + ("_acx" if accel == "acx" else ""))


def ipt_dense(theta, delta, idx=None, z0=None, tol=1e-12, max_iter=DEFAULT_MAX_ITER,
              div_norm=DEFAULT_DIV_NORM, div_growth=DEFAULT_DIV_GROWTH, resid=True, accel="picard") -> Result:
    """IPT (Alg. 1 per requested column; Alg. 2 when idx covers every index) on a
    dense Delta.  Returns the certified iterate z (entry idx[c] of column c is 1),
    lambda = theta_i + (Delta z)_i, and the per-column status.  accel="acx" replaces
    the plain update by alternating cyclic extrapolation (Alg. 3); sweeps then
    counts applications of F."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    n = theta.shape[0]
    assert delta.shape == (n, n)
    if idx is None:
        idx = np.arange(n, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    k = idx.shape[0]
    if z0 is not None:
        z0 = np.ascontiguousarray(z0, dtype=np.float64)
        assert z0.shape == (n, k)
    z = np.empty((n, k)); lam = np.empty(k); st = np.empty(k, np.int32); sw = np.empty(k, np.int32)
    stp = np.empty(k); res = np.empty(k) if resid else None
    rc = _fn("oracle_ipt_dense", accel)(n, _ptr(theta), _ptr(delta), n, k, _ptr(idx), _ptr(z0), k, tol, max_iter,
                                  div_norm, div_growth, _ptr(z), k, _ptr(lam), _ptr(st), _ptr(sw), _ptr(stp),
                                  _ptr(res))
    return _finish(rc, z, lam, st, sw, stp, res)


def ipt_dense_cont(theta, delta, alpha, idx=None, z0=None, tol=1e-12, max_iter=DEFAULT_MAX_ITER,
                   div_norm=DEFAULT_DIV_NORM, div_growth=DEFAULT_DIV_GROWTH, resid=True) -> Result:
    """IPT with the non-autonomous continuation of the concluding discussion (the
    3 x 3 example): sweep t applies f_i to the partition D + (1 - alpha^t) Delta, so
    the map tends to the autonomous one; a column is certified only on a sweep whose
    scale has reached exactly 1 in FP64.  0 < alpha < 1; otherwise as ipt_dense."""
    if not (0.0 < alpha < 1.0):
        raise ValueError("alpha must be in (0, 1)")
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    n = theta.shape[0]
    assert delta.shape == (n, n)
    if idx is None:
        idx = np.arange(n, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    k = idx.shape[0]
    if z0 is not None:
        z0 = np.ascontiguousarray(z0, dtype=np.float64)
        assert z0.shape == (n, k)
    z = np.empty((n, k)); lam = np.empty(k); st = np.empty(k, np.int32); sw = np.empty(k, np.int32)
    stp = np.empty(k); res = np.empty(k) if resid else None
    rc = _load().oracle_ipt_dense_cont(n, _ptr(theta), _ptr(delta), n, k, _ptr(idx), _ptr(z0), k, float(alpha), tol,
                                       max_iter, div_norm, div_growth, _ptr(z), k, _ptr(lam), _ptr(st), _ptr(sw),
                                       _ptr(stp), _ptr(res))
    return _finish(rc, z, lam, st, sw, stp, res)


def ipt_dense_homotopy(theta, delta, stages, idx=None, z0=None, tol=1e-12, max_iter=DEFAULT_MAX_ITER,
                       div_norm=DEFAULT_DIV_NORM, div_growth=DEFAULT_DIV_GROWTH, resid=True, accel="picard") -> Result:
    """The homotopy restart of the concluding section: for q = 1..stages, IPT on the
    partition D + (q/stages) Delta (each entry of Delta times the FP64 number
    q/stages), started from the previous stage's vectors (the first stage from z0,
    or e_i); the last stage is the problem itself and decides.  Reading: "the
    diagonal matrix thus obtained as initial condition" is the matrix of the previous
    stage's eigenvectors, the chart z_i = 1 kept.  Returns the last stage's result
    with sweeps summed over the stages; accel as for ipt_dense, in every stage."""
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    z, total = z0, None
    for q in range(1, stages + 1):
        scale = float(q) / float(stages)
        r = ipt_dense(theta, delta * scale if q < stages else delta, idx=idx, z0=z, tol=tol, max_iter=max_iter,
                      div_norm=div_norm, div_growth=div_growth, resid=resid and q == stages, accel=accel)
        total = r.sweeps.copy() if total is None else total + r.sweeps
        z = r.z
    r["sweeps"] = total
    return r


def ipt_dense_z(theta, delta, idx=None, z0=None, tol=1e-12, max_iter=DEFAULT_MAX_ITER,
                div_norm=DEFAULT_DIV_NORM, div_growth=DEFAULT_DIV_GROWTH, resid=True) -> Result:
    """IPT over C^n (Sec. 2 states the method for complex M): theta, delta, z0 complex
    (numpy complex128, stored as (re, im) pairs); z and lam are complex.  Otherwise
    as ipt_dense (Alg. 1 per requested column)."""
    theta = np.ascontiguousarray(theta, dtype=np.complex128)
    delta = np.ascontiguousarray(delta, dtype=np.complex128)
    n = theta.shape[0]
    assert delta.shape == (n, n)
    if idx is None:
        idx = np.arange(n, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    k = idx.shape[0]
    if z0 is not None:
        z0 = np.ascontiguousarray(z0, dtype=np.complex128)
        assert z0.shape == (n, k)
    z = np.empty((n, k), np.complex128); lam = np.empty(k, np.complex128); st = np.empty(k, np.int32)
    sw = np.empty(k, np.int32); stp = np.empty(k); res = np.empty(k) if resid else None
    rc = _load().oracle_ipt_dense_z(n, _ptr(theta), _ptr(delta), n, k, _ptr(idx), _ptr(z0), k, tol, max_iter,
                                    div_norm, div_growth, _ptr(z), k, _ptr(lam), _ptr(st), _ptr(sw), _ptr(stp),
                                    _ptr(res))
    return _finish(rc, z, lam, st, sw, stp, res)


def ipt_csr(theta, row_ptr, col, val, idx, z0=None, tol=1e-10, max_iter=DEFAULT_MAX_ITER,
            div_norm=DEFAULT_DIV_NORM, div_growth=DEFAULT_DIV_GROWTH, resid=True, accel="picard") -> Result:
    """IPT on a CSR Delta for the requested columns (Alg. 1 per column; accel as for
    ipt_dense)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    n = theta.shape[0]
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    k = idx.shape[0]
    if z0 is not None:
        z0 = np.ascontiguousarray(z0, dtype=np.float64)
        assert z0.shape == (n, k)
    z = np.empty((n, k)); lam = np.empty(k); st = np.empty(k, np.int32); sw = np.empty(k, np.int32)
    stp = np.empty(k); res = np.empty(k) if resid else None
    rc = _fn("oracle_ipt_csr", accel)(n, _ptr(theta), _ptr(row_ptr), _ptr(col), _ptr(val), k, _ptr(idx), _ptr(z0), k,
                                tol, max_iter, div_norm, div_growth, _ptr(z), k, _ptr(lam), _ptr(st), _ptr(sw),
                                _ptr(stp), _ptr(res))
    return _finish(rc, z, lam, st, sw, stp, res)


def ipt_trace(theta, delta, i, t, z_start=None) -> np.ndarray:
    """Iterates z^(0..t) of f_i (eq. single_line_dyn) from e_i (or z_start), rows of
    a (t+1) x n array, with no stopping test."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    n = theta.shape[0]
    if z_start is not None:
        z_start = np.ascontiguousarray(z_start, dtype=np.float64)
    out = np.empty((t + 1, n))
    _load().oracle_ipt_trace(n, _ptr(theta), _ptr(delta), n, int(i), _ptr(z_start), int(t), _ptr(out))
    return out


def ipt_map(theta, delta, i, z):
    """One application of f_i (eq. single_line_dyn); returns (f_i(z), (Delta z)_i)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    w = np.empty_like(z)
    d = _load().oracle_ipt_map(theta.shape[0], _ptr(theta), _ptr(delta), theta.shape[0], int(i), _ptr(z), _ptr(w))
    return w, d


def ipt_batched(ns, theta_pool, delta_pool, theta_off, delta_off, tol=1e-10, max_iter=64,
                div_norm=DEFAULT_DIV_NORM, div_growth=DEFAULT_DIV_GROWTH, accel="picard", pair_tau=None):
    """Independent dense full-spectrum IPT solves over a packed batch.  z of problem
    b is returned row-major at z_pool[delta_off[b]:][:n_b*n_b].  With pair_tau, each
    problem is first re-partitioned by ``choose_d`` and its eigenvectors rotated back
    (``pair_back_rotate``)."""
    if accel != "picard" or pair_tau is not None:
        ns = np.asarray(ns)
        z = np.empty(np.asarray(delta_pool).shape[0]); lam = np.empty(np.asarray(theta_pool).shape[0])
        st = np.empty(lam.shape[0], np.int32); sw = np.empty(lam.shape[0], np.int32)
        for b in range(ns.shape[0]):
            n, to, do = int(ns[b]), int(theta_off[b]), int(delta_off[b])
            th = np.asarray(theta_pool[to:to + n]); de = np.asarray(delta_pool[do:do + n * n]).reshape(n, n)
            if pair_tau is not None:
                th, de, partner, cs = choose_d(th, de, pair_tau)
            r = ipt_dense(th, de, tol=tol, max_iter=max_iter, div_norm=div_norm, div_growth=div_growth, resid=False,
                          accel=accel)
            zb = r.z if pair_tau is None else pair_back_rotate(r.z, partner, cs)
            z[do:do + n * n] = zb.ravel(); lam[to:to + n] = r.lam; st[to:to + n] = r.status; sw[to:to + n] = r.sweeps
        return Result(z=z, lam=lam, status=st, sweeps=sw, step=None, resid=None)
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    theta_off = np.ascontiguousarray(theta_off, dtype=np.int64)
    delta_off = np.ascontiguousarray(delta_off, dtype=np.int64)
    theta_pool = np.ascontiguousarray(theta_pool, dtype=np.float64)
    delta_pool = np.ascontiguousarray(delta_pool, dtype=np.float64)
    z = np.empty_like(delta_pool); lam = np.empty_like(theta_pool)
    st = np.empty(theta_pool.shape[0], np.int32); sw = np.empty(theta_pool.shape[0], np.int32)
    rc = _load().oracle_ipt_batched(ns.shape[0], _ptr(ns), _ptr(theta_off), _ptr(delta_off), _ptr(delta_off),
                                    _ptr(theta_pool), _ptr(delta_pool), tol, max_iter, div_norm, div_growth,
                                    _ptr(z), _ptr(lam), _ptr(st), _ptr(sw))
    return _finish(rc, z, lam, st, sw, None, None)


# ------------------------------------------------------------------ NumPy parts

def pair_partners(theta, delta, tau):
    """Near-degenerate pairs (reading: the concluding section's freedom in choosing D,
    applied to pairs).  The coupling of i and k relative to their gap is
    r_ik = |Delta_ik| / |theta_i - theta_k| (k != i).  i and j = argmax_k r_ik (the
    first index on ties) form a pair when i is also the argmax for j, r_ij > tau, and
    Delta_ij == Delta_ji exactly (the 2x2 block is then symmetric).  Returns partner[i]
    (-1 when unpaired) and the row maxima of r."""
    theta = np.asarray(theta, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    n = theta.shape[0]
    partner = np.full(n, -1, dtype=np.int64)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.abs(delta) / np.abs(theta[:, None] - theta[None, :])
    np.fill_diagonal(r, -1.0)
    best = np.argmax(r, axis=1)  # the first index among equal maxima
    rmax = r[np.arange(n), best]
    for i in range(n):
        j = best[i]
        if n > 1 and best[j] == i and rmax[i] > tau and delta[i, j] == delta[j, i]:
            partner[i] = j
    return partner, rmax


def jacobi_cs(a, b, d):
    """The rotation J = [[c, s], [-s, c]] with J^T [[a, b], [b, d]] J diagonal (the
    symmetric Schur decomposition of a 2x2 block: t = tan of the angle, |angle| <=
    pi/4)."""
    if b == 0.0:
        return 1.0, 0.0
    zeta = (d - a) / (2.0 * b)
    t = (1.0 if zeta >= 0.0 else -1.0) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta))
    c = 1.0 / np.sqrt(1.0 + t * t)
    return c, t * c


def pair_rotation(theta, delta, tau):
    """M = diag(theta) + Delta -> M' = R^T M R with R the product of the pairs' 2x2
    rotations (R_ii = R_jj = c, R_ij = s, R_ji = -s for the pair i < j).  The new
    partition keeps every unpaired theta_k and Delta_kk; a pair's theta'_i, theta'_j
    are the diagonal of its rotated 2x2 block, whose entries leave Delta' (the
    pair's coupling is gone).  M' has the eigenvalues of M, and an eigenvector z' of
    M' is R^T z for the eigenvector z of M.  Returns (theta', Delta', partner, cs)
    with cs[i] = (c, s) for both members of a pair."""
    theta = np.asarray(theta, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    n = theta.shape[0]
    partner, _ = pair_partners(theta, delta, tau)
    M = np.diag(theta) + delta
    R = np.eye(n)
    cs = np.zeros((n, 2))
    cs[:, 0] = 1.0
    for i in range(n):
        j = partner[i]
        if j > i:
            c, s = jacobi_cs(M[i, i], M[i, j], M[j, j])
            R[i, i] = R[j, j] = c
            R[i, j], R[j, i] = s, -s
            cs[i] = cs[j] = (c, s)
    Mr = R.T @ M @ R
    th2 = theta.copy()
    de2 = delta.copy()
    paired = partner >= 0
    for i in range(n):
        for k in range(n):
            if paired[i] or paired[k]:
                de2[i, k] = Mr[i, k]
    for i in np.where(paired)[0]:
        j = partner[i]
        th2[i] = Mr[i, i]
        de2[i, i] = 0.0
        de2[i, j] = 0.0
    return th2, de2, partner, cs


def choose_d(theta, delta, tau):
    """The partition M = D' + Delta' used with the choice of D: the near-degenerate
    pairs rotated out (``pair_rotation``), then the level shifts moved into D, to
    first order (diag Delta) and second order (the RS energy shift
    s_i = sum_{k != i} Delta_ik Delta_ki / (theta_i - theta_k), on the folded theta;
    terms with Delta_ik Delta_ki = 0 are 0):
      theta'_i = (theta_i + Delta_ii) + s_i,  Delta'_ii = -s_i,  Delta'_ik = Delta_ik.
    The matrix is the rotated M (up to the rounding of theta'); the gaps of G become
    those of the shifted levels, so a level shift comparable to a small gap no longer
    makes the fixed point repelling.  Returns (theta', Delta', partner, cs)."""
    th1, de1, partner, cs = pair_rotation(theta, delta, tau)
    n = th1.shape[0]
    th2 = th1 + np.diag(de1)
    off = de1 - np.diag(np.diag(de1))
    prod = off * off.T
    with np.errstate(divide="ignore", invalid="ignore"):
        terms = np.where(prod != 0.0, prod / (th2[:, None] - th2[None, :]), 0.0)
    np.fill_diagonal(terms, 0.0)
    shift = np.zeros(n)
    for i in range(n):  # in index order
        acc = 0.0
        for k in range(n):
            acc += terms[i, k]
        shift[i] = acc
    return th2 + shift, off - np.diag(shift), partner, cs


def pair_back_rotate(z, partner, cs):
    """Eigenvectors of M from those of M': z = R z' (rows i and j of a pair mix)."""
    z = np.array(z, dtype=np.float64, copy=True)
    out = z.copy()
    for i in range(z.shape[0]):
        j = partner[i]
        if j > i:
            c, s = cs[i]
            out[i] = c * z[i] + s * z[j]
            out[j] = -s * z[i] + c * z[j]
    return out


def inverse_gaps(theta):
    """G_jk = 1/(theta_j - theta_k) for j != k, G_jj = 0 (Sec. 3, inverse gaps matrix)."""
    theta = np.asarray(theta, dtype=np.float64)
    diff = theta[:, None] - theta[None, :]
    g = np.zeros_like(diff)
    off = ~np.eye(theta.shape[0], dtype=bool)
    g[off] = 1.0 / diff[off]
    return g


def rs_series(theta, delta, order):
    """Rayleigh-Schroedinger corrections Z^[0..order] of M = D + eps*Delta
    (eq. ARS-alpha; App. B): Z^[0] = I and
    Z^[l] = G o ( sum_{s=0}^{l-1} Z^[l-1-s] D(Delta Z^[s]) - Delta Z^[l-1] ).
    Returns a list of n x n arrays; Z_RS^(k) = sum_l eps^l Z^[l]."""
    theta = np.asarray(theta, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    n = theta.shape[0]
    g = inverse_gaps(theta)
    zs = [np.eye(n)]
    dz = [delta @ zs[0]]                       # Delta Z^[s], kept for the diagonal terms
    for l in range(1, order + 1):
        acc = np.zeros((n, n))
        for s in range(l):
            acc += zs[l - 1 - s] * np.diag(dz[s])[None, :]   # Z^[l-1-s] D(Delta Z^[s])
        zl = g * (acc - dz[l - 1])
        zs.append(zl)
        dz.append(delta @ zl)
    return zs


def rs_eigenvalues(theta, delta, order):
    """lambda^[0] = theta, lambda^[l] = (Delta Z^[l-1])_ii (App. B)."""
    zs = rs_series(theta, delta, order - 1 if order > 0 else 0)
    lam = [np.asarray(theta, dtype=np.float64).copy()]
    for l in range(1, order + 1):
        lam.append(np.diag(np.asarray(delta) @ zs[l - 1]).copy())
    return lam


def norm1(theta, delta=None, csr=None):
    """|M|_1 = max_k sum_j |M_jk| with M = diag(theta) + Delta (max absolute column sum)."""
    theta = np.asarray(theta, dtype=np.float64)
    if delta is not None:
        m = np.array(delta, dtype=np.float64, copy=True)
        m[np.diag_indices_from(m)] += theta
        return float(np.abs(m).sum(axis=0).max())
    row_ptr, col, val = csr
    n = theta.shape[0]
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    colsum = np.zeros(n)
    diag = theta.copy()
    on = rows == col
    np.add.at(diag, col[on], val[on])
    np.add.at(colsum, col[~on], np.abs(val[~on]))
    return float((colsum + np.abs(diag)).max())


def eigen_residual(theta, delta, z, lam):
    """|M z_c - lambda_c z_c|_2 / |z_c|_2 per column (plain definition)."""
    theta = np.asarray(theta, dtype=np.float64)
    mz = theta[:, None] * z + np.asarray(delta) @ z
    return np.linalg.norm(mz - z * lam[None, :], axis=0) / np.linalg.norm(z, axis=0)

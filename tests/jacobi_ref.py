"""Brute-force cyclic Jacobi eigensolver for tiny real symmetric matrices (a
textbook method, independent of IPT), used only to pin the oracle."""
import math

import numpy as np


def cyclic_jacobi(a, sweeps=100, tol=1e-30):
    """Returns (eigenvalues, eigenvectors as columns) of a symmetric matrix by
    cyclic plane rotations that annihilate one off-diagonal pair at a time."""
    a = np.array(a, dtype=np.float64, copy=True)
    n = a.shape[0]
    v = np.eye(n)
    for _ in range(sweeps):
        off = sum(a[p, q] ** 2 for p in range(n) for q in range(n) if p != q)
        if off <= tol:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                if a[p, q] == 0.0:
                    continue
                tau = (a[q, q] - a[p, p]) / (2.0 * a[p, q])
                t = math.copysign(1.0, tau) / (abs(tau) + math.sqrt(1.0 + tau * tau))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = t * c
                rot = np.eye(n)
                rot[p, p] = c
                rot[q, q] = c
                rot[p, q] = s
                rot[q, p] = -s
                a = rot.T @ a @ rot
                v = v @ rot
    return np.diag(a).copy(), v

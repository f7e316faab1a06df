"""CPU checks of the parity rule itself (tests/parity.py)."""
import numpy as np
import pytest

from parity import check


class _Ref:
    def __init__(self, status, step, sweeps, n=3):
        self.status = np.asarray(status)
        self.step = np.asarray(step, dtype=float)
        self.sweeps = np.asarray(sweeps)
        k = len(status)
        self.z = np.eye(n, k)
        self.lam = np.arange(k, dtype=float)


def test_failure_label_at_the_sweep_cap_is_free_only_there():
    ref = _Ref([0, 2, 1], [1e-12, 2.0, 0.9], [4, 100, 100])
    z, lam = ref.z.copy(), ref.lam.copy()
    check(z, lam, [0, 1, 2], ref, 1.0, 1e-10, max_iter=100)       # swapped labels at the cap
    with pytest.raises(AssertionError):
        check(z, lam, [0, 1, 2], ref, 1.0, 1e-10)                 # without max_iter: exact labels
    with pytest.raises(AssertionError):
        check(z, lam, [0, 0, 2], ref, 1.0, 1e-10, max_iter=100)   # CONVERGED is never accepted for a failure
    early = _Ref([0, 2, 1], [1e-12, 2.0, 0.9], [4, 9, 100])
    with pytest.raises(AssertionError):
        check(z, lam, [0, 1, 1], early, 1.0, 1e-10, max_iter=100)  # a divergence before the cap must match


def test_converged_columns_are_compared():
    ref = _Ref([0, 0], [1e-12, 1e-12], [4, 4])
    z, lam = ref.z.copy(), ref.lam.copy()
    lam[1] += 1e-9
    with pytest.raises(AssertionError):
        check(z, lam, [0, 0], ref, 1.0, 1e-10)
    z2 = ref.z.copy()
    z2[2, 0] = 1e-6
    with pytest.raises(AssertionError):
        check(z2, ref.lam, [0, 0], ref, 1.0, 1e-10)


def test_ladder_failure_labels_are_free_before_the_cap():
    """On a ladder solve the growth count runs on exact sweeps only, so a failing
    column's label may differ from the FP64 oracle's anywhere; CONVERGED against a
    failure is still a mismatch."""
    early = _Ref([0, 2, 1], [1e-12, 2.0, 0.9], [4, 9, 100])
    z, lam = early.z.copy(), early.lam.copy()
    check(z, lam, [0, 1, 2], early, 1.0, 1e-10, max_iter=100, ladder=True)
    with pytest.raises(AssertionError):
        check(z, lam, [0, 1, 1], early, 1.0, 1e-10, max_iter=100)
    with pytest.raises(AssertionError):
        check(z, lam, [0, 0, 1], early, 1.0, 1e-10, max_iter=100, ladder=True)
    with pytest.raises(AssertionError):
        check(z, lam, [2, 2, 1], early, 1.0, 1e-10, max_iter=100, ladder=True)

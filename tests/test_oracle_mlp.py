"""Pins of the FP64 MLP reference: its gradient equals central finite differences of
its own loss (an independent computation), and bf16 rounding is round-to-nearest-even."""
import numpy as np

from oracle import mlp


def test_gradient_matches_finite_differences():
    dims = (2, 7, 2, 5)
    rng = np.random.default_rng(0)
    nparam = sum(li * lo + lo for li, lo in mlp.layer_sizes(*dims))
    p = rng.standard_normal(nparam) * 0.5
    x = rng.standard_normal((9, 2))
    t = rng.standard_normal((9, 5))
    _, g = mlp.loss_grad(p, x, t, dims)
    h = 1e-6
    fd = np.empty_like(p)
    for q in range(nparam):
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd[q] = (mlp.loss_grad(pp, x, t, dims)[0] - mlp.loss_grad(pm, x, t, dims)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-8 * max(1.0, np.abs(g).max())


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.14159265, 1e-30])
    r = mlp.to_bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie to even
    assert r[2] == 1.0 + 4 * 2 ** -8        # tie to even (upwards)
    assert r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-12
    assert np.all(np.abs(r - vals) <= np.abs(vals) * 2 ** -8)

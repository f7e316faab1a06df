"""Pins of the BF16 network reference (oracle.mlp.network_bf16) and of its bounds.

Without the roundings it is the plain FP64 network, whose gradient the finite-difference
pin fixes.  With them, an independent FP32 evaluation of the same rounding points (NumPy
float32 products, whose accumulation order differs from the reference's) lands inside
the bounds on every element, the bounds are small next to the values, and planted
mistakes of the kind a kernel could make (a wrong tanh derivative, a missing rounding
point, a transposed weight, a dropped bias gradient) fall outside them."""
import numpy as np
import pytest

from oracle import mlp


def _bf(a):
    """BF16 rounding of FP32 values, kept as float32."""
    return mlp.to_bf16(np.asarray(a, dtype=np.float32)).astype(np.float32)


def _emulate(params, x, t, dims, mistake=None, row_weights=None):
    """The network at the kernels' rounding points, in FP32 arithmetic."""
    layers = mlp.unpack(params, *dims)
    f = np.float32
    h = _bf(x)
    hs = [h]
    for l, (w, b) in enumerate(layers):
        pre = h @ _bf(w).T + (0 if mistake == "no_hidden_bias" and l == 1 else b.astype(f))
        if l < len(layers) - 1:
            v = np.tanh(pre)
            h = v.astype(f) if mistake == "unrounded_activation" else _bf(v)
            hs.append(h)
        else:
            y = pre
    t = t.astype(f)
    w = np.ones((y.shape[0], 1), dtype=f) if row_weights is None else row_weights.astype(f).reshape(-1, 1)
    d = (y - t) * w
    count = y.size
    loss = float(np.sum(d.astype(np.float64) ** 2) / count)
    if mistake == "unweighted_gradient":
        w = np.ones_like(w)
    g = _bf(f((1.0 if mistake == "half_scale" else 2.0) / count) * w * d)
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        wb = _bf(layers[l][0])
        gw = g.T @ hs[l]
        gb = g.sum(axis=0, dtype=f)
        if mistake == "no_bias_grad" and l == len(layers) - 1:
            gb = np.zeros_like(gb)
        grads.append((gw, gb))
        if l > 0:
            dh = g @ (wb.T if mistake == "transposed_weight" and l == 1 else wb)
            hl = hs[l]
            der = (1.0 - hl) if mistake == "tanh_derivative" else (1.0 - hl * hl)
            gn = dh * der.astype(f)
            g = _bf(gn)
    out = []
    for gw, gb in reversed(grads):
        out += [gw.ravel(), gb]
    return loss, np.concatenate(out).astype(np.float64), y.astype(np.float64)


def _case(seed, dims, batch, scale=0.3):
    rng = np.random.default_rng(seed)
    nparam = sum(li * lo + lo for li, lo in mlp.layer_sizes(*dims))
    p = (rng.standard_normal(nparam) * scale).astype(np.float32).astype(np.float64)
    x = rng.standard_normal((batch, dims[0])).astype(np.float32)
    t = rng.standard_normal((batch, dims[-1])).astype(np.float32)
    return p, x, t


def test_without_roundings_it_is_the_plain_network():
    dims = (2, 9, 2, 7)
    p, x, t = _case(0, dims, 11)
    loss, g, y, *_ = mlp.network_bf16(p, x, t, dims, round_points=False)
    loss0, g0 = mlp.loss_grad(p, x, t, dims)
    assert abs(loss - loss0) <= 1e-14 * loss0
    assert np.max(np.abs(g - g0)) <= 1e-13 * np.abs(g0).max()
    np.testing.assert_allclose(y, mlp.forward(p, x, dims)[-1], rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed,dims,batch", [(1, (2, 64, 2, 300), 37), (2, (2, 48, 3, 130), 64),
                                             (3, (3, 128, 2, 257), 200)])
def test_fp32_evaluation_lands_inside_the_bounds(seed, dims, batch):
    p, x, t = _case(seed, dims, batch)
    loss, g, y, lb, gb, yb = mlp.network_bf16(p, x, t, dims)
    el, eg, ey = _emulate(p, x, t, dims)
    assert abs(el - loss) <= lb
    assert np.all(np.abs(eg - g) <= gb)
    assert np.all(np.abs(ey - y) <= yb)
    # the bounds are small next to the values, and not vacuous
    assert np.median(gb / np.maximum(np.abs(g), 1e-30)) < 5e-2
    assert np.median(yb / np.abs(y)) < 1e-2
    assert np.max(np.abs(ey - y) / yb) > 1e-3


@pytest.mark.parametrize("mistake", ["tanh_derivative", "unrounded_activation", "transposed_weight", "no_bias_grad",
                                     "half_scale", "no_hidden_bias"])
def test_planted_mistakes_fall_outside(mistake):
    dims = (2, 64, 2, 300)
    p, x, t = _case(1, dims, 37)
    loss, g, y, lb, gb, yb = mlp.network_bf16(p, x, t, dims)
    el, eg, ey = _emulate(p, x, t, dims, mistake)
    outside = np.sum(np.abs(eg - g) > gb) + np.sum(np.abs(ey - y) > yb) + int(abs(el - loss) > lb)
    assert outside > 0, mistake


def test_row_weights():
    """Per-example weights: without roundings the loss is the weighted plain loss and its
    gradient equals central finite differences; the FP32 evaluation with the weights lands
    inside the bounds, and forgetting the weights in the gradient falls outside."""
    dims = (2, 9, 2, 7)
    p, x, t = _case(5, dims, 11)
    w = np.random.default_rng(6).uniform(0.0, 1.0, 11).astype(np.float32)
    loss, g, *_ = mlp.network_bf16(p, x, t, dims, round_points=False, row_weights=w)
    ws = w.astype(np.float64).reshape(-1, 1)
    y = mlp.forward(p, x, dims)[-1]
    assert abs(loss - np.sum((ws * (y - t)) ** 2) / y.size) <= 1e-14 * loss
    h = 1e-6
    for q in np.random.default_rng(7).choice(p.shape[0], 25, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd = (mlp.network_bf16(pp, x, t, dims, False, w)[0] - mlp.network_bf16(pm, x, t, dims, False, w)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-7 * max(1.0, np.abs(g).max())
    dims = (2, 64, 2, 300)
    p, x, t = _case(1, dims, 37)
    w = np.random.default_rng(8).uniform(0.0, 1.0, 37).astype(np.float32)
    loss, g, y, lb, gb, yb = mlp.network_bf16(p, x, t, dims, row_weights=w)
    el, eg, ey = _emulate(p, x, t, dims, row_weights=w)
    assert abs(el - loss) <= lb
    assert np.all(np.abs(eg - g) <= gb)
    el, eg, ey = _emulate(p, x, t, dims, mistake="unweighted_gradient", row_weights=w)
    assert np.sum(np.abs(eg - g) > gb) > 0

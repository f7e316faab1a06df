"""FP64 reference of the warm-start MLP -- TEST INFRASTRUCTURE ONLY.

x -> [Linear -> tanh] x depth -> Linear -> y, mean squared error loss, and its exact
gradient by the chain rule, in NumPy float64.  Parameters use the library's layout:
per layer W (out x in, row-major) followed by b (out).  The HIP kernels compute the
same network with BF16 weights and BF16-rounded GEMM inputs; pass
round_bf16=True to evaluate with the weights rounded the same way.  network_bf16 is
the network with every BF16 rounding point of the kernels and exact arithmetic in
between, with element-wise bounds on what FP32 arithmetic may change (the reference
the GPU gradients are checked against)."""
import numpy as np


def layer_sizes(in_dim, hidden, depth, out_dim):
    dims = [in_dim] + [hidden] * depth + [out_dim]
    return list(zip(dims[:-1], dims[1:]))


def unpack(params, in_dim, hidden, depth, out_dim):
    params = np.asarray(params, dtype=np.float64)
    layers, off = [], 0
    for li, lo in layer_sizes(in_dim, hidden, depth, out_dim):
        w = params[off:off + li * lo].reshape(lo, li)
        off += li * lo
        b = params[off:off + lo]
        off += lo
        layers.append((w, b))
    assert off == params.shape[0]
    return layers


def to_bf16(a):
    """Round float values to bfloat16 (round to nearest even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, x, dims, round_bf16=False):
    layers = unpack(params, *dims)
    hs = [np.asarray(x, dtype=np.float64)]
    for l, (w, b) in enumerate(layers):
        if round_bf16:
            w = to_bf16(w)
        pre = hs[-1] @ w.T + b
        hs.append(pre if l == len(layers) - 1 else np.tanh(pre))
    return hs


def loss_grad(params, x, t, dims, round_bf16=False):
    """Mean squared error over all outputs and its gradient (same layout as params)."""
    layers = unpack(params, *dims)
    hs = forward(params, x, dims, round_bf16)
    y = hs[-1]
    t = np.asarray(t, dtype=np.float64)
    count = y.size
    loss = float(np.sum((y - t) ** 2) / count)
    d = 2.0 * (y - t) / count
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        w, _ = layers[l]
        if round_bf16:
            w = to_bf16(w)
        gw = d.T @ hs[l]
        gb = d.sum(axis=0)
        grads.append((gw, gb))
        if l > 0:
            d = (d @ w) * (1.0 - hs[l] ** 2)
    out = []
    for gw, gb in reversed(grads):
        out.append(gw.ravel())
        out.append(gb)
    return loss, np.concatenate(out)


# ------------------------------------------------------------------ the kernels' network
# The library evaluates the network with BF16 GEMM operands: the input x, the weights,
# each hidden activation tanh(pre), the output gradient g = s (y - t) with
# s = 2 / (batch out), and each hidden gradient (g_{l+1} W_{l+1}) o (1 - H_l^2) (H_l the
# BF16 activation) are rounded to BF16 from FP32 values; products are accumulated in
# FP32, biases added in FP32, tanh evaluated in FP32; the bias gradient sums the BF16
# gradient values, the loss the FP32 squares (y - t)^2.
# ``network_bf16`` is that network with every rounding to BF16 done as the kernels do
# (from the FP32 value, round to nearest even) and everything else exact (FP64), and
# ``bf16_bounds`` bounds, element by element, how far a computation that differs from
# it only by FP32 arithmetic (accumulation in any order, the bias add, tanh to within
# 4 ulp) can land: the FP32 errors propagate through the network, and a BF16 rounding
# can come out one BF16 step different only where the FP32 error interval of the value
# being rounded straddles a rounding boundary.
U_F32 = 2.0 ** -24


def _gamma(k):
    """Higham's gamma_k = k u / (1 - k u) for FP32: a sum of k terms accumulated in FP32
    in any order is within gamma_k * (sum of the terms' moduli) of the exact sum."""
    ku = k * U_F32
    return ku / (1.0 - ku)


def _r(a):
    """BF16 rounding of the FP32 value of a (the kernels round FP32 values)."""
    return to_bf16(np.asarray(a, dtype=np.float32))


def _round_err(v, d):
    """The rounded value r(v) and a bound on |r(w) - r(v)| over every w with
    |w - v| <= d (r is monotone, so the interval's end points bound it)."""
    rv = _r(v)
    lo, hi = _r(v - d), _r(v + d)
    return rv, np.maximum(hi - rv, rv - lo)


def network_bf16(params, x, t, dims, round_points=True, row_weights=None):
    """Loss, gradient (parameter layout) and output y of the network as the kernels
    define it, with exact arithmetic between the BF16 roundings, together with bounds
    on |kernel - this| for each: returns (loss, grad, y, loss_bound, grad_bound,
    y_bound).  round_points=False skips the roundings (the plain FP64 network).
    row_weights (one FP32 weight w_b per example) make the loss
    sum_b w_b^2 sum_q (y_bq - t_bq)^2 / (batch out); the kernels form w (y - t) and
    scale w (w (y - t)) in FP32."""
    global _r
    if not round_points:
        saved, _r = _r, lambda a: np.asarray(a, dtype=np.float64)
        try:
            return network_bf16(params, x, t, dims, row_weights=row_weights)
        finally:
            _r = saved
    layers = unpack(params, *dims)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    hs, ehs = [_r(x)], [np.zeros_like(x)]
    for l, (w, b) in enumerate(layers):
        wr = _r(w)
        aw = np.abs(wr)
        h, eh = hs[-1], ehs[-1]
        pre = h @ wr.T + b
        e_pre = eh @ aw.T + _gamma(h.shape[1] + 1) * ((np.abs(h) + eh) @ aw.T + np.abs(b))
        if l < len(layers) - 1:
            v = np.tanh(pre)
            hr, e = _round_err(v, e_pre + 4.0 * U_F32 * np.abs(v))
            hs.append(hr)
            ehs.append(e)
        else:
            hs.append(pre)
            ehs.append(e_pre)
    y, ey = hs[-1], ehs[-1]
    count = y.size
    s = 2.0 / count
    w = np.ones((y.shape[0], 1)) if row_weights is None else \
        np.asarray(row_weights, dtype=np.float32).astype(np.float64).reshape(-1, 1)
    d = w * (y - t)
    loss = float(np.sum(d * d) / count)
    # FP32: y - t, then the product with w
    ed = w * (ey + U_F32 * (np.abs(y - t) + ey)) + U_F32 * (np.abs(d) + w * ey)
    loss_bound = float((np.sum(2.0 * np.abs(d) * ed + ed * ed) + _gamma(66) * np.sum((np.abs(d) + ed) ** 2)) / count
                       + 2.0 * U_F32 * loss)
    gv = s * w * d
    # FP32: the scale (rounded once), its product with w, then with d
    g, eg = _round_err(gv, s * w * ed + 3.0 * U_F32 * (np.abs(gv) + s * w * ed))
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        wr = _r(layers[l][0])
        aw = np.abs(wr)
        h, eh = hs[l], ehs[l]
        ag = np.abs(g)
        nb = g.shape[0]
        gw = g.T @ h
        e_gw = eg.T @ np.abs(h) + ag.T @ eh + eg.T @ eh + _gamma(nb) * ((ag + eg).T @ (np.abs(h) + eh))
        gb = g.sum(axis=0)
        e_gb = eg.sum(axis=0) + _gamma(nb) * (ag + eg).sum(axis=0)
        grads.append((gw, gb, e_gw, e_gb))
        if l > 0:
            dh = g @ wr
            e_dh = eg @ aw + _gamma(wr.shape[0]) * ((ag + eg) @ aw)
            one = 1.0 - h * h
            e_one = 2.0 * np.abs(h) * eh + eh * eh
            gn = dh * one
            e_gn = e_dh * np.abs(one) + (np.abs(dh) + e_dh) * e_one
            # FP32 evaluation of dh (1 - h h): the square and the difference round with
            # absolute errors (near saturation 1 - h^2 is small), then the product
            e_gn = (e_gn + U_F32 * (1.0 + U_F32) * (np.abs(dh) + e_dh) * (h * h + np.abs(one) + e_one)
                    + U_F32 * (np.abs(gn) + e_gn))
            g, eg = _round_err(gn, e_gn)
    out, bnd = [], []
    for gw, gb, e_gw, e_gb in reversed(grads):
        out += [gw.ravel(), gb]
        bnd += [e_gw.ravel(), e_gb]
    return loss, np.concatenate(out), y, loss_bound, np.concatenate(bnd), ey

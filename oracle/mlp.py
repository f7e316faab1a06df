"""FP64 reference of the warm-start MLP -- TEST INFRASTRUCTURE ONLY.

x -> [Linear -> tanh] x depth -> Linear -> y, mean squared error loss, and its exact
gradient by the chain rule, in NumPy float64.  Parameters use the library's layout:
per layer W (out x in, row-major) followed by b (out).  The HIP kernels compute the
same network with BF16 weights and BF16-rounded GEMM inputs; pass
round_bf16=True to evaluate with the weights rounded the same way."""
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

"""Oracle of the skeleton-proposal network (test infrastructure only): a plain numpy FP64
multilayer perceptron with ReLU hidden layers, its loss and a hand-written backward pass.

Loss per sample: binary cross entropy with logits on the first nout/2 outputs (labels 0/1),
wmse times the squared error on the others; the batch loss is the mean over samples.
Parameters are packed per linear map l as W_l (out x in, column major) then b_l, the
packing of the library.
"""
import numpy as np


def dims(shape):
    nin, nh, nl, nout = shape
    return [nin] + [nh] * nl + [nout]


def offsets(shape):
    d = dims(shape)
    off, o = [], 0
    for l in range(len(d) - 1):
        off.append((o, o + d[l + 1] * d[l]))       # W_l
        o += d[l + 1] * d[l]
        off.append((o, o + d[l + 1]))              # b_l
        o += d[l + 1]
    return off, o


def unpack(params, shape):
    d = dims(shape)
    off, _ = offsets(shape)
    out = []
    for l in range(len(d) - 1):
        (w0, w1), (b0, b1) = off[2 * l], off[2 * l + 1]
        W = np.asarray(params[w0:w1], float).reshape(d[l], d[l + 1]).T    # column major out x in
        out.append((W, np.asarray(params[b0:b1], float)))
    return out


def pack(layers):
    parts = []
    for W, b in layers:
        parts.append(W.T.reshape(-1))
        parts.append(b)
    return np.concatenate(parts)


def forward(params, shape, X):
    """X (B, nin) -> outputs (B, nout) and the pre-activations and activations per layer."""
    layers = unpack(params, shape)
    H = [np.asarray(X, float)]
    Z = [None]
    for l, (W, b) in enumerate(layers):
        z = H[-1] @ W.T + b
        Z.append(z)
        H.append(np.maximum(z, 0.0) if l + 1 < len(layers) else z)
    return Z[-1], (Z, H)


def loss(out, Y, wmse):
    """Batch-mean loss and its gradient with respect to the outputs."""
    B, nout = out.shape
    ns = nout // 2
    z, y = out[:, :ns], Y[:, :ns]
    bce = np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))
    d = out[:, ns:] - Y[:, ns:]
    L = (bce.sum() + wmse * (d * d).sum()) / B
    g = np.empty_like(out)
    g[:, :ns] = 1.0 / (1.0 + np.exp(-z)) - y
    g[:, ns:] = 2.0 * wmse * d
    return L, g / B


def backward(params, shape, cache, dout):
    """Gradient of the loss with respect to the packed parameters (chain rule by layer)."""
    layers = unpack(params, shape)
    Z, H = cache
    grads = [None] * len(layers)
    dz = dout
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (dz.T @ H[l], dz.sum(axis=0))
        if l > 0:
            dh = dz @ W
            dz = dh * (Z[l] > 0)
    return pack(grads)


def value_and_grad(params, shape, X, Y, wmse):
    out, cache = forward(params, shape, X)
    L, g = loss(out, Y, wmse)
    return out, L, backward(params, shape, cache, g)

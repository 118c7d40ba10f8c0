"""Plain numpy FP64 reference of the surrogate network -- TEST INFRASTRUCTURE
ONLY (used by the tests to check the HIP training and inference kernels).

Network: L = depth + 1 linear layers n_in -> width -> ... -> n_out, SiLU
between them, inputs scaled to [-1, 1], outputs standardised, loss = mean
squared error over all outputs of the batch.  Flat parameter layout: W_1
[out][in], ..., W_L, then b_1, ..., b_L.  With ``bf16=True`` the values the
device keeps in BF16 (scaled inputs, weights, hidden activations and the
back-propagated dZ fed to the matrix products) are rounded to BF16 at the same
points; all arithmetic is FP64.
"""
import numpy as np


def bf16_round(x):
    """Round to the nearest BF16 (ties to even) through the FP32 value."""
    x32 = np.asarray(x, np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return ((u << 16).astype(np.uint32)).view(np.float32).astype(np.float64)


def dims(n_in, width, depth, n_out):
    L = depth + 1
    din = [n_in] + [width] * depth
    dout = [width] * depth + [n_out]
    return L, din, dout


def unpack(p, n_in, width, depth, n_out):
    L, din, dout = dims(n_in, width, depth, n_out)
    Ws, bs, off = [], [], 0
    for l in range(L):
        Ws.append(np.asarray(p[off:off + din[l] * dout[l]], np.float64).reshape(dout[l], din[l]))
        off += din[l] * dout[l]
    for l in range(L):
        bs.append(np.asarray(p[off:off + dout[l]], np.float64))
        off += dout[l]
    return Ws, bs


def pack(Ws, bs):
    return np.concatenate([w.reshape(-1) for w in Ws] + [b for b in bs])


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def scale_inputs(X, lo, hi):
    return 2.0 * (np.asarray(X, np.float64) - lo) / (hi - lo) - 1.0


def forward(p, Xs, shape, bf16=False):
    """Xs: already scaled inputs.  Returns pre-activations Z and inputs H of each layer."""
    Ws, bs = unpack(p, *shape)
    r = bf16_round if bf16 else (lambda v: v)
    h = r(Xs)
    Zs, Hs = [], [h]
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = h @ r(W).T + b
        Zs.append(z)
        if l < len(Ws) - 1:
            h = r(silu(z))
            Hs.append(h)
    return Zs, Hs


def _backward(p, Xs, Ys, shape, bf16, magnitudes):
    Ws, bs = unpack(p, *shape)
    r = bf16_round if bf16 else (lambda v: v)
    Zs, Hs = forward(p, Xs, shape, bf16)
    out = Zs[-1]
    n = out.size
    loss = np.sum((out - Ys) ** 2) / n
    dz = 2.0 * (out - Ys) / n
    gW, gb = [None] * len(Ws), [None] * len(Ws)
    mag = np.abs if magnitudes else (lambda v: v)
    for l in range(len(Ws) - 1, -1, -1):
        gW[l] = mag(r(dz)).T @ mag(Hs[l])
        gb[l] = mag(dz).sum(axis=0)
        if l > 0:
            dh = r(dz) @ r(Ws[l])
            dz = dh * dsilu(Zs[l - 1])
    return loss, pack(gW, gb)


def loss_and_grads(p, Xs, Ys, shape, bf16=False):
    """Standardised targets Ys.  Returns (loss, flat gradient)."""
    return _backward(p, Xs, Ys, shape, bf16, False)


def grad_scales(p, Xs, Ys, shape, bf16=False):
    """Per parameter, the sum of the magnitudes of the terms that make up its
    gradient (|dZ|^T |H| for a weight, sum |dZ| for a bias), from the same
    forward and backward pass as loss_and_grads: the condition of each sum.
    Changing every term by a relative u moves the element by at most u times
    this, so rounding the BF16 operands differently (one BF16 ulp, u = 2^-8)
    or accumulating in another order stays within a small multiple of it."""
    return _backward(p, Xs, Ys, shape, bf16, True)[1]


def output_scales(p, Xs, shape, bf16=False):
    """Per sample and output, |W_L| |h_{L-1}| + |b_L|: the condition of the
    last layer's sum (standardised units), the same role as grad_scales."""
    Ws, bs = unpack(p, *shape)
    r = bf16_round if bf16 else (lambda v: v)
    _, Hs = forward(p, Xs, shape, bf16)
    return np.abs(Hs[-1]) @ np.abs(r(Ws[-1])).T + np.abs(bs[-1])

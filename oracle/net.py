"""FP64 reference of the learned initial-guess network (test infrastructure).

A 3-D convolution with 3x3x3 kernels, zero padding and "same" output size,
written as plain loops over the 27 taps (each tap is one einsum over the
channel index): out[b, z, y, x, o] = bias[o] + sum_{tap, i} w[tap, o, i] *
in[b, z+dz, y+dy, x+dx, i], taps ordered (dz, dy, dx) with dx fastest,
offsets -1..1.  Activations are channel-last [batch, z, y, x, channel].

The network: conv(2->16) -> ReLU -> conv(16->16) -> ReLU -> conv(16->1), the
loss the masked mean squared error.  Backward passes (data and weight
gradients) are the same loops transposed; they are pinned by central finite
differences in tests/test_oracle_net.py.  Adam follows Kingma & Ba (2015)
with bias correction.
"""
import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
LAYERS = [(2, 16), (16, 16), (16, 1)]


def n_params():
    return sum(27 * ci * co + co for ci, co in LAYERS)


def unpack(theta):
    """Flat parameter vector -> [(w[27, co, ci], b[co]), ...] (packing order of the ABI)."""
    out, k = [], 0
    for ci, co in LAYERS:
        w = theta[k:k + 27 * co * ci].reshape(27, co, ci)
        k += 27 * co * ci
        b = theta[k:k + co]
        k += co
        out.append((w, b))
    return out


def pack(params):
    return np.concatenate([np.concatenate([w.reshape(-1), b]) for w, b in params])


def _shift(a, dz, dy, dx):
    """b[:, z, y, x] = a[:, z+dz, y+dy, x+dx], zero outside."""
    out = np.zeros_like(a)
    B, Z, Y, X = a.shape[:4]
    sz = slice(max(0, -dz), min(Z, Z - dz))
    sy = slice(max(0, -dy), min(Y, Y - dy))
    sx = slice(max(0, -dx), min(X, X - dx))
    tz = slice(max(0, dz), min(Z, Z + dz))
    ty = slice(max(0, dy), min(Y, Y + dy))
    tx = slice(max(0, dx), min(X, X + dx))
    out[:, sz, sy, sx] = a[:, tz, ty, tx]
    return out


def conv_fwd(x, w, b):
    y = np.zeros(x.shape[:4] + (w.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += np.einsum("bzyxi,oi->bzyxo", _shift(x, dz, dy, dx), w[t])
    return y + b


def conv_bwd_data(gy, w):
    """d loss / d x for y = conv_fwd(x, w, b)."""
    gx = np.zeros(gy.shape[:4] + (w.shape[2],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        gx += _shift(np.einsum("bzyxo,oi->bzyxi", gy, w[t]), -dz, -dy, -dx)
    return gx


def conv_bwd_weight(x, gy):
    """d loss / d w and d loss / d b."""
    gw = np.zeros((27, gy.shape[-1], x.shape[-1]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        gw[t] = np.einsum("bzyxo,bzyxi->oi", gy, _shift(x, dz, dy, dx))
    gb = gy.reshape(-1, gy.shape[-1]).sum(0)
    return gw, gb


def forward(params, x):
    acts = [x]
    h = x
    for li, (w, b) in enumerate(params):
        h = conv_fwd(h, w, b)
        if li < len(params) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return acts


def loss_and_grads(params, x, target, mask):
    """Masked MSE: sum(mask (y - t)^2) / sum(mask).  Returns (loss, grads)."""
    acts = forward(params, x)
    y = acts[-1]
    cnt = mask.sum()
    diff = (y - target) * mask
    loss = float((diff ** 2).sum() / cnt)
    g = 2.0 * diff / cnt
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        w, b = params[li]
        gw, gb = conv_bwd_weight(acts[li], g)
        grads[li] = (gw, gb)
        if li > 0:
            g = conv_bwd_data(g, w)
            g = g * (acts[li] > 0)
    return loss, grads


def adam(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round FP32 values to bfloat16 (round to nearest even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)

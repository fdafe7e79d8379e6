"""Plain FP64 reference of the encoder-decoder layers (test infrastructure).

Each function is the definition of the operation written out with numpy,
in NHWC layout (x[b, y, x, c]); 3x3 weights are w[cout, tap, cin] with
tap = 3 (dy + 1) + (dx + 1) and zero padding.  Used only by tests to check
the GPU kernels of include/mdfnn.h; never imported by the product path.
"""
import numpy as np

TAPS = [(t // 3 - 1, t % 3 - 1) for t in range(9)]


def shifted(x, dy, dx):
    """s[b, y, x, c] = x[b, y + dy, x + dx, c], zero outside."""
    B, H, W, C = x.shape
    out = np.zeros_like(x)
    ys = slice(max(0, -dy), min(H, H - dy))
    xs = slice(max(0, -dx), min(W, W - dx))
    yd = slice(max(0, dy), min(H, H + dy))
    xd = slice(max(0, dx), min(W, W + dx))
    out[:, ys, xs, :] = x[:, yd, xd, :]
    return out


def conv3x3(x, w, bias=None):
    """y[b,y,x,co] = bias[co] + sum_{tap,ci} w[co,tap,ci] x[b,y+dy,x+dx,ci]."""
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (dy, dx) in enumerate(TAPS):
        y += np.tensordot(shifted(x, dy, dx), w[:, t, :], axes=([3], [1]))
    if bias is not None:
        y += bias
    return y


def conv3x3_dgrad(dy, w):
    """dx[b,y,x,ci] = sum_{tap,co} w[co,tap,ci] dy[b,y-dy,x-dx,co]."""
    dx = np.zeros(dy.shape[:3] + (w.shape[2],))
    for t, (ddy, ddx) in enumerate(TAPS):
        dx += np.tensordot(shifted(dy, -ddy, -ddx), w[:, t, :], axes=([3], [0]))
    return dx


def conv3x3_wgrad(x, dy):
    """dw[co,tap,ci] = sum_{b,y,x} dy[b,y,x,co] x[b,y+dy,x+dx,ci]; db = sum dy."""
    co, ci = dy.shape[3], x.shape[3]
    dw = np.zeros((co, 9, ci))
    for t, (ddy, ddx) in enumerate(TAPS):
        s = shifted(x, ddy, ddx)
        dw[:, t, :] = np.tensordot(dy, s, axes=([0, 1, 2], [0, 1, 2]))
    return dw, dy.sum(axis=(0, 1, 2))


def avgpool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_bwd(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_bwd(dy):
    B, H2, W2, C = dy.shape
    return dy.reshape(B, H2 // 2, 2, W2 // 2, 2, C).sum(axis=(2, 4))


def head(x, w, b):
    """y[p, o] = b[o] + sum_c w[o, c] x[p, c] over pixels p."""
    return x @ w.T + b


def head_bwd(x, dy, w):
    return dy @ w, dy.T @ x, dy.sum(axis=0)


def mse(y, t, wt):
    """L = sum_{p,c} wt[p] (y - t)^2 / (sum_p wt[p] C) and dL/dy."""
    C = y.shape[1]
    den = wt.sum() * C
    d = y - t
    return float((wt[:, None] * d * d).sum() / den), 2.0 * wt[:, None] * d / den


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

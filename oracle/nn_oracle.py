"""Oracle of the learned preconditioner network (test infrastructure only).

A 3D convolutional network over the spacetime grid [tau][y][x] of a 2+1D
spinor field, with the real and imaginary parts of the two spinor components
as 4 channels: conv 4->16, ReLU, 16->16, ReLU, 16->16, ReLU, 16->4, all with
3x3x3 taps, periodic padding in space and zero padding in time.  Plain FP64
numpy, written from the definitions of convolution, ReLU, the relative
squared-error loss and the Adam update.  Optional emulation of bfloat16
round-to-nearest-even at the points where the GPU kernels round (layer inputs,
weights, back-propagated gradients), so that results can be compared with the
GPU at tight tolerance.

Parameter vector layout (FP32 on the GPU, FP64 here): for each layer l,
W_l[27][cin][cout] then b_l[cout]; tap t = (dt+1)*9 + (dy+1)*3 + (dx+1).
"""
from __future__ import annotations

import numpy as np

CH = [4, 16, 16, 16, 4]
TAPS = [(dt, dy, dx) for dt in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def param_layout():
    out, off = [], 0
    for l in range(4):
        ci, co = CH[l], CH[l + 1]
        out.append((off, off + 27 * ci * co, off + 27 * ci * co + co, ci, co))
        off += 27 * ci * co + co
    return out, off


LAYOUT, NPARAM = param_layout()


def unpack(p):
    res = []
    for (w0, b0, e, ci, co) in LAYOUT:
        res.append((p[w0:b0].reshape(27, ci, co), p[b0:e]))
    return res


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(x, dt, dy, dx):
    """s[tau, y, x] = x[tau+dt, y+dy, x+dx]: periodic in y, x; zero outside time."""
    r = np.roll(x, shift=(-dy, -dx), axis=(1, 2))
    out = np.zeros_like(r)
    nt = x.shape[0]
    if dt == 0:
        out[:] = r
    elif dt > 0:
        out[:nt - dt] = r[dt:]
    else:
        out[-dt:] = r[:nt + dt]
    return out


def conv(x, W, b):
    """y[p, co] = b[co] + sum_{t, ci} x[p + t, ci] W[t, ci, co]."""
    y = np.zeros(x.shape[:3] + (W.shape[2],)) + b
    for t, (dt, dy, dx) in enumerate(TAPS):
        y += np.einsum("tyxc,co->tyxo", shift(x, dt, dy, dx), W[t])
    return y


def conv_transpose(g, W):
    """Adjoint of conv in its input: dx[q, ci] = sum_{t, co} g[q - t, co] W[t, ci, co]."""
    dx = np.zeros(g.shape[:3] + (W.shape[1],))
    for t, (dt, dy, dx_) in enumerate(TAPS):
        dx += shift(np.einsum("tyxo,co->tyxc", g, W[t]), -dt, -dy, -dx_)
    return dx


def weight_grad(x, g):
    """dW[t, ci, co] = sum_p x[p + t, ci] g[p, co]."""
    return np.stack([np.einsum("tyxc,tyxo->co", shift(x, dt, dy, dx), g) for (dt, dy, dx) in TAPS])


def forward(p, x, emulate=True):
    """x: [nt, ny, nx, 4].  Returns (out, activations a0..a3)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, np.float64))
    layers = unpack(p)
    a = [r(x)]
    for l, (W, b) in enumerate(layers):
        pre = conv(a[-1], r(W), b)
        if l < 3:
            a.append(r(np.maximum(pre, 0.0)))
        else:
            out = pre
    return out, a


def backward(p, acts, dout, emulate=True):
    """Gradients of the parameters for dL/dout (layout of the parameter vector)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, np.float64))
    layers = unpack(p)
    grad = np.zeros(NPARAM)
    g = r(dout)
    for l in range(3, -1, -1):
        W, b = layers[l]
        w0, b0, e, ci, co = LAYOUT[l]
        grad[w0:b0] = weight_grad(acts[l], g).reshape(-1)
        grad[b0:e] = g.sum(axis=(0, 1, 2))
        if l > 0:
            da = conv_transpose(g, r(W))
            g = r(da * (acts[l] > 0))
    return grad


def loss(out, target):
    """Relative squared error ||out - target||^2 / ||target||^2 and its gradient."""
    den = np.sum(target * target)
    d = out - target
    return np.sum(d * d) / den, 2.0 * d / den


def adam(p, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He initialisation of the weights (normal, std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM)
    for (w0, b0, e, ci, co) in LAYOUT:
        p[w0:b0] = rng.standard_normal(b0 - w0) * np.sqrt(2.0 / (27 * ci))
    return p


def as_channels(v, nt, ny, nx):
    """Complex spinor vector [nt][ny][nx][2] -> real channels [nt, ny, nx, 4]
    (re0, im0, re1, im1)."""
    return np.stack([v.real, v.imag], axis=-1).reshape(nt, ny, nx, 4)


def from_channels(c):
    c = c.reshape(-1, 2)
    return c[:, 0] + 1j * c[:, 1]


def precondition(p, v, nt, ny, nx, emulate=True):
    """z = (||v|| / sqrt(n)) N(v sqrt(n) / ||v||), n the number of complex entries."""
    n = v.size
    nv = np.linalg.norm(v)
    s = np.sqrt(n) / nv
    out, _ = forward(p, as_channels(v * s, nt, ny, nx), emulate)
    return from_channels(out) / s

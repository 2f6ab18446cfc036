"""Pins of the network oracle: a brute-force convolution, the adjoint identity,
central finite differences of the loss, bfloat16 rounding against torch's
conversion, and the closed form of the first Adam step."""
import numpy as np
import pytest
import torch

from oracle import nn_oracle as N


def test_parameter_count():
    # 4->16, 16->16, 16->16, 16->4 with 3x3x3 taps and biases
    assert N.NPARAM == 27 * (4 * 16 + 16 * 16 + 16 * 16 + 16 * 4) + 16 * 3 + 4 == 17332


def test_conv_matches_brute_force():
    rng = np.random.default_rng(0)
    nt, ny, nx, ci, co = 3, 4, 5, 2, 3
    x = rng.standard_normal((nt, ny, nx, ci))
    W = rng.standard_normal((27, ci, co))
    b = rng.standard_normal(co)
    y = N.conv(x, W, b)
    for t in range(nt):
        for j in range(ny):
            for i in range(nx):
                acc = b.copy()
                for dt in (-1, 0, 1):
                    if not 0 <= t + dt < nt:
                        continue          # zero padding in time
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            tap = (dt + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                            acc = acc + x[t + dt, (j + dy) % ny, (i + dx) % nx] @ W[tap]
                assert np.allclose(y[t, j, i], acc, atol=1e-13)


def test_conv_transpose_is_adjoint_and_weight_grad():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 3, 5, 3))
    g = rng.standard_normal((4, 3, 5, 2))
    W = rng.standard_normal((27, 3, 2))
    lhs = np.sum(N.conv(x, W, np.zeros(2)) * g)
    assert np.isclose(lhs, np.sum(x * N.conv_transpose(g, W)), rtol=1e-12)
    # d<conv(x, W), g>/dW equals weight_grad(x, g)
    assert np.isclose(lhs, np.sum(W * N.weight_grad(x, g)), rtol=1e-12)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(2)
    p = N.init_params(3) * 0.7
    p[N.LAYOUT[0][1]:N.LAYOUT[0][2]] = 0.05   # positive biases keep ReLUs away from kinks
    x = rng.standard_normal((3, 4, 4, 4))
    t = rng.standard_normal((3, 4, 4, 4))
    out, acts = N.forward(p, x, emulate=False)
    L, dout = N.loss(out, t)
    g = N.backward(p, acts, dout, emulate=False)
    idx = np.concatenate([rng.choice(N.NPARAM, 40, replace=False),
                          [N.LAYOUT[l][1] for l in range(4)]])   # include biases
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (N.loss(N.forward(pp, x, False)[0], t)[0] - N.loss(N.forward(pm, x, False)[0], t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7 * np.abs(g).max(), (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(4)
    a = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.bf16(a), ref)
    # ties go to even: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert N.bf16(1.0 + 2 ** -8) == 1.0 and N.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_adam_first_step():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = N.adam(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    # bias-corrected first step: lr * g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)


def test_precondition_is_scale_equivariant():
    rng = np.random.default_rng(5)
    p = N.init_params(6)
    v = rng.standard_normal(2 * 3 * 4 * 5 * 2)
    v = v[::2] + 1j * v[1::2]
    z1 = N.precondition(p, v, 3, 4, 5, emulate=False)
    z2 = N.precondition(p, 7.5 * v, 3, 4, 5, emulate=False)
    assert np.allclose(z2, 7.5 * z1, rtol=1e-12)

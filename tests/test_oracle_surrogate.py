"""Pins of the surrogate oracle (oracle/surrogate.py), none of which calls
the oracle against itself:
  * bfloat16 rounding: hand-worked ties and torch's own conversion;
  * the periodic 3x3 convolution against a brute-force loop; the identity
    kernel; commuting with circular shifts;
  * both backward products against central finite differences;
  * the network's backpropagation against finite differences of its own
    loss with the bf16 rounding switched off (which makes it smooth);
  * Adam's first two steps in closed form;
  * coarse-graining: hand-placed particles, total mass, an aligned state.
"""
import math

import numpy as np
import pytest

from oracle import surrogate as S


def test_bf16_rounding_by_hand_and_by_torch():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8 + 2 ** -12), 3.0e38,
                  1.5 * 2 ** -130, 0.0, -0.0, 65504.0, 1 / 3])
    r = S.to_bf16(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # tie: to the even neighbour
    assert r[2] == 1 + 2 ** -6               # tie: 1 + 2^-6 has the even last bit
    assert r[3] == -(1 + 2 ** -7)            # above the tie: away from 1
    import torch
    t = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(r, t)
    g = np.random.default_rng(0).normal(0, 10, 10000)
    t = torch.tensor(g, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.to_bf16(g), t)


def _brute_conv(x, w, b):
    H, W, Ci = x.shape
    Co = w.shape[3]
    y = np.zeros((H, W, Co))
    for i in range(H):
        for j in range(W):
            for o in range(Co):
                s = b[o]
                for a in range(3):
                    for c in range(3):
                        for k in range(Ci):
                            s += x[(i + a - 1) % H, (j + c - 1) % W, k] * w[a, c, k, o]
                y[i, j, o] = s
    return y


def test_conv_against_brute_force():
    g = np.random.default_rng(1)
    x = g.normal(size=(5, 4, 3))
    w = g.normal(size=(3, 3, 3, 2))
    b = g.normal(size=2)
    assert np.allclose(S.conv3x3(x, w, b), _brute_conv(x, w, b), atol=1e-12)


def test_conv_identity_and_shift_equivariance():
    g = np.random.default_rng(2)
    x = g.normal(size=(8, 6, 4))
    w = np.zeros((3, 3, 4, 4))
    w[1, 1] = np.eye(4)
    assert np.allclose(S.conv3x3(x, w), x)
    w = g.normal(size=(3, 3, 4, 5))
    y = S.conv3x3(x, w)
    xs = np.roll(x, (3, -2), axis=(0, 1))
    assert np.allclose(S.conv3x3(xs, w), np.roll(y, (3, -2), axis=(0, 1)), atol=1e-12)
    # a kernel with one tap at (a, c) reads x[i + a - 1, j + c - 1]
    w = np.zeros((3, 3, 4, 4))
    w[0, 2] = np.eye(4)
    assert np.allclose(S.conv3x3(x, w), np.roll(x, (1, -1), axis=(0, 1)))


def test_backward_products_against_finite_differences():
    g = np.random.default_rng(3)
    x = g.normal(size=(5, 6, 3))
    w = g.normal(size=(3, 3, 3, 4))
    b = g.normal(size=4)
    gy = g.normal(size=(5, 6, 4))
    L = lambda x_, w_, b_: float(np.sum(S.conv3x3(x_, w_, b_) * gy))
    dx = S.conv3x3_grad_input(gy, w)
    dw, db = S.conv3x3_grad_weights(x, gy)
    h = 1e-6
    for idx in [(0, 0, 0), (4, 5, 2), (2, 3, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((L(x + e, w, b) - L(x - e, w, b)) / (2 * h) - dx[idx]) < 1e-6
    for idx in [(0, 0, 0, 0), (2, 1, 2, 3), (1, 2, 0, 1)]:
        e = np.zeros_like(w)
        e[idx] = h
        assert abs((L(x, w + e, b) - L(x, w - e, b)) / (2 * h) - dw[idx]) < 1e-6
    e = np.zeros_like(b)
    e[2] = h
    assert abs((L(x, w, b + e) - L(x, w, b - e)) / (2 * h) - db[2]) < 1e-6


def test_network_backprop_against_finite_differences(monkeypatch):
    monkeypatch.setattr(S, "to_bf16", lambda a: np.asarray(a, np.float64))
    g = np.random.default_rng(4)
    params = S.init_params(seed=5)
    for p in params:
        p[1] = g.normal(0, 0.05, p[1].shape)
    params[3][1][3:] = 0.0
    u = np.zeros((6, 5, S.C_IN))
    u[..., :3] = g.normal(0, 0.3, (6, 5, 3))
    target = u[..., :3] + g.normal(0, 0.1, (6, 5, 3))
    loss, _, grads = S.loss_and_grads(params, u, target)
    h = 1e-6
    checks = [(0, 0, (1, 1, 0, 3)), (1, 0, (0, 2, 5, 7)), (2, 0, (2, 0, 31, 1)),
              (3, 0, (1, 1, 4, 2)), (0, 1, (5,)), (3, 1, (1,))]
    for layer, which, idx in checks:
        p = params[layer][which]
        old = p[idx]
        p[idx] = old + h
        lp = S.loss_and_grads(params, u, target)[0]
        p[idx] = old - h
        lm = S.loss_and_grads(params, u, target)[0]
        p[idx] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grads[layer][which][idx]) < 1e-7 + 1e-5 * abs(fd), (layer, which, idx)


def test_adam_first_two_steps():
    g1 = np.array([0.5, -2.0, 1e-3])
    g2 = np.array([-1.0, -1.0, 2e-3])
    p = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    S.adam_step(p, g1, m, v, 1, lr, b1, b2, eps)
    assert np.allclose(p, -lr * g1 / (np.abs(g1) + eps), rtol=1e-12)
    p1 = p.copy()
    S.adam_step(p, g2, m, v, 2, lr, b1, b2, eps)
    mh = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    assert np.allclose(p, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=1e-12)


def test_coarse_graining_by_hand():
    L, G = 16.0, 4            # bins of side 4, area 16
    x = np.array([0.0, 3.999, 4.0, 15.99, 16.0, 9.0])
    y = np.array([0.0, 0.5, 0.5, 15.99, 8.0, 9.0])
    th = np.array([0.0, math.pi / 2, math.pi, -math.pi / 2, 0.3, 1.0])
    rho, px, py = S.coarse_grain(x, y, th, L, G)
    assert rho[0, 0] == 2 / 16 and rho[0, 1] == 1 / 16 and rho[3, 3] == 1 / 16
    assert rho[2, 3] == 1 / 16 and rho[2, 2] == 1 / 16       # x = L clamps into the last bin
    assert abs(px[0, 0] - 1 / 16) < 1e-15 and abs(py[0, 0] - 1 / 16) < 1e-15
    assert abs(px[0, 1] + 1 / 16) < 1e-15 and abs(py[3, 3] + 1 / 16) < 1e-15
    assert abs(rho.sum() * 16 - len(x)) < 1e-12


def test_coarse_graining_aligned_state():
    g = np.random.default_rng(6)
    N, L, G, a = 20000, 32.0, 8, 0.7
    x, y = g.uniform(0, L, N), g.uniform(0, L, N)
    rho, px, py = S.coarse_grain(x, y, np.full(N, a), L, G)
    assert np.allclose(px, rho * math.cos(a)) and np.allclose(py, rho * math.sin(a))
    assert abs(S.polar_order(rho, px, py) - 1.0) < 1e-12
    u = S.network_input(rho, px, py, N / L ** 2)
    assert u.shape == (G, G, S.C_IN) and not u[..., 3:].any()
    assert abs(u[..., 0].mean()) < 1e-12

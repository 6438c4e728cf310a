"""Oracle of the learned field surrogate -- TEST INFRASTRUCTURE ONLY.

Plain numpy (binary64) statement of what the surrogate's GPU kernels compute:
the coarse-graining of a particle state onto a grid of fields, a 3x3
periodic convolution layer (forward, the two backward products), the loss
and the Adam update.  Only tests/, the smoke check and the benchmark's CPU
baseline use it; the library never does, and it shares no code with the
HIP kernels.

Definitions followed:
  * fields of a state (Sec. 3.4 measures the same quantities globally): on a
    G x G grid of square bins of side L / G, the number density
    rho = n / (L / G)^2 and the polarisation density p = sum e^{i theta} /
    (L / G)^2 of the particles in each bin; a particle's bin is
    floor(x G / L) in binary64 from its binary32 coordinate, clamped to
    G - 1;
  * the network input u = (rho / rho0 - 1, p_x / rho0, p_y / rho0), rho0 =
    N / L^2, zero-padded to 16 channels; channel-last layout [H, W, C];
  * conv: y[i, j, o] = b[o] + sum_{a, c in 0..2} sum_k
    x[(i + a - 1) mod H, (j + c - 1) mod W, k] w[a, c, k, o]  (periodic box,
    so circular padding), weights [3, 3, Cin, Cout];
  * network: three conv + ReLU layers (16 -> 32 -> 32 -> 32 channels) and a
    linear conv layer (32 -> 16); prediction = u + output, first three
    channels; activations between layers and all weights are rounded to
    bfloat16 (round to nearest even), products accumulated exactly here;
  * loss: mean of (prediction - target)^2 over the three channels and the
    grid; Adam (Kingma and Ba, ICLR 2015) with bias correction.
"""
import numpy as np

G_DEFAULT = 128
C_IN = 16          # padded input channels
C_HID = 32
C_OUT = 16         # padded output channels (three used)


# --------------------------------------------------------------------------
# bfloat16: round to nearest, ties to even, of a binary32 value
# --------------------------------------------------------------------------
def to_bf16(a):
    """Values of a (rounded first to binary32) rounded to bfloat16, as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# coarse-graining
# --------------------------------------------------------------------------
def coarse_grain(x, y, th, L, G=G_DEFAULT):
    """(rho, p_x, p_y) on a G x G grid, arrays [G, G] indexed [row (y), col (x)]."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    th = np.asarray(th, np.float64)
    s = G / L
    bx = np.minimum((x * s).astype(np.int64), G - 1)
    by = np.minimum((y * s).astype(np.int64), G - 1)
    area = (L / G) ** 2
    rho = np.zeros((G, G))
    px = np.zeros((G, G))
    py = np.zeros((G, G))
    np.add.at(rho, (by, bx), 1.0)
    np.add.at(px, (by, bx), np.cos(th))
    np.add.at(py, (by, bx), np.sin(th))
    return rho / area, px / area, py / area


def network_input(rho, px, py, rho0):
    """u = (rho / rho0 - 1, p / rho0), [G, G, 16] with channels 3..15 zero."""
    G = rho.shape[0]
    u = np.zeros((G, G, C_IN))
    u[..., 0] = rho / rho0 - 1.0
    u[..., 1] = px / rho0
    u[..., 2] = py / rho0
    return u


# --------------------------------------------------------------------------
# 3x3 periodic convolution and its two backward products
# --------------------------------------------------------------------------
def conv3x3(x, w, b=None):
    """x [H, W, Cin], w [3, 3, Cin, Cout] -> [H, W, Cout] (binary64)."""
    H, W, _ = x.shape
    out = np.zeros((H, W, w.shape[3]))
    for a in range(3):
        for c in range(3):
            xs = np.roll(x, shift=(1 - a, 1 - c), axis=(0, 1))   # xs[i, j] = x[i + a - 1, j + c - 1]
            out += xs @ w[a, c]
    if b is not None:
        out += b
    return out


def conv3x3_grad_input(dy, w):
    """dL/dx of y = conv3x3(x, w) given dL/dy: each x[i', j'] feeds
    y[i' - a + 1, j' - c + 1] through w[a, c]."""
    H, W, _ = dy.shape
    dx = np.zeros((H, W, w.shape[2]))
    for a in range(3):
        for c in range(3):
            ds = np.roll(dy, shift=(a - 1, c - 1), axis=(0, 1))   # ds[i, j] = dy[i - a + 1, j - c + 1]
            dx += ds @ w[a, c].T
    return dx


def conv3x3_grad_weights(x, dy):
    """dL/dw [3, 3, Cin, Cout] and dL/db [Cout] of y = conv3x3(x, w, b)."""
    Cin, Cout = x.shape[2], dy.shape[2]
    dw = np.zeros((3, 3, Cin, Cout))
    dyf = dy.reshape(-1, Cout)
    for a in range(3):
        for c in range(3):
            xs = np.roll(x, shift=(1 - a, 1 - c), axis=(0, 1)).reshape(-1, Cin)
            dw[a, c] = xs.T @ dyf
    return dw, dyf.sum(axis=0)


# --------------------------------------------------------------------------
# the network
# --------------------------------------------------------------------------
def init_params(seed=0, scale=1.0):
    """He-initialised weights (normal, std sqrt(2 / fan_in)), zero biases;
    the last layer's unused output channels are zero.  Weights are kept in
    binary64; the network rounds them to bfloat16 where it uses them."""
    g = np.random.default_rng(seed)
    shapes = [(C_IN, C_HID), (C_HID, C_HID), (C_HID, C_HID), (C_HID, C_OUT)]
    params = []
    for k, (ci, co) in enumerate(shapes):
        fan_in = 9 * (3 if k == 0 else ci)
        w = g.normal(0.0, scale * np.sqrt(2.0 / fan_in), (3, 3, ci, co))
        if k == 0:
            w[:, :, 3:, :] = 0.0
        if k == 3:
            w[..., 3:] = 0.0
            w *= 0.1
        params.append([w, np.zeros(co)])
    return params


def forward(params, u):
    """Activations [a0 = bf16(u), a1, a2, a3] (bf16 values) and the
    prediction [H, W, 3] (binary64)."""
    acts = [to_bf16(u)]
    for k in range(3):
        w, b = params[k]
        z = conv3x3(acts[-1], to_bf16(w), b)
        acts.append(to_bf16(np.maximum(z, 0.0)))
    w, b = params[3]
    out = conv3x3(acts[-1], to_bf16(w), b)
    pred = u[..., :3] + out[..., :3]
    return acts, pred


def loss_and_grads(params, u, target):
    """MSE loss and the gradients of every weight and bias (binary64, with
    the bf16 operands of the forward pass; the backpropagated gradients are
    rounded to bf16 where the GPU feeds them to a product)."""
    acts, pred = forward(params, u)
    diff = pred - target
    n = diff.size
    loss = float(np.mean(diff ** 2))
    dout = np.zeros(acts[-1].shape[:2] + (C_OUT,))
    dout[..., :3] = 2.0 * diff / n
    grads = [None] * 4
    dy = to_bf16(dout)
    for k in range(3, -1, -1):
        w, _ = params[k]
        dw, db = conv3x3_grad_weights(acts[k], dy)
        grads[k] = [dw, db]
        if k > 0:
            dx = conv3x3_grad_input(dy, to_bf16(w))
            dy = to_bf16(dx * (acts[k] > 0.0))
    return loss, pred, grads


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t >= 1) in place; returns nothing."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p -= lr * mh / (np.sqrt(vh) + eps)


def polar_order(rho, px, py):
    """|sum p| / sum rho of a field (the coarse-grained polar order)."""
    return float(np.hypot(px.sum(), py.sum()) / rho.sum())

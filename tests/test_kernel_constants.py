"""The numerical constants written into the HIP kernels, checked against the
mathematics on the CPU (no GPU, no oracle): the polynomial arctangent of
the Vicsek update and the Cody-Waite split of pi/2 of the sine/cosine.
The binary32 arithmetic of the kernels is emulated with numpy float32."""
import math
import os
import re
from fractions import Fraction

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2211_15630_amd", "csrc", "aap_kernels.hip")
PI = Fraction("3.14159265358979323846264338327950288419716939937510582097494459")


def _body(start, end):
    s = open(SRC).read()
    i = s.index(start)
    return s[i:s.index(end, i)]


def test_polynomial_arctangent_error_bound():
    body = _body("float atan2_poly", "return __builtin_copysignf")
    c = [np.float32(float.fromhex(t)) for t in re.findall(r"(-?0x1\.[0-9a-f]+p-?\d+)f", body)]
    assert len(c) == 8
    f32 = np.float32
    rng = np.random.default_rng(3)
    t = np.concatenate([np.linspace(-math.pi, math.pi, 400001),
                        [0.0, math.pi / 4, -math.pi / 4, math.pi / 2, math.pi]])
    r = np.exp(rng.uniform(-6, 6, t.size))
    x = (r * np.cos(t)).astype(f32)
    y = (r * np.sin(t)).astype(f32)
    ax, ay = np.abs(x), np.abs(y)
    mn, mx = np.minimum(ax, ay), np.maximum(ax, ay)
    a = (mn / mx).astype(f32)
    s = (a * a).astype(f32)
    p = c[0]
    for v in c[1:]:
        p = (p * s + v).astype(f32)
    res = (a * p).astype(f32)
    res = np.where(ay > ax, f32(1.57079637) - res, res).astype(f32)
    res = np.where(x < 0, f32(3.14159274) - res, res).astype(f32)
    res = np.copysign(res, y)
    exact = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    err = np.abs((res - exact + math.pi) % (2 * math.pi) - math.pi)
    assert err.max() < 3.5e-7


def test_cody_waite_split_of_half_pi():
    body = _body("void sincos_small", "const float s = r * r;")
    parts = [Fraction(float.fromhex(t)) for t in re.findall(r"(-?0x1\.[0-9a-f]+p[-+]?\d+)f", body)]
    # P1 + P2 + P3 = pi/2 to far below binary32 precision, each part exact in binary32
    assert len(parts) == 3
    assert all(float(np.float32(float(v))) == float(v) for v in parts)
    assert abs(sum(parts) - PI / 2) < Fraction(1, 2 ** 72)
    # each part holds the leading bits of what remains
    assert abs(parts[0] - PI / 2) < Fraction(1, 2 ** 23)
    assert abs(parts[0] + parts[1] - PI / 2) < Fraction(1, 2 ** 47)


def _lawson_arctan(deg=7, npts=4001, iters=200):
    """Minimax fit of atan(a) by a P(a^2) on [0, 1] (P of degree deg) with
    Lawson's iteratively reweighted least squares: start from equal weights
    on Chebyshev-distributed nodes, solve the weighted least-squares problem,
    multiply each weight by the node's absolute error, normalise, repeat.
    The weights concentrate on the extrema and the error curve approaches
    equioscillation.  Returns (coefficients in ascending powers of a^2,
    maximum absolute error on the nodes)."""
    a = 0.5 + 0.5 * np.cos(np.linspace(math.pi, 0.0, npts))
    A = a[:, None] * (a * a)[:, None] ** np.arange(deg + 1)[None, :]
    f = np.arctan(a)
    w = np.full(npts, 1.0 / npts)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(A * sw[:, None], f * sw, rcond=None)
        e = np.abs(A @ c - f)
        w = w * e
        w /= w.sum()
    return c, float(e.max())


def test_arctangent_polynomial_is_the_lawson_minimax_fit():
    """How the kernel's coefficients were obtained: the degree-7 (in a^2)
    Lawson fit above, rounded to binary32 and adjusted by a few ulps.  The
    refit lands within 5e-7 of every kernel coefficient, its error
    equioscillates at 3.75e-8, and the kernel's polynomial (evaluated
    exactly) stays within twice that optimum -- far below the binary32
    evaluation error checked above."""
    c, emax = _lawson_arctan()
    assert 3.5e-8 < emax < 4.0e-8
    body = _body("float atan2_poly", "return __builtin_copysignf")
    k = [float.fromhex(t) for t in re.findall(r"(-?0x1\.[0-9a-f]+p-?\d+)f", body)][::-1]
    assert np.max(np.abs(np.array(k) - c)) < 5e-7
    a = np.linspace(0.0, 1.0, 200001)
    s = a * a
    pk = a * sum(kj * s ** j for j, kj in enumerate(k))
    ek = np.abs(pk - np.arctan(a))
    assert ek.max() < 2.0 * emax
    # near-equioscillation of the refit: its error reaches the maximum at
    # deg + 2 = 9 alternating extrema (counted as sign changes of the error)
    pr = a * sum(cj * s ** j for j, cj in enumerate(c))
    er = pr - np.arctan(a)
    big = np.abs(er) > 0.9 * emax
    signs = np.sign(er[big])
    assert np.count_nonzero(np.diff(signs)) + 1 >= 8

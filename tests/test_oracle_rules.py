"""Pins of the oracle's rule variants: the nematic Vicsek model (Eq. (3))
and the interaction order o of the Langevin dynamics (Eq. (5)).

  * the sign of Eq. (3) equals the sign of cos(th_i - th~_j) evaluated in
    exact rational arithmetic (pi to 80 digits) for binary32 angles,
    including pairs whose difference is within an ulp of +-pi/2 and
    +-3pi/2, tiny angles and every mirror combination;
  * two NVM particles with no noise: partners within pi/2 take the
    bisector, partners further apart end antiparallel on the bisector of
    one angle and the other turned by pi;
  * NVM: turning a subset of particles by pi leaves every other new angle
    unchanged and turns theirs by pi (nematic symmetry); VM does not;
  * NVM = VM on states whose angles all lie within a quarter turn;
  * NVM next to a reflecting wall: the mirror image's sign is taken with
    the mirrored angle (hand-derived sums);
  * order o: two particles give A = +-sin(o phi); o = 2 is blind to turns
    by pi; the mirror image enters as sin(o (pi - th_j - th_i)); one
    Euler step of the Langevin dynamics with o = 3 by hand.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

PI = Fraction("3.14159265358979323846264338327950288419716939937510582097494459230781640628620899")


def _exact_sign(thi, thj, mx, my):
    """sign(cos(th_i - th~_j)) from the definition, in rationals."""
    t = Fraction(float(thj))
    if mx:
        t = PI - t
    if my:
        t = -t
    d = Fraction(float(thi)) - t
    # reduce to (-pi, pi]: cos >= 0 iff |d| <= pi/2
    k = math.floor((d + PI) / (2 * PI))
    d -= 2 * PI * k
    return 1 if abs(d) <= PI / 2 else -1


def _adversarial_pairs(rng, count):
    f32 = np.float32
    out = []
    ti = rng.uniform(-math.pi, math.pi, count).astype(f32)
    for a in ti:
        a64 = float(a)
        for base in (a64 - math.pi / 2, a64 + math.pi / 2, a64 - 1.5 * math.pi,
                     a64 + 1.5 * math.pi, -a64 + math.pi / 2, -a64 - math.pi / 2,
                     math.pi / 2 - a64 + math.pi, -a64 + 1.5 * math.pi):
            b = (base + math.pi) % (2 * math.pi) - math.pi
            c = f32(b)
            for _ in range(3):
                out.append((a, c))
                c = np.nextafter(c, f32(4))
            c = f32(b)
            for _ in range(2):
                c = np.nextafter(c, f32(-4))
                out.append((a, c))
    return out


def test_nvm_sign_is_exact(orc):
    rng = np.random.default_rng(17)
    pairs = _adversarial_pairs(rng, 60)
    f32 = np.float32
    h = f32(math.pi / 2)
    tiny = [f32(1e-30), f32(-1e-30), f32(2.0 ** -29), f32(0.0), f32(3e-9)]
    for hv in (h, np.nextafter(h, f32(0)), -h, np.nextafter(-h, f32(0))):
        for tv in tiny:
            pairs += [(hv, tv), (tv, hv)]
    pi32 = f32(math.pi)
    pairs += [(pi32, -pi32), (pi32, f32(math.pi / 2)), (-pi32, f32(-math.pi / 2)),
              (f32(0), f32(0)), (pi32, pi32)]
    pairs += [(f32(a), f32(b)) for a, b in rng.uniform(-math.pi, math.pi, (200, 2))]
    wrong = []
    for a, b in pairs:
        for mx in (0, 1):
            for my in (0, 1):
                if orc.nvm_sign(float(a), float(b), mx, my) != _exact_sign(a, b, mx, my):
                    wrong.append((float(a), float(b), mx, my))
    assert not wrong, wrong[:5]
    assert len(pairs) > 1000


def _two(orc, phi, rule, order=1, L=10.0, **kw):
    p = orc.Params(N=2, Lx=L, Ly=L, v=0.5, eta=0.0, rule=rule, order=order, **kw)
    x = np.array([5.0, 5.4])
    y = np.array([5.0, 5.3])
    th = np.array([0.0, phi])
    return p, orc.step(x, y, th, p, 0)


def _ang(a, b):
    return abs((a - b + math.pi) % (2 * math.pi) - math.pi)


@pytest.mark.parametrize("phi", [0.4, -1.2, 1.5, 1.7, 2.5, -2.9, 3.1])
def test_nvm_two_particles(orc, phi):
    _, (_, _, tn, n, C, S, A) = _two(orc, phi, orc.RULE_NVM)
    assert n.tolist() == [1, 1]
    if abs(phi) < math.pi / 2:
        assert _ang(tn[0], phi / 2) < 1e-12 and _ang(tn[1], phi / 2) < 1e-12
    else:
        # the partner enters as e^{i (angle + pi)}: bisectors of (0, phi + pi)
        # and (phi, pi)
        assert _ang(tn[0], (phi - math.copysign(math.pi, phi)) / 2) < 1e-12
        assert _ang(tn[1], (phi + math.copysign(math.pi, phi)) / 2) < 1e-12
        assert _ang(tn[1], tn[0] + math.pi) < 1e-12


def test_nvm_nematic_symmetry(orc):
    rng = np.random.default_rng(8)
    N, L = 600, 12.0
    x, y = rng.uniform(0, L, N), rng.uniform(0, L, N)
    th = rng.uniform(-math.pi, math.pi, N)
    flip = rng.random(N) < 0.5
    th2 = np.where(flip, th - math.pi, th)
    th2 = np.where(th2 < -math.pi, th2 + 2 * math.pi, th2)
    for rule, symmetric in ((2, True), (0, False)):
        p = orc.Params(N=N, Lx=L, Ly=L, v=0.5, eta=0.4, rule=rule, seed=3)
        _, _, t1, *_ = orc.step(x, y, th, p, 5)
        _, _, t2, *_ = orc.step(x, y, th2, p, 5)
        d = _ang(t2, np.where(flip, t1 + math.pi, t1))
        if symmetric:
            assert np.all(d < 1e-9)
        else:
            assert np.mean(d > 1e-3) > 0.5


def test_nvm_equals_vm_within_a_quarter_turn(orc):
    rng = np.random.default_rng(4)
    N, L = 800, 14.0
    x, y = rng.uniform(0, L, N), rng.uniform(0, L, N)
    th = rng.uniform(-0.7, 0.7, N)
    pv = orc.Params(N=N, Lx=L, Ly=L, v=0.5, eta=0.2, rule=orc.RULE_VM, seed=1)
    pn = orc.Params(N=N, Lx=L, Ly=L, v=0.5, eta=0.2, rule=orc.RULE_NVM, seed=1)
    a = orc.step(x, y, th, pv, 2)
    b = orc.step(x, y, th, pn, 2)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_nvm_at_reflecting_wall_by_hand(orc):
    # i at x = 0.2, j at x = 0.5 (same y) next to the wall x = 0; R = 1.
    # j is a neighbour directly (distance 0.3) and through its mirror image
    # at x = -0.5 (distance 0.7) with angle pi - th_j; i's own image at -0.2
    # is not a neighbour.
    ti, tj = 0.3, 2.0
    p = orc.Params(N=2, Lx=10, Ly=10, v=0.5, eta=0.0, rule=orc.RULE_NVM, bx=1, by=1)
    n, C, S, _ = orc.neighbours_brute([0.2, 0.5], [5.0, 5.0], [ti, tj], p)
    # direct: cos(0.3 - 2.0) < 0 -> -e^{i 2.0}; image: cos(0.3 - (pi - 2)) > 0
    Ce = math.cos(ti) - math.cos(tj) + math.cos(math.pi - tj)
    Se = math.sin(ti) - math.sin(tj) + math.sin(math.pi - tj)
    assert n[0] == 2 and abs(C[0] - Ce) < 1e-14 and abs(S[0] - Se) < 1e-14
    # j sees i directly (cos(2 - 0.3) < 0 -> -e^{0.3 i}) and i's image at
    # -0.2 (distance 0.7, angle pi - 0.3: cos(2 - pi + 0.3) > 0); j's own
    # image at -0.5 is 1.0 away but is j itself
    Ce = math.cos(tj) - math.cos(ti) + math.cos(math.pi - ti)
    Se = math.sin(tj) - math.sin(ti) + math.sin(math.pi - ti)
    assert n[1] == 2 and abs(C[1] - Ce) < 1e-14 and abs(S[1] - Se) < 1e-14
    nc, Cc, Sc, _ = orc.neighbours_cells([0.2, 0.5], [5.0, 5.0], [ti, tj], p)
    assert np.array_equal(nc, n) and np.allclose(Cc, C, atol=1e-14) and np.allclose(Sc, S, atol=1e-14)


@pytest.mark.parametrize("order", [1, 2, 3, 5])
@pytest.mark.parametrize("phi", [0.3, 1.9, -2.6])
def test_order_two_particles(orc, order, phi):
    p = orc.Params(N=2, Lx=10, Ly=10, rule=orc.RULE_LANGEVIN, order=order, dt=0.1)
    _, _, _, A = orc.neighbours_brute([5.0, 5.4], [5.0, 5.3], [0.0, phi], p)
    assert abs(A[0] - math.sin(order * phi)) < 1e-14
    assert abs(A[1] + math.sin(order * phi)) < 1e-14


def test_order_two_blind_to_half_turns(orc):
    rng = np.random.default_rng(21)
    N, L = 500, 10.0
    x, y = rng.uniform(0, L, N), rng.uniform(0, L, N)
    th = rng.uniform(-math.pi, math.pi, N)
    th2 = np.where(rng.random(N) < 0.5, th + math.pi, th)
    for order, same in ((2, True), (4, True), (1, False), (3, False)):
        p = orc.Params(N=N, Lx=L, Ly=L, rule=orc.RULE_LANGEVIN, order=order, dt=0.1)
        A1 = orc.neighbours_cells(x, y, th, p)[3]
        A2 = orc.neighbours_cells(x, y, th2, p)[3]
        assert (np.max(np.abs(A1 - A2)) < 1e-11) == same


@pytest.mark.parametrize("order", [2, 3])
def test_order_mirror_image_by_hand(orc, order):
    # the geometry of the wall test above, y wall and x wall in turn
    ti, tj = 0.3, 2.0
    p = orc.Params(N=2, Lx=10, Ly=10, rule=orc.RULE_LANGEVIN, order=order, dt=0.1, bx=1, by=1)
    _, _, _, A = orc.neighbours_brute([0.2, 0.5], [5.0, 5.0], [ti, tj], p)
    Ae = math.sin(order * (tj - ti)) + math.sin(order * (math.pi - tj - ti))
    assert abs(A[0] - Ae) < 1e-14
    _, _, _, A = orc.neighbours_brute([5.0, 5.0], [0.2, 0.5], [ti, tj], p)
    Ae = math.sin(order * (tj - ti)) + math.sin(order * (-tj - ti))
    assert abs(A[0] - Ae) < 1e-14


def test_langevin_order_three_euler_step(orc):
    phi, dt, gamma, om = 0.8, 0.05, 1.5, 0.2
    p = orc.Params(N=2, Lx=10, Ly=10, v=0.5, eta=0.0, omega=om, gamma=gamma, dt=dt,
                   rule=orc.RULE_LANGEVIN, order=3)
    x, y, th = np.array([5.0, 5.4]), np.array([5.0, 5.3]), np.array([0.0, phi])
    xn, yn, tn, *_ = orc.step(x, y, th, p, 0)
    assert abs(tn[0] - (dt * (gamma * math.sin(3 * phi) + om))) < 1e-14
    assert abs(tn[1] - (phi + dt * (-gamma * math.sin(3 * phi) + om))) < 1e-14
    # positions with the old angles (Euler-Maruyama)
    assert abs(xn[1] - (5.4 + 0.5 * dt * math.cos(phi))) < 1e-14

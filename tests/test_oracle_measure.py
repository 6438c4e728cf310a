"""Pins of the oracle's measurement suite (Sec. 3.4): the nematic order
parameter q and the histograms of the angles and of the neighbour numbers.

  * q closed forms: two particles at 0 and phi give p = |cos(phi/2)| and
    q = |cos phi|; a state split evenly between a and a + pi has p = 0 and
    q = 1; three- and four-fold symmetric states have q = 0; q does not
    change when any subset of particles is turned by pi (p does);
  * angle bins cover [-pi, pi) in equal parts: hand-placed angles, the
    clamp of +pi into the last bin;
  * neighbour-number bins: n >= bins - 1 fall into the last bin;
  * every measured state adds N to each histogram, and the mean read off
    the neighbour histogram is the nbar series' mean;
  * eta = 1: new angles are i.i.d. uniform and positions stay i.i.d.
    uniform, so the angle histogram is flat and n of one particle is
    Binomial(N - 1, pi R^2 / (Lx Ly)) on a periodic box with R < L / 2;
  * a run split in two at step K equals the whole run (noise keyed by
    the step, Sec. 2.5), including q and the histograms.
"""
import math

import numpy as np
import pytest
from scipy import stats


def _q(orc, th):
    return orc.state_observables(np.asarray(th, np.float64), np.zeros(len(th), np.int64))


@pytest.mark.parametrize("phi", [0.0, 0.3, 1.2, math.pi / 2, 2.5, math.pi])
def test_two_particles_p_and_q(orc, phi):
    p, _, q = _q(orc, [0.0, phi])
    assert abs(p - abs(math.cos(phi / 2))) < 1e-15
    assert abs(q - abs(math.cos(phi))) < 1e-15


def test_antiparallel_state_is_nematic(orc):
    rng = np.random.default_rng(3)
    a = 0.7
    th = np.where(np.arange(1000) % 2 == 0, a, a - math.pi)
    rng.shuffle(th)
    p, _, q = _q(orc, th)
    assert p < 1e-14 and abs(q - 1.0) < 1e-14
    p, _, q = _q(orc, np.full(17, -2.2))
    assert abs(p - 1.0) < 1e-14 and abs(q - 1.0) < 1e-14


@pytest.mark.parametrize("k", [3, 4, 6])
def test_k_fold_symmetric_states_have_no_nematic_order(orc, k):
    th = 0.4 + 2 * math.pi * np.arange(5 * k) / k
    th = (th + math.pi) % (2 * math.pi) - math.pi
    p, _, q = _q(orc, th)
    assert p < 1e-13 and q < 1e-13


def test_q_blind_to_half_turns(orc):
    rng = np.random.default_rng(11)
    th = rng.normal(0.3, 0.5, 500)
    flip = rng.random(500) < 0.4
    th2 = np.where(flip, th - math.pi, th)
    p1, _, q1 = _q(orc, th)
    p2, _, q2 = _q(orc, th2)
    assert abs(q1 - q2) < 1e-13
    assert p1 - p2 > 0.2


def test_q_of_isotropic_angles(orc):
    # E[q^2] = 1/N for i.i.d. uniform angles
    rng = np.random.default_rng(5)
    N, T = 64, 4000
    q2 = np.array([_q(orc, rng.uniform(-math.pi, math.pi, N))[2] ** 2 for _ in range(T)])
    assert abs(q2.mean() - 1 / N) < 5 * q2.std() / math.sqrt(T)


def test_angle_bins_by_hand(orc):
    # four bins: [-pi,-pi/2), [-pi/2,0), [0,pi/2), [pi/2,pi); +pi is clamped
    th = np.array([-math.pi, -3.0, -1.0, -1e-9, 0.0, 1.0, 1.6, 3.0, math.pi])
    ht, hn = orc.histograms(th, np.zeros(len(th), np.int64), 4, 1)
    assert ht.tolist() == [2, 2, 2, 3]
    assert hn.tolist() == [len(th)]
    ht, _ = orc.histograms(th, np.zeros(len(th), np.int64), 3, 2)
    # thirds: [-pi,-pi/3), [-pi/3,pi/3), [pi/3,pi)
    assert ht.tolist() == [2, 4, 3]
    # angles outside [-pi, pi] fall into the end bins
    ht, _ = orc.histograms(np.array([-7.0, 7.0, 1e30, -1e30]), np.zeros(4, np.int64), 5, 1)
    assert ht.tolist() == [2, 0, 0, 0, 2]


def test_neighbour_bins_saturate(orc):
    n = np.array([0, 1, 2, 3, 7, 100, 2], np.int64)
    _, hn = orc.histograms(np.zeros(len(n)), n, 1, 4)
    assert hn.tolist() == [1, 1, 2, 3]
    _, hn = orc.histograms(np.zeros(len(n)), n, 1, 200)
    assert hn[[0, 1, 2, 3, 7, 100]].tolist() == [1, 1, 2, 1, 1, 1] and hn.sum() == len(n)


def test_histograms_count_every_measured_state(orc):
    N, L, T = 512, 16.0, 40
    p = orc.Params(N=N, Lx=L, Ly=L, v=0.5, eta=0.3, seed=4)
    x, y, th = orc.init_state(p)
    _, _, _, m = orc.run_measured(x, y, th, p, 0, T, bins=(24, 64))
    assert m["hist_theta"].sum() == N * T and m["hist_n"].sum() == N * T
    # 64 bins hold every count at this density, so the histogram's mean is nbar
    mean_n = np.dot(np.arange(64), m["hist_n"]) / (N * T)
    assert abs(mean_n - m["nbar"].mean()) < 1e-12
    _, _, _, ps, ns = orc.run(x, y, th, p, 0, T)
    assert np.array_equal(ps, m["p"]) and np.array_equal(ns, m["nbar"])


def test_full_noise_histograms_follow_closed_forms(orc):
    N, L, T, R = 1024, 32.0, 60, 1.0
    p = orc.Params(N=N, Lx=L, Ly=L, R=R, v=0.5, eta=1.0, seed=6)
    x, y, th = orc.init_state(p)
    bt, bn = 16, 12
    _, _, _, m = orc.run_measured(x, y, th, p, 0, T, bins=(bt, bn))
    # angles: flat (chi^2 over the bins; counts within a state are independent)
    ht = m["hist_theta"]
    chi2 = np.sum((ht - N * T / bt) ** 2 / (N * T / bt))
    assert stats.chi2.sf(chi2, bt - 1) > 1e-4
    # neighbour numbers: Binomial(N-1, pi R^2 / L^2); the n of one state are
    # dependent (pairs are counted twice), so compare the pooled frequencies
    # with a bound from the per-state spread rather than a chi^2 test
    pk = stats.binom.pmf(np.arange(bn), N - 1, math.pi * R * R / (L * L))
    pk[-1] = 1.0 - pk[:-1].sum()
    freq = m["hist_n"] / (N * T)
    assert np.all(np.abs(freq - pk) < 6 * np.sqrt(pk * (1 - pk) * 2 / (N * T)) + 1e-4)
    assert abs(np.dot(np.arange(bn), freq) - (N - 1) * math.pi / (L * L)) < 0.02


def test_split_run_equals_whole_run(orc):
    N, L, K = 700, 20.0, 25
    p = orc.Params(N=N, Lx=L, Ly=L, v=0.5, eta=0.35, seed=12)
    x, y, th = orc.init_state(p)
    xa, ya, ta, ma = orc.run_measured(x, y, th, p, 0, 2 * K, bins=(10, 20))
    x1, y1, t1, m1 = orc.run_measured(x, y, th, p, 0, K, bins=(10, 20))
    x2, y2, t2, m2 = orc.run_measured(x1, y1, t1, p, K, K, bins=(10, 20))
    for u, v in ((xa, x2), (ya, y2), (ta, t2)):
        assert np.array_equal(u, v)
    assert np.array_equal(ma["q"], np.concatenate([m1["q"], m2["q"]]))
    assert np.array_equal(ma["hist_theta"], m1["hist_theta"] + m2["hist_theta"])
    assert np.array_equal(ma["hist_n"], m1["hist_n"] + m2["hist_n"])


"""Pins of the oracle's counter-based generator and of the noise it feeds.

The paper draws uniform numbers from a Mersenne twister and Gaussians by
Box-Muller (Sec. 3.1).  The oracle replaces the twister by Philox4x32-10 so
every (particle, step) draw is addressable.  Bit identity to the published
generator is pinned against rocRAND's engine in test_oracle_philox_rocrand.py;
what the method needs from it -- uniform, independent draws -- and the two
Weyl constants, which follow from closed forms, are pinned here.
"""
import math

import numpy as np
import pytest


def test_weyl_constants_from_closed_forms(orc):
    c = orc.philox_constants()
    # floor((phi - 1) 2^32) with phi = (1 + sqrt 5)/2, in exact integers
    w0 = (math.isqrt(5 << 64) - (1 << 32)) // 2
    # floor((sqrt 3 - 1) 2^32)
    w1 = math.isqrt(3 << 64) - (1 << 32)
    assert int(c[2]) == w0
    assert int(c[3]) == w1


def _numpy_philox(ctr, key, rounds=10):
    """Second, vectorised statement of the Salmon et al. round function,
    used to cross-check the C oracle over many counters."""
    c = [np.asarray(ctr[:, k], dtype=np.uint64) for k in range(4)]
    k0 = np.full(len(ctr), key[0], dtype=np.uint64)
    k1 = np.full(len(ctr), key[1], dtype=np.uint64)
    mask = np.uint64(0xFFFFFFFF)
    for r in range(rounds):
        if r:
            k0 = (k0 + np.uint64(0x9E3779B9)) & mask
            k1 = (k1 + np.uint64(0xBB67AE85)) & mask
        p0 = np.uint64(0xD2511F53) * c[0]
        p1 = np.uint64(0xCD9E8D57) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=1).astype(np.uint32)


def test_two_implementations_agree(orc):
    g = np.random.default_rng(7)
    ctr = g.integers(0, 2 ** 32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    key = g.integers(0, 2 ** 32, size=2, dtype=np.uint64).astype(np.uint32)
    ref = _numpy_philox(ctr, key)
    for k in range(0, 2000, 97):
        out = orc.philox4x32(ctr[k], key)
        assert np.array_equal(out, ref[k])
    # the batch entry uses counter (id, step, replica, purpose), key = seed
    ids = np.arange(1000, dtype=np.uint32)
    seed = 0x123456789ABCDEF
    b = orc.philox_batch(seed, ids, step=42, replica=3, purpose=1)
    ctr2 = np.stack([ids, np.full(1000, 42), np.full(1000, 3), np.full(1000, 1)],
                    axis=1).astype(np.uint32)
    ref2 = _numpy_philox(ctr2, np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32))
    assert np.array_equal(b, ref2)


def test_uniformity_chi2(orc):
    ids = np.arange(1 << 16, dtype=np.uint32)
    w = orc.philox_batch(0, ids, step=5, replica=0, purpose=0).ravel()
    # top byte of each word, 256 bins: chi2 with 255 dof, mean 255, sd ~22.6
    top = (w >> 24).astype(np.int64)
    cnt = np.bincount(top, minlength=256)
    e = len(top) / 256.0
    chi2 = float(((cnt - e) ** 2 / e).sum())
    assert 255 - 6 * 22.6 < chi2 < 255 + 6 * 22.6
    u = (w >> 8).astype(np.float64) * 2.0 ** -24
    assert abs(u.mean() - 0.5) < 6 * math.sqrt(1 / 12 / len(u))
    assert abs(u.var() - 1 / 12) < 0.002


def test_independence_across_counter_words(orc):
    ids = np.arange(1 << 15, dtype=np.uint32)
    a = orc.philox_batch(1, ids, step=0, replica=0, purpose=0)[:, 0]
    b = orc.philox_batch(1, ids, step=1, replica=0, purpose=0)[:, 0]   # next step
    c = orc.philox_batch(1, ids, step=0, replica=0, purpose=1)[:, 0]   # other purpose
    d = orc.philox_batch(2, ids, step=0, replica=0, purpose=0)[:, 0]   # other seed
    ua = a.astype(np.float64) / 2 ** 32
    lim = 6 / math.sqrt(len(ids))
    for other in (b, c, d):
        uo = other.astype(np.float64) / 2 ** 32
        assert abs(np.corrcoef(ua, uo)[0, 1]) < lim
    # adjacent ids
    assert abs(np.corrcoef(ua[:-1], ua[1:])[0, 1]) < lim


def test_avalanche(orc):
    g = np.random.default_rng(3)
    key = np.array([11, 22], dtype=np.uint32)
    flips = []
    for _ in range(300):
        ctr = g.integers(0, 2 ** 32, size=4, dtype=np.uint64).astype(np.uint32)
        bit = int(g.integers(0, 128))
        ctr2 = ctr.copy()
        ctr2[bit // 32] ^= np.uint32(1 << (bit % 32))
        o1, o2 = orc.philox4x32(ctr, key), orc.philox4x32(ctr2, key)
        flips.append(sum(bin(int(v)).count("1") for v in (o1 ^ o2)))
    # 128 output bits, each flipped with probability 1/2: mean 64, sd 5.66
    m = np.mean(flips)
    assert abs(m - 64) < 6 * 5.66 / math.sqrt(300)


def test_uniform_noise_range_and_moments(orc):
    # xi of Eq. (1) is uniform on [-pi, pi]: mean 0, variance pi^2/3
    xs = np.array([orc.noise_vm(9, i, 3) for i in range(20000)])
    assert xs.min() >= -math.pi and xs.max() < math.pi
    assert abs(xs.mean()) < 6 * math.sqrt(math.pi ** 2 / 3 / len(xs))
    assert abs(xs.var() / (math.pi ** 2 / 3) - 1) < 0.05
    # Kolmogorov distance to U[-pi, pi]
    s = np.sort(xs)
    F = (s + math.pi) / (2 * math.pi)
    D = np.max(np.abs(F - (np.arange(1, len(s) + 1) / len(s))))
    assert D < 1.95 / math.sqrt(len(s))


def test_gaussian_noise_moments(orc):
    # Box-Muller output is standard normal (Sec. 3.1)
    gs = np.array([orc.noise_gauss(4, i, 11) for i in range(40000)])
    n = len(gs)
    assert abs(gs.mean()) < 6 / math.sqrt(n)
    assert abs(gs.var() - 1) < 6 * math.sqrt(2 / n)
    kurt = np.mean(gs ** 4) / np.mean(gs ** 2) ** 2
    assert abs(kurt - 3) < 0.15
    from scipy.stats import kstest
    assert kstest(gs, "norm").pvalue > 1e-4


def test_replica_keys_the_noise_and_the_initial_state(orc):
    # an isolated VM particle with eta = 1 and no chirality turns by exactly
    # pi (2u - 1), u = U24 of word 0 of Philox(seed; id, step, replica, 0)
    seed, t, r = 0x5EED, 17, 9
    p = orc.Params(N=1, Lx=10, Ly=10, v=0.0, eta=1.0, seed=seed, replica=r)
    tn = orc.step([5.0], [5.0], [0.0], p, t)[2][0]
    w = _numpy_philox(np.array([[0, t, r, 0]], dtype=np.uint32),
                      np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32))[0]
    u = (int(w[0]) >> 8) * 2.0 ** -24
    assert abs(tn - np.pi * (2 * u - 1)) < 1e-15
    # replicas of one seed start from different states; replica 0 is the default
    a = orc.init_state(orc.Params(N=64, Lx=8, Ly=8, seed=seed))
    b = orc.init_state(orc.Params(N=64, Lx=8, Ly=8, seed=seed, replica=0))
    c = orc.init_state(orc.Params(N=64, Lx=8, Ly=8, seed=seed, replica=1))
    assert all(np.array_equal(u_, v_) for u_, v_ in zip(a, b))
    assert not np.array_equal(a[0], c[0])

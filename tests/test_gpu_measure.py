"""GPU measurement suite (Sec. 3.4) and checkpoint/resume (Sec. 3.6)
through the C ABI.

  * the angle and neighbour-number histograms of one measured state equal
    the oracle's counts exactly (bins decided in binary64 from the binary32
    angle on both sides; n is exact), edge angles included;
  * the nematic order q of that state agrees with the oracle's within the
    fixed-point rounding of its unit vectors;
  * at full size with eta = 1 the angle histogram is flat and the
    neighbour-number histogram follows Binomial(N - 1, pi R^2 / (Lx Ly));
  * a run checkpointed at step K and resumed in a new simulation ends
    bit-identical to the uninterrupted run: state, observables, histograms.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle as orc
from paper_2211_15630_amd import binding as B
from paper_2211_15630_amd import workloads as W

from _parity import oracle_params, sim_for

pytestmark = pytest.mark.gpu


def _counts(h, N, steps):
    c = np.asarray(h) * (N * steps)
    r = np.rint(c)
    assert np.all(np.abs(c - r) < 1e-6)
    return r.astype(np.int64)


def _one_state(cfg, x, y, th, bt, bn, step=3):
    sim = sim_for(cfg, binnum_theta=bt, binnum_neighbors=bn)
    try:
        sim.set_state(x, y, th, step)
        sim.step(1, measure=True)
        ob = sim.observables()
        ht, hn = sim.histograms()
    finally:
        sim.close()
    return ob, ht, hn


@pytest.mark.parametrize("kind,bt,bn", [("uniform", 37, 20), ("uniform", 4096, 4096),
                                        ("clustered", 12, 9), ("edges", 64, 3)])
def test_histograms_and_q_of_one_state(kind, bt, bn):
    cfg = W.workload("vm_small", N=6000, Lx=48.0, Ly=40.0)
    N = cfg["N"]
    if kind == "clustered":
        x, y, th = W.clustered_state(N, 48.0, 40.0, 4)
    else:
        x, y, th = W.uniform_state(N, 48.0, 40.0, 7)
    if kind == "edges":
        # angles on every bin edge in binary32, both ends of [-pi, pi] and
        # the binary32 values just outside it
        k = np.arange(N) % (bt + 1)
        th = (-math.pi + 2 * math.pi * k / bt).astype(np.float32)
        pi32 = np.float32(math.pi)
        th[::7] = pi32
        th[3::7] = -pi32
        th[5::11] = np.nextafter(pi32, np.float32(0))
    ob, ht, hn = _one_state(cfg, x, y, th, bt, bn)
    th64 = th.astype(np.float64)
    n, *_ = orc.neighbours_cells(x, y, th, oracle_params(cfg))
    ot, on = orc.histograms(th64, n, bt, bn)
    assert np.array_equal(_counts(ht, N, 1), ot)
    assert np.array_equal(_counts(hn, N, 1), on)
    p0, nbar0, q0 = orc.state_observables(th64, n)
    # each cos 2 th, sin 2 th is within ~2^-21 of the exact value (binary32
    # sincos of the angle, 2^-27 fixed point, one binary64 square)
    assert ob["steps_measured"] == 1
    assert abs(ob["q_last"] - q0) < 2e-6
    assert abs(ob["q_mom"][0] - ob["q_last"]) < 1e-15
    assert abs(ob["q_mom"][1] - ob["q_last"] ** 2) < 1e-12
    assert abs(ob["p_last"] - p0) < 2e-6 and abs(ob["nbar_last"] - nbar0) < 1e-12


def test_q_of_a_nematic_state():
    cfg = W.workload("vm_small")
    x, y, _ = W.uniform_state(4096, 64.0, 64.0, 3)
    th = np.where(np.arange(4096) % 2 == 0, 0.6, 0.6 - math.pi).astype(np.float32)
    ob, _, _ = _one_state(cfg, x, y, th, 8, 4)
    assert ob["p_last"] < 1e-6 and abs(ob["q_last"] - 1.0) < 1e-6


def test_histograms_over_many_steps_are_consistent():
    cfg = W.workload("vm_small", eta=0.25, seed=2)
    # n <= N - 1 = bn - 1: no count saturates
    N, T, bn = cfg["N"], 300, 4096
    sim = sim_for(cfg, binnum_theta=30, binnum_neighbors=bn)
    try:
        sim.step(T, measure=True)
        ob = sim.observables()
        ht, hn = sim.histograms()
        sim.reset_observables()
        ht0, hn0 = sim.histograms()
    finally:
        sim.close()
    ct, cn = _counts(ht, N, T), _counts(hn, N, T)
    assert ct.sum() == N * T and cn.sum() == N * T
    assert abs(np.dot(np.arange(bn), cn) / (N * T) - ob["nbar_mom"][0]) < 1e-9
    assert not ht0.any() and not hn0.any()


def test_full_noise_histograms_full_size():
    cfg = W.workload("vm_large", eta=1.0, seed=4)
    N, T, bt, bn = cfg["N"], 10, 64, 16
    sim = sim_for(cfg, binnum_theta=bt, binnum_neighbors=bn)
    try:
        sim.step(T, measure=True)
        ht, hn = sim.histograms()
    finally:
        sim.close()
    ct = _counts(ht, N, T)
    chi2 = np.sum((ct - N * T / bt) ** 2 / (N * T / bt))
    assert stats.chi2.sf(chi2, bt - 1) > 1e-4
    pk = stats.binom.pmf(np.arange(bn), N - 1, math.pi / (cfg["Lx"] * cfg["Ly"]))
    pk[-1] = 1.0 - pk[:-1].sum()
    freq = _counts(hn, N, T) / (N * T)
    assert np.all(np.abs(freq - pk) < 6 * np.sqrt(pk * (1 - pk) * 2 / (N * T)) + 1e-6)


def _run_and_collect(sim, K):
    sim.step(K, measure=True)
    x, y, th, st = sim.get_state()
    ob = sim.observables()
    h = sim.histograms() if sim.params.bins_theta else (None, None)
    return (x, y, th, st), ob, h


@pytest.mark.parametrize("name,over", [
    ("vm_small", dict(eta=0.3, seed=9)),
    ("langevin_walls", dict(N=16384, Lx=64.0, Ly=64.0, D=0.05)),
])
def test_checkpoint_resume_bit_identical(name, over, tmp_path):
    cfg = W.workload(name, **over)
    K = 150
    a = sim_for(cfg, binnum_theta=50, binnum_neighbors=40)
    b = sim_for(cfg, binnum_theta=50, binnum_neighbors=40)
    try:
        a.step(K, measure=True)
        data = a.checkpoint()
        path = str(tmp_path / "sim.ckpt")
        a.save(path)
        sa, oa, ha = _run_and_collect(a, K)
        b.step(7)                    # whatever b held before is replaced
        b.load(path)
        sb, ob, hb = _run_and_collect(b, K)
        b.restore(data)
        sc, oc, hc = _run_and_collect(b, K)
    finally:
        a.close()
        b.close()
    assert sa[3] == sb[3] == sc[3] == 2 * K
    for other, oo, hh in ((sb, ob, hb), (sc, oc, hc)):
        for u, v in zip(sa[:3], other[:3]):
            assert np.array_equal(u, v)
        assert oa == oo
        assert np.array_equal(ha[0], hh[0]) and np.array_equal(ha[1], hh[1])
    assert oa["steps_measured"] == 2 * K


def test_checkpoint_rejects_other_simulations():
    cfg = W.workload("vm_small")
    a = sim_for(cfg, binnum_theta=10, binnum_neighbors=10)
    b = sim_for(cfg, eta=0.31, binnum_theta=10, binnum_neighbors=10)
    c = sim_for(cfg)
    try:
        a.step(3)
        data = a.checkpoint()
        for other in (b, c):
            with pytest.raises(B.AapError) as e:
                other.restore(data)
            assert e.value.code == B.AAP_EINVAL
        bad = bytearray(data)
        bad[0] ^= 1
        with pytest.raises(B.AapError):
            a.restore(bytes(bad))
        with pytest.raises(B.AapError):
            a.restore(data[:-8])
        # a refused load leaves the simulation as it was
        before = a.get_state()
        a.restore(data)
        after = a.get_state()
        assert all(np.array_equal(u, v) for u, v in zip(before[:3], after[:3]))
    finally:
        a.close()
        b.close()
        c.close()


_CHILD = r"""
import os, signal, sys
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, os.path.join(sys.argv[1], "tests"))
from paper_2211_15630_amd import workloads as W
from _parity import sim_for
sim = sim_for(W.workload("vm_small", eta=0.35, seed=21), binnum_theta=16, binnum_neighbors=16)
sim.step(int(sys.argv[3]), measure=True)
sim.save(sys.argv[2])
sim.sync()
print("saved", flush=True)
os.kill(os.getpid(), signal.SIGKILL)   # the process dies without closing anything
"""


def test_killed_process_resumes_from_its_checkpoint(tmp_path):
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = str(tmp_path / "killed.ckpt")
    K = 120
    r = subprocess.run([sys.executable, "-c", _CHILD, root, path, str(K)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == -9 and "saved" in r.stdout, (r.returncode, r.stderr[-2000:])
    cfg = W.workload("vm_small", eta=0.35, seed=21)
    a = sim_for(cfg, binnum_theta=16, binnum_neighbors=16)
    b = sim_for(cfg, binnum_theta=16, binnum_neighbors=16)
    try:
        a.step(K, measure=True)
        sa, oa, ha = _run_and_collect(a, K)
        b.load(path)
        sb, ob, hb = _run_and_collect(b, K)
    finally:
        a.close()
        b.close()
    for u, v in zip(sa, sb):
        assert np.array_equal(u, v)
    assert oa == ob
    assert np.array_equal(ha[0], hb[0]) and np.array_equal(ha[1], hb[1])

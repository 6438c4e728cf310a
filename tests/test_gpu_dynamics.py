"""GPU multi-step behaviour through the C ABI: determinism, the measured
observables, closed forms that hold at any size, and statistical parity
with the oracle's long runs (16 seeds, stored by
tests/golden/make_oracle_stats.py)."""
import json
import math
import os

import numpy as np
import pytest

import oracle as orc
from paper_2211_15630_amd import binding as B
from paper_2211_15630_amd import workloads as W

from _parity import oracle_params, sim_for

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_stats.json")


def test_run_twice_bit_identical():
    cfg = W.workload("vm_small", eta=0.2, seed=5)
    outs = []
    for _ in range(2):
        sim = sim_for(cfg)
        try:
            ps = sim.step(300, series=True)
            x, y, th, st = sim.get_state()
            ob = sim.observables()
        finally:
            sim.close()
        outs.append((ps, x, y, th, ob))
    a, b = outs
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)
    assert a[4] == b[4]


def test_langevin_walls_run_twice_bit_identical():
    cfg = W.workload("langevin_walls", N=16384, Lx=64.0, Ly=64.0, D=0.05)
    res = []
    for _ in range(2):
        sim = sim_for(cfg)
        try:
            ps = sim.step(100, series=True)
            res.append((ps,) + sim.get_state()[:3])
        finally:
            sim.close()
    for u, v in zip(res[0], res[1]):
        assert np.array_equal(u, v)


def test_measured_state_zero_is_the_given_state():
    cfg = W.workload("vm_small")
    x, y, th = W.uniform_state(4096, 64.0, 64.0, 2)
    sim = sim_for(cfg)
    try:
        sim.set_state(x, y, th, 0)
        ps0 = sim.step(1, series=True)
        ob0 = sim.observables()
        ps = np.concatenate([ps0, sim.step(2, series=True)])
        ob = sim.observables()
    finally:
        sim.close()
    p0 = abs(np.mean(np.exp(1j * th.astype(np.float64))))
    assert abs(ps[0] - p0) < 1e-6
    # nbar of state 0: the exact integer sum of the oracle's n over N
    n, *_ = orc.neighbours_cells(x, y, th, oracle_params(cfg))
    assert ob0["steps_measured"] == 1
    assert ob0["nbar_mom"][0] == np.sum(n) / len(n)
    assert ob["steps_measured"] == 3
    assert abs(ob["p_mom"][0] - ps.mean()) < 1e-12
    # oracle steps from the same state: p of states 1 and 2 agree closely
    _, _, _, po, no = orc.run(x, y, th, oracle_params(cfg), 0, 3)
    assert np.allclose(ps, po, atol=1e-5)


def test_mean_neighbour_number_uniform_full_size():
    # E[nbar] = (N-1) pi R^2 / (Lx Ly) for uniform positions (Eq. (6)); the
    # initial state is uniform, and with eta = 1 positions stay uniform
    cfg = W.workload("vm_large", eta=1.0, seed=3)
    sim = sim_for(cfg)
    try:
        sim.step(20, measure=True)
        ob = sim.observables()
    finally:
        sim.close()
    N = cfg["N"]
    expect = (N - 1) * math.pi / (cfg["Lx"] * cfg["Ly"])
    # sd of nbar for one configuration ~ sqrt(2 E / N); 20 states
    assert abs(ob["nbar_mom"][0] - expect) < 5 * math.sqrt(2 * expect / N / 20) + 1e-9


def test_full_noise_polarisation_moments():
    # eta = 1: new angles i.i.d. uniform -> <p^2> = 1/N, <p^4> = (2N-1)/N^3
    N, L, T = 64, 12.0, 20000
    cfg = W.workload("vm_small", N=N, Lx=L, Ly=L, eta=1.0, seed=8)
    sim = sim_for(cfg)
    try:
        ps = sim.step(T, series=True)[1:]
    finally:
        sim.close()
    m2, m4 = np.mean(ps ** 2), np.mean(ps ** 4)
    assert abs(m2 - 1 / N) < 5 * np.std(ps ** 2) / math.sqrt(len(ps))
    assert abs(m4 - (2 * N - 1) / N ** 3) < 5 * np.std(ps ** 4) / math.sqrt(len(ps))


def test_aligned_without_noise_stays_polar():
    cfg = W.workload("vm_small", eta=0.0)
    x, y, th = W.aligned_state(4096, 64.0, 64.0, 1, angle=0.4)
    sim = sim_for(cfg)
    try:
        sim.set_state(x, y, th, 0)
        ps = sim.step(500, series=True)
    finally:
        sim.close()
    assert np.all(np.abs(ps - 1.0) < 1e-6)


def test_nvm_walls_run_twice_bit_identical():
    cfg = W.workload("nvm_small", bx=1, by=0, omega=0.1)
    res = []
    for _ in range(2):
        sim = sim_for(cfg)
        try:
            ps = sim.step(200, series=True)
            res.append((ps,) + sim.get_state()[:3])
        finally:
            sim.close()
    for u, v in zip(res[0], res[1]):
        assert np.array_equal(u, v)


def test_nvm_full_noise_polarisation_moments():
    # eta = 1: new angles i.i.d. uniform whatever the rule
    N, L, T = 64, 12.0, 20000
    cfg = W.workload("nvm_small", N=N, Lx=L, Ly=L, eta=1.0, seed=8)
    sim = sim_for(cfg)
    try:
        ps = sim.step(T, series=True)[1:]
    finally:
        sim.close()
    m2, m4 = np.mean(ps ** 2), np.mean(ps ** 4)
    assert abs(m2 - 1 / N) < 5 * np.std(ps ** 2) / math.sqrt(len(ps))
    assert abs(m4 - (2 * N - 1) / N ** 3) < 5 * np.std(ps ** 4) / math.sqrt(len(ps))


def test_antiparallel_state_stays_nematic_under_nvm_only():
    # Eq. (3) aligns antiparallel neighbours without turning them: from a
    # state split between a and a + pi the NVM keeps q high and p near 0,
    # while the VM turns it polar
    x, y, _ = W.uniform_state(8192, 64.0, 64.0, 3)
    th = np.where(np.arange(8192) % 2 == 0, 0.6, 0.6 - math.pi).astype(np.float32)
    out = {}
    for rule in (W.RULE_NVM, W.RULE_VM):
        sim = sim_for(W.workload("nvm_small", rule=rule))
        try:
            sim.set_state(x, y, th, 0)
            sim.step(299)
            sim.step(1, measure=True)
            ob = sim.observables()
        finally:
            sim.close()
        out[rule] = (ob["p_last"], ob["q_last"])
    assert out[W.RULE_NVM][1] > 0.9 and out[W.RULE_NVM][0] < 0.05
    assert out[W.RULE_VM][0] > 0.9


def test_reflecting_containment_langevin():
    cfg = W.workload("langevin_walls", N=1 << 18, Lx=256.0, Ly=256.0, D=0.2, v=4.0)
    sim = sim_for(cfg)
    try:
        for _ in range(4):
            sim.step(50)
            x, y, th, _ = sim.get_state()
            assert np.all((x >= 0) & (x <= 256.0) & (y >= 0) & (y <= 256.0))
            assert np.all(np.abs(th) <= np.float32(math.pi))
    finally:
        sim.close()


def test_every_id_present_after_many_steps():
    cfg = W.workload("vm_small", eta=0.1)
    sim = sim_for(cfg)
    try:
        sim.step(2000)
        sim.debug_enable(True)
        sim.step(1)
        d = sim.debug_last_step()
    finally:
        sim.close()
    assert np.array_equal(np.sort(d["order"]), np.arange(4096, dtype=np.uint32))
    assert d["start"][-1] == 4096 and np.all(np.diff(d["start"].astype(np.int64)) >= 0)


def test_timing_samples_every_kth_step():
    cfg = W.workload("vm_small", eta=0.3)
    sim = sim_for(cfg)
    try:
        with pytest.raises(B.AapError):
            sim.timing_enable(-1)
        sim.timing_enable(4)
        sim.step(9)
        t = sim.timing_read()
        sim.timing_enable(0)
        sim.step(3)
        assert all(v[1] == 0 for v in sim.timing_read().values())
    finally:
        sim.close()
    # steps 0, 4, 8 of the nine carry events: step 0 (fresh state) sorts with
    # k_scan + k_scatter, steps 4 and 8 with k_sort; k_nbr runs every step
    launches = {k: v[1] for k, v in t.items()}
    assert launches == {"k_scan": 1, "k_scatter": 1, "k_sort": 2, "k_nbr": 3}, launches
    for name, (ms, n) in t.items():
        assert 0.0 < ms < 50.0, (name, ms)


def _z(a, b):
    a, b = np.asarray(a), np.asarray(b)
    se = math.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b))
    return abs(a.mean() - b.mean()) / se if se > 0 else 0.0


def _binder_jackknife(p2, p4):
    p2, p4 = np.asarray(p2), np.asarray(p4)
    U = 1 - p4.mean() / (3 * p2.mean() ** 2)
    n = len(p2)
    loo = np.array([1 - np.delete(p4, k).mean() / (3 * np.delete(p2, k).mean() ** 2)
                    for k in range(n)])
    se = math.sqrt((n - 1) / n * np.sum((loo - loo.mean()) ** 2))
    return U, se


@pytest.mark.parametrize("name", ["vm_eta0.2", "vm_eta0.4", "vm_eta0.6",
                                  "langevin_D0.05", "langevin_D0.2",
                                  "nvm_eta0.1", "nvm_eta0.3", "langevin_o2_D0.05",
                                  "vm65536_eta0.2", "vm65536_eta0.4", "vm65536_eta0.6"])
def test_statistical_parity_16_seeds(name):
    gold = json.load(open(GOLDEN))
    pt = next(q for q in gold["points"] if q["params"]["name"] == name)
    P = pt["params"]
    w = W.inverse_n_weights(4096) if P["weights"] == "inverse_n_4096" else None
    rows = []
    for s in range(16):
        sim = B.Sim(N=P["N"], Lx=P["Lx"], Ly=P["Ly"], R=P["R"], v=P["v"], eta=P["eta"],
                    rule=P["rule"], order=P.get("order", 1), bx=P["bx"], by=P["by"],
                    gamma=P["gamma"], dt=P["dt"], seed=s, weights=w)
        try:
            sim.step(P["discard"])
            ps = sim.step(P["steps"] - P["discard"], series=True)
            ob = sim.observables()
        finally:
            sim.close()
        q = ob["q_mom"]
        rows.append((ps.mean(), np.mean(ps ** 2), np.mean(ps ** 4), ob["nbar_mom"][0],
                     q[0], q[1], q[3]))
    g = np.array(rows)
    o = np.array([[r["p1"], r["p2"], r["p4"], r["nbar"]] for r in pt["seeds"]])
    zp = _z(g[:, 0], o[:, 0])
    Ug, seg = _binder_jackknife(g[:, 1], g[:, 2])
    Uo, seo = _binder_jackknife(o[:, 1], o[:, 2])
    zU = abs(Ug - Uo) / math.sqrt(seg ** 2 + seo ** 2) if seg + seo > 0 else 0.0
    zn = _z(g[:, 3], o[:, 3])
    print(name, "p", g[:, 0].mean(), o[:, 0].mean(), "z", zp, "U", Ug, Uo, "z", zU, "nbar z", zn)
    assert zp <= 3.0
    assert zU <= 3.0
    assert zn <= 3.0
    if P.get("q"):
        oq = np.array([[r["q1"], r["q2"], r["q4"]] for r in pt["seeds"]])
        zq = _z(g[:, 4], oq[:, 0])
        Vg, sg = _binder_jackknife(g[:, 5], g[:, 6])
        Vo, so = _binder_jackknife(oq[:, 1], oq[:, 2])
        zV = abs(Vg - Vo) / math.sqrt(sg ** 2 + so ** 2) if sg + so > 0 else 0.0
        print(name, "q", g[:, 4].mean(), oq[:, 0].mean(), "z", zq, "U(q)", Vg, Vo, "z", zV)
        assert zq <= 3.0
        assert zV <= 3.0


def test_full_size_statistics_16_seeds():
    """The standard Vicsek model at full size (N = 2^20, L = 1024, density 1)
    over 16 seeds, 10^4 steps each, the first 2000 discarded, for the noise
    sweep eta = 0.2, 0.4, 0.6.  The oracle cannot run these (1.6e11 particle
    updates per point), so the statistics are checked against what holds at
    any size: <p> falls with the noise; the low-noise runs order (<p> far
    above the 1/sqrt(N) of independent angles, and a Binder cumulant above
    the disordered one); the high-noise runs are disordered (U within 3
    standard errors of the Gaussian value 1/3, <p> of order 1/sqrt(N)); and
    the mean neighbour number lies above its uniform-state value
    (N-1) pi R^2 / L^2 and rises with order (clustering)."""
    N, L = 1 << 20, 1024.0
    res = {}
    for eta in (0.2, 0.4, 0.6):
        rows = []
        for s in range(16):
            sim = B.Sim(N=N, Lx=L, Ly=L, R=1.0, v=0.5, eta=eta, seed=s)
            try:
                sim.step(2000)
                ps = sim.step(8000, series=True)
                ob = sim.observables()
            finally:
                sim.close()
            rows.append((ps.mean(), np.mean(ps ** 2), np.mean(ps ** 4), ob["nbar_mom"][0]))
        g = np.array(rows)
        U, se = _binder_jackknife(g[:, 1], g[:, 2])
        res[eta] = dict(p=g[:, 0].mean(), p_se=g[:, 0].std(ddof=1) / 4.0, U=U, U_se=se,
                        nbar=g[:, 3].mean())
        print("N=2^20 eta", eta, res[eta], flush=True)
    assert res[0.2]["p"] > res[0.4]["p"] > res[0.6]["p"]
    assert res[0.2]["p"] > 100.0 / math.sqrt(N) and res[0.2]["U"] > res[0.6]["U"]
    assert abs(res[0.6]["U"] - 1.0 / 3.0) <= 3.0 * res[0.6]["U_se"] + 1e-3
    assert res[0.6]["p"] < 10.0 / math.sqrt(N)
    nbar0 = (N - 1) * math.pi / (L * L)
    assert nbar0 < res[0.6]["nbar"] < res[0.2]["nbar"]

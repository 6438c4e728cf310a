"""Batches of replicas through the C ABI (one launch per kernel and step
for every replica; optional captured graphs).

  * replica r of a batch evolves bit for bit as a single system with the
    same parameters and replica index: state, step and measured moments,
    for VM, NVM with walls and Langevin of order 2;
  * graph replays give the eager results, with eager steps and measurement
    changes between replays, several replays in a row;
  * the replica index is word 2 of the noise counter: one-step parity of a
    single system of replica 5 with the oracle's replica 5;
  * the 256-replica noise sweep at full size: sampled replicas equal their
    single-system runs; measured order falls with the noise;
  * one batched step (batched sort + batched neighbour kernel) against the
    oracle, replica by replica: next cells, cell starts and the (cell, id)
    order exact, n exact, C and S within the fixed-point bound, theta', x',
    y' within the one-step tolerances -- for replicas of uneven N and
    densities 0.25 .. 4, the VM, the NVM with walls and chirality, and the
    Langevin rule of order 1 (walls) and 2; and on sampled replicas of the
    full 256-replica sweep.
"""
import numpy as np
import pytest

from paper_2211_15630_amd import binding as B
from paper_2211_15630_amd import workloads as W

import oracle as orc

from _parity import (compare_cells, compare_sums, compare_update, one_step_parity,
                     oracle_params, sim_for)

pytestmark = pytest.mark.gpu


def _small_batch(rule=W.RULE_VM, **over):
    sizes = [(1024, 0.5), (3000, 1.0), (4096, 2.0), (777, 4.0), (2048, 1.5)]
    out = []
    for r, (n, rho) in enumerate(sizes):
        L = float(np.sqrt(n / rho))
        cfg = W.workload("vm_small", N=n, Lx=L, Ly=L, eta=0.15 + 0.1 * r, seed=7, replica=r,
                         rule=rule)
        cfg.update(over)
        out.append(W.model_params(cfg))
    return out


def _single(kw, steps, measure_plan):
    sim = B.Sim(**kw)
    try:
        for n, m in measure_plan:
            sim.step(n, measure=m)
        return sim.get_state(), sim.observables()
    finally:
        sim.close()


def _batch(reps, measure_plan, graph_steps=0):
    b = B.Batch(reps, graph_steps=graph_steps)
    try:
        for n, m in measure_plan:
            b.step(n, measure=m)
        b.sync()
        return [b.get_state(r) for r in range(b.count)], b.observables()
    finally:
        b.close()


PLAN = [(1, True), (20, True), (7, False), (16, True)]


@pytest.mark.parametrize("rule,over", [
    (W.RULE_VM, dict()),
    (W.RULE_NVM, dict(bx=1, by=1, omega=0.1)),
    (W.RULE_LANGEVIN, dict(order=2, dt=0.1, weights=W.inverse_n_weights(64))),
])
def test_batch_equals_single_systems(rule, over):
    reps = _small_batch(rule, **over)
    states, obs = _batch(reps, PLAN)
    for r, kw in enumerate(reps):
        st, ob = _single(kw, 0, PLAN)
        for u, v in zip(states[r][:3], st[:3]):
            assert np.array_equal(u, v), f"replica {r}"
        assert states[r][3] == st[3] == sum(n for n, _ in PLAN)
        assert obs[r] == ob, f"replica {r}"


def test_batch_graph_equals_eager():
    reps = _small_batch()
    plan = [(1, True), (9, True), (16, True), (3, False), (12, False), (1, True), (24, True)]
    s0, o0 = _batch(reps, plan, graph_steps=0)
    s1, o1 = _batch(reps, plan, graph_steps=4)
    for r in range(len(reps)):
        for u, v in zip(s0[r], s1[r]):
            assert np.array_equal(u, v)
        assert o0[r] == o1[r]


def test_replicas_are_independent_streams():
    reps = _small_batch()
    same = [dict(kw, replica=0) for kw in reps[:2]]
    a = _single(reps[1], 0, [(5, False)])[0]
    b = _single(same[1], 0, [(5, False)])[0]
    assert not np.array_equal(a[2], b[2])


def test_replica_one_step_parity_with_oracle():
    cfg = W.workload("vm_small", replica=5, eta=0.6)
    one_step_parity(cfg, W.uniform_state(4096, 64.0, 64.0, 12))


def test_batch_256_noise_sweep_full_size():
    cfgs = W.batch_replicas()
    reps = [W.model_params(c) for c in cfgs]
    plan = [(1, True), (120, True)]
    b = B.Batch(reps, graph_steps=8)
    try:
        for n, m in plan:
            b.step(n, measure=m)
        b.sync()
        obs = b.observables()
        sampled = {r: b.get_state(r) for r in (0, 97, 255)}
    finally:
        b.close()
    for r, st in sampled.items():
        st1, ob1 = _single(reps[r], 0, plan)
        for u, v in zip(st[:3], st1[:3]):
            assert np.array_equal(u, v), f"replica {r}"
        assert obs[r] == ob1
    p = np.array([o["p_mom"][0] for o in obs])
    assert np.all(np.isfinite(p)) and all(o["steps_measured"] == 121 for o in obs)
    # low-noise replicas order faster than high-noise ones (same mix of sizes)
    assert p[:64].mean() > p[-64:].mean()


def test_workgroup_sizes_and_autotune_do_not_change_results():
    reps = _small_batch(W.RULE_VM)
    ref_states, ref_obs = _batch(reps, [(1, True), (48, True), (10, True)])
    for threads in (64, 128):
        b = B.Batch(reps)
        try:
            b.threads(threads)
            b.step(1, True)
            b.step(58, True)
            b.sync()
            for r in range(b.count):
                for u, v in zip(b.get_state(r), ref_states[r]):
                    assert np.array_equal(u, v)
            assert b.observables() == ref_obs
        finally:
            b.close()
    b = B.Batch(reps)
    try:
        # 1 first step + 3 sizes x 2 graph settings x 2 trials x 4 steps = 49
        threads, graph = b.autotune(4, True)
        assert threads in (64, 128, 256) and graph in (0, 4)
        sort_ms, nbr_ms = b.kernel_times(4, True)
        assert 0.0 < sort_ms < 10.0 and 0.0 < nbr_ms < 10.0
        b.step(6, True)
        b.sync()
        for r in range(b.count):
            for u, v in zip(b.get_state(r), ref_states[r]):
                assert np.array_equal(u, v)
        assert b.observables() == ref_obs
    finally:
        b.close()


def _uneven_batch(rule, **over):
    """Replica configurations of uneven size and density 0.25 .. 4 (Eq. (6)
    neighbourhoods from sparse to dense), with per-replica noise."""
    sizes = [(1500, 0.25), (5000, 0.5), (2048, 1.0), (4096, 2.0), (3000, 4.0), (777, 3.0)]
    cfgs = []
    for r, (n, rho) in enumerate(sizes):
        L = float(np.sqrt(n / rho))
        cfg = W.workload("vm_small", N=n, Lx=L, Ly=L, eta=0.1 + 0.1 * r, seed=11, replica=r,
                         rule=rule)
        cfg.update(over)
        cfgs.append(cfg)
    return cfgs


def _batched_step_parity(cfgs, replicas, warm=12):
    """warm steps (the first sorts each initial state, the others run the
    batched kernels), then one batched step with debug output, compared
    replica by replica with the oracle from the state it read."""
    b = B.Batch([W.model_params(c) for c in cfgs])
    try:
        b.step(warm, measure=True)
        b.sync()
        before = {r: b.get_state(r) for r in replicas}
        keys = {r: b.debug_keys(r) for r in replicas}
        b.debug_enable(True)
        b.step(1, measure=True)
        b.sync()
        after = {r: b.get_state(r) for r in replicas}
        dbg = {r: b.debug_last_step(r) for r in replicas}
    finally:
        b.close()
    reps = {}
    for r in replicas:
        cfg = cfgs[r]
        x1, y1, t1, st = before[r]
        assert st == warm
        p = oracle_params(cfg)
        # the next cells the last batched neighbour kernel wrote
        assert np.array_equal(keys[r], orc.cell_keys(x1, y1, p.Lx, p.Ly, p.R)), f"replica {r}"
        # the batched sort of that state, then the batched neighbour sums
        compare_cells(None, x1, y1, t1, cfg, dbg[r])
        n, C, S, A = compare_sums(cfg, x1, y1, t1, dbg[r])
        xg, yg, tg, st2 = after[r]
        assert st2 == warm + 1
        reps[r] = compare_update(cfg, x1, y1, t1, n, C, S, A, xg, yg, tg, st)
    return reps


@pytest.mark.parametrize("rule,over", [
    (W.RULE_VM, dict()),
    (W.RULE_NVM, dict(bx=1, by=1, omega=0.1)),
    (W.RULE_LANGEVIN, dict(order=1, dt=0.1, bx=1, by=1, weights=W.inverse_n_weights(64))),
    (W.RULE_LANGEVIN, dict(order=2, dt=0.1, weights=W.inverse_n_weights(64))),
])
def test_batched_step_against_oracle(rule, over):
    cfgs = _uneven_batch(rule, **over)
    reps = _batched_step_parity(cfgs, range(len(cfgs)))
    print(rule, reps)


def test_batch_256_full_size_sampled_against_oracle():
    cfgs = W.batch_replicas()
    Ns = np.array([c["N"] for c in cfgs])
    rho = np.array([c["density"] for c in cfgs])
    pick = sorted({int(np.argmin(Ns)), int(np.argmax(Ns)), int(np.argmin(rho)),
                   int(np.argmax(rho)), 0, 128, 255})
    reps = _batched_step_parity(cfgs, pick, warm=40)
    print(reps)

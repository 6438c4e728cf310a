"""Steps replayed from captured HIP graphs (aap_graph) against the same
steps launched one by one, through the C ABI: after every call (each a run
of several graph replays with the program's own launches and
synchronisations between them) the positions, angles, observables and
histograms are bit-identical -- the replayed kernels read the step number
the noise is keyed by from device memory, and the sums are exact."""
import numpy as np
import pytest

from paper_2211_15630_amd import workloads as W

from _parity import sim_for

pytestmark = pytest.mark.gpu

# (steps, measure, series) per call: unmeasured and measured runs longer
# than several graphs, a series call (launched one by one), odd lengths
CALLS = [(37, False, False), (53, True, False), (20, True, True), (3, True, False),
         (33, False, False), (40, True, False)]


def _run(cfg, graph, over, state=None):
    sim = sim_for(cfg, **over)
    out = []
    try:
        if graph:
            sim.graph(graph)
        if state is not None:
            sim.set_state(*state)
        for n, meas, series in CALLS:
            if series:
                ps = sim.step(n, series=True)
            else:
                ps = None
                sim.step(n, measure=meas)
            x, y, th, st = sim.get_state()
            out.append((x, y, th, st, ps, sim.observables(),
                        sim.histograms() if over.get("binnum_theta") else None))
    finally:
        sim.close()
    return out


def _same(a, b):
    for ra, rb in zip(a, b):
        for u, v in zip(ra[:4], rb[:4]):
            assert np.array_equal(u, v)
        if ra[4] is not None:
            assert np.array_equal(ra[4], rb[4])
        assert ra[5] == rb[5]
        if ra[6] is not None:
            for u, v in zip(ra[6], rb[6]):
                assert np.array_equal(u, v)


@pytest.mark.parametrize("name,cfg_over,over,graph", [
    ("vm_small", dict(eta=0.3, seed=3), dict(), 16),
    ("vm_small", dict(eta=0.3, seed=3), dict(binnum_theta=32, binnum_neighbors=16), 8),
    ("vm_small", dict(eta=0.2, seed=4, bx=1, by=1), dict(), 2),
    ("langevin_walls", dict(N=16384, Lx=64.0, Ly=64.0, D=0.05), dict(), 16),
    ("nvm_large", dict(N=8192, Lx=64.0, Ly=64.0), dict(), 16),
    # 1500^2 cells in 1099 sort tiles: the tile offsets come from their own
    # scan kernel, captured with the rest
    ("vm_small", dict(N=65536, Lx=1500.0, Ly=1500.0, eta=0.4, seed=2), dict(), 8),
])
def test_graph_replays_equal_direct_steps(name, cfg_over, over, graph):
    cfg = W.workload(name, **cfg_over)
    _same(_run(cfg, 0, over), _run(cfg, graph, over))


def test_graph_after_a_set_state_and_a_changed_length():
    cfg = W.workload("vm_small", eta=0.25, seed=6)
    state = W.clustered_state(cfg["N"], cfg["Lx"], cfg["Ly"], 6)
    direct = _run(cfg, 0, {}, state=state)
    sim = sim_for(cfg)
    got = []
    try:
        sim.graph(16)
        sim.set_state(*state)
        for k, (n, meas, series) in enumerate(CALLS):
            if k == 2:
                sim.graph(4)
            if k == 4:
                sim.graph(0)
            if k == 5:
                sim.graph(32)
            ps = sim.step(n, series=True) if series else sim.step(n, measure=meas)
            x, y, th, st = sim.get_state()
            got.append((x, y, th, st, ps, sim.observables(), None))
    finally:
        sim.close()
    _same(direct, got)

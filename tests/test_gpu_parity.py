"""GPU parity through the C ABI against the oracle, one step from identical
binary32 states: cell ids, cell starts, the (cell, id) order and neighbour
counts bit-exact; neighbour sums, angles and positions within the derived
tolerances.  Workloads at full size (N = 4096, 2^20 and 4*2^20) and
structures: uniform, travelling bands, dense clusters, adversarial edges."""
import math

import numpy as np
import pytest

import oracle as orc
from paper_2211_15630_amd import workloads as W

from _parity import cs_tolerance, one_step_parity, oracle_params, second_step_parity, sim_for

pytestmark = pytest.mark.gpu


def _state(kind, cfg, seed):
    N, Lx, Ly, bx, by = cfg["N"], cfg["Lx"], cfg["Ly"], cfg["bx"], cfg["by"]
    if kind == "uniform":
        return W.uniform_state(N, Lx, Ly, seed, bx, by)
    if kind == "banded":
        return W.banded_state(N, Lx, Ly, seed, bx, by)
    if kind == "clustered":
        # ~250 extra particles per cluster of radius ~2: a few times the mean
        # density, like the dense regions of band states
        return W.clustered_state(N, Lx, Ly, seed, bx, by, clusters=max(16, N // 256),
                                 sigma=2.0, frac=0.3)
    if kind == "edge":
        M = orc.cells_per_axis(Lx, cfg["R"])
        return W.edge_state(N, Lx, Ly, seed, Lx / M, Ly / M, cfg["R"], bx, by)
    raise KeyError(kind)


@pytest.mark.parametrize("kind", ["uniform", "banded", "clustered", "edge"])
def test_vm_small_one_step(kind):
    cfg = W.workload("vm_small")
    rep, _ = one_step_parity(cfg, _state(kind, cfg, 11))
    print(kind, rep)


@pytest.mark.parametrize("bx,by", [(1, 1), (0, 1), (1, 0)])
@pytest.mark.parametrize("kind", ["uniform", "edge"])
def test_vm_small_walls_one_step(kind, bx, by):
    cfg = W.workload("vm_small", bx=bx, by=by)
    one_step_parity(cfg, _state(kind, cfg, 3))


@pytest.mark.parametrize("kind", ["uniform", "clustered", "edge"])
def test_langevin_small_one_step(kind):
    cfg = W.workload("langevin_walls", N=16384, Lx=64.0, Ly=64.0)
    one_step_parity(cfg, _state(kind, cfg, 5))


def test_langevin_periodic_additive_one_step():
    cfg = W.workload("langevin_walls", N=8192, Lx=48.0, Ly=40.0, bx=0, by=0,
                     weights=None, omega=0.3)
    one_step_parity(cfg, _state("uniform", cfg, 8))


@pytest.mark.parametrize("kind", ["uniform", "banded"])
def test_vm_large_one_step(kind):
    cfg = W.workload("vm_large", eta=0.4)
    rep, _ = one_step_parity(cfg, _state(kind, cfg, 2))
    print(kind, rep)


@pytest.mark.parametrize("D", [0.05, 0.2])
def test_langevin_walls_full_one_step(D):
    cfg = W.workload("langevin_walls", D=D)
    rep, _ = one_step_parity(cfg, _state("uniform", cfg, 4))
    print(D, rep)


def test_full_size_sampled_brute_force():
    # at full size, sampled particles against the plain definition (all N
    # particles and all images, one by one)
    cfg = W.workload("langevin_walls", D=0.2)
    x, y, th = _state("clustered", cfg, 9)
    sim = sim_for(cfg)
    try:
        sim.set_state(x, y, th, 3)
        sim.debug_enable(True)
        sim.step(1)
        d = sim.debug_last_step()
    finally:
        sim.close()
    p = oracle_params(cfg)
    g = np.random.default_rng(0)
    idx = g.choice(cfg["N"], 256, replace=False)
    n, C, S, _ = orc.neighbours_brute(x, y, th, p, idx)
    assert np.array_equal(d["n"][idx].astype(np.int64), n)
    tol = cs_tolerance(n)
    assert np.all(np.abs(d["C"][idx].astype(np.float64) - C) <= tol)
    assert np.all(np.abs(d["S"][idx].astype(np.float64) - S) <= tol)


def test_dense_cluster_exactly():
    # ~700 particles within a radius of ~1.5 cells (about 100 per cell)
    cfg = W.workload("vm_small")
    g = np.random.default_rng(4)
    x, y, th = W.uniform_state(4096, 64.0, 64.0, 4)
    k = 700
    x[:k] = (20.0 + g.normal(0, 0.5, k)).astype(np.float32)
    y[:k] = (30.0 + g.normal(0, 0.5, k)).astype(np.float32)
    one_step_parity(cfg, (x, y, th))


def test_overfull_cell_exactly():
    # 1200 particles in one cell, and a crowd at a reflecting corner
    cfg = W.workload("vm_small")
    x, y, th = W.uniform_state(4096, 64.0, 64.0, 4)
    x[:1200] = np.float32(10.5)
    y[:1200] = np.linspace(10.1, 10.9, 1200).astype(np.float32)
    one_step_parity(cfg, (x, y, th))
    cfgw = W.workload("vm_small", bx=1, by=1)
    x, y, th = W.uniform_state(4096, 64.0, 64.0, 5, 1, 1)
    x[:500] = np.linspace(0.0, 0.9, 500).astype(np.float32)
    y[:500] = np.linspace(0.9, 0.0, 500).astype(np.float32)
    one_step_parity(cfgw, (x, y, th))


@pytest.mark.parametrize("N", [1, 2, 3, 17])
def test_tiny_systems(N):
    cfg = W.workload("vm_small", N=N, Lx=6.0, Ly=5.0)
    x, y, th = W.uniform_state(N, 6.0, 5.0, N)
    one_step_parity(cfg, (x, y, th))
    cfgw = W.workload("vm_small", N=N, Lx=6.0, Ly=5.0, bx=1, by=1)
    x, y, th = W.uniform_state(N, 6.0, 5.0, N, 1, 1)
    one_step_parity(cfgw, (x, y, th))


def test_vanishing_sum_keeps_own_angle():
    # arg(0) read as the particle's own angle.  Particle 0 (angle 0) sees
    # particle 1 (angle 0) and particle 2 (angle just below pi) both directly
    # and through the wall at y = 0 (theta -> -theta); particle 1's image and
    # particle 0's own image lie beyond R.  In 2^-27 fixed point the four
    # vectors cancel exactly, (1, 0) + (1, 0) + (-1, s) + (-1, -s) = 0, so
    # the library takes the own-angle branch; the oracle's binary64 sum is
    # (2.3e-14, 0), whose argument is the same angle 0.
    cfg = W.workload("vm_small", N=3, Lx=8.0, Ly=8.0, eta=0.0, bx=0, by=1)
    x = np.array([4.0, 4.5, 4.0], np.float32)
    y = np.array([0.6, 0.9, 0.2], np.float32)
    th = np.array([0.0, 0.0, np.nextafter(np.float32(np.pi), np.float32(0))], np.float32)
    sim = sim_for(cfg)
    try:
        sim.set_state(x, y, th, 3)
        sim.debug_enable(True)
        sim.step(1)
        dbg = sim.debug_last_step()
        _, _, tg, _ = sim.get_state()
    finally:
        sim.close()
    assert list(dbg["n"][:3]) == [3, 2, 3]
    assert dbg["C"][0] == 0.0 and dbg["S"][0] == 0.0
    assert tg[0] == 0.0
    one_step_parity(cfg, (x, y, th), step=3)


def test_non_power_of_two_box():
    # the run-time scan's box L = sqrt(N / 0.6366) is not a binary32 number;
    # the library rounds it once and both sides use the rounded value
    cfg = W.workload("runtime_vs_n", N=20000)
    x, y, th = W.uniform_state(cfg["N"], float(np.float32(cfg["Lx"])) * 0.999999,
                               float(np.float32(cfg["Ly"])) * 0.999999, 1)
    one_step_parity(cfg, (x, y, th))


def test_init_matches_oracle():
    cfg = W.workload("vm_small", seed=123)
    sim = sim_for(cfg)
    try:
        xg, yg, tg, st = sim.get_state()
    finally:
        sim.close()
    assert st == 0
    xo, yo, to = orc.init_state(oracle_params(cfg))
    # L = 64 is a power of two: L * u is exact in binary32
    assert np.array_equal(xg, xo.astype(np.float32))
    assert np.array_equal(yg, yo.astype(np.float32))
    assert np.max(np.abs(tg - to)) < 4e-7


def test_set_state_validation():
    cfg = W.workload("vm_small")
    sim = sim_for(cfg)
    from paper_2211_15630_amd import binding as B
    try:
        x, y, th = W.uniform_state(4096, 64.0, 64.0, 0)
        x[5] = 64.0          # periodic: outside [0, L)
        with pytest.raises(B.AapError) as e:
            sim.set_state(x, y, th)
        assert e.value.code == B.AAP_EINVAL
        x[5] = np.nan
        with pytest.raises(B.AapError):
            sim.set_state(x, y, th)
        x[5] = 1.0
        pi32 = np.float32(math.pi)
        th[7] = np.nextafter(pi32, np.float32(4))   # just above pi in binary32
        with pytest.raises(B.AapError):
            sim.set_state(x, y, th)
        th[7] = -pi32                               # the ends of [-pi, pi] are accepted
        th[8] = pi32
        sim.set_state(x, y, th)
        with pytest.raises(B.AapError):
            sim.debug_last_step()   # no captured step yet
    finally:
        sim.close()


def test_unit_vectors_dense_angles():
    # Isolated particles (grid spacing 2.5 R, steps of 0.2 R): each sum is
    # the particle's own unit vector, rounded to 2^-27 and then to binary32.
    # Checked against binary64 cos/sin over a dense angle grid that includes
    # the quadrant boundaries and +-pi: first the vectors made from the
    # state set on the host, then those of the angles one step stores.
    side, sp = 256, 2.5
    N, L = side * side, side * sp
    cfg = W.workload("vm_small", N=N, Lx=L, Ly=L, v=0.2, eta=0.3, seed=4)
    g = (np.arange(side) * sp + sp / 2).astype(np.float32)
    x, y = (a.ravel().copy() for a in np.meshgrid(g, g))
    th = np.linspace(-np.pi, np.pi, N, endpoint=False).astype(np.float32)
    q = np.pi / 4
    special = [0.0, 1e-30, -1e-30, 1e-8, -1e-8, q, -q, 2 * q, -2 * q, 3 * q, -3 * q,
               np.pi, -np.pi, np.nextafter(np.float32(q), np.float32(0)),
               np.nextafter(np.float32(q), np.float32(1)),
               np.nextafter(np.float32(3 * q), np.float32(4))]
    th[:len(special)] = np.array(special, dtype=np.float32)
    tol = 2.0 ** -21
    sim = sim_for(cfg)
    try:
        sim.set_state(x, y, th, 0)
        sim.debug_enable(True)
        sim.step(1)
        d1 = sim.debug_last_step()
        _, _, th1, _ = sim.get_state()
        sim.step(1)
        d2 = sim.debug_last_step()
    finally:
        sim.close()
    for d, t in ((d1, th), (d2, th1)):
        assert np.all(d["n"] == 0)
        t64 = t.astype(np.float64)
        ec = np.abs(d["C"].astype(np.float64) - np.cos(t64))
        es = np.abs(d["S"].astype(np.float64) - np.sin(t64))
        assert ec.max() <= tol, (ec.max(), t[np.argmax(ec)])
        assert es.max() <= tol, (es.max(), t[np.argmax(es)])


@pytest.mark.parametrize("kind", ["uniform", "banded", "clustered", "edge"])
@pytest.mark.parametrize("walls", [0, 1])
def test_second_step_sorted_path(kind, walls):
    cfg = W.workload("vm_small", bx=walls, by=walls)
    second_step_parity(cfg, _state(kind, cfg, 11 + walls))


def test_second_step_sorted_path_large():
    # N = 2^20: 512 counting-sort tiles, the look-back across them, and the
    # cyclic row windows at the top and bottom of the box
    cfg = W.workload("vm_large", eta=0.4)
    second_step_parity(cfg, _state("banded", cfg, 5))


def test_second_step_sorted_path_many_tiles():
    # L = 2100: 2099^2 cells in 2152 sort tiles, past the point where each
    # tile's offset comes from the scan of the tile counts
    cfg = W.workload("vm_large", Lx=2100.0, Ly=2100.0, eta=0.4)
    second_step_parity(cfg, _state("clustered", cfg, 14))


def test_second_step_sorted_path_langevin_walls():
    cfg = W.workload("langevin_walls", N=65536, Lx=128.0, Ly=128.0, D=0.05)
    second_step_parity(cfg, _state("clustered", cfg, 6))


def test_second_step_sorted_path_fast_particles():
    # v = 2.7 cell sides per step: each tile gathers arrivals from three rows
    # on either side
    cfg = W.workload("vm_small", v=2.7, eta=0.2)
    second_step_parity(cfg, _state("uniform", cfg, 8))


# --- nematic Vicsek rule (Eq. (3)) and interaction order o >= 2 (Eq. (5)) ---

@pytest.mark.parametrize("bx,by", [(0, 0), (1, 1), (1, 0)])
@pytest.mark.parametrize("kind", ["uniform", "banded", "clustered", "edge"])
def test_nvm_small_one_step(kind, bx, by):
    # chirality on the walled boxes
    cfg = W.workload("nvm_small", bx=bx, by=by, omega=0.2 if bx else 0.0)
    rep, _ = one_step_parity(cfg, _state(kind, cfg, 13))
    print(kind, bx, by, rep)


@pytest.mark.parametrize("bx,by", [(0, 0), (1, 1), (0, 1)])
def test_nvm_quarter_turn_pairs(bx, by):
    # partners a quarter (or three quarters) turn apart to within 2 ulps,
    # directly and through wall images: the exact sign test decides
    x, y, th = W.quarter_turn_pairs(48.0, 40.0, 21 + bx + 2 * by, bx, by)
    cfg = W.workload("nvm_small", N=len(x), Lx=48.0, Ly=40.0, bx=bx, by=by)
    one_step_parity(cfg, (x, y, th))


def test_nvm_large_one_step():
    cfg = W.workload("nvm_large")
    one_step_parity(cfg, _state("banded", cfg, 2))


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("bx,by", [(0, 0), (1, 1), (1, 0)])
@pytest.mark.parametrize("kind", ["clustered", "edge"])
def test_langevin_order_one_step(kind, order, bx, by):
    cfg = W.workload("langevin_nematic", order=order, bx=bx, by=by, omega=0.15)
    one_step_parity(cfg, _state(kind, cfg, 4 + order))


@pytest.mark.parametrize("name,over", [
    ("nvm_small", dict()),
    ("nvm_small", dict(bx=1, by=1)),
    ("langevin_nematic", dict()),
    ("langevin_nematic", dict(order=3, bx=1, by=1)),
])
def test_second_step_sorted_path_rules(name, over):
    cfg = W.workload(name, **over)
    second_step_parity(cfg, _state("clustered", cfg, 9))


@pytest.mark.parametrize("N", [12000, 20000])
def test_second_step_sort_beyond_one_chunk(N):
    """Two counting-sort tiles (63 x 63 cells) with more sources each than
    one register chunk of the sort (4096): the kept chunk (N = 12000) and
    the re-read later chunks (N = 20000), and the neighbour kernel still
    writes the oracle's (cell, id) order."""
    cfg = W.workload("vm_small", N=N)
    second_step_parity(cfg, _state("clustered", cfg, 13))


@pytest.mark.parametrize("rule,over", [
    (W.RULE_VM, dict()),
    (W.RULE_VM, dict(bx=1, by=1)),
    (W.RULE_NVM, dict(bx=1, omega=0.2)),
    (W.RULE_LANGEVIN, dict(bx=1, by=1, dt=0.1, weights=W.inverse_n_weights(4096))),
    (W.RULE_LANGEVIN, dict(order=2, dt=0.1, weights=W.inverse_n_weights(4096))),
])
def test_dense_rows_one_and_two_steps(rule, over):
    """About 30 particles per cell everywhere (30000 in a 32 x 32 box): a wave
    spans two or three cells, its three tile rows hold ~150 records each --
    too many together for the per-wave tile, few enough one row at a time,
    so the interior waves take the row-by-row staged path; a denser patch
    (~120 per cell) has rows longer than the tile, staged in pieces."""
    cfg = W.workload("vm_small", N=30000, Lx=32.0, Ly=32.0, rule=rule, eta=0.25, **over)
    g = np.random.default_rng(21)
    x, y, th = W.uniform_state(30000, 32.0, 32.0, 21, cfg["bx"], cfg["by"])
    k = 2000
    x[:k] = (8.0 + g.uniform(0.0, 2.0, k)).astype(np.float32)
    y[:k] = (20.0 + g.uniform(0.0, 2.0, k)).astype(np.float32)
    rep, _ = one_step_parity(cfg, (x, y, th))
    rep2 = second_step_parity(cfg, (x, y, th))
    print(rule, over, rep, rep2)


@pytest.mark.parametrize("rule,rho", [(W.RULE_VM, 4), (W.RULE_VM, 8), (W.RULE_VM, 12),
                                      (W.RULE_VM, 20), (W.RULE_NVM, 8), (W.RULE_LANGEVIN, 8)])
def test_wrapped_tile_densities(rule, rho):
    """Periodic 64 x 64 box at rho particles per cell.  The waves across the
    x seam (end of one row, start of the next) stage all nine of their
    segments in LDS at rho = 4, only the three range segments at rho = 8
    and 12 (the six wrapped cells are read from the cell-sorted array), none
    at rho = 20; the one-row waves of the first and the last row read the
    row across the y edge from the same staged tile."""
    over = {}
    if rule == W.RULE_LANGEVIN:
        over = dict(order=2, dt=0.1, weights=W.inverse_n_weights(4096))
    cfg = W.workload("vm_small", N=rho * 4096, rule=rule, eta=0.25, **over)
    st = W.uniform_state(cfg["N"], 64.0, 64.0, 40 + rho, 0, 0)
    rep, _ = one_step_parity(cfg, st)
    rep2 = second_step_parity(cfg, st)
    print(rule, rho, rep, rep2)


@pytest.mark.parametrize("rule,per_row", [(W.RULE_VM, 128), (W.RULE_VM, 384), (W.RULE_NVM, 128),
                                          (W.RULE_LANGEVIN, 128)])
def test_row_aligned_waves(rule, per_row):
    """Every cell row of a periodic 64 x 64 box holds a multiple of 64
    particles, so every row starts and ends a wave: the first and last wave
    of each row are one-row waves with a lane in column 0 or Mx - 1, which
    read the cell across the x edge (seen at x -+ L) from their staged tile
    in rows 2 .. My - 3 and take the image-map walk in the other rows."""
    over = {}
    if rule == W.RULE_LANGEVIN:
        over = dict(order=2, dt=0.1, weights=W.inverse_n_weights(4096))
    M = orc.cells_per_axis(64.0, 1.0)
    cs = 64.0 / M
    g = np.random.default_rng(per_row + rule)
    ys = [j * cs + g.uniform(0.01, cs - 0.01, per_row) for j in range(M)]
    y = np.concatenate(ys).astype(np.float32)
    x = g.uniform(0.0, 63.99, y.size).astype(np.float32)
    th = g.uniform(-np.pi, np.pi, y.size).astype(np.float32)
    cfg = W.workload("vm_small", N=int(y.size), rule=rule, eta=0.25, **over)
    key = orc.cell_keys(x, y, 64.0, 64.0, 1.0).astype(np.int64)
    assert np.all(np.bincount(key // M, minlength=M) == per_row)
    rep, _ = one_step_parity(cfg, (x, y, th))
    rep2 = second_step_parity(cfg, (x, y, th))
    print(rule, per_row, rep, rep2)


@pytest.mark.parametrize("Lx,Ly,bx,by", [(3.2, 64.0, 0, 0), (64.0, 3.2, 0, 0), (3.2, 64.0, 0, 1),
                                         (64.0, 3.2, 1, 0), (3.2, 3.2, 0, 0)])
def test_narrow_boxes_wrapped_tiles(Lx, Ly, bx, by):
    """Boxes three cells wide or high, 40 particles per cell: seam waves and
    one-row waves whose wrapped cell or row is one of only three, next to
    walls on the other axis, and a 3 x 3 box where every wave touches an
    edge."""
    Mx, My = orc.cells_per_axis(Lx, 1.0), orc.cells_per_axis(Ly, 1.0)
    N = 40 * Mx * My
    cfg = W.workload("vm_small", N=N, Lx=Lx, Ly=Ly, bx=bx, by=by, eta=0.25)
    st = W.uniform_state(N, Lx, Ly, 50 + Mx + My, bx, by)
    one_step_parity(cfg, st)
    second_step_parity(cfg, st)


def test_uneven_xcd_pieces():
    """N = 70001 in a periodic 264 x 264 box: 1094 neighbour workgroups and
    34 sort tiles, neither a multiple of 8, so the four pieces each XCD is
    dealt (systems of 2^16 to 2^21 particles) differ in length; every
    particle must still be handled once, in one and two steps."""
    cfg = W.workload("vm_small", N=70001, Lx=264.0, Ly=264.0, eta=0.3)
    st = W.uniform_state(cfg["N"], 264.0, 264.0, 77, 0, 0)
    one_step_parity(cfg, st)
    second_step_parity(cfg, st)

"""The allocation-free fields entry point (aap_fields_noalloc) against
aap_fields with a caller-provided scratch, through the C ABI: two calls in a
row on one GPU (the second on a smaller system and grid, so it reuses the
static scratch the first left behind), the largest grid the static scratch
allows, and the error beyond it.  The fields are exact integer sums scaled
once, so both entry points must agree bit for bit."""
import numpy as np
import pytest
import torch

from paper_2211_15630_amd import binding as B
from paper_2211_15630_amd import workloads as W

pytestmark = pytest.mark.gpu

MAX_G = 512


def _sim(N, L, seed):
    cfg = W.workload("vm_small", N=N, Lx=L, Ly=L, eta=0.3, seed=seed)
    sim = B.Sim(**W.model_params(cfg))
    sim.step(7, measure=False)
    return sim


def _both(sim, G):
    ref = B.sim_fields(sim, G).cpu().numpy()
    out = torch.full((3, G, G), float("nan"), dtype=torch.float32, device=sim.device)
    B.sim_fields_noalloc(sim, G, out)
    sim.stream.synchronize()
    return out.cpu().numpy(), ref


def test_noalloc_fields_equal_fields_two_calls_second_smaller():
    big = _sim(1 << 18, 512.0, 3)
    small = _sim(3000, 48.0, 4)
    try:
        got, ref = _both(big, 256)
        assert np.array_equal(got, ref)
        assert np.sum(ref[0]) > 0
        # second call: fewer particles and a smaller grid, same static scratch
        got, ref = _both(small, 40)
        assert np.array_equal(got, ref)
        # total mass: every particle counted once (densities per unit area)
        side = 48.0 / 40
        assert abs(np.sum(got[0].astype(np.float64)) * side * side - 3000) < 1e-3
    finally:
        big.close()
        small.close()


def test_noalloc_fields_largest_grid_and_beyond():
    sim = _sim(1 << 16, 256.0, 5)
    try:
        got, ref = _both(sim, MAX_G)
        assert np.array_equal(got, ref)
        out = torch.empty((3, MAX_G + 1, MAX_G + 1), dtype=torch.float32, device=sim.device)
        with pytest.raises(RuntimeError, match="grid side"):
            B.sim_fields_noalloc(sim, MAX_G + 1, out)
        # the failed call left the simulation usable, and repeated calls agree
        got2, _ = _both(sim, MAX_G)
        assert np.array_equal(got2, got)
    finally:
        sim.close()

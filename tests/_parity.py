"""Shared helpers of the GPU parity tests: build a simulation through the C
ABI from a seeded synthetic state, run the oracle on the same state, and
compare with the tolerances derived from the binary32 arithmetic."""
import math

import numpy as np

import oracle as orc
from paper_2211_15630_amd import binding as B
from paper_2211_15630_amd import workloads as W

TWO_M24 = 2.0 ** -24


def sim_for(cfg, **over):
    kw = W.model_params(cfg)
    kw.update(over)
    return B.Sim(**kw)


def oracle_params(cfg):
    kw = W.model_params(cfg)
    # the library rounds the box sides to binary32; the oracle gets the same
    kw["Lx"] = float(np.float32(kw["Lx"]))
    kw["Ly"] = float(np.float32(kw["Ly"]))
    return orc.Params(**kw)


def cs_tolerance(n):
    """|C_gpu - C_orc| bound for n+1 unit-vector terms: each binary32
    sincosf term is within 4 ulp (<= 2^-22 for |v| < 1) of the exact value,
    is rounded once to a multiple of 2^-27, the terms are added exactly in
    integers, and the total (|C| <= n+1) is rounded once to binary32
    (<= (n+1) 2^-24).  Sum: < (n+1) 2^-21."""
    n = np.asarray(n, dtype=np.float64)
    return (n + 1.0) * 2.0 ** -21 + 1e-12


def angle_diff(a, b):
    d = (np.asarray(a, np.float64) - np.asarray(b, np.float64) + math.pi) % (2 * math.pi) - math.pi
    return np.abs(d)


def periodic_diff(a, b, L):
    d = (np.asarray(a, np.float64) - np.asarray(b, np.float64) + L / 2) % L - L / 2
    return np.abs(d)


def compare_cells(sim, x, y, th, cfg, debug):
    """Exact comparison of keys, cell starts and order; returns the oracle
    cell counts."""
    p = oracle_params(cfg)
    key = orc.cell_keys(x, y, p.Lx, p.Ly, p.R)
    Mx, My = orc.cells_per_axis(p.Lx, p.R), orc.cells_per_axis(p.Ly, p.R)
    count, start, order = orc.cell_lists(key, Mx * My)
    assert np.array_equal(debug["start"], start), "cell starts differ"
    assert np.array_equal(debug["order"], order), "cell-list order differs"
    return key


def compare_sums(cfg, x, y, th, debug):
    """n exact; C, S within cs_tolerance.  For the Langevin rule of order
    o >= 2 the library's C, S are the sums of the o-th harmonics, which
    enter only through A = S cos(o th_i) - C sin(o th_i): A is compared with
    the oracle's sum of sin(o (th~_j - th_i)) within the bound of its two
    terms."""
    p = oracle_params(cfg)
    n, C, S, A = orc.neighbours_cells(x, y, th, p)
    assert np.array_equal(debug["n"].astype(np.int64), n), \
        f"neighbour counts differ at {np.flatnonzero(debug['n'] != n)[:10]}"
    tol = cs_tolerance(n)
    Cg = debug["C"].astype(np.float64)
    Sg = debug["S"].astype(np.float64)
    if p.rule == orc.RULE_LANGEVIN and p.order != 1:
        o_th = p.order * np.asarray(th, np.float64)
        Ag = Sg * np.cos(o_th) - Cg * np.sin(o_th)
        dA = np.abs(Ag - A)
        assert np.all(dA <= 2 * tol), f"A max excess {np.max(dA - 2 * tol)}"
        return n, C, S, A
    dC = np.abs(Cg - C)
    dS = np.abs(Sg - S)
    assert np.all(dC <= tol), f"C max excess {np.max(dC - tol)} at {np.argmax(dC - tol)}"
    assert np.all(dS <= tol), f"S max excess {np.max(dS - tol)} at {np.argmax(dS - tol)}"
    return n, C, S, A


def compare_update(cfg, x, y, th, n, C, S, A, xg, yg, tg, step):
    """One-step parity of theta', x', y' from the same binary32 state.

    theta': 1e-5 rad, widened where arg[C + iS] is ill-conditioned by the
    bound on |(dC, dS)| / |C + iS| (VM only).  Positions: 1e-5 L (modulo L
    on periodic axes).  A particle whose wall crossing differs between the
    two sides (it ends within rounding of a wall) may show the mirrored
    orientation instead."""
    p = oracle_params(cfg)
    xo, yo, to = orc.update(x, y, th, n, C, S, A, p, step)
    tol_t = np.full(len(xo), 1e-5)
    if p.rule != orc.RULE_LANGEVIN:
        r = np.hypot(C, S)
        with np.errstate(divide="ignore"):
            tol_t = np.maximum(tol_t, 1e-5 + 2.0 * cs_tolerance(n) / r)
    dt_ = angle_diff(tg, to)
    bad = dt_ > tol_t
    n_mirrored = 0
    if bad.any():
        # A particle that ends within rounding of a reflecting wall may cross
        # it on one side and not on the other: then its angle is the
        # oracle's mirrored by that wall (pi - theta at an x wall, -theta at
        # a y wall, theta - pi when both flips differ), and nothing else.
        eps = 1e-4
        near_x = np.zeros(len(xo), bool)
        near_y = np.zeros(len(xo), bool)
        if p.bx:
            near_x = (xo < eps) | (xo > p.Lx - eps)
        if p.by:
            near_y = (yo < eps) | (yo > p.Ly - eps)
        to64 = np.asarray(to, np.float64)
        mirrored = near_x & (angle_diff(tg, math.pi - to64) <= tol_t)
        mirrored |= near_y & (angle_diff(tg, -to64) <= tol_t)
        mirrored |= near_x & near_y & (angle_diff(tg, to64 - math.pi) <= tol_t)
        wrong = bad & ~mirrored
        assert not np.any(wrong), \
            f"theta' differs at {np.flatnonzero(wrong)[:10]}: max {dt_[wrong].max()}"
        n_mirrored = int(np.sum(bad))
        dt_ = np.where(bad, 0.0, dt_)
    tol_x = 1e-5 * p.Lx
    tol_y = 1e-5 * p.Ly
    dx = periodic_diff(xg, xo, p.Lx) if not p.bx else np.abs(xg - xo)
    dy = periodic_diff(yg, yo, p.Ly) if not p.by else np.abs(yg - yo)
    assert np.all(dx <= tol_x), f"x' max diff {dx.max()}"
    assert np.all(dy <= tol_y), f"y' max diff {dy.max()}"
    n_wide = int(np.sum(tol_t > 1e-5 + 1e-12))
    return dict(max_dtheta=float(dt_.max()), max_dx=float(dx.max()),
                max_dy=float(dy.max()), widened=n_wide, mirrored=n_mirrored)


def one_step_parity(cfg, state, step=7):
    x, y, th = state
    sim = sim_for(cfg)
    try:
        sim.set_state(x, y, th, step)
        key_gpu, _, _ = sim.debug_keys()
        p = oracle_params(cfg)
        key = orc.cell_keys(x, y, p.Lx, p.Ly, p.R)
        assert np.array_equal(key_gpu, key), "cell ids differ"
        sim.debug_enable(True)
        sim.step(1)
        dbg = sim.debug_last_step()
        compare_cells(sim, x, y, th, cfg, dbg)
        n, C, S, A = compare_sums(cfg, x, y, th, dbg)
        xg, yg, tg, st = sim.get_state()
        assert st == step + 1
        rep = compare_update(cfg, x, y, th, n, C, S, A, xg, yg, tg, step)
        return rep, (xg, yg, tg)
    finally:
        sim.close()


def second_step_parity(cfg, state, step=7):
    """Parity of the second step after set_state: the state the first step
    produced is cell-sorted on the device, so the second step sorts it with
    the counting-sort kernel of later steps.  The oracle starts from that
    state as read back."""
    x, y, th = state
    sim = sim_for(cfg)
    try:
        sim.set_state(x, y, th, step)
        sim.step(1)
        x1, y1, t1, st = sim.get_state()
        assert st == step + 1
        key_gpu, _, _ = sim.debug_keys()
        p = oracle_params(cfg)
        assert np.array_equal(key_gpu, orc.cell_keys(x1, y1, p.Lx, p.Ly, p.R)), "next cells differ"
        sim.debug_enable(True)
        sim.step(1)
        dbg = sim.debug_last_step()
        compare_cells(sim, x1, y1, t1, cfg, dbg)
        n, C, S, A = compare_sums(cfg, x1, y1, t1, dbg)
        xg, yg, tg, st2 = sim.get_state()
        assert st2 == step + 2
        return compare_update(cfg, x1, y1, t1, n, C, S, A, xg, yg, tg, step + 1)
    finally:
        sim.close()

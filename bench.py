"""Throughput of the metric Vicsek step on one MI355X.

One "step" is the whole hot path for every particle: the counting sort into
cells, 3x3-stencil neighbour sums + noisy angle update + streaming (+ the
per-step polarisation measurement).  Default workload: standard Vicsek
model, N = 2^20 particles, periodic L = 1024 (density 1), R = 1, v = 0.5,
eta = 0.4, seed 0, measurement on, state resident in HBM.

Other workloads (--workload):
  vm_small        the same model at N = 4096, L = 64, eta = 0.3 (1000 steps);
  dram_control    the same model at N = 2^24 (or --N), L = sqrt(N), a working
                  set beyond the last-level cache;
  langevin_walls  the overdamped Langevin model with reflecting walls, N = 4 *
                  2^20, L = 1024, h(n) = 1/n, dt = 0.1, --D (0.05 or 0.2),
                  --order o (1 unless given);
  nvm_large       the nematic Vicsek model of Sec. 5 (N = 2^19, L = 512,
                  eta = 0.065);
  batch_replicas  256 standard-Vicsek replicas of uneven N (log-uniform in
                  [1024, 65536]), density (uniform in [0.25, 4]) and noise
                  (spaced over [0.1, 0.7]) stepped as one batch (two launches
                  per step for all replicas, captured graphs and workgroup size
                  chosen by the autotuner), against the same replicas stepped
                  one by one as single systems from the same states for the
                  same measured steps -- identical trajectories, hence matched
                  <phi> error -- and the <phi>(eta) curve per density quartile;
  surrogate       the learned field model on N = 4 * 2^20, L = 1024, eta = 0.4
                  Vicsek runs (see surrogate.py).

Prints one JSON line: particle-updates/s over the timed steps; the roofline
position of the dominant kernel (its minimal bytes per launch over its
average device time from HIP events on the dispatches of sampled timed
steps, on the simulation's stream) and of the whole step; repeats of the
timed region, the rate without measurement, a plain copy kernel's bandwidth,
the environment, and the oracle's rate on the host cores on a bounded sample
of the same workload.
"""
import argparse
import copy
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle-updates/s (Vicsek N=2^20); batched vs plain at matched "
          "⟨φ⟩ error")
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("paper_2211_15630_amd/csrc/aap_kernels.hip",
                  "paper_2211_15630_amd/csrc/aap_internal.h")
WORKLOADS = ("vm_large", "vm_small", "dram_control", "nvm_large", "langevin_walls",
             "batch_replicas", "surrogate")
MFMA_BF16_PEAK_TFLOPS = 2500.0


def algorithmic_bytes(N, cells):
    """The minimal bytes of one step of the counting-sort + 3x3-stencil
    structure, each required stream counted once (candidates re-read by
    neighbouring particles come from the caches):
      sort share      record read 16 B + written 16 B, next cell read 4 B per
                      particle; count and start written per cell (8 B);
      neighbour share sorted record read 16 B, x, y, theta written 12 B, next
                      cell written 4 B per particle; start read per cell (4 B).
    Sum: 68 B per particle + 12 B per cell."""
    return {
        "k_sort": 36 * N + 8 * cells,
        "k_nbr": 32 * N + 4 * cells,
        "step": 68 * N + 12 * cells,
    }


def design_bytes(N, cells):
    """Bytes the kernels of this library move per launch with its own record
    layout (Cand 16 B = x, y, cos, sin; Ori 8 B = theta, id; next cell 4 B;
    start 4 B per cell).  k_scan and k_scatter sort only the first step after
    an initial or restored state."""
    return {
        # count read and cleared, start written
        "k_scan": 12 * cells,
        # (cell, slot), Cand, Ori read; Cand, Ori written; start read
        "k_scatter": N * (8 + 16 + 8 + 16 + 8) + cells * 4,
        # next cell, Cand, Ori read; Cand, Ori written; start written
        "k_sort": N * (4 + 16 + 8 + 16 + 8) + cells * 4,
        # Cand, Ori read; Cand, Ori, next cell written; start read
        "k_nbr": N * (16 + 8 + 16 + 8 + 4) + cells * 4,
    }


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_profile(workload):
    return os.path.join(ROOT, "profiles", f"k_nbr_{workload}_traffic.md")


def measured_traffic(workload="vm_large"):
    """HBM bytes per k_nbr launch from the committed counter summary of the
    workload, or None when there is none or it was taken on other kernel
    sources."""
    path = traffic_profile(workload)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_val or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_val.group(1))


def cpu_baseline(cfg, budget_s):
    """The oracle (binary64, OpenMP over particles) on the same workload:
    init, then whole steps until the time budget is spent, on every core it
    may use; then, for a third of the budget (at least one step), on one
    core."""
    import oracle as orc
    from paper_2211_15630_amd import workloads as W
    p = orc.Params(**W.model_params(cfg))

    def timed(budget):
        x, y, th = orc.init_state(p)
        steps = 0
        t0 = time.perf_counter()
        while True:
            x, y, th, _, _ = orc.run(x, y, th, p, steps, 1, measure=True)
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return steps, el

    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    if threads <= 0 or threads > cores:
        threads = cores
    orc.set_threads(threads)
    threads = orc.max_threads()
    steps, el = timed(budget_s)
    orc.set_threads(1)
    steps1, el1 = timed(budget_s / 3)
    orc.set_threads(threads)
    return {
        "value": cfg["N"] * steps / el,
        "unit": "particle-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{steps} full steps of the same workload (N={cfg['N']}) after init, "
                  f"{el:.1f} s wall, binary64, cell lists",
        "one_core": {"value": cfg["N"] * steps1 / el1, "cores": 1,
                     "sample": f"{steps1} full steps, {el1:.1f} s wall"},
    }


# The paper's own serial rate for the standard Vicsek model with cell lists
# (context, other hardware): the two guide lines of its run-time figure
# (Fig. 7) give 0.0072 s x N for init + 10^4 steps at large N, and
# 150 s x rho0 for 10^4 steps of N = 10^5 at large density.
PAPER_SERIAL = {
    "value_range": [1.4e6, 6.7e6],
    "unit": "particle-updates/s per core",
    "hardware": "one CPU core of the Brain-Cluster (Greifswald), serial C in binary64; "
                "CPU model not stated",
    "source": "Fig. 7 guide lines: 1/(0.0072 s / 1e4) at large N; 1/(150 s x rho0 / (1e5 x 1e4)) "
              "at rho0 = 1",
}


def run_batch(a, steps, warmup, plain_steps=None):
    """The replica batch against single systems (see the module docstring);
    returns the JSON object.  plain_steps: steps of the one-by-one
    comparison (default: all the batch's steps; 0 skips it).  The batch's
    observables are read after exactly plain_steps steps for the comparison,
    so both sides are compared on the same measured states."""
    import numpy as np
    import torch
    from paper_2211_15630_amd import binding as B
    from paper_2211_15630_amd import workloads as W

    cfgs = W.batch_replicas()
    reps = [W.model_params(c) for c in cfgs]
    Ns = np.array([c["N"] for c in cfgs], dtype=np.int64)
    Ntot = int(Ns.sum())
    b = B.Batch(reps)
    b.step(1, measure=True)
    b.step(warmup, measure=True)
    threads, graph = b.autotune(16, True)
    sort_ms, nbr_ms = b.kernel_times(100, True)
    b.sync()
    print(f"# batch of {len(reps)} replicas, {Ntot} particles: workgroup {threads}, "
          f"graph {graph} steps; sort {sort_ms*1e3:.1f} us, nbr {nbr_ms*1e3:.1f} us",
          file=sys.stderr, flush=True)
    psteps = steps if plain_steps is None else min(plain_steps, steps)
    states = [b.get_state(r) for r in range(len(reps))]
    b.reset_observables()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wall_b_cmp = None
    obs_cmp = None
    if 0 < psteps < steps:
        b.step(psteps, measure=True)
        b.sync()
        wall_b_cmp = time.perf_counter() - t0
        obs_cmp = b.observables()        # the measured states 0 .. psteps-1
        t1 = time.perf_counter()
        b.step(steps - psteps, measure=True)
        b.sync()
        wall_b = wall_b_cmp + (time.perf_counter() - t1)
    else:
        b.step(steps, measure=True)
        b.sync()
        wall_b = time.perf_counter() - t0
    torch.cuda.synchronize()
    obs_b = b.observables()
    if obs_cmp is None:
        obs_cmp = obs_b
        wall_b_cmp = wall_b
    cells = 0
    for r in range(len(reps)):
        mx = cells_per_axis(reps[r]["Lx"], reps[r]["R"])
        cells += mx * mx
    b.close()
    # the same replicas one by one, from the same states, for psteps steps
    wall_p = 0.0
    dphi = None
    dbinder = None
    for r, kw in enumerate(reps if psteps > 0 else []):
        sim = B.Sim(**kw)
        x, y, th, st = states[r]
        sim.set_state(x, y, th, st)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(psteps, measure=True)
        sim.sync()
        wall_p += time.perf_counter() - t0
        ob = sim.observables()
        d = abs(ob["p_mom"][0] - obs_cmp[r]["p_mom"][0])
        dphi = d if dphi is None else max(dphi, d)
        du = abs(ob["binder"] - obs_cmp[r]["binder"])
        dbinder = du if dbinder is None else max(dbinder, du)
        sim.close()
    if psteps > 0:
        print(f"# {psteps} steps: batched {wall_b_cmp:.3f} s, one by one {wall_p:.3f} s; "
              f"max |d<phi>| = {dphi:.3g}, max |dU| = {dbinder:.3g}",
              file=sys.stderr, flush=True)
    value = Ntot * steps / wall_b
    plain = Ntot * psteps / wall_p if wall_p > 0 else None
    batched_cmp = Ntot * psteps / wall_b_cmp if psteps > 0 else None
    alg = algorithmic_bytes(Ntot, cells)
    dom = "k_nbr" if nbr_ms >= sort_ms else "k_sort"
    dom_ms = max(nbr_ms, sort_ms)
    achieved = alg[dom] / (dom_ms * 1e-3) / 1e9
    step_achieved = alg["step"] / (wall_b / steps) / 1e9
    rho = np.array([c["density"] for c in cfgs])
    eta = np.array([c["eta"] for c in cfgs])
    phi = np.array([o["p_mom"][0] for o in obs_b])
    # per-replica standard error of <phi> from its time series moments,
    # assuming independent states (a lower bound: successive states are
    # correlated)
    var = np.array([max(o["p_mom"][1] - o["p_mom"][0] ** 2, 0.0) for o in obs_b])
    se = np.sqrt(var / steps)
    edges = np.quantile(rho, [0, 0.25, 0.5, 0.75, 1.0])
    curves = []
    for q in range(4):
        sel = (rho >= edges[q]) & ((rho < edges[q + 1]) if q < 3 else (rho <= edges[q + 1]))
        idx = np.flatnonzero(sel)
        idx = idx[np.argsort(eta[idx])]
        curves.append({"density": [round(float(edges[q]), 3), round(float(edges[q + 1]), 3)],
                       "eta": [round(float(e), 4) for e in eta[idx]],
                       "phi": [round(float(v), 4) for v in phi[idx]],
                       "phi_se_iid": [float("%.2g" % v) for v in se[idx]],
                       "N": [int(n) for n in Ns[idx]]})
    if psteps > 0:
        phi_error = {"compared_steps": psteps,
                     "max_abs_dphi": dphi, "max_abs_dbinder": dbinder,
                     "note": "the same states stepped by the same kernels: the trajectories, "
                             "hence <phi> and its statistical error, are identical, so the "
                             "time ratio at equal steps is the ratio at matched <phi> error"}
    else:
        phi_error = None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall_b / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (uniform isotropic initial states from Philox, seed 0, replica r)",
        "config": {"workload": "batch_replicas: 256 standard-Vicsek replicas, N log-uniform in "
                               "[1024, 65536], density uniform in [0.25, 4], eta spaced over "
                               "[0.1, 0.7], R=1, v=0.5, periodic, measured every step",
                   "replicas": len(reps), "particles": Ntot, "parallelism": "single GPU",
                   "workgroup": threads, "steps_per_graph": graph},
        "batched_vs_plain": {"steps": psteps, "batched": batched_cmp, "plain": plain,
                             "ratio": batched_cmp / plain if plain else None,
                             "plain_ms_per_step": wall_p / psteps * 1e3 if plain else None,
                             "phi_error": phi_error},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": dom + "_b", "avg_us": dom_ms * 1e3, "launches": 100,
                     "alg_bytes_per_launch": alg[dom],
                     "step": {"alg_bytes": alg["step"], "achieved": step_achieved,
                              "frac": step_achieved / HBM_PEAK_GBS}},
        "kernels": {"k_sort_b": {"avg_us": round(sort_ms * 1e3, 3), "alg_bytes": alg["k_sort"]},
                    "k_nbr_b": {"avg_us": round(nbr_ms * 1e3, 3), "alg_bytes": alg["k_nbr"]}},
        "phi_eta_curves": curves,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(cfgs, a.cpu_seconds)
    return out


def cells_per_axis(L, R):
    """Cells per axis of a box side (the library's rule, floor(L / (R (1 + 2^-20))))."""
    import math
    import numpy as np
    return int(math.floor(float(np.float32(L)) / (R * (1.0 + 2.0 ** -20))))


def cpu_baseline_batch(cfgs, budget_s):
    """The oracle on the replicas in order, 20 steps each, until the budget
    is spent."""
    import oracle as orc
    from paper_2211_15630_amd import workloads as W
    done = 0
    t0 = time.perf_counter()
    used = 0
    for c in cfgs:
        p = orc.Params(**W.model_params(c))
        x, y, th = orc.init_state(p)
        orc.run(x, y, th, p, 0, 20, measure=True)
        done += c["N"] * 20
        used += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    cores = len(os.sched_getaffinity(0))
    if threads <= 0 or threads > cores:
        threads = cores
    return {"value": done / el, "unit": "particle-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {used} replicas of the batch, 20 steps each from init, "
                      f"{el:.1f} s wall, binary64, cell lists"}


def run_surrogate(a):
    """The learned field surrogate against the particle simulation."""
    import torch
    from paper_2211_15630_amd import binding as B
    from paper_2211_15630_amd import surrogate as SG
    from paper_2211_15630_amd import workloads as W

    log = lambda m: print("# " + m, file=sys.stderr, flush=True)
    cfg = SG.surrogate_config()
    snaps, gst = SG.generate(cfg, log)
    log(f"generated {gst}")
    cnn, tst = SG.train(snaps, cfg, epochs=a.epochs, log=log)
    ev = SG.evaluate(cnn, snaps, cfg)
    log(f"evaluation {ev}")
    # rollouts over the whole held-out run, judged by its particle fields
    # every K predictions with fallback to them (tolerances: half the
    # persistence error, and 0.02 in the coarse polar order)
    rho0 = cfg["N"] / cfg["L"] ** 2
    judged = []
    for K in (1, 5, 10, 25):
        jr = SG.judged_rollout(cnn, snaps[cfg["train_runs"]], rho0, K,
                               0.5 * ev["mse_persistence"], 0.02)
        log(f"judged rollout {jr}")
        judged.append(jr)
    G = cfg["G"]
    t1 = SG.time_forward(cnn, G, 1)
    t16 = SG.time_forward(cnn, G, cnn.max_batch)
    cnn.close()
    del snaps
    torch.cuda.empty_cache()
    # the plain particle path on one run of the same system: 50 steps
    w = W.workload("vm_small", N=cfg["N"], Lx=cfg["L"], Ly=cfg["L"], eta=cfg["eta"], seed=0)
    sim = B.Sim(**W.model_params(w))
    sim.step(200)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(1000)
    sim.sync()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / 1000
    sim.close()
    N, every = cfg["N"], cfg["every"]
    value = N * every / t1
    flops = SG.forward_flops(G)
    achieved = flops * cnn.max_batch / t16 / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s (equivalent: N x 50 steps per prediction)",
        "n_gpus": 1,
        "steps": every,
        "warmup": cfg["warmup"],
        "ms_per_step": t1 / every * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 (fp32 accumulation)",
        "data": "synthetic: fields of the library's own Vicsek runs (seeds 0..8)",
        "config": {"workload": "surrogate: 4-layer 3x3 periodic CNN, 32 channels, bf16 MFMA, on "
                               "128x128 (rho, p_x, p_y) fields of standard-Vicsek runs, N=4*2^20, "
                               "L=1024, density 4, eta=0.4, predicting 50 steps ahead; 2000 "
                               "training pairs from 8 runs, evaluated on a held-out run",
                   "N": N, "L": cfg["L"], "grid": G, "parallelism": "single GPU"},
        "surrogate_vs_plain": {"prediction_ms": t1 * 1e3, "plain_50_steps_ms": t_step * every * 1e3,
                               "speedup": t_step * every / t1,
                               "plain_particle_updates_per_s": N / t_step,
                               "field_mse_cnn": ev["mse_cnn"],
                               "field_mse_persistence": ev["mse_persistence"],
                               "field_mse_ratio": ev["mse_ratio"],
                               "judged_rollouts": judged,
                               "phi_drift_after_500_steps": ev["phi_drift_mean"],
                               "phi_drift_max": ev["phi_drift_max"],
                               "phi_true_mean": ev["phi_true_mean"]},
        "training": {"pairs": tst["pairs"], "adam_steps": tst["adam_steps"], "batch": tst["batch"],
                     "seconds": tst["train_seconds"], "epoch_loss": tst["epoch_loss"],
                     "data_seconds": gst["sim_seconds"]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": None,
                     "kernel": "cnn forward (4 conv layers, batch %d)" % cnn.max_batch,
                     "flops_per_field": flops, "avg_us": t16 * 1e6},
    }
    print(json.dumps(out), flush=True)


def describe(name, cfg):
    if name == "vm_large":
        return ("vm_large: standard Vicsek (plain method) N=2^20, periodic L=1024, R=1, "
                "v=0.5, eta=%g, polarisation measured every step" % cfg["eta"])
    if name == "vm_small":
        return ("vm_small: standard Vicsek (plain method) N=4096, periodic L=64, R=1, "
                "v=0.5, eta=%g, polarisation measured every step" % cfg["eta"])
    if name == "dram_control":
        return ("dram_control: standard Vicsek N=%d, periodic L=%g (density 1), R=1, v=0.5, "
                "eta=%g, measured every step (working set beyond the last-level cache)"
                % (cfg["N"], cfg["Lx"], cfg["eta"]))
    if name == "nvm_large":
        return ("nvm_large: nematic Vicsek (Eq. 3) N=2^19, periodic L=512, R=1, v=0.5, "
                "eta=%g, polar and nematic order measured every step" % cfg["eta"])
    return ("langevin_walls: overdamped Langevin (Eq. 5) order %d, h(n)=1/n, N=4*2^20, "
            "L=1024 with reflecting walls, dt=0.1, D=%g (eta=sqrt(2D)=%g), measured every step"
            % (cfg["order"], cfg["eta"] ** 2 / 2.0, cfg["eta"]))


def env_info():
    """ROCm version, GPU architecture, host CPU model and GPU clocks (where
    the tools report them)."""
    import subprocess
    import torch
    info = {}
    try:
        info["rocm"] = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        info["rocm"] = None
    info["torch"] = torch.__version__
    try:
        prop = torch.cuda.get_device_properties(0)
        info["gpu"] = f"{prop.name} ({getattr(prop, 'gcnArchName', '?')}, "  \
                      f"{prop.multi_processor_count} CUs, {prop.total_memory >> 30} GiB)"
    except Exception:
        info["gpu"] = None
    info["cpu_model"] = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    info["host_cores_usable"] = len(os.sched_getaffinity(0))
    try:
        r = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True,
                           timeout=20)
        clk = [ln.strip() for ln in r.stdout.splitlines() if "sclk" in ln or "mclk" in ln]
        info["clocks"] = clk[:4] if clk else None
    except Exception:
        info["clocks"] = None
    return info


def copy_bandwidth(mib=1024, reps=5):
    """Device-to-device copy of mib MiB (torch's copy kernel): read + written
    bytes over the median time of reps copies, in GB/s; beside the 8 TB/s
    peak it shows what a plain streaming kernel reaches on this GPU."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    t = sorted(times)[len(times) // 2]
    return {"bytes": 2 * (mib << 20), "median_us": t * 1e6,
            "GBps": 2 * (mib << 20) / t / 1e9, "frac_of_peak": 2 * (mib << 20) / t / 1e9 /
            HBM_PEAK_GBS}


def run_system(a):
    """One simulation of the chosen workload: warm-up, the timed region, then
    repeats, a run without measurement, and the report."""
    import numpy as np
    import torch
    from paper_2211_15630_amd import binding as B
    from paper_2211_15630_amd import workloads as W

    over = dict(seed=0)
    if a.eta is not None:
        over["eta"] = a.eta
    if a.order is not None:
        if a.workload != "langevin_walls":
            sys.exit("bench.py: --order applies to the langevin_walls workload only")
        over["order"] = a.order
    if a.D is not None:
        if a.workload != "langevin_walls":
            sys.exit("bench.py: --D applies to the langevin_walls workload only")
        over["D"] = a.D
    if a.workload == "dram_control":
        N = a.N if a.N else 1 << 24
        L = float(np.sqrt(N))
        cfg = W.workload("vm_large", N=N, Lx=L, Ly=L, **over)
    else:
        if a.N:
            sys.exit("bench.py: --N applies to the dram_control workload only")
        cfg = W.workload(a.workload, **over)
    N = cfg["N"]
    if a.copy_mb > 0:
        # one plain device copy of known size: the scale of the traffic counters
        src = torch.ones(a.copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# calibration copy: {a.copy_mb} MiB read + {a.copy_mb} MiB written",
              file=sys.stderr, flush=True)
        del src, dst
    sim = B.Sim(**W.model_params(cfg))
    mx, my = sim.cells()
    cells = mx * my
    print(f"# workload {a.workload} N={N} cells={mx}x{my} eta={cfg['eta']:g} "
          f"order={cfg['order']}", file=sys.stderr, flush=True)

    sim.step(a.warmup, measure=True)
    sim.sync()
    sim.reset_observables()

    # timed region: the kernels of every te-th step carry HIP events on
    # their own dispatch (the simulation's stream); at least four steps are
    # sampled however short the region
    te = max(1, min(a.time_every, -(-a.steps // 4)))
    sim.timing_enable(te)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(a.steps, measure=True)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = sim.timing_read()
    sim.timing_enable(False)
    ob = sim.observables()
    print(f"# timed {a.steps} steps: wall {wall:.4f} s, "
          f"<p>={ob['p_mom'][0]:.5f} U={ob['binder']:.4f}", file=sys.stderr, flush=True)

    sim.close()

    def rerun(measure, graph=0):
        """The same workload again from its initial state (the same
        trajectory, no events): warm-up, then the timed steps; graph > 0
        replays runs of that many steps from captured HIP graphs."""
        s2 = B.Sim(**W.model_params(cfg))
        if graph:
            s2.graph(graph)
        s2.step(a.warmup, measure=measure)
        s2.sync()
        torch.cuda.synchronize()
        t = time.perf_counter()
        s2.step(a.steps, measure=measure)
        s2.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        s2.close()
        return el

    # repeats of the whole timed region, then the same without measurement
    walls = [wall] + [rerun(True) for _ in range(a.repeats - 1)]
    wall_off = None if a.no_off else rerun(False)
    # the same again with the steps replayed from HIP graphs, against the
    # event-free reruns
    graph_leg = None
    if a.graph > 0:
        wall_graph = rerun(True, a.graph)
        plain = walls[1:] if len(walls) > 1 else [rerun(True)]
        wall_plain = float(np.median(plain))
        graph_leg = {"steps_per_graph": a.graph, "value": N * a.steps / wall_graph,
                     "value_launched": N * a.steps / wall_plain,
                     "delta": wall_plain / wall_graph - 1.0,
                     "what": "the same measured steps from the initial state, replayed from "
                             "captured graphs, against the same steps launched one by one "
                             "(both without timing events); results are bit-identical"}
        print(f"# graphs of {a.graph} steps: {wall_graph:.4f} s against {wall_plain:.4f} s "
              f"launched", file=sys.stderr, flush=True)

    alg = algorithmic_bytes(N, cells)
    dsg = design_bytes(N, cells)
    dominant = max((k for k in kt if kt[k][1] > 0), key=lambda k: kt[k][0])
    avg_ms, launches = kt[dominant]
    achieved = alg[dominant] / (avg_ms * 1e-3) / 1e9
    kernels = {k: {"avg_us": round(v[0] * 1e3, 3), "launches": v[1],
                   "alg_bytes": alg.get(k), "design_bytes": dsg.get(k, 0),
                   "GBps_alg": round(alg[k] / (v[0] * 1e-3) / 1e9, 1) if k in alg else None}
               for k, v in kt.items() if v[1] > 0 and v[0] > 0}
    print("# kernels " + json.dumps(kernels), file=sys.stderr, flush=True)
    # the committed counter summaries are of each workload's default
    # configuration only
    default_cfg = a.eta is None and a.order is None and a.D is None and a.N is None
    traffic = measured_traffic(a.workload) if dominant == "k_nbr" and default_cfg else None
    step_s = wall / a.steps
    step_gbs = alg["step"] / step_s / 1e9

    value = N * a.steps / wall
    rates = sorted(N * a.steps / w for w in walls)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (uniform isotropic initial state from Philox, seed 0)",
        "config": {"workload": describe(a.workload, cfg),
                   "N": N, "L": cfg["Lx"], "cells": [mx, my], "eta": cfg["eta"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": dominant, "avg_us": avg_ms * 1e3, "launches": launches,
                     "alg_bytes_per_launch": alg[dominant],
                     "design_bytes_per_launch": dsg[dominant],
                     "step": {"alg_bytes": alg["step"], "achieved": step_gbs,
                              "frac": step_gbs / HBM_PEAK_GBS, "target_frac": 0.6},
                     "what_bounds_it": "k_nbr: VALU issue and the latency of its per-wave "
                                       "load chain (counter summary in profiles/), not HBM "
                                       "bandwidth; k_sort: the latency of its three dependent "
                                       "memory round trips"},
        "kernels": kernels,
        "repeats": {"count": len(walls), "steps_each": a.steps,
                    "what": "the same workload rerun from its initial state (same trajectory); "
                            "the first run, which carries the timing events, is the headline",
                    "median": rates[len(rates) // 2], "min": rates[0], "max": rates[-1]},
        "graph": graph_leg,
        "measure_off": ({"value": N * a.steps / wall_off, "steps": a.steps}
                        if wall_off else None),
        "observables": {"p_mean": ob["p_mom"][0], "binder": ob["binder"],
                        "nbar_mean": ob["nbar_mom"][0]},
    }
    if cfg["rule"] == 0:
        out["paper_serial"] = PAPER_SERIAL
    return out, cfg


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 10000; vm_small 1000; langevin_walls 5000; "
                         "dram_control 1000; batch_replicas 2000)")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", choices=WORKLOADS, default="vm_large")
    ap.add_argument("--eta", type=float, default=None,
                    help="noise (vm_large default 0.4; others: the workload's)")
    ap.add_argument("--order", type=int, default=None,
                    help="interaction order o (langevin_walls only; default 1)")
    ap.add_argument("--D", type=float, default=None,
                    help="rotational diffusion D (langevin_walls only; eta = sqrt(2D); "
                         "default 0.2)")
    ap.add_argument("--N", type=int, default=None,
                    help="particles of the dram_control workload (default 2^24)")
    ap.add_argument("--time-every", type=int, default=25,
                    help="kernels of every k-th timed step carry HIP events (at most "
                         "ceil(steps / 4), so that at least four steps are sampled)")
    ap.add_argument("--graph", type=int, default=16,
                    help="steps per captured HIP graph for the graph leg (even; 0 skips it)")
    ap.add_argument("--repeats", type=int, default=3,
                    help="timed regions of --steps steps (the first is the headline)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="batch_replicas: skip the one-by-one comparison")
    ap.add_argument("--plain-steps", type=int, default=None,
                    help="batch_replicas: steps of the one-by-one comparison (default all)")
    ap.add_argument("--epochs", type=int, default=10, help="surrogate: training epochs")
    ap.add_argument("--no-batch", action="store_true",
                    help="vm_large: skip the short batched-against-one-by-one comparison")
    ap.add_argument("--no-off", action="store_true",
                    help="skip the run without measurement")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first copy this many MiB device-to-device (counter calibration)")
    ap.add_argument("--no-env", action="store_true",
                    help="skip the copy-bandwidth and environment report")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {a.gpus} is not supported "
              f"(sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    if a.steps is None:
        a.steps = {"batch_replicas": 2000, "vm_small": 1000, "langevin_walls": 5000,
                   "dram_control": 1000}.get(a.workload, 10000)
    if a.steps < 1 or a.time_every < 1 or a.repeats < 1:
        sys.exit("bench.py: --steps, --time-every and --repeats must be >= 1")
    if a.graph < 0 or a.graph % 2:
        sys.exit("bench.py: --graph must be 0 or even")

    import torch
    from paper_2211_15630_amd import binding as B

    if not os.path.exists(B.LIB_PATH):
        from __graft_entry__ import build
        build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if a.workload == "surrogate":
        run_surrogate(a)
        return
    if a.workload == "batch_replicas":
        ps = 0 if a.no_plain else a.plain_steps
        out = run_batch(a, a.steps, a.warmup, ps)
        if not a.no_env:
            out["environment"] = env_info()
        print(json.dumps(out), flush=True)
        return

    out, cfg = run_system(a)
    if not a.no_env:
        out["copy_kernel"] = copy_bandwidth()
        out["environment"] = env_info()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, a.cpu_seconds)
        out["cpu_baseline"]["cpu_model"] = out.get("environment", {}).get("cpu_model")
        print(f"# cpu baseline {out['cpu_baseline']}", file=sys.stderr, flush=True)
    if a.workload == "vm_large" and not a.no_batch:
        # the 256-replica noise sweep, batched against one by one at equal steps
        nb = copy.copy(a)
        nb.no_cpu_baseline = True
        bo = run_batch(nb, 300, 100, 300)
        out["batched"] = {"workload": bo["config"]["workload"],
                          "particles": bo["config"]["particles"], "steps": bo["steps"],
                          "batched_vs_plain": bo["batched_vs_plain"],
                          "k_nbr_b_us": bo["kernels"]["k_nbr_b"]["avg_us"],
                          "k_sort_b_us": bo["kernels"]["k_sort_b"]["avg_us"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""The learned field surrogate end to end: snapshot pairs from the particle
simulation, training, and evaluation against the simulation.

Every step runs in libaap.so (batched particle steps, coarse-graining,
network forward, backward and Adam); this module only sequences the calls
and keeps the snapshot tensors in device memory.

Workload (the defaults): standard Vicsek model, N = 4 * 2^20, L = 1024
(density 4), R = 1, v = 0.5, eta = 0.4, periodic; fields on a 128 x 128 grid
every 50 steps after a warm-up of 20000 steps; 8 training runs (seeds 0..7,
250 snapshot pairs each: 2000 pairs) and one held-out run (seed 8).  From a
uniform start these runs order slowly: the polar order is about 0.05 after
5000 steps, 0.2 after 20000 and 0.45 after 32500, so the snapshot window
(steps 20000 .. 32500) is the ordering regime, where the fields carry a
growing polarisation for the network to advance.
"""
import math
import time

import numpy as np

from . import binding as B
from . import workloads as W


def surrogate_config(N=4 << 20, L=1024.0, eta=0.4, G=128, every=50, warmup=20000,
                     pairs_per_run=250, train_runs=8, test_runs=1):
    return dict(N=N, L=L, eta=eta, G=G, every=every, warmup=warmup,
                pairs_per_run=pairs_per_run, train_runs=train_runs, test_runs=test_runs)


def generate(cfg, log=None):
    """Snapshots [runs, pairs + 1, 3, G, G] (device float32) of train_runs +
    test_runs independent runs stepped as one batch; returns (snaps, stats)."""
    import torch
    runs = cfg["train_runs"] + cfg["test_runs"]
    reps = []
    for r in range(runs):
        w = W.workload("vm_small", N=cfg["N"], Lx=cfg["L"], Ly=cfg["L"], eta=cfg["eta"], seed=r)
        reps.append(W.model_params(w))
    G = cfg["G"]
    nsnap = cfg["pairs_per_run"] + 1
    snaps = torch.empty((runs, nsnap, 3, G, G), dtype=torch.float32, device="cuda")
    b = B.Batch(reps, graph_steps=cfg["every"] if cfg["every"] % 2 == 0 else 0)
    t0 = time.perf_counter()
    try:
        b.step(1, measure=False)
        b.step(cfg["warmup"] - 1, measure=False)
        for k in range(nsnap):
            if k:
                b.step(cfg["every"], measure=False)
            for r in range(runs):
                snaps[r, k] = B.batch_fields(b, r, G)
            if log and k % 50 == 0:
                log(f"snapshot {k}/{nsnap - 1}: {time.perf_counter() - t0:.1f} s")
        b.sync()
    finally:
        b.close()
    torch.cuda.synchronize()
    return snaps, {"sim_seconds": time.perf_counter() - t0,
                   "steps": cfg["warmup"] + cfg["every"] * (nsnap - 1), "runs": runs}


def init_params(seed=0):
    """He-initialised weights, zero biases, the padding channels zero, the
    last layer scaled by 0.1 (the network starts close to persistence)."""
    g = np.random.default_rng(seed)
    out = []
    for k, (ci, co) in enumerate([(16, 32), (32, 32), (32, 32), (32, 16)]):
        fan_in = 9 * (3 if k == 0 else ci)
        w = g.normal(0.0, math.sqrt(2.0 / fan_in), (3, 3, ci, co))
        if k == 0:
            w[:, :, 3:, :] = 0.0
        if k == 3:
            w[..., 3:] = 0.0
            w *= 0.1
        out += [w.ravel(), np.zeros(co)]
    return np.concatenate(out).astype(np.float32)


def train(snaps, cfg, epochs=10, batch=16, lr=1e-3, seed=0, log=None):
    """Adam on the training runs' (t, t + every) pairs; returns (cnn, stats)."""
    import torch
    G = cfg["G"]
    rho0 = cfg["N"] / cfg["L"] ** 2
    tr = cfg["train_runs"]
    P = cfg["pairs_per_run"]
    inp = snaps[:tr, :P].reshape(tr * P, 3, G, G)
    tgt = snaps[:tr, 1:P + 1].reshape(tr * P, 3, G, G)
    cnn = B.CNN(G, batch)
    cnn.set_params(init_params(seed))
    g = np.random.default_rng(seed)
    n = inp.shape[0]
    losses = []
    t0 = time.perf_counter()
    steps = 0
    for e in range(epochs):
        order = torch.tensor(g.permutation(n), device="cuda")
        el = []
        # cosine decay of the learning rate over the run
        for s in range(0, n - batch + 1, batch):
            idx = order[s:s + batch]
            xb = inp.index_select(0, idx).contiguous()
            yb = tgt.index_select(0, idx).contiguous()
            frac = steps / max(1, epochs * (n // batch))
            el.append(cnn.train_step(xb, yb, rho0, lr * 0.5 * (1 + math.cos(math.pi * frac))))
            steps += 1
        losses.append(float(np.mean(el)))
        if log:
            log(f"epoch {e}: loss {losses[-1]:.3e} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return cnn, {"train_seconds": time.perf_counter() - t0, "adam_steps": steps,
                 "epoch_loss": losses, "pairs": n, "batch": batch}


def polar_order(f):
    """|sum p| / sum rho of fields [..., 3, G, G] (torch)."""
    import torch
    return (torch.hypot(f[..., 1, :, :].sum((-1, -2)), f[..., 2, :, :].sum((-1, -2)))
            / f[..., 0, :, :].sum((-1, -2)))


def evaluate(cnn, snaps, cfg, rollout=10):
    """On the held-out runs: mean squared error (in units of rho0^2) of the
    prediction and of persistence, and the drift of the coarse polar order
    over a rollout of `rollout` predictions from every start."""
    import torch
    G = cfg["G"]
    rho0 = cfg["N"] / cfg["L"] ** 2
    tr = cfg["train_runs"]
    test = snaps[tr:]
    P = cfg["pairs_per_run"]
    mse, per = [], []
    for r in range(test.shape[0]):
        for s in range(0, P, cnn.max_batch):
            nbat = min(cnn.max_batch, P - s)
            x = test[r, s:s + nbat].contiguous()
            y = test[r, s + 1:s + 1 + nbat]
            pr = cnn.forward(x, rho0)
            mse.append(float(((pr - y) / rho0).pow(2).mean()) * nbat)
            per.append(float(((x - y) / rho0).pow(2).mean()) * nbat)
    n = test.shape[0] * P
    starts = list(range(0, P - rollout + 1, max(1, (P - rollout) // 16)))[:16]
    drift = []
    for r in range(test.shape[0]):
        x = torch.stack([test[r, s] for s in starts]).contiguous()
        for k in range(rollout):
            x = cnn.forward(x, rho0)
        truth = torch.stack([test[r, s + rollout] for s in starts])
        drift.append((polar_order(x) - polar_order(truth)).abs().cpu().numpy())
    drift = np.concatenate(drift)
    phi_true = float(polar_order(test[:, rollout:]).mean())
    return {"mse_cnn": sum(mse) / n, "mse_persistence": sum(per) / n,
            "mse_ratio": (sum(mse) / n) / (sum(per) / n),
            "phi_drift_mean": float(drift.mean()), "phi_drift_max": float(drift.max()),
            "rollout_steps": rollout * cfg["every"], "phi_true_mean": phi_true}


def judged_rollout(cnn, truth, rho0, check_every, tol_mse, tol_phi):
    """A surrogate rollout judged by the particle simulation, which is also
    its fallback.

    truth [T + 1, 3, G, G]: fields of one particle run every `every` steps
    (the plain path).  The surrogate starts from truth[0] and advances the
    fields one prediction (`every` steps) at a time.  After every
    check_every-th prediction it is compared with the particle fields of the
    same time: when the mean squared field error (in units of rho0^2)
    exceeds tol_mse or the coarse polar order |sum p| / sum rho differs by
    more than tol_phi, the rollout hands back to the particle path -- the
    surrogate continues from the particle fields of that time.

    Returns the time means of the coarse polar order of the rollout and of
    the particle run over the T predicted times, their difference, the
    number of checks and of fallbacks, and the largest judged errors."""
    import torch
    T = truth.shape[0] - 1
    x = truth[0:1].contiguous()
    phi_s, phi_t = [], []
    checks = falls = 0
    worst_mse = worst_dphi = 0.0
    for k in range(1, T + 1):
        x = cnn.forward(x, rho0)
        ps = float(polar_order(x)[0])
        pt = float(polar_order(truth[k:k + 1])[0])
        phi_s.append(ps)
        phi_t.append(pt)
        if k % check_every == 0:
            checks += 1
            mse = float(((x[0] - truth[k]) / rho0).pow(2).mean())
            dphi = abs(ps - pt)
            worst_mse = max(worst_mse, mse)
            worst_dphi = max(worst_dphi, dphi)
            if mse > tol_mse or dphi > tol_phi:
                falls += 1
                x = truth[k:k + 1].contiguous()
    torch.cuda.synchronize()
    ms, mt = float(np.mean(phi_s)), float(np.mean(phi_t))
    return {"predictions": T, "check_every": check_every, "tol_mse": tol_mse, "tol_phi": tol_phi,
            "phi_surrogate_mean": ms, "phi_plain_mean": mt, "phi_error": abs(ms - mt),
            "checks": checks, "fallbacks": falls, "worst_judged_mse": worst_mse,
            "worst_judged_dphi": worst_dphi}


def time_forward(cnn, G, nb, reps=50):
    """Mean time of one forward of nb fields (device events on the current stream)."""
    import torch
    x = torch.rand((nb, 3, G, G), device="cuda") + 3.5
    for _ in range(5):
        cnn.forward(x, 4.0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        cnn.forward(x, 4.0)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def forward_flops(G):
    """Multiply-adds x 2 of one forward on the padded layers."""
    return 2 * G * G * 9 * (16 * 32 + 32 * 32 + 32 * 32 + 32 * 16)

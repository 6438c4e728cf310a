"""Write tests/golden/oracle_stats.json: long-run statistics of the oracle
(physics mode, binary64 state) that the GPU statistical-parity test compares
against.  Calls only the oracle package.

Recipe (one entry per parameter point, 16 seeds each, the oracle's own
uniform isotropic initial state from the seed):
  * VM, N=4096, L=64 periodic (density 1), R=1, v=0.5,
    eta in {0.2, 0.4, 0.6}; 10^4 steps, the first 2000 discarded;
  * Langevin with h(n)=1/n, Gamma=1, dt=0.1, v=0.5, reflecting walls,
    N=16384, L=64 (density 4), eta=sqrt(2D), D in {0.05, 0.2}; 3000 steps,
    the first 1000 discarded;
  * nematic Vicsek model (Eq. (3)), N=4096, L=64 periodic, R=1, v=0.5,
    eta in {0.1, 0.3}; 6000 steps, the first 2000 discarded;
  * Langevin of order 2 (Eq. (5)) with h(n)=1/n, Gamma=1, dt=0.1, v=0.5,
    periodic, N=16384, L=64, D=0.05; 3000 steps, the first 1000 discarded;
  * VM at the larger size N=65536, L=256 periodic (density 1), R=1, v=0.5,
    eta in {0.2, 0.4, 0.6}; 10^4 steps, the first 2000 discarded.
Per seed it stores the time means of p, p^2, p^4 and nbar over the kept
steps, and for the nematic points those of q, q^2, q^4 too.
Usage: python tests/golden/make_oracle_stats.py [--jobs J] [--only NAME ...]
(--only recomputes the named points and keeps the others of the file).
"""
import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "oracle_stats.json")

SEEDS = list(range(16))


def points():
    pts = []
    for eta in (0.2, 0.4, 0.6):
        pts.append(dict(name=f"vm_eta{eta}", N=4096, Lx=64.0, Ly=64.0, R=1.0, v=0.5,
                        eta=eta, rule=0, bx=0, by=0, gamma=1.0, dt=1.0,
                        weights="none", steps=10000, discard=2000))
    for D in (0.05, 0.2):
        pts.append(dict(name=f"langevin_D{D}", N=16384, Lx=64.0, Ly=64.0, R=1.0, v=0.5,
                        eta=math.sqrt(2 * D), rule=1, bx=1, by=1, gamma=1.0, dt=0.1,
                        weights="inverse_n_4096", steps=3000, discard=1000))
    for eta in (0.1, 0.3):
        pts.append(dict(name=f"nvm_eta{eta}", N=4096, Lx=64.0, Ly=64.0, R=1.0, v=0.5,
                        eta=eta, rule=2, bx=0, by=0, gamma=1.0, dt=1.0,
                        weights="none", steps=6000, discard=2000, q=True))
    pts.append(dict(name="langevin_o2_D0.05", N=16384, Lx=64.0, Ly=64.0, R=1.0, v=0.5,
                    eta=math.sqrt(2 * 0.05), rule=1, order=2, bx=0, by=0, gamma=1.0,
                    dt=0.1, weights="inverse_n_4096", steps=3000, discard=1000, q=True))
    for eta in (0.2, 0.4, 0.6):
        pts.append(dict(name=f"vm65536_eta{eta}", N=65536, Lx=256.0, Ly=256.0, R=1.0, v=0.5,
                        eta=eta, rule=0, bx=0, by=0, gamma=1.0, dt=1.0,
                        weights="none", steps=10000, discard=2000))
    return pts


def run_one(args):
    pt, seed = args
    os.environ["OMP_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    import numpy as np
    import oracle as orc
    w = None
    if pt["weights"] == "inverse_n_4096":
        w = np.zeros(4096)
        w[1:] = 1.0 / np.arange(1, 4096)
    p = orc.Params(N=pt["N"], Lx=pt["Lx"], Ly=pt["Ly"], R=pt["R"], v=pt["v"],
                   eta=pt["eta"], rule=pt["rule"], order=pt.get("order", 1), bx=pt["bx"],
                   by=pt["by"], gamma=pt["gamma"], dt=pt["dt"], seed=seed, weights=w)
    x, y, th = orc.init_state(p)
    _, _, _, m = orc.run_measured(x, y, th, p, 0, pt["steps"])
    k = pt["discard"]
    ps, ns, qs = m["p"][k:], m["nbar"][k:], m["q"][k:]
    r = dict(seed=seed, p1=float(np.mean(ps)), p2=float(np.mean(ps ** 2)),
             p4=float(np.mean(ps ** 4)), nbar=float(np.mean(ns)))
    if pt.get("q"):
        r.update(q1=float(np.mean(qs)), q2=float(np.mean(qs ** 2)), q4=float(np.mean(qs ** 4)))
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 4)
    ap.add_argument("--only", nargs="*", default=None)
    a = ap.parse_args()
    t0 = time.time()
    old = {}
    if a.only is not None and os.path.exists(OUT):
        old = {q["params"]["name"]: q for q in json.load(open(OUT))["points"]}
    out = dict(recipe=__doc__, points=[])
    with ProcessPoolExecutor(a.jobs) as ex:
        for pt in points():
            if a.only is not None and pt["name"] not in a.only and pt["name"] in old:
                out["points"].append(old[pt["name"]])
                continue
            res = list(ex.map(run_one, [(pt, s) for s in SEEDS]))
            out["points"].append(dict(params=pt, seeds=res))
            print(pt["name"], "done", round(time.time() - t0, 1), "s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()

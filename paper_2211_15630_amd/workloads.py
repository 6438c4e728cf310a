"""Workload definitions and seeded synthetic input states.

This module holds no arithmetic of the method: it only names the parameter
sets of the workloads and draws seeded synthetic particle states (numpy's
PCG64 generator) of the shapes and structures those workloads produce.  Both
the GPU tests and the oracle tests take their inputs from here.

Workloads (model parameters as in Sec. 2 of the paper; units of R):
  * ``vm_small``  -- standard Vicsek model, N=4096, periodic L=64, v=0.5,
    eta=0.3, 1000 steps with the polar order recorded every step;
  * ``vm_large``  -- standard Vicsek model, N=2^20, periodic L=1024, v=0.5,
    eta in {0.2, 0.4, 0.6}, 10^4 steps;
  * ``langevin_walls`` -- overdamped Langevin alignment with weight
    h(n)=1/n, Gamma=1, order 1, eta=sqrt(2D) for D in {0.05, 0.2}, dt=0.1,
    v=0.5, reflecting walls on both axes, N=4*2^20, L=1024, 5000 steps;
  * ``runtime_vs_n`` / ``runtime_vs_rho`` -- the run-time scans of Sec. 5.2
    (Fig. 7): R=1, v=1, eta=0.45 at density 0.6366, and eta=0.85 at N=10^5;
  * ``nvm_large`` -- nematic Vicsek model with the parameters of the NVM
    snapshots of Sec. 5 (N=524288, R=1, v=0.5, eta=0.065, omega=0); the box
    side is not printed there: periodic L=512 (density 2);
  * ``nvm_small`` -- the same model at N=8192, L=64 (density 2);
  * ``langevin_nematic`` -- the Langevin workload at order o=2 (nematic
    alignment, Eq. (5)), N=16384, L=64, periodic, D=0.05;
  * ``batch_replicas`` -- a noise sweep across the transition as one batch:
    256 standard-Vicsek replicas, N log-uniform in [1024, 65536], density
    uniform in [0.25, 4] (L = sqrt(N / density)), eta spaced uniformly over
    [0.1, 0.7], R=1, v=0.5, periodic, one seed, replica index r.
"""
import math

import numpy as np

RULE_VM = 0
RULE_LANGEVIN = 1
RULE_NVM = 2


def inverse_n_weights(length=4096):
    """Weight table h(n) = 1/n for n >= 1 and h(0) = 0 (n < length).

    The paper tabulates the weight function once for n = 0..len-1 and uses
    the last entry beyond the table (Sec. 4).
    """
    h = np.zeros(length, dtype=np.float64)
    h[1:] = 1.0 / np.arange(1, length, dtype=np.float64)
    return h


def workload(name, **over):
    """Parameter dict for a named workload (keyword names of Sec. 4)."""
    base = dict(R=1.0, omega=0.0, gamma=1.0, dt=1.0, order=1, bx=0, by=0,
                seed=0, weights=None, replica=0)
    if name == "vm_small":
        base.update(N=4096, Lx=64.0, Ly=64.0, v=0.5, eta=0.3, rule=RULE_VM,
                    steps=1000)
    elif name == "vm_large":
        base.update(N=1 << 20, Lx=1024.0, Ly=1024.0, v=0.5, eta=0.4,
                    rule=RULE_VM, steps=10000)
    elif name == "langevin_walls":
        D = over.pop("D", 0.2)
        base.update(N=4 << 20, Lx=1024.0, Ly=1024.0, v=0.5,
                    eta=math.sqrt(2.0 * D), rule=RULE_LANGEVIN, gamma=1.0,
                    dt=0.1, bx=1, by=1, weights=inverse_n_weights(),
                    steps=5000)
    elif name == "runtime_vs_n":
        N = over.pop("N", 1 << 16)
        L = math.sqrt(N / 0.6366)
        base.update(N=N, Lx=L, Ly=L, v=1.0, eta=0.45, rule=RULE_VM,
                    steps=10000)
    elif name == "runtime_vs_rho":
        rho = over.pop("rho", 1.0)
        N = over.pop("N", 100000)
        L = math.sqrt(N / rho)
        base.update(N=N, Lx=L, Ly=L, v=1.0, eta=0.85, rule=RULE_VM,
                    steps=10000)
    elif name == "nvm_large":
        base.update(N=1 << 19, Lx=512.0, Ly=512.0, v=0.5, eta=0.065,
                    rule=RULE_NVM, steps=10000)
    elif name == "nvm_small":
        base.update(N=8192, Lx=64.0, Ly=64.0, v=0.5, eta=0.065,
                    rule=RULE_NVM, steps=1000)
    elif name == "langevin_nematic":
        D = over.pop("D", 0.05)
        base.update(N=16384, Lx=64.0, Ly=64.0, v=0.5, eta=math.sqrt(2.0 * D),
                    rule=RULE_LANGEVIN, order=2, gamma=1.0, dt=0.1,
                    weights=inverse_n_weights(), steps=5000)
    else:
        raise KeyError(name)
    base.update(over)
    return base


def model_params(cfg):
    """The subset of a workload dict that parametrises the model."""
    keys = ("N", "Lx", "Ly", "R", "v", "eta", "omega", "gamma", "dt", "rule",
            "order", "bx", "by", "seed", "weights", "replica")
    return {k: cfg[k] for k in keys}


# ---------------------------------------------------------------------------
# Synthetic states (float32, arrays indexed by particle id)
# ---------------------------------------------------------------------------
def _finish(x, y, th, Lx, Ly, bx, by):
    x = x.astype(np.float32)
    y = y.astype(np.float32)
    th = th.astype(np.float32)
    Lxf, Lyf = np.float32(Lx), np.float32(Ly)
    # keep every coordinate inside the box of its boundary type
    if bx:
        x = np.clip(x, np.float32(0), Lxf)
    else:
        x = np.where(x >= Lxf, np.float32(0), np.where(x < 0, np.float32(0), x))
    if by:
        y = np.clip(y, np.float32(0), Lyf)
    else:
        y = np.where(y >= Lyf, np.float32(0), np.where(y < 0, np.float32(0), y))
    pi32 = np.float32(np.pi)
    th = np.where(th >= pi32, -pi32, th)
    th = np.where(th < -pi32, -pi32, th)
    return np.ascontiguousarray(x), np.ascontiguousarray(y), np.ascontiguousarray(th)


def uniform_state(N, Lx, Ly, seed, bx=0, by=0):
    """Uniform positions and isotropic orientations."""
    g = np.random.default_rng(seed)
    x = g.random(N) * Lx
    y = g.random(N) * Ly
    th = (g.random(N) * 2.0 - 1.0) * np.pi
    return _finish(x, y, th, Lx, Ly, bx, by)


def banded_state(N, Lx, Ly, seed, bx=0, by=0, bands=3, width=None,
                 frac_in_bands=0.7, spread=0.3):
    """Travelling-band-like structure: dense stripes normal to x, polar
    order along x inside the stripes, a disordered gas outside."""
    g = np.random.default_rng(seed)
    width = width if width is not None else max(Lx / (8.0 * bands), 1.0)
    nb = int(N * frac_in_bands)
    centres = (np.arange(bands) + 0.5) * Lx / bands
    which = g.integers(0, bands, nb)
    xb = centres[which] + g.normal(0.0, width, nb)
    xb = np.mod(xb, Lx)
    xg = g.random(N - nb) * Lx
    x = np.concatenate([xb, xg])
    y = g.random(N) * Ly
    thb = g.normal(0.0, spread, nb)
    thg = (g.random(N - nb) * 2.0 - 1.0) * np.pi
    th = np.concatenate([thb, thg])
    th = np.mod(th + np.pi, 2 * np.pi) - np.pi
    perm = g.permutation(N)
    return _finish(x[perm], y[perm], th[perm], Lx, Ly, bx, by)


def clustered_state(N, Lx, Ly, seed, bx=0, by=0, clusters=8, sigma=1.5,
                    frac=0.5):
    """Dense Gaussian clusters on a uniform background: cells far above the
    mean occupancy."""
    g = np.random.default_rng(seed)
    nc = int(N * frac)
    cx = g.random(clusters) * Lx
    cy = g.random(clusters) * Ly
    which = g.integers(0, clusters, nc)
    x = np.concatenate([cx[which] + g.normal(0, sigma, nc), g.random(N - nc) * Lx])
    y = np.concatenate([cy[which] + g.normal(0, sigma, nc), g.random(N - nc) * Ly])
    x = np.mod(x, Lx) if not bx else np.clip(x, 0, Lx)
    y = np.mod(y, Ly) if not by else np.clip(y, 0, Ly)
    th = (g.random(N) * 2.0 - 1.0) * np.pi
    perm = g.permutation(N)
    return _finish(x[perm], y[perm], th[perm], Lx, Ly, bx, by)


def aligned_state(N, Lx, Ly, seed, angle=0.7, bx=0, by=0):
    """Uniform positions, every orientation equal."""
    g = np.random.default_rng(seed)
    x = g.random(N) * Lx
    y = g.random(N) * Ly
    th = np.full(N, angle)
    return _finish(x, y, th, Lx, Ly, bx, by)


def edge_state(N, Lx, Ly, seed, cell_x, cell_y, R=1.0, bx=0, by=0):
    """Adversarial placements: coordinates on cell edges, on the walls
    (0 and L), pairs at exactly representable distance R, pairs whose
    distance rounds to R, plus a uniform filler.  ``cell_x``/``cell_y`` are
    the cell sides to place particles on."""
    g = np.random.default_rng(seed)
    pts = []
    Mx = int(round(Lx / cell_x))
    My = int(round(Ly / cell_y))
    k = max(N // 6, 1)
    # on cell edges
    ex = np.float32(cell_x) * g.integers(0, Mx, k).astype(np.float32)
    ey = np.float32(cell_y) * g.integers(0, My, k).astype(np.float32)
    pts.append((ex, g.random(k) * Ly))
    pts.append((g.random(k) * Lx, ey))
    # on the walls / box edges
    wall = np.array([0.0, Lx if bx else 0.0], dtype=np.float64)
    pts.append((wall[g.integers(0, 2, k)], g.random(k) * Ly))
    wally = np.array([0.0, Ly if by else 0.0], dtype=np.float64)
    pts.append((g.random(k) * Lx, wally[g.integers(0, 2, k)]))
    # exact-distance pairs along an axis (half-integers are exact in binary)
    h = k // 2
    ax = np.floor(g.random(h) * (Lx - 2 * R)) + 0.5
    ay = np.floor(g.random(h) * Ly) + 0.25
    pts.append((np.concatenate([ax, ax + R]), np.concatenate([ay, ay])))
    # 3-4-5 pairs: distance rounds to R
    bx0 = g.random(h) * (Lx - 2 * R)
    by0 = g.random(h) * (Ly - 2 * R)
    pts.append((np.concatenate([bx0, bx0 + 0.6 * R]),
                np.concatenate([by0, by0 + 0.8 * R])))
    x = np.concatenate([p[0] for p in pts])
    y = np.concatenate([p[1] for p in pts])
    if len(x) < N:
        x = np.concatenate([x, g.random(N - len(x)) * Lx])
        y = np.concatenate([y, g.random(N - len(y)) * Ly])
    x, y = x[:N], y[:N]
    th = (g.random(N) * 2.0 - 1.0) * np.pi
    perm = g.permutation(N)
    return _finish(x[perm], y[perm], th[perm], Lx, Ly, bx, by)


def quarter_turn_pairs(Lx, Ly, seed, bx=0, by=0, R=1.0):
    """Isolated pairs of particles (sites 3R apart, partners 0.5R apart)
    whose orientations differ by a quarter or three quarters of a turn to
    within a few binary32 ulps: the pairs on which the nematic rule's sign
    (Eq. (3)) is hardest to decide.  Next to a reflecting wall the pairs sit
    0.2R and 0.5R from it, so that the partner's mirror image is a
    neighbour, and the angles put that image's orientation (pi - theta for
    an x wall, -theta for a y wall) a quarter turn away instead.  Returns
    float32 (x, y, theta) with N = 2 * sites."""
    g = np.random.default_rng(seed)
    f32 = np.float32
    sx = np.arange(1.5 * R, Lx - 1.5 * R, 3.0 * R)
    sy = np.arange(1.5 * R, Ly - 1.5 * R, 3.0 * R)
    X, Y = np.meshgrid(sx, sy)
    X, Y = X.ravel(), Y.ravel()
    n = len(X)
    wall = np.zeros(n, dtype=np.int64)   # 0 none, 1 x wall at 0, 2 y wall at 0
    xi, yi = X.copy(), Y.copy()
    xj, yj = X + 0.3 * R, Y + 0.4 * R
    if bx:
        m = X == sx[0]
        xi[m], xj[m], yj[m] = 0.2 * R, 0.5 * R, Y[m]
        wall[m] = 1
    if by:
        m = (Y == sy[0]) & (wall == 0)
        yi[m], yj[m], xj[m] = 0.2 * R, 0.5 * R, X[m]
        wall[m] = 2
    ti = g.uniform(-np.pi, np.pi, n)
    k = g.choice(np.array([-3, -1, 1, 3]), n)
    # the partner's (image) orientation a quarter turn (or three) from ti
    tgt = ti + k * (np.pi / 2)
    tj = np.where(wall == 1, np.pi - tgt, np.where(wall == 2, -tgt, tgt))
    tj = np.mod(tj + np.pi, 2 * np.pi) - np.pi
    tj32 = tj.astype(f32)
    steps = g.integers(-2, 3, n)
    for s in (-2, -1, 1, 2):
        sel = steps == s
        d = np.sign(s)
        for _ in range(abs(s)):
            tj32[sel] = np.nextafter(tj32[sel], f32(4 * d))
    x = np.empty(2 * n)
    y = np.empty(2 * n)
    th = np.empty(2 * n)
    x[0::2], x[1::2] = xi, xj
    y[0::2], y[1::2] = yi, yj
    th[0::2], th[1::2] = ti.astype(f32), tj32
    return _finish(x, y, th, Lx, Ly, bx, by)


def batch_replicas(count=256, seed=0, rng_seed=1, eta_lo=0.1, eta_hi=0.7):
    """Parameter dicts of the replica batch (see the module docstring): the
    sizes and densities are drawn with numpy's PCG64 from rng_seed, the
    noise values are spaced uniformly over [eta_lo, eta_hi] in replica
    order."""
    g = np.random.default_rng(rng_seed)
    N = np.rint(np.exp(g.uniform(math.log(1024), math.log(65536), count))).astype(np.int64)
    rho = g.uniform(0.25, 4.0, count)
    eta = np.linspace(eta_lo, eta_hi, count) if count > 1 else np.array([eta_lo])
    out = []
    for r in range(count):
        L = math.sqrt(N[r] / rho[r])
        cfg = workload("vm_small", N=int(N[r]), Lx=L, Ly=L, eta=float(eta[r]), seed=seed,
                       replica=r)
        cfg["density"] = float(rho[r])
        out.append(cfg)
    return out

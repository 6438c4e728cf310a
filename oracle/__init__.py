"""Double-precision CPU oracle for the metric Vicsek-class step (test only).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  It is independent of the GPU
library: it shares no source, header, table or helper with it.

The arithmetic lives in ``aap_oracle.c`` (binary64, no FP contraction).  This
module adds the parts whose plain definition is a library primitive:
  * the cell-list bin of every particle is ``orc_cell_keys``;
  * the per-cell counts are a histogram (``numpy.bincount``) and the cell
    starts its exclusive prefix sum, as the per-cell lists of Sec. 3.2;
  * the order of the binned particles is a stable sort by (cell, id);
  * the moments of p and of the mean neighbour number of Sec. 3.4 and the
    Binder cumulant of Fig. 5.

Pins (tests that fix the oracle against something other than itself) are in
``tests/test_oracle_*.py``.  The generator's bit stream is pinned to an
independent implementation of Philox4x32-10 (rocRAND's engine, built from its
headers for the host); its statistics and its Weyl constants are pinned too.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build_oracle

RULE_VM = 0
RULE_LANGEVIN = 1
RULE_NVM = 2

_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_int = ctypes.c_int
_dbl = ctypes.c_double
_p = ctypes.c_void_p


class _Params(ctypes.Structure):
    _fields_ = [
        ("Lx", _dbl), ("Ly", _dbl), ("R", _dbl), ("v", _dbl), ("eta", _dbl),
        ("omega", _dbl), ("gamma", _dbl), ("dt", _dbl),
        ("rule", _int), ("order", _int), ("bx", _int), ("by", _int),
        ("seed", _u64), ("weights", _p), ("weight_len", _int), ("replica", _u32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = ctypes.CDLL(LIB)
        L.orc_philox4x32.argtypes = [_p, _p, _int, _p]
        L.orc_philox_constants.argtypes = [_p]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_philox_batch.argtypes = [_u64, _p, _i64, _u64, _u32, _u32, _p]
        L.orc_cells_per_axis.argtypes = [_dbl, _dbl]
        L.orc_cells_per_axis.restype = _int
        L.orc_wrap_angle_export.argtypes = [_dbl]
        L.orc_wrap_angle_export.restype = _dbl
        L.orc_cell_keys.argtypes = [_i64, _p, _p, _dbl, _dbl, _dbl, _p]
        L.orc_neighbours_brute.argtypes = [
            _i64, _p, _p, _p, _dbl, _dbl, _dbl, _int, _int, _int, _int, _p, _i64,
            _p, _p, _p, _p]
        L.orc_neighbours_cells.argtypes = [
            _i64, _p, _p, _p, _dbl, _dbl, _dbl, _int, _int, _int, _int,
            _p, _p, _p, _p]
        L.orc_nvm_sign.argtypes = [_dbl, _dbl, _int, _int]
        L.orc_nvm_sign.restype = _int
        L.orc_noise_vm.argtypes = [_u64, _u32, _u64]
        L.orc_noise_vm.restype = _dbl
        L.orc_noise_gauss.argtypes = [_u64, _u32, _u64]
        L.orc_noise_gauss.restype = _dbl
        L.orc_update.argtypes = [_i64, ctypes.POINTER(_Params), _u64, _p,
                                 _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]
        L.orc_init.argtypes = [_i64, _dbl, _dbl, _int, _int, _u64, _u32, _p, _p, _p]
        L.orc_state_observables.argtypes = [_i64, _p, _p, _p, _p, _p]
        L.orc_histograms.argtypes = [_i64, _p, _p, _int, _int, _p, _p]
        L.orc_run.argtypes = [_i64, ctypes.POINTER(_Params), _u64, _i64,
                              _p, _p, _p, _p, _p, _p, _int, _int, _p, _p]
        L.orc_run.restype = _int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Parameters (the keyword names of the paper's aappp_init, Sec. 4)
# --------------------------------------------------------------------------
class Params:
    """Model parameters; names follow the keyword arguments of Sec. 4."""

    def __init__(self, N, Lx, Ly, R=1.0, v=0.5, eta=0.3, omega=0.0,
                 gamma=1.0, dt=1.0, rule=RULE_VM, order=1, bx=0, by=0,
                 seed=0, weights=None, replica=0):
        self.N = int(N)
        self.Lx, self.Ly, self.R = float(Lx), float(Ly), float(R)
        self.v, self.eta, self.omega = float(v), float(eta), float(omega)
        self.gamma, self.dt = float(gamma), float(dt)
        self.rule, self.order = int(rule), int(order)
        self.bx, self.by = int(bx), int(by)
        self.seed = int(seed)
        self.weights = None if weights is None else _f64(weights)
        self.replica = int(replica)

    def c_struct(self):
        s = _Params()
        for k in ("Lx", "Ly", "R", "v", "eta", "omega", "gamma", "dt",
                  "rule", "order", "bx", "by", "seed", "replica"):
            setattr(s, k, getattr(self, k))
        if self.weights is not None:
            s.weights = self.weights.ctypes.data_as(_p).value
            s.weight_len = len(self.weights)
        else:
            s.weights = None
            s.weight_len = 0
        return s


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------
def philox4x32(ctr, key, rounds=10):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32(_ptr(c), _ptr(k), int(rounds), _ptr(out))
    return out


def set_threads(n):
    """Threads of the oracle's OpenMP loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads():
    return int(lib().orc_max_threads())


def philox_constants():
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox_constants(_ptr(out))
    return out


def philox_batch(seed, ids, step, replica, purpose):
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    out = np.zeros((len(ids), 4), dtype=np.uint32)
    lib().orc_philox_batch(int(seed), _ptr(ids), len(ids), int(step),
                           int(replica), int(purpose), _ptr(out))
    return out


def noise_vm(seed, pid, t):
    return lib().orc_noise_vm(int(seed), int(pid), int(t))


def noise_gauss(seed, pid, t):
    return lib().orc_noise_gauss(int(seed), int(pid), int(t))


# --------------------------------------------------------------------------
# Geometry and the cell-list binning
# --------------------------------------------------------------------------
def cells_per_axis(L, R):
    return lib().orc_cells_per_axis(float(L), float(R))


def wrap_angle(th):
    return lib().orc_wrap_angle_export(float(th))


def cell_keys(x, y, Lx, Ly, R):
    x, y = _f64(x), _f64(y)
    key = np.zeros(len(x), dtype=np.uint32)
    lib().orc_cell_keys(len(x), _ptr(x), _ptr(y), float(Lx), float(Ly),
                        float(R), _ptr(key))
    return key


def cell_lists(key, ncells):
    """Per-cell counts, exclusive starts (ncells+1) and the particle order.

    The order lists the particles cell by cell and, within a cell, by
    ascending id: a stable sort by cell of the id-ordered particle list.
    """
    key = np.asarray(key, dtype=np.int64)
    count = np.bincount(key, minlength=ncells).astype(np.uint32)
    start = np.zeros(ncells + 1, dtype=np.int64)
    np.cumsum(count, out=start[1:])
    order = np.argsort(key, kind="stable").astype(np.uint32)
    return count, start.astype(np.uint32), order


# --------------------------------------------------------------------------
# Neighbour sums
# --------------------------------------------------------------------------
def neighbours_brute(x, y, th, p: Params, idx=None):
    x, y, th = _f64(x), _f64(y), _f64(th)
    N = len(x)
    idx = np.arange(N, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    m = len(idx)
    n = np.zeros(m, dtype=np.int64)
    C, S, A = (np.zeros(m) for _ in range(3))
    lib().orc_neighbours_brute(N, _ptr(x), _ptr(y), _ptr(th), p.Lx, p.Ly, p.R,
                               p.bx, p.by, p.rule, p.order, _ptr(idx), m,
                               _ptr(n), _ptr(C), _ptr(S), _ptr(A))
    return n, C, S, A


def neighbours_cells(x, y, th, p: Params):
    x, y, th = _f64(x), _f64(y), _f64(th)
    N = len(x)
    n = np.zeros(N, dtype=np.int64)
    C, S, A = (np.zeros(N) for _ in range(3))
    lib().orc_neighbours_cells(N, _ptr(x), _ptr(y), _ptr(th), p.Lx, p.Ly, p.R,
                               p.bx, p.by, p.rule, p.order,
                               _ptr(n), _ptr(C), _ptr(S), _ptr(A))
    return n, C, S, A


def nvm_sign(thi, thj, mirror_x=False, mirror_y=False):
    """sign(cos(th_i - th~_j)) of Eq. (3) for the image of j (sign(0) = +1)."""
    return lib().orc_nvm_sign(float(thi), float(thj), int(bool(mirror_x)), int(bool(mirror_y)))


# --------------------------------------------------------------------------
# Steps
# --------------------------------------------------------------------------
def update(x, y, th, n, C, S, A, p: Params, t, ids=None):
    """Apply the update rule to every particle given its neighbour sums."""
    x, y, th = _f64(x).copy(), _f64(y).copy(), _f64(th).copy()
    N = len(x)
    ids = np.arange(N, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
    n = np.ascontiguousarray(n, dtype=np.int64)
    C, S, A = _f64(C), _f64(S), _f64(A)
    ps = p.c_struct()
    lib().orc_update(N, ctypes.byref(ps), int(t), _ptr(ids), _ptr(x), _ptr(y),
                     _ptr(th), _ptr(n), _ptr(C), _ptr(S), _ptr(A),
                     _ptr(x), _ptr(y), _ptr(th))
    return x, y, th


def step(x, y, th, p: Params, t, ids=None):
    """One full step t -> t+1 from the given state (arrays in id order)."""
    n, C, S, A = neighbours_cells(x, y, th, p)
    xn, yn, tn = update(x, y, th, n, C, S, A, p, t, ids)
    return xn, yn, tn, n, C, S, A


def init_state(p: Params):
    N = p.N
    x, y, th = np.zeros(N), np.zeros(N), np.zeros(N)
    lib().orc_init(N, p.Lx, p.Ly, p.bx, p.by, p.seed, p.replica, _ptr(x), _ptr(y), _ptr(th))
    return x, y, th


def state_observables(th, n):
    """(p, nbar, q) of one state (Sec. 3.4)."""
    th = _f64(th)
    n = np.ascontiguousarray(n, dtype=np.int64)
    pv, nv, qv = _dbl(), _dbl(), _dbl()
    lib().orc_state_observables(len(th), _ptr(th), _ptr(n),
                                ctypes.byref(pv), ctypes.byref(nv), ctypes.byref(qv))
    return pv.value, nv.value, qv.value


def histograms(th, n, bt, bn):
    """Counts of one state in bt angle bins and bn neighbour-number bins."""
    th = _f64(th)
    n = np.ascontiguousarray(n, dtype=np.int64)
    ht = np.zeros(bt, np.int64)
    hn = np.zeros(bn, np.int64)
    lib().orc_histograms(len(th), _ptr(th), _ptr(n), int(bt), int(bn), _ptr(ht), _ptr(hn))
    return ht, hn


def run(x, y, th, p: Params, t0, nsteps, measure=True):
    """nsteps physics-mode steps in place; returns the p and nbar series."""
    x, y, th, m = run_measured(x, y, th, p, t0, nsteps, measure=measure)
    return x, y, th, m.get("p"), m.get("nbar")


def run_measured(x, y, th, p: Params, t0, nsteps, measure=True, bins=None):
    """nsteps physics-mode steps; returns (x, y, th, results) with the p,
    nbar and q series of the measured states and, when bins = (bt, bn), the
    histogram counts of all measured states."""
    x, y, th = _f64(x).copy(), _f64(y).copy(), _f64(th).copy()
    ps_ = np.zeros(nsteps) if measure else None
    ns_ = np.zeros(nsteps) if measure else None
    qs_ = np.zeros(nsteps) if measure else None
    bt, bn = bins if (measure and bins) else (0, 0)
    ht = np.zeros(bt, np.int64) if bt else None
    hn = np.zeros(bn, np.int64) if bn else None
    pc = p.c_struct()
    rc = lib().orc_run(len(x), ctypes.byref(pc), int(t0), int(nsteps),
                       _ptr(x), _ptr(y), _ptr(th), _ptr(ps_), _ptr(ns_), _ptr(qs_),
                       int(bt), int(bn), _ptr(ht), _ptr(hn))
    if rc != 0:
        raise MemoryError("oracle run failed")
    res = {}
    if measure:
        res.update(p=ps_, nbar=ns_, q=qs_)
    if bt:
        res.update(hist_theta=ht, hist_n=hn)
    return x, y, th, res


def moments(series):
    """First four raw moments of a measured series (Sec. 3.4, normalised)."""
    s = np.asarray(series, dtype=np.float64)
    return np.array([np.mean(s ** k) for k in (1, 2, 3, 4)])


def binder(p_moments):
    """U = 1 - <p^4> / (3 <p^2>^2), Fig. 5."""
    return 1.0 - p_moments[3] / (3.0 * p_moments[1] ** 2)

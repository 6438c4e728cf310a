"""Thin ctypes binding of libaap.so (include/aap.h).

Every function of the C ABI has a Python function of the same name here that
only marshals arguments; all computation happens in the library's HIP
kernels.  PyTorch provides the device workspace (a uint8 tensor) and the HIP
stream.  There is no fallback: if the library is not built, loading raises.

``Sim`` is a convenience wrapper that owns a workspace tensor and a handle;
its keyword names follow the paper's ``aappp_init`` (Sec. 4).
"""
import ctypes
import os

import numpy as np

# AAP_LIB selects another build of the same sources (the host-sanitizer
# check loads libaap_san.so this way)
LIB_PATH = os.environ.get("AAP_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                     "libaap.so")

AAP_OK = 0
AAP_EINVAL = -1
AAP_ENOMEM = -2
AAP_EHIP = -3
AAP_RULE_VM = 0
AAP_RULE_LANGEVIN = 1
AAP_RULE_NVM = 2

_c_int = ctypes.c_int
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_dbl = ctypes.c_double
_p = ctypes.c_void_p


class aap_params(ctypes.Structure):
    _fields_ = [
        ("N", _u64), ("Lx", _dbl), ("Ly", _dbl), ("R", _dbl),
        ("v", _dbl), ("eta", _dbl), ("omega", _dbl), ("gamma", _dbl),
        ("dt", _dbl), ("rule", _i32), ("order", _i32), ("bx", _i32),
        ("by", _i32), ("seed", _u64), ("weights", ctypes.POINTER(_dbl)),
        ("weight_len", _i32), ("bins_theta", _i32), ("bins_n", _i32), ("replica", ctypes.c_uint32),
    ]


class aap_observables_t(ctypes.Structure):
    _fields_ = [
        ("steps_measured", _i64), ("p_mom", _dbl * 4), ("nbar_mom", _dbl * 4),
        ("binder", _dbl), ("p_last", _dbl), ("nbar_last", _dbl),
        ("q_mom", _dbl * 4), ("q_last", _dbl),
    ]


class AapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"aap error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libaap.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_2211_15630_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.aap_params_default.restype = aap_params
        L.aap_params_default.argtypes = []
        L.aap_workspace_bytes.argtypes = [P(aap_params), P(ctypes.c_size_t)]
        L.aap_create.argtypes = [P(aap_params), _p, ctypes.c_size_t, _p, P(_p)]
        L.aap_destroy.argtypes = [_p]
        L.aap_step.argtypes = [_p, _i64, _c_int, P(_dbl)]
        L.aap_graph.argtypes = [_p, _i32]
        L.aap_observables.argtypes = [_p, P(aap_observables_t)]
        L.aap_reset_observables.argtypes = [_p]
        L.aap_get_state.argtypes = [_p, _p, _p, _p, P(_u64)]
        L.aap_set_state.argtypes = [_p, _p, _p, _p, _u64]
        L.aap_sync.argtypes = [_p]
        L.aap_debug_keys.argtypes = [_p, _p, P(_i32), P(_i32)]
        L.aap_debug_enable.argtypes = [_p, _c_int]
        L.aap_debug_last_step.argtypes = [_p, _p, _p, _p, _p, _p]
        L.aap_timing_enable.argtypes = [_p, _c_int]
        L.aap_timing_read.argtypes = [_p, P(ctypes.c_char_p), P(_dbl), P(_i64), P(_i32)]
        L.aap_histograms.argtypes = [_p, _p, _i32, _p, _i32]
        L.aap_checkpoint_bytes.argtypes = [_p, P(ctypes.c_size_t)]
        L.aap_checkpoint_save.argtypes = [_p, _p, ctypes.c_size_t]
        L.aap_checkpoint_load.argtypes = [_p, _p, ctypes.c_size_t]
        L.aap_batch_workspace_bytes.argtypes = [_p, _i32, P(ctypes.c_size_t)]
        L.aap_batch_create.argtypes = [_p, _i32, _p, ctypes.c_size_t, _p, P(_p)]
        L.aap_batch_destroy.argtypes = [_p]
        L.aap_batch_graph.argtypes = [_p, _i32]
        L.aap_batch_step.argtypes = [_p, _i64, _c_int]
        L.aap_batch_sync.argtypes = [_p]
        L.aap_batch_observables.argtypes = [_p, _p, _i32]
        L.aap_batch_reset_observables.argtypes = [_p]
        L.aap_batch_get_state.argtypes = [_p, _i32, _p, _p, _p, P(_u64)]
        L.aap_batch_threads.argtypes = [_p, _i32]
        L.aap_batch_kernel_times.argtypes = [_p, _i32, _c_int, P(_dbl), P(_dbl)]
        L.aap_batch_autotune.argtypes = [_p, _i32, _c_int, P(_i32), P(_i32)]
        L.aap_batch_debug_enable.argtypes = [_p, _c_int]
        L.aap_batch_debug_keys.argtypes = [_p, _i32, _p, P(_i32), P(_i32)]
        L.aap_batch_debug_last_step.argtypes = [_p, _i32, _p, _p, _p, _p, _p]
        L.aap_fields_scratch_bytes.argtypes = [_i32, P(ctypes.c_size_t)]
        L.aap_fields.argtypes = [_p, _i32, _p, _p, ctypes.c_size_t]
        L.aap_batch_fields.argtypes = [_p, _i32, _i32, _p, _p, ctypes.c_size_t]
        L.aap_fields_noalloc.argtypes = [_p, _i32, _p]
        L.aap_cnn_param_count.argtypes = []
        L.aap_cnn_param_count.restype = ctypes.c_size_t
        L.aap_cnn_workspace_bytes.argtypes = [_i32, _i32, P(ctypes.c_size_t)]
        L.aap_cnn_create.argtypes = [_i32, _i32, _p, ctypes.c_size_t, _p, P(_p)]
        L.aap_cnn_destroy.argtypes = [_p]
        L.aap_cnn_set_params.argtypes = [_p, _p, ctypes.c_size_t]
        L.aap_cnn_get_params.argtypes = [_p, _p, ctypes.c_size_t]
        L.aap_cnn_forward.argtypes = [_p, _p, _i32, _dbl, _p]
        L.aap_cnn_train_step.argtypes = [_p, _p, _p, _i32, _dbl, ctypes.c_float, P(_dbl)]
        L.aap_cnn_debug_read.argtypes = [_p, _i32, _p, ctypes.c_size_t]
        L.aap_last_error.restype = ctypes.c_char_p
        L.aap_last_error.argtypes = []
        for name in ("aap_workspace_bytes", "aap_create", "aap_destroy", "aap_step",
                     "aap_observables", "aap_reset_observables", "aap_get_state",
                     "aap_set_state", "aap_sync", "aap_debug_keys", "aap_debug_enable",
                     "aap_debug_last_step", "aap_timing_enable", "aap_timing_read",
                     "aap_histograms", "aap_checkpoint_bytes", "aap_checkpoint_save",
                     "aap_checkpoint_load", "aap_batch_workspace_bytes", "aap_batch_create",
                     "aap_batch_destroy", "aap_batch_graph", "aap_batch_step", "aap_batch_sync",
                     "aap_batch_observables", "aap_batch_reset_observables",
                     "aap_batch_get_state", "aap_batch_threads", "aap_batch_kernel_times",
                     "aap_batch_autotune", "aap_batch_debug_enable", "aap_batch_debug_keys",
                     "aap_batch_debug_last_step", "aap_fields_scratch_bytes", "aap_fields",
                     "aap_batch_fields", "aap_fields_noalloc", "aap_cnn_workspace_bytes",
                     "aap_cnn_create",
                     "aap_cnn_destroy", "aap_cnn_set_params", "aap_cnn_get_params",
                     "aap_cnn_forward", "aap_cnn_train_step", "aap_cnn_debug_read"):
            getattr(L, name).restype = _c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != AAP_OK:
        raise AapError(rc, load().aap_last_error().decode(errors="replace"))
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_p)


# ---------------------------------------------------------------------------
# one function per C entry point
# ---------------------------------------------------------------------------
def aap_params_default():
    return load().aap_params_default()


def aap_workspace_bytes(p):
    n = ctypes.c_size_t()
    _check(load().aap_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def aap_create(p, d_workspace, nbytes, hip_stream):
    h = _p()
    _check(load().aap_create(ctypes.byref(p), _p(d_workspace), nbytes,
                             _p(hip_stream), ctypes.byref(h)))
    return h


def aap_destroy(h):
    _check(load().aap_destroy(h))


def aap_step(h, nsteps, measure=0, p_series=None):
    ptr = None if p_series is None else p_series.ctypes.data_as(ctypes.POINTER(_dbl))
    _check(load().aap_step(h, int(nsteps), int(measure), ptr))


def aap_graph(h, steps_per_graph):
    _check(load().aap_graph(h, int(steps_per_graph)))


def aap_observables(h):
    o = aap_observables_t()
    _check(load().aap_observables(h, ctypes.byref(o)))
    return o


def aap_reset_observables(h):
    _check(load().aap_reset_observables(h))


def aap_get_state(h, x, y, theta):
    st = _u64()
    _check(load().aap_get_state(h, _ptr(x), _ptr(y), _ptr(theta), ctypes.byref(st)))
    return st.value


def aap_set_state(h, x, y, theta, step):
    _check(load().aap_set_state(h, _ptr(x), _ptr(y), _ptr(theta), int(step)))


def aap_sync(h):
    _check(load().aap_sync(h))


def aap_debug_keys(h, key):
    mx, my = _i32(), _i32()
    _check(load().aap_debug_keys(h, _ptr(key), ctypes.byref(mx), ctypes.byref(my)))
    return mx.value, my.value


def aap_debug_enable(h, on):
    _check(load().aap_debug_enable(h, int(on)))


def aap_debug_last_step(h, start, order, n, C, S):
    _check(load().aap_debug_last_step(h, _ptr(start), _ptr(order), _ptr(n), _ptr(C), _ptr(S)))


def aap_timing_enable(h, every):
    _check(load().aap_timing_enable(h, int(every)))


def aap_timing_read(h):
    cnt = _i32(16)
    names = (ctypes.c_char_p * 16)()
    ms = (_dbl * 16)()
    launches = (_i64 * 16)()
    _check(load().aap_timing_read(h, names, ms, launches, ctypes.byref(cnt)))
    return {names[k].decode(): (ms[k], launches[k]) for k in range(cnt.value)}


def aap_histograms(h, theta_hist, n_hist):
    _check(load().aap_histograms(h, _ptr(theta_hist), len(theta_hist), _ptr(n_hist),
                                 len(n_hist)))


def aap_checkpoint_bytes(h):
    n = ctypes.c_size_t()
    _check(load().aap_checkpoint_bytes(h, ctypes.byref(n)))
    return n.value


def aap_checkpoint_save(h, buf):
    _check(load().aap_checkpoint_save(h, _ptr(buf), buf.nbytes))


def aap_checkpoint_load(h, buf):
    _check(load().aap_checkpoint_load(h, _ptr(buf), buf.nbytes))


def aap_last_error():
    return load().aap_last_error().decode(errors="replace")


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------
def make_params(N=4096, Lx=64.0, Ly=None, R=1.0, v=0.5, eta=0.3, omega=0.0,
                gamma=1.0, dt=1.0, rule=AAP_RULE_VM, order=1, bx=0, by=0,
                seed=0, weights=None, binnum_theta=0, binnum_neighbors=0, replica=0):
    """aap_params from keyword arguments (the paper's names, Sec. 4);
    returns (params, keepalive)."""
    p = aap_params_default()
    p.bins_theta, p.bins_n = int(binnum_theta), int(binnum_neighbors)
    p.replica = int(replica)
    p.N, p.Lx, p.Ly, p.R = int(N), float(Lx), float(Lx if Ly is None else Ly), float(R)
    p.v, p.eta, p.omega, p.gamma, p.dt = float(v), float(eta), float(omega), float(gamma), float(dt)
    p.rule, p.order, p.bx, p.by = int(rule), int(order), int(bx), int(by)
    p.seed = int(seed)
    keep = None
    if weights is not None:
        keep = np.ascontiguousarray(weights, dtype=np.float64)
        p.weights = keep.ctypes.data_as(ctypes.POINTER(_dbl))
        p.weight_len = len(keep)
    return p, keep


class Sim:
    """A simulation on one GPU: workspace tensor + library handle."""

    def __init__(self, device=None, stream=None, **kw):
        import torch
        load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        # the weights array the parameters point into stays alive with the Sim
        self.params, self._keep = make_params(**kw)
        self.N = int(self.params.N)
        nbytes = aap_workspace_bytes(self.params)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.handle = aap_create(self.params, self.workspace.data_ptr(), nbytes,
                                     self.stream.cuda_stream)
        self.nbytes = nbytes

    def step(self, nsteps=1, measure=False, series=False):
        if series:
            out = np.zeros(int(nsteps), dtype=np.float64)
            aap_step(self.handle, nsteps, 1, out)
            return out
        aap_step(self.handle, nsteps, int(bool(measure)), None)
        return None

    def observables(self):
        o = aap_observables(self.handle)
        return dict(steps_measured=o.steps_measured, p_mom=list(o.p_mom),
                    nbar_mom=list(o.nbar_mom), binder=o.binder, p_last=o.p_last,
                    nbar_last=o.nbar_last, q_mom=list(o.q_mom), q_last=o.q_last)

    def histograms(self):
        """(angle histogram, neighbour-number histogram), normalised."""
        th = np.zeros(self.params.bins_theta, np.float64)
        nh = np.zeros(self.params.bins_n, np.float64)
        aap_histograms(self.handle, th, nh)
        return th, nh

    def checkpoint(self):
        """The whole simulation as bytes (aap_checkpoint_save)."""
        buf = np.zeros(aap_checkpoint_bytes(self.handle), np.uint8)
        aap_checkpoint_save(self.handle, buf)
        return buf.tobytes()

    def restore(self, data):
        """Load bytes made by checkpoint() of a simulation with the same parameters."""
        aap_checkpoint_load(self.handle, np.frombuffer(data, dtype=np.uint8).copy())

    def save(self, path):
        with open(path, "wb") as f:
            f.write(self.checkpoint())

    def load(self, path):
        with open(path, "rb") as f:
            self.restore(f.read())

    def reset_observables(self):
        aap_reset_observables(self.handle)

    def get_state(self):
        x = np.zeros(self.N, np.float32)
        y = np.zeros(self.N, np.float32)
        th = np.zeros(self.N, np.float32)
        step = aap_get_state(self.handle, x, y, th)
        return x, y, th, step

    def set_state(self, x, y, th, step=0):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        th = np.ascontiguousarray(th, dtype=np.float32)
        assert len(x) == len(y) == len(th) == self.N
        aap_set_state(self.handle, x, y, th, step)

    def sync(self):
        aap_sync(self.handle)

    def debug_keys(self):
        key = np.zeros(self.N, np.uint32)
        mx, my = aap_debug_keys(self.handle, key)
        return key, mx, my

    def cells(self):
        return aap_debug_keys(self.handle, None)

    def debug_enable(self, on=True):
        aap_debug_enable(self.handle, on)

    def debug_last_step(self):
        mx, my = self.cells()
        start = np.zeros(mx * my + 1, np.uint32)
        order = np.zeros(self.N, np.uint32)
        n = np.zeros(self.N, np.uint32)
        C = np.zeros(self.N, np.float32)
        S = np.zeros(self.N, np.float32)
        aap_debug_last_step(self.handle, start, order, n, C, S)
        return dict(start=start, order=order, n=n, C=C, S=S)

    def timing_enable(self, every=1):
        """Time the kernels of every every-th step (True = 1; 0/False off)."""
        aap_timing_enable(self.handle, int(every))

    def graph(self, steps_per_graph):
        """Replay runs of steps_per_graph steps from captured HIP graphs (0 = off)."""
        aap_graph(self.handle, int(steps_per_graph))

    def timing_read(self):
        return aap_timing_read(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            aap_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# batches of replicas
# ---------------------------------------------------------------------------
def _params_array(plist):
    arr = (aap_params * len(plist))(*plist)
    return arr


def aap_batch_workspace_bytes(plist):
    arr = _params_array(plist)
    n = ctypes.c_size_t()
    _check(load().aap_batch_workspace_bytes(ctypes.cast(arr, _p), len(plist), ctypes.byref(n)))
    return n.value


def aap_batch_create(plist, d_workspace, nbytes, hip_stream):
    arr = _params_array(plist)
    h = _p()
    _check(load().aap_batch_create(ctypes.cast(arr, _p), len(plist), _p(d_workspace), nbytes,
                                   _p(hip_stream), ctypes.byref(h)))
    return h


def aap_batch_destroy(h):
    _check(load().aap_batch_destroy(h))


def aap_batch_graph(h, steps_per_graph):
    _check(load().aap_batch_graph(h, int(steps_per_graph)))


def aap_batch_step(h, nsteps, measure):
    _check(load().aap_batch_step(h, int(nsteps), int(bool(measure))))


def aap_batch_sync(h):
    _check(load().aap_batch_sync(h))


def aap_batch_observables(h, count):
    out = (aap_observables_t * count)()
    _check(load().aap_batch_observables(h, ctypes.cast(out, _p), count))
    return list(out)


def aap_batch_reset_observables(h):
    _check(load().aap_batch_reset_observables(h))


def aap_batch_debug_enable(h, on):
    _check(load().aap_batch_debug_enable(h, int(on)))


def aap_batch_debug_keys(h, replica, key):
    mx, my = _i32(), _i32()
    _check(load().aap_batch_debug_keys(h, int(replica), _ptr(key), ctypes.byref(mx),
                                       ctypes.byref(my)))
    return mx.value, my.value


def aap_batch_debug_last_step(h, replica, start, order, n, C, S):
    _check(load().aap_batch_debug_last_step(h, int(replica), _ptr(start), _ptr(order), _ptr(n),
                                            _ptr(C), _ptr(S)))


def aap_batch_get_state(h, replica, x, y, theta):
    st = _u64()
    _check(load().aap_batch_get_state(h, int(replica), _ptr(x), _ptr(y), _ptr(theta),
                                      ctypes.byref(st)))
    return st.value


def aap_batch_threads(h, threads):
    _check(load().aap_batch_threads(h, int(threads)))


def aap_batch_kernel_times(h, steps, measure):
    a, c = _dbl(), _dbl()
    _check(load().aap_batch_kernel_times(h, int(steps), int(bool(measure)), ctypes.byref(a),
                                         ctypes.byref(c)))
    return a.value, c.value


def aap_batch_autotune(h, steps, measure):
    t, g = _i32(), _i32()
    _check(load().aap_batch_autotune(h, int(steps), int(bool(measure)), ctypes.byref(t),
                                     ctypes.byref(g)))
    return t.value, g.value


class Batch:
    """Replicas stepped together on one GPU: one workspace tensor, one handle.
    ``replicas`` is a list of keyword dicts as for Sim."""

    def __init__(self, replicas, device=None, stream=None, graph_steps=0):
        import torch
        load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        made = [make_params(**kw) for kw in replicas]
        self.params = [m[0] for m in made]
        self._keep = [m[1] for m in made]
        self.count = len(self.params)
        self.N = [int(p.N) for p in self.params]
        nbytes = aap_batch_workspace_bytes(self.params)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.handle = aap_batch_create(self.params, self.workspace.data_ptr(), nbytes,
                                           self.stream.cuda_stream)
        self.nbytes = nbytes
        if graph_steps:
            aap_batch_graph(self.handle, graph_steps)

    def graph(self, steps_per_graph):
        aap_batch_graph(self.handle, steps_per_graph)

    def threads(self, n):
        aap_batch_threads(self.handle, n)

    def kernel_times(self, steps, measure=True):
        """(sort ms, neighbour ms) means over `steps` timed ordinary steps."""
        return aap_batch_kernel_times(self.handle, steps, measure)

    def autotune(self, steps=16, measure=True):
        """Keeps the fastest (workgroup size, steps per graph); returns it."""
        return aap_batch_autotune(self.handle, steps, measure)

    def step(self, nsteps=1, measure=False):
        aap_batch_step(self.handle, nsteps, measure)

    def sync(self):
        aap_batch_sync(self.handle)

    def observables(self):
        return [dict(steps_measured=o.steps_measured, p_mom=list(o.p_mom),
                     nbar_mom=list(o.nbar_mom), binder=o.binder, p_last=o.p_last,
                     nbar_last=o.nbar_last, q_mom=list(o.q_mom), q_last=o.q_last)
                for o in aap_batch_observables(self.handle, self.count)]

    def reset_observables(self):
        aap_batch_reset_observables(self.handle)

    def debug_enable(self, on=True):
        """Every later step also records n, C, S per particle (parity tests)."""
        aap_batch_debug_enable(self.handle, on)

    def debug_keys(self, replica):
        """The next cells of replica's particles by id, as the last step wrote them."""
        key = np.zeros(self.N[replica], np.uint32)
        aap_batch_debug_keys(self.handle, replica, key)
        return key

    def debug_last_step(self, replica):
        """Cell starts, sorted ids, and n, C, S by id of the state the last
        step of replica read (as Sim.debug_last_step)."""
        n = self.N[replica]
        mx, my = aap_batch_debug_keys(self.handle, replica, None)
        start = np.zeros(mx * my + 1, np.uint32)
        order = np.zeros(n, np.uint32)
        nn = np.zeros(n, np.uint32)
        C = np.zeros(n, np.float32)
        S = np.zeros(n, np.float32)
        aap_batch_debug_last_step(self.handle, replica, start, order, nn, C, S)
        return dict(start=start, order=order, n=nn, C=C, S=S)

    def get_state(self, replica):
        n = self.N[replica]
        x = np.zeros(n, np.float32)
        y = np.zeros(n, np.float32)
        th = np.zeros(n, np.float32)
        step = aap_batch_get_state(self.handle, replica, x, y, th)
        return x, y, th, step

    def close(self):
        if self.handle:
            aap_batch_destroy(self.handle)
            self.handle = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# learned field surrogate
# ---------------------------------------------------------------------------
def aap_fields_scratch_bytes(G):
    n = ctypes.c_size_t()
    _check(load().aap_fields_scratch_bytes(int(G), ctypes.byref(n)))
    return n.value


def aap_fields(h, G, d_fields, d_scratch, nbytes):
    _check(load().aap_fields(h, int(G), _p(d_fields), _p(d_scratch), nbytes))


def aap_batch_fields(h, replica, G, d_fields, d_scratch, nbytes):
    _check(load().aap_batch_fields(h, int(replica), int(G), _p(d_fields), _p(d_scratch), nbytes))


def aap_fields_noalloc(h, G, d_fields):
    _check(load().aap_fields_noalloc(h, int(G), _p(d_fields)))


def aap_cnn_param_count():
    return int(load().aap_cnn_param_count())


def _fields_into(fn, handle, G, device, extra=()):
    import torch
    nbytes = aap_fields_scratch_bytes(G)
    scratch = torch.empty(nbytes, dtype=torch.uint8, device=device)
    out = torch.empty((3, G, G), dtype=torch.float32, device=device)
    fn(handle, *extra, G, out.data_ptr(), scratch.data_ptr(), nbytes)
    return out, scratch


def sim_fields(sim, G):
    """(rho, p_x, p_y) of a Sim's current state: a torch tensor [3, G, G]."""
    out, scratch = _fields_into(aap_fields, sim.handle, G, sim.device)
    sim.stream.synchronize()
    return out


def sim_fields_noalloc(sim, G, out):
    """The fields of a Sim's state into out (a float32 device tensor [3, G, G]
    the caller allocated), through the entry point that allocates nothing."""
    assert out.dtype.is_floating_point and out.numel() == 3 * G * G and out.is_contiguous()
    aap_fields_noalloc(sim.handle, G, out.data_ptr())
    return out


def batch_fields(batch, replica, G):
    out, scratch = _fields_into(aap_batch_fields, batch.handle, G, batch.device, (int(replica),))
    batch.stream.synchronize()
    return out


class CNN:
    """The field surrogate: workspace tensor + library handle."""

    def __init__(self, G, max_batch, device=None, stream=None):
        import torch
        load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.G, self.max_batch = int(G), int(max_batch)
        n = ctypes.c_size_t()
        _check(load().aap_cnn_workspace_bytes(self.G, self.max_batch, ctypes.byref(n)))
        self.nbytes = n.value
        self.nparam = aap_cnn_param_count()
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = _p()
            _check(load().aap_cnn_create(self.G, self.max_batch, _p(self.workspace.data_ptr()),
                                         self.nbytes, _p(self.stream.cuda_stream),
                                         ctypes.byref(h)))
        self.handle = h

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(load().aap_cnn_set_params(self.handle, _ptr(a), a.size))

    def get_params(self):
        a = np.zeros(self.nparam, np.float32)
        _check(load().aap_cnn_get_params(self.handle, _ptr(a), a.size))
        return a

    def forward(self, fields, rho0):
        """fields: torch float32 [nb, 3, G, G] on the device -> predicted fields."""
        import torch
        assert fields.dtype == torch.float32 and fields.is_contiguous()
        out = torch.empty_like(fields)
        _check(load().aap_cnn_forward(self.handle, _p(fields.data_ptr()), fields.shape[0],
                                      float(rho0), _p(out.data_ptr())))
        return out

    def train_step(self, inp, target, rho0, lr):
        loss = _dbl()
        _check(load().aap_cnn_train_step(self.handle, _p(inp.data_ptr()), _p(target.data_ptr()),
                                         inp.shape[0], float(rho0), float(lr),
                                         ctypes.byref(loss)))
        return loss.value

    def debug_read(self, which, shape, dtype):
        a = np.zeros(shape, dtype)
        _check(load().aap_cnn_debug_read(self.handle, int(which), _ptr(a), a.nbytes))
        return a

    def close(self):
        if self.handle:
            _check(load().aap_cnn_destroy(self.handle))
            self.handle = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes binding of liblj_bh.so (C ABI in include/lj_bh.h).

Argument marshalling only: torch tensors provide device memory and the
stream; every step of the method runs in the library's HIP kernels.  The
library must be built (paper_2510_25938_amd/build.py); importing a function
without it raises instead of falling back to anything else.
"""
import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblj_bh.so")

FP64, MIXED = 0, 1
CONVERGED, MAXITER, LSFAIL, NONFINITE, SWITCHED, BADSIZE = 0, 1, 2, 3, 4, 5
OK, E_ARG, E_HIP, E_WORKSPACE, E_UNSUPPORTED = 0, -1, -2, -3, -4
MAX_ATOMS_EVAL, MAX_ATOMS_MIN, MAX_M, MAX_CANDS = 4096, 1024, 10, 64
SCHED_EVAL, SCHED_MIN_LARGE = 0, 1
SCHED_MIN_CLASS = (2, 3, 4)  # minimiser shape of size classes 0, 1, 2
# shapes per class: (clusters per workgroup, largest N) for each shape index
CLASS_SHAPES = {0: ((1, 64), (1, 16), (2, 32), (4, 16)) * 2, 1: ((1, 128), (1, 128)),
                2: ((1, 256), (1, 192))}
EXPORTED = ["lj_energy_grad_batch", "lj_lbfgs_defaults", "lj_minimize_workspace_bytes",
            "lj_bh_minimize_batch", "lj_bh_workspace_bytes", "lj_bh_step", "lj_set_schedule",
            "lj_get_schedule", "lj_autotune_workspace_bytes", "lj_autotune", "lj_status_string",
            "lj_last_error", "lj_abi_version", "lj_bh_minimize_batch_noalloc",
            "lj_bh_graph_captures"]
NOALLOC_SCRATCH_BYTES, NOALLOC_MAX_ATOMS, NOALLOC_MAX_CLUSTERS = 1 << 20, 256, 262016


PAIRS = {"lj": 0, "morse": 1}  # LJ_PAIR_LJ (Eq. 1), LJ_PAIR_MORSE


class Batch(C.Structure):
    _fields_ = [("num", C.c_int32), ("offset", C.c_void_p), ("max_n", C.c_int32),
                ("total_atoms", C.c_int64), ("pair", C.c_int32), ("pair_rho", C.c_double),
                ("sigma", C.c_double), ("epsilon", C.c_double)]


class LbfgsParams(C.Structure):
    _fields_ = [("m", C.c_int32), ("gtol", C.c_double), ("max_iter", C.c_int32),
                ("max_step", C.c_double), ("c1", C.c_double), ("max_ls", C.c_int32),
                ("curv_eps", C.c_double), ("gtol_mixed_per_atom", C.c_double),
                ("polish", C.c_int32), ("ls_noise", C.c_double)]


class BhParams(C.Structure):
    _fields_ = [("cands", C.c_int32), ("kT", C.c_double), ("adapt_interval", C.c_int32),
                ("target_rate", C.c_double), ("factor", C.c_double), ("seed", C.c_uint64)]


class BhState(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("xyz_cur", "e_cur", "step", "win_accepts",
                                          "step_index", "e_best_seen", "e_best_acc",
                                          "xyz_best")]


class BhTrace(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("e_trial", "accepted", "e_best", "e_best_acc", "e_cur",
                                          "step", "e_cand", "polish_status")] + [
        ("capacity_steps", C.c_int32)]


class LJError(RuntimeError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LJError(f"{LIB_PATH} is missing: build it with paper_2510_25938_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.lj_energy_grad_batch.argtypes = [C.POINTER(Batch), vp, vp, vp, i32, vp]
        L.lj_energy_grad_batch.restype = i32
        L.lj_lbfgs_defaults.argtypes = [C.POINTER(LbfgsParams)]
        L.lj_lbfgs_defaults.restype = None
        L.lj_minimize_workspace_bytes.argtypes = [C.POINTER(Batch), C.POINTER(LbfgsParams), i32]
        L.lj_minimize_workspace_bytes.restype = C.c_size_t
        L.lj_bh_minimize_batch.argtypes = [C.POINTER(Batch), vp, vp, vp, vp, vp, vp, vp,
                                           C.POINTER(LbfgsParams), i32, vp, C.c_size_t, vp]
        L.lj_bh_minimize_batch.restype = i32
        L.lj_bh_minimize_batch_noalloc.argtypes = [C.POINTER(Batch), vp, vp, vp, vp, vp, vp, vp,
                                                   C.POINTER(LbfgsParams), i32, vp]
        L.lj_bh_minimize_batch_noalloc.restype = i32
        L.lj_bh_workspace_bytes.argtypes = [C.POINTER(Batch), C.POINTER(BhParams),
                                            C.POINTER(LbfgsParams), i32]
        L.lj_bh_workspace_bytes.restype = C.c_size_t
        L.lj_bh_step.argtypes = [C.POINTER(Batch), C.POINTER(BhState), C.POINTER(BhParams),
                                 C.POINTER(LbfgsParams), i32, i32, C.POINTER(BhTrace), vp,
                                 C.c_size_t, vp]
        L.lj_bh_step.restype = i32
        L.lj_set_schedule.argtypes = [i32, i32, i32, i32, i32]
        L.lj_set_schedule.restype = i32
        L.lj_get_schedule.argtypes = [i32, i32, i32, C.POINTER(i32), C.POINTER(i32)]
        L.lj_get_schedule.restype = i32
        L.lj_autotune_workspace_bytes.argtypes = [C.POINTER(Batch), i32]
        L.lj_autotune_workspace_bytes.restype = C.c_size_t
        L.lj_autotune.argtypes = [C.POINTER(Batch), vp, i32, vp, C.c_size_t, vp,
                                  C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.lj_autotune.restype = i32
        L.lj_status_string.argtypes = [i32]
        L.lj_status_string.restype = C.c_char_p
        L.lj_last_error.argtypes = []
        L.lj_last_error.restype = C.c_char_p
        L.lj_abi_version.argtypes = []
        L.lj_abi_version.restype = i32
        L.lj_bh_graph_captures.argtypes = []
        L.lj_bh_graph_captures.restype = C.c_int64
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        L = lib()
        raise LJError(f"{L.lj_status_string(status).decode()}: {L.lj_last_error().decode()}",
                      status)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _order(stream, *tensors):
    """Work on `stream` that uses tensors made on the current stream: the
    stream first waits for the current stream's queued work, and the tensors
    are recorded as in use on it (so the caching allocator does not hand their
    memory out again before that work is done)."""
    if stream is None or torch.cuda.is_current_stream_capturing():
        return  # under capture the caller orders its streams
    cur = torch.cuda.current_stream(stream.device)
    if stream.cuda_stream == cur.cuda_stream:
        return
    stream.wait_stream(cur)
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def precision_code(p):
    if isinstance(p, int):
        return p
    return {"fp64": FP64, "mixed": MIXED}[p]


def lbfgs_params(**kw):
    p = LbfgsParams()
    lib().lj_lbfgs_defaults(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class ClusterBatch:
    """A ragged batch: host sizes plus the device int32 prefix-sum offsets, and
    the pair potential ("lj": Eq. (1); "morse": the Morse pair of range rho,
    well depth 1 at r = 1), both in reduced units."""

    def __init__(self, offset, device="cuda", pair="lj", rho=6.0):
        if pair not in PAIRS:
            raise ValueError(f"pair must be one of {sorted(PAIRS)}")
        self.pair, self.rho = pair, float(rho)
        off = np.asarray(offset, dtype=np.int64)
        if off.ndim != 1 or off.size < 1 or off[0] != 0 or np.any(np.diff(off) < 0):
            raise ValueError("offset must be nondecreasing prefix sums starting at 0")
        self.sizes = np.diff(off)
        self.num = int(self.sizes.size)
        self.total = int(off[-1])
        self.max_n = int(self.sizes.max()) if self.num else 0
        self.offset_host = off.astype(np.int32)
        self.offset = torch.from_numpy(self.offset_host).to(device)

    def desc(self, max_n=None, sigma=1.0, epsilon=1.0):
        """The C descriptor; sigma / epsilon: the units of the coordinates and
        energies passed in and out (the library converts; kernels work in
        reduced units)."""
        return Batch(self.num, self.offset.data_ptr(), self.max_n if max_n is None else max_n,
                     self.total, PAIRS[self.pair], self.rho, float(sigma), float(epsilon))


def energy_grad(batch, xyz, precision="fp64", grad=True, stream=None, sigma=1.0, epsilon=1.0):
    """Energies [num] and gradient planes [3][total] (None if grad=False) of the
    batch's pair potential, for coordinates in units of sigma and energies in
    units of epsilon."""
    assert xyz.dtype == torch.float64 and xyz.is_contiguous() and xyz.shape == (3, batch.total)
    E = torch.empty(batch.num, dtype=torch.float64, device=xyz.device)
    g = torch.empty_like(xyz) if grad else None
    _order(stream, xyz, E, g, batch.offset)
    _check(lib().lj_energy_grad_batch(C.byref(batch.desc(sigma=sigma, epsilon=epsilon)),
                                      _ptr(xyz), _ptr(E), _ptr(g), precision_code(precision),
                                      _stream(stream)))
    return E, g


def minimize_workspace_bytes(batch, params=None, precision="fp64"):
    params = params or lbfgs_params()
    return int(lib().lj_minimize_workspace_bytes(C.byref(batch.desc()), C.byref(params),
                                                 precision_code(precision)))


def minimize(batch, xyz, params=None, precision="fp64", switch_point=False, workspace=None,
             stream=None, inplace=False, sigma=1.0, epsilon=1.0):
    """Local minimisation of every cluster; returns a dict of device tensors.
    Coordinates (in and out) are in units of sigma, energies and gradient norms
    in units of epsilon (sigma / sigma); params are in reduced units."""
    params = params or lbfgs_params()
    assert xyz.dtype == torch.float64 and xyz.is_contiguous() and xyz.shape == (3, batch.total)
    dev = xyz.device
    x = xyz if inplace else xyz.clone()
    out = dict(xyz=x, energy=torch.empty(batch.num, dtype=torch.float64, device=dev),
               gnorm=torch.empty(batch.num, dtype=torch.float64, device=dev),
               iters=torch.empty(batch.num, dtype=torch.int32, device=dev),
               evals=torch.empty(batch.num, dtype=torch.int32, device=dev),
               status=torch.empty(batch.num, dtype=torch.int32, device=dev))
    out["xyz_switch"] = torch.zeros_like(x) if switch_point else None
    if workspace is None:
        nb = minimize_workspace_bytes(batch, params, precision)
        if nb == 0 and batch.num > 0:
            _check(E_ARG)
        workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    _order(stream, x, workspace, batch.offset, *out.values())
    _check(lib().lj_bh_minimize_batch(C.byref(batch.desc(sigma=sigma, epsilon=epsilon)),
                                      _ptr(x), _ptr(out["energy"]),
                                      _ptr(out["gnorm"]), _ptr(out["iters"]), _ptr(out["evals"]),
                                      _ptr(out["status"]), _ptr(out["xyz_switch"]),
                                      C.byref(params), precision_code(precision),
                                      _ptr(workspace), workspace.numel(), _stream(stream)))
    return out


def minimize_noalloc(batch, xyz, params=None, precision="fp64", switch_point=False,
                     stream=None, inplace=False, sigma=1.0, epsilon=1.0):
    """`minimize` through the allocation-free entry point: no workspace, the
    library's fixed per-device scratch instead (at most NOALLOC_MAX_ATOMS atoms
    per cluster and NOALLOC_MAX_CLUSTERS clusters; overlapping calls on one
    device race).  The output tensors are allocated here, by the caller."""
    params = params or lbfgs_params()
    assert xyz.dtype == torch.float64 and xyz.is_contiguous() and xyz.shape == (3, batch.total)
    dev = xyz.device
    x = xyz if inplace else xyz.clone()
    out = dict(xyz=x, energy=torch.empty(batch.num, dtype=torch.float64, device=dev),
               gnorm=torch.empty(batch.num, dtype=torch.float64, device=dev),
               iters=torch.empty(batch.num, dtype=torch.int32, device=dev),
               evals=torch.empty(batch.num, dtype=torch.int32, device=dev),
               status=torch.empty(batch.num, dtype=torch.int32, device=dev))
    out["xyz_switch"] = torch.zeros_like(x) if switch_point else None
    _order(stream, x, batch.offset, *out.values())
    _check(lib().lj_bh_minimize_batch_noalloc(
        C.byref(batch.desc(sigma=sigma, epsilon=epsilon)), _ptr(x), _ptr(out["energy"]), _ptr(out["gnorm"]),
        _ptr(out["iters"]), _ptr(out["evals"]), _ptr(out["status"]), _ptr(out["xyz_switch"]),
        C.byref(params), precision_code(precision), _stream(stream)))
    return out


def set_schedule(kind, precision, max_n, w, a=1):
    _check(lib().lj_set_schedule(kind, precision_code(precision), int(max_n), int(w), int(a)))


def eval_shape_default(max_n):
    """The library's built-in pair-kernel shape (W, A) for max_n atoms."""
    n = max(int(max_n), 1)
    for lim, shape in ((64, (1, 1)), (128, (2, 1)), (256, (4, 1)), (512, (8, 1)),
                       (1024, (16, 1)), (2048, (16, 2))):
        if n <= lim:
            return shape
    return (16, 4)


def get_schedule(kind, precision, max_n=0):
    w, a = C.c_int32(), C.c_int32()
    _check(lib().lj_get_schedule(kind, precision_code(precision), int(max_n), C.byref(w),
                                 C.byref(a)))
    return w.value, a.value


def autotune(batch, xyz, precision="mixed", stream=None, cache=None):
    """Time every launch schedule for this batch shape and keep the fastest.

    Synchronises the stream.  With `cache` (a JSON path) the chosen schedules
    are merged into that file; `load_schedules` installs them in a new process.
    Returns {"eval": (W, A, ms), "min_large": shape or None, "min_ms": ms of a
    minimisation with the chosen shapes or None, "min_class": {class: shape}
    for the size classes the batch holds}.
    """
    prec = precision_code(precision)
    nb = int(lib().lj_autotune_workspace_bytes(C.byref(batch.desc()), prec))
    if nb == 0:
        _check(E_ARG)
    ws = torch.empty(nb, dtype=torch.uint8, device=xyz.device)
    _order(stream, xyz, ws, batch.offset)
    t_eval, t_min = C.c_float(), C.c_float()
    _check(lib().lj_autotune(C.byref(batch.desc()), _ptr(xyz), prec, _ptr(ws), nb,
                             _stream(stream), C.byref(t_eval), C.byref(t_min)))
    w, a = get_schedule(SCHED_EVAL, prec, batch.max_n)
    res = {"eval": (w, a, t_eval.value), "min_large": None, "min_ms": None, "min_class": {}}
    if t_min.value >= 0:
        res["min_ms"] = t_min.value
        if batch.max_n > 256:
            res["min_large"] = get_schedule(SCHED_MIN_LARGE, prec)[0]
        for c in range(3):
            if c <= _class_of(batch.max_n):
                k = get_schedule(SCHED_MIN_CLASS[c], prec, batch.max_n)[0]
                if k >= 0:
                    res["min_class"][c] = k
    if cache:
        import json
        table = {}
        if os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
        key = "fp64" if prec == FP64 else "mixed"
        p2 = 1
        while p2 < max(batch.max_n, 1):
            p2 *= 2
        table.setdefault(key, {}).setdefault("eval", {})[str(p2)] = [w, a]
        if res["min_large"] is not None:
            table[key]["min_large"] = res["min_large"]
        if res["min_class"]:
            table[key].setdefault("min_class", {})[str(batch.max_n)] = {
                str(c): k for c, k in res["min_class"].items()}
        with open(cache, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    return res


def load_schedules(cache):
    """Install schedules saved by `autotune(..., cache=path)`."""
    import json
    with open(cache) as fh:
        table = json.load(fh)
    for key, entry in table.items():
        prec = FP64 if key == "fp64" else MIXED
        for p2, (w, a) in entry.get("eval", {}).items():
            set_schedule(SCHED_EVAL, prec, int(p2), w, a)
        if "min_large" in entry:
            set_schedule(SCHED_MIN_LARGE, prec, 0, entry["min_large"], 0)
        for max_n, shapes in entry.get("min_class", {}).items():
            for c, k in shapes.items():
                set_schedule(SCHED_MIN_CLASS[int(c)], prec, int(max_n), k, 0)


def _class_of(n):
    for c, lim in enumerate((64, 128, 256, MAX_ATOMS_MIN)):
        if n <= lim:
            return c
    return -1


def bh_params(cands=8, kT=0.8, adapt_interval=10, target_rate=0.5, factor=0.9, seed=0):
    return BhParams(cands, kT, adapt_interval, target_rate, factor, seed)


class BasinHopping:
    """Device state of many independent basin-hopping chains.

    `xyz_min` / `e_min` must be local minima (e.g. from `minimize`); the
    chains start there with step size `step0`.
    """

    def __init__(self, batch, xyz_min, e_min, bh, params=None, precision="fp64", step0=0.4,
                 trace_steps=0, trace_candidates=False):
        self.batch, self.bh = batch, bh
        self.params = params or lbfgs_params()
        self.precision = precision_code(precision)
        dev = xyz_min.device
        C_ = batch.num
        self.xyz_cur = xyz_min.clone()
        self.xyz_best = xyz_min.clone()
        self.e_cur = e_min.clone().to(torch.float64)
        self.e_best_acc = self.e_cur.clone()
        self.e_best_seen = torch.full((C_,), float("inf"), dtype=torch.float64, device=dev)
        self.step_size = torch.full((C_,), float(step0), dtype=torch.float64, device=dev)
        self.win_accepts = torch.zeros(C_, dtype=torch.int32, device=dev)
        self.step_index = torch.zeros(C_, dtype=torch.int64, device=dev)
        self.state = BhState(*[t.data_ptr() for t in (self.xyz_cur, self.e_cur, self.step_size,
                                                      self.win_accepts, self.step_index,
                                                      self.e_best_seen, self.e_best_acc,
                                                      self.xyz_best)])
        self.trace = None
        self._trace_desc = None
        if trace_steps > 0:
            f = dict(dtype=torch.float64, device=dev)
            self.trace = dict(e_trial=torch.full((C_, trace_steps), float("nan"), **f),
                              accepted=torch.zeros((C_, trace_steps), dtype=torch.int8, device=dev),
                              e_best=torch.full((C_, trace_steps), float("nan"), **f),
                              e_best_acc=torch.full((C_, trace_steps), float("nan"), **f),
                              e_cur=torch.full((C_, trace_steps), float("nan"), **f),
                              step=torch.full((C_, trace_steps), float("nan"), **f))
            self.trace["e_cand"] = (torch.full((C_, trace_steps, bh.cands), float("nan"), **f)
                                    if trace_candidates else None)
            self.trace["polish_status"] = torch.full((C_, trace_steps), -1, dtype=torch.int8,
                                                     device=dev)
            self._trace_desc = BhTrace(*[None if self.trace[k] is None else self.trace[k].data_ptr()
                                         for k in ("e_trial", "accepted", "e_best", "e_best_acc",
                                                   "e_cur", "step", "e_cand", "polish_status")],
                                       trace_steps)
        nb = int(lib().lj_bh_workspace_bytes(C.byref(batch.desc()), C.byref(bh),
                                             C.byref(self.params), self.precision))
        if nb == 0:
            _check(E_ARG)
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
        # Every step is ordered after the previous one (or, for the first, after
        # the initialisation above): a step on a stream other than the last
        # one's first waits for the event recorded behind the last step.
        self._last_stream = torch.cuda.current_stream(dev)
        self._last_event = torch.cuda.Event()
        self._last_event.record(self._last_stream)
        self._recorded = {self._last_stream.cuda_stream}

    def _tensors(self):
        ts = [self.xyz_cur, self.xyz_best, self.e_cur, self.e_best_acc, self.e_best_seen,
              self.step_size, self.win_accepts, self.step_index, self.workspace, self.batch.offset]
        if self.trace is not None:
            ts += [t for t in self.trace.values() if t is not None]
        return ts

    def step(self, num_steps=1, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.xyz_cur.device)
        capturing = torch.cuda.is_current_stream_capturing()
        if not capturing:  # under capture the caller orders its streams
            if s.cuda_stream != self._last_stream.cuda_stream:
                s.wait_event(self._last_event)
            if s.cuda_stream not in self._recorded:
                for t in self._tensors():
                    t.record_stream(s)
                self._recorded.add(s.cuda_stream)
        tr = C.byref(self._trace_desc) if self._trace_desc is not None else None
        _check(lib().lj_bh_step(C.byref(self.batch.desc()), C.byref(self.state), C.byref(self.bh),
                                C.byref(self.params), self.precision, int(num_steps), tr,
                                _ptr(self.workspace), self.workspace.numel(), _stream(s)))
        if not capturing:
            self._last_event = torch.cuda.Event()
            self._last_event.record(s)
            self._last_stream = s


def graph_captures():
    """Step graphs captured by this process so far (lj_bh_step's cache)."""
    return int(lib().lj_bh_graph_captures())

"""ctypes binding of libdpc (include/libdpc.h).

Argument marshalling only: every step of the method runs in the HIP library.
Tensors must live on the current ROCm device; PyTorch provides device memory
and the stream handle.  There is no fallback: if libdpc.so is missing, every
call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpc.so")

OK, ERR_INVALID_ARG, ERR_RANGE, ERR_NOT_FOREST, ERR_OOM, ERR_HIP, ERR_SCRATCH = range(7)
NOALLOC_SCRATCH_BYTES = 64 << 20  # DPC_NOALLOC_SCRATCH_BYTES
SKIP_NOISE_DEPENDENTS = 1
TIME_STAGES = 2
COUNT_WORK = 4
FENWICK_DEPENDENTS = 8
PST_DEPENDENTS = 16
# DPC_BACKEND_PRIORITY_TREE, DPC_BACKEND_FENWICK, DPC_BACKEND_PRIORITY_SEARCH_TREE
BACKENDS = ("priority_tree", "fenwick", "priority_search_tree")
INF = (1 << 63) - 1
STAGES = ("index", "density", "priority", "dependent", "labels")

EXPORTED = ("dpc_density", "dpc_dependent", "dpc_cluster", "dpc_run", "dpc_batch_run", "dpc_last_stats",
            "dpc_status_str", "dpc_square_threshold", "dpc_workspace_bytes", "dpc_density_sweep",
            "dpc_cluster_sweep", "dpc_server_create",
            "dpc_server_submit", "dpc_server_poll", "dpc_server_wait", "dpc_server_get_stats",
            "dpc_server_destroy", "dpc_set_leaf_size", "dpc_leaf_size", "dpc_autotune", "dpc_plan_create",
            "dpc_plan_launch", "dpc_plan_capture", "dpc_plan_status", "dpc_plan_destroy",
            "dpc_set_dependent_backend", "dpc_dependent_backend", "dpc_autotune_dependent",
            "dpc_plan_create_batch", "dpc_run_noalloc")


class Stats(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("stage_ms", ctypes.c_double * len(STAGES)),
                ("density_pairs", ctypes.c_int64), ("density_nodes", ctypes.c_int64),
                ("density_contained", ctypes.c_int64), ("dependent_pairs", ctypes.c_int64),
                ("dependent_nodes", ctypes.c_int64), ("density_wave_nodes", ctypes.c_int64),
                ("density_wave_points", ctypes.c_int64), ("dependent_wave_nodes", ctypes.c_int64),
                ("dependent_wave_points", ctypes.c_int64), ("workspace_bytes", ctypes.c_uint64)]

WORK_FIELDS = ("density_pairs", "density_nodes", "density_contained", "dependent_pairs", "dependent_nodes",
               "density_wave_nodes", "density_wave_points", "dependent_wave_nodes", "dependent_wave_points")


class Instance(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("d_cut", ctypes.c_double), ("rho_min", ctypes.c_int32), ("delta_min", ctypes.c_double),
                ("rho", ctypes.c_void_p), ("dep", ctypes.c_void_p), ("delta2", ctypes.c_void_p),
                ("label", ctypes.c_void_p), ("status", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("submit_ns", ctypes.c_int64),
                ("admit_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64), ("footprint", ctypes.c_uint64),
                ("batch_size", ctypes.c_int32), ("slot", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("max_batch_seen", ctypes.c_int64), ("max_slots_busy", ctypes.c_int32),
                ("max_admitted_bytes", ctypes.c_uint64), ("max_workspace_bytes", ctypes.c_uint64),
                ("over_footprint", ctypes.c_int64), ("in_flight_bytes", ctypes.c_uint64),
                ("queued", ctypes.c_int64)]


_lib = None


class DPCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} (status {status})")


def load():
    """Load libdpc.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32, u32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    lib.dpc_density.argtypes = [P, i64, i32, dbl, P, P]
    lib.dpc_density.restype = ctypes.c_int
    lib.dpc_dependent.argtypes = [P, i64, i32, P, i32, P, P, P]
    lib.dpc_dependent.restype = ctypes.c_int
    lib.dpc_cluster.argtypes = [i64, P, P, P, i32, dbl, P, P]
    lib.dpc_cluster.restype = ctypes.c_int
    lib.dpc_run.argtypes = [P, i64, i32, dbl, i32, dbl, u32, P, P, P, P, P]
    lib.dpc_run.restype = ctypes.c_int
    lib.dpc_run_noalloc.argtypes = [P, i64, i32, dbl, i32, dbl, u32, P, P, P, P, P]
    lib.dpc_run_noalloc.restype = ctypes.c_int
    lib.dpc_status_str.argtypes = [ctypes.c_int]
    lib.dpc_status_str.restype = ctypes.c_char_p
    lib.dpc_square_threshold.argtypes = [dbl, i32, P]
    lib.dpc_square_threshold.restype = ctypes.c_int
    lib.dpc_batch_run.argtypes = [ctypes.POINTER(Instance), ctypes.c_int32, u32, P]
    lib.dpc_batch_run.restype = ctypes.c_int
    lib.dpc_last_stats.argtypes = [ctypes.POINTER(Stats)]
    lib.dpc_last_stats.restype = ctypes.c_int
    lib.dpc_density_sweep.argtypes = [P, i64, i32, ctypes.POINTER(dbl), i32, P, P]
    lib.dpc_density_sweep.restype = ctypes.c_int
    lib.dpc_cluster_sweep.argtypes = [i64, P, P, P, ctypes.POINTER(i32), ctypes.POINTER(dbl), i32, P, P]
    lib.dpc_cluster_sweep.restype = ctypes.c_int
    lib.dpc_set_leaf_size.argtypes = [i32, i32]
    lib.dpc_set_leaf_size.restype = ctypes.c_int
    lib.dpc_leaf_size.argtypes = [i32]
    lib.dpc_leaf_size.restype = ctypes.c_int32
    lib.dpc_autotune.argtypes = [P, i64, i32, dbl, i32, dbl, P, ctypes.POINTER(dbl), ctypes.POINTER(i32)]
    lib.dpc_autotune.restype = ctypes.c_int
    lib.dpc_workspace_bytes.argtypes = [i64, i32]
    lib.dpc_workspace_bytes.restype = ctypes.c_uint64
    lib.dpc_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]
    lib.dpc_server_create.restype = ctypes.c_int
    lib.dpc_server_submit.argtypes = [P, ctypes.POINTER(Instance), u32, ctypes.POINTER(ctypes.c_uint64)]
    lib.dpc_server_submit.restype = ctypes.c_int
    lib.dpc_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(RequestInfo)]
    lib.dpc_server_poll.restype = ctypes.c_int
    lib.dpc_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(RequestInfo)]
    lib.dpc_server_wait.restype = ctypes.c_int
    lib.dpc_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.dpc_server_get_stats.restype = ctypes.c_int
    lib.dpc_server_destroy.argtypes = [P]
    lib.dpc_server_destroy.restype = ctypes.c_int
    lib.dpc_plan_create.argtypes = [P, i64, i32, dbl, i32, dbl, u32, P, P, P, P, P, ctypes.POINTER(P)]
    lib.dpc_plan_create.restype = ctypes.c_int
    lib.dpc_plan_create_batch.argtypes = [ctypes.POINTER(Instance), ctypes.c_int32, u32, P, ctypes.POINTER(P)]
    lib.dpc_plan_create_batch.restype = ctypes.c_int
    lib.dpc_plan_launch.argtypes = [P, P]
    lib.dpc_plan_launch.restype = ctypes.c_int
    lib.dpc_plan_capture.argtypes = [P, P]
    lib.dpc_plan_capture.restype = ctypes.c_int
    lib.dpc_plan_status.argtypes = [P, P, ctypes.POINTER(i32)]
    lib.dpc_plan_status.restype = ctypes.c_int
    lib.dpc_plan_destroy.argtypes = [P]
    lib.dpc_plan_destroy.restype = ctypes.c_int
    lib.dpc_set_dependent_backend.argtypes = [i32, i32]
    lib.dpc_set_dependent_backend.restype = ctypes.c_int
    lib.dpc_dependent_backend.argtypes = [i32]
    lib.dpc_dependent_backend.restype = ctypes.c_int32
    lib.dpc_autotune_dependent.argtypes = [P, i64, i32, dbl, i32, dbl, P, ctypes.POINTER(dbl), ctypes.POINTER(i32)]
    lib.dpc_autotune_dependent.restype = ctypes.c_int
    _lib = lib
    return lib


def status_str(status: int) -> str:
    return load().dpc_status_str(int(status)).decode()


def square_threshold(r: float, round_up: bool = False) -> int:
    out = ctypes.c_int64(0)
    st = load().dpc_square_threshold(float(r), int(bool(round_up)), ctypes.byref(out))
    if st != OK:
        raise DPCError(st, "dpc_square_threshold")
    return out.value


# ---------------------------------------------------------------------------
# device calls


def _torch():
    import torch

    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _check_points(points):
    torch = _torch()
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a device tensor")
    if points.dtype != torch.int32 or points.dim() != 2 or not points.is_contiguous():
        raise TypeError("points must be a contiguous int32 [n, d] tensor")
    return points.shape[0], points.shape[1]


def _out(t, n, dtype, device):
    torch = _torch()
    if t is None:
        return torch.empty(n, dtype=dtype, device=device)
    if t.dtype != dtype or t.numel() != n or not t.is_contiguous() or t.device != device:
        raise TypeError(f"output must be a contiguous {dtype} tensor of {n} elements on {device}")
    return t


def _vec(t, n, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or t.numel() != n \
            or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} device tensor of {n} elements")
    return t


def density(points, d_cut: float, out=None, stream=None):
    """rho (int32 [n]) for int32 [n, d] device points."""
    torch = _torch()
    n, d = _check_points(points)
    rho = _out(out, n, torch.int32, points.device)
    st = load().dpc_density(_ptr(points), n, d, float(d_cut), _ptr(rho), _stream(stream))
    if st != OK:
        raise DPCError(st, "dpc_density")
    return rho


def dependent(points, rho, rho_min: int = 0, dep=None, delta2=None, stream=None):
    """(dep int32 [n], delta2 int64 [n]) for given densities."""
    torch = _torch()
    n, d = _check_points(points)
    _vec(rho, n, torch.int32, "rho")
    dep = _out(dep, n, torch.int32, points.device)
    delta2 = _out(delta2, n, torch.int64, points.device)
    st = load().dpc_dependent(_ptr(points), n, d, _ptr(rho), int(rho_min), _ptr(dep), _ptr(delta2),
                              _stream(stream))
    if st != OK:
        raise DPCError(st, "dpc_dependent")
    return dep, delta2


def cluster(rho, dep, delta2, rho_min: int, delta_min: float, label=None, stream=None):
    """label (int32 [n]): -1 for noise, else the index of the cluster centre."""
    torch = _torch()
    n = rho.numel()
    _vec(rho, n, torch.int32, "rho")
    _vec(dep, n, torch.int32, "dep")
    _vec(delta2, n, torch.int64, "delta2")
    label = _out(label, n, torch.int32, rho.device)
    st = load().dpc_cluster(n, _ptr(rho), _ptr(dep), _ptr(delta2), int(rho_min), float(delta_min), _ptr(label),
                            _stream(stream))
    if st != OK:
        raise DPCError(st, "dpc_cluster")
    return label


def last_stats() -> dict:
    """Measurements of this thread's last run() made with time_stages/count_work."""
    s = Stats()
    st = load().dpc_last_stats(ctypes.byref(s))
    if st != OK:
        raise DPCError(st, "dpc_last_stats")
    out = {"flags": s.flags, "stage_ms": dict(zip(STAGES, list(s.stage_ms)))}
    out.update({k: getattr(s, k) for k in WORK_FIELDS})
    out["workspace_bytes"] = s.workspace_bytes
    return out


def run(points, d_cut: float, rho_min: int, delta_min: float, skip_noise: bool = False, out=None,
        stream=None, time_stages: bool = False, count_work: bool = False, fenwick: bool = False,
        pst: bool = False):
    """(rho, dep, delta2, label) of the whole method on device points.

    time_stages / count_work record per-step GPU times / work counters of
    this call for last_stats() (measurement only).  fenwick finds the
    dependent points with the Fenwick tree of k-d trees, pst with the
    priority-search k-d tree that stores one point per node, instead of the
    default k-d tree (same outputs)."""
    torch = _torch()
    n, d = _check_points(points)
    dev = points.device
    if out is None:
        out = (None, None, None, None)
    rho = _out(out[0], n, torch.int32, dev)
    dep = _out(out[1], n, torch.int32, dev)
    delta2 = _out(out[2], n, torch.int64, dev)
    label = _out(out[3], n, torch.int32, dev)
    flags = (SKIP_NOISE_DEPENDENTS if skip_noise else 0) | (TIME_STAGES if time_stages else 0) \
        | (COUNT_WORK if count_work else 0) | (FENWICK_DEPENDENTS if fenwick else 0) \
        | (PST_DEPENDENTS if pst else 0)
    st = load().dpc_run(_ptr(points), n, d, float(d_cut), int(rho_min), float(delta_min), flags, _ptr(rho),
                        _ptr(dep), _ptr(delta2), _ptr(label), _stream(stream))
    if st != OK:
        raise DPCError(st, "dpc_run")
    return rho, dep, delta2, label


def run_noalloc(points, d_cut: float, rho_min: int, delta_min: float, skip_noise: bool = False, out=None,
                stream=None):
    """dpc_run_noalloc: the whole method with the library's fixed device
    scratch instead of any allocation (outputs as for run; pass `out` to
    allocate nothing at all)."""
    torch = _torch()
    n, d = _check_points(points)
    dev = points.device
    if out is None:
        out = (None, None, None, None)
    rho = _out(out[0], n, torch.int32, dev)
    dep = _out(out[1], n, torch.int32, dev)
    delta2 = _out(out[2], n, torch.int64, dev)
    label = _out(out[3], n, torch.int32, dev)
    flags = SKIP_NOISE_DEPENDENTS if skip_noise else 0
    st = load().dpc_run_noalloc(_ptr(points), n, d, float(d_cut), int(rho_min), float(delta_min), flags,
                                _ptr(rho), _ptr(dep), _ptr(delta2), _ptr(label), _stream(stream))
    if st != OK:
        raise DPCError(st, "dpc_run_noalloc")
    return rho, dep, delta2, label


def density_sweep(points, d_cuts, out=None, stream=None):
    """rho for several radii ([len(d_cuts), n] int32), one index build."""
    torch = _torch()
    n, d = _check_points(points)
    k = len(d_cuts)
    rho = out if out is not None else torch.empty((k, n), dtype=torch.int32, device=points.device)
    if rho.dtype != torch.int32 or tuple(rho.shape) != (k, n) or not rho.is_contiguous():
        raise TypeError(f"out must be a contiguous int32 [{k}, {n}] tensor")
    arr = (ctypes.c_double * max(k, 1))(*[float(x) for x in d_cuts])
    st = load().dpc_density_sweep(_ptr(points), n, d, arr, k, _ptr(rho), _stream(stream))
    if st != OK:
        raise DPCError(st, "dpc_density_sweep")
    return rho


def cluster_sweep(rho, dep, delta2, pairs, out=None, stream=None):
    """Labels for several (rho_min, delta_min) pairs ([len(pairs), n] int32)."""
    torch = _torch()
    n = rho.numel()
    k = len(pairs)
    label = out if out is not None else torch.empty((k, n), dtype=torch.int32, device=rho.device)
    if label.dtype != torch.int32 or tuple(label.shape) != (k, n) or not label.is_contiguous():
        raise TypeError(f"out must be a contiguous int32 [{k}, {n}] tensor")
    rm = (ctypes.c_int32 * max(k, 1))(*[int(p[0]) for p in pairs])
    dm = (ctypes.c_double * max(k, 1))(*[float(p[1]) for p in pairs])
    st = load().dpc_cluster_sweep(n, _ptr(rho), _ptr(dep), _ptr(delta2), rm, dm, k, _ptr(label), _stream(stream))
    if st != OK:
        raise DPCError(st, "dpc_cluster_sweep")
    return label


class Batch:
    """A prepared dpc_batch_run call: the instance records are built once, so
    that repeated calls on the same tensors marshal nothing.

    problems: sequence of (points, d_cut, rho_min, delta_min) with points an
    int32 [n, d] device tensor; outs (optional) supplies the output tensors
    [(rho, dep, delta2, label), ...].  The tensors must stay alive while the
    batch is used."""

    def __init__(self, problems, skip_noise: bool = False, outs=None):
        torch = _torch()
        self.count = len(problems)
        self.recs = (Instance * max(self.count, 1))()
        self.flags = SKIP_NOISE_DEPENDENTS if skip_noise else 0
        self.points = []
        self.results = []
        for i, (points, d_cut, rho_min, delta_min) in enumerate(problems):
            n, d = _check_points(points)
            dev = points.device
            o = outs[i] if outs is not None else (None, None, None, None)
            rho = _out(o[0], n, torch.int32, dev)
            dep = _out(o[1], n, torch.int32, dev)
            delta2 = _out(o[2], n, torch.int64, dev)
            label = _out(o[3], n, torch.int32, dev)
            self.recs[i] = Instance(_ptr(points).value, n, d, float(d_cut), int(rho_min), float(delta_min),
                                    _ptr(rho).value, _ptr(dep).value, _ptr(delta2).value, _ptr(label).value, -1)
            self.points.append(points)
            self.results.append((rho, dep, delta2, label))

    def run(self, stream=None, check: bool = True):
        """One dpc_batch_run over every instance; returns the call's status
        (raises on failure with check)."""
        st = load().dpc_batch_run(self.recs, self.count, self.flags, _stream(stream))
        if check and st != OK:
            raise DPCError(st, "dpc_batch_run")
        return st

    def statuses(self):
        return [self.recs[i].status for i in range(self.count)]


def batch_run(problems, skip_noise: bool = False, outs=None, stream=None, check: bool = True):
    """Runs many independent instances in one call.

    problems: sequence of (points, d_cut, rho_min, delta_min) with points an
    int32 [n, d] device tensor.  Returns [(rho, dep, delta2, label), ...] and
    the per-instance statuses.  outs (optional) supplies the output tensors.
    With check, a failing instance raises."""
    b = Batch(problems, skip_noise, outs)
    b.run(stream, check)
    return b.results, b.statuses()


def workspace_bytes(n: int, d: int) -> int:
    """Upper bound on the device workspace of one instance (dpc_workspace_bytes)."""
    return int(load().dpc_workspace_bytes(int(n), int(d)))


def _info(ri) -> dict:
    return {f: getattr(ri, f) for f, _ in RequestInfo._fields_}


class Server:
    """A dpc_server: requests are queued with submit() and run in batches on
    `slots` streams as the HBM budget allows (see include/libdpc.h).

    The tensors of a request are kept referenced until its result has been
    collected with poll() or wait()."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 2, max_batch: int = 64):
        self._h = ctypes.c_void_p()
        cfg = ServerConfig(int(hbm_budget_bytes), int(slots), int(max_batch))
        st = load().dpc_server_create(ctypes.byref(cfg), ctypes.byref(self._h))
        if st != OK:
            raise DPCError(st, "dpc_server_create")
        self._keep = {}

    def submit(self, points, d_cut: float, rho_min: int, delta_min: float, out=None, skip_noise: bool = False):
        """Queues one request; returns (ticket, (rho, dep, delta2, label))."""
        torch = _torch()
        n, d = _check_points(points)
        dev = points.device
        o = out if out is not None else (None, None, None, None)
        res = (_out(o[0], n, torch.int32, dev), _out(o[1], n, torch.int32, dev), _out(o[2], n, torch.int64, dev),
               _out(o[3], n, torch.int32, dev))
        rec = Instance(_ptr(points).value, n, d, float(d_cut), int(rho_min), float(delta_min), _ptr(res[0]).value,
                       _ptr(res[1]).value, _ptr(res[2]).value, _ptr(res[3]).value, -1)
        t = ctypes.c_uint64()
        st = load().dpc_server_submit(self._h, ctypes.byref(rec), SKIP_NOISE_DEPENDENTS if skip_noise else 0,
                                      ctypes.byref(t))
        if st != OK:
            raise DPCError(st, "dpc_server_submit")
        self._keep[t.value] = (points, res)
        return t.value, res

    def poll(self, ticket: int):
        """The request's state (a dict; 'done' 0 or 1) without blocking."""
        ri = RequestInfo()
        st = load().dpc_server_poll(self._h, ticket, ctypes.byref(ri))
        if st != OK:
            raise DPCError(st, "dpc_server_poll")
        if ri.done:
            self._keep.pop(ticket, None)
        return _info(ri)

    def wait(self, ticket: int) -> dict:
        """Blocks until the request is done; returns its state."""
        ri = RequestInfo()
        st = load().dpc_server_wait(self._h, ticket, ctypes.byref(ri))
        if st != OK:
            raise DPCError(st, "dpc_server_wait")
        self._keep.pop(ticket, None)
        return _info(ri)

    def stats(self) -> dict:
        ss = ServerStats()
        st = load().dpc_server_get_stats(self._h, ctypes.byref(ss))
        if st != OK:
            raise DPCError(st, "dpc_server_get_stats")
        return {f: getattr(ss, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            st = load().dpc_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()
            if st != OK:
                raise DPCError(st, "dpc_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Plan:
    """A dpc_plan: run() recorded once on `points` and the output tensors,
    then replayed with launch() (optionally as a HIP graph after capture())
    on the current contents of `points` (see include/libdpc.h)."""

    def __init__(self, points, d_cut: float, rho_min: int, delta_min: float, skip_noise: bool = False, out=None,
                 stream=None):
        torch = _torch()
        n, d = _check_points(points)
        dev = points.device
        o = out if out is not None else (None, None, None, None)
        self.out = (_out(o[0], n, torch.int32, dev), _out(o[1], n, torch.int32, dev),
                    _out(o[2], n, torch.int64, dev), _out(o[3], n, torch.int32, dev))
        self.points = points
        self._h = ctypes.c_void_p()
        st = load().dpc_plan_create(_ptr(points), n, d, float(d_cut), int(rho_min), float(delta_min),
                                    SKIP_NOISE_DEPENDENTS if skip_noise else 0, _ptr(self.out[0]),
                                    _ptr(self.out[1]), _ptr(self.out[2]), _ptr(self.out[3]), _stream(stream),
                                    ctypes.byref(self._h))
        if st != OK:
            raise DPCError(st, "dpc_plan_create")

    def launch(self, stream=None):
        """Enqueues one replay; returns the output tensors."""
        st = load().dpc_plan_launch(self._h, _stream(stream))
        if st != OK:
            raise DPCError(st, "dpc_plan_launch")
        return self.out

    def capture(self, stream=None):
        """Captures the replay into a HIP graph on a non-default stream."""
        torch = _torch()
        if stream is None:
            stream = torch.cuda.Stream()
        st = load().dpc_plan_capture(self._h, _stream(stream))
        if st != OK:
            raise DPCError(st, "dpc_plan_capture")

    def status(self, stream=None) -> int:
        """The last replay's status (OK, or ERR_RANGE if the points left the
        planned bounds); waits for `stream`."""
        v = ctypes.c_int32()
        st = load().dpc_plan_status(self._h, _stream(stream), ctypes.byref(v))
        if st != OK:
            raise DPCError(st, "dpc_plan_status")
        return v.value

    def close(self):
        if self._h:
            st = load().dpc_plan_destroy(self._h)
            self._h = ctypes.c_void_p()
            if st != OK:
                raise DPCError(st, "dpc_plan_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class BatchPlan(Plan):
    """A dpc_plan of a whole batch: batch_run() recorded once on the
    problems' point tensors and the output tensors, then replayed with
    launch() (optionally as a HIP graph after capture()).  results holds the
    outputs per problem."""

    def __init__(self, problems, skip_noise: bool = False, outs=None, stream=None):
        self._b = Batch(problems, skip_noise, outs)
        self.results = self._b.results
        self.out = self.results
        self._h = ctypes.c_void_p()
        st = load().dpc_plan_create_batch(self._b.recs, self._b.count, self._b.flags, _stream(stream),
                                          ctypes.byref(self._h))
        if st != OK:
            raise DPCError(st, "dpc_plan_create_batch")

    def statuses(self):
        return self._b.statuses()


LEAF_SIZES = (16, 32, 64)


def set_leaf_size(d: int, leaf_points: int) -> None:
    """Points per k-d tree leaf (16, 32 or 64) for dimension d; never changes outputs."""
    st = load().dpc_set_leaf_size(int(d), int(leaf_points))
    if st != OK:
        raise DPCError(st, "dpc_set_leaf_size")


def leaf_size(d: int) -> int:
    return int(load().dpc_leaf_size(int(d)))


def autotune(points, d_cut: float, rho_min: int, delta_min: float, stream=None) -> dict:
    """Times every leaf size on this instance and keeps the fastest for its
    dimension; returns {"ms": {16: t16, 32: t32, 64: t64}, "chosen": size}."""
    n, d = _check_points(points)
    ms = (ctypes.c_double * len(LEAF_SIZES))()
    ch = ctypes.c_int32()
    st = load().dpc_autotune(_ptr(points), n, d, float(d_cut), int(rho_min), float(delta_min), _stream(stream), ms,
                             ctypes.byref(ch))
    if st != OK:
        raise DPCError(st, "dpc_autotune")
    return {"ms": {size: ms[c] for c, size in enumerate(LEAF_SIZES)}, "chosen": ch.value}


def set_dependent_backend(d: int, backend: str) -> None:
    """Dependent-point backend dpc_run uses for dimension d: "priority_tree"
    or "fenwick" (same outputs)."""
    if backend not in BACKENDS:
        raise ValueError(f"backend must be one of {BACKENDS}")
    st = load().dpc_set_dependent_backend(int(d), BACKENDS.index(backend))
    if st != OK:
        raise DPCError(st, "dpc_set_dependent_backend")


def dependent_backend(d: int) -> str:
    b = load().dpc_dependent_backend(int(d))
    if b < 0:
        raise DPCError(ERR_INVALID_ARG, "dpc_dependent_backend")
    return BACKENDS[b]


def autotune_dependent(points, d_cut: float, rho_min: int, delta_min: float, stream=None) -> dict:
    """Times every dependent-point backend on this instance and keeps the
    fastest for its dimension; returns {"ms": {backend: t}, "chosen": backend}."""
    n, d = _check_points(points)
    ms = (ctypes.c_double * len(BACKENDS))()
    ch = ctypes.c_int32()
    st = load().dpc_autotune_dependent(_ptr(points), n, d, float(d_cut), int(rho_min), float(delta_min),
                                       _stream(stream), ms, ctypes.byref(ch))
    if st != OK:
        raise DPCError(st, "dpc_autotune_dependent")
    return {"ms": {b: ms[i] for i, b in enumerate(BACKENDS)}, "chosen": BACKENDS[ch.value]}

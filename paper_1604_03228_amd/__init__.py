"""Python binding of libkcenter: the k-center hot path of McClintock & Wirth,
"Efficient Parallel Algorithms for k-Center Clustering" (arXiv 1604.03228),
on AMD MI355X (gfx950).

This module only marshals arguments: torch tensors (device memory and the
current HIP stream) go to the C ABI of ``libkcenter.so``
(``include/kcenter.h``) as plain pointers; every step of the computation runs
in the library's HIP kernels.  If the library is missing the import of any
entry point raises -- there is no CPU fallback.
"""
import atexit
import ctypes
import os
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkcenter.so")

KC_FP32 = 0
KC_BF16_RESCORE = 1
ALGO_GON, ALGO_MRG, ALGO_EIM = 0, 1, 2

_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


class KcPoints(ctypes.Structure):
    _fields_ = [("f32", _p), ("bf16", _p), ("n", _i64), ("d", _i32),
                ("ld", _i64), ("prec", _i32)]


class KcEimParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("phi", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("max_iters", _i32)]


class KcEimIter(ctypes.Structure):
    _fields_ = [("r_size", _i64), ("ds_size", _i64), ("h_size", _i64),
                ("s_size", _i64), ("tau", ctypes.c_double),
                ("p_s", ctypes.c_double), ("p_h", ctypes.c_double)]


class KcProblem(ctypes.Structure):
    _fields_ = [("pts", KcPoints), ("algo", _i32), ("k", _i64),
                ("first", _i64), ("offsets", _p), ("m", _i32),
                ("eim", KcEimParams), ("centers", _p), ("n_centers", _p),
                ("radius", _p)]


class KCenterError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("kcenter status %d: %s" % (status, msg))
        self.status = status


EXPORTS = ["kc_create", "kc_destroy", "kc_strerror", "kc_last_error",
           "kc_set_option", "kc_device_status", "kc_timing_read",
           "kc_counter_read", "kc_tune_report",
           "kcenter_gonzalez", "kcenter_gonzalez_noalloc",
           "kcenter_gonzalez_resume",
           "kcenter_mrg", "kcenter_mrg_rounds", "kcenter_assign", "kcenter_eim",
           "kcenter_batch", "kcenter_batch_plan", "kcenter_batch_run",
           "kcenter_batch_free"]

_lib = None


def load_library(path=LIB_PATH):
    """Load libkcenter.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libkcenter.so not built: run "
                          "`python -m paper_1604_03228_amd.build`")
    L = ctypes.CDLL(path)
    L.kc_create.argtypes = [ctypes.POINTER(_p)]
    L.kc_destroy.argtypes = [_p]
    L.kc_destroy.restype = None
    L.kc_strerror.argtypes = [ctypes.c_int]
    L.kc_strerror.restype = ctypes.c_char_p
    L.kc_last_error.argtypes = [_p]
    L.kc_last_error.restype = ctypes.c_char_p
    L.kc_set_option.argtypes = [_p, ctypes.c_char_p, _i64]
    L.kc_device_status.argtypes = [_p, _p, ctypes.POINTER(ctypes.c_uint32)]
    L.kc_timing_read.argtypes = [_p, ctypes.c_char_p,
                                 ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
    L.kc_counter_read.argtypes = [_p, ctypes.c_char_p, ctypes.POINTER(_i64)]
    L.kc_tune_report.argtypes = [_p, ctypes.c_char_p, _i64,
                                 ctypes.POINTER(_i64)]
    L.kcenter_gonzalez.argtypes = [_p, ctypes.POINTER(KcPoints), _i64, _i64,
                                   _p, _p, _p, _p]
    L.kcenter_gonzalez_noalloc.argtypes = [_p, ctypes.POINTER(KcPoints),
                                           _i64, _i64, _p, _p, _p, _p]
    L.kcenter_gonzalez_resume.argtypes = [_p, ctypes.POINTER(KcPoints), _p,
                                          _i64, _i64, _p, _p, _p, _p]
    L.kcenter_mrg.argtypes = [_p, ctypes.POINTER(KcPoints), _p, _i32, _i64,
                              _p, _p, _p, _p, _p, _p, _p, _p, _p]
    L.kcenter_mrg_rounds.argtypes = [_p, ctypes.POINTER(KcPoints), _i64, _i64,
                                     _p, _p, _p, ctypes.POINTER(_i32), _p]
    L.kcenter_assign.argtypes = [_p, ctypes.POINTER(KcPoints), _p, _i64, _p,
                                 _p, _p]
    L.kcenter_eim.argtypes = [_p, ctypes.POINTER(KcPoints), _i64,
                              ctypes.POINTER(KcEimParams), _p, _p, _p, _p,
                              ctypes.POINTER(_i64), _p,
                              ctypes.POINTER(_i32), _p]
    L.kcenter_batch.argtypes = [_p, _p, _i32, _p]
    L.kcenter_batch_plan.argtypes = [_p, _p, _i32, ctypes.POINTER(_p)]
    L.kcenter_batch_run.argtypes = [_p, _p, _p]
    L.kcenter_batch_free.argtypes = [_p]
    L.kcenter_batch_free.restype = None
    for name in ("kc_create", "kc_set_option", "kc_device_status",
                 "kc_timing_read", "kc_counter_read", "kc_tune_report",
                 "kcenter_gonzalez", "kcenter_gonzalez_noalloc",
                 "kcenter_gonzalez_resume",
                 "kcenter_mrg", "kcenter_mrg_rounds",
                 "kcenter_assign",
                 "kcenter_eim", "kcenter_batch", "kcenter_batch_plan",
                 "kcenter_batch_run"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _stream():
    return _p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return _p(t.data_ptr()) if t is not None else None


_live = weakref.WeakSet()


@atexit.register
def _close_all():
    """Release every live handle while the HIP runtime is still up.  Python's
    exit handlers run before the C runtime's; a handle still holding
    instantiated graphs, events and device buffers when the runtime (or a
    profiler wrapping it) tears down would otherwise be released after the
    library's code objects are gone."""
    hs = list(_live)
    if not hs:
        return
    try:
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for h in hs:
        try:
            h.close()
        except Exception:
            pass


class Handle:
    """Owns a kc_handle (workspace, captured graphs) on the current device."""

    def __init__(self, graphs=True, resident=True):
        L = load_library()
        h = _p()
        rc = L.kc_create(ctypes.byref(h))
        if rc != 0:
            raise KCenterError(rc, L.kc_strerror(rc).decode())
        self._h = h
        _live.add(self)
        self.set_option("graphs", int(graphs))
        self.set_option("resident", int(resident))

    def close(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            load_library().kc_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise KCenterError(rc, load_library().kc_last_error(self._h)
                               .decode())

    def set_option(self, name, value):
        self._check(load_library().kc_set_option(self._h, name.encode(),
                                                 int(value)))

    def timing_read(self, name):
        """(milliseconds, kernel launches, intervals) recorded under `name`
        since the last read (needs option timing=1); synchronises."""
        ms = ctypes.c_double(0)
        la = _i64(0)
        iv = _i64(0)
        self._check(load_library().kc_timing_read(
            self._h, name.encode(), ctypes.byref(ms), ctypes.byref(la),
            ctypes.byref(iv)))
        return ms.value, la.value, iv.value

    def counter(self, name):
        """A work counter of the last BF16 run (see kc_counter_read)."""
        v = _i64(0)
        self._check(load_library().kc_counter_read(self._h, name.encode(),
                                                   ctypes.byref(v)))
        return v.value

    def tune_report(self):
        """The autotuner's choices: {key: (variant, [ms per variant])}."""
        L = load_library()
        need = _i64(0)
        L.kc_tune_report(self._h, None, 0, ctypes.byref(need))
        buf = ctypes.create_string_buffer(max(int(need.value), 1))
        self._check(L.kc_tune_report(self._h, buf, len(buf), ctypes.byref(need)))
        out = {}
        for line in buf.value.decode().splitlines():
            f = line.split()
            out[f[0]] = (int(f[1]), [float(x) for x in f[2:]])
        return out

    def device_status(self):
        """Synchronise the current stream and read/clear the status word."""
        w = ctypes.c_uint32(0)
        rc = load_library().kc_device_status(self._h, _stream(),
                                             ctypes.byref(w))
        if rc not in (0, -7):
            self._check(rc)
        return w.value


def points(X, bf16=None):
    """Describe a CUDA FP32 tensor [n, d] (row-major, rows may be strided)
    and an optional BF16 copy (int16/uint16 bits or torch.bfloat16) of the
    same shape and row stride."""
    if not (isinstance(X, torch.Tensor) and X.is_cuda and
            X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1):
        raise ValueError("points: need a CUDA float32 [n, d] tensor with "
                         "unit column stride")
    p = KcPoints()
    p.f32 = X.data_ptr()
    p.n, p.d = X.shape
    p.ld = X.stride(0)
    p.prec = KC_FP32
    p.bf16 = None
    if bf16 is not None:
        if bf16.shape != X.shape or bf16.stride(0) != X.stride(0) or \
                bf16.element_size() != 2 or not bf16.is_cuda:
            raise ValueError("bf16 copy must match the FP32 layout")
        p.bf16 = bf16.data_ptr()
        p.prec = KC_BF16_RESCORE
    return p


_default = None


def default_handle():
    global _default
    if _default is None:
        _default = Handle()
    return _default


def gonzalez(X, k, first=0, bf16=None, handle=None, out=None):
    """Gonzalez's traversal.  Returns (centers int64[k], radius_trace f64[k],
    n_chosen int64[1]) as CUDA tensors (asynchronous)."""
    h = handle or default_handle()
    dev = X.device
    if out is None:
        out = (torch.empty(k, dtype=torch.int64, device=dev),
               torch.empty(k, dtype=torch.float64, device=dev),
               torch.empty(1, dtype=torch.int64, device=dev))
    centers, trace, nch = out
    p = points(X, bf16)
    h._check(load_library().kcenter_gonzalez(
        h._h, ctypes.byref(p), int(k), int(first), _ptr(centers),
        _ptr(trace), _ptr(nch), _stream()))
    return centers, trace, nch


def gonzalez_resume(X, prefix, k, handle=None):
    """Gonzalez's traversal with its first centers forced to `prefix` (a host
    sequence of distinct indices, e.g. the first p centers of an earlier
    run), continued to k centers.  Returns (centers int64[k], trace f64[k],
    n_chosen int64[1]) as CUDA tensors (asynchronous)."""
    import numpy as np
    h = handle or default_handle()
    dev = X.device
    pre = np.ascontiguousarray(np.asarray(prefix, dtype=np.int64))
    out = (torch.empty(k, dtype=torch.int64, device=dev),
           torch.empty(k, dtype=torch.float64, device=dev),
           torch.empty(1, dtype=torch.int64, device=dev))
    p = points(X, None)
    h._check(load_library().kcenter_gonzalez_resume(
        h._h, ctypes.byref(p), pre.ctypes.data_as(_p), len(pre), int(k),
        _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _stream()))
    return out


def gonzalez_noalloc(X, k, first=0, handle=None, out=None):
    """Gonzalez's traversal through the entry point that allocates no device
    memory (its workspace is the library's fixed per-GPU array).  `out`, if
    given, is (centers int64[k], trace f64[k], n_chosen int64[1]); with it
    the call allocates nothing.  Returns those tensors (asynchronous)."""
    h = handle or default_handle()
    dev = X.device
    if out is None:
        out = (torch.empty(k, dtype=torch.int64, device=dev),
               torch.empty(k, dtype=torch.float64, device=dev),
               torch.empty(1, dtype=torch.int64, device=dev))
    centers, trace, nch = out
    p = points(X, None)
    h._check(load_library().kcenter_gonzalez_noalloc(
        h._h, ctypes.byref(p), int(k), int(first), _ptr(centers),
        _ptr(trace), _ptr(nch), _stream()))
    return centers, trace, nch


def mrg(X, offsets, k, bf16=None, handle=None, details=False):
    """Two-round MRG.  offsets: host sequence of m+1 ints.  Returns
    (centers, n_centers, radius) and, with details, a dict of round1, r1,
    union, n_union, r2."""
    import numpy as np
    h = handle or default_handle()
    dev = X.device
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    m = len(off) - 1
    centers = torch.empty(k, dtype=torch.int64, device=dev)
    nc = torch.empty(1, dtype=torch.int64, device=dev)
    radius = torch.empty(1, dtype=torch.float64, device=dev)
    extra = None
    if details:
        extra = dict(round1=torch.empty(m * k, dtype=torch.int64, device=dev),
                     r1=torch.empty(m, dtype=torch.float64, device=dev),
                     union=torch.empty(max(m * k, 1), dtype=torch.int64,
                                       device=dev),
                     n_union=torch.empty(1, dtype=torch.int64, device=dev),
                     r2=torch.empty(1, dtype=torch.float64, device=dev))
    p = points(X, bf16)
    g = (lambda n: _ptr(extra[n])) if details else (lambda n: None)
    h._check(load_library().kcenter_mrg(
        h._h, ctypes.byref(p), off.ctypes.data_as(_p), m, int(k),
        _ptr(centers), _ptr(nc), _ptr(radius), g("round1"), g("r1"),
        g("union"), g("n_union"), g("r2"), _stream()))
    if details:
        return centers, nc, radius, extra
    return centers, nc, radius


def mrg_rounds(X, k, capacity, handle=None):
    """Multi-round MRG with per-machine capacity.  Returns (centers,
    n_centers, radius) CUDA tensors and the number of rounds (host int);
    reads |S| once per pass."""
    h = handle or default_handle()
    dev = X.device
    centers = torch.empty(k, dtype=torch.int64, device=dev)
    nc = torch.empty(1, dtype=torch.int64, device=dev)
    radius = torch.empty(1, dtype=torch.float64, device=dev)
    rounds = _i32(0)
    p = points(X, None)
    h._check(load_library().kcenter_mrg_rounds(
        h._h, ctypes.byref(p), int(k), int(capacity), _ptr(centers), _ptr(nc),
        _ptr(radius), ctypes.byref(rounds), _stream()))
    return centers, nc, radius, rounds.value


def assign(X, centers, bf16=None, labels=True, handle=None):
    """Nearest-center labels (int32[n] or None) and exact radius f64[1]."""
    h = handle or default_handle()
    dev = X.device
    centers = centers.to(device=dev, dtype=torch.int64).contiguous()
    lab = torch.empty(X.shape[0], dtype=torch.int32, device=dev) \
        if labels else None
    radius = torch.empty(1, dtype=torch.float64, device=dev)
    p = points(X, bf16)
    h._check(load_library().kcenter_assign(
        h._h, ctypes.byref(p), _ptr(centers), centers.numel(), _ptr(lab),
        _ptr(radius), _stream()))
    return lab, radius


def eim(X, k, eps, phi, seed, max_iters=64, bf16=None, want_sample=True,
        handle=None):
    """EIM sampling pass + Gonzalez on the sample.  Returns (centers,
    n_centers, radius, sample or None, iteration records).  Synchronises
    the stream once per iteration."""
    h = handle or default_handle()
    dev = X.device
    n = X.shape[0]
    centers = torch.empty(k, dtype=torch.int64, device=dev)
    nc = torch.empty(1, dtype=torch.int64, device=dev)
    radius = torch.empty(1, dtype=torch.float64, device=dev)
    sample = torch.empty(n, dtype=torch.int64, device=dev) \
        if want_sample else None
    prm = KcEimParams(float(eps), float(phi), int(seed), int(max_iters))
    iters = (KcEimIter * max(1, max_iters))()
    ns = _i64(0)
    ni = _i32(0)
    p = points(X, bf16)
    h._check(load_library().kcenter_eim(
        h._h, ctypes.byref(p), int(k), ctypes.byref(prm), _ptr(centers),
        _ptr(nc), _ptr(radius), _ptr(sample), ctypes.byref(ns),
        ctypes.cast(iters, _p), ctypes.byref(ni), _stream()))
    recs = [dict(r_size=it.r_size, ds_size=it.ds_size, h_size=it.h_size,
                 s_size=it.s_size, tau=it.tau, p_s=it.p_s, p_h=it.p_h)
            for it in iters[:ni.value]]
    if sample is not None:
        sample = sample[:ns.value]
    return centers, nc, radius, sample, recs


def _problem_array(problems):
    """The kc_problem array of a list of problem dicts, the output tensors
    and the host arrays the array points into."""
    import numpy as np
    arr = (KcProblem * len(problems))()
    keep = []
    outs = []
    for i, pr in enumerate(problems):
        X = pr["X"]
        dev = X.device
        k = int(pr["k"])
        c = torch.empty(k, dtype=torch.int64, device=dev)
        nc = torch.empty(1, dtype=torch.int64, device=dev)
        r = torch.empty(1, dtype=torch.float64, device=dev)
        outs.append((c, nc, r))
        q = arr[i]
        q.pts = points(X, pr.get("bf16"))
        q.algo = {"gon": ALGO_GON, "mrg": ALGO_MRG, "eim": ALGO_EIM}[pr["algo"]]
        q.k = k
        q.first = int(pr.get("first", 0))
        if pr["algo"] == "mrg":
            off = np.ascontiguousarray(np.asarray(pr["offsets"], np.int64))
            keep.append(off)
            q.offsets = off.ctypes.data
            q.m = len(off) - 1
        if pr["algo"] == "eim":
            q.eim = KcEimParams(float(pr["eps"]), float(pr["phi"]),
                                int(pr["seed"]), int(pr.get("max_iters", 64)))
        q.centers = c.data_ptr()
        q.n_centers = nc.data_ptr()
        q.radius = r.data_ptr()
    return arr, outs, keep


def batch(problems, handle=None):
    """Solve independent problems.  Each entry is a dict with X (CUDA
    FP32), algo ('gon' | 'mrg' | 'eim'), k, and first / offsets / eps,
    phi, seed as the algorithm needs.  Returns a list of (centers,
    n_centers, radius) CUDA tensors."""
    h = handle or default_handle()
    arr, outs, keep = _problem_array(problems)
    h._check(load_library().kcenter_batch(h._h, ctypes.cast(arr, _p),
                                          len(problems), _stream()))
    return outs


class BatchPlan:
    """A batch planned once (kcenter_batch_plan) and run many times
    (kcenter_batch_run on the current stream).  `outs` holds the (centers,
    n_centers, radius) tensors every run writes; the problems' point tensors
    must stay alive and unchanged in shape."""

    def __init__(self, problems, handle=None):
        self.handle = handle or default_handle()
        arr, self.outs, _ = _problem_array(problems)
        self._points = [pr["X"] for pr in problems]
        pl = _p()
        self.handle._check(load_library().kcenter_batch_plan(
            self.handle._h, ctypes.cast(arr, _p), len(problems),
            ctypes.byref(pl)))
        self._plan = pl
        _live.add(self)

    def run(self):
        self.handle._check(load_library().kcenter_batch_run(
            self.handle._h, self._plan, _stream()))
        return self.outs

    def close(self):
        if getattr(self, "_plan", None):
            pl, self._plan = self._plan, None
            load_library().kcenter_batch_free(pl)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

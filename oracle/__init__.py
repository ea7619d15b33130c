"""FP64 CPU oracle for the k-center hot path (arXiv 1604.03228).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product library never
imports, links or calls anything here.

This module is a thin ctypes layer over ``kc_oracle.c``; every function
converts numpy inputs and returns numpy outputs.  The arithmetic lives in the
C file (plain FP64, one point per loop iteration, no blocking).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kc_oracle.c")
_LIB = os.path.join(_HERE, "libkc_oracle.so")

_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_p = ctypes.c_void_p


class EimIter(ctypes.Structure):
    _fields_ = [("r_size", _i64), ("ds_size", _i64), ("h_size", _i64),
                ("s_size", _i64), ("tau", _f64), ("p_s", _f64),
                ("p_h", _f64)]


def build():
    """Compile the oracle with gcc (FP contraction off, OpenMP on)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-o", _LIB, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or (
                os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_gon.argtypes = [_p, _i64, ctypes.c_int, _i64, _i64, _i64, _p,
                              _p, _p]
        L.orc_gon.restype = _i64
        L.orc_gon_replay.argtypes = [_p, _i64, ctypes.c_int, _i64, _i64, _p,
                                     _i64, _f64, _p, _p]
        L.orc_gon_replay.restype = _i64
        L.orc_assign.argtypes = [_p, _i64, ctypes.c_int, _i64, _p, _i64, _p,
                                 _p]
        L.orc_assign.restype = _f64
        L.orc_mrg.argtypes = [_p, _i64, ctypes.c_int, _i64, _p, ctypes.c_int,
                              _i64, _p, _p, _p, _p, _p, _p, _p]
        L.orc_mrg.restype = _f64
        L.orc_mrg_rounds.argtypes = [_p, _i64, ctypes.c_int, _i64, _i64, _i64,
                                     _p, _p, _p, _p, _p]
        L.orc_gon_resume.argtypes = [_p, _i64, ctypes.c_int, _i64, _i64, _p,
                                     _i64, _p, _p]
        L.orc_gon_resume.restype = _i64
        L.orc_mrg_rounds.restype = _f64
        L.orc_philox4x64_10.argtypes = [_p, _p, _p]
        L.orc_philox4x64_10.restype = None
        L.orc_eim.argtypes = [_p, _i64, ctypes.c_int, _i64, _i64, _f64, _f64,
                              ctypes.c_uint64, ctypes.c_int, _p, _p, _p, _p,
                              _p, _p, _p, _p, _p, _p]
        L.orc_eim_uniform_pair.argtypes = [ctypes.c_uint64, _i64,
                                           ctypes.c_int, _p]
        L.orc_eim_uniform_pair.restype = None
        L.orc_eim_draw_flags.argtypes = [ctypes.c_uint64, ctypes.c_int, _p,
                                         _i64, _f64, _f64, _p]
        L.orc_eim_draw_flags.restype = _i64
        L.orc_min_dist2_to_set.argtypes = [_p, ctypes.c_int, _i64, _i64, _p,
                                           _i64, _p]
        L.orc_min_dist2_to_set.restype = _f64
        L.orc_eim.restype = _f64
        L.orc_opt_bruteforce.argtypes = [_p, _i64, ctypes.c_int, _i64, _i64]
        L.orc_opt_bruteforce.restype = _f64
        _lib = L
    return _lib


def set_threads(t):
    """Threads for the per-point loops; returns the count in force."""
    return lib().orc_set_threads(int(t))


def _pts(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    assert X.ndim == 2
    return X, X.shape[0], X.shape[1]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def gon(X, k, first=0, want_mind=False):
    """Gonzalez (Section 3.1).  Returns (centers[k], trace[k], n_chosen)
    and, if asked, the final squared min-distances."""
    X, n, d = _pts(X)
    centers = np.full(k, -1, np.int64)
    trace = np.zeros(k, np.float64)
    mind = np.zeros(n, np.float64) if want_mind else None
    got = lib().orc_gon(_ptr(X), n, d, d, k, first, _ptr(centers),
                        _ptr(trace), _ptr(mind) if want_mind else None)
    if got < 0:
        raise MemoryError("oracle gon")
    if want_mind:
        return centers, trace, int(got), mind
    return centers, trace, int(got)


def gon_replay(X, k, seq, band):
    """Replay a center sequence; see orc_gon_replay.  Returns
    (first_bad_step or -1, n_certified_ties, oracle trace along seq)."""
    X, n, d = _pts(X)
    seq = np.ascontiguousarray(seq, dtype=np.int64)
    trace = np.zeros(max(len(seq), 1), np.float64)
    ties = ctypes.c_int64(0)
    bad = lib().orc_gon_replay(_ptr(X), n, d, d, k, _ptr(seq), len(seq),
                               float(band), _ptr(trace), ctypes.byref(ties))
    return int(bad), int(ties.value), trace[:len(seq)]


def assign(X, centers, want_mind=False):
    """Nearest-center labels (lowest position on ties) and covering radius."""
    X, n, d = _pts(X)
    centers = np.ascontiguousarray(centers, dtype=np.int64)
    labels = np.zeros(n, np.int32)
    mind = np.zeros(n, np.float64) if want_mind else None
    R = lib().orc_assign(_ptr(X), n, d, d, _ptr(centers), len(centers),
                         _ptr(labels), _ptr(mind) if want_mind else None)
    if want_mind:
        return labels, R, mind
    return labels, R


def mrg(X, offsets, k):
    """Two-round MRG (Algorithm 1).  Returns a dict."""
    X, n, d = _pts(X)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    m = len(offsets) - 1
    centers = np.full(k, -1, np.int64)
    nc = ctypes.c_int64(0)
    round1 = np.full(m * k, -1, np.int64)
    r1 = np.zeros(m, np.float64)
    uni = np.zeros(max(m * k, 1), np.int64)
    nu = ctypes.c_int64(0)
    r2 = ctypes.c_double(0)
    R = lib().orc_mrg(_ptr(X), n, d, d, _ptr(offsets), m, k, _ptr(centers),
                      ctypes.byref(nc), _ptr(round1), _ptr(r1), _ptr(uni),
                      ctypes.byref(nu), ctypes.byref(r2))
    return dict(centers=centers, n_centers=int(nc.value), radius=R,
                round1=round1.reshape(m, k), r1=r1,
                union=uni[:nu.value].copy(), r2=r2.value)


def mrg_rounds(X, k, capacity):
    """Multi-round MRG (Algorithm 1 with its loop, Lemma 3).  `sample` is the
    set S the last round runs on."""
    X, n, d = _pts(X)
    centers = np.full(k, -1, np.int64)
    nc = ctypes.c_int64(0)
    rounds = ctypes.c_int(0)
    s_out = np.zeros(n, np.int64)
    ns = ctypes.c_int64(0)
    R = lib().orc_mrg_rounds(_ptr(X), n, d, d, k, capacity, _ptr(centers),
                             ctypes.byref(nc), ctypes.byref(rounds),
                             _ptr(s_out), ctypes.byref(ns))
    return dict(centers=centers, n_centers=int(nc.value), radius=R,
                rounds=rounds.value, sample=s_out[:ns.value].copy())


def gon_resume(X, k, prefix):
    """Gonzalez with centers 0..p-1 forced to `prefix`, then continued to k.
    Returns (centers[k], trace[k], n_chosen); raises on an invalid prefix."""
    X, n, d = _pts(X)
    prefix = np.ascontiguousarray(prefix, dtype=np.int64)
    centers = np.full(k, -1, np.int64)
    trace = np.zeros(k, np.float64)
    got = lib().orc_gon_resume(_ptr(X), n, d, d, k, _ptr(prefix), len(prefix),
                               _ptr(centers), _ptr(trace))
    if got < 0:
        raise ValueError("oracle gon_resume: invalid prefix")
    return centers, trace, int(got)


def philox4x64_10(ctr, key):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint64)
    key = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_ptr(ctr), _ptr(key), _ptr(out))
    return out


def eim(X, k, eps, phi, seed, max_iters=64):
    """EIM (Algorithms 2 and 3 with the Section 4.1 changes) plus Gonzalez
    on the sample.  Returns a dict (radius -1 when it did not converge)."""
    X, n, d = _pts(X)
    centers = np.full(k, -1, np.int64)
    nc = ctypes.c_int64(0)
    sample = np.zeros(n, np.int64)
    ns = ctypes.c_int64(0)
    sset = np.zeros(n, np.int64)
    nss = ctypes.c_int64(0)
    rset = np.zeros(n, np.int64)
    nrs = ctypes.c_int64(0)
    iters = (EimIter * max(max_iters, 1))()
    ni = ctypes.c_int(0)
    R = lib().orc_eim(_ptr(X), n, d, d, k, float(eps), float(phi),
                      ctypes.c_uint64(seed), max_iters, _ptr(centers),
                      ctypes.byref(nc), _ptr(sample), ctypes.byref(ns),
                      _ptr(sset), ctypes.byref(nss), _ptr(rset),
                      ctypes.byref(nrs), ctypes.cast(iters, ctypes.c_void_p),
                      ctypes.byref(ni))
    its = [dict(r_size=it.r_size, ds_size=it.ds_size, h_size=it.h_size,
                s_size=it.s_size, tau=it.tau, p_s=it.p_s, p_h=it.p_h)
           for it in iters[:ni.value]]
    return dict(centers=centers, n_centers=int(nc.value), radius=R,
                sample=sample[:ns.value].copy(), S=sset[:nss.value].copy(),
                R=rset[:nrs.value].copy(), iters=its)


def eim_uniform_pair(seed, x, it):
    """EIM's (u_S, u_H) for point x in iteration it."""
    out = np.zeros(2, np.float64)
    lib().orc_eim_uniform_pair(ctypes.c_uint64(seed), int(x), int(it),
                               _ptr(out))
    return float(out[0]), float(out[1])


def eim_draw_flags(seed, it, R, p_s, p_h):
    """EIM's draws of iteration `it` for the listed points R: uint8 flags
    (bit 0 into S, bit 1 into H)."""
    R = np.ascontiguousarray(R, dtype=np.int64)
    f = np.zeros(max(len(R), 1), np.uint8)
    lib().orc_eim_draw_flags(ctypes.c_uint64(seed), int(it), _ptr(R), len(R),
                             float(p_s), float(p_h), _ptr(f))
    return f[:len(R)]


def min_dist2_to_set(X, x, idx):
    """(min squared distance of point x to the listed points, position)."""
    X, n, d = _pts(X)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    arg = ctypes.c_int64(-1)
    v = lib().orc_min_dist2_to_set(_ptr(X), d, d, int(x), _ptr(idx), len(idx),
                                   ctypes.byref(arg))
    return v, int(arg.value)


def opt_bruteforce(X, k):
    X, n, d = _pts(X)
    return lib().orc_opt_bruteforce(_ptr(X), n, d, d, k)

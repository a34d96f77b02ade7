"""CPU FP64 oracle for the decomposed-TV min-cut method (arXiv:1503.01563).

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct reference code used
by the test-suite, the smoke check and the benchmark's CPU-baseline leg.  The
product path (the GPU library and its binding) never imports it, and the two
share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, built with gcc) and the
conv-net reference in ``convnet.py`` (numpy FP64); this module only marshals
numpy arrays into the C functions.

Conventions: grid ``[D][H][W]`` with W contiguous (2D grids pass ``dims=(H, W)``);
``a[j]`` holds the weights of the edges ``(i, i + stride_j)`` along axis ``j``
(0 = W, 1 = H, 2 = D), ignored on the last slice; cut energy
``E(S) = sum_{i in S} w_i + sum_e a_e [e crosses S]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_LIB_OMP = os.path.join(_HERE, "liborc_omp.so")
_lib = None
_lib_omp = None

_CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]


def _compile(out, extra):
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run(["gcc"] + _CFLAGS + extra + ["-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain IEEE FP64, no contraction): liborc.so on
    one thread, and liborc_omp.so, the same source with OpenMP (the all-core
    CPU baseline; identical results)."""
    if force or not os.path.exists(_LIB):
        _compile(_LIB, ["-Wno-unknown-pragmas"])
    if force or not os.path.exists(_LIB_OMP):
        _compile(_LIB_OMP, ["-fopenmp"])
    return _LIB


class OrcStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("cert", ctypes.c_double), ("energy", ctypes.c_double),
                ("lower_bound", ctypes.c_double), ("tv_gap", ctypes.c_double),
                ("tau_used", ctypes.c_double)]


def _load(threads: int = 1):
    """The plain library, or with threads > 1 the OpenMP build set to that
    many threads."""
    global _lib, _lib_omp
    if threads > 1:
        if _lib_omp is None:
            if not os.path.exists(_LIB_OMP):
                build(force=False)
            _lib_omp = _declare(ctypes.CDLL(_LIB_OMP))
        _lib_omp.orc_set_threads(int(threads))
        return _lib_omp
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def threads_used(threads: int) -> int:
    """Threads the OpenMP build runs with after asking for `threads`."""
    return int(_load(max(2, threads)).orc_set_threads(0)) if threads > 1 else 1


def _declare(lib):
    """argtypes of every exported function."""
    P = ctypes.c_void_p
    lib.orc_tv1d.argtypes = [ctypes.c_long, P, P, P, P]
    lib.orc_tv1d.restype = ctypes.c_int
    lib.orc_cut_energy.argtypes = [ctypes.c_int, P, P, P, P]
    lib.orc_cut_energy.restype = ctypes.c_double
    lib.orc_bruteforce.argtypes = [ctypes.c_int, P, P, P, P, P, P]
    lib.orc_bruteforce.restype = ctypes.c_double
    lib.orc_mincut.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
    lib.orc_mincut.restype = ctypes.c_double
    lib.orc_dr_solve.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 P, P, P, P, P, P, ctypes.POINTER(OrcStats)]
    lib.orc_dr_solve.restype = ctypes.c_int
    lib.orc_prox_family.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, P, P]
    lib.orc_prox_family.restype = ctypes.c_int
    lib.orc_lower_bound.argtypes = [ctypes.c_int, P, P, P, P, P, P]
    lib.orc_lower_bound.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads.restype = ctypes.c_int
    return lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(x):
    return x.ctypes.data_as(ctypes.c_void_p) if x is not None else None


class _PtrArray:
    """Keeps a C array of double* alive together with the arrays it points to."""

    def __init__(self, arrays):
        self.arrays = [_f64(a) for a in arrays]
        self.c = (ctypes.c_void_p * 3)(*([a.ctypes.data for a in self.arrays] + [None] * (3 - len(self.arrays))))

    @property
    def ptr(self):
        return ctypes.cast(self.c, ctypes.c_void_p)


def _dims(dims):
    return (ctypes.c_long * 3)(*(list(dims) + [0] * (3 - len(dims))))


def tv1d(v, a):
    """Weighted 1D-TV prox of one chain: returns (x, p) with x = v - D^T p."""
    lib = _load()
    v = _f64(v).ravel()
    m = v.size
    a = _f64(a).ravel()
    if a.size < max(m - 1, 0):
        raise ValueError("need m-1 weights")
    a_buf = a if a.size > 0 else np.zeros(1)
    x = np.empty(m)
    p = np.empty(max(m - 1, 1))
    rc = lib.orc_tv1d(m, _ptr(v), _ptr(a_buf), _ptr(x), _ptr(p))
    if rc != 0:
        raise RuntimeError("orc_tv1d failed: %d" % rc)
    return x, p[: m - 1]


def prox_family(dims, axis, v, a_axis):
    """Prox of every chain along `axis`; returns (x, p) as grid-shaped float64."""
    lib = _load()
    dims = tuple(int(d) for d in dims)
    v = _f64(v)
    a_axis = _f64(a_axis)
    x = np.empty(dims)
    p = np.empty(dims)
    rc = lib.orc_prox_family(len(dims), _dims(dims), axis, _ptr(v), _ptr(a_axis), _ptr(x), _ptr(p))
    if rc != 0:
        raise RuntimeError("orc_prox_family failed: %d" % rc)
    return x, p


def cut_energy(w, a, labels):
    """E(S) for S = {labels != 0} in FP64 (exact for integer/dyadic data)."""
    lib = _load()
    w = _f64(w)
    pa = _PtrArray(a)
    lab = np.ascontiguousarray(labels, dtype=np.uint8)
    return lib.orc_cut_energy(w.ndim, _dims(w.shape), _ptr(w), pa.ptr, _ptr(lab))


def bruteforce(w, a):
    """Exhaustive minimum over all labellings (n <= 22): (E*, min_set, max_set, count)."""
    lib = _load()
    w = _f64(w)
    pa = _PtrArray(a)
    mn = np.empty(w.shape, np.uint8)
    mx = np.empty(w.shape, np.uint8)
    cnt = ctypes.c_long(0)
    e = lib.orc_bruteforce(w.ndim, _dims(w.shape), _ptr(w), pa.ptr, _ptr(mn), _ptr(mx),
                           ctypes.cast(ctypes.pointer(cnt), ctypes.c_void_p))
    return e, mn, mx, cnt.value


def mincut(w, a, method="dinic"):
    """Exact minimum cut by max-flow: (E*, minimal optimal set, maximal optimal set)."""
    lib = _load()
    w = _f64(w)
    pa = _PtrArray(a)
    mn = np.empty(w.shape, np.uint8)
    mx = np.empty(w.shape, np.uint8)
    m = {"ek": 0, "edmonds_karp": 0, "dinic": 1}[method]
    e = lib.orc_mincut(m, w.ndim, _dims(w.shape), _ptr(w), pa.ptr, _ptr(mn), _ptr(mx), None)
    return e, mn, mx


def lower_bound(w, a, p):
    """(LB(y), TV gap) for y = sum_j D_j^T clip(p_j)."""
    lib = _load()
    w = _f64(w)
    pa = _PtrArray(a)
    pp = _PtrArray(p)
    lb = ctypes.c_double(0)
    gap = ctypes.c_double(0)
    lib.orc_lower_bound(w.ndim, _dims(w.shape), _ptr(w), pa.ptr, pp.ptr,
                        ctypes.cast(ctypes.pointer(lb), ctypes.c_void_p),
                        ctypes.cast(ctypes.pointer(gap), ctypes.c_void_p))
    return lb.value, gap.value


def dr_solve(w, a, variant=None, max_iters=500, gap_tol=1e-3, tv_tol=0.0, tau0=1e-3,
             z0=None, history=False, return_z=False, threads=1):
    """FP64 Douglas-Rachford (averaged alternating reflections).

    variant 0 = two-set form (2D only), 1 = product space.  Default: 0 for 2D,
    1 for 3D.  threads > 1 runs the OpenMP build (same results).  Returns a
    dict with x, labels, stats (and histories / z).
    """
    lib = _load(threads)
    w = _f64(w)
    nd = w.ndim
    if variant is None:
        variant = 0 if nd == 2 else 1
    pa = _PtrArray(a)
    n = w.size
    nz = n if variant == 0 else nd * n
    x = np.empty(w.shape)
    lab = np.empty(w.shape, np.uint8)
    zout = np.empty(nz) if return_z else None
    ch = np.full(max_iters, np.nan) if history else None
    th = np.full(max_iters, np.nan) if history else None
    z0a = _f64(z0).ravel() if z0 is not None else None
    if z0a is not None and z0a.size != nz:
        raise ValueError("z0 must have %d entries" % nz)
    st = OrcStats()
    rc = lib.orc_dr_solve(nd, _dims(w.shape), _ptr(w), pa.ptr, variant, max_iters, gap_tol,
                          tv_tol, tau0, _ptr(z0a), _ptr(x), _ptr(lab), _ptr(zout), _ptr(ch),
                          _ptr(th), ctypes.byref(st))
    if rc != 0:
        raise RuntimeError("orc_dr_solve failed: %d" % rc)
    out = {"x": x, "labels": lab, "iters": st.iters, "status": st.status, "cert": st.cert,
           "energy": st.energy, "lower_bound": st.lower_bound, "tv_gap": st.tv_gap,
           "tau_used": st.tau_used}
    if history:
        out["cert_hist"] = ch[: st.iters]
        out["tvgap_hist"] = th[: st.iters]
    if return_z:
        out["z"] = zout
    return out

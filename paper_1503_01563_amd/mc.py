"""Python binding of libmc (include/mc.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module checks tensor
shapes, dtypes and devices, passes device pointers and the current HIP stream,
and converts the returned status into exceptions.  There is no fallback: if
libmc.so is missing or cannot be loaded, every call raises.

Arrays are torch tensors on a ROCm device: ``w`` of the grid shape (H, W) or
(D, H, W), float32, contiguous; ``a`` a sequence with one tensor of the same
shape per axis (axis 0 = W, 1 = H, 2 = D), or four for an 8-connected 2D grid
(W, H, diagonal, anti-diagonal; see include/mc.h).
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmc.so")

MC_OK = 0
MC_NOT_CONVERGED = 1
MC_VALIDATE = 1
MC_PROFILE = 2
MC_WARM_MOVES = 4
MC_WHOLE_CHAINS = 8
MC_PIECE_CHAINS = 16
MC_BATCH_PERSISTENT = 32
MC_DEBUG = 64
MC_FP64_STATE = 128
VARIANT_AUTO, VARIANT_TWO_SET, VARIANT_PRODUCT = 0, 1, 2
VARIANT_BCD, VARIANT_AP, VARIANT_FISTA = 3, 4, 5
VARIANT_BCD_DR = 6
V_POTTS, V_TRUNC_LINEAR = 0, 1


class McError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libmc error %d: %s" % (code, msg))
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("conn", ctypes.c_int32),
                ("dims", ctypes.c_int64 * 3)]


class Opts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("gap_tol", ctypes.c_double), ("variant", ctypes.c_int32),
                ("tau0", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("batch_items", ctypes.c_int32), ("bcd_iters", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("cert_gap", ctypes.c_double), ("energy", ctypes.c_double),
                ("lower_bound", ctypes.c_double), ("tv_gap", ctypes.c_double),
                ("tau_used", ctypes.c_float), ("ms", ctypes.c_float),
                ("sweep_ms", ctypes.c_double), ("sweep_launches", ctypes.c_int32),
                ("checks", ctypes.c_int32), ("items", ctypes.c_int32), ("whole_chains", ctypes.c_int32),
                ("dual_sweep_ms", ctypes.c_double), ("dual_sweep_launches", ctypes.c_int32)]


class MLStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("cycles", ctypes.c_int32), ("moves", ctypes.c_int32),
                ("accepted", ctypes.c_int32), ("uncertified", ctypes.c_int32), ("skipped", ctypes.c_int32),
                ("dr_iters", ctypes.c_int64), ("energy0", ctypes.c_double), ("energy", ctypes.c_double),
                ("ms", ctypes.c_float), ("reserved2", ctypes.c_float)]


_lib = None
_lib_lock = threading.Lock()


def load_library():
    """Load libmc.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise McError(-100, "libmc.so not found at %s; run paper_1503_01563_amd.build" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.mc_opts_default.argtypes = [ctypes.POINTER(Opts)]
        lib.mc_opts_default.restype = None
        lib.mc_ctx_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        lib.mc_ctx_create.restype = ctypes.c_int
        lib.mc_ctx_destroy.argtypes = [P]
        lib.mc_ctx_destroy.restype = ctypes.c_int
        lib.mc_tv_solve.argtypes = [P, ctypes.POINTER(Grid), P, P, P, P, P, P,
                                    ctypes.POINTER(Stats), ctypes.POINTER(Opts), P]
        lib.mc_tv_solve.restype = ctypes.c_int
        lib.mc_tv_solve_noalloc.argtypes = lib.mc_tv_solve.argtypes
        lib.mc_tv_solve_noalloc.restype = ctypes.c_int
        lib.mc_tv_prox_chains.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int, P, P, P, P, P]
        lib.mc_tv_prox_chains.restype = ctypes.c_int
        lib.mc_cut_energy.argtypes = [P, ctypes.POINTER(Grid), P, P, P, ctypes.POINTER(ctypes.c_double), P]
        lib.mc_cut_energy.restype = ctypes.c_int
        lib.mc_tv_solve_batched.argtypes = [P, ctypes.c_int, ctypes.POINTER(Grid), P, P, P, P, P,
                                            ctypes.POINTER(Stats), ctypes.POINTER(Opts), P]
        lib.mc_tv_solve_batched.restype = ctypes.c_int
        lib.mc_ws_param_count.argtypes = []
        lib.mc_ws_param_count.restype = ctypes.c_int
        I, F = ctypes.c_int, ctypes.c_float
        lib.mc_ws_forward.argtypes = [P, P, I, I, I, P, P, P, P, P]
        lib.mc_ws_forward.restype = ctypes.c_int
        lib.mc_ws_backward.argtypes = [P, P, I, I, I, P, P, P, P, P, ctypes.POINTER(ctypes.c_double), P]
        lib.mc_ws_backward.restype = ctypes.c_int
        lib.mc_ws_adam_step.argtypes = [P, P, P, P, P, I, F, F, F, F, P]
        lib.mc_ws_adam_step.restype = ctypes.c_int
        lib.mc_ws_warm_state.argtypes = [P, ctypes.POINTER(Grid), P, P, F, P, P]
        lib.mc_ws_warm_state.restype = ctypes.c_int
        lib.mc_expansion_problem.argtypes = [P, ctypes.POINTER(Grid), I, P, P, I, F, P, I, P, P, P]
        lib.mc_expansion_problem.restype = ctypes.c_int
        lib.mc_ml_energy.argtypes = [P, ctypes.POINTER(Grid), I, P, P, I, F, P, ctypes.POINTER(ctypes.c_double), P]
        lib.mc_ml_energy.restype = ctypes.c_int
        lib.mc_alpha_expansion.argtypes = [P, ctypes.POINTER(Grid), I, P, P, I, F, P, I,
                                           ctypes.POINTER(MLStats), ctypes.POINTER(Opts), P]
        lib.mc_alpha_expansion.restype = ctypes.c_int
        lib.mc_status_string.argtypes = [ctypes.c_int]
        lib.mc_status_string.restype = ctypes.c_char_p
        lib.mc_last_error.argtypes = []
        lib.mc_last_error.restype = ctypes.c_char_p
        _lib = lib
        return lib


def _check(rc, allow_not_converged=False):
    if rc == MC_OK or (allow_not_converged and rc == MC_NOT_CONVERGED):
        return rc
    lib = load_library()
    raise McError(rc, "%s: %s" % (lib.mc_status_string(rc).decode(), lib.mc_last_error().decode()))


_ctx = {}


def context(device: int):
    """Per-(thread, device) libmc context."""
    key = (threading.get_ident(), device)
    if key not in _ctx:
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.mc_ctx_create(ctypes.byref(h), device))
        _ctx[key] = h
    return _ctx[key]


def _grid(shape, conn=0):
    g = Grid()
    g.ndim = len(shape)
    g.conn = int(conn)
    if g.ndim not in (2, 3):
        raise ValueError("grid must be 2D or 3D")
    for k, s in enumerate(shape):
        g.dims[k] = int(s)
    return g


def _conn_of(a, nd):
    """8-connected when a 2D grid comes with four weight arrays."""
    if nd == 2 and len(a) == 4:
        return 8
    return 0


def _dev_f32(t, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a torch tensor on a ROCm device" % name)
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32" % name)
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("%s must be contiguous with shape %s" % (name, tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _aptrs(a, shape, nd):
    k = len(a)
    if k != nd and not (nd == 2 and k == 4):
        raise ValueError("need one weight array per axis (four for an 8-connected 2D grid)")
    return (ctypes.c_void_p * 4)(*([_dev_f32(a[j], shape, "a[%d]" % j).value for j in range(k)]
                                   + [None] * (4 - k)))


@dataclass
class SolveResult:
    labels: torch.Tensor
    x: Optional[torch.Tensor]
    z: Optional[torch.Tensor]
    status: int
    iters: int
    cert_gap: float
    energy: float
    lower_bound: float
    tau_used: float
    ms: float
    tv_gap: float = float("nan")
    sweep_ms: float = 0.0
    sweep_launches: int = 0
    checks: int = 0
    whole_chains: int = 0
    dual_sweep_ms: float = 0.0
    dual_sweep_launches: int = 0

    @property
    def converged(self):
        return self.status == MC_OK


def make_opts(max_iters=500, check_every=1, gap_tol=1e-3, variant=VARIANT_AUTO, tau0=1e-3,
              validate=False, profile=False, whole_chains=None, debug=False, fp64_state=False):
    """whole_chains: None = chosen by the solver from its first sweeps, True =
    whole-chain sweeps, False = overlapping pieces.  debug: MC_DEBUG.
    fp64_state: MC_FP64_STATE."""
    o = Opts()
    load_library().mc_opts_default(ctypes.byref(o))
    o.max_iters = int(max_iters)
    o.check_every = int(check_every)
    o.gap_tol = float(gap_tol)
    o.variant = int(variant)
    o.tau0 = float(tau0)
    o.flags = ((MC_VALIDATE if validate else 0) | (MC_PROFILE if profile else 0) | (MC_DEBUG if debug else 0)
               | (MC_FP64_STATE if fp64_state else 0))
    if whole_chains is not None:
        o.flags |= MC_WHOLE_CHAINS if whole_chains else MC_PIECE_CHAINS
    return o


def tv_solve(w: torch.Tensor, a: Sequence[torch.Tensor], z0: Optional[torch.Tensor] = None,
             max_iters=500, check_every=1, gap_tol=1e-3, variant=VARIANT_AUTO, tau0=1e-3,
             validate=False, return_x=True, return_z=False, labels_out=None,
             profile=False, whole_chains=None, debug=False, fp64_state=False) -> SolveResult:
    """Minimum cut of one grid by mc_tv_solve.  debug: MC_DEBUG (state and
    dual checks every iteration; 4- and 6-connected splitting solves).
    fp64_state: MC_FP64_STATE (the splitting in FP64, a slow debug path)."""
    return _solve("mc_tv_solve", w, a, z0, max_iters, check_every, gap_tol, variant, tau0, validate,
                  return_x, return_z, labels_out, profile, whole_chains, debug, fp64_state)


def tv_solve_noalloc(w: torch.Tensor, a: Sequence[torch.Tensor], z0: Optional[torch.Tensor] = None,
                     max_iters=500, check_every=1, gap_tol=1e-3, variant=VARIANT_AUTO, tau0=1e-3,
                     validate=False, return_x=True, return_z=False, labels_out=None,
                     whole_chains=None) -> SolveResult:
    """Minimum cut of one grid by mc_tv_solve_noalloc (the library's static
    device scratch instead of context workspace; outputs are still allocated
    here unless passed in)."""
    return _solve("mc_tv_solve_noalloc", w, a, z0, max_iters, check_every, gap_tol, variant, tau0, validate,
                  return_x, return_z, labels_out, False, whole_chains)


def _solve(entry, w, a, z0, max_iters, check_every, gap_tol, variant, tau0, validate, return_x, return_z,
           labels_out, profile, whole_chains, debug=False, fp64_state=False) -> SolveResult:
    lib = load_library()
    shape = tuple(w.shape)
    nd = len(shape)
    dev = w.device.index if w.device.index is not None else torch.cuda.current_device()
    wp = _dev_f32(w, shape, "w")
    ap = _aptrs(a, shape, nd)
    conn = _conn_of(a, nd)
    two_set = conn != 8 and ((variant == VARIANT_TWO_SET) or (variant == VARIANT_AUTO and nd == 2))
    nz = w.numel() if two_set else (4 if conn == 8 else nd) * w.numel()  # product space / BCD / AP / FISTA: r*n
    z0p = None
    if z0 is not None:
        if z0.device != w.device or z0.dtype != torch.float32 or not z0.is_contiguous() or z0.numel() != nz:
            raise ValueError("z0 must be a contiguous float32 device tensor with %d entries" % nz)
        z0p = ctypes.c_void_p(z0.data_ptr())
    labels = labels_out if labels_out is not None else torch.empty(shape, dtype=torch.uint8, device=w.device)
    if labels.dtype != torch.uint8 or tuple(labels.shape) != shape or not labels.is_contiguous():
        raise ValueError("labels_out must be contiguous uint8 of the grid shape")
    x = torch.empty(shape, dtype=torch.float32, device=w.device) if return_x else None
    z = torch.empty(nz, dtype=torch.float32, device=w.device) if return_z else None
    st = Stats()
    o = make_opts(max_iters, check_every, gap_tol, variant, tau0, validate, profile, whole_chains, debug,
                  fp64_state)
    rc = getattr(lib, entry)(context(dev), ctypes.byref(_grid(shape, conn)), wp,
                         ctypes.cast(ap, ctypes.c_void_p), z0p,
                         ctypes.c_void_p(x.data_ptr()) if x is not None else None,
                         ctypes.c_void_p(labels.data_ptr()),
                         ctypes.c_void_p(z.data_ptr()) if z is not None else None,
                         ctypes.byref(st), ctypes.byref(o), _stream(dev))
    _check(rc, allow_not_converged=True)
    return SolveResult(labels, x, z, st.status, st.iters, st.cert_gap, st.energy,
                       st.lower_bound, st.tau_used, st.ms, st.tv_gap, st.sweep_ms,
                       st.sweep_launches, st.checks, st.whole_chains, st.dual_sweep_ms, st.dual_sweep_launches)


def tv_prox_chains(v: torch.Tensor, a_axis: torch.Tensor, axis: int, return_p=False,
                   x_out=None, p_out=None):
    """Exact weighted 1D-TV prox of every line of `v` along `axis` (mc_tv_prox_chains)."""
    lib = load_library()
    shape = tuple(v.shape)
    dev = v.device.index if v.device.index is not None else torch.cuda.current_device()
    vp = _dev_f32(v, shape, "v")
    apn = _dev_f32(a_axis, shape, "a_axis")
    x = x_out if x_out is not None else torch.empty_like(v)
    p = (p_out if p_out is not None else torch.empty_like(v)) if return_p else None
    _dev_f32(x, shape, "x_out")
    if p is not None:
        _dev_f32(p, shape, "p_out")
    rc = lib.mc_tv_prox_chains(context(dev), ctypes.byref(_grid(shape)), int(axis), vp, apn,
                               ctypes.c_void_p(x.data_ptr()),
                               ctypes.c_void_p(p.data_ptr()) if p is not None else None,
                               _stream(dev))
    _check(rc)
    return (x, p) if return_p else x


def cut_energy(w: torch.Tensor, a: Sequence[torch.Tensor], labels: torch.Tensor) -> float:
    """E(S) in FP64 on the device (mc_cut_energy)."""
    lib = load_library()
    shape = tuple(w.shape)
    nd = len(shape)
    dev = w.device.index if w.device.index is not None else torch.cuda.current_device()
    wp = _dev_f32(w, shape, "w")
    ap = _aptrs(a, shape, nd)
    if labels.dtype != torch.uint8 or tuple(labels.shape) != shape or not labels.is_contiguous():
        raise ValueError("labels must be contiguous uint8 of the grid shape")
    e = ctypes.c_double(0)
    rc = lib.mc_cut_energy(context(dev), ctypes.byref(_grid(shape, _conn_of(a, nd))), wp,
                           ctypes.cast(ap, ctypes.c_void_p), ctypes.c_void_p(labels.data_ptr()),
                           ctypes.byref(e), _stream(dev))
    _check(rc)
    return e.value


@dataclass
class BatchResult:
    labels: list
    x: Optional[list]
    status: list
    iters: list
    cert_gap: list
    energy: list
    ms: list
    items: int
    z: Optional[list] = None

    @property
    def converged(self):
        return all(s == MC_OK for s in self.status)


def tv_solve_batched(ws: Sequence[torch.Tensor], As: Sequence[Sequence[torch.Tensor]], max_iters=500,
                     check_every=8, gap_tol=1e-3, tau0=1e-3, items=0, return_x=False,
                     return_z=False, persistent=False) -> BatchResult:
    """Minimum cuts of several 2D grids at once (mc_tv_solve_batched).

    ws[g] is the (H_g, W_g) unary tensor of grid g, As[g] = (a_x, a_y).
    items > 0 fixes the work items per sweep launch (0: tuned on first use).
    return_z: also the splitting state of each grid after its last check.
    persistent: each check period as one persistent launch (MC_BATCH_PERSISTENT).
    The checks run on the device without a host round trip, so a sparse
    cadence pays: on 64 uneven grids (H, W in [128, 1024]) the per-grid time
    to the exact cut was p50 142 / p99 248 ms with checks every 8 iterations
    against 162 / 282 ms every 2 (repeat calls of one session).
    """
    lib = load_library()
    ng = len(ws)
    if ng < 1 or len(As) != ng:
        raise ValueError("need one weight pair per grid")
    dev = ws[0].device.index if ws[0].device.index is not None else torch.cuda.current_device()
    grids = (Grid * ng)()
    wp = (ctypes.c_void_p * ng)()
    ap = (ctypes.c_void_p * (2 * ng))()
    lp = (ctypes.c_void_p * ng)()
    xp = (ctypes.c_void_p * ng)()
    zp = (ctypes.c_void_p * ng)()
    labels, xs, zs = [], [], []
    for g in range(ng):
        shape = tuple(ws[g].shape)
        if len(shape) != 2:
            raise ValueError("batched grids must be 2D")
        grids[g] = _grid(shape)
        wp[g] = _dev_f32(ws[g], shape, "w[%d]" % g).value
        ap[2 * g] = _dev_f32(As[g][0], shape, "a_x[%d]" % g).value
        ap[2 * g + 1] = _dev_f32(As[g][1], shape, "a_y[%d]" % g).value
        lab = torch.empty(shape, dtype=torch.uint8, device=ws[g].device)
        labels.append(lab)
        lp[g] = lab.data_ptr()
        if return_x:
            x = torch.empty(shape, dtype=torch.float32, device=ws[g].device)
            xs.append(x)
            xp[g] = x.data_ptr()
        if return_z:
            z = torch.empty(shape, dtype=torch.float32, device=ws[g].device)
            zs.append(z)
            zp[g] = z.data_ptr()
    st = (Stats * ng)()
    o = make_opts(max_iters, check_every, gap_tol, VARIANT_AUTO, tau0)
    o.batch_items = int(items)
    if persistent:
        o.flags |= MC_BATCH_PERSISTENT
    rc = lib.mc_tv_solve_batched(context(dev), ng, grids, ctypes.cast(wp, ctypes.c_void_p),
                                 ctypes.cast(ap, ctypes.c_void_p), ctypes.cast(lp, ctypes.c_void_p),
                                 ctypes.cast(xp, ctypes.c_void_p) if return_x else None,
                                 ctypes.cast(zp, ctypes.c_void_p) if return_z else None,
                                 st, ctypes.byref(o), _stream(dev))
    _check(rc, allow_not_converged=True)
    return BatchResult(labels, xs if return_x else None, [s.status for s in st],
                       [s.iters for s in st], [s.cert_gap for s in st], [s.energy for s in st],
                       [s.ms for s in st], st[0].items, zs if return_z else None)


# ---- learned warm start ------------------------------------------------------------

def ws_param_count() -> int:
    return int(load_library().mc_ws_param_count())


def _images(w, a_x, a_y):
    """Accept (H, W) or (B, H, W) tensors; returns the batch shape and pointers."""
    if w.dim() == 2:
        w, a_x, a_y = w.unsqueeze(0), a_x.unsqueeze(0), a_y.unsqueeze(0)
    if w.dim() != 3:
        raise ValueError("images must be (H, W) or (B, H, W)")
    shape = tuple(w.shape)
    return shape, (_dev_f32(w, shape, "w"), _dev_f32(a_x, shape, "a_x"), _dev_f32(a_y, shape, "a_y"))


def _params(params):
    return _dev_f32(params, (ws_param_count(),), "params")


def ws_forward(params: torch.Tensor, w: torch.Tensor, a_x: torch.Tensor, a_y: torch.Tensor,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Network output (B, 2, H, W) for images (B, H, W) or (H, W) (mc_ws_forward)."""
    lib = load_library()
    (B, H, W), ptrs = _images(w, a_x, a_y)
    dev = w.device.index if w.device.index is not None else torch.cuda.current_device()
    o = out if out is not None else torch.empty((B, 2, H, W), dtype=torch.float32, device=w.device)
    op = _dev_f32(o, (B, 2, H, W), "out")
    _check(lib.mc_ws_forward(context(dev), _params(params), B, H, W, *ptrs, op, _stream(dev)))
    return o


def ws_backward(params, w, a_x, a_y, target, grad: Optional[torch.Tensor] = None, want_loss=True):
    """(grad, loss) of the mean-squared error against target (B, 2, H, W)."""
    lib = load_library()
    (B, H, W), ptrs = _images(w, a_x, a_y)
    dev = w.device.index if w.device.index is not None else torch.cuda.current_device()
    if target.dim() == 3:
        target = target.unsqueeze(0)
    tp = _dev_f32(target, (B, 2, H, W), "target")
    g = grad if grad is not None else torch.empty(ws_param_count(), dtype=torch.float32, device=w.device)
    gp = _dev_f32(g, (ws_param_count(),), "grad")
    loss = ctypes.c_double(float("nan"))
    _check(lib.mc_ws_backward(context(dev), _params(params), B, H, W, *ptrs, tp, gp,
                              ctypes.byref(loss) if want_loss else None, _stream(dev)))
    return g, (loss.value if want_loss else None)


def ws_adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of params, m, v (mc_ws_adam_step)."""
    lib = load_library()
    n = ws_param_count()
    dev = params.device.index if params.device.index is not None else torch.cuda.current_device()
    ptrs = [_dev_f32(t, (n,), name) for t, name in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v"))]
    _check(lib.mc_ws_adam_step(context(dev), *ptrs, int(step), float(lr), float(beta1), float(beta2),
                               float(eps), _stream(dev)))


def ws_warm_state(out: torch.Tensor, a_x: torch.Tensor, c: float = 0.0) -> torch.Tensor:
    """Starting state z0 (H, W) of the two-set splitting from out (2, H, W)."""
    lib = load_library()
    if out.dim() == 4:
        if out.shape[0] != 1:
            raise ValueError("one image at a time")
        out = out[0]
    H, W = int(out.shape[1]), int(out.shape[2])
    dev = out.device.index if out.device.index is not None else torch.cuda.current_device()
    op = _dev_f32(out, (2, H, W), "out")
    ap = _dev_f32(a_x, (H, W), "a_x")
    z0 = torch.empty((H, W), dtype=torch.float32, device=out.device)
    _check(lib.mc_ws_warm_state(context(dev), ctypes.byref(_grid((H, W))), op, ap, float(c),
                                ctypes.c_void_p(z0.data_ptr()), _stream(dev)))
    return z0


# ---- multi-label energies by alpha-expansion ----------------------------------------

def _ml_args(data, lam, labels):
    if data.dim() != 3:
        raise ValueError("data must be (n_labels, H, W)")
    L, H, W = (int(x) for x in data.shape)
    dp = _dev_f32(data, (L, H, W), "data")
    if len(lam) != 2:
        raise ValueError("lam must hold two arrays (along W, along H)")
    lp = (ctypes.c_void_p * 2)(_dev_f32(lam[0], (H, W), "lam[0]").value, _dev_f32(lam[1], (H, W), "lam[1]").value)
    if (not isinstance(labels, torch.Tensor) or labels.device != data.device or labels.dtype != torch.int32
            or tuple(labels.shape) != (H, W) or not labels.is_contiguous()):
        raise ValueError("labels must be a contiguous int32 device tensor of shape (H, W)")
    dev = data.device.index if data.device.index is not None else torch.cuda.current_device()
    return L, H, W, dp, lp, dev


def expansion_problem(data, lam, labels, alpha, kind=V_TRUNC_LINEAR, trunc=2.0):
    """Binary problem (w, [a_x, a_y]) of the expansion move of `alpha` (mc_expansion_problem)."""
    lib = load_library()
    L, H, W, dp, lp, dev = _ml_args(data, lam, labels)
    w = torch.empty((H, W), dtype=torch.float32, device=data.device)
    a = [torch.empty((H, W), dtype=torch.float32, device=data.device) for _ in range(2)]
    ap = (ctypes.c_void_p * 2)(a[0].data_ptr(), a[1].data_ptr())
    _check(lib.mc_expansion_problem(context(dev), ctypes.byref(_grid((H, W))), L, dp, ctypes.cast(lp, ctypes.c_void_p),
                                    int(kind), float(trunc), ctypes.c_void_p(labels.data_ptr()), int(alpha),
                                    ctypes.c_void_p(w.data_ptr()), ctypes.cast(ap, ctypes.c_void_p), _stream(dev)))
    return w, a


def ml_energy(data, lam, labels, kind=V_TRUNC_LINEAR, trunc=2.0) -> float:
    """Multi-label energy E(f) in FP64 on the device (mc_ml_energy)."""
    lib = load_library()
    L, H, W, dp, lp, dev = _ml_args(data, lam, labels)
    e = ctypes.c_double(0)
    _check(lib.mc_ml_energy(context(dev), ctypes.byref(_grid((H, W))), L, dp, ctypes.cast(lp, ctypes.c_void_p),
                            int(kind), float(trunc), ctypes.c_void_p(labels.data_ptr()), ctypes.byref(e),
                            _stream(dev)))
    return e.value


@dataclass
class MLResult:
    status: int
    cycles: int
    moves: int
    accepted: int
    uncertified: int
    dr_iters: int
    energy0: float
    energy: float
    ms: float
    skipped: int = 0

    @property
    def converged(self):
        return self.status == MC_OK


def alpha_expansion(data, lam, labels, kind=V_TRUNC_LINEAR, trunc=2.0, max_cycles=50, max_iters=2000,
                    check_every=2, gap_tol=1e-3, validate=False, warm=None, whole_chains=True,
                    variant=VARIANT_AUTO) -> MLResult:
    """Alpha-expansion from `labels`, in place (mc_alpha_expansion); every move
    is an exact mc_tv_solve.  Defaults, measured on the 384 x 288 stereo
    stand-in (16 labels):
    - `warm` (None: on for the two-set splitting, the only form it applies
      to): each move starts from the same label's previous move (the reuse
      of dual vectors across related problems): 319 ms against 338 ms cold;
    - `whole_chains`: one lane per chain, since move problems are flat where
      the labels agree and their chain proxes have long constant segments
      (overlapping pieces: 867 ms);
    - `check_every` = 2: moves certify after a few iterations each (cold
      moves: 339 ms against 413 ms with checks every 4, 351 ms every
      iteration)."""
    lib = load_library()
    L, H, W, dp, lp, dev = _ml_args(data, lam, labels)
    st = MLStats()
    o = make_opts(max_iters, check_every, gap_tol, variant, 1e-3, validate, False, whole_chains)
    if warm is None:
        warm = variant in (VARIANT_AUTO, VARIANT_TWO_SET)
    if warm:
        o.flags |= MC_WARM_MOVES
    rc = lib.mc_alpha_expansion(context(dev), ctypes.byref(_grid((H, W))), L, dp, ctypes.cast(lp, ctypes.c_void_p),
                                int(kind), float(trunc), ctypes.c_void_p(labels.data_ptr()), int(max_cycles),
                                ctypes.byref(st), ctypes.byref(o), _stream(dev))
    _check(rc, allow_not_converged=True)
    return MLResult(st.status, st.cycles, st.moves, st.accepted, st.uncertified, st.dr_iters, st.energy0,
                    st.energy, st.ms, st.skipped)

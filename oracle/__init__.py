"""FP64 CPU oracle for continuous sensor registration.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does.  It
shares no code with the GPU path.

Two independent implementations of the same definitions live here:
  * ``cvo_oracle.c`` (plain C, FP64, brute force over all pairs, optional
    threads over target blocks), wrapped with ctypes below;
  * ``np_oracle.py`` (NumPy, FP64, tiny inputs only), used to cross-check the
    C code and for the finite-difference pins.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cvo_oracle.c")
_LIB = os.path.join(_HERE, "libcvo_oracle.so")
_lib = None

ENOOVERLAP = -4
EINVAL = -1


def build(force=True):
    """Compile the C oracle with gcc (IEEE FP64 semantics, no fast-math)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-o", _LIB, _SRC, "-lm", "-lpthread"])
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        f32p, f64p, i32p, i64p = P(ctypes.c_float), P(ctypes.c_double), P(ctypes.c_int), P(ctypes.c_longlong)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        L.cvo_oracle_eval.argtypes = [c_int, f32p, f32p, c_int, f32p, f32p, c_int,
                                      c_double, c_double, c_double, c_double, c_double, c_double,
                                      f64p, c_int, i32p, c_int, f64p, f64p, i64p, f64p]
        L.cvo_oracle_eval.restype = c_int
        L.cvo_oracle_eval_h.argtypes = L.cvo_oracle_eval.argtypes
        L.cvo_oracle_eval_h.restype = c_int
        L.cvo_oracle_eval_grid.argtypes = L.cvo_oracle_eval.argtypes
        L.cvo_oracle_eval_grid.restype = c_int
        L.cvo_oracle_expmap.argtypes = [f64p, f64p, f64p, f64p]
        L.cvo_oracle_expmap.restype = None
        L.cvo_oracle_mean_sqnorm.argtypes = [c_int, f32p]
        L.cvo_oracle_mean_sqnorm.restype = c_double
        L.cvo_oracle_register.argtypes = [c_int, f32p, f32p, c_int, f32p, f32p, c_int,
                                          c_double, c_double, c_double, c_double, c_double, c_double,
                                          c_int, i32p, f64p, c_int, c_double, c_double, c_int, c_int, f64p,
                                          c_int, f64p, f64p, i32p, i32p, c_int, f64p, c_double]
        L.cvo_oracle_register.restype = c_int
        L.cvo_oracle_quartic.argtypes = [c_int, f32p, f32p, c_int, f32p, f32p, c_int,
                                         c_double, c_double, c_double, c_double, f64p, f64p, f64p, c_int,
                                         f64p, f64p]
        L.cvo_oracle_quartic.restype = c_int
        L.cvo_oracle_quartic_step.argtypes = [f64p, f64p]
        L.cvo_oracle_quartic_step.restype = c_int
        L.cvo_oracle_quartic_step_bounded.argtypes = [f64p, c_double, f64p]
        L.cvo_oracle_quartic_step_bounded.restype = c_int
        _lib = L
    return _lib


def _f32(a, cols):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.ndim == 2 and a.shape[1] == cols, a.shape
    return a


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def default_threads():
    return max(1, min(16, os.cpu_count() or 1))


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


def mean_sqnorm(x):
    x = _f32(x, 3)
    return _load().cvo_oracle_mean_sqnorm(x.shape[0], _ptr(x, ctypes.c_float))


def eval(src_xyz, src_feat, tgt_xyz, tgt_feat, T, *, sigma=0.1, feat_scale=0.2, ell=0.1,
         kappa=0.0, a2=None, b2=1.0, sel=None, nthreads=None, per_target=False, paper_pose=False,
         grid=False):
    """F, omega, v at pose T (library convention: T acts on target points).

    Returns dict(g=[F, w0, w1, w2, v0, v1, v2], abs=[same with |terms|],
    within=int, examined=int, per_target=[nsel,7] or None).
    With paper_pose=True, T is read as the paper's h (= library T^-1).
    grid=True (needs kappa > 0) enumerates the cutoff pairs through the
    oracle's own uniform source grid instead of testing every pair: the same
    pair set (pinned against the brute force), for clouds too large for it;
    `examined` then counts the grid's candidates.
    """
    L = _load()
    x = _f32(src_xyz, 3)
    fd = np.asarray(src_feat).shape[1]
    lx = _f32(src_feat, fd)
    z = _f32(tgt_xyz, 3)
    lz = _f32(tgt_feat, fd)
    if a2 is None:
        a2 = mean_sqnorm(x)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
    nth = nthreads or default_threads()
    out = np.zeros(7)
    absout = np.zeros(7)
    counts = np.zeros(2, dtype=np.int64)
    if sel is not None:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        nsel = sel.size
        selp = _ptr(sel, ctypes.c_int)
    else:
        nsel = 0
        selp = None
    pt = None
    if per_target:
        pt = np.zeros((nsel if sel is not None else z.shape[0], 7))
    if grid and paper_pose:
        raise ValueError("grid enumeration takes the library pose")
    fn = L.cvo_oracle_eval_grid if grid else (L.cvo_oracle_eval_h if paper_pose else L.cvo_oracle_eval)
    rc = fn(x.shape[0], _ptr(x, ctypes.c_float), _ptr(lx, ctypes.c_float),
            z.shape[0], _ptr(z, ctypes.c_float), _ptr(lz, ctypes.c_float), fd,
            sigma, feat_scale, ell, kappa, a2, b2, _ptr(T, ctypes.c_double), nsel, selp, nth,
            _ptr(out, ctypes.c_double), _ptr(absout, ctypes.c_double),
            _ptr(counts, ctypes.c_longlong), _ptr(pt, ctypes.c_double) if pt is not None else None)
    if rc != 0:
        raise OracleError(rc)
    return dict(g=out, abs=absout, within=int(counts[0]), examined=int(counts[1]), per_target=pt)


def expmap(w, u):
    """Closed-form SE(3) exponential of the twist (w^, u): returns 4x4."""
    L = _load()
    w = np.ascontiguousarray(w, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    dR = np.zeros(9)
    dT = np.zeros(3)
    L.cvo_oracle_expmap(_ptr(w, ctypes.c_double), _ptr(u, ctypes.c_double),
                        _ptr(dR, ctypes.c_double), _ptr(dT, ctypes.c_double))
    E = np.eye(4)
    E[:3, :3] = dR.reshape(3, 3)
    E[:3, 3] = dT
    return E


def quartic(src_xyz, src_feat, tgt_xyz, tgt_feat, T, w, u, *, sigma=0.1, feat_scale=0.2, ell=0.1,
            kappa=0.0, nthreads=None):
    """Taylor coefficients of G(t) = F(h exp(t (w^, u))) at t = 0 (eq. fourth),
    T = h^-1: returns (coef[5] = F, A1..A4, abs[5] = sums of |terms|)."""
    L = _load()
    x = _f32(src_xyz, 3)
    fd = np.asarray(src_feat).shape[1]
    lx = _f32(src_feat, fd)
    z = _f32(tgt_xyz, 3)
    lz = _f32(tgt_feat, fd)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
    w = np.ascontiguousarray(w, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(5)
    absout = np.zeros(5)
    rc = L.cvo_oracle_quartic(x.shape[0], _ptr(x, ctypes.c_float), _ptr(lx, ctypes.c_float),
                              z.shape[0], _ptr(z, ctypes.c_float), _ptr(lz, ctypes.c_float), fd,
                              sigma, feat_scale, ell, kappa, _ptr(T, ctypes.c_double), _ptr(w, ctypes.c_double),
                              _ptr(u, ctypes.c_double), nthreads or default_threads(),
                              _ptr(out, ctypes.c_double), _ptr(absout, ctypes.c_double))
    if rc != 0:
        raise OracleError(rc)
    return out, absout


def quartic_step(coef, tmax=None):
    """t > 0 maximising P(t) = A1 t + A2 t^2 + A3 t^3 + A4 t^4 (coef[1:5]) among
    its local maxima (those at t <= tmax when given), or None when P has none
    there."""
    A = np.ascontiguousarray(coef, dtype=np.float64)
    assert A.shape == (5,)
    t = np.zeros(1)
    if tmax is None:
        ok = _load().cvo_oracle_quartic_step(_ptr(A, ctypes.c_double), _ptr(t, ctypes.c_double))
    else:
        ok = _load().cvo_oracle_quartic_step_bounded(_ptr(A, ctypes.c_double), float(tmax), _ptr(t, ctypes.c_double))
    return float(t[0]) if ok else None


TRACE_COLS = 26
STEP_RULES = {"fixed": 0, "quartic": 1, "conjugate": 2}


def register(src_xyz, src_feat, tgt_xyz, tgt_feat, *, sigma=0.1, feat_scale=0.2, a2=None, b2=1.0,
             eta=1.0, kappa=0.0, stage_iters=(), stage_ell=(0.1,), max_iters=50, tol=0.0, grad_tol=0.0,
             step_rule="fixed", dof_mask=0, T0=None, nthreads=None, grid=False, stage_tol=0.0):
    """Run the registration iteration; returns dict(T, iters, converged,
    trace[iters,26], abs[iters,7] (sums of |terms| per iteration), rc).
    step_rule "fixed": tau = eta ell^2 / F; "quartic": the maximiser of the
    fourth-order model (eq. fourth), falling back to the fixed rule when the
    model has no maximum on t > 0; "conjugate": the same line search along
    Polak-Ribiere conjugate directions (restarts at each stage, every 6
    steps, and on a non-ascent direction).  grid=True (kappa > 0) evaluates
    through the oracle's grid enumeration (same pair set as the brute
    force).  stage_tol > 0 ends a length-scale stage early once the applied
    twist |tau d| < stage_tol (stage_iters then bound the stages)."""
    L = _load()
    x = _f32(src_xyz, 3)
    fd = np.asarray(src_feat).shape[1]
    lx = _f32(src_feat, fd)
    z = _f32(tgt_xyz, 3)
    lz = _f32(tgt_feat, fd)
    ns = len(stage_ell)
    si = np.ascontiguousarray(list(stage_iters) + [0] * (ns - len(stage_iters)), dtype=np.int32)
    se = np.ascontiguousarray(stage_ell, dtype=np.float64)
    T0 = np.eye(4) if T0 is None else np.asarray(T0, dtype=np.float64)
    T0 = np.ascontiguousarray(T0).reshape(16)
    Tout = np.zeros(16)
    trace = np.zeros((max_iters, TRACE_COLS))
    abs_trace = np.zeros((max_iters, 7))
    it = np.zeros(1, dtype=np.int32)
    cv = np.zeros(1, dtype=np.int32)
    rc = L.cvo_oracle_register(x.shape[0], _ptr(x, ctypes.c_float), _ptr(lx, ctypes.c_float),
                               z.shape[0], _ptr(z, ctypes.c_float), _ptr(lz, ctypes.c_float), fd,
                               sigma, feat_scale, -1.0 if a2 is None else a2, b2, eta, kappa, ns,
                               _ptr(si, ctypes.c_int), _ptr(se, ctypes.c_double), max_iters, tol, grad_tol,
                               STEP_RULES[step_rule], dof_mask, _ptr(T0, ctypes.c_double), nthreads or default_threads(),
                               _ptr(Tout, ctypes.c_double), _ptr(trace, ctypes.c_double),
                               _ptr(it, ctypes.c_int), _ptr(cv, ctypes.c_int), 1 if grid else 0,
                               _ptr(abs_trace, ctypes.c_double), stage_tol)
    return dict(T=Tout.reshape(4, 4), iters=int(it[0]), converged=bool(cv[0]),
                trace=trace[: int(it[0])], abs=abs_trace[: int(it[0])], rc=rc)

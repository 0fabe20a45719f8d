"""Python access to the plain FP64 CPU oracle (``oracle/oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the GPU path.  Arrays are per-trajectory rows (``[n][d]``, ``[n][P]``),
the natural layout for a one-trajectory-at-a-time reference.

What each call follows in the paper:
  record  -- the adaptive solve with embedded error estimate, RMS acceptance
             test and step-size controller (Section 2.1), keeping the accepted
             mesh (Section 3.1) and the states at requested times, each
             reached by one extra step (Section 3.4).
  replay  -- the fixed chain of eq. (replay) on a frozen mesh, in double,
             dual numbers (forward mode) or complex arithmetic (complex step).
  adjoint -- the reverse sweep of that chain with the mesh held fixed
             (Section 3.1, the sg[h] convention).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

LORENZ, VDP, ROBERTSON, HIRES, LV_UDE, LINEAR = 1, 2, 3, 4, 5, 6
TSIT5, VERN7, RODAS, ROS23 = 1, 2, 3, 4
ST_OK, ST_MAX_STEPS, ST_DT_UNDERFLOW, ST_NONFINITE, ST_NOSPACE = 0, 1, 2, 3, 4
LOSS_SUMSQ, LOSS_MSE_TARGET, LOSS_COTANGENT = 0, 1, 2

_lib = None

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)


def use_library(path):
    """Load the oracle from another build of the same source (the benchmark's
    CPU baseline uses one tuned for its host); must precede the first call."""
    global _lib, LIB_PATH
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    LIB_PATH = path


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        lib = C.CDLL(LIB_PATH)
        I, L, D = C.c_int, C.c_int64, C.c_double
        lib.oracle_dims.argtypes = [I, C.POINTER(I), C.POINTER(I)]
        lib.oracle_erk_tableau.argtypes = [I, _d, _d, _d, _d, C.POINTER(I), C.POINTER(I)]
        lib.oracle_root_inv.argtypes = [D, I]
        lib.oracle_root_inv.restype = D
        lib.oracle_rhs.argtypes = [I, _d, _d, _d]
        lib.oracle_jac.argtypes = [I, _d, _d, _d]
        lib.oracle_jac_vjp.argtypes = [I, _d, _d, _d, _d, _d, _d]
        lib.oracle_ros_tableau.argtypes = [I, _d, _d, _d, _d, _d, C.POINTER(I), C.POINTER(I),
                                           C.POINTER(I)]
        lib.oracle_vjp.argtypes = [I, _d, _d, _d, _d, _d]
        lib.oracle_ros_trial.argtypes = [I, I, _d, _d, D, _d, _d]
        lib.oracle_refresh.argtypes = [I, I, I, I, _d, _d, D, D, D, D, L, I, _d, L, _d, _i32,
                                       D, L, _d, _i32, _i32, _i32, _d, _d, _i64, _i32]
        lib.oracle_record.argtypes = [I, I, I, I, _d, _d, D, D, D, D, D, L, I, _d, L,
                                      _d, _i32, _i32, _i32, _d, _d, _i64]
        lib.oracle_replay.argtypes = [I, I, I, I, _d, _d, L, _d, _i32, I, _i32, _d, _d, I]
        lib.oracle_replay_dual.argtypes = [I, I, I, _d, _d, _d, _d, L, _d, _i32, I,
                                           _i32, _d, _d, _d, I]
        lib.oracle_replay_complex.argtypes = [I, I, I, _d, _d, _d, _d, D, L, _d, _i32,
                                              I, _i32, _d, _d, _d, I]
        lib.oracle_adjoint.argtypes = [I, I, I, I, _d, _d, L, _d, _i32, I, _i32, _d,
                                       I, _d, D, _d, _d, _d, I]
        lib.oracle_count_ops.argtypes = [I, I, _i64]
        lib.oracle_count_system.argtypes = [I, _i64]
        lib.oracle_count_lu.argtypes = [I, _i64]
        for f in ("oracle_count_ops", "oracle_count_system", "oracle_count_lu", "oracle_dims", "oracle_erk_tableau", "oracle_rhs", "oracle_vjp", "oracle_jac",
                  "oracle_jac_vjp", "oracle_ros_tableau",
                  "oracle_record", "oracle_replay", "oracle_replay_dual",
                  "oracle_replay_complex", "oracle_adjoint"):
            getattr(lib, f).restype = I
        _lib = lib
    return _lib


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def dims(system):
    d, p = C.c_int(), C.c_int()
    if _load().oracle_dims(system, C.byref(d), C.byref(p)) != 0:
        raise ValueError(f"unknown system {system}")
    return d.value, p.value


def erk_tableau(method):
    c = np.zeros(16); a = np.zeros(256); b = np.zeros(16); ew = np.zeros(16)
    o, q = C.c_int(), C.c_int()
    s = _load().oracle_erk_tableau(method, _p(c), _p(a), _p(b), _p(ew), C.byref(o), C.byref(q))
    if s < 0:
        raise ValueError(f"no explicit tableau for method {method}")
    return dict(s=s, c=c[:s].copy(), A=a[: s * s].reshape(s, s).copy(), b=b[:s].copy(),
                ew=ew[:s].copy(), order=o.value, q_emb=q.value)


COUNT_UNITS = ("trial", "accept", "side_fwd", "adj_step", "adj_side", "adj_zero", "dense_fwd",
               "dense_adj")


def count_ops(method, system):
    """Floating-point operations of one unit of work, counted by running the
    oracle's own step routines on an operation-counting scalar (fma 2; +, -,
    *, /, min, max, sqrt, tanh and the controller's root 1; negation, abs and
    comparisons 0).  Returns a dict over COUNT_UNITS."""
    out = np.zeros(8, np.int64)
    if _load().oracle_count_ops(method, system, _p(out, _i64)) != 0:
        raise ValueError(f"no counts for method {method} on system {system}")
    return dict(zip(COUNT_UNITS, (int(v) for v in out)))


def count_lu(system):
    """(factorisation, solve, transposed solve) operation counts of W =
    I/(gamma h) - J at the counting point, operations on exact zeros left
    out, and the number of rows the pivoting moved there (0: the zeros are
    the Jacobian's structural zeros)."""
    out = np.zeros(4, np.int64)
    if _load().oracle_count_lu(system, _p(out, _i64)) != 0:
        raise ValueError(f"no linear algebra for system {system}")
    return tuple(int(v) for v in out)


def count_system(system):
    """(f, VJP, Jacobian, Jacobian-VJP) operation counts of one evaluation."""
    out = np.zeros(4, np.int64)
    if _load().oracle_count_system(system, _p(out, _i64)) != 0:
        raise ValueError(f"unknown system {system}")
    return tuple(int(v) for v in out)


def root_inv(x, k):
    """The controller's x^(-1/k) (k = 4..8)."""
    return _load().oracle_root_inv(float(x), int(k))


def rhs(system, y, p):
    y, p = _f64(y), _f64(p)
    f = np.zeros_like(y)
    _load().oracle_rhs(system, _p(y), _p(p), _p(f))
    return f


def jac(system, y, p):
    y, p = _f64(y), _f64(p)
    d = len(y)
    J = np.zeros(d * d)
    if _load().oracle_jac(system, _p(y), _p(p), _p(J)) != 0:
        raise ValueError("no Jacobian for this system")
    return J.reshape(d, d)


def jac_vjp(system, y, p, u, v):
    """(d/dy, d/dp) of u^T J(y, p) v."""
    y, p, u, v = _f64(y), _f64(p), _f64(u), _f64(v)
    gy = np.zeros_like(y); gp = np.zeros_like(p)
    if _load().oracle_jac_vjp(system, _p(y), _p(p), _p(u), _p(v), _p(gy), _p(gp)) != 0:
        raise ValueError("no Jacobian for this system")
    return gy, gp


def ros_tableau(method=RODAS):
    """A Rosenbrock method in transformed form (a, c, m, error weights e;
    the first su stages enter y_new)."""
    g = C.c_double(); a = np.zeros(36); c = np.zeros(36); m = np.zeros(6); e = np.zeros(6)
    o, q, su = C.c_int(), C.c_int(), C.c_int()
    s = _load().oracle_ros_tableau(method, C.byref(g), _p(a), _p(c), _p(m), _p(e), C.byref(o),
                                   C.byref(q), C.byref(su))
    if s < 0:
        raise ValueError(f"not a Rosenbrock method: {method}")
    return dict(s=s, su=su.value, gamma=g.value, a=a[:s * s].reshape(s, s).copy(),
                c=c[:s * s].reshape(s, s).copy(), m=m[:s].copy(), e=e[:s].copy(),
                order=o.value, q_emb=q.value)


def ros_trial(method, system, y, p, h):
    """One Rosenbrock trial step: (y_new, error estimate vector)."""
    y, p = _f64(y), _f64(p)
    yn = np.zeros_like(y); e = np.zeros_like(y)
    if _load().oracle_ros_trial(method, system, _p(y), _p(p), float(h), _p(yn), _p(e)) != 0:
        raise ValueError("oracle_ros_trial rejected its arguments")
    return yn, e


def vjp(system, y, p, w):
    y, p, w = _f64(y), _f64(p), _f64(w)
    gy = np.zeros_like(y)
    gp = np.zeros_like(p)
    _load().oracle_vjp(system, _p(y), _p(p), _p(w), _p(gy), _p(gp))
    return gy, gp


def record(system, method, y0, p, t0, t1, rtol, atol, save_t=None, h0=0.0,
           max_steps=100000, cap=None, params_shared=False):
    """Adaptive record.  Returns a dict with the mesh and the save states."""
    y0, p = _f64(y0), _f64(p)
    n, d = y0.shape
    save_t = np.array([t1] if save_t is None else save_t, dtype=np.float64)
    ns = len(save_t)
    if cap is None:
        cap = 4096
    h = np.zeros((n, cap)); S = np.zeros(n, np.int32); st = np.zeros(n, np.int32)
    sidx = np.zeros((n, ns), np.int32); sdt = np.zeros((n, ns)); ys = np.zeros((n, ns, d))
    ntr = np.zeros(n, np.int64)
    rc = _load().oracle_record(system, method, n, int(params_shared), _p(y0), _p(p), t0, t1,
                               rtol, atol, h0, max_steps, ns, _p(save_t), cap, _p(h),
                               _p(S, _i32), _p(st, _i32), _p(sidx, _i32), _p(sdt), _p(ys),
                               _p(ntr, _i64))
    if rc != 0:
        raise ValueError("oracle_record rejected its arguments")
    return dict(h=h, S=S, status=st, save_idx=sidx, save_dt=sdt, y_save=ys, n_trial=ntr,
                save_t=save_t, system=system, method=method)


def refresh(system, method, y0, p, t0, t1, rtol, atol, old, save_t=None, slack=1.0,
            max_steps=100000, cap=None, params_shared=False):
    """Refresh the old record's mesh (dict with h [n][cap], S [n]) at new
    inputs: keep each lane's old steps while their error estimates stay <= slack,
    then continue adaptively.  Returns a record dict plus drift_at (steps kept)."""
    y0, p = _f64(y0), _f64(p)
    n, d = y0.shape
    fh = _f64(old["h"])
    fS = np.ascontiguousarray(old["S"], np.int32)
    save_t = np.array([t1] if save_t is None else save_t, dtype=np.float64)
    ns = len(save_t)
    if cap is None:
        cap = 4096
    h = np.zeros((n, cap)); S = np.zeros(n, np.int32); st = np.zeros(n, np.int32)
    sidx = np.zeros((n, ns), np.int32); sdt = np.zeros((n, ns)); ys = np.zeros((n, ns, d))
    ntr = np.zeros(n, np.int64); drift = np.zeros(n, np.int32)
    rc = _load().oracle_refresh(system, method, n, int(params_shared), _p(y0), _p(p), t0, t1,
                                rtol, atol, max_steps, ns, _p(save_t), fh.shape[1], _p(fh),
                                _p(fS, _i32), float(slack), cap, _p(h), _p(S, _i32),
                                _p(st, _i32), _p(sidx, _i32), _p(sdt), _p(ys), _p(ntr, _i64),
                                _p(drift, _i32))
    if rc != 0:
        raise ValueError("oracle_refresh rejected its arguments")
    return dict(h=h, S=S, status=st, save_idx=sidx, save_dt=sdt, y_save=ys, n_trial=ntr,
                save_t=save_t, system=system, method=method, drift_at=drift)


def _mesh(mesh):
    h = _f64(mesh["h"])
    return (h, h.shape[1], np.ascontiguousarray(mesh["S"], np.int32),
            np.ascontiguousarray(mesh["save_idx"], np.int32), _f64(mesh["save_dt"]))


def replay(system, method, y0, p, mesh, params_shared=False, dense=False):
    """Save states on a frozen mesh: by one extra step from each save's base
    point, or (dense) by the continuous extension of the step holding it."""
    y0, p = _f64(y0), _f64(p)
    h, cap, S, sidx, sdt = _mesh(mesh)
    n, d = y0.shape
    ns = sidx.shape[1]
    ys = np.zeros((n, ns, d))
    _load().oracle_replay(system, method, n, int(params_shared), _p(y0), _p(p), cap, _p(h),
                          _p(S, _i32), ns, _p(sidx, _i32), _p(sdt), _p(ys), int(dense))
    return ys


def replay_dual(system, method, y0, p, dy0, dp, mesh, dense=False):
    y0, p, dy0, dp = _f64(y0), _f64(p), _f64(dy0), _f64(dp)
    h, cap, S, sidx, sdt = _mesh(mesh)
    n, d = y0.shape
    ns = sidx.shape[1]
    ys = np.zeros((n, ns, d)); dys = np.zeros((n, ns, d))
    _load().oracle_replay_dual(system, method, n, _p(y0), _p(p), _p(dy0), _p(dp), cap, _p(h),
                               _p(S, _i32), ns, _p(sidx, _i32), _p(sdt), _p(ys), _p(dys),
                               int(dense))
    return ys, dys


def replay_complex(system, method, y0, p, dy0, dp, eps, mesh, dense=False):
    y0, p, dy0, dp = _f64(y0), _f64(p), _f64(dy0), _f64(dp)
    h, cap, S, sidx, sdt = _mesh(mesh)
    n, d = y0.shape
    ns = sidx.shape[1]
    re = np.zeros((n, ns, d)); im = np.zeros((n, ns, d))
    _load().oracle_replay_complex(system, method, n, _p(y0), _p(p), _p(dy0), _p(dp), eps, cap,
                                  _p(h), _p(S, _i32), ns, _p(sidx, _i32), _p(sdt), _p(re),
                                  _p(im), int(dense))
    return re, im


def adjoint(system, method, y0, p, mesh, loss_kind=LOSS_SUMSQ, loss_data=None, scale=1.0,
            params_shared=False, dense=False):
    """Discrete adjoint on a frozen mesh: (grad_p [n][P], grad_y0 [n][d], loss [n]);
    dense: the save states from the continuous extension."""
    y0, p = _f64(y0), _f64(p)
    h, cap, S, sidx, sdt = _mesh(mesh)
    n, d = y0.shape
    ns = sidx.shape[1]
    np_ = dims(system)[1]
    gp = np.zeros((n, np_)); gy = np.zeros((n, d)); ll = np.zeros(n)
    ld = _f64(loss_data) if loss_data is not None else None
    _load().oracle_adjoint(system, method, n, int(params_shared), _p(y0), _p(p), cap, _p(h),
                           _p(S, _i32), ns, _p(sidx, _i32), _p(sdt), loss_kind,
                           _p(ld) if ld is not None else None, scale, _p(gp), _p(gy), _p(ll),
                           int(dense))
    return gp, gy, ll

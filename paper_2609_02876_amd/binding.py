"""Python binding of the C ABI (``include/ensode.h``), same names as there.

torch supplies device memory and the stream; all computation runs in the HIP
kernels of ``libensode.so``.  There is no CPU path: without a GPU and the
built library these functions raise.

Layouts (trajectory index fastest): y0 [d, n], params [P, n] (or [P] when
shared), save states [n_save, d, n], grad_params [P, n], grad_y0 [d, n].
"""
import ctypes as C
import math

import torch

from . import _abi as A

_DT = {torch.float64: A.F64, torch.float32: A.F32}
SHARED_ONLY = ("ude",)   # systems whose parameters are always shared


def _sysinfo(system):
    if system not in A.SYSTEMS:
        raise ValueError(f"unknown system {system!r}; have {sorted(A.SYSTEMS)}")
    return A.SYSTEMS[system]


def _require_gpu(*ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("ensode works on GPU tensors only")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class _Spec:
    """Problem + ivp structs with the host arrays they point to kept alive."""

    def __init__(self, system, method, y0, params, t0, t1, rtol, atol, save_times,
                 h0, max_steps, params_shared, dense=False):
        sid, d, npar = _sysinfo(system)
        if method not in A.METHODS:
            raise ValueError(f"unknown method {method!r}")
        if y0.dtype not in _DT:
            raise ValueError("y0 must be float64 or float32")
        if params.dtype != y0.dtype:
            raise ValueError("params must have the dtype of y0")
        if y0.dim() != 2 or y0.shape[0] != d:
            raise ValueError(f"y0 must be [{d}, n]")
        n = y0.shape[1]
        want_p = (npar,) if params_shared else (npar, n)
        if tuple(params.shape) != want_p:
            raise ValueError(f"params must be {list(want_p)}")
        _require_gpu(y0, params)
        self.system, self.method, self.d, self.npar, self.n = system, method, d, npar, n
        self.dtype = y0.dtype
        self.y0, self.params = y0, params
        self.prob = A.Problem(sid, A.METHODS[method], _DT[y0.dtype], d, npar, int(params_shared))
        st = [] if save_times is None else [float(x) for x in save_times]
        if len(st) > A.MAX_SAVE:
            raise ValueError(f"at most {A.MAX_SAVE} save times")
        self._st = (C.c_double * max(1, len(st)))(*st) if st else None
        self.n_save = max(1, len(st))
        self.save_times = st
        self.dense = bool(dense)
        self.ivp = A.Ivp(n, y0.data_ptr(), params.data_ptr(), float(t0), float(t1), float(rtol),
                         float(atol), float(h0), int(max_steps), len(st),
                         C.cast(self._st, C.POINTER(C.c_double)) if st else None, int(dense))


class RecordHandle:
    """A record inside its pool (keeps the pool and the inputs alive)."""

    def __init__(self, spec, pool, rec, y_save, status):
        self.spec, self.pool, self.rec = spec, pool, rec
        self.y_save, self.status = y_save, status

    @property
    def n(self):
        return self.spec.n

    def steps(self):
        return _view_i32(self.rec.steps, self.n, self.pool)

    def n_trial(self):
        return _view_i32(self.rec.n_trial, self.n, self.pool)

    def save_index(self):
        """[n_save, n] int32: the mesh index of each save's base point."""
        ns = self.spec.n_save
        return _view_i32(self.rec.save_idx, ns * self.n, self.pool).view(ns, self.n)

    def save_offset(self):
        """[n_save, n] float64: each save's side-step size t_s - t_base."""
        ns = self.spec.n_save
        off = self.rec.save_dt - self.pool.data_ptr()
        return self.pool[off: off + 8 * ns * self.n].view(torch.float64).view(ns, self.n)


def _view_i32(ptr, n, pool):
    off = ptr - pool.data_ptr()
    return pool[off: off + 4 * n].view(torch.int32)


def ensemble_record_bytes(system, method, n, t0, t1, steps_hint, n_save=0,
                          dtype=torch.float64, ckpt_every=0, params_shared=None, dense=False):
    sid, d, npar = _sysinfo(system)
    if params_shared is None:
        params_shared = system in SHARED_ONLY
    prob = A.Problem(sid, A.METHODS[method], _DT[dtype], d, npar, int(params_shared))
    st = (C.c_double * max(1, n_save))(*([t1] * max(1, n_save)))
    ivp = A.Ivp(n, None, None, float(t0), float(t1), 1e-6, 1e-6, 0.0, 0, int(n_save),
                C.cast(st, C.POINTER(C.c_double)), int(dense))
    out = C.c_size_t()
    A.check(A.load().ensemble_record_bytes(C.byref(prob), C.byref(ivp), int(steps_hint),
                                           int(ckpt_every), C.byref(out)))
    return out.value


def plan_tape(system, method, n, t0, t1, steps_hint, n_save=0, dtype=torch.float64,
              budget_bytes=None, ckpt_every=64, shared=None):
    """Tape layout for a record: 0 (full tape) when its planned pool fits the
    HBM budget, else ckpt_every (one state per segment, the segment replayed
    in the reverse sweep).  Raises when neither fits."""
    full = ensemble_record_bytes(system, method, n, t0, t1, steps_hint, n_save, dtype, 0, shared)
    if budget_bytes is None or full <= budget_bytes:
        return 0
    ck = ensemble_record_bytes(system, method, n, t0, t1, steps_hint, n_save, dtype, ckpt_every,
                               shared)
    if ck > budget_bytes:
        raise ValueError(f"record needs {ck} bytes even with checkpoints every {ckpt_every} "
                         f"steps; budget is {budget_bytes}")
    return ckpt_every


def ensemble_solve(system, method, y0, params, t0, t1, rtol, atol, save_times=None, h0=0.0,
                   max_steps=0, params_shared=False, dense=False):
    """Forward solve: (states at the save times [n_save, d, n], lane status [n]).
    dense: save states from the continuous extension instead of extra steps."""
    spec = _Spec(system, method, y0, params, t0, t1, rtol, atol, save_times, h0, max_steps,
                 params_shared, dense)
    y_out = torch.empty((spec.n_save, spec.d, spec.n), dtype=spec.dtype, device=y0.device)
    status = torch.empty(spec.n, dtype=torch.int32, device=y0.device)
    A.check(A.load().ensemble_solve(C.byref(spec.prob), C.byref(spec.ivp), _ptr(y_out),
                                    _ptr(status), _stream()))
    return y_out, status


def _pool_for(spec, steps_hint, pool, steps_per_traj, ckpt_every=0):
    """(pool tensor, tape config): a given pool, or one planned for steps_hint."""
    if pool is not None:
        _require_gpu(pool)
        if pool.dtype != torch.uint8:
            raise ValueError("pool must be a uint8 tensor")
        spt = int(steps_per_traj or 0)
    else:
        nbytes = ensemble_record_bytes(spec.system, spec.method, spec.n, spec.ivp.t0,
                                       spec.ivp.t1, steps_hint, spec.ivp.n_save, spec.dtype,
                                       ckpt_every, bool(spec.prob.params_shared), spec.dense)
        pool = torch.empty(nbytes, dtype=torch.uint8, device=spec.y0.device)
        spt = int(steps_hint)
    return pool, A.TapeCfg(pool.data_ptr(), pool.numel(), int(ckpt_every), spt)


def ensemble_record(system, method, y0, params, t0, t1, rtol, atol, save_times=None, h0=0.0,
                    max_steps=0, params_shared=False, steps_hint=512, pool=None,
                    steps_per_traj=None, ckpt_every=0, tape_budget_bytes=None, dense=False):
    """Adaptive record.  Returns a RecordHandle (.y_save, .status, .pool).

    Without a pool, one is planned that reserves steps_hint taped steps per
    trajectory (plus overflow).  With a pool, steps_per_traj sets the
    per-trajectory reservation (None: 7/8 of the pool evenly).
    ckpt_every="auto" keeps the full tape unless its plan exceeds
    tape_budget_bytes, then checkpoints every 64 steps (plan_tape).  dense: save
    states from the continuous extension of the accepted step (no extra step)."""
    spec = _Spec(system, method, y0, params, t0, t1, rtol, atol, save_times, h0, max_steps,
                 params_shared, dense)
    if ckpt_every == "auto":
        ckpt_every = plan_tape(system, method, spec.n, t0, t1, steps_hint, spec.ivp.n_save,
                               spec.dtype, tape_budget_bytes, shared=bool(params_shared))
    pool, tc = _pool_for(spec, steps_hint, pool, steps_per_traj, ckpt_every)
    rec = A.Record()
    y_save = torch.empty((spec.n_save, spec.d, spec.n), dtype=spec.dtype, device=y0.device)
    status = torch.empty(spec.n, dtype=torch.int32, device=y0.device)
    A.check(A.load().ensemble_record(C.byref(spec.prob), C.byref(spec.ivp), C.byref(tc),
                                     C.byref(rec), _ptr(y_save), _ptr(status), _stream()))
    return RecordHandle(spec, pool, rec, y_save, status)


def ensemble_replay_mesh(system, method, y0, params, t0, t1, h, steps, save_times=None,
                         params_shared=False, pool=None, steps_per_traj=None, ckpt_every=0,
                         dense=False):
    """Record on a given mesh h [cap, n] (float64), steps [n] (int32)."""
    spec = _Spec(system, method, y0, params, t0, t1, 1e-6, 1e-6, save_times, 0.0, 0,
                 params_shared, dense)
    _require_gpu(h, steps)
    if h.dtype != torch.float64 or steps.dtype != torch.int32:
        raise ValueError("h must be float64 and steps int32")
    if h.dim() != 2 or h.shape[1] != spec.n or steps.shape != (spec.n,):
        raise ValueError("h must be [cap, n] and steps [n]")
    cap = h.shape[0]
    pool, tc = _pool_for(spec, cap, pool, steps_per_traj, ckpt_every)
    rec = A.Record()
    y_save = torch.empty((spec.n_save, spec.d, spec.n), dtype=spec.dtype, device=y0.device)
    status = torch.empty(spec.n, dtype=torch.int32, device=y0.device)
    A.check(A.load().ensemble_replay_mesh(C.byref(spec.prob), C.byref(spec.ivp), C.byref(tc),
                                          _ptr(h), _ptr(steps), cap, C.byref(rec), _ptr(y_save),
                                          _ptr(status), _stream()))
    return RecordHandle(spec, pool, rec, y_save, status)


def ensemble_refresh(system, method, y0, params, t0, t1, rtol, atol, h, steps, slack=1.0,
                     save_times=None, h0=0.0, max_steps=0, params_shared=False, steps_hint=None,
                     pool=None, steps_per_traj=None, ckpt_every=0, dense=False):
    """Refresh an old mesh h [cap, n] (float64), steps [n] (int32) at new
    inputs: each trajectory keeps its old steps while their error estimates
    stay <= slack, then records adaptively (the mesh-drift policy).
    Returns (RecordHandle, drift_at [n] int32: old steps kept).  (dense
    output is refused by the library here.)"""
    spec = _Spec(system, method, y0, params, t0, t1, rtol, atol, save_times, h0, max_steps,
                 params_shared, dense)
    _require_gpu(h, steps)
    if h.dtype != torch.float64 or steps.dtype != torch.int32:
        raise ValueError("h must be float64 and steps int32")
    if h.dim() != 2 or h.shape[1] != spec.n or steps.shape != (spec.n,):
        raise ValueError("h must be [cap, n] and steps [n]")
    cap = h.shape[0]
    pool, tc = _pool_for(spec, steps_hint or cap, pool, steps_per_traj, ckpt_every)
    rec = A.Record()
    y_save = torch.empty((spec.n_save, spec.d, spec.n), dtype=spec.dtype, device=y0.device)
    status = torch.empty(spec.n, dtype=torch.int32, device=y0.device)
    drift = torch.empty(spec.n, dtype=torch.int32, device=y0.device)
    A.check(A.load().ensemble_refresh(C.byref(spec.prob), C.byref(spec.ivp), C.byref(tc),
                                      _ptr(h), _ptr(steps), cap, float(slack), C.byref(rec),
                                      _ptr(y_save), _ptr(status), _ptr(drift), _stream()))
    return RecordHandle(spec, pool, rec, y_save, status), drift


def refresh_record(handle, y0, params, slack=1.0, steps_hint=None):
    """The mesh-drift policy on a record: its mesh refreshed at new y0 and
    params with the record's own system, method, span, tolerances and save
    times.  Returns (new RecordHandle, drift_at)."""
    sp = handle.spec
    h, S = ensemble_mesh_export(handle)
    return ensemble_refresh(sp.system, sp.method, y0, params, sp.ivp.t0, sp.ivp.t1,
                            sp.ivp.rtol, sp.ivp.atol, h, S, slack=slack,
                            save_times=sp.save_times or None,
                            max_steps=sp.ivp.max_steps,
                            params_shared=bool(sp.prob.params_shared),
                            steps_hint=steps_hint or max(int(h.shape[0]), 16))


def ensemble_mesh_export(handle, cap=None):
    """The record's mesh as the zero-padded rectangle (h [cap, n], steps [n])."""
    n = handle.n
    dev = handle.pool.device
    if cap is None:
        cap = int(handle.steps().max().item()) if n else 1
    cap = max(1, cap)
    h = torch.empty((cap, n), dtype=torch.float64, device=dev)
    s = torch.empty(n, dtype=torch.int32, device=dev)
    A.check(A.load().ensemble_mesh_export(C.byref(handle.rec), _ptr(h), _ptr(s), cap, _stream()))
    return h, s


_LOSS = {"sumsq": A.LOSS_SUMSQ, "mse": A.LOSS_MSE_TARGET, "cotangent": A.LOSS_COTANGENT}


def ensemble_adjoint_workspace_bytes(handle):
    out = C.c_size_t()
    A.check(A.load().ensemble_adjoint_workspace_bytes(C.byref(handle.rec), C.byref(out)))
    return out.value


def ensemble_adjoint(handle, loss="sumsq", data=None, scale=1.0, want_y0=True,
                     want_loss=True, workspace=None):
    """Reverse sweep: (grad_params, grad_y0 [d, n] or None, loss [n] or None).

    grad_params is [P, n], or [P] (summed over trajectories in a fixed order)
    when the parameters are shared."""
    spec = handle.spec
    if loss not in _LOSS:
        raise ValueError(f"loss must be one of {sorted(_LOSS)}")
    if data is not None:
        _require_gpu(data)
        if data.dtype != spec.dtype or tuple(data.shape) != (spec.n_save, spec.d, spec.n):
            raise ValueError(f"loss data must be [{spec.n_save}, {spec.d}, {spec.n}] {spec.dtype}")
    dev = spec.y0.device
    shared = bool(spec.prob.params_shared)
    gp = torch.empty((spec.npar,) if shared else (spec.npar, spec.n), dtype=spec.dtype,
                     device=dev)
    gy = torch.empty((spec.d, spec.n), dtype=spec.dtype, device=dev) if want_y0 else None
    ll = torch.empty(spec.n, dtype=torch.float64, device=dev) if want_loss else None
    ws_bytes = ensemble_adjoint_workspace_bytes(handle)
    if ws_bytes and workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    lo = A.Loss(_LOSS[loss], data.data_ptr() if data is not None else None, float(scale))
    A.check(A.load().ensemble_adjoint(C.byref(spec.prob), C.byref(spec.ivp), C.byref(handle.rec),
                                      C.byref(lo), _ptr(gp), _ptr(gy), _ptr(ll),
                                      _ptr(workspace), int(workspace.numel()) if workspace is not None else 0,
                                      _stream()))
    return gp, gy, ll


def ensemble_adjoint_static(handle, loss="sumsq", data=None, scale=1.0, want_y0=True,
                            want_loss=True, out=None):
    """ensemble_adjoint with the library's static device workspace (no
    workspace is allocated for it).  out = (grad_params, grad_y0, loss)
    tensors to write into (any may be None); missing outputs are allocated
    here, by torch, as ensemble_adjoint does."""
    spec = handle.spec
    if loss not in _LOSS:
        raise ValueError(f"loss must be one of {sorted(_LOSS)}")
    if data is not None:
        _require_gpu(data)
        if data.dtype != spec.dtype or tuple(data.shape) != (spec.n_save, spec.d, spec.n):
            raise ValueError(f"loss data must be [{spec.n_save}, {spec.d}, {spec.n}] {spec.dtype}")
    dev = spec.y0.device
    shared = bool(spec.prob.params_shared)
    gp, gy, ll = out if out is not None else (None, None, None)
    if gp is None:
        gp = torch.empty((spec.npar,) if shared else (spec.npar, spec.n), dtype=spec.dtype,
                         device=dev)
    if gy is None and want_y0:
        gy = torch.empty((spec.d, spec.n), dtype=spec.dtype, device=dev)
    if ll is None and want_loss:
        ll = torch.empty(spec.n, dtype=torch.float64, device=dev)
    lo = A.Loss(_LOSS[loss], data.data_ptr() if data is not None else None, float(scale))
    A.check(A.load().ensemble_adjoint_static(C.byref(spec.prob), C.byref(spec.ivp),
                                             C.byref(handle.rec), C.byref(lo), _ptr(gp),
                                             _ptr(gy), _ptr(ll), _stream()))
    return gp, gy, ll


def ensemble_jvp(handle, dy0=None, dparams=None, loss="sumsq", data=None, scale=1.0,
                 want_states=True, want_loss=True):
    """Forward mode on the recorded mesh: (y_save_dot [n_save, d, n] or None,
    loss_dot [n] or None) along the tangent dy0 [d, n], dparams [P, n]
    (None: zero).  Per-trajectory parameters only."""
    spec = handle.spec
    if loss not in _LOSS:
        raise ValueError(f"loss must be one of {sorted(_LOSS)}")
    for name, t, shape in (("dy0", dy0, (spec.d, spec.n)), ("dparams", dparams, (spec.npar, spec.n)),
                           ("loss data", data, (spec.n_save, spec.d, spec.n))):
        if t is not None:
            _require_gpu(t)
            if t.dtype != spec.dtype or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {list(shape)} {spec.dtype} tensor")
    dev = spec.y0.device
    ysd = (torch.empty((spec.n_save, spec.d, spec.n), dtype=spec.dtype, device=dev)
           if want_states else None)
    ld = torch.empty(spec.n, dtype=torch.float64, device=dev) if want_loss else None
    lo = A.Loss(_LOSS[loss], data.data_ptr() if data is not None else None, float(scale))
    A.check(A.load().ensemble_jvp(C.byref(spec.prob), C.byref(spec.ivp), C.byref(handle.rec),
                                  _ptr(dy0), _ptr(dparams), C.byref(lo), _ptr(ysd), _ptr(ld),
                                  _stream()))
    return ysd, ld


def register_system(name, source, dim, nparams, jacobian=False):
    """Register a system given as source (see ensemble_system_register in
    ensode.h: a struct System with rhs, vjp and, with jacobian=True, jac and
    jac_vjp); afterwards `name` works wherever a system name does.  Returns
    the system id."""
    if name in A.SYSTEMS:
        raise ValueError(f"system {name!r} exists")
    sid = C.c_int32()
    A.check(A.load().ensemble_system_register(source.encode(), int(dim), int(nparams),
                                              int(bool(jacobian)), C.byref(sid)))
    A.SYSTEMS[name] = (sid.value, int(dim), int(nparams))
    return sid.value


def ensemble_record_stats(handle):
    st = A.Stats()
    A.check(A.load().ensemble_record_stats(C.byref(handle.rec), C.byref(st), _stream()))
    return dict(overflow_pages_used=st.overflow_pages_used, steps_accepted=st.steps_accepted, trials=st.trials,
                side_steps=st.side_steps, n_pages=handle.rec.n_pages)


def steps_hint_for(mean_steps, margin=1.15):
    """Pool plan per trajectory from an expected mean step count."""
    return int(math.ceil(mean_steps * margin)) + 16

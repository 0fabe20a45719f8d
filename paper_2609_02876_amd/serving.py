"""Python binding of the serving entry points (ensemble_server_* in ensode.h).

A Server owns a device pool (a torch byte tensor) and runs submitted
ensemble-gradient jobs -- record plus reverse sweep on each job's own
trajectories -- as they arrive: admission by the memory a job's record
needs, packing of admitted jobs of one (system, method, dtype) family into
persistent launches, several launches in flight on separate streams.

The server works on its own streams.  submit() waits for torch's current
stream first, so inputs written there are complete; once a job is done its
outputs are complete for any later work.
"""
import ctypes as C

import torch

from . import _abi as A
from .binding import _DT, _LOSS, _Spec, _ptr, _require_gpu


class ServedJob:
    """Outputs of one job: y_save [n_save, d, n], status [n], grad_params
    [P, n], grad_y0 [d, n] or None, loss [n] or None."""

    def __init__(self, server, jid, spec, y_save, status, gp, gy, ll, keep):
        self.server, self.id, self.spec = server, jid, spec
        self.y_save, self.status, self.grad_params, self.grad_y0, self.loss = (
            y_save, status, gp, gy, ll)
        self._keep = keep

    def state(self):
        return self.server.poll(self)

    def done(self):
        return self.state() == A.JOB_DONE


class Server:
    def __init__(self, pool_bytes, n_slots=4, device=None):
        dev = torch.device(device) if device is not None else torch.device("cuda")
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=dev)
        h = C.c_void_p()
        A.check(A.load().ensemble_server_create(_ptr(self.pool), self.pool.numel(),
                                                int(n_slots), C.byref(h)))
        self._h = h
        self._jobs = {}

    def submit(self, system, method, y0, params, t0, t1, rtol, atol, save_times=None,
               loss="sumsq", data=None, scale=1.0, steps_hint=0, max_steps=0, want_y0=True,
               want_loss=True):
        spec = _Spec(system, method, y0, params, t0, t1, rtol, atol, save_times, 0.0, max_steps,
                     False)
        if loss not in _LOSS:
            raise ValueError(f"loss must be one of {sorted(_LOSS)}")
        if data is not None:
            _require_gpu(data)
            if data.dtype != spec.dtype or tuple(data.shape) != (spec.n_save, spec.d, spec.n):
                raise ValueError(f"loss data must be [{spec.n_save}, {spec.d}, {spec.n}]")
        dev = y0.device
        ys = torch.empty((spec.n_save, spec.d, spec.n), dtype=spec.dtype, device=dev)
        st = torch.empty(spec.n, dtype=torch.int32, device=dev)
        gp = torch.empty((spec.npar, spec.n), dtype=spec.dtype, device=dev)
        gy = torch.empty((spec.d, spec.n), dtype=spec.dtype, device=dev) if want_y0 else None
        ll = torch.empty(spec.n, dtype=torch.float64, device=dev) if want_loss else None
        job = A.Job(spec.prob, spec.ivp,
                    A.Loss(_LOSS[loss], data.data_ptr() if data is not None else None,
                           float(scale)),
                    int(steps_hint), ys.data_ptr(), st.data_ptr(), gp.data_ptr(),
                    gy.data_ptr() if gy is not None else None,
                    ll.data_ptr() if ll is not None else None)
        torch.cuda.current_stream().synchronize()
        jid = C.c_int64()
        A.check(A.load().ensemble_server_submit(self._h, C.byref(job), C.byref(jid)))
        sj = ServedJob(self, jid.value, spec, ys, st, gp, gy, ll, (y0, params, data))
        self._jobs[jid.value] = sj
        return sj

    def progress(self):
        a = C.c_int32()
        A.check(A.load().ensemble_server_progress(self._h, C.byref(a)))
        return a.value

    def poll(self, job):
        s = C.c_int32()
        A.check(A.load().ensemble_server_poll(self._h, int(job.id), C.byref(s)))
        return s.value

    def wait(self, job):
        A.check(A.load().ensemble_server_wait(self._h, int(job.id)))
        return self.poll(job)

    def drain(self):
        A.check(A.load().ensemble_server_drain(self._h))

    def stats(self):
        s = A.ServerStats()
        A.check(A.load().ensemble_server_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in A.ServerStats._fields_}

    def close(self):
        if self._h:
            A.check(A.load().ensemble_server_destroy(self._h))
            self._h = None
            self._jobs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""torch.autograd integration: the record as forward, the reverse sweep as backward.

``odeint(...)`` returns the ensemble's states at the save times,
[n_save, d, n], as a differentiable function of y0 [d, n] and params
([P, n], or [P] when shared).  Its backward runs ``ensemble_adjoint`` with
the incoming gradient as the save-state cotangent.  The derivative is the
record-and-replay one (paper, Section 3.1): the exact gradient of the
discrete solution with the recorded mesh held fixed.

``frozen_mesh(...)`` records a mesh once.  Passing it back as ``mesh=`` makes
the forward a replay of that mesh (``ensemble_replay_mesh``).  That is the
function finite differences see when they perturb inputs "inside the same
recorded replay" (Appendix B.6), and it is how one record is reused while
the parameters move (Section 3.1).
"""
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import binding as B


@dataclass
class Mesh:
    """A recorded mesh as the zero-padded rectangle h [cap, n] with steps [n]."""
    h: torch.Tensor
    steps: torch.Tensor


@dataclass
class _Cfg:
    system: str
    method: str
    t0: float
    t1: float
    rtol: float
    atol: float
    save_times: Optional[Sequence[float]]
    mesh: Optional[Mesh]
    params_shared: bool
    steps_hint: int
    max_steps: int
    ckpt_every: object
    tape_budget_bytes: Optional[int]


class _EnsembleODE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, params, cfg: _Cfg):
        # the record reads y0 and params through their storage (the sweep
        # reuses them); saving the inputs lets torch's version counters
        # refuse a backward after either was changed in place
        ctx.save_for_backward(y0, params)
        y0 = y0.detach().contiguous()
        params = params.detach().contiguous()
        if cfg.mesh is None:
            rec = B.ensemble_record(cfg.system, cfg.method, y0, params, cfg.t0, cfg.t1, cfg.rtol,
                                    cfg.atol, save_times=cfg.save_times,
                                    params_shared=cfg.params_shared, steps_hint=cfg.steps_hint,
                                    max_steps=cfg.max_steps, ckpt_every=cfg.ckpt_every,
                                    tape_budget_bytes=cfg.tape_budget_bytes)
        else:
            rec = B.ensemble_replay_mesh(cfg.system, cfg.method, y0, params, cfg.t0, cfg.t1,
                                         cfg.mesh.h, cfg.mesh.steps, save_times=cfg.save_times,
                                         params_shared=cfg.params_shared,
                                         ckpt_every=cfg.ckpt_every)
        ctx.rec = rec
        ctx.mark_non_differentiable(rec.status)
        return rec.y_save, rec.status

    @staticmethod
    def backward(ctx, g, _gs):
        ctx.saved_tensors  # raises if y0 or params changed in place since forward
        rec = ctx.rec
        if g is None:
            return None, None, None
        gp, gy, _ = B.ensemble_adjoint(rec, "cotangent", g.contiguous(),
                                       want_y0=ctx.needs_input_grad[0], want_loss=False)
        return gy, (gp if ctx.needs_input_grad[1] else None), None


def odeint(system, method, y0, params, t0, t1, rtol=1e-6, atol=1e-8, save_times=None,
           mesh: Optional[Mesh] = None, params_shared=False, steps_hint=512, max_steps=0,
           ckpt_every=0, tape_budget_bytes=None, return_status=False):
    """States at the save times [n_save, d, n] (t1 alone when save_times is None).

    ckpt_every > 0 records a checkpointed tape (one state per segment of that
    many steps); the gradient is the same to the bit, the tape about 4x smaller.
    ckpt_every="auto" checkpoints every 64 steps only when the full tape's
    plan exceeds tape_budget_bytes."""
    if ckpt_every != "auto":
        ckpt_every = int(ckpt_every)
    if mesh is not None and ckpt_every == "auto":
        ckpt_every = 0
    cfg = _Cfg(system, method, float(t0), float(t1), float(rtol), float(atol),
               list(save_times) if save_times is not None else None, mesh, bool(params_shared),
               int(steps_hint), int(max_steps), ckpt_every, tape_budget_bytes)
    ys, status = _EnsembleODE.apply(y0, params, cfg)
    return (ys, status) if return_status else ys


def frozen_mesh(system, method, y0, params, t0, t1, rtol=1e-6, atol=1e-8, save_times=None,
                params_shared=False, steps_hint=512) -> Mesh:
    """Record once and return the mesh for later replays."""
    with torch.no_grad():
        rec = B.ensemble_record(system, method, y0.detach().contiguous(),
                                params.detach().contiguous(), t0, t1, rtol, atol,
                                save_times=save_times, params_shared=params_shared,
                                steps_hint=steps_hint)
        h, s = B.ensemble_mesh_export(rec)
    return Mesh(h, s)

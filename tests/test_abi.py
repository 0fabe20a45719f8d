"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_2609_02876_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ensode.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(ensemble_\w+)\(", src, re.M)))


def test_header_and_binding_agree():
    assert _declared() == sorted(A.EXPORTS)


def test_library_exports_every_symbol():
    if not os.path.exists(A.LIB_PATH):
        pytest.skip("libensode.so not built")
    lib = C.CDLL(A.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def _lib():
    if not os.path.exists(A.LIB_PATH):
        pytest.skip("libensode.so not built")
    return A.load(build_if_missing=False)


def _prob(**kw):
    d = dict(system=A.SYS_LORENZ, method=A.TSIT5, dtype=A.F64, dim=3, nparams=3, params_shared=0)
    d.update(kw)
    return A.Problem(**d)


def _ivp(**kw):
    st = (C.c_double * 2)(0.5, 1.0)
    d = dict(n=1024, y0=None, params=None, t0=0.0, t1=1.0, rtol=1e-6, atol=1e-8, h0=0.0,
             max_steps=0, n_save=2, save_times=C.cast(st, C.POINTER(C.c_double)))
    d.update(kw)
    v = A.Ivp(**d)
    v._keep = st
    return v


@pytest.mark.parametrize("system,method,d,np_", [
    (A.SYS_ROBERTSON, A.RODAS4, 3, 3), (A.SYS_HIRES, A.RODAS4, 8, 12),
    (A.SYS_LINEAR, A.RODAS4, 2, 2), (A.SYS_LINEAR, A.VERN7, 2, 2),
    (A.SYS_ROBERTSON, A.ROS23, 3, 3), (A.SYS_HIRES, A.ROS23, 8, 12),
    (A.SYS_LINEAR, A.ROS23, 2, 2)])
def test_supported_combinations_plan(system, method, d, np_):
    lib = _lib()
    out = C.c_size_t()
    prob = _prob(system=system, method=method, dim=d, nparams=np_)
    assert lib.ensemble_record_bytes(C.byref(prob), C.byref(_ivp()), 64, 0, C.byref(out)) == 0
    assert out.value > 0


def test_record_bytes_plan():
    lib = _lib()
    out = C.c_size_t()
    assert lib.ensemble_record_bytes(C.byref(_prob()), C.byref(_ivp()), 64, 0, C.byref(out)) == 0
    # 1024 trajectories x 4 pages of 16 steps x 32 bytes, plus links and the fixed part
    assert out.value > 1024 * 4 * 512
    small = out.value
    assert lib.ensemble_record_bytes(C.byref(_prob()), C.byref(_ivp()), 640, 0, C.byref(out)) == 0
    assert out.value > 9 * small


@pytest.mark.parametrize("prob,ivp,code", [
    (dict(system=99), {}, A.ENS_EUNSUPPORTED),
    (dict(dim=2), {}, A.ENS_EINVAL),
    (dict(method=7), {}, A.ENS_EUNSUPPORTED),
    (dict(dtype=5), {}, A.ENS_EUNSUPPORTED),
    ({}, dict(n=0), A.ENS_EINVAL),
    ({}, dict(t1=0.0), A.ENS_EINVAL),
    ({}, dict(rtol=-1.0), A.ENS_EINVAL),
    ({}, dict(rtol=0.0, atol=0.0), A.ENS_EINVAL),
    ({}, dict(n_save=65), A.ENS_EINVAL),
    # the Rosenbrock method: stiff systems and the linear one, FP64 only
    (dict(method=A.RODAS4), {}, A.ENS_EUNSUPPORTED),
    (dict(system=A.SYS_ROBERTSON, method=A.RODAS4, dtype=A.F32), {}, A.ENS_EUNSUPPORTED),
    (dict(system=A.SYS_ROBERTSON, method=A.TSIT5), {}, A.ENS_EUNSUPPORTED),
    (dict(system=A.SYS_HIRES, method=A.RODAS4, dim=8, nparams=3), {}, A.ENS_EINVAL),
    (dict(method=A.ROS23), {}, A.ENS_EUNSUPPORTED),
    (dict(system=A.SYS_ROBERTSON, method=A.ROS23, dtype=A.F32), {}, A.ENS_EUNSUPPORTED),
])
def test_validation_errors(prob, ivp, code):
    lib = _lib()
    out = C.c_size_t()
    rc = lib.ensemble_record_bytes(C.byref(_prob(**prob)), C.byref(_ivp(**ivp)), 64, 0, C.byref(out))
    assert rc == code
    assert len(lib.ensemble_last_error()) > 0


def test_bad_save_times_rejected():
    lib = _lib()
    st = (C.c_double * 2)(0.7, 0.2)
    v = _ivp(save_times=C.cast(st, C.POINTER(C.c_double)))
    out = C.c_size_t()
    assert lib.ensemble_record_bytes(C.byref(_prob()), C.byref(v), 64, 0, C.byref(out)) == A.ENS_EINVAL
    assert b"nondecreasing" in lib.ensemble_last_error()
    st2 = (C.c_double * 2)(0.5, 1.5)
    v = _ivp(save_times=C.cast(st2, C.POINTER(C.c_double)))
    assert lib.ensemble_record_bytes(C.byref(_prob()), C.byref(v), 64, 0, C.byref(out)) == A.ENS_EINVAL


def test_null_pointers_rejected_before_launch():
    lib = _lib()
    rec = A.Record()
    assert lib.ensemble_solve(None, None, None, None, None) == A.ENS_EINVAL
    # y0 / params NULL: refused by validation, no device call is made
    tc = A.TapeCfg(None, 0, 0)
    assert lib.ensemble_record(C.byref(_prob()), C.byref(_ivp()), C.byref(tc), C.byref(rec),
                               None, None, None) == A.ENS_EINVAL
    assert lib.ensemble_adjoint(C.byref(_prob()), C.byref(_ivp()), None, None, None, None, None,
                                None, 0, None) == A.ENS_EINVAL


def test_adjoint_workspace_plan():
    """The sweep's workspace: each save's cotangent for its base state
    ([n_save][dim][n]), plus the shared-parameter partials and the segment
    replay records of a checkpointed tape, each 256-byte aligned."""
    lib = _lib()
    out = C.c_size_t()
    rec = A.Record(n=1024, system=A.SYS_LORENZ, method=A.TSIT5, dtype=A.F64, dim=3, nparams=3,
                   params_shared=0, n_save=20, page_steps=16, ckpt_every=0)
    cot = 20 * 3 * 1024 * 8
    assert lib.ensemble_adjoint_workspace_bytes(C.byref(rec), C.byref(out)) == 0
    assert out.value == cot
    rec.params_shared = 1   # 4 blocks x 3 params x 8 bytes, 256-aligned
    assert lib.ensemble_adjoint_workspace_bytes(C.byref(rec), C.byref(out)) == 0
    assert out.value == 256 + cot
    rec.params_shared, rec.ckpt_every, rec.page_steps = 0, 64, 64   # one 64-step segment each
    assert lib.ensemble_adjoint_workspace_bytes(C.byref(rec), C.byref(out)) == 0
    assert out.value == 1024 * 64 * 32 + cot
    rec.n, rec.n_save, rec.ckpt_every, rec.page_steps = 1000, 1, 0, 16   # ragged: aligned up
    assert lib.ensemble_adjoint_workspace_bytes(C.byref(rec), C.byref(out)) == 0
    assert out.value == (3 * 1000 * 8 + 255) // 256 * 256


def test_checkpoint_plan_is_smaller():
    lib = _lib()
    full, ck = C.c_size_t(), C.c_size_t()
    assert lib.ensemble_record_bytes(C.byref(_prob()), C.byref(_ivp()), 640, 0, C.byref(full)) == 0
    assert lib.ensemble_record_bytes(C.byref(_prob()), C.byref(_ivp()), 640, 64, C.byref(ck)) == 0
    assert ck.value < full.value / 3
    assert lib.ensemble_record_bytes(C.byref(_prob()), C.byref(_ivp()), 640, 48, C.byref(ck)) == A.ENS_EINVAL


def test_tape_plan_switches_to_checkpoints_over_budget():
    """Full tape while its plan fits the HBM budget, checkpoint-64 above it,
    an error when even the checkpointed plan does not fit (host logic only)."""
    _lib()
    from paper_2609_02876_amd import binding as B
    args = ("lorenz", "tsit5", 1 << 20, 0.0, 10.0, 352, 20)
    full = B.ensemble_record_bytes(*args)
    ck = B.ensemble_record_bytes(*args, ckpt_every=64)
    assert ck < full / 3
    assert B.plan_tape(*args) == 0
    assert B.plan_tape(*args, budget_bytes=full) == 0
    assert B.plan_tape(*args, budget_bytes=full - 1) == 64
    with pytest.raises(ValueError):
        B.plan_tape(*args, budget_bytes=ck - 1)


@pytest.mark.parametrize("kw,code", [
    ({}, 0),
    (dict(params_shared=0), A.ENS_EINVAL),
    (dict(dtype=A.F64), A.ENS_EUNSUPPORTED),
    (dict(method=A.VERN7), A.ENS_EUNSUPPORTED),
])
def test_ude_problem_checks(kw, code):
    """The UDE runs Tsit5 in F32 with its 1218 network weights shared."""
    lib = _lib()
    out = C.c_size_t()
    d = dict(system=A.SYS_LV_UDE, method=A.TSIT5, dtype=A.F32, dim=2, nparams=1218,
             params_shared=1)
    d.update(kw)
    rc = lib.ensemble_record_bytes(C.byref(A.Problem(**d)), C.byref(_ivp()), 64, 0, C.byref(out))
    assert rc == code


def test_ude_pool_plan_through_the_binding():
    _lib()
    import torch
    from paper_2609_02876_amd import binding as B
    full = B.ensemble_record_bytes("ude", "tsit5", 4096, 0.0, 10.0, 256, 20, torch.float32)
    ck = B.ensemble_record_bytes("ude", "tsit5", 4096, 0.0, 10.0, 256, 20, torch.float32, 64)
    assert 0 < ck < full
    assert B.plan_tape("ude", "tsit5", 4096, 0.0, 10.0, 256, 20, torch.float32,
                       budget_bytes=full - 1) == 64


def test_refresh_rejects_bad_slack_and_the_ude():
    """ensemble_refresh's argument checks run on the host, before any launch."""
    lib = _lib()
    rec = A.Record()
    tc = A.TapeCfg(1 << 20, 1 << 20, 0, 0)
    dummy = C.c_void_p(1 << 20)   # never dereferenced: the checks fail first
    for slack in (-1.0, float("nan")):
        rc = lib.ensemble_refresh(C.byref(_prob()), C.byref(_ivp()), C.byref(tc), dummy, dummy,
                                  4, slack, C.byref(rec), dummy, None, None, None)
        assert rc == A.ENS_EINVAL and b"slack" in lib.ensemble_last_error()
    ude = _prob(system=A.SYS_LV_UDE, dtype=A.F32, dim=2, nparams=1218, params_shared=1)
    rc = lib.ensemble_refresh(C.byref(ude), C.byref(_ivp()), C.byref(tc), dummy, dummy, 4, 1.0,
                              C.byref(rec), dummy, None, None, None)
    assert rc == A.ENS_EUNSUPPORTED
    rc = lib.ensemble_refresh(C.byref(_prob()), C.byref(_ivp()), C.byref(tc), None, dummy, 4,
                              1.0, C.byref(rec), dummy, None, None, None)
    assert rc == A.ENS_EINVAL

"""Systems registered at run time (compiled with hipRTC), through the C ABI.

A registered copy of a built-in system, written with the same operations,
runs the same kernels compiled from the same headers with the same flags, so
its record, reverse sweep and forward mode equal the built-in system's to the
bit; the built-in systems are pinned to the oracle (test_gpu_parity,
test_gpu_rosenbrock, test_gpu_jvp), which pins the registered path in turn.
Registered Lorenz and Robertson are also compared with the oracle directly
(mesh statistics against its adaptive record; states, gradients and forward
tangents against it on the GPU's mesh).  A system with no built-in
counterpart has no oracle: its gradients are checked against central
differences of the replay on the frozen mesh and against the forward mode.
"""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import own_mesh_parity
from paper_2609_02876_amd import _abi as A
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import serving as SV
from paper_2609_02876_amd import user_systems as U
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _name(base):
    if base not in A.SYSTEMS:
        src = {"rtc_lorenz": U.LORENZ, "rtc_robertson": U.ROBERTSON}[base]
        B.register_system(base, src, 3, 3, jacobian=(base == "rtc_robertson"))
    return base


def _run(system, method, y0, p, t1, rtol, atol, st, dtype, **kw):
    h = B.ensemble_record(system, method, _dev(y0.T, dtype), _dev(p.T, dtype), 0.0, t1, rtol,
                          atol, save_times=st, steps_hint=2048 if method == "ros23" else 512,
                          **kw)
    gp, gy, ll = B.ensemble_adjoint(h)
    rng = np.random.default_rng(4)
    dp = _dev((rng.standard_normal(p.shape) * p).T, dtype)
    ysd, ld = B.ensemble_jvp(h, None, dp)
    torch.cuda.synchronize()
    return [h.y_save, h.status, h.steps(), gp, gy, ll, ysd, ld]


@pytest.mark.parametrize("base,system,method,t1,rtol,atol", [
    ("rtc_lorenz", O.LORENZ, "tsit5", 10.0, 1e-6, 1e-8),
    ("rtc_lorenz", O.LORENZ, "vern7", 10.0, 1e-8, 1e-8),
    ("rtc_robertson", O.ROBERTSON, "rodas4", 1e5, 1e-6, 1e-10),
    ("rtc_robertson", O.ROBERTSON, "ros23", 1e5, 1e-6, 1e-10),
])
def test_registered_systems_match_oracle(base, system, method, t1, rtol, atol):
    """A registered system against the oracle itself, not only against the
    built-in kernel: its adaptive mesh by the statistics, its save states,
    sweep gradients and forward-mode tangents on its own mesh."""
    print(f"case registered {base} {method} against the oracle", flush=True)
    n = 500
    y0, p = (W.lorenz if system == O.LORENZ else W.robertson)(n, seed=9)
    st = list(W.save_times(0.0, t1, 20))
    mo = {"tsit5": O.TSIT5, "vern7": O.VERN7, "rodas4": O.RODAS, "ros23": O.ROS23}[method]
    h = B.ensemble_record(_name(base), method, _dev(y0.T), _dev(p.T), 0.0, t1, rtol, atol,
                          save_times=st, steps_hint=2048 if method == "ros23" else 512)
    gp, gy, _ = B.ensemble_adjoint(h)
    rng = np.random.default_rng(10)
    dp = rng.standard_normal(p.shape) * p
    ysd, _ = B.ensemble_jvp(h, None, _dev(dp.T))
    torch.cuda.synchronize()
    assert np.all(h.status.cpu().numpy() == 0)
    ref = O.record(system, mo, y0, p, 0.0, t1, rtol, atol, save_t=st)
    own_mesh_parity(h, system, mo, y0, p, ref, 1e-11, gp=gp, gy=gy)
    from gpu_helpers import oracle_mesh, rel
    _, dys = O.replay_dual(system, mo, y0, p, np.zeros_like(y0), dp, oracle_mesh(h))
    e = rel(ysd.cpu().numpy(), np.transpose(dys, (1, 2, 0))).max()
    print(f"  forward tangents vs oracle dual replay: {e:.2e}")
    assert e <= 1e-11


@pytest.mark.parametrize("method,dtype", [("tsit5", torch.float64), ("vern7", torch.float64),
                                          ("tsit5", torch.float32)])
def test_registered_lorenz_equals_builtin(method, dtype):
    print(f"case registered lorenz {method} {dtype}", flush=True)
    n = 1000
    y0, p = W.lorenz(n, seed=2)
    st = list(W.save_times(0.0, 10.0, 20))
    a = _run("lorenz", method, y0, p, 10.0, 1e-6, 1e-8, st, dtype)
    b = _run(_name("rtc_lorenz"), method, y0, p, 10.0, 1e-6, 1e-8, st, dtype)
    assert np.all(a[1].cpu().numpy() == 0)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("method", ["rodas4", "ros23"])
def test_registered_robertson_rosenbrock_equals_builtin(method):
    print(f"case registered robertson {method}", flush=True)
    n = 513
    y0, p = W.robertson(n, seed=3)
    st = list(W.save_times(0.0, 1e5, 20))
    a = _run("robertson", method, y0, p, 1e5, 1e-6, 1e-10, st, torch.float64)
    b = _run(_name("rtc_robertson"), method, y0, p, 1e5, 1e-6, 1e-10, st, torch.float64)
    assert np.all(a[1].cpu().numpy() == 0)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_registered_checkpointed_and_shared():
    n = 700
    y0, p = W.lorenz(n, seed=5)
    st = list(W.save_times(0.0, 10.0, 20))
    for kw in (dict(ckpt_every=16),):
        a = _run("lorenz", "tsit5", y0, p, 10.0, 1e-6, 1e-8, st, torch.float64, **kw)
        b = _run(_name("rtc_lorenz"), "tsit5", y0, p, 10.0, 1e-6, 1e-8, st, torch.float64, **kw)
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    # shared parameters: one (sigma, rho, beta) for all trajectories
    outs = []
    for system in ("lorenz", _name("rtc_lorenz")):
        h = B.ensemble_record(system, "tsit5", _dev(y0.T), _dev(p[0]), 0.0, 10.0, 1e-6, 1e-8,
                              save_times=st, params_shared=True, steps_hint=512)
        outs.append(B.ensemble_adjoint(h))
    torch.cuda.synchronize()
    for x, y in zip(*outs):
        assert torch.equal(x, y)


BRUSSELATOR = """
struct System {
  // Brusselator, p = (a, b): x' = a - (b + 1) x + x^2 y,  y' = b x - x^2 y
  template <class T>
  __device__ static void rhs(const T* y, const T* p, T* f) {
    const T xxy = (y[0] * y[0]) * y[1];
    f[0] = fmaT(-(p[1] + T(1)), y[0], p[0] + xxy);
    f[1] = fmaT(p[1], y[0], -xxy);
  }
  template <class T>
  __device__ static void vjp(const T* y, const T* p, const T* w, T* gy, T* gp) {
    const T d = w[0] - w[1];
    const T xy2 = T(2) * (y[0] * y[1]);
    gy[0] = fmaT(xy2, d, fmaT(p[1], w[1], -((p[1] + T(1)) * w[0])));
    gy[1] = (y[0] * y[0]) * d;
    gp[0] = gp[0] + w[0];
    gp[1] = fmaT(y[0], w[1] - w[0], gp[1]);
  }
};
"""


def test_new_system_gradients_against_differences_and_forward_mode():
    """A system with no built-in copy: the reverse gradient against central
    differences of the replay on the frozen mesh (relative step 1e-6) and
    against one forward pass per parameter."""
    if "rtc_brusselator" not in A.SYSTEMS:
        B.register_system("rtc_brusselator", BRUSSELATOR, 2, 2)
    n = 256
    rng = np.random.default_rng(6)
    y0 = np.column_stack([1.0 + 0.5 * rng.random(n), 2.0 + 0.5 * rng.random(n)])
    p = np.column_stack([1.0 + 0.2 * rng.random(n), 2.5 + 0.5 * rng.random(n)])
    st = list(W.save_times(0.0, 8.0, 20))
    h = B.ensemble_record("rtc_brusselator", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 8.0, 1e-8,
                          1e-10, save_times=st, steps_hint=1024)
    gp, gy, ll = B.ensemble_adjoint(h)
    cap = int(h.steps().max().item())
    hm, sm = B.ensemble_mesh_export(h, cap)
    torch.cuda.synchronize()
    assert np.all(h.status.cpu().numpy() == 0)
    g = gp.cpu().numpy()
    for k in range(2):
        eps = 1e-6 * p[:, k]
        losses = []
        for sgn in (1.0, -1.0):
            q = p.copy()
            q[:, k] += sgn * eps
            r = B.ensemble_replay_mesh("rtc_brusselator", "tsit5", _dev(y0.T), _dev(q.T), 0.0,
                                       8.0, hm, sm, save_times=st)
            _, _, lq = B.ensemble_adjoint(r)
            torch.cuda.synchronize()
            losses.append(lq.cpu().numpy())
        fd = (losses[0] - losses[1]) / (2 * eps)
        e_fd = np.max(np.abs(fd - g[k]) / np.maximum(np.abs(g[k]), 1e-3 * np.abs(g[k]).max()))
        t = torch.zeros((2, n), dtype=torch.float64, device="cuda")
        t[k] = 1.0
        _, ld = B.ensemble_jvp(h, None, t, want_states=False)
        torch.cuda.synchronize()
        e_fw = np.max(np.abs(ld.cpu().numpy() - g[k])) / np.abs(g[k]).max()
        print(f"  param {k}: reverse vs differences {e_fd:.2e}, vs forward {e_fw:.2e}")
        assert e_fd <= 1e-6 and e_fw <= 1e-12


def test_registered_systems_are_not_served():
    y0, p = W.lorenz(64, seed=0)
    srv = SV.Server(1 << 28, n_slots=1)
    with pytest.raises(A.EnsembleError, match="not served"):
        srv.submit(_name("rtc_lorenz"), "tsit5", _dev(y0.T), _dev(p.T), 0.0, 1.0, 1e-6, 1e-8)
    srv.close()


@pytest.mark.parametrize("method", ["rodas4", "ros23"])
def test_registered_jacobian_pattern(method):
    """A registered system may declare its Jacobian's nonzero pattern
    (JAC_ROWS); the Rosenbrock factorisation then skips the structural
    zeros.  A registered Robertson with its pattern gives the same bits as
    the built-in one (which declares the same) and as a registered copy
    without it (the dense factorisation)."""
    print(f"case registered robertson with JAC_ROWS, {method}", flush=True)
    if "rtc_robertson_pattern" not in A.SYSTEMS:
        src = U.ROBERTSON.replace("struct System {",
                                  "struct System {\n  static constexpr unsigned JAC_ROWS[3] = "
                                  "{0x7u, 0x7u, 0x2u};", 1)
        B.register_system("rtc_robertson_pattern", src, 3, 3, jacobian=True)
    n = 300
    y0, p = W.robertson(n, seed=12)
    st = list(W.save_times(0.0, 1e5, 10))
    pat = _run("rtc_robertson_pattern", method, y0, p, 1e5, 1e-6, 1e-10, st, torch.float64)
    built = _run("robertson", method, y0, p, 1e5, 1e-6, 1e-10, st, torch.float64)
    dense = _run(_name("rtc_robertson"), method, y0, p, 1e5, 1e-6, 1e-10, st, torch.float64)
    for a, b, c in zip(pat, built, dense):
        if a is None:
            continue
        assert torch.equal(a, b) and torch.equal(a, c)


def _chain16_source():
    """A 16-dimensional linear chain written out term by term (no loops in a
    registered source): f_i = -p_(i mod 4) y_i + y_(i+1 mod 16)."""
    d = 16
    rhs = "\n".join(f"    f[{i}] = fmaT(-p[{i % 4}], y[{i}], y[{(i + 1) % d}]);" for i in range(d))
    gy = "\n".join(f"    gy[{i}] = fmaT(-p[{i % 4}], w[{i}], w[{(i - 1) % d}]);" for i in range(d))
    gp = "\n".join(f"    gp[{k}] = gp[{k}] - (" + " + ".join(f"y[{i}] * w[{i}]" for i in range(k, d, 4))
                   + ");" for k in range(4))
    return ("struct System {\n  template <class T>\n  __device__ static void rhs(const T* y, const T* p, T* f) {\n"
            + rhs + "\n  }\n  template <class T>\n"
            "  __device__ static void vjp(const T* y, const T* p, const T* w, T* gy, T* gp) {\n"
            + gy + "\n" + gp + "\n  }\n};\n")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_registered_wide_system_tape(dtype):
    """The widest registered state (16 components: 136-byte FP64 records, a group
    of four records is 34 chunks of 16 bytes, one group per cooperative write
    round and 152 KB of LDS a block): replaying the exported mesh, whose tape
    each lane writes on its own, gives the record's save states and gradients
    to the bit."""
    if "rtc_chain16" not in A.SYSTEMS:
        B.register_system("rtc_chain16", _chain16_source(), 16, 4)
    n, t1 = 200, 4.0
    rng = np.random.default_rng(16)
    y0 = rng.standard_normal((n, 16))
    p = 0.5 + rng.random((n, 4))
    st = [1.0, 2.0, 2.5, 4.0]
    print(f"case registered chain16 {dtype} n={n}", flush=True)
    h = B.ensemble_record("rtc_chain16", "tsit5", _dev(y0.T, dtype), _dev(p.T, dtype), 0.0, t1,
                          1e-6, 1e-8, save_times=st, steps_hint=256)
    gp, gy, ll = B.ensemble_adjoint(h)
    hm, S = B.ensemble_mesh_export(h)
    r = B.ensemble_replay_mesh("rtc_chain16", "tsit5", _dev(y0.T, dtype), _dev(p.T, dtype), 0.0,
                               t1, hm, S, save_times=st)
    gp2, gy2, ll2 = B.ensemble_adjoint(r)
    torch.cuda.synchronize()
    assert np.all(h.status.cpu().numpy() == 0) and int(S.min().item()) > 8
    assert torch.equal(h.y_save, r.y_save)
    assert torch.equal(gp, gp2) and torch.equal(gy, gy2) and torch.equal(ll, ll2)

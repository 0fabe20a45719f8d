"""Seeded synthetic ensembles (inputs only; no solver arithmetic here).

Both the GPU path and the CPU oracle are fed from these generators, so the
two sides see the same float64 arrays.  Shapes follow the paper's problem
statement (Section 2: n trajectories of y' = f(t, y, theta), theta per
trajectory) with the parameter spreads of the workloads this library is
measured on.  Arrays are per-trajectory rows: y0 [n, d], params [n, P].
"""
import numpy as np

LORENZ_Y0 = (1.0, 0.0, 0.0)
VDP_Y0 = (2.0, 0.0)


def save_times(t0, t1, k=20):
    """k evenly spaced save times t0 + (t1 - t0) s / k, s = 1..k; the last is t1 exactly."""
    t = [t0 + (t1 - t0) * s / k for s in range(1, k + 1)]
    t[-1] = t1
    return np.array(t, dtype=np.float64)


def lorenz(n, seed=0):
    """Lorenz ensemble: y0 = (1,0,0); sigma ~ U[9,11], rho ~ U[27,29], beta ~ U[2.5,3]."""
    u = np.random.default_rng(seed).random((n, 3))
    p = np.stack([9.0 + 2.0 * u[:, 0], 27.0 + 2.0 * u[:, 1], 2.5 + 0.5 * u[:, 2]], 1)
    y0 = np.tile(np.array(LORENZ_Y0), (n, 1))
    return y0, p


def lorenz_paper_timing(n, seed=0):
    """The paper's Lorenz timing ensemble (Appendix A): sigma = 10, beta = 8/3, rho ~ U[0,21]."""
    rho = 21.0 * np.random.default_rng(seed).random(n)
    p = np.stack([np.full(n, 10.0), rho, np.full(n, 8.0 / 3.0)], 1)
    return np.tile(np.array(LORENZ_Y0), (n, 1)), p


def vdp(n, seed=0):
    """Van der Pol ensemble: y0 = (2, 0); mu ~ U[0.5, 2]."""
    u = np.random.default_rng(seed).random((n, 1))
    return np.tile(np.array(VDP_Y0), (n, 1)), 0.5 + 1.5 * u


ROBERTSON_K = (0.04, 3e7, 1e4)
HIRES_THETA = (1.71, 0.43, 8.32, 0.0007, 8.75, 10.03, 0.035, 1.12, 1.745, 280.0, 0.69, 1.81)
HIRES_Y0 = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0057)


def robertson(n, seed=0):
    """Robertson kinetics: y0 = (1,0,0); (k1, k2, k3) = (0.04, 3e7, 1e4), each
    scaled by exp(U[log 0.8, log 1.25]) (log-uniform in [0.8, 1.25])."""
    rng = np.random.default_rng(seed)
    k = np.array(ROBERTSON_K) * np.exp(rng.uniform(np.log(0.8), np.log(1.25), (n, 3)))
    return np.tile([1.0, 0.0, 0.0], (n, 1)), k


def hires(n, seed=0):
    """HIRES: y0 = (1,0,0,0,0,0,0,0.0057); the twelve rate constants each scaled by U[0.9, 1.1]."""
    rng = np.random.default_rng(seed)
    return np.tile(np.array(HIRES_Y0), (n, 1)), np.array(HIRES_THETA) * rng.uniform(0.9, 1.1, (n, 12))


UDE_HIDDEN = 32
UDE_NP = 2 * 32 + 32 + 32 * 32 + 32 + 32 * 2 + 2   # 1218


def ude_weights(seed=0, scale=0.1):
    """MLP 2-32-32-2 parameters in the order W1 [32][2], b1, W2 [32][32], b2,
    W3 [2][32], b3: Glorot-uniform weights (bound sqrt(6 / (fan_in + fan_out)))
    times `scale`, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((32, 2), (32, 32), (2, 32)):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(scale * rng.uniform(-a, a, (fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    th = np.concatenate(parts)
    assert th.size == UDE_NP
    return th


def ude(n, seed=0):
    """Lotka-Volterra UDE ensemble: y0 ~ U[0.5, 2]^2 per trajectory; the MLP
    weights (shared by all trajectories) from ude_weights(seed 0)."""
    y0 = np.random.default_rng(seed).uniform(0.5, 2.0, (n, 2))
    return y0, ude_weights(0)


def ude_teacher():
    """Teacher weights of the synthetic targets (seed 1)."""
    return ude_weights(1)


def damped_rotation(n, seed=0):
    """Linear test ensemble y' = A y, A = [[-a, -w], [w, -a]]: a ~ U[0.05,0.35], w ~ U[0.5,2.5], y0 ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    u = rng.random((n, 2))
    p = np.stack([0.05 + 0.3 * u[:, 0], 0.5 + 2.0 * u[:, 1]], 1)
    return rng.normal(size=(n, 2)), p


# Named workloads.  "lorenz_2p20_t10" is the headline measurement: 2^20
# Lorenz trajectories on [0, 10], Tsit5, FP64, rtol 1e-6, atol 1e-8, loss =
# sum of squared states at 20 evenly spaced save times, gradient with respect
# to the three per-trajectory parameters.  "lorenz_1024_t1" is the small
# parity case: loss = sum of squared final states on [0, 1].
WORKLOADS = {
    "lorenz_1024_t1": dict(system="lorenz", method="tsit5", n=1024, t0=0.0, t1=1.0,
                           rtol=1e-6, atol=1e-8, n_save=0),
    "lorenz_2p20_t10": dict(system="lorenz", method="tsit5", n=1 << 20, t0=0.0, t1=10.0,
                            rtol=1e-6, atol=1e-8, n_save=20),
    # the same with a checkpointed tape: a state every 64 steps and the step
    # sizes, the segments replayed in the sweep
    "lorenz_2p20_t10_ckpt64": dict(system="lorenz", method="tsit5", n=1 << 20, t0=0.0,
                                   t1=10.0, rtol=1e-6, atol=1e-8, n_save=20, ckpt_every=64),
    # stiff: Rodas4, FP64, rtol 1e-6, atol 1e-10, loss on 20 save states
    "robertson_2p18_t1e5": dict(system="robertson", method="rodas4", n=1 << 18, t0=0.0,
                                t1=1e5, rtol=1e-6, atol=1e-10, n_save=20),
    "hires_2p18": dict(system="hires", method="rodas4", n=1 << 18, t0=0.0, t1=321.8122,
                       rtol=1e-6, atol=1e-10, n_save=20),
    # the same two with checkpointed tapes (a state every 64 steps)
    "robertson_2p18_t1e5_ckpt64": dict(system="robertson", method="rodas4", n=1 << 18,
                                       t0=0.0, t1=1e5, rtol=1e-6, atol=1e-10, n_save=20,
                                       ckpt_every=64),
    "hires_2p18_ckpt64": dict(system="hires", method="rodas4", n=1 << 18, t0=0.0,
                              t1=321.8122, rtol=1e-6, atol=1e-10, n_save=20, ckpt_every=64),
    # the same two with Rosenbrock23 (order 2, three stages in a trial step)
    "robertson_ros23_2p18_t1e5": dict(system="robertson", method="ros23", n=1 << 18, t0=0.0,
                                      t1=1e5, rtol=1e-6, atol=1e-10, n_save=20),
    "hires_ros23_2p18": dict(system="hires", method="ros23", n=1 << 18, t0=0.0,
                             t1=321.8122, rtol=1e-6, atol=1e-10, n_save=20),
    # UDE: Lotka-Volterra + MLP 2-32-32-2 (weights shared), Tsit5, FP32,
    # rtol = atol = 1e-6, 20 save times t = 0.5 s, loss = MSE to the teacher
    # network's trajectories, tape checkpointed every 64 steps (or full)
    "ude_2p16": dict(system="ude", method="tsit5", n=1 << 16, t0=0.0, t1=10.0, rtol=1e-6,
                     atol=1e-6, n_save=20, dtype="f32", shared=True, loss="mse",
                     ckpt_every=64),
    "ude_2p16_full": dict(system="ude", method="tsit5", n=1 << 16, t0=0.0, t1=10.0,
                          rtol=1e-6, atol=1e-6, n_save=20, dtype="f32", shared=True,
                          loss="mse", ckpt_every=0),
    # the paper's forward-only timing (Section 4.1, Appendix A): Lorenz with
    # sigma = 10, beta = 8/3, rho ~ U[0, 21], y0 = (1, 0, 0), t in [0, 1],
    # Tsit5, rtol 1e-6, atol 1e-9, 2^20 trajectories, to the final state
    "lorenz_paper_fwd_2p20": dict(system="lorenz", method="tsit5", n=1 << 20, t0=0.0, t1=1.0,
                                  rtol=1e-6, atol=1e-9, n_save=0, gen="lorenz_paper_timing"),
    "lorenz_paper_fwd_2p20_f32": dict(system="lorenz", method="tsit5", n=1 << 20, t0=0.0,
                                      t1=1.0, rtol=1e-6, atol=1e-9, n_save=0, dtype="f32",
                                      gen="lorenz_paper_timing"),
}

GENERATORS = {"lorenz": lorenz, "vdp": vdp, "robertson": robertson, "hires": hires,
              "linear": damped_rotation, "ude": ude}


def make(name, n=None, seed=0):
    """(config, y0, params, save_t) of a named workload, optionally resized."""
    cfg = dict(WORKLOADS[name])
    if n is not None:
        cfg["n"] = n
    gen = {"lorenz_paper_timing": lorenz_paper_timing}[cfg["gen"]] if "gen" in cfg else \
        GENERATORS[cfg["system"]]
    y0, p = gen(cfg["n"], seed)
    st = save_times(cfg["t0"], cfg["t1"], cfg["n_save"]) if cfg["n_save"] else np.array([cfg["t1"]])
    return cfg, y0, p, st

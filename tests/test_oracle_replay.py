"""Pins for the oracle's replay map Phi (paper, eq. stages/update/replay).

* P2: convergence order 5 (Tsit5) and 7 (Vern7) of the fixed-step replay.
* P3: for y' = A y the replay is exactly y_S = prod_i R(h_i A) y0 with R the
  stability polynomial of the tableau, built here from b^T A^(k-1) 1 -- a
  different computation from the stage loop.
* P9: zero-length steps appended to a mesh change nothing (paper, Section 3.1,
  zero padding).
* the record and the replay of its mesh give bit-identical states.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
from oracle_helpers import (lorenz_params, make_mesh, mesh_times, rot_matrix,
                            stability_coeffs, stability_matrix)

RNG = np.random.default_rng(0)


@pytest.mark.parametrize("method,p,N", [(O.TSIT5, 5, 160), (O.VERN7, 7, 40)])
def test_convergence_order_linear(method, p, N):
    a, w, T = 0.1, 1.0, 10.0
    y0 = np.array([[1.0, 0.5]])
    errs = []
    for n_steps in (N, 2 * N):
        m = make_mesh([[T / n_steps] * n_steps], [T], 0.0, T)
        ys = O.replay(O.LINEAR, method, y0, np.array([[a, w]]), m)[0, -1]
        exact = expm(rot_matrix(a, w) * T) @ y0[0]
        errs.append(np.linalg.norm(ys - exact))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - p) < 0.25, (errs, rate)


@pytest.mark.parametrize("method,p,N,T", [(O.TSIT5, 5, 400, 1.0), (O.VERN7, 7, 100, 1.0)])
def test_convergence_order_lorenz(method, p, N, T):
    y0 = np.array([[1.0, 0.0, 0.0]]); prm = np.array([[10.0, 28.0, 8.0 / 3.0]])
    sol = []
    for n_steps in (N, 2 * N, 4 * N):
        m = make_mesh([[T / n_steps] * n_steps], [T], 0.0, T)
        sol.append(O.replay(O.LORENZ, method, y0, prm, m)[0, -1])
    r = np.linalg.norm(sol[0] - sol[1]) / np.linalg.norm(sol[1] - sol[2])
    assert abs(np.log2(r) - p) < 0.25, np.log2(r)


@pytest.mark.parametrize("method", [O.TSIT5, O.VERN7])
def test_discrete_closed_form_linear(method):
    g = stability_coeffs(method)
    n = 6
    prm = np.stack([0.05 + 0.3 * RNG.random(n), 0.5 + 2 * RNG.random(n)], 1)
    y0 = RNG.normal(size=(n, 2))
    save_t = np.linspace(0.5, 8.0, 16)
    rec = O.record(O.LINEAR, method, y0, prm, 0.0, 8.0, 1e-6, 1e-8, save_t=save_t)
    assert np.all(rec["status"] == O.ST_OK)
    ys = O.replay(O.LINEAR, method, y0, prm, rec)
    for l in range(n):
        A = rot_matrix(*prm[l])
        y = y0[l].copy(); states = [y.copy()]
        for i in range(rec["S"][l]):
            y = stability_matrix(g, rec["h"][l, i] * A) @ y
            states.append(y.copy())
        for s in range(len(save_t)):
            base = states[rec["save_idx"][l, s]]
            ref = stability_matrix(g, rec["save_dt"][l, s] * A) @ base
            assert np.allclose(ys[l, s], ref, rtol=1e-12, atol=1e-14 * np.linalg.norm(ref))


def test_replay_reproduces_record_bitwise():
    n = 64
    y0 = np.tile([1.0, 0.0, 0.0], (n, 1)); prm = lorenz_params(n)
    for method in (O.TSIT5, O.VERN7):
        st = [0.5 * s for s in range(1, 21)]
        rec = O.record(O.LORENZ, method, y0, prm, 0.0, 10.0, 1e-6, 1e-8, save_t=st)
        assert np.all(rec["status"] == O.ST_OK)
        assert np.array_equal(O.replay(O.LORENZ, method, y0, prm, rec), rec["y_save"])


def test_save_time_bookkeeping():
    n = 32
    y0 = np.tile([2.0, 0.0], (n, 1)); mu = 0.5 + 1.5 * RNG.random((n, 1))
    st = [6.3 * s / 20 for s in range(1, 20)] + [6.3]
    rec = O.record(O.VDP, O.TSIT5, y0, mu, 0.0, 6.3, 1e-6, 1e-8, save_t=st)
    for l in range(n):
        S = rec["S"][l]
        t = mesh_times(rec["h"][l], S, 0.0, 6.3)
        assert abs(np.sum(rec["h"][l, :S]) - 6.3) < 1e-12
        for s, ts in enumerate(st):
            i = rec["save_idx"][l, s]
            assert t[i] <= ts and (i == S or t[i + 1] > ts)
            assert rec["save_dt"][l, s] == ts - t[i]
        assert rec["save_idx"][l, -1] == S and rec["save_dt"][l, -1] == 0.0
        assert np.array_equal(rec["y_save"][l, -1], O.replay(O.VDP, O.TSIT5, y0[l:l + 1], mu[l:l + 1], {k: (v[l:l + 1] if hasattr(v, 'shape') and v.ndim else v) for k, v in rec.items() if k in ('h', 'S', 'save_idx', 'save_dt')})[0, -1])


@pytest.mark.parametrize("method", [O.TSIT5, O.VERN7])
def test_zero_padding_is_identity(method):
    n = 16
    y0 = np.tile([1.0, 0.0, 0.0], (n, 1)); prm = lorenz_params(n, seed=3)
    st = [0.25, 0.5, 1.0]
    rec = O.record(O.LORENZ, method, y0, prm, 0.0, 1.0, 1e-6, 1e-8, save_t=st)
    S = rec["S"]; Smax = int(S.max()) + 7
    pad = dict(h=np.zeros((n, Smax)), S=np.full(n, Smax, np.int32),
               save_idx=rec["save_idx"].copy(), save_dt=rec["save_dt"].copy())
    for l in range(n):
        pad["h"][l, : S[l]] = rec["h"][l, : S[l]]
        pad["save_idx"][l][pad["save_idx"][l] == S[l]] = Smax
    assert np.array_equal(O.replay(O.LORENZ, method, y0, prm, pad), rec["y_save"])
    g1 = O.adjoint(O.LORENZ, method, y0, prm, rec)
    g2 = O.adjoint(O.LORENZ, method, y0, prm, pad)
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)

"""Helpers shared by the oracle pin tests (no method arithmetic in here)."""
import numpy as np

import oracle as O
from paper_2609_02876_amd import workloads


def mesh_times(h_row, S, t0, t1):
    """Mesh points t_0..t_S rebuilt by the same additions the record makes."""
    t = [t0]
    for i in range(S):
        t.append(t1 if i == S - 1 else t[-1] + h_row[i])
    return np.array(t)


def make_mesh(h_lists, save_t, t0, t1=None):
    """Mesh dict for explicit per-lane step lists (the last point is t1)."""
    n = len(h_lists)
    cap = max(1, max(len(h) for h in h_lists))
    save_t = np.asarray(save_t, float)
    H = np.zeros((n, cap)); S = np.zeros(n, np.int32)
    sidx = np.zeros((n, len(save_t)), np.int32); sdt = np.zeros((n, len(save_t)))
    for l, hl in enumerate(h_lists):
        H[l, : len(hl)] = hl; S[l] = len(hl)
        tl = mesh_times(hl, len(hl), t0, t1 if t1 is not None else t0 + float(np.sum(hl)))
        for s, ts in enumerate(save_t):
            i = int(np.max(np.nonzero(tl <= ts)[0]))
            sidx[l, s] = i; sdt[l, s] = ts - tl[i]
    return dict(h=H, S=S, save_idx=sidx, save_dt=sdt)


def lorenz_params(n, seed=0):
    return workloads.lorenz(n, seed)[1]


def rot_matrix(a, w):
    return np.array([[-a, -w], [w, -a]])


def stability_coeffs(method):
    """g_k = b^T A^(k-1) 1, k = 0..s (g_0 = 1): R(z) = sum_k g_k z^k."""
    tb = O.erk_tableau(method)
    A, b = tb["A"], tb["b"]
    g = [1.0]
    v = np.ones(tb["s"])
    for _ in range(tb["s"]):
        g.append(float(b @ v))
        v = A @ v
    return np.array(g)


def stability_matrix(g, Z):
    """R(Z) = sum_k g_k Z^k for a square matrix Z (complex allowed)."""
    R = np.zeros_like(Z); P = np.eye(Z.shape[0], dtype=Z.dtype)
    for gk in g:
        R = R + gk * P
        P = P @ Z
    return R

"""The noise floor of an adaptive mesh (the reading behind the mesh
statistics of the GPU tests).

The error estimate e = h sum_j (b_j - bhat_j) k_j is a small difference of
large stage terms: at rtol 1e-6 on Lorenz it is about 1e-6 of |h k|, so one
rounding of the stages moves it by about 1e-10 relative, and the controller
passes that on to the next step size.  Two controllers that form the same
factor 0.9 err^(-1/5) to within an ulp -- here err^(-1/5) against
(err^2)^(-1/10), and the same factor moved by one ulp -- therefore give
meshes with the same step counts whose step sizes differ by 1e-11..1e-8
relative within 50 steps: bit-identical meshes need bit-identical
controller arithmetic, and agreement far below 1e-8 is not a property the
method has.  A plain float64 Tsit5 loop on the CPU (coefficients from the
oracle) shows it.
"""
import numpy as np

import oracle as O
from paper_2609_02876_amd import workloads as W


def _run(tb, y0, p, t1, factor, rtol=1e-6, atol=1e-8):
    A, ew, s = tb["A"], tb["ew"], tb["s"]

    def f(y):
        return np.array([p[0] * (y[1] - y[0]), y[0] * (p[1] - y[2]) - y[1],
                         y[0] * y[1] - p[2] * y[2]])

    y, t, k1, h, prev, hs = y0.copy(), 0.0, f(y0), 1e-3, False, []
    while t < t1:
        last = t + h >= t1
        if last:
            h = t1 - t
        ks = [k1]
        for i in range(1, s):
            ks.append(f(y + h * sum(A[i, j] * ks[j] for j in range(i))))
        ynew = y + h * sum(A[s - 1, j] * ks[j] for j in range(s - 1))
        e = h * sum(ew[j] * ks[j] for j in range(s))
        ms = float(np.mean((e / (atol + rtol * np.maximum(abs(y), abs(ynew)))) ** 2))
        fac = factor(ms)
        if ms <= 1.0:
            hs.append(h)
            t, y, k1 = (t1 if last else t + h), ynew, ks[-1]
            h, prev = h * max(0.2, min(1.0 if prev else 10.0, fac)), False
        else:
            h, prev = h * max(0.2, fac), True
    return np.array(hs)


def test_one_ulp_in_the_factor_moves_later_steps_far_above_an_ulp():
    tb = O.erk_tableau(O.TSIT5)
    y0, p = W.lorenz(12, seed=0)
    root = lambda ms: 0.9 * np.sqrt(ms) ** -0.2
    sq = lambda ms: 0.9 * ms ** -0.1
    ulp = lambda ms: np.nextafter(0.9 * ms ** -0.1, np.inf)
    diffs = []
    for l in range(len(y0)):
        a, b, c = (_run(tb, y0[l], p[l], 1.0, g) for g in (root, sq, ulp))
        assert len(a) == len(b) == len(c)           # the step counts agree
        diffs += [np.max(np.abs(a / b - 1)), np.max(np.abs(b / c - 1))]
    diffs = np.array(diffs)
    # far above an ulp, yet far below anything that would change a count
    assert np.median(diffs) > 1e-12
    assert np.median(diffs) < 1e-8 and diffs.max() < 1e-6

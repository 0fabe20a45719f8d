"""Algorithmic floating-point work of the record and the reverse sweep.

Counting rules: fma = 2; add, sub, mul, div, min, max = 1; sqrt, tanh and the
controller's root (a power) = 1; abs, negation, selects and comparisons = 0.
Time bookkeeping (t + h, the end-of-span clip, the underflow test) is not
counted, nor is work a lane performs only because its wavefront is busy
(masked lanes).

Per-unit figures, per (method, system):
  trial      one trial step of the record: the stages, y_new, the error
             estimate and its RMS norm, the controller's proposed factor and
             the next step size as after a rejection.  Rejected trials count
             (they are needed to find the mesh).
  accept     what an accepted trial adds: the controller's acceptance bound,
             and the slope at the new state for a pair without
             first-same-as-last
  side_fwd   one save-time side step of nonzero size in the record (the
             stages that enter y_new, and y_new; the base slope is known)
  adj_step   one mesh step of the reverse sweep (recomputed stages, stage
             cotangents, vector-Jacobian products; for the Rosenbrock methods
             also the Jacobian, the LU, the transposed solves and the
             Jacobian-VJP terms)
  adj_side   one save-time side step of nonzero size in the reverse sweep:
             adj_step plus y_new from the recomputed stages, the loss
             cotangent and term, and the addition into the base cotangent
  adj_zero   one save time on a mesh point in the reverse sweep
  dense_fwd  one dense save of the record (dense output): the continuous
             extension from the step's end states and slopes
  dense_adj  one dense save of the sweep: the extension recomputed, the loss
             cotangent and term, its reverse (a VJP at each end state), and
             the two additions into the end states' cotangents

These are operation counts of the method's steps exactly as the plain CPU
reference performs them, counted there by an operation-counting scalar; a
CPU test keeps every entry equal to that count.  In the linear algebra of
the Rosenbrock methods (W = I/(gamma h) - J factored and solved) operations
on the structural zeros of the Jacobian are not counted: the count is that
of the sparse factorisation without interchanges.
"""

UNITS = ("trial", "accept", "side_fwd", "adj_step", "adj_side", "adj_zero", "dense_fwd",
         "dense_adj")

PER_UNIT = {
    ("tsit5", "lorenz"): (257, 1, 184, 417, 468, 12, 40, 113),
    ("vern7", "lorenz"): (431, 9, 313, 705, 762, 12, 40, 113),
    ("tsit5", "vdp"): (171, 1, 121, 274, 308, 8, 26, 74),
    ("vern7", "vdp"): (286, 6, 206, 464, 502, 8, 26, 74),
    ("tsit5", "linear"): (177, 1, 126, 286, 320, 8, 28, 78),
    ("vern7", "linear"): (295, 7, 214, 482, 520, 8, 28, 78),
    # Lotka-Volterra + 2-32-32-2 tanh MLP: the field costs 2,377 and its
    # vector-Jacobian product 7,257 (it recomputes the hidden layers)
    ("tsit5", "ude"): (14403, 1, 11981, 57970, 58004, 8, 4770, 19306),
    ("rodas4", "robertson"): (373, 1, 347, 954, 969, 12, 40, 121),
    ("rodas4", "hires"): (1135, 1, 1074, 2755, 2795, 32, 136, 386),
    ("rodas4", "linear"): (233, 1, 214, 539, 549, 8, 28, 78),
    ("ros23", "robertson"): (166, 1, 92, 236, 260, 12, 40, 121),
    ("ros23", "hires"): (505, 1, 290, 699, 763, 32, 136, 386),
    ("ros23", "linear"): (101, 1, 52, 123, 139, 8, 28, 78),
}

# (state dim, f, its VJP, the Jacobian, d/d(y, p) of u^T J v) per evaluation
SYSTEMS = {
    "lorenz": (3, 8, 20, 0, 0),
    "vdp": (2, 5, 13, 0, 0),
    "robertson": (3, 8, 24, 6, 25),
    "hires": (8, 36, 81, 3, 49),
    "linear": (2, 6, 14, 0, 8),
    "ude": (2, 2377, 7257, 0, 0),
}


def per_unit(method, system):
    return dict(zip(UNITS, PER_UNIT[(method, system)]))


def record_flops(method, system, trials, accepted, side_steps, dense=False):
    """side_steps: saves of nonzero offset from their base point (extra steps,
    or with dense output, interpolated saves)."""
    u = per_unit(method, system)
    per_save = u["dense_fwd"] if dense else u["side_fwd"]
    return u["trial"] * trials + u["accept"] * accepted + per_save * side_steps


def adjoint_flops(method, system, accepted, side_steps, zero_sides, dense=False):
    u = per_unit(method, system)
    per_save = u["dense_adj"] if dense else u["adj_side"]
    return u["adj_step"] * accepted + per_save * side_steps + u["adj_zero"] * zero_sides


# ------------------------------------------------------------ forward mode --
# Work of a replay step in dual numbers (value and one tangent): a sum 2, a
# product 4, an fma 6 (product rule); a combination with constant
# coefficients costs twice its primal work.
TABLEAUX = {
    "tsit5": dict(S=7, SU=6,
                  rows=[[], [0], [0, 1], [0, 1, 2], [0, 1, 2, 3], [0, 1, 2, 3, 4],
                        [0, 1, 2, 3, 4, 5]],
                  b=[0, 1, 2, 3, 4, 5]),
    "vern7": dict(S=10, SU=9,
                  rows=[[], [0], [0, 1], [0, 2], [0, 2, 3], [0, 2, 3, 4], [0, 2, 3, 4, 5],
                        [0, 2, 3, 4, 5, 6], [0, 2, 3, 4, 5, 6, 7], [0, 2, 3, 4, 5, 6]],
                  b=[0, 3, 4, 5, 6, 7, 8]),
}

# the right-hand side in dual numbers
RHS_DUAL = {"lorenz": 24, "vdp": 16, "linear": 20, "robertson": 26}

# Rosenbrock methods: nonzero counts of the rows of A (stage inputs) and C
# (stage right-hand sides); SU of the S stages enter y_new; new_at_input:
# y_new is the last stage's input (Rosenbrock23) rather than Y_s + u_s
ROS_TABLEAUX = {
    "rodas4": dict(S=6, SU=6, a_nnz=[0, 1, 2, 3, 4, 5], c_nnz=[0, 1, 2, 3, 4, 5],
                   new_at_input=False),
    "ros23": dict(S=3, SU=2, a_nnz=[0, 1, 2], c_nnz=[0, 1, 2], new_at_input=True),
}


def _combo(m):
    """sum of m weighted terms then fma(h, acc, y): 2m - 1 + 2."""
    return 2 * m + 1


# Jacobian entries in dual numbers (Rodas4 forward mode)
JAC_DUAL = {"robertson": 18, "linear": 0}


def _ros_jvp_per_step(method, system):
    """A Rodas4 step in dual numbers: the Jacobian, the LU and every solve
    with variable operands (a division or an fma 6, a product 4, a sum 2),
    the stage combinations with constant coefficients twice."""
    t = ROS_TABLEAUX[method]
    D = SYSTEMS[system][0]
    S, SU = t["S"], t["SU"]
    lu = 6 * D + sum(4 * m + 6 * m * m for m in range(1, D))   # reciprocals, then products
    factor = JAC_DUAL[system] + 2 + 2 * D + lu
    solve = 6 * D * D - 2 * D
    stage_in = sum(2 * z for z in t["a_nnz"][:SU]) * D
    stage_rhs = sum(2 * w + 1 for w in t["c_nnz"][:SU] if w) * D
    update = 2 * (2 * t["a_nnz"][S - 1] * D if t["new_at_input"] else D)
    return (factor + 1 + SU * solve + 2 * stage_in + SU * RHS_DUAL[system] + 2 * stage_rhs
            + update)


def jvp_per_step(method, system):
    """One replay step of the forward mode (explicit pairs): the stages'
    right-hand sides in dual numbers, and the stage and update combinations
    twice (the tangent of a combination with constant coefficients is the
    same combination of tangents)."""
    if method in ROS_TABLEAUX:
        return _ros_jvp_per_step(method, system)
    t = TABLEAUX[method]
    D = SYSTEMS[system][0]
    SU, rows = t["SU"], t["rows"]
    combos = (sum(_combo(len(rows[i])) for i in range(1, SU)) + _combo(len(t["b"]))) * D
    return SU * RHS_DUAL[system] + 2 * combos


def jvp_flops(method, system, accepted, side_steps, n_saves):
    """A forward-mode pass: every mesh step and every nonzero save step, plus
    the loss tangent (one fma per save component)."""
    D = SYSTEMS[system][0]
    return jvp_per_step(method, system) * (accepted + side_steps) + 2 * D * n_saves

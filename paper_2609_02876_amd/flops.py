"""Algorithmic floating-point work of the record and the reverse sweep
(explicit Runge-Kutta pairs and the Rodas4 Rosenbrock method).

Counting rules: fma = 2; add, sub, mul, div, min, max = 1; sqrt and the
controller's root = 1; abs, negation, selects and comparisons = 0.  Work the
method needs is counted once (a first-same-as-last stage is not recounted;
for a pair without that property the slope at the new state is counted once
per accepted step); work a lane performs only because its wavefront is busy
(masked lanes, rejected trials' unused side results) is not counted.

Per-unit figures:
  trial      one trial step of the record (stages, update, error estimate,
             RMS norm, controller) -- rejected trials count (they are needed
             to find the mesh)
  accept     extra work per accepted step (the new first stage for pairs
             without first-same-as-last)
  side_fwd   one save-time step of nonzero size in the record
  adj_step   one mesh step of the reverse sweep (recomputed stages, stage
             cotangents, VJPs, adjoint update)
  adj_side   one save-time step of nonzero size in the reverse sweep (adds
             the forward update of the save state and the loss cotangent)
  adj_zero   one save time on a mesh point in the reverse sweep
"""

# nonzero pattern (0-based column indices) of each stage row, b and the
# error weights; these mirror the tableaux of the kernels.
TABLEAUX = {
    "tsit5": dict(S=7, SU=6, fsal=True,
                  rows=[[], [0], [0, 1], [0, 1, 2], [0, 1, 2, 3], [0, 1, 2, 3, 4],
                        [0, 1, 2, 3, 4, 5]],
                  b=[0, 1, 2, 3, 4, 5], ew=[0, 1, 2, 3, 4, 5, 6]),
    "vern7": dict(S=10, SU=9, fsal=False,
                  rows=[[], [0], [0, 1], [0, 2], [0, 2, 3], [0, 2, 3, 4], [0, 2, 3, 4, 5],
                        [0, 2, 3, 4, 5, 6], [0, 2, 3, 4, 5, 6, 7], [0, 2, 3, 4, 5, 6]],
                  b=[0, 3, 4, 5, 6, 7, 8], ew=[0, 3, 4, 5, 6, 7, 8, 9]),
}

# (state dim, rhs flops, vjp flops)
SYSTEMS = {
    "lorenz": (3, 8, 20),
    "vdp": (2, 5, 13),
    "robertson": (3, 8, 20),
    "hires": (8, 36, 77),
    "linear": (2, 6, 14),
    # Lotka-Volterra + 2-32-32-2 tanh MLP (tanh = 1): the field is layers
    # 128 + 2048 + 128, two tanh layers 64, bias/LV 14; the VJP recomputes the
    # hidden layers (2240) and adds dW3/db3 130, delta2 and db2 224, W2^T
    # delta2 2048, delta1/db1/dW1 256, W1^T delta1 + LV 136 and dW2 2048
    "ude": (2, 2382, 7082),
}

# forward mode: flops of the right-hand side in dual numbers (a sum 2, a
# product 4, an fma 6: value plus tangent by the product rule)
RHS_DUAL = {"lorenz": 24, "vdp": 16, "linear": 20, "robertson": 26}

# (jacobian flops, flops of d/d(y, p) of u^T J v) for the stiff path
JACOBIANS = {
    "robertson": (5, 24),
    "hires": (3, 49),
    "linear": (0, 8),
}

# Rosenbrock methods: nonzero counts of the rows of A (stage inputs) and C
# (stage right-hand sides); SU of the S stages enter y_new; e_nnz: nonzero
# error weights; new_at_input: y_new is the last stage's input (Rosenbrock23)
# rather than Y_s + u_s (Rodas4)
ROS_TABLEAUX = {
    "rodas4": dict(S=6, SU=6, a_nnz=[0, 1, 2, 3, 4, 5], c_nnz=[0, 1, 2, 3, 4, 5], e_nnz=1,
                   new_at_input=False),
    "ros23": dict(S=3, SU=2, a_nnz=[0, 1, 2], c_nnz=[0, 1, 2], e_nnz=3, new_at_input=True),
}


def _lu(D):
    """LU with partial pivoting of a D x D matrix: a reciprocal per pivot;
    for column k, D-k-1 multipliers (a product with it) and (D-k-1)^2 fma
    updates."""
    return D + sum(m * (1 + 2 * m) for m in range(1, D))


def _ros_per_unit(method, system):
    t = ROS_TABLEAUX[method]
    D, F, V = SYSTEMS[system]
    J, JV = JACOBIANS[system]
    S, SU = t["S"], t["SU"]
    a_nnz, c_nnz = t["a_nnz"], t["c_nnz"]
    solve = 2 * D * D - D                       # L and U sweeps, D products by 1/U_kk
    factor = J + 2 + D + _lu(D)                 # jac, 1/(gamma h), diagonal, LU

    def stage_in(k):                            # inputs of the first k stages
        return sum(2 * z for z in a_nnz[:k]) * D

    def stages(k):                              # 1: 1/h
        return 1 + stage_in(k) + k * F + sum(2 * w + 1 for w in c_nnz[:k] if w) * D + k * solve

    # y_new: Y_s + u_s, or the last stage's input (counted with the stages
    # of a trial, formed on its own after the SU stages of a replay)
    upd_trial = 0 if t["new_at_input"] else D
    upd_replay = 2 * a_nnz[S - 1] * D if t["new_at_input"] else D
    e_combo = (2 * t["e_nnz"] - 1) * D if t["e_nnz"] > 1 else 0
    err = e_combo + 3 * D + (3 * D + 1)
    controller = 7
    trial = factor + stages(S) + upd_trial + err + controller
    side_fwd = factor + stages(SU) + upd_replay
    push = sum(2 * (z + w) for z, w in zip(a_nnz[:SU], c_nnz[:SU])) * D
    reverse = (SU * D + SU * solve + SU * D + stage_in(SU) + SU * V + SU * D + SU * JV + push
               + D)
    update = upd_replay
    adj_step = factor + stages(SU) + reverse
    cot = 3 * D
    adj_side = adj_step + update + cot + D
    adj_zero = cot + D
    return dict(trial=trial, accept=0, side_fwd=side_fwd, adj_step=adj_step,
                adj_side=adj_side, adj_zero=adj_zero)


def _combo(m):
    """sum of m weighted terms then fma(h, acc, y): 2m - 1 + 2."""
    return 2 * m + 1


def per_unit(method, system):
    if method in ROS_TABLEAUX:
        return _ros_per_unit(method, system)
    t = TABLEAUX[method]
    D, F, V = SYSTEMS[system]
    S, SU = t["S"], t["SU"]
    rows = t["rows"]
    stages_all = sum(_combo(len(rows[i])) for i in range(1, S)) * D
    stages_su = sum(_combo(len(rows[i])) for i in range(1, SU)) * D
    update = _combo(len(t["b"])) * D
    err = 2 * len(t["ew"]) * D + 3 * D + (3 * D + 1)
    controller = 7
    trial = stages_all + (S - 1) * F + (0 if t["fsal"] else update) + err + controller
    accept = 0 if t["fsal"] else F
    side_fwd = stages_su + (SU - 1) * F + update
    # reverse: each stage j, terms = [b_j != 0] + #{l in (j, SU): a_lj != 0}
    rev = 0
    for j in range(SU):
        terms = (1 if j in t["b"] else 0) + sum(1 for l in range(j + 1, SU) if j in rows[l])
        rev += (2 * terms if terms else 1) * D
    adj_step = F + stages_su + (SU - 1) * F + rev + SU * V + SU * D
    cot = 3 * D  # sum of squares: w = 2 s v (mul), loss += v v (fma)
    adj_side = adj_step + update + cot + D
    adj_zero = cot + D
    return dict(trial=trial, accept=accept, side_fwd=side_fwd, adj_step=adj_step,
                adj_side=adj_side, adj_zero=adj_zero)


def record_flops(method, system, trials, accepted, side_steps):
    u = per_unit(method, system)
    return u["trial"] * trials + u["accept"] * accepted + u["side_fwd"] * side_steps


def adjoint_flops(method, system, accepted, side_steps, zero_sides):
    u = per_unit(method, system)
    return u["adj_step"] * accepted + u["adj_side"] * side_steps + u["adj_zero"] * zero_sides


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

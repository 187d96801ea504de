"""FP64 oracle for trajectory optimisation (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the product library never loads it.

The variables are a trajectory Q = [q_0 .. q_{T-1}] (time-major, one
configuration per timestep, Sec. II: each configuration interacts with its
temporal neighbours).  Residuals (Sec. III-C costs, each weighted):

* start and goal pose: the joint pose cost at q_0 and q_{T-1};
* joint limits at every timestep;
* smoothness: q_t - q_{t-1};
* velocity limit: max(0, |q_t - q_{t-1}| - v_max dt);
* acceleration and jerk: the five-point stencils centred at t = 2 .. T-3,
  (-q_{t-2} + 16 q_{t-1} - 30 q_t + 16 q_{t+1} - q_{t+2}) / (12 dt^2) and
  (-q_{t-2} + 2 q_{t-1} - 2 q_{t+1} + q_{t+2}) / (2 dt^3).

The solver is the IK oracle's Levenberg-Marquardt controller (Sec. III-A)
over all T*n variables with a dense Jacobian and an exact FP64 solve.  Row
order: start pose (6), goal pose (6), limits [T][n], smoothness [T-1][n],
velocity [T-1][n], acceleration [T-4][n], jerk [T-4][n].
"""
from __future__ import annotations

import numpy as np

import oracle

# Five-point stencils on offsets -2..2 (times dt^2, resp. dt^3).
ACC = np.array([-1.0, 16.0, -30.0, 16.0, -1.0]) / 12.0
JERK = np.array([-1.0, 2.0, 0.0, -2.0, 1.0]) / 2.0


def _pose_w(c):
    return {"w_pos": c["w_pos"], "w_rot": c["w_rot"], "w_limit": 0.0, "w_rest": 0.0}


def _limits(tree):
    vj = tree.var_joints
    return np.asarray(tree.lower, np.float64)[vj], np.asarray(tree.upper, np.float64)[vj]


def residual(tree, start, goal, c, Q):
    """Residual vector of trajectory Q [T, n]; start / goal targets [1, 7]."""
    Q = np.asarray(Q, np.float64)
    T = Q.shape[0]
    lo, hi = _limits(tree)
    dt = c["dt"]
    r0 = oracle.residual(tree, start, _pose_w(c), Q[0])[0][:6]
    r1 = oracle.residual(tree, goal, _pose_w(c), Q[-1])[0][:6]
    lim = c["w_limit"] * (np.maximum(0.0, Q - hi) + np.maximum(0.0, lo - Q))
    dQ = Q[1:] - Q[:-1]
    smooth = c["w_smooth"] * dQ
    vel = c["w_vel"] * np.maximum(0.0, np.abs(dQ) - np.asarray(c["vmax"]) * dt)
    acc = sum(ACC[k] * Q[k:T - 4 + k] for k in range(5)) * (c["w_acc"] / dt ** 2)
    jerk = sum(JERK[k] * Q[k:T - 4 + k] for k in range(5)) * (c["w_jerk"] / dt ** 3)
    return np.concatenate([r0, r1, lim.ravel(), smooth.ravel(), vel.ravel(), acc.ravel(),
                           jerk.ravel()])


def jacobian(tree, start, goal, c, Q):
    """Dense Jacobian [rows, T*n], variable t*n + i."""
    Q = np.asarray(Q, np.float64)
    T, n = Q.shape
    lo, hi = _limits(tree)
    dt = c["dt"]
    rows = 12 + T * n + 2 * (T - 1) * n + 2 * (T - 4) * n
    J = np.zeros((rows, T * n))
    J[0:6, 0:n] = oracle.jacobian(tree, start, _pose_w(c), Q[0])[:6]
    J[6:12, (T - 1) * n:T * n] = oracle.jacobian(tree, goal, _pose_w(c), Q[-1])[:6]
    row = 12
    for t in range(T):
        for i in range(n):
            q = Q[t, i]
            J[row, t * n + i] = c["w_limit"] if q > hi[i] else (-c["w_limit"] if q < lo[i] else 0.0)
            row += 1
    for t in range(1, T):
        for i in range(n):
            J[row, t * n + i] = c["w_smooth"]
            J[row, (t - 1) * n + i] = -c["w_smooth"]
            row += 1
    vmax = np.asarray(c["vmax"])
    for t in range(1, T):
        for i in range(n):
            d = Q[t, i] - Q[t - 1, i]
            if abs(d) - vmax[i] * dt > 0.0:
                s = c["w_vel"] * np.sign(d)
                J[row, t * n + i] = s
                J[row, (t - 1) * n + i] = -s
            row += 1
    for coef, scale in [(ACC, c["w_acc"] / dt ** 2), (JERK, c["w_jerk"] / dt ** 3)]:
        for t in range(2, T - 2):
            for i in range(n):
                for k in range(5):
                    J[row, (t - 2 + k) * n + i] = coef[k] * scale
                row += 1
    return J


def cost(tree, start, goal, c, Q):
    r = residual(tree, start, goal, c, Q)
    return float(r @ r)


def endpoint_errors(tree, start, goal, Q):
    """(pos, rot) errors of the start and goal poses, [2] each."""
    w = {"w_pos": 1.0, "w_rot": 1.0, "w_limit": 0.0, "w_rest": 0.0}
    _, p0, r0 = oracle.residual(tree, start, w, Q[0])
    _, p1, r1 = oracle.residual(tree, goal, w, Q[-1])
    return np.array([p0[0], p1[0]]), np.array([r0[0], r1[0]])


def lm_solve(tree, start, goal, c, o, Q0):
    """Levenberg-Marquardt on one trajectory, the IK controller's rules:
    damping lambda * diag(max(A_jj, floor)); accept iff the cost strictly
    decreases, lambda /= nu_down (>= lambda_min), else lambda *= nu_up
    (<= lambda_max; a reject at lambda_max stalls); every trial is one
    iteration; with early_exit the run stops once both endpoint poses are
    within tolerance.  Returns the trajectory, cost, counters and status
    (CONVERGED when both endpoint poses meet the tolerance at the end), the
    accept sequence and, per iteration, whether its decision was a near-tie
    (|c' - c| <= 1e-5 c, as the IK oracle flags them)."""
    Q = np.array(Q0, np.float64)
    T, n = Q.shape
    cst = cost(tree, start, goal, c, Q)
    lam = o["lambda0"]
    iters = accepts = 0
    stalled = False

    def meets(Qx):
        pe, re = endpoint_errors(tree, start, goal, Qx)
        return bool(np.all(pe <= o["tol_pos"]) and np.all(re <= o["tol_rot"]))

    done = o["early_exit"] and meets(Q)
    trace, ties = [], []
    while not done and iters < o["max_iters"]:
        r = residual(tree, start, goal, c, Q)
        J = jacobian(tree, start, goal, c, Q)
        A = J.T @ J
        g = J.T @ r
        D = np.maximum(np.diag(A), o["damping_floor"])
        d = np.linalg.solve(A + lam * np.diag(D), -g)
        Qt = Q + d.reshape(T, n)
        ct = cost(tree, start, goal, c, Qt)
        iters += 1
        ties.append(int(np.isfinite(ct) and abs(ct - cst) <= 1e-5 * cst))
        if ct < cst:
            Q, cst = Qt, ct
            lam = max(lam / o["nu_down"], o["lambda_min"])
            accepts += 1
            trace.append(1)
            if o["early_exit"] and meets(Q):
                done = True
        else:
            trace.append(0)
            if lam >= o["lambda_max"]:
                stalled = True
                done = True
            lam = min(lam * o["nu_up"], o["lambda_max"])
    ok = meets(Q)
    pe, re = endpoint_errors(tree, start, goal, Q)
    status = oracle.CONVERGED if ok else (oracle.STALLED if stalled else oracle.MAX_ITERS)
    return {"Q": Q, "cost": cst, "iters": iters, "accepts": accepts, "status": status,
            "pos_err": pe, "rot_err": re, "trace_acc": np.array(trace, np.int32),
            "trace_tie": np.array(ties, np.int32)}

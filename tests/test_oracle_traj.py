"""Pins of the trajectory-optimisation oracle (Sec. III-C smoothness, velocity
limit and five-point acceleration/jerk costs; LM as for IK).

The stencils are checked on polynomials (the five-point second- and
third-derivative formulas are exact up to degree 5 and 4), the residual's
pieces against their definitions at hand-made trajectories, the Jacobian
against central differences, and the solver against a closed form: with
smoothness as the only trajectory cost, the interior of the optimum is the
straight line between its endpoints.
"""
import numpy as np

import oracle
import synth
from oracle import traj

ARM = synth.arm7(0)


def _costs(**kw):
    c = {"T": 12, "dt": 0.1, "w_pos": 1.0, "w_rot": 0.5, "w_limit": 0.0, "w_smooth": 0.0,
         "w_vel": 0.0, "vmax": [1.0] * 7, "w_acc": 0.0, "w_jerk": 0.0}
    c.update(kw)
    return c


def _targets(qa, qb):
    return oracle.targets_from(ARM, np.stack([qa, qb]), round_f32=False)


def _parts(c, T, n=7):
    sizes = [6, 6, T * n, (T - 1) * n, (T - 1) * n, (T - 4) * n, (T - 4) * n]
    return np.cumsum([0] + sizes)


def test_stencils_are_exact_on_polynomials():
    T, dt = 12, 0.1
    t = np.arange(T) * dt
    rng = np.random.default_rng(1)
    co = rng.normal(size=(5, 7))                     # degree-4 polynomial per joint
    Q = sum(co[k][None, :] * t[:, None] ** k for k in range(5))
    d2 = sum(k * (k - 1) * co[k][None, :] * t[:, None] ** (k - 2) for k in range(2, 5))
    d3 = sum(k * (k - 1) * (k - 2) * co[k][None, :] * t[:, None] ** (k - 3) for k in range(3, 5))
    qa, qb = Q[0], Q[-1]
    st, gl = _targets(qa, qb)
    cut = _parts(None, T)
    r = traj.residual(ARM, st, gl, _costs(T=T, dt=dt, w_acc=1.0, w_jerk=1.0), Q)
    np.testing.assert_allclose(r[cut[5]:cut[6]].reshape(T - 4, 7), d2[2:T - 2], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(r[cut[6]:cut[7]].reshape(T - 4, 7), d3[2:T - 2], rtol=1e-9, atol=1e-8)


def test_linear_trajectory_pieces():
    T = 10
    qa, qb = synth.uniform_configs(ARM, 2, 3)
    s = np.linspace(0, 1, T)[:, None]
    Q = (1 - s) * qa + s * qb
    st, gl = _targets(qa, qb)
    c = _costs(T=T, w_smooth=0.3, w_vel=2.0, vmax=[0.5] * 7, w_acc=1.0, w_jerk=1.0, w_limit=10.0)
    r = traj.residual(ARM, st, gl, c, Q)
    cut = _parts(c, T)
    np.testing.assert_allclose(r[:12], 0.0, atol=1e-12)          # endpoints on their poses
    np.testing.assert_allclose(r[cut[2]:cut[3]], 0.0)               # within limits
    step = (qb - qa) / (T - 1)
    np.testing.assert_allclose(r[cut[3]:cut[4]].reshape(T - 1, 7), 0.3 * np.tile(step, (T - 1, 1)),
                               rtol=1e-12)
    vel = 2.0 * np.maximum(0.0, np.abs(step) - 0.5 * 0.1)
    np.testing.assert_allclose(r[cut[4]:cut[5]].reshape(T - 1, 7), np.tile(vel, (T - 1, 1)),
                               rtol=1e-12)
    np.testing.assert_allclose(r[cut[5]:], 0.0, atol=1e-9)          # no acceleration, no jerk


def test_limit_rows_per_timestep():
    T = 6
    Q = np.zeros((T, 7))
    Q[2, 3] = ARM.upper[3] + 0.25
    Q[4, 0] = ARM.lower[0] - 0.5
    st, gl = _targets(Q[0], Q[-1])
    r = traj.residual(ARM, st, gl, _costs(T=T, w_limit=10.0), Q)
    lim = r[12:12 + T * 7].reshape(T, 7)
    want = np.zeros((T, 7))
    want[2, 3] = 2.5
    want[4, 0] = 5.0
    np.testing.assert_allclose(lim, want, rtol=1e-6)


def test_jacobian_matches_finite_differences():
    T = 8
    wl = synth.workload("traj", targets=3)
    for b in range(3):
        Q = wl["init"][b][np.linspace(0, 31, T).astype(int)]
        st, gl = _targets(wl["start_q"][b], wl["goal_q"][b])
        c = dict(wl["costs"], T=T)
        J = traj.jacobian(ARM, st, gl, c, Q)
        h = 1e-6
        Jf = np.zeros_like(J)
        for v in range(T * 7):
            e = np.zeros(T * 7)
            e[v] = h
            Jf[:, v] = (traj.residual(ARM, st, gl, c, Q + e.reshape(T, 7)) -
                        traj.residual(ARM, st, gl, c, Q - e.reshape(T, 7))) / (2 * h)
        rel = np.linalg.norm(J - Jf) / np.linalg.norm(Jf)
        assert rel < 1e-6, rel


def test_smoothness_only_optimum_is_a_straight_line():
    """With smoothness the only trajectory cost, the optimum's interior is the
    linear interpolation of its endpoints (sum of squared steps with fixed
    ends is minimised by equal steps).  The endpoints keep creeping along the
    arm's self-motion (shortening the path) long after the interior has
    settled, so the check holds to 1e-4 after 60 iterations (5e-6 after
    200)."""
    T = 12
    qa, qb = synth.uniform_configs(ARM, 2, 8)
    st, gl = _targets(qa, qb)
    rng = np.random.default_rng(9)
    s = np.linspace(0, 1, T)[:, None]
    Q0 = (1 - s) * qa + s * qb + 0.2 * np.sin(np.pi * s) * rng.normal(size=7)
    c = _costs(T=T, w_smooth=0.05, w_pos=10.0, w_rot=5.0)
    o = {"max_iters": 60, "lambda0": 1e-3, "nu_up": 10.0, "nu_down": 10.0, "lambda_min": 1e-10,
         "lambda_max": 1e10, "early_exit": False, "tol_pos": 1e-3, "tol_rot": 1e-2,
         "damping_floor": 1e-6, "pivot_rel": 1e-6}
    res = traj.lm_solve(ARM, st, gl, c, o, Q0)
    Q = res["Q"]
    line = (1 - s) * Q[0] + s * Q[-1]
    np.testing.assert_allclose(Q, line, atol=1e-4)
    assert res["cost"] < traj.cost(ARM, st, gl, c, Q0)
    # one accept flag and one near-tie flag per iteration (this run's
    # decisions all move the cost by more than 1e-5 of itself)
    assert len(res["trace_acc"]) == len(res["trace_tie"]) == res["iters"] == 60
    assert set(np.unique(res["trace_acc"])) <= {0, 1} and not res["trace_tie"].any()
    assert res["accepts"] == res["trace_acc"].sum()

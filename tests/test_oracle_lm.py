"""Pins for the oracle's damped normal equations, Cholesky and LM controller.

Sec. III-A: Levenberg-Marquardt over the weighted sum of squared residuals,
limits as penalties.  Pinned by: numpy's LAPACK Cholesky/solve; closed-form
LM iterates for problems whose residual is linear (rest-only, limit-only);
exactly determined IK with a known unique answer (1-DoF, planar 2-link full
pose) and with two closed-form branches (planar 2-link position-only); a
brute-force grid on a 2-DoF problem; and invariants (accepted cost strictly
decreasing, counters, status codes, best-of-K rule).
"""
import math

import numpy as np
import pytest

import synth

rng = np.random.default_rng(7)


def opts(**kw):
    o = {"max_iters": 50, "lambda0": 1e-3, "nu_up": 10.0, "nu_down": 10.0,
         "lambda_min": 1e-10, "lambda_max": 1e10, "early_exit": False, "tol_pos": 1e-3,
         "tol_rot": 1e-2, "damping_floor": 1e-6, "pivot_rel": 1e-6}
    o.update(kw)
    return o


def weights(**kw):
    w = {"w_pos": 1.0, "w_rot": 0.5, "w_limit": 10.0, "w_rest": 0.0, "q_rest": None}
    w.update(kw)
    return w


@pytest.mark.parametrize("n", [1, 2, 7, 16, 34, 64])
def test_cholesky_matches_lapack(ora, n):
    M = rng.normal(size=(n, n))
    A = M @ M.T + n * np.eye(n)
    L, ok, ratio = ora.cholesky(A)
    assert ok and ratio > 0
    np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=1e-12, atol=1e-12)
    b = rng.normal(size=n)
    np.testing.assert_allclose(ora.chol_solve(L, b), np.linalg.solve(A, b), rtol=1e-10)


def test_cholesky_rejects_indefinite(ora):
    A = np.diag([1.0, -1e-3, 2.0])
    _, ok, ratio = ora.cholesky(A)
    assert not ok and ratio < 0


def test_step_solves_damped_normal_equations(ora):
    tree = synth.arm7(0)
    w = weights(w_rest=0.01)
    q = synth.uniform_configs(tree, 1, 1)[0]
    tg = ora.targets_from(tree, synth.uniform_configs(tree, 1, 2))[0]
    r, _, _ = ora.residual(tree, tg, w, q)
    J = ora.jacobian(tree, tg, w, q)
    for lam in [1e-3, 1.0, 1e3]:
        A = J.T @ J
        D = np.diag(np.maximum(np.diag(A), 1e-6))
        want = np.linalg.solve(A + lam * D, -J.T @ r)
        d, ok, _ = ora.lm_step(tree, tg, w, opts(), q, lam)
        assert ok
        np.testing.assert_allclose(d, want, rtol=1e-9, atol=1e-12)


def _rest_only_problem():
    tree = synth.chain("zyz", seed=3)
    # Pose rows carry zero weight, limits are far away: r = w (q - q_rest).
    w = weights(w_pos=0.0, w_rot=0.0, w_limit=0.0, w_rest=0.5,
                q_rest=np.array([0.1, -0.2, 0.3]))
    tg = np.zeros((1, 7))
    tg[0, 3] = 1.0
    return tree, w, tg


def test_rest_only_iterates_closed_form(ora):
    # J = w I, A = w^2 I, D = w^2 I: q_{t+1} - q_rest = lam_t/(1+lam_t) (q_t - q_rest),
    # every step accepted, lam_{t+1} = lam_t / 10.
    tree, w, tg = _rest_only_problem()
    q0 = np.array([1.0, 0.5, -0.7])
    res = ora.lm_solve(tree, tg, w, opts(max_iters=5, lambda0=1.0), q0, n_trace=5)
    qr, lam, q = w["q_rest"], 1.0, q0.copy()
    for t in range(5):
        q = qr + lam / (1 + lam) * (q - qr)
        lam /= 10
        np.testing.assert_allclose(res["trace_q"][t], q, rtol=0, atol=1e-14)
        assert res["trace_acc"][t] == 1
    assert res["accepts"] == 5 and res["iters"] == 5


def test_limit_only_iterates_closed_form(ora):
    # From above the upper limit u: r = w (q - u), J = w.  Same geometric
    # approach to u, from outside.
    tree = synth.one_joint(lim=1.0)
    w = weights(w_pos=0.0, w_rot=0.0, w_limit=3.0)
    tg = np.zeros((1, 7))
    tg[0, 3] = 1.0
    u = tree.upper[0]
    res = ora.lm_solve(tree, tg, w, opts(max_iters=5, lambda0=0.5), np.array([2.0]), n_trace=5)
    lam, q = 0.5, 2.0
    for t in range(5):
        q = u + lam / (1 + lam) * (q - u)
        lam /= 10
        assert res["trace_q"][t][0] == pytest.approx(q, abs=1e-14)
        assert res["trace_q"][t][0] > u


def test_one_dof_converges_to_unique_answer(ora):
    tree = synth.one_joint(kind=synth.EE_POSITION)
    for qs in [-2.5, 0.4, 2.9]:
        tg = ora.targets_from(tree, np.array([[qs]]))[0]
        seed = np.array([qs + rng.uniform(-1.2, 1.2)])
        res = ora.lm_solve(tree, tg, weights(w_limit=0.0), opts(), seed)
        # the FP32-rounded target pins q* to ~1e-7 rad
        assert res["q"][0] == pytest.approx(qs, abs=1e-6)
        assert res["status"] & 0xff == ora.CONVERGED


def test_planar_full_pose_converges_to_unique_answer(ora):
    tree = synth.planar2(0.6, 0.4)
    for qs in synth.uniform_configs(tree, 5, 21) * 0.9:
        tg = ora.targets_from(tree, qs[None], round_f32=False)[0]
        seed = qs + rng.uniform(-0.5, 0.5, size=2)
        res = ora.lm_solve(tree, tg, weights(w_limit=0.0), opts(), seed)
        np.testing.assert_allclose(res["q"], qs, atol=1e-8)


def test_planar_position_only_reaches_a_closed_form_branch(ora):
    l1, l2 = 0.6, 0.4
    tree = synth.planar2(l1, l2, kind=synth.EE_POSITION)
    for qs in synth.uniform_configs(tree, 6, 22) * 0.9:
        tg = ora.targets_from(tree, qs[None], round_f32=False)[0]
        x, y = tg[0, 0], tg[0, 1]
        c2 = (x * x + y * y - l1 * l1 - l2 * l2) / (2 * l1 * l2)
        branches = []
        for s in (+1, -1):
            q2 = s * math.acos(max(-1.0, min(1.0, c2)))
            q1 = math.atan2(y, x) - math.atan2(l2 * math.sin(q2), l1 + l2 * math.cos(q2))
            branches.append(np.array([q1, q2]))
        res = ora.lm_solve(tree, tg, weights(w_limit=0.0), opts(), qs + rng.uniform(-0.4, 0.4, 2))
        wrap = lambda a: (a + math.pi) % (2 * math.pi) - math.pi
        d = min(np.max(np.abs(wrap(res["q"] - b))) for b in branches)
        # near the workspace boundary the joint error is ~sqrt(position error)
        assert res["pos_err"][0] < 1e-12
        assert d < 1e-6


def test_best_of_eight_reaches_brute_force_grid_minimum(ora):
    # Target out of reach: the minimum cost is positive and found by a grid.
    tree = synth.planar2(0.6, 0.4, lim=2.5)
    tg = np.array([[1.3, 0.4, 0.05, math.cos(0.6), 0.0, 0.0, math.sin(0.6)]])
    w = weights(w_limit=1.0)
    g = np.linspace(-3.0, 3.0, 241)
    best = min(ora.cost(tree, tg, w, np.array([a, b])) for a in g for b in g)
    seeds = synth.uniform_configs(tree, 8, 23)
    out = ora.lm_solve_batch(tree, tg, seeds, 8, w, opts(max_iters=100), threads=2)
    # grid spacing 0.025 rad: the grid's best is within O(h^2) of the optimum
    assert out["cost"].min() <= best + 1e-12
    assert out["cost"].min() >= best - 5e-3


@pytest.mark.parametrize("tree", [synth.arm7(0), synth.tree34(5), synth.hand16(8)],
                         ids=lambda t: t.name)
def test_accepted_costs_strictly_decrease(ora, tree):
    tg = ora.targets_from(tree, synth.uniform_configs(tree, 6, 31))
    seeds = synth.uniform_configs(tree, 6, 32)
    w = weights(w_rest=0.01)
    for t, s in zip(tg, seeds):
        c0 = ora.cost(tree, t, w, s)
        res = ora.lm_solve(tree, t, w, opts(max_iters=30), s, n_trace=30)
        prev = c0
        for acc, c in zip(res["trace_acc"], res["trace_cost"]):
            assert c >= 0
            if acc:
                assert c < prev
            else:
                assert c == prev
            prev = c
        assert res["accepts"] == res["trace_acc"].sum()
        assert res["cost"] == pytest.approx(ora.cost(tree, t, w, res["q"]), rel=1e-15)


def test_early_exit_and_iters_to_tol(ora):
    tree = synth.arm7(0)
    tg = ora.targets_from(tree, synth.uniform_configs(tree, 40, 41))
    seeds = synth.uniform_configs(tree, 40, 42)
    w = weights(w_rest=0.01)
    full = ora.lm_solve_batch(tree, tg, seeds, 1, w, opts(max_iters=30))
    ee = ora.lm_solve_batch(tree, tg, seeds, 1, w, opts(max_iters=30, early_exit=True))
    conv = full["iters_to_tol"] >= 0
    assert conv.any()
    np.testing.assert_array_equal(ee["iters_to_tol"], full["iters_to_tol"])
    np.testing.assert_array_equal(ee["iters"][conv], full["iters_to_tol"][conv])
    assert np.all(ee["status"][conv] & 0xff == ora.CONVERGED)


def test_seed_already_at_target_exits_at_zero(ora):
    tree = synth.arm7(0)
    q = synth.uniform_configs(tree, 1, 43)
    tg = ora.targets_from(tree, q)[0]
    res = ora.lm_solve(tree, tg, weights(), opts(early_exit=True), q[0])
    assert res["iters"] == 0 and res["iters_to_tol"] == 0 and res["status"] & 0xff == ora.CONVERGED


def test_status_codes(ora):
    tree = synth.arm7(0)
    q = synth.uniform_configs(tree, 2, 44)
    tg = ora.targets_from(tree, q[:1])[0]
    # max_iters = 0 leaves the seed unchanged.
    res = ora.lm_solve(tree, tg, weights(), opts(max_iters=0), q[1])
    np.testing.assert_array_equal(res["q"], q[1])
    assert res["iters"] == 0 and res["status"] & 0xff == ora.MAX_ITERS
    # Non-finite target.
    bad = tg.copy()
    bad[0, 1] = np.nan
    res = ora.lm_solve(tree, bad, weights(), opts(), q[1])
    assert res["status"] == ora.NONFINITE and np.array_equal(res["q"], q[1])
    # Unreachable target straight ahead of a stretched planar arm: the gradient
    # is exactly zero, every trial is rejected, lambda climbs to lambda_max.
    pl = synth.planar2(0.6, 0.4, kind=synth.EE_POSITION)
    far = np.array([[2.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0]])
    res = ora.lm_solve(pl, far, weights(w_limit=0.0), opts(lambda0=1e8), np.zeros(2))
    assert res["status"] & 0xff == ora.STALLED
    assert res["accepts"] == 0 and res["iters"] == 3


def test_fallback_flag_on_rank_deficient_system(ora):
    # 7 joints, 6 pose rows, no rest cost: J^T J is singular, so once lambda is
    # small the smallest pivot ratio drops below 1e-6.
    tree = synth.arm7(0)
    q = synth.uniform_configs(tree, 1, 45)
    tg = ora.targets_from(tree, q)[0]
    seed = q[0] + 0.05
    res = ora.lm_solve(tree, tg, weights(w_limit=0.0), opts(max_iters=12), seed)
    assert res["flags"] & ora.FLAG_FP64
    res = ora.lm_solve(tree, tg, weights(w_limit=0.0, w_rest=0.1), opts(max_iters=12), seed)
    assert not res["flags"] & ora.FLAG_FP64


def test_best_of_k_rule(ora):
    st = np.array([1, 0, 0, 1,   1, 1, 1, 1,   0, 0, 1, 1], np.int32)
    cost = np.array([0.1, 0.5, 0.2, 0.0,   3, 2, 2, 5,   0.3, 0.3, 0, 0])
    pose = np.array([0.0, 0.5, 0.2, 0.0,   3, 1, 1, 5,   0.3, 0.3, 0, 0])
    best, succ = ora.best_of_k(st, cost, pose, 4)
    np.testing.assert_array_equal(best, [2, 1, 0])
    np.testing.assert_array_equal(succ, [True, False, True])


def test_batch_matches_single_and_is_thread_invariant(ora):
    tree = synth.arm7(0)
    wl = synth.workload("arm131k", targets=12)
    g = wl["groups"][0]
    tg = ora.targets_from(tree, g["q_star"])
    a = ora.lm_solve_batch(tree, tg, g["seeds"], 8, wl["weights"], wl["options"], threads=1)
    b = ora.lm_solve_batch(tree, tg, g["seeds"], 8, wl["weights"], wl["options"], threads=5)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    for p in [0, 17, 95]:
        s = ora.lm_solve(tree, tg[p // 8], wl["weights"], wl["options"], g["seeds"][p])
        np.testing.assert_array_equal(s["q"], a["q"][p])
        assert s["iters"] == a["iters"][p]

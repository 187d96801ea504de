"""Pins of the oracle's IK-Beam (Sec. V-C): the survivor selection and the
two-stage schedule, checked against independent routines and special cases
that reduce to plain LM + best-of-K."""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _keys(st, c, pc):
    """Independent statement of the survivor order as a sort key (a seed within
    tolerance first; its total cost, or the pose-only cost of one that is not;
    NaN after every number; then the index)."""
    out = []
    for k in range(len(st)):
        conv = (st[k] & 0xFF) == oracle.CONVERGED
        v = c[k] if conv else pc[k]
        out.append((0 if conv else 1, 1 if np.isnan(v) else 0, 0.0 if np.isnan(v) else v, k))
    return out


def _random_case(rng, T, K, nan_frac=0.0, tie_frac=0.0):
    st = np.where(rng.random(T * K) < 0.3, oracle.CONVERGED,
                  rng.choice([oracle.MAX_ITERS, oracle.STALLED], T * K)).astype(np.int32)
    st |= np.where(rng.random(T * K) < 0.1, oracle.FLAG_FP64, 0).astype(np.int32)
    c = rng.random(T * K)
    pc = rng.random(T * K)
    if tie_frac:
        tie = rng.random(T * K) < tie_frac
        c[tie] = 0.5
        pc[tie] = 0.25
    if nan_frac:
        c[rng.random(T * K) < nan_frac] = np.nan
        pc[rng.random(T * K) < nan_frac] = np.nan
    return st, c, pc


@pytest.mark.parametrize("K,keep,nan_frac,tie_frac", [(8, 3, 0.0, 0.0), (64, 4, 0.0, 0.0),
                                                      (16, 16, 0.2, 0.3), (5, 1, 0.4, 0.5)])
def test_beam_select_is_the_head_of_the_sorted_order(K, keep, nan_frac, tie_frac):
    rng = np.random.default_rng(K * 100 + keep)
    T = 40
    st, c, pc = _random_case(rng, T, K, nan_frac, tie_frac)
    kept = oracle.beam_select(st, c, pc, K, keep)
    assert kept.shape == (T, keep)
    for t in range(T):
        sl = slice(t * K, (t + 1) * K)
        order = [key[3] for key in sorted(_keys(st[sl], c[sl], pc[sl]))]
        assert list(kept[t]) == order[:keep]


def test_beam_select_first_is_best_of_k_without_nan():
    rng = np.random.default_rng(3)
    for K in [1, 2, 7, 64]:
        st, c, pc = _random_case(rng, 50, K, tie_frac=0.2)
        kept = oracle.beam_select(st, c, pc, K, 1)
        best, _ = oracle.best_of_k(st, c, pc, K)
        np.testing.assert_array_equal(kept[:, 0], best)


def test_beam_select_brute_force_dominance_tiny():
    """Every kept seed precedes every dropped one, and the kept list is in
    order: checked pairwise over all seeds of all small cases."""
    vals = [0.0, 1.0, np.nan]
    for conv_bits in itertools.product([0, 1], repeat=3):
        for cv in itertools.product(vals, repeat=3):
            st = np.array([oracle.CONVERGED if b else oracle.MAX_ITERS for b in conv_bits], np.int32)
            c = np.array(cv)
            pc = np.array(cv[::-1])
            for keep in (1, 2, 3):
                kept = list(oracle.beam_select(st, c, pc, 3, keep)[0])
                keys = _keys(st, c, pc)
                assert len(set(kept)) == keep
                for a, b in zip(kept, kept[1:]):
                    assert keys[a] < keys[b]
                for d in set(range(3)) - set(kept):
                    assert all(keys[a] < keys[d] for a in kept)


def test_beam_select_permutation_equivariant():
    rng = np.random.default_rng(11)
    K, keep, T = 32, 4, 20
    st, c, pc = _random_case(rng, T, K)
    kept = oracle.beam_select(st, c, pc, K, keep)
    perm = rng.permutation(K)
    idx = (np.arange(T)[:, None] * K + perm[None, :]).ravel()
    kept_p = oracle.beam_select(st[idx], c[idx], pc[idx], K, keep)
    # distinct values, so the kept seeds are the same seeds, relabelled
    np.testing.assert_array_equal(perm[kept_p], kept)


def _arm_case(T):
    wl = synth.workload("beam", targets=T)
    g = wl["groups"][0]
    tree = g["tree"]
    return tree, oracle.targets_from(tree, g["q_star"]), g["seeds"], wl


def test_beam_without_stage1_iterations_is_best_of_k():
    """iters1 = 0: stage 1 only re-evaluates the survivors, so the result is
    the best-of-K choice of plain LM with iters0 iterations."""
    tree, tg, seeds, wl = _arm_case(12)
    r = oracle.ik_beam(tree, tg, seeds, 64, 6, 4, 0, wl["weights"], wl["options"])
    o = dict(wl["options"], max_iters=6)
    s = oracle.lm_solve_batch(tree, tg, seeds, 64, wl["weights"], o)
    best, succ = oracle.best_of_k(s["status"], s["cost"], s["pose_cost"], 64)
    np.testing.assert_array_equal(r["best_index"], best)
    np.testing.assert_array_equal(r["success"], succ)
    np.testing.assert_array_equal(r["best_q"], s["q"][np.arange(12) * 64 + best])
    np.testing.assert_array_equal(r["pick"], 0)


def test_beam_keeping_every_seed_from_the_start_is_plain_lm():
    """iters0 = 0 and keep = n_seeds: every seed goes through stage 1, so the
    result is best-of-K of plain LM with iters1 iterations."""
    tree, tg, seeds, wl = _arm_case(6)
    K = 16
    sd = seeds.reshape(6, 64, -1)[:, :K].reshape(6 * K, -1)
    r = oracle.ik_beam(tree, tg, sd, K, 0, K, 10, wl["weights"], wl["options"])
    o = dict(wl["options"], max_iters=10)
    s = oracle.lm_solve_batch(tree, tg, sd, K, wl["weights"], o)
    best, succ = oracle.best_of_k(s["status"], s["cost"], s["pose_cost"], K)
    np.testing.assert_array_equal(r["best_index"], best)
    np.testing.assert_array_equal(r["success"], succ)
    np.testing.assert_array_equal(r["best_q"], s["q"][np.arange(6) * K + best])


def test_beam_stages_chain_and_lambda_restarts():
    """Stage 1 starts from the survivors' stage-0 joints with lambda back at
    lambda0: each survivor's stage-1 result equals a fresh LM solve from
    those joints; the returned entries are the picked survivor's."""
    tree, tg, seeds, wl = _arm_case(4)
    r = oracle.ik_beam(tree, tg, seeds, 64, 6, 4, 10, wl["weights"], wl["options"])
    o = dict(wl["options"], max_iters=10)
    for t in range(4):
        for j in range(4):
            q0 = r["stage0"]["q"][t * 64 + r["kept"][t, j]]
            one = oracle.lm_solve(tree, tg[t], wl["weights"], o, q0)
            np.testing.assert_array_equal(one["q"], r["stage1"]["q"][t * 4 + j])
        p = t * 4 + r["pick"][t]
        np.testing.assert_array_equal(r["best_q"][t], r["stage1"]["q"][p])
        assert r["best_index"][t] == r["kept"][t, r["pick"][t]]
    # the schedule helps: the beam solves at least as many targets as stage 0
    st0 = (r["stage0"]["status"].reshape(4, 64) & 0xFF) == 0
    assert r["success"].sum() >= st0.any(1).sum()

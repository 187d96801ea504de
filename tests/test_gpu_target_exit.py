"""GPU checks of target_exit on the per-lane kernel: with it, a problem also
ends (status TARGET_SOLVED) in the pass in which another problem of its
target, in the same run of consecutive lanes of its wavefront, meets the
tolerance.  Against the same batch solved without it: every target's success
and first iteration at the tolerance are unchanged; a problem it does not end
gives bit-identical results; a problem it ends stops in the pass of its run's
first convergence, with no more iterations than before; the best-of-K pick
meets the tolerance.  The seeded pipeline with target_exit on its passes
solves the same targets from the same sources."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    import paper_2505_03728_amd as pk
    c = pk.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def arm(ctx):
    return ctx.upload(synth.arm7(0))


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(DEV)


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items() if not k.startswith("_")}


def _solve(ctx, rid, targets, seeds, T, K, w, o):
    out = ctx.alloc_outputs(rid, T, K, best=True)
    ctx.ik_solve(rid, targets, seeds, K, w, o, out)
    return out


@pytest.mark.parametrize("K", [8, 3, 128])
def test_target_exit_plain_solve(ctx, arm, K):
    import paper_2505_03728_amd as pk
    import torch
    tree = synth.arm7(0)
    T = {8: 1024, 3: 1000, 128: 64}[K]
    wl = synth.workload("seeder", targets=T)
    tg = oracle.targets_from(tree, wl["eval_q_star"])
    targets = torch.from_numpy(pk.pack_targets(tree.ee_kind, tg)).to(DEV)
    seeds = _dev(synth.uniform_configs(tree, T * K, 29).T)
    w = pk.Weights.from_dict(wl["weights"])
    o = pk.Options.from_dict(wl["options"], early_exit=True)
    ot = pk.Options.from_dict(wl["options"], early_exit=True, target_exit=True)
    a = _np(_solve(ctx, arm, targets, seeds, T, K, w, o))
    b = _np(_solve(ctx, arm, targets, seeds, T, K, w, ot))
    torch.cuda.synchronize()
    N = T * K
    st_a, st_b = a["status"] & 0xff, b["status"] & 0xff
    assert not np.any(st_a == pk.TARGET_SOLVED)
    np.testing.assert_array_equal(a["target_success"], b["target_success"])

    def first_tol(itt):
        v = np.where(itt >= 0, itt, 1 << 30).reshape(T, K).min(axis=1)
        return np.where(v == 1 << 30, -1, v)
    np.testing.assert_array_equal(first_tol(a["iters_to_tol"]), first_tol(b["iters_to_tol"]))
    ended = st_b == pk.TARGET_SOLVED
    kept = ~ended
    for key in ["iters", "accepts", "status", "iters_to_tol", "cost", "pose_cost"]:
        np.testing.assert_array_equal(a[key][kept], b[key][kept], err_msg=key)
    np.testing.assert_array_equal(a["joints"][:, kept], b["joints"][:, kept])
    # runs: consecutive problems of one target within one 64-problem wavefront
    p = np.arange(N)
    t = p // K
    run = np.cumsum(np.r_[True, (t[1:] != t[:-1]) | (p[1:] % 64 == 0)]) - 1
    itt_b = b["iters_to_tol"]
    first_in_run = np.full(run.max() + 1, 1 << 30)
    np.minimum.at(first_in_run, run[itt_b >= 0], itt_b[itt_b >= 0])
    assert np.all(first_in_run[run[ended]] < 1 << 30)
    np.testing.assert_array_equal(b["iters"][ended], first_in_run[run[ended]])
    assert np.all(b["iters"][ended] <= a["iters"][ended])
    assert np.all(itt_b[ended] == -1)
    # the pick meets the tolerance (it is a converged problem)
    succ = b["target_success"].astype(bool)
    bi = b["best_index"]
    assert np.all(st_b[np.nonzero(succ)[0] * K + bi[succ]] == pk.CONVERGED)
    bj = b["best_joints"].T.astype(np.float64)
    for tt in np.nonzero(succ)[0][:100]:
        _, pe, re = oracle.residual(tree, tg[tt], wl["weights"], bj[tt])
        assert pe[0] <= 1e-3 * 1.05 and re[0] <= 1e-2 * 1.05
    saved = 1.0 - b["iters"].sum() / a["iters"].sum()
    print(f"K={K}: {int(ended.sum())} of {N} problems ended by their target, "
          f"{saved:.1%} fewer LM iterations, success {succ.mean():.4f}")
    if K in (8, 128):
        assert ended.sum() > 0


def test_target_exit_seeded_pipeline(ctx, arm):
    """The seeded pipeline with target_exit on its refinement, restart and
    fallback passes: the same targets solved from the same sources, with the
    same first iteration at the tolerance, and fewer LM iterations."""
    import paper_2505_03728_amd as pk
    import torch
    tree = synth.arm7(0)
    T = 2048
    wl = synth.workload("seeder", targets=T)
    mc = wl["mlp"]
    K = wl["K"]
    sd = pk.Seeder(ctx, arm, K=K, hidden=mc["hidden"], depth=mc["depth"],
                   init=synth.mlp_init([7] + [mc["hidden"]] * mc["depth"] + [7 * K], mc["init_seed"]))
    S = 65536
    qtr = _dev(wl["train_q"][:S].T)
    perm = torch.from_numpy(np.stack([synth.epoch_permutation(S, mc["shuffle_seed"], e)
                                      for e in range(3)])).to(DEV)
    sd.train(qtr, batch=mc["batch"], epochs=3, lr=mc["lr"], perm=perm)
    tg = oracle.targets_from(tree, wl["eval_q_star"])
    targets = torch.from_numpy(pk.pack_targets(tree.ee_kind, tg)).to(DEV)
    Kf = 64
    rseeds = _dev(synth.uniform_configs(tree, T * Kf, 17).T)
    w = pk.Weights.from_dict(wl["weights"])
    res = {}
    for te in (False, True):
        ref = pk.Options.from_dict(wl["options"], max_iters=10, early_exit=True, target_exit=te)
        fb = pk.Options.from_dict(wl["options"], early_exit=True, target_exit=te)
        res[te] = ctx.ik_solve_seeded(arm, targets, sd, w, ref, fallback=fb, fallback_seeds=rseeds,
                                      fallback_K=Kf, counters=True, restart_iters=20)
    torch.cuda.synchronize()
    a, b = _np(res[False]), _np(res[True])
    for key in ["target_success", "source", "iters_to_tol", "n_restart", "n_fallback"]:
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)
    succ = b["target_success"].astype(bool)
    bj = b["best_joints"].T.astype(np.float64)
    for tt in np.nonzero(succ)[0][:150]:
        _, pe, re = oracle.residual(tree, tg[tt], wl["weights"], bj[tt])
        assert pe[0] <= 1e-3 * 1.05 and re[0] <= 1e-2 * 1.05
    its = {k: int(r["refine_iters"].sum() + r["restart_iters"].sum() + r["fallback_iters"].sum())
           for k, r in ((False, a), (True, b))}
    assert its[True] < its[False]
    print(f"seeded pipeline: success {succ.mean():.4f}; LM iterations {its[False]} -> {its[True]}")

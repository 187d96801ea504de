"""The allocation-free IK entry point (pk_ik_solve_noalloc) against pk_ik_solve:
same kernels, so every output is bit-identical, on two calls in a row (the
second smaller, so it reads scratch the first call left behind), with
best-of-K taking its cost, pose-only cost and status from the library's
scratch array; the size limit is refused before anything is launched."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import soa, targets_dev

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
KEYS = ["joints", "pos_err", "rot_err", "iters", "accepts", "iters_to_tol", "best_index",
        "best_joints", "target_success"]


@pytest.fixture(scope="module")
def ctx():
    import paper_2505_03728_amd as pk
    c = pk.Context(0)
    yield c
    c.close()


def _outputs(ctx, rid, T, K):
    """Outputs with best-of-K but no cost, pose-only cost or status buffers,
    so best-of-K runs on the library's scratch."""
    out = ctx.alloc_outputs(rid, T, K, best=True)
    for k in ("cost", "pose_cost", "status"):
        out.pop(k)
    return out


def _solve(ctx, rid, tree, tg, seeds, K, wl, noalloc):
    import paper_2505_03728_amd as pk
    import torch
    T = tg.shape[0]
    out = _outputs(ctx, rid, T, K)
    fn = ctx.ik_solve_noalloc if noalloc else ctx.ik_solve
    fn(rid, targets_dev(tree, tg, DEV), soa(seeds, DEV), K, pk.Weights.from_dict(wl["weights"]),
       pk.Options.from_dict(wl["options"]), out)
    torch.cuda.synchronize()
    return {k: out[k].cpu().numpy() for k in KEYS}


@pytest.mark.parametrize("wl_name,targets", [("arm131k", (2048, 300)), ("tree4k", (96, 40))])
def test_noalloc_matches_ik_solve_two_calls(ctx, wl_name, targets):
    wl = synth.workload(wl_name, targets=targets[0])
    g = wl["groups"][0]
    tree, K = g["tree"], g["K"]
    rid = ctx.upload(tree)
    tg = oracle.targets_from(tree, g["q_star"])
    for T in targets:            # the second call is smaller than the first
        ref = _solve(ctx, rid, tree, tg[:T], g["seeds"][:T * K], K, wl, noalloc=False)
        got = _solve(ctx, rid, tree, tg[:T], g["seeds"][:T * K], K, wl, noalloc=True)
        for k in KEYS:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{wl_name} T={T} {k}")
        print(f"{wl_name} T={T} K={K}: identical, {int(got['target_success'].sum())} targets solved")


def test_noalloc_refuses_more_than_its_limit(ctx):
    import paper_2505_03728_amd as pk
    import torch
    tree = synth.arm7(0)
    rid = ctx.upload(tree)
    K = 8
    T = pk.NOALLOC_MAX_PROBLEMS // K + 1
    targets = torch.zeros((7, T), dtype=torch.float32, device=DEV)
    seeds = torch.zeros((7, T * K), dtype=torch.float32, device=DEV)
    out = _outputs(ctx, rid, T, K)
    wl = synth.workload("arm131k", targets=1)
    with pytest.raises(pk.PkError, match="limit"):
        ctx.ik_solve_noalloc(rid, targets, seeds, K, pk.Weights.from_dict(wl["weights"]),
                             pk.Options.from_dict(wl["options"]), out)

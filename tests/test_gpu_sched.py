"""Mixed-robot persistent scheduler: results independent of the schedule
(iterations per launch, persistent grid size, graph or eager), equal to
separate launches, and in agreement with the FP64 oracle on a sample."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import check_excused, compare_outcome, soa, targets_dev

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    import paper_2505_03728_amd as pk
    c = pk.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def batch(ctx):
    import paper_2505_03728_amd as pk
    wl = synth.workload("mixed84k", scale=0.02)      # 1200 arm, 400 hand, 81 tree
    groups = []
    for g in wl["groups"]:
        tree = g["tree"]
        rid = ctx.upload(tree)
        tg = oracle.targets_from(tree, g["q_star"])
        groups.append({"rid": rid, "tree": tree, "tg": tg, "seeds_np": g["seeds"],
                       "targets": targets_dev(tree, tg, DEV), "seeds": soa(g["seeds"], DEV),
                       "K": g["K"], "weights": pk.Weights.from_dict(g["weights"]), "wd": g["weights"]})
    return wl, groups


def _fresh(ctx, groups, best=False):
    for g in groups:
        g["out"] = ctx.alloc_outputs(g["rid"], g["tg"].shape[0], g["K"], best=best)
    return groups


def _host(groups):
    return [{k: v.cpu().numpy() for k, v in g["out"].items() if not k.startswith("_")} for g in groups]


KEYS = ["joints", "pos_err", "rot_err", "cost", "iters", "accepts", "status", "iters_to_tol"]


def test_mixed_equals_separate_launches(ctx, batch):
    import paper_2505_03728_amd as pk
    import torch
    wl, groups = batch
    opt = pk.Options.from_dict(wl["options"])
    sep = _fresh(ctx, [dict(g) for g in groups])
    for g in sep:
        ctx.ik_solve(g["rid"], g["targets"], g["seeds"], g["K"], g["weights"], opt, g["out"])
    torch.cuda.synchronize()
    ref = _host(sep)
    S, PG = pk.SCHED_SINGLE, pk.SCHED_PER_GROUP
    for mode, k, wpc, wg, graph in [(S, 5, 2, 64, True), (S, 10, 4, 128, True), (S, 0, 1, 64, False),
                                    (S, 3, 8, 256, False), (S, 1, 4, 64, True), (PG, 5, 2, 64, True),
                                    (PG, 0, 4, 64, False)]:
        gs = _fresh(ctx, [dict(g) for g in groups])
        ctx.ik_solve_mixed(gs, opt, iters_per_launch=k, waves_per_cu=wpc, workgroup_size=wg,
                           use_graph=graph, mode=mode)
        if graph:       # replay the cached graph once more on the same buffers
            ctx.ik_solve_mixed(gs, opt, iters_per_launch=k, waves_per_cu=wpc, workgroup_size=wg,
                               use_graph=graph, mode=mode)
        torch.cuda.synchronize()
        got = _host(gs)
        for gi, (a, b) in enumerate(zip(ref, got)):
            for key in KEYS:
                np.testing.assert_array_equal(a[key], b[key], err_msg=f"mode={mode} k={k} group {gi} {key}")
        print(f"mode={mode} k={k} waves/CU={wpc} workgroup={wg} graph={graph}: identical to separate launches")


def test_mixed_per_group_variants_equal_separate_launches(ctx, batch):
    """Every group on the wave mapping (64 lanes per problem) through the
    scheduler equals pk_ik_solve with the wave variant, bit for bit."""
    import paper_2505_03728_amd as pk
    import torch
    wl, groups = batch
    sep = _fresh(ctx, [dict(g) for g in groups])
    opt_w = pk.Options.from_dict(wl["options"], variant=pk.VARIANT_WAVE)
    for g in sep:
        ctx.ik_solve(g["rid"], g["targets"], g["seeds"], g["K"], g["weights"], opt_w, g["out"])
    torch.cuda.synchronize()
    ref = _host(sep)
    opt = pk.Options.from_dict(wl["options"])
    gs = _fresh(ctx, [dict(g) for g in groups])
    ctx.ik_solve_mixed(gs, opt, iters_per_launch=10, waves_per_cu=4, use_graph=True,
                       variants=[pk.VARIANT_WAVE] * len(groups))
    torch.cuda.synchronize()
    got = _host(gs)
    for gi, (a, b) in enumerate(zip(ref, got)):
        for key in KEYS:
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"group {gi} {key}")
    # a lane mapping requested for the tree robot is refused
    with pytest.raises(pk.PkError):
        ctx.ik_solve_mixed(_fresh(ctx, [dict(g) for g in groups]), opt, iters_per_launch=10,
                           waves_per_cu=4, variants=[0, 0, pk.VARIANT_LANE])


def test_autotune_and_oracle_sample(ctx, batch):
    import paper_2505_03728_amd as pk
    import torch
    wl, groups = batch
    opt = pk.Options.from_dict(wl["options"])
    gs = _fresh(ctx, [dict(g) for g in groups], best=True)
    tuned = ctx.autotune_mixed(gs, opt)
    print(f"autotuned: {tuned}")
    k, variants = tuned["k"], tuned["variants"]
    assert k in (1, 2, 5, 10, 25, 0) and tuned["waves_per_cu"] in (2, 4, 8, 16) and tuned["ms"] > 0
    assert tuned["mode"] in (pk.SCHED_SINGLE, pk.SCHED_PER_GROUP)
    assert tuned["workgroup_size"] in (64, 128, 256)
    assert ctx.autotune_lookup(gs, opt) == tuned
    # the tree robot has only the wave mapping; the others may take either
    assert variants[2] == pk.VARIANT_WAVE and all(v in (pk.VARIANT_LANE, pk.VARIANT_WAVE) for v in variants)
    gs = _fresh(ctx, [dict(g) for g in groups], best=True)
    ctx.ik_solve_mixed(gs, opt)            # uses the tuned entry
    torch.cuda.synchronize()
    got = _host(gs)
    rng = np.random.default_rng(3)
    bad, excused, n = [], [], 0
    for g, out in zip(groups, got):
        N = g["seeds_np"].shape[0]
        for p in rng.choice(N, min(N, 40), replace=False):
            o = oracle.lm_solve(g["tree"], g["tg"][p // g["K"]], g["wd"], wl["options"],
                                g["seeds_np"][p], n_trace=wl["options"]["max_iters"])
            v, why = compare_outcome(ctx, g["rid"], g["tree"], g["tg"][p], g["seeds_np"][p], g["wd"],
                                     wl["options"], out["status"][p], out["iters_to_tol"][p], o)
            n += 1
            if v == "bad":
                print(f"{g['tree'].name} problem {p}: gpu iters {out['iters'][p]} status {out['status'][p]}, "
                      f"oracle {o['iters']} status {o['status']} ({why})")
                bad.append((g["tree"].name, int(p)))
            elif v == "excused":
                excused.append((g["tree"].name, int(p), why))
        print(f"{g['tree'].name}: success {np.mean((out['status'] & 0xff) == 0):.3f}")
    print(f"oracle sample: {bad} unexplained, {len(excused)} excused of {n}")
    assert not bad
    check_excused("scheduler oracle sample", excused, n)


def test_full_size_mixed84k_sampled(ctx):
    """The mixed benchmark's full batch (60000 arm + 20000 hand + 4096 tree, early
    exit, <= 50 iterations) in one scheduled graph launch with the schedule the
    autotuner picks for it, checked on a sample of each group."""
    import paper_2505_03728_amd as pk
    import torch
    wl = synth.workload("mixed84k")
    groups = []
    for g in wl["groups"]:
        tree = g["tree"]
        rid = ctx.upload(tree)
        tg = oracle.targets_from(tree, g["q_star"])
        groups.append({"rid": rid, "tree": tree, "tg": tg, "seeds_np": g["seeds"],
                       "targets": targets_dev(tree, tg, DEV), "seeds": soa(g["seeds"], DEV),
                       "K": 1, "weights": pk.Weights.from_dict(g["weights"]), "wd": g["weights"]})
    opt = pk.Options.from_dict(wl["options"])
    gs = _fresh(ctx, groups)
    ctx.ik_solve_mixed(gs, opt, iters_per_launch=25, waves_per_cu=8, use_graph=True,
                       variants=[pk.VARIANT_LANE, pk.VARIANT_LANE, pk.VARIANT_WAVE])
    torch.cuda.synchronize()
    got = _host(gs)
    rng = np.random.default_rng(17)
    bad, excused, n = [], [], 0
    for g, out in zip(groups, got):
        st = out["status"] & 0xff
        assert np.all(np.isin(st, [0, 1, 2]))
        # early exit: converged problems stop at their first point within tolerance
        np.testing.assert_array_equal(out["iters_to_tol"][st == 0], out["iters"][st == 0])
        for p in rng.choice(g["tg"].shape[0], 20, replace=False):
            o = oracle.lm_solve(g["tree"], g["tg"][p], g["wd"], wl["options"], g["seeds_np"][p],
                                n_trace=wl["options"]["max_iters"])
            v, why = compare_outcome(ctx, g["rid"], g["tree"], g["tg"][p], g["seeds_np"][p], g["wd"],
                                     wl["options"], out["status"][p], out["iters_to_tol"][p], o)
            n += 1
            if v == "bad":
                bad.append((g["tree"].name, int(p), why))
            elif v == "excused":
                excused.append((g["tree"].name, int(p), why))
        print(f"{g['tree'].name}: {st.size} problems, success {np.mean(st == 0):.4f}")
    print(f"mixed84k sample: {bad} unexplained, {len(excused)} excused of {n}")
    assert not bad
    check_excused("mixed84k sample", excused, n)


def test_autotune_table_json_round_trip(ctx, batch, tmp_path, monkeypatch):
    """The tuned schedule is stored as JSON keyed by the batch's robot classes
    (n, m, EE kind), options and architecture; a new context reads it from the
    file named by PK_AUTOTUNE_TABLE (and through autotune_load) and finds the
    same entry for the same robot classes (under its own robot ids)."""
    import json

    import paper_2505_03728_amd as pk
    wl, groups = batch
    opt = pk.Options.from_dict(wl["options"])
    gs = _fresh(ctx, [dict(g) for g in groups])
    tuned = ctx.autotune_lookup(gs, opt) or ctx.autotune_mixed(gs, opt)
    path = tmp_path / "autotune.json"
    ctx.autotune_save(str(path))
    doc = json.loads(path.read_text())
    assert doc["format"] == "pkmi-autotune-1"
    keys = [e["key"] for e in doc["entries"]]
    print(keys)
    assert any(k.startswith("n7_m1_pose+n16_m4_position+n34_m4_pose|") and "|gfx" in k for k in keys)
    monkeypatch.setenv("PK_AUTOTUNE_TABLE", str(path))
    c2 = pk.Context(0)
    try:
        g2 = []
        for g in groups:
            d = dict(g)
            d["rid"] = c2.upload(g["tree"])
            g2.append(d)
        g2 = _fresh(c2, g2)
        got = c2.autotune_lookup(g2, opt)
        fields = ("mode", "k", "waves_per_cu", "workgroup_size", "variants")
        assert got is not None and {k: got[k] for k in fields} == {k: tuned[k] for k in fields}
        assert c2.autotune_load(str(path)) == len(keys)
    finally:
        c2.close()

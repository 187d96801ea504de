"""GPU parity of the learned seeder's MFMA kernels against the FP64 MLP
oracle in BF16-emulation mode: forward within 1e-3 relative (Frobenius per
tensor) and every element within 1e-2 of the tensor's RMS; gradients within
2e-2 relative and every element within 5e-2 of the tensor's RMS; Adam over
several steps (parameters and both moments, element by element) against the
oracle's Adam fed the GPU's own gradients; the training/inference/checkpoint
paths; and the seeded pipeline with the seeder trained at full size."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from tests.gpu_util import borderline, check_excused

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


def _inputs(B, seed):
    tree = synth.arm7(0)
    q = synth.uniform_configs(tree, B, seed)
    tg = oracle.targets_from(tree, q)[:, 0, :]
    reach = float(np.sum(np.linalg.norm(tree.offset, axis=1)) + np.linalg.norm(tree.ee_offset[0]))
    x = mlp.encode_targets(tg[:, :3], tg[:, 3:], reach).astype(np.float32).astype(np.float64)
    return x, q


def _dev(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(DEV)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-30))


def _max_over_rms(a, b):
    """Largest element-wise difference over the reference tensor's RMS: a
    wrong row or column stands out here even where the Frobenius norm of the
    whole tensor hides it."""
    b = np.asarray(b, dtype=np.float64)
    rms = max(float(np.sqrt(np.mean(b * b))), 1e-30)
    return float(np.abs(np.asarray(a, dtype=np.float64) - b).max() / rms)


@pytest.mark.parametrize("hidden,depth,B", [(128, 2, 200), (512, 3, 300)])
def test_forward_matches_bf16_oracle(ctx, arm, hidden, depth, B):
    import paper_2505_03728_amd as pk
    import torch
    init = synth.mlp_init([7] + [hidden] * depth + [56], 21)
    sd = pk.Seeder(ctx, arm, K=8, hidden=hidden, depth=depth, init=init)
    x, _ = _inputs(B, 5)
    y = sd.forward(_dev(x))
    torch.cuda.synchronize()
    yo, _ = mlp.forward(init, x, emulate_bf16=True)
    rel = _rel(y.cpu().numpy(), yo)
    el = _max_over_rms(y.cpu().numpy(), yo)
    print(f"forward h={hidden} d={depth}: rel err {rel:.2e}, max element err / RMS {el:.2e}")
    assert rel <= 1e-3 and el <= 1e-2
    # parameters round-trip through the padded device layout
    got = sd.get(0)
    for (W, b), (Wg, bg) in zip(init, got):
        np.testing.assert_array_equal(Wg, W.astype(np.float32))
        np.testing.assert_array_equal(bg, b.astype(np.float32))


@pytest.mark.parametrize("hidden,depth,K", [(128, 1, 8), (256, 2, 8), (512, 3, 8), (256, 2, 4),
                                            (384, 2, 8)])
def test_fused_forward_equals_layer_path(ctx, arm, hidden, depth, K):
    """The fused inference kernel (activations kept on chip) takes each
    layer's reduction in the same order as the layer-by-layer GEMMs, so the
    two give identical outputs; also after the weights change (training).
    K=4 has 28 real outputs of the 64 computed; hidden width 384 is a shape
    the fused kernel leaves to the GEMMs."""
    import paper_2505_03728_amd as pk
    import torch
    init = synth.mlp_init([7] + [hidden] * depth + [7 * K], 31)
    sd = pk.Seeder(ctx, arm, K=K, hidden=hidden, depth=depth, init=init)
    for B in (300, 1024):
        x, _ = _inputs(B, 6 + B)
        xd = _dev(x)
        yf = sd.forward(xd)
        yl = sd.forward(xd, layers=True)
        torch.cuda.synchronize()
        assert torch.isfinite(yf).all()
        assert torch.equal(yf, yl), (B, float((yf - yl).abs().max()))
        yo, _ = mlp.forward(init, x, emulate_bf16=True)
        assert _rel(yf.cpu().numpy(), yo) <= 1e-3
    # new weights: two training steps, then both paths again
    q = synth.uniform_configs(synth.arm7(0), 256, 9)
    sd.train(_dev(q.T), batch=128, epochs=1, lr=1e-2)
    x, _ = _inputs(300, 77)
    xd = _dev(x)
    yf, yl = sd.forward(xd), sd.forward(xd, layers=True)
    torch.cuda.synchronize()
    assert torch.equal(yf, yl)
    yo, _ = mlp.forward(sd.get(0), x, emulate_bf16=True)
    assert _rel(yf.cpu().numpy(), yo) <= 1e-3


@pytest.mark.parametrize("hidden,depth,B", [(128, 2, 256), (512, 3, 512)])
def test_gradients_match_bf16_oracle(ctx, arm, hidden, depth, B):
    import paper_2505_03728_amd as pk
    import torch
    init = synth.mlp_init([7] + [hidden] * depth + [56], 22)
    sd = pk.Seeder(ctx, arm, K=8, hidden=hidden, depth=depth, init=init)
    x, q = _inputs(B, 6)
    loss = sd.grad(_dev(x), _dev(q))
    torch.cuda.synchronize()
    g = sd.get(1)
    y, cache = mlp.forward(init, x, emulate_bf16=True)
    lo, _, dy = mlp.min_over_k_loss(y, q, 8)
    go = mlp.backward(init, cache, dy, emulate_bf16=True)
    assert abs(loss.item() - lo) <= 1e-3 * lo
    for li, ((gW, gb), (oW, ob)) in enumerate(zip(g, go)):
        rw, rb = _rel(gW, oW), _rel(gb, ob)
        ew, eb = _max_over_rms(gW, oW), _max_over_rms(gb, ob)
        print(f"layer {li}: dW rel {rw:.2e} (max element / RMS {ew:.2e}), db rel {rb:.2e} ({eb:.2e})")
        assert rw <= 2e-2 and rb <= 2e-2
        assert ew <= 5e-2 and eb <= 5e-2


def test_adam_step_closed_form_and_training(ctx, arm):
    import paper_2505_03728_amd as pk
    import torch
    init = synth.mlp_init([7, 128, 128, 56], 23)
    sd = pk.Seeder(ctx, arm, K=8, hidden=128, depth=2, init=init)
    tree = synth.arm7(0)
    qtr = synth.uniform_configs(tree, 1024, 24)
    qdev = _dev(qtr.T)
    # one step on the first 1024 samples in index order
    log = torch.zeros(1, device=DEV)
    sd.train(qdev, batch=1024, epochs=1, lr=1e-3, loss_log=log)
    torch.cuda.synchronize()
    g = sd.get(1)
    p1 = sd.get(0)
    for (W0, b0), (W1, b1), (gW, gb) in zip(init, p1, g):
        np.testing.assert_allclose(W1 - W0.astype(np.float32), -1e-3 * gW / (np.abs(gW) + 1e-8),
                                   atol=2e-7)
        np.testing.assert_allclose(b1 - b0.astype(np.float32), -1e-3 * gb / (np.abs(gb) + 1e-8),
                                   atol=2e-7)
    # a few epochs reduce the loss
    S = 8192
    q = synth.uniform_configs(tree, S, 25)
    perm = np.stack([synth.epoch_permutation(S, 26, e) for e in range(6)])
    log = torch.zeros(6 * (S // 1024), device=DEV)
    sd.train(_dev(q.T), batch=1024, epochs=6, lr=1e-3,
             perm=torch.from_numpy(perm).to(DEV), loss_log=log)
    torch.cuda.synchronize()
    L = log.cpu().numpy()
    print("loss", L[0], L[len(L) // 2], L[-1])
    assert np.all(np.isfinite(L)) and L[-8:].mean() < 0.8 * L[:8].mean()


def test_adam_several_steps_elementwise(ctx, arm):
    """Four training steps on one fixed batch (index order, the batch is the
    whole set): after each, the GPU's parameters and both Adam moments equal,
    element by element, the oracle's Adam fed the gradients the GPU reports
    for that step, from the same initial parameters.  The oracle takes the
    hyperparameters as the library receives them (FP32-rounded lr, betas and
    eps, promoted).  Tolerances: v to 1e-6 relative (a sum of squares); m to
    1e-6 of the same recursion run on |g| (m may cancel to near zero while its
    terms do not); parameters to 2e-7 + 1e-6 |p| (the bias corrections
    1 - beta^t lose digits in FP32 at small t, about 1e-5 of a step of lr)."""
    import paper_2505_03728_amd as pk
    import torch
    f32 = lambda v: float(np.float32(v))
    init = synth.mlp_init([7, 128, 128, 56], 41)
    sd = pk.Seeder(ctx, arm, K=8, hidden=128, depth=2, init=init)
    q = synth.uniform_configs(synth.arm7(0), 1024, 42)
    qdev = _dev(q.T)
    cur = [(W.astype(np.float64), b.astype(np.float64)) for W, b in init]
    opt = mlp.Adam(cur, lr=f32(1e-3), b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8))
    scale = [[np.zeros(np.shape(W)), np.zeros(np.shape(b))] for W, b in cur]
    worst = {"p": 0.0, "m": 0.0, "v": 0.0}
    for step in range(4):
        sd.train(qdev, batch=1024, epochs=1, lr=1e-3)
        torch.cuda.synchronize()
        g = [(W.astype(np.float64), b.astype(np.float64)) for W, b in sd.get(1)]
        cur = opt.step(cur, g)
        gp, gm, gv = sd.get(0), sd.get(2), sd.get(3)
        for li in range(len(cur)):
            for j in range(2):
                scale[li][j] = opt.b1 * scale[li][j] + (1 - opt.b1) * np.abs(g[li][j])
                dp = np.abs(gp[li][j] - cur[li][j])
                assert np.all(dp <= 2e-7 + 1e-6 * np.abs(cur[li][j])), (step, li, j, dp.max())
                dm = np.abs(gm[li][j] - opt.m[li][j])
                assert np.all(dm <= 1e-6 * scale[li][j] + 1e-30), (step, li, j, dm.max())
                dv = np.abs(gv[li][j] - opt.v[li][j])
                assert np.all(dv <= 1e-6 * np.abs(opt.v[li][j]) + 1e-30), (step, li, j, dv.max())
                worst["p"] = max(worst["p"], float(dp.max()))
                worst["m"] = max(worst["m"], float((dm / (scale[li][j] + 1e-30)).max()))
                worst["v"] = max(worst["v"], float((dv / (np.abs(opt.v[li][j]) + 1e-30)).max()))
    print(f"Adam over 4 steps: max |dp| {worst['p']:.2e}, max dm / scale {worst['m']:.2e}, "
          f"max rel dv {worst['v']:.2e}")


def test_infer_seeds_within_limits_and_checkpoint(ctx, arm, tmp_path):
    import paper_2505_03728_amd as pk
    import torch
    tree = synth.arm7(0)
    init = synth.mlp_init([7, 128, 128, 56], 27)
    sd = pk.Seeder(ctx, arm, K=8, hidden=128, depth=2, init=init)
    q = synth.uniform_configs(tree, 300, 28)
    tg = oracle.targets_from(tree, q)
    targets = torch.from_numpy(pk.pack_targets(tree.ee_kind, tg)).to(DEV)
    seeds = sd.infer(targets)
    torch.cuda.synchronize()
    s = seeds.cpu().numpy()
    assert s.shape == (7, 300 * 8)
    assert np.all(s >= tree.lower[:, None].astype(np.float32) - 1e-7)
    assert np.all(s <= tree.upper[:, None].astype(np.float32) + 1e-7)
    # seeds equal the clamped network output on the encoded targets
    reach = float(np.sum(np.linalg.norm(tree.offset, axis=1)) + np.linalg.norm(tree.ee_offset[0]))
    x = mlp.encode_targets(tg[:, 0, :3], tg[:, 0, 3:], reach)
    y = sd.forward(_dev(x)).cpu().numpy().reshape(300, 8, 7)
    want = np.clip(y, tree.lower.astype(np.float32), tree.upper.astype(np.float32))
    d = np.abs(s.T.reshape(300, 8, 7) - want)
    # the device encodes in FP32, this side in FP64: a BF16 input may round
    # the other way now and then
    assert np.mean(d <= 1e-4) >= 0.99 and d.max() <= 5e-2
    path = tmp_path / "seeder.bin"
    sd.save(path)
    sd2 = pk.Seeder(ctx, arm, K=8, hidden=128, depth=2)
    sd2.load(path)
    for (W, b), (W2, b2) in zip(sd.get(0), sd2.get(0)):
        np.testing.assert_array_equal(W, W2)
        np.testing.assert_array_equal(b, b2)


@pytest.fixture(scope="module")
def trained(ctx, arm):
    """The seeder at the learned-seed workload's full size: MLP
    7-512-512-512-56 (K = 8), trained on its 2M (FK(q), q) pairs for 20
    epochs, batch 8192, Adam lr 1e-3, its seeded initial weights and epoch
    orders."""
    import paper_2505_03728_amd as pk
    import torch
    wl = synth.workload("seeder")
    mc = wl["mlp"]
    init = synth.mlp_init([7] + [mc["hidden"]] * mc["depth"] + [7 * wl["K"]], mc["init_seed"])
    sd = pk.Seeder(ctx, arm, K=wl["K"], hidden=mc["hidden"], depth=mc["depth"], init=init)
    S, E = wl["train_q"].shape[0], mc["epochs"]
    perm = np.stack([synth.epoch_permutation(S, mc["shuffle_seed"], e) for e in range(E)])
    log = torch.zeros(E * (S // mc["batch"]), device=DEV)
    sd.train(_dev(wl["train_q"].T), batch=mc["batch"], epochs=E, lr=mc["lr"],
             perm=torch.from_numpy(perm).to(DEV), loss_log=log)
    torch.cuda.synchronize()
    return sd, log


def test_trained_full_size_net_matches_oracle(ctx, arm, trained):
    """The trained full-size network (its parameters read back) against the
    oracle's BF16-emulated forward on a sample of fresh targets, element by
    element, through both the fused inference kernel and the layer path."""
    import torch
    sd, log = trained
    L = log.cpu().numpy()
    assert np.all(np.isfinite(L)) and L[-50:].mean() < 0.5 * L[:50].mean()
    x, _ = _inputs(512, 61)
    xd = _dev(x)
    yf, yl = sd.forward(xd), sd.forward(xd, layers=True)
    torch.cuda.synchronize()
    assert torch.equal(yf, yl)
    yo, _ = mlp.forward(sd.get(0), x, emulate_bf16=True)
    rel, el = _rel(yf.cpu().numpy(), yo), _max_over_rms(yf.cpu().numpy(), yo)
    print(f"trained 512x3 net: loss {L[0]:.3f} -> {L[-50:].mean():.3f}; forward rel {rel:.2e}, "
          f"max element / RMS {el:.2e}")
    assert rel <= 1e-3 and el <= 1e-2


def test_seeded_pipeline_and_gain_over_random_seeds(ctx, arm, trained):
    """A seeder trained briefly on (FK(q), q) pairs gives seeds from which
    10 LM iterations solve more targets than 10 iterations from random seeds;
    the pipeline's per-target results follow its own rules."""
    import paper_2505_03728_amd as pk
    import torch
    tree = synth.arm7(0)
    sd, log = trained
    T = 2048
    wl = synth.workload("seeder", targets=T)
    tg = oracle.targets_from(tree, wl["eval_q_star"])
    targets = torch.from_numpy(pk.pack_targets(tree.ee_kind, tg)).to(DEV)
    rseeds = _dev(wl["plain_seeds"].T)
    w = pk.Weights.from_dict(wl["weights"])
    ref = pk.Options.from_dict(wl["options"], max_iters=10, early_exit=True)
    fb = pk.Options.from_dict(wl["options"], max_iters=30)
    learned = ctx.ik_solve_seeded(arm, targets, sd, w, ref, fallback=None, fallback_K=0)
    both = ctx.ik_solve_seeded(arm, targets, sd, w, ref, fallback=fb, fallback_seeds=rseeds,
                               fallback_K=8, counters=True)
    plain = ctx.alloc_outputs(arm, T, 8, best=True)
    ctx.ik_solve(arm, targets, rseeds, 8, w, ref, plain)
    torch.cuda.synchronize()
    s_learn = learned["target_success"].cpu().numpy().astype(bool)
    s_both = both["target_success"].cpu().numpy().astype(bool)
    s_plain = plain["target_success"].cpu().numpy().astype(bool)
    src = both["source"].cpu().numpy()
    nfb = int(both["n_fallback"].item())
    print(f"loss {log[0].item():.3f} -> {log[-1].item():.3f}; 10-iteration success: "
          f"learned {s_learn.mean():.4f}, random {s_plain.mean():.4f}; with fallback "
          f"{s_both.mean():.4f} ({nfb} targets re-solved)")
    assert s_learn.mean() > s_plain.mean()
    np.testing.assert_array_equal(s_both[src == 0], True)
    np.testing.assert_array_equal(src == 0, s_learn)
    assert nfb == int((~s_learn).sum())
    assert np.all(s_both >= s_learn)
    fi = both["fallback_iters"].cpu().numpy().reshape(T, 8)
    assert np.all(fi[s_learn] == 0) and np.all(fi[~s_learn] > 0)
    # returned joints meet the tolerance where success is claimed
    bj = both["best_joints"].cpu().numpy().T.astype(np.float64)
    for t in np.nonzero(s_both)[0][:200]:
        _, pe, re = oracle.residual(tree, tg[t], wl["weights"], bj[t])
        assert pe[0] <= 1e-3 * 1.05 and re[0] <= 1e-2 * 1.05
    # the fallback in stages of c seeds: the same targets solved, every run
    # problem's counters as in the single stage, a stage prefix of each
    # fallback target's seeds run, and a target stops short of all 8 seeds
    # only once a stage has solved it
    fi_all = fi
    nfp = int(both["n_fallback_problems"].item())
    assert nfp == 8 * nfb
    for c in (2, 3):
        st = ctx.ik_solve_seeded(arm, targets, sd, w, ref, fallback=fb, fallback_seeds=rseeds,
                                 fallback_K=8, counters=True, fallback_chunk=c)
        torch.cuda.synchronize()
        for key in ["target_success", "source", "n_fallback", "refine_iters"]:
            np.testing.assert_array_equal(st[key].cpu().numpy(), both[key].cpu().numpy(),
                                          err_msg=f"chunk {c} {key}")
        fi_c = st["fallback_iters"].cpu().numpy().reshape(T, 8)
        kr = (fi_c > 0).sum(axis=1)
        ends = set(range(c, 8, c)) | {8}
        s_c = st["target_success"].cpu().numpy().astype(bool)
        for t in np.nonzero(~s_learn)[0]:
            assert kr[t] in ends, (c, t, kr[t])
            np.testing.assert_array_equal(fi_c[t, :kr[t]], fi_all[t, :kr[t]])
            assert kr[t] == 8 or s_c[t], (c, t)
        assert np.all(kr[s_learn] == 0)
        assert int(st["n_fallback_problems"].item()) == int(kr.sum())
        itt_c = st["iters_to_tol"].cpu().numpy()
        itt_b = both["iters_to_tol"].cpu().numpy()
        fb_ok = src == 1
        assert np.all(itt_c[fb_ok] >= itt_b[fb_ok])
        bj_c = st["best_joints"].cpu().numpy().T.astype(np.float64)
        for t in np.nonzero(fb_ok)[0][:100]:
            _, pe, re = oracle.residual(tree, tg[t], wl["weights"], bj_c[t])
            assert pe[0] <= 1e-3 * 1.05 and re[0] <= 1e-2 * 1.05
        print(f"fallback in stages of {c}: {int(kr.sum())} of {nfp} fallback problems run")
    # a restart pass between the refinement and the fallback: only targets the
    # refinement did not solve are restarted (their K problems, from the
    # refined joints), a restart success keeps the fallback off that target,
    # and the fallback then re-solves only what is left
    rs = ctx.ik_solve_seeded(arm, targets, sd, w, ref, fallback=fb, fallback_seeds=rseeds, fallback_K=8,
                             counters=True, restart_iters=20)
    torch.cuda.synchronize()
    src_r = rs["source"].cpu().numpy()
    s_r = rs["target_success"].cpu().numpy().astype(bool)
    ri = rs["restart_iters"].cpu().numpy().reshape(T, 8)
    fi_r = rs["fallback_iters"].cpu().numpy().reshape(T, 8)
    print(f"with a 20-iteration restart: success {s_r.mean():.4f} (restart solved {np.mean(src_r == 2):.4f}, "
          f"fallback {np.mean(src_r == 1):.4f})")
    assert int(rs["n_restart"].item()) == int((~s_learn).sum())
    np.testing.assert_array_equal(src_r == 0, s_learn)
    assert np.all(ri[s_learn] == 0) and np.all(ri[~s_learn] > 0)
    assert np.all(ri <= 20)
    restarted_ok = src_r == 2
    assert np.all(~s_learn[restarted_ok])
    assert np.all(fi_r[restarted_ok | s_learn] == 0)
    assert int(rs["n_fallback"].item()) == int((~s_learn & ~restarted_ok).sum())
    np.testing.assert_array_equal(s_r, np.isin(src_r, [0, 1, 2]))
    bj_r = rs["best_joints"].cpu().numpy().T.astype(np.float64)
    for t in np.nonzero(restarted_ok)[0][:100]:
        _, pe, re = oracle.residual(tree, tg[t], wl["weights"], bj_r[t])
        assert pe[0] <= 1e-3 * 1.05 and re[0] <= 1e-2 * 1.05
    itt_r = rs["iters_to_tol"].cpu().numpy()
    assert np.all(itt_r[restarted_ok] > 10) and np.all(itt_r[restarted_ok] <= 30)
    # the compacted refinement schedule (k iterations per launch) gives the
    # same per-target results as the single launch
    for k in (2, 3):
        comp = ctx.ik_solve_seeded(arm, targets, sd, w, ref, fallback=fb, fallback_seeds=rseeds,
                                   fallback_K=8, counters=True, refine_iters_per_launch=k,
                                   refine_blocks_per_cu=4)
        torch.cuda.synchronize()
        for key in ["best_joints", "target_success", "source", "iters_to_tol", "refine_iters",
                    "refine_accepts", "fallback_iters"]:
            np.testing.assert_array_equal(comp[key].cpu().numpy(), both[key].cpu().numpy(),
                                          err_msg=f"k={k} {key}")


def test_seeded_pipeline_full_size_sampled(ctx, arm, trained):
    """The seeded benchmark's size (131072 fresh targets, K = 8, <= 10 refinement
    iterations with early exit, 8 random seeds x 30 iterations as fallback):
    on a sample of targets the learned pass succeeds exactly where the FP64
    oracle, started from the same learned seeds, reaches the tolerance with
    one of them; claimed successes meet the tolerance at the returned joints."""
    import paper_2505_03728_amd as pk
    import torch
    tree = synth.arm7(0)
    sd, _ = trained
    wl = synth.workload("seeder")
    T = wl["eval_q_star"].shape[0]
    tg = oracle.targets_from(tree, wl["eval_q_star"])
    targets = torch.from_numpy(pk.pack_targets(tree.ee_kind, tg)).to(DEV)
    w = pk.Weights.from_dict(wl["weights"])
    ref = pk.Options.from_dict(wl["options"], max_iters=10, early_exit=True)
    fb = pk.Options.from_dict(wl["options"], max_iters=30)
    res = ctx.ik_solve_seeded(arm, targets, sd, w, ref, fallback=fb,
                              fallback_seeds=_dev(wl["plain_seeds"].T), fallback_K=8, counters=True,
                              restart_iters=20)
    seeds = sd.infer(targets)
    torch.cuda.synchronize()
    src = res["source"].cpu().numpy()
    succ = res["target_success"].cpu().numpy().astype(bool)
    sn = seeds.cpu().numpy().T.astype(np.float64)           # [T*K, n]
    assert np.all(sn >= tree.lower - 1e-6) and np.all(sn <= tree.upper + 1e-6)
    assert int(res["n_restart"].item()) == int((src != 0).sum())
    assert int(res["n_fallback"].item()) == int(((src != 0) & (src != 2)).sum())
    o = dict(wl["options"], max_iters=10, early_exit=True)
    o_r = dict(wl["options"], max_iters=20, early_exit=True)

    def near(outs):
        return any(r["trace_tie"].any() or borderline({"pos_err": [r["pos_err"]], "rot_err": [r["rot_err"]]}, 0)
                   for r in outs)
    rng = np.random.default_rng(23)
    bad, excused = 0, []
    # every restarted target among the first 2000 and a random sample: pass A
    # from the learned seeds, then (where pass A fails) the restart from its
    # final joints, on the oracle
    sample = np.unique(np.concatenate([rng.choice(T, 64, replace=False),
                                       np.nonzero(src[:2000] != 0)[0][:40]]))
    n_restarted = 0
    for t in sample:
        outs = [oracle.lm_solve(tree, tg[t], wl["weights"], o, sn[t * 8 + k], n_trace=10) for k in range(8)]
        so = any((r["status"] & 0xff) == 0 for r in outs)
        if so != (src[t] == 0):
            if near(outs):
                excused.append((int(t), "near-tie or borderline"))
            else:
                bad += 1
            continue
        if so:
            continue
        n_restarted += 1
        outs_r = [oracle.lm_solve(tree, tg[t], wl["weights"], o_r, r["q"], n_trace=20) for r in outs]
        sr = any((r["status"] & 0xff) == 0 for r in outs_r)
        if sr != (src[t] == 2):
            if near(outs) or near(outs_r):
                excused.append((int(t), "near-tie or borderline (restart)"))
            else:
                print(f"target {t}: restart success gpu {src[t] == 2}, oracle {sr}")
                bad += 1
    bj = res["best_joints"].cpu().numpy().T.astype(np.float64)
    for t in np.nonzero(succ)[0][:: max(1, int(succ.sum()) // 300)]:
        _, pe, re = oracle.residual(tree, tg[t], wl["weights"], bj[t])
        assert pe[0] <= 1e-3 * 1.05 and re[0] <= 1e-2 * 1.05
    print(f"seeded 131072: success {succ.mean():.4f}, learned {np.mean(src == 0):.4f}, restart "
          f"{np.mean(src == 2):.4f}; sample {bad} unexplained, {len(excused)} excused of {len(sample)} "
          f"({n_restarted} restarted on the oracle)")
    assert n_restarted >= 20
    assert bad == 0
    check_excused("seeded 131072 sample", excused, len(sample))

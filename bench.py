"""Benchmark: batched LM IK solves/s on one MI355X.

Headline workload (one step): 16384 reachable targets x 8 random in-limit
seeds on the seeded 7-DoF arm (131072 LM problems), FP32, at most 30 LM
iterations with early exit at 1 mm / 0.01 rad, pose + joint-limit + rest
(0.01) residuals, best-of-8 per target.  Inputs are resident in HBM before
timing (targets are FK of seeded configurations, computed on the GPU).  The
step (LM launch + best-of-K launch) is captured once into a HIP graph; the
step time is the median over the timed replays, each bracketed by HIP events.
value = successful targets (1 mm / 0.01 rad) per second of that time.

The same line carries the learned-seed comparison: the seeder MLP
(7-512-512-512-56, BF16 matrix cores) trained here on 2M (FK(q), q) pairs,
then learned seeds + <= 6 LM iterations + restart + random-seed fallback against plain
LM from 8 random seeds, on 131072 fresh targets (success, solves/s,
iterations to tolerance, FP32 roofline fraction of each form).

Prints one JSON line.  The roofline entry is for the LM kernel, timed alone
with HIP events on its stream; the CPU baseline is the FP64 oracle on a
bounded sample of the headline workload on the host's cores (and on one).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VALU_PEAK = 157.3      # TFLOP/s, MI355X FP32 vector (datasheet; packed FP32)
FP32_VALU_UNPACKED = 78.6   # TFLOP/s, 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz
BF16_MFMA_PEAK = 2500.0     # TFLOP/s, MI355X dense BF16 matrix cores (datasheet)

# HBM traffic per launch of the arm LM kernel: rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads for
# a 256 MiB device-to-device copy (--copy-probe).  Valid only while the kernel
# sources hash to `sha256` and the run is the profiled workload; otherwise the
# bench reports traffic as null.
LANE_KERNEL_SOURCES = ["paper_2505_03728_amd/csrc/lm_lane.hip", "paper_2505_03728_amd/csrc/lm_lane.hpp",
                       "paper_2505_03728_amd/csrc/lm_lane_kernels.hpp", "paper_2505_03728_amd/csrc/pk_device.hpp",
                       "paper_2505_03728_amd/csrc/pk_internal.hpp", "include/pkmi.h"]
ARM_TRAFFIC = {"sha256": "e230fbc486226fec", "fetch_kib": 2842.0, "write_kib": 7680.0, "fetch_scale": 2.0,
               "write_scale": 1.0,
               "workload": {"targets": 16384, "K": 8, "max_iters": 30, "early_exit": True},
               "profile": "profiles/lm_lane_arm131k_hbm_counters.md"}


def sources_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def arm_traffic_bytes(workload):
    """HBM bytes per launch from the stored counter readings, or None when the
    kernel sources or the workload differ from the profiled ones."""
    t = ARM_TRAFFIC
    if t["sha256"] is None or t["sha256"] != sources_hash(LANE_KERNEL_SOURCES) or \
            workload != t["workload"]:
        return None
    return round(1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="headline only (skip the learned-seed comparison)")
    ap.add_argument("--targets", type=int, default=16384)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--fixed-budget", action="store_true",
                    help="early exit off (every problem runs all its iterations)")
    ap.add_argument("--workload", default="arm131k",
                    choices=["arm131k", "tree4k", "mixed84k", "seeder", "beam", "mobile", "traj"])
    ap.add_argument("--epochs", type=int, default=None)   # None: the seeder workload's
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device-to-device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def host_cpu():
    """CPU model, logical CPUs of the host and CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    return {"cpu_model": model, "host_logical_cpus": os.cpu_count(), "affinity_cpus": aff}


# A GPU's share of its host is 16 CPUs: the oracle's thread pool is sized to
# the CPUs this process may run on, at most that share.
CPU_SHARE = 16


def oracle_threads():
    return max(1, min(CPU_SHARE, host_cpu()["affinity_cpus"]))


def cpu_baseline(tree, wl, T_full, K, budget_s):
    """FP64 oracle on the host: whole chunks of targets until the budget is
    spent, on the pool's threads; then a shorter sample on one thread."""
    import oracle
    import synth
    threads = oracle_threads()
    g = synth.workload("arm131k", targets=T_full)["groups"][0]

    def run(nthreads, budget, chunk):
        done_t = succ = 0
        elapsed = 0.0
        while done_t < T_full and elapsed < budget:
            a, b = done_t, min(T_full, done_t + chunk)
            tg = oracle.targets_from(tree, g["q_star"][a:b])
            s0 = time.perf_counter()
            r = oracle.lm_solve_batch(tree, tg, g["seeds"][a * K:b * K], K, wl["weights"],
                                      wl["options"], threads=nthreads)
            _, ok = oracle.best_of_k(r["status"], r["cost"], r["pose_cost"], K)
            elapsed += time.perf_counter() - s0
            succ += int(ok.sum())
            done_t = b
        return succ, done_t, elapsed

    succ, done_t, elapsed = run(threads, budget_s, 512)
    s1, d1, e1 = run(1, budget_s / 3, 32)
    cpu = host_cpu()
    return {"value": succ / elapsed if elapsed > 0 else 0.0, "unit": "solves/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {done_t} of {T_full} targets x {K} seeds, FP64, at most "
                      f"{wl['options']['max_iters']} iterations (early exit "
                      f"{'on' if wl['options']['early_exit'] else 'off'}), {elapsed:.1f} s on "
                      f"{threads} threads (FK of targets not timed); one thread: first {d1} "
                      f"targets, {e1:.1f} s",
            "success_rate": succ / max(done_t, 1),
            "value_1thread": s1 / e1 if e1 > 0 else 0.0,
            **cpu}


def _replay_times(fn, steps, warmup):
    """Per-step times (ms) of fn, each bracketed by HIP events on the current
    stream, after warmup untimed calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for e0, e1 in ev:
        e0.record(st)
        fn()
        e1.record(st)
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in ev]


def _stats(ts):
    import numpy as np
    a = np.asarray(ts)
    return {"median": float(np.median(a)), "p10": float(np.percentile(a, 10)),
            "p90": float(np.percentile(a, 90)), "mean": float(a.mean()), "reps": int(a.size)}


def _itt_per_target(itt, T, K):
    """Iterations to tolerance per target: the fewest over its seeds (solved
    targets only), mean and median."""
    import numpy as np
    itt = itt.reshape(T, K)
    best = np.where(itt >= 0, itt, 10 ** 6).min(1)
    ok = best < 10 ** 6
    return (float(best[ok].mean()) if ok.any() else None,
            float(np.median(best[ok])) if ok.any() else None)


def headline(args, ctx):
    """The benchmark's step, graph-captured; the LM kernel timed alone for the
    roofline."""
    import numpy as np
    import torch

    import paper_2505_03728_amd as pk
    from paper_2505_03728_amd.flops import lm_bytes, lm_flops
    import synth

    dev = "cuda:0"
    wl = synth.workload("arm131k", targets=args.targets)
    wl["options"]["early_exit"] = not args.fixed_budget
    g = wl["groups"][0]
    tree, K = g["tree"], g["K"]
    T = g["q_star"].shape[0]
    N = T * K
    rid = ctx.upload(tree)
    info = ctx.robot_info(rid)

    qstar = torch.from_numpy(np.ascontiguousarray(g["q_star"].T.astype(np.float32))).to(dev)
    ee = ctx.fk(rid, qstar)                                   # [m, 7, T]
    planes = [ee[k, :(7 if kd == 0 else 3)] for k, kd in enumerate(tree.ee_kind)]
    targets = torch.cat(planes, 0).contiguous()
    seeds = torch.from_numpy(np.ascontiguousarray(g["seeds"].T.astype(np.float32))).to(dev)
    w = pk.Weights.from_dict(wl["weights"])
    o = pk.Options.from_dict(wl["options"], variant=args.variant)
    out = ctx.alloc_outputs(rid, T, K, best=True, full=False)
    out["status"] = torch.empty(N, dtype=torch.int32, device=dev)
    out["cost"] = torch.empty(N, dtype=torch.float32, device=dev)

    # warm up eagerly (the library sizes its workspace here), then capture
    for _ in range(max(1, args.warmup)):
        ctx.ik_solve(rid, targets, seeds, K, w, o, out)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(graph, stream=cap):
            ctx.ik_solve(rid, targets, seeds, K, w, o, out)
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    print(f"# graph captured; warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
    ts = _replay_times(graph.replay, args.steps, args.warmup)
    st = _stats(ts)
    ms_step = st["median"]
    success = int(out["target_success"].sum().item())
    value = success / (ms_step / 1e3)
    print(f"# timed {args.steps} graph replays: median {ms_step:.4f} ms/step", file=sys.stderr, flush=True)

    # LM kernel alone (no best-of-K launch), HIP events on the same stream.
    out2 = ctx.alloc_outputs(rid, T, K, best=False, full=True)
    kts = _replay_times(lambda: ctx.ik_solve(rid, targets, seeds, K, w, o, out2), max(5, args.steps), 1)
    k_ms = float(np.mean(kts))
    iters = int(out2["iters"].sum().item())
    accepts = int(out2["accepts"].sum().item())
    blocks = [info["chain_len"]] * info["chains"] if (info["chains"] and args.variant != 2) else None
    flops = lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, blocks, iters, accepts, N)
    achieved = flops / (k_ms / 1e3) / 1e12
    conv = ((out2["status"] & 0xFF) == pk.CONVERGED).float().mean().item()
    fp64 = ((out2["status"] & pk.FLAG_FP64) != 0).float().mean().item()
    itt_mean, itt_med = _itt_per_target(out2["iters_to_tol"].cpu().numpy(), T, K)
    hbm = lm_bytes(info["n"], info["m"], info["target_floats"], N, T)
    wkey = {"targets": T, "K": K, "max_iters": wl["options"]["max_iters"],
            "early_exit": bool(wl["options"]["early_exit"])}

    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("# copy probe: 268435456 bytes read + written", file=sys.stderr, flush=True)

    res = {
        "metric": "IK solves/sec at 1mm/0.01rad success",
        "value": round(value, 1),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"7-DoF arm LM IK: {T} targets x {K} random seeds = {N} problems, "
                               f"at most {wl['options']['max_iters']} iterations (early exit "
                               f"{'on' if wl['options']['early_exit'] else 'off'}), pose(1.0/0.5) + "
                               f"limit(10) + rest(0.01), best-of-{K}", "targets": T,
                   "seeds_per_target": K, "problems": N, "lm_iters": wl["options"]["max_iters"],
                   "early_exit": bool(wl["options"]["early_exit"]),
                   "variant": ["auto", "lane", "wave"][args.variant]},
        "timing": {"method": "HIP graph of the step (LM + best-of-K launches), replayed; "
                             "each replay bracketed by HIP events; ms_per_step = median",
                   **{k: (round(v, 5) if isinstance(v, float) else v) for k, v in st.items()}},
        "success_rate": success / T,
        "problem_convergence": round(conv, 5),
        "fp64_fallback_fraction": round(fp64, 5),
        "iters_to_tol_per_target": {"mean": itt_mean, "median": itt_med},
        "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": FP32_VALU_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VALU_PEAK, 5),
                     "traffic": arm_traffic_bytes(wkey) if args.variant != 2 else None,
                     "traffic_source": ARM_TRAFFIC["profile"],
                     "kernel": "lm_lane_kernel<1,7,pose>" if args.variant != 2
                     else "lm_path_kernel<8,4>", "kernel_ms": round(k_ms, 5),
                     "algorithmic_flops": flops, "algorithmic_hbm_bytes": hbm,
                     "peak_unpacked_fp32": FP32_VALU_UNPACKED,
                     "frac_of_unpacked": round(achieved / FP32_VALU_UNPACKED, 5),
                     "lm_problem_iterations": iters, "accepted": accepts},
    }
    return res, tree, wl, T, K


# Learned form's passes: LM iterations from the learned seeds, the restart
# budget, and random seeds per target for the fallback (also the plain form's
# seed count for its >= 99% comparison).  Six refinement iterations leave more
# targets to the restart than ten but cost less overall (same success).
REFINE_ITERS = 6
RESTART_ITERS = 20
FALLBACK_K = 128


def learned_vs_random(args, ctx, epochs=None):
    """The learned-seed form against plain random-seed LM on the seeder
    workload: 131072 fresh targets of the 7-DoF arm, K = 8."""
    import numpy as np
    import torch

    import paper_2505_03728_amd as pk
    from paper_2505_03728_amd.flops import lm_flops
    import synth
    wl = synth.workload("seeder")
    tree, K = wl["tree"], wl["K"]
    mc = wl["mlp"]
    rid = ctx.upload(tree)
    init = synth.mlp_init([7] + [mc["hidden"]] * mc["depth"] + [7 * K], mc["init_seed"])
    sd = pk.Seeder(ctx, rid, K=K, hidden=mc["hidden"], depth=mc["depth"], init=init)
    S = wl["train_q"].shape[0]
    E = epochs or mc["epochs"]
    qtr = torch.from_numpy(np.ascontiguousarray(wl["train_q"].T.astype(np.float32))).cuda()
    perm = torch.from_numpy(np.stack([synth.epoch_permutation(S, mc["shuffle_seed"], e)
                                      for e in range(E)])).cuda()
    steps_tr = E * (S // mc["batch"])
    log = torch.zeros(steps_tr, device="cuda")
    t0 = time.perf_counter()
    sd.train(qtr, batch=mc["batch"], epochs=E, lr=mc["lr"], perm=perm, loss_log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del perm, qtr
    print(f"# trained {steps_tr} steps in {train_s:.2f} s, loss {log[0].item():.4f} -> "
          f"{log[-1].item():.4f}", file=sys.stderr, flush=True)
    T = wl["eval_q_star"].shape[0]
    targets = _dev_targets(ctx, rid, tree, wl["eval_q_star"])
    # random in-limit seeds: the first 8 per target are the plain form's, all
    # FALLBACK_K of them serve the learned form's fallback and the plain form at
    # FALLBACK_K seeds
    rseeds_all = torch.from_numpy(np.ascontiguousarray(
        synth.uniform_configs(tree, T * FALLBACK_K, 17).T.astype(np.float32))).cuda()
    rseeds = rseeds_all[:, :T * K].contiguous()
    w = pk.Weights.from_dict(wl["weights"])
    plain_o = pk.Options.from_dict(wl["options"], early_exit=True)          # <= 30 iterations
    ref_o = pk.Options.from_dict(wl["options"], max_iters=REFINE_ITERS, early_exit=True)
    plain = ctx.alloc_outputs(rid, T, K, best=True)
    ts_plain = _replay_times(lambda: ctx.ik_solve(rid, targets, rseeds, K, w, plain_o, plain),
                             args.steps, args.warmup)
    plain10 = ctx.alloc_outputs(rid, T, K, best=True)
    ts_plain10 = _replay_times(lambda: ctx.ik_solve(rid, targets, rseeds, K, w, ref_o, plain10),
                               args.steps, args.warmup)
    plain_big = ctx.alloc_outputs(rid, T, FALLBACK_K, best=True)
    ts_plain_big = _replay_times(lambda: ctx.ik_solve(rid, targets, rseeds_all, FALLBACK_K, w, plain_o,
                                                      plain_big), max(5, args.steps // 4), 1)
    res_l = {}

    def learned():
        res_l["o"] = ctx.ik_solve_seeded(rid, targets, sd, w, ref_o, fallback=plain_o,
                                         fallback_seeds=rseeds_all, fallback_K=FALLBACK_K, counters=True,
                                         restart_iters=RESTART_ITERS)
    ts_learn = _replay_times(learned, args.steps, args.warmup)
    # both forms again with target_exit: a problem also ends once another
    # problem of its target in its run of lanes met the tolerance (per-target
    # success and first iteration at the tolerance unchanged)
    plain_te_o = pk.Options.from_dict(wl["options"], early_exit=True, target_exit=True)
    ref_te_o = pk.Options.from_dict(wl["options"], max_iters=REFINE_ITERS, early_exit=True,
                                    target_exit=True)
    plain_te = ctx.alloc_outputs(rid, T, K, best=True)
    ts_plain_te = _replay_times(lambda: ctx.ik_solve(rid, targets, rseeds, K, w, plain_te_o, plain_te),
                                args.steps, args.warmup)
    res_t = {}

    def learned_te():
        res_t["o"] = ctx.ik_solve_seeded(rid, targets, sd, w, ref_te_o, fallback=plain_te_o,
                                         fallback_seeds=rseeds_all, fallback_K=FALLBACK_K, counters=True,
                                         restart_iters=RESTART_ITERS)
    ts_learn_te = _replay_times(learned_te, args.steps, args.warmup)
    seeds_buf = torch.empty((7, T * K), device="cuda")
    ts_infer = _replay_times(lambda: sd.infer(targets, seeds_buf), args.steps, args.warmup)
    torch.cuda.synchronize()
    ms_learn, ms_plain = _stats(ts_learn)["median"], _stats(ts_plain)["median"]
    ms_plain10, ms_infer = _stats(ts_plain10)["median"], _stats(ts_infer)["median"]
    lo = res_l["o"]
    s_plain = int(plain["target_success"].sum())
    s_plain10 = int(plain10["target_success"].sum())
    s_learn = int(lo["target_success"].sum())
    src = lo["source"].cpu().numpy()
    itt_l = lo["iters_to_tol"].cpu().numpy()
    itt_p_mean, itt_p_med = _itt_per_target(plain["iters_to_tol"].cpu().numpy(), T, K)
    blocks = [7]
    fl_plain = lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, blocks, int(plain["iters"].sum()),
                        int(plain["accepts"].sum()), T * K)
    n_fb = int(lo["n_fallback"].item())
    n_rs = int(lo["n_restart"].item())
    fl_lm = lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, blocks, int(lo["refine_iters"].sum()),
                     int(lo["refine_accepts"].sum()), T * K)
    fl_lm += lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, blocks, int(lo["restart_iters"].sum()),
                      int(lo["restart_accepts"].sum()), n_rs * K)
    fl_lm += lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, blocks, int(lo["fallback_iters"].sum()),
                      int(lo["fallback_accepts"].sum()), n_fb * FALLBACK_K)
    ms_big = _stats(ts_plain_big)["median"]
    s_big = int(plain_big["target_success"].sum())
    fl_big = lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, blocks, int(plain_big["iters"].sum()),
                      int(plain_big["accepts"].sum()), T * FALLBACK_K)
    itt_b_mean, itt_b_med = _itt_per_target(plain_big["iters_to_tol"].cpu().numpy(), T, FALLBACK_K)
    dims = [7] + [mc["hidden"]] * mc["depth"] + [7 * K]
    fl_mlp = 2.0 * T * sum(a * b for a, b in zip(dims[:-1], dims[1:]))
    v_learn = s_learn / (ms_learn / 1e3)
    v_plain = s_plain / (ms_plain / 1e3)
    ms_learn_te, ms_plain_te = _stats(ts_learn_te)["median"], _stats(ts_plain_te)["median"]
    lt = res_t["o"]
    s_learn_te = int(lt["target_success"].sum())
    s_plain_te = int(plain_te["target_success"].sum())
    v_learn_te = s_learn_te / (ms_learn_te / 1e3)
    v_plain_te = s_plain_te / (ms_plain_te / 1e3)
    its_te = int(lt["refine_iters"].sum() + lt["restart_iters"].sum() + lt["fallback_iters"].sum())
    its_pp = int(lo["refine_iters"].sum() + lo["restart_iters"].sum() + lo["fallback_iters"].sum())
    ok_l = itt_l >= 0
    tfl = lambda f, ms: f / (ms / 1e3) / 1e12
    return {
        "targets": T, "seeds_per_target": K,
        "timing": "median of per-call HIP-event times (eager launches)",
        "learned": {"solves_per_s": round(v_learn, 1), "success_rate": s_learn / T,
                    "ms": round(ms_learn, 5),
                    "success_from_learned_seeds": float(np.mean(src == 0)),
                    "success_from_restart": float(np.mean(src == 2)),
                    "success_from_fallback": float(np.mean(src == 1)),
                    "restarted_targets": n_rs, "fallback_targets": n_fb,
                    "iters_to_tol_mean": float(itt_l[ok_l].mean()) if ok_l.any() else None,
                    "iters_to_tol_median": float(np.median(itt_l[ok_l])) if ok_l.any() else None,
                    "lm_tflops": round(tfl(fl_lm, ms_learn), 4),
                    "frac_fp32": round(tfl(fl_lm, ms_learn) / FP32_VALU_PEAK, 6),
                    "inference_ms": round(ms_infer, 5),
                    "inference_frac_bf16": round(tfl(fl_mlp, ms_infer) / BF16_MFMA_PEAK, 5),
                    "schedule": f"seeder ({K} seeds) -> <= {REFINE_ITERS} LM iterations (early exit) -> unsolved "
                                f"targets: LM restarted from the refined joints, <= {RESTART_ITERS} "
                                f"iterations -> still unsolved: {FALLBACK_K} random seeds x <= 30 "
                                f"iterations"},
        "plain_random": {"solves_per_s": round(v_plain, 1), "success_rate": s_plain / T,
                         "ms": round(ms_plain, 5),
                         "iters_to_tol_mean": itt_p_mean, "iters_to_tol_median": itt_p_med,
                         "tflops": round(tfl(fl_plain, ms_plain), 4),
                         "frac_fp32": round(tfl(fl_plain, ms_plain) / FP32_VALU_PEAK, 6),
                         "success_rate_10_iters": s_plain10 / T,
                         "solves_per_s_10_iters": round(s_plain10 / (ms_plain10 / 1e3), 1)},
        "plain_random_many_seeds": {"seeds_per_target": FALLBACK_K,
                                    "solves_per_s": round(s_big / (ms_big / 1e3), 1),
                                    "success_rate": s_big / T, "ms": round(ms_big, 5),
                                    "iters_to_tol_mean": itt_b_mean, "iters_to_tol_median": itt_b_med,
                                    "frac_fp32": round(tfl(fl_big, ms_big) / FP32_VALU_PEAK, 6)},
        "speedup_learned_vs_plain": round(v_learn / v_plain, 3),
        "target_exit": {"rule": "both forms with target_exit: a problem also ends in the pass in which "
                                "another problem of its target in its run of lanes met the tolerance",
                        "learned": {"solves_per_s": round(v_learn_te, 1), "success_rate": s_learn_te / T,
                                    "ms": round(ms_learn_te, 5), "lm_iterations": its_te,
                                    "lm_iterations_without": its_pp},
                        "plain_random": {"solves_per_s": round(v_plain_te, 1), "success_rate": s_plain_te / T,
                                         "ms": round(ms_plain_te, 5),
                                         "lm_iterations": int(plain_te["iters"].sum()),
                                         "lm_iterations_without": int(plain["iters"].sum())}},
        "speedup_learned_vs_plain_target_exit": round(v_learn_te / v_plain_te, 3),
        "speedup_learned_vs_plain_many_seeds": round(v_learn / (s_big / (ms_big / 1e3)), 3),
        "seeder_training": {"samples": S, "epochs": E, "batch": mc["batch"], "steps": steps_tr,
                            "seconds": round(train_s, 3), "loss_first": float(log[0]),
                            "loss_last": float(log[-1])},
        "mlp_flops": fl_mlp,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)
    if args.workload != "arm131k":
        {"tree4k": run_tree, "mixed84k": run_mixed, "seeder": run_seeder,
         "beam": run_beam, "mobile": run_mobile, "traj": run_traj}[args.workload](args)
        return
    import paper_2505_03728_amd as pk
    ctx = pk.Context(0)
    res, tree, wl, T, K = headline(args, ctx)
    if not args.no_learned:
        print("# learned seeds vs random seeds ...", file=sys.stderr, flush=True)
        res["learned_vs_random"] = learned_vs_random(args, ctx, args.epochs)
    if not args.no_cpu:
        print("# cpu baseline (FP64 oracle) ...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(tree, wl, T, K, args.cpu_seconds)
    print(json.dumps(res), flush=True)
    ctx.close()


# ------------------------------------------------------------------ extra workloads

def _line(metric, value, unit, args, ms, config, **kw):
    d = {"metric": metric, "value": round(value, 1), "unit": unit, "n_gpus": 1,
         "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
         "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
         "data": "synthetic", "config": config}
    d.update(kw)
    return d


def _time(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _dev_targets(ctx, rid, tree, q_star):
    import numpy as np
    import torch
    q = torch.from_numpy(np.ascontiguousarray(q_star.T.astype(np.float32))).cuda()
    ee = ctx.fk(rid, q)
    return torch.cat([ee[k, :(7 if kd == 0 else 3)] for k, kd in enumerate(tree.ee_kind)], 0).contiguous()


def _oracle_rate(groups, weights, options, budget_s):
    """FP64 oracle over the groups' problems (round robin chunks) within the budget."""
    import oracle
    threads = oracle_threads()
    done = succ = 0
    elapsed = 0.0
    off = [0] * len(groups)
    while elapsed < budget_s and any(o < g["q_star"].shape[0] for o, g in zip(off, groups)):
        for gi, g in enumerate(groups):
            a = off[gi]
            if a >= g["q_star"].shape[0]:
                continue
            b = min(g["q_star"].shape[0], a + 256)
            tg = oracle.targets_from(g["tree"], g["q_star"][a:b])
            s0 = time.perf_counter()
            r = oracle.lm_solve_batch(g["tree"], tg, g["seeds"][a * g["K"]:b * g["K"]], g["K"],
                                      g.get("w", weights), options, threads=threads)
            _, ok = oracle.best_of_k(r["status"], r["cost"], r["pose_cost"], g["K"])
            elapsed += time.perf_counter() - s0
            succ += int(ok.sum())
            done += b - a
            off[gi] = b
    return succ / elapsed if elapsed else 0.0, threads, done, elapsed


def run_tree(args):
    """34-DoF tree, 4 pose EEs, 4096 problems, 40 iterations (one problem per wavefront,
    path-pair layout)."""
    import numpy as np
    import torch

    import paper_2505_03728_amd as pk
    from paper_2505_03728_amd.flops import lm_flops
    import synth
    wl = synth.workload("tree4k")
    g = wl["groups"][0]
    tree, K = g["tree"], 1
    T = g["q_star"].shape[0]
    ctx = pk.Context(0)
    rid = ctx.upload(tree)
    targets = _dev_targets(ctx, rid, tree, g["q_star"])
    seeds = torch.from_numpy(np.ascontiguousarray(g["seeds"].T.astype(np.float32))).cuda()
    w, o = pk.Weights.from_dict(wl["weights"]), pk.Options.from_dict(wl["options"])
    out = ctx.alloc_outputs(rid, T, K)
    ms = _time(lambda: ctx.ik_solve(rid, targets, seeds, K, w, o, out), args.steps, args.warmup)
    conv = int(((out["status"] & 0xFF) == 0).sum().item())
    flops = lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, None, int(out["iters"].sum()),
                     int(out["accepts"].sum()), T)
    ach = flops / (ms / 1e3) / 1e12
    res = _line("IK solves/sec at 1mm/0.01rad success", conv / (ms / 1e3), "solves/s", args, ms,
                {"workload": f"34-DoF tree (torso 6 + 4x7), 4 pose EEs, {T} problems x 1 seed, "
                             f"{wl['options']['max_iters']} iterations, pose + limit", "problems": T},
                success_rate=conv / T,
                fp64_fallback_fraction=float(((out["status"] & 0x100) != 0).float().mean()),
                roofline={"bound": "alu", "achieved": round(ach, 4), "peak": FP32_VALU_PEAK,
                          "unit": "TFLOP/s", "frac": round(ach / FP32_VALU_PEAK, 6), "traffic": None,
                          "kernel": "lm_path_kernel<16,4,12>", "kernel_ms": round(ms, 5),
                          "algorithmic_flops": flops})
    if not args.no_cpu:
        rate, th, done, el = _oracle_rate([{"tree": tree, "q_star": g["q_star"], "seeds": g["seeds"],
                                            "K": 1}], wl["weights"], wl["options"], args.cpu_seconds)
        res["cpu_baseline"] = {"value": rate, "unit": "solves/s", "cores": th, "kind": "oracle",
                               "sample": f"first {done} of {T} problems, {el:.1f} s"}
    print(json.dumps(res), flush=True)


def run_mixed(args):
    """60000 arm + 20000 hand + 4096 tree problems in one scheduled graph launch."""
    import numpy as np
    import torch

    import paper_2505_03728_amd as pk
    from paper_2505_03728_amd.flops import lm_flops
    import synth
    wl = synth.workload("mixed84k")
    ctx = pk.Context(0)
    groups = []
    for g in wl["groups"]:
        tree = g["tree"]
        rid = ctx.upload(tree)
        T = g["q_star"].shape[0]
        groups.append({"rid": rid, "tree": tree, "K": 1, "q_star": g["q_star"], "seeds_np": g["seeds"],
                       "targets": _dev_targets(ctx, rid, tree, g["q_star"]),
                       "seeds": torch.from_numpy(np.ascontiguousarray(g["seeds"].T.astype(np.float32))).cuda(),
                       "weights": pk.Weights.from_dict(g["weights"]), "wd": g["weights"],
                       "out": ctx.alloc_outputs(rid, T, 1)})
    o = pk.Options.from_dict(wl["options"])
    tuned = ctx.autotune_mixed(groups, o)
    k, wpc, wg, variants = tuned["k"], tuned["waves_per_cu"], tuned["workgroup_size"], tuned["variants"]
    mode = "single persistent launch" if tuned["mode"] == pk.SCHED_SINGLE else "per-group launches"
    vnames = ["lane" if v == pk.VARIANT_LANE else "wave" for v in variants]
    print(f"# autotuned {mode} k={k} waves/CU={wpc} workgroup={wg} variants={vnames} ({tuned['ms']:.3f} ms)",
          file=sys.stderr, flush=True)
    ms = _time(lambda: ctx.ik_solve_mixed(groups, o), args.steps, args.warmup)
    # the best of the other mode on the same groups, for comparison
    other = pk.SCHED_PER_GROUP if tuned["mode"] == pk.SCHED_SINGLE else pk.SCHED_SINGLE
    ms_other = min(_time(lambda: ctx.ik_solve_mixed(groups, o, iters_per_launch=kk, waves_per_cu=ww,
                                                    variants=variants, mode=other), args.steps, args.warmup)
                   for kk in (0, 25) for ww in (4, 8))
    # the same groups launched one by one without the scheduler
    ms_sep = _time(lambda: [ctx.ik_solve(g["rid"], g["targets"], g["seeds"], 1, g["weights"], o, g["out"])
                            for g in groups], args.steps, args.warmup)
    ctx.ik_solve_mixed(groups, o)
    torch.cuda.synchronize()
    conv, flops, per = 0, 0.0, {}
    for g in groups:
        out, tree = g["out"], g["tree"]
        c = int(((out["status"] & 0xFF) == 0).sum().item())
        conv += c
        info = ctx.robot_info(g["rid"])
        blocks = [info["chain_len"]] * info["chains"] if info["chains"] else None
        flops += lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, blocks, int(out["iters"].sum()),
                          int(out["accepts"].sum()), out["joints"].shape[1])
        per[tree.name] = {"problems": out["joints"].shape[1], "success_rate": c / out["joints"].shape[1],
                          "mean_iters": float(out["iters"].float().mean())}
    N = sum(g["out"]["joints"].shape[1] for g in groups)
    ach = flops / (ms / 1e3) / 1e12
    res = _line("IK solves/sec at 1mm/0.01rad success", conv / (ms / 1e3), "solves/s", args, ms,
                {"workload": "mixed batch in one graph launch: 60000 7-DoF arm + 20000 16-DoF hand "
                             "(4 fingertip positions) + 4096 34-DoF tree problems, early exit, <= 50 "
                             "iterations", "problems": N, "schedule": mode, "iters_per_launch": k,
                 "waves_per_cu": wpc, "workgroup_size": wg,
                 "lanes_per_problem": {g["tree"].name: (1 if v == pk.VARIANT_LANE else 64)
                                       for g, v in zip(groups, variants)}},
                success_rate=conv / N, groups=per, ms_separate_launches=round(ms_sep, 5),
                ms_other_schedule={"schedule": "per-group launches" if other == pk.SCHED_PER_GROUP
                                   else "single persistent launch", "ms": round(ms_other, 5)},
                roofline={"bound": "alu", "achieved": round(ach, 4), "peak": FP32_VALU_PEAK,
                          "unit": "TFLOP/s", "frac": round(ach / FP32_VALU_PEAK, 6), "traffic": None,
                          "kernel": "lm_mixed_kernel (one persistent launch over all groups)"
                          if tuned["mode"] == pk.SCHED_SINGLE else
                          "persistent lm_lane / lm_path kernels (one per group, concurrent)",
                          "algorithmic_flops": flops})
    if not args.no_cpu:
        rate, th, done, el = _oracle_rate(
            [{"tree": g["tree"], "q_star": g["q_star"], "seeds": g["seeds_np"], "K": 1, "w": g["wd"]}
             for g in groups], wl["weights"], wl["options"], args.cpu_seconds)
        res["cpu_baseline"] = {"value": rate, "unit": "solves/s", "cores": th, "kind": "oracle",
                               "sample": f"{done} of {N} problems (round robin over the groups), {el:.1f} s"}
    print(json.dumps(res), flush=True)


def run_seeder(args):
    """Learned seeder (trained here) + <= 6 LM iterations, restart and fallback, against
    8 random seeds x 30 iterations, on 131072 fresh targets of the 7-DoF arm."""
    import paper_2505_03728_amd as pk
    import synth
    ctx = pk.Context(0)
    lv = learned_vs_random(args, ctx, args.epochs)
    wl = synth.workload("seeder")
    L, P = lv["learned"], lv["plain_random"]
    res = _line("IK solves/sec at 1mm/0.01rad success", L["solves_per_s"], "solves/s", args, L["ms"],
                {"workload": f"7-DoF arm, {lv['targets']} fresh targets: learned seeder (MLP "
                             f"7-512-512-512-56, K={lv['seeds_per_target']}, BF16 MFMA) + <={REFINE_ITERS} LM "
                             f"iterations (early exit) + restart + fallback to random seeds, vs plain "
                             f"random seeds", "targets": lv["targets"], "seeds_per_target": lv["seeds_per_target"],
                 "epochs": lv["seeder_training"]["epochs"]},
                success_rate=L["success_rate"], learned_vs_random=lv,
                roofline={"bound": "mfma", "achieved": round(lv["mlp_flops"] / (L["inference_ms"] / 1e3) / 1e12, 3),
                          "peak": BF16_MFMA_PEAK, "unit": "TFLOP/s", "frac": L["inference_frac_bf16"],
                          "traffic": None,
                          "kernel": "seeder inference (fused BF16 MFMA MLP kernel + encode + seeds)",
                          "kernel_ms": L["inference_ms"], "algorithmic_flops": lv["mlp_flops"]})
    if not args.no_cpu:
        g = {"tree": wl["tree"], "q_star": wl["eval_q_star"], "seeds": wl["plain_seeds"], "K": wl["K"]}
        rate, th, done, el = _oracle_rate([g], wl["weights"], dict(wl["options"], early_exit=True),
                                          args.cpu_seconds)
        res["cpu_baseline"] = {"value": rate, "unit": "solves/s", "cores": th, "kind": "oracle",
                               "sample": f"plain form: first {done} of {lv['targets']} targets x "
                                         f"{wl['K']} seeds, {el:.1f} s", **host_cpu()}
    print(json.dumps(res), flush=True)
    ctx.close()


# IK-Beam GPU times of the paper's Table II (analytic Jacobians, RTX 4090,
# Franka Panda), ms per batch: context only (other robot and hardware).
PAPER_BEAM_MS = {1: 3.6, 10: 3.6, 100: 4.7, 1000: 15.5, 2000: 32.8}


def run_beam(args):
    """IK-Beam (64 seeds, 6 iterations, 4 kept, 10 iterations) on the 7-DoF arm
    at the paper's batch sizes; value = targets per second at batch 2000."""
    import numpy as np
    import torch

    import paper_2505_03728_amd as pk
    from paper_2505_03728_amd.flops import lm_flops
    import synth
    wl = synth.workload("beam")
    g = wl["groups"][0]
    tree, K, sch = g["tree"], g["K"], wl["schedule"]
    ctx = pk.Context(0)
    rid = ctx.upload(tree)
    w, o = pk.Weights.from_dict(wl["weights"]), pk.Options.from_dict(wl["options"])
    batches = {}
    for B in wl["batches"]:
        targets = _dev_targets(ctx, rid, tree, g["q_star"][:B])
        seeds = torch.from_numpy(np.ascontiguousarray(g["seeds"][:B * K].T.astype(np.float32))).cuda()
        out = ctx.alloc_beam_outputs(rid, B, K, sch["keep"])
        ms = _time(lambda: ctx.ik_beam(rid, targets, seeds, w, o, out=out, **sch), args.steps,
                   args.warmup)
        pe = out["pos_err"][0].cpu().numpy() * 1e3
        re = out["rot_err"][0].cpu().numpy()
        batches[B] = {"ms": round(ms, 4), "success": float(out["target_success"].float().mean()),
                      "p98_pos_err_mm": float(np.percentile(pe, 98)),
                      "p98_rot_err_rad": float(np.percentile(re, 98)),
                      "paper_ms_context": PAPER_BEAM_MS.get(B)}
        print(f"# batch {B}: {ms:.4f} ms", file=sys.stderr, flush=True)
    B = wl["batches"][-1]
    ms = batches[B]["ms"]
    # The dominant kernel, stage 0 (B*64 problems, 6 iterations), timed alone.
    targets = _dev_targets(ctx, rid, tree, g["q_star"][:B])
    seeds = torch.from_numpy(np.ascontiguousarray(g["seeds"][:B * K].T.astype(np.float32))).cuda()
    o0 = pk.Options.from_dict(dict(wl["options"], max_iters=sch["iters0"]))
    out0 = ctx.alloc_outputs(rid, B, K)
    k_ms = _time(lambda: ctx.ik_solve(rid, targets, seeds, K, w, o0, out0), max(5, args.steps), 1)
    info = ctx.robot_info(rid)
    blocks = [info["chain_len"]] * info["chains"]
    flops = lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, blocks, int(out0["iters"].sum()),
                     int(out0["accepts"].sum()), B * K)
    ach = flops / (k_ms / 1e3) / 1e12
    res = _line("IK-Beam targets/sec (batch 2000)", B / (ms / 1e3), "targets/s", args, ms,
                {"workload": f"IK-Beam on the 7-DoF arm: {B} targets x {K} seeds, "
                             f"{sch['iters0']} LM iterations, best {sch['keep']} kept, "
                             f"{sch['iters1']} more, best returned; pose(1.0/0.5) + limit(10)",
                 "targets": B, "schedule": sch},
                success_rate=batches[B]["success"], batches=batches,
                roofline={"bound": "alu", "achieved": round(ach, 4), "peak": FP32_VALU_PEAK,
                          "unit": "TFLOP/s", "frac": round(ach / FP32_VALU_PEAK, 6),
                          "traffic": None, "kernel": "lm_lane_kernel<1,7,pose> (stage 0)",
                          "kernel_ms": round(k_ms, 5), "algorithmic_flops": flops})
    if not args.no_cpu:
        import oracle
        threads = oracle_threads()
        done = succ = 0
        el = 0.0
        while done < B and el < args.cpu_seconds:
            a, b = done, min(B, done + 100)
            tg = oracle.targets_from(tree, g["q_star"][a:b])
            t0 = time.perf_counter()
            r = oracle.ik_beam(tree, tg, g["seeds"][a * K:b * K], K, sch["iters0"], sch["keep"],
                               sch["iters1"], wl["weights"], wl["options"], threads=threads)
            el += time.perf_counter() - t0
            succ += int(r["success"].sum())
            done = b
        res["cpu_baseline"] = {"value": done / el if el else 0.0, "unit": "targets/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"first {done} of {B} targets in batches of 100, FP64, "
                                         f"{el:.1f} s", "success_rate": succ / max(done, 1)}
    print(json.dumps(res), flush=True)
    ctx.close()


def run_mobile(args):
    """IK with a mobile base (Sec. V-B): 4096 translated targets x 4 seeds on the
    arm with its SE(2) base pose as variables (prismatic x, y + revolute yaw: a
    10-joint chain on the per-lane kernel); the same targets with the base
    fixed at the origin (arm alone) are solved once for the success comparison."""
    import numpy as np
    import torch

    import paper_2505_03728_amd as pk
    from paper_2505_03728_amd.flops import lm_flops
    import synth
    wl = synth.workload("mobile")
    g = wl["groups"][0]
    mob, K = g["tree"], g["K"]
    T = g["q_star"].shape[0]
    N = T * K
    ctx = pk.Context(0)
    rid = ctx.upload(mob)
    targets = _dev_targets(ctx, rid, mob, g["q_star"])
    seeds = torch.from_numpy(np.ascontiguousarray(g["seeds"].T.astype(np.float32))).cuda()
    w, o = pk.Weights.from_dict(wl["weights"]), pk.Options.from_dict(wl["options"])
    out = ctx.alloc_outputs(rid, T, K, best=True)
    ms = _time(lambda: ctx.ik_solve(rid, targets, seeds, K, w, o, out), args.steps, args.warmup)
    succ = int(out["target_success"].sum().item())
    st = out["status"].cpu().numpy()
    pe = out["pos_err"].cpu().numpy()[0].reshape(T, K)
    bi = out["best_index"].cpu().numpy()
    flops = lm_flops(mob.parent, mob.ee_joint, mob.ee_kind, None, int(out["iters"].sum()),
                     int(out["accepts"].sum()), T * K)
    ach = flops / (ms / 1e3) / 1e12
    # fixed base: the arm alone on the same targets, seeds without the base part
    arm = synth.arm7(0)
    rid_a = ctx.upload(arm)
    seeds_a = torch.from_numpy(np.ascontiguousarray(wl["fixed_base"]["seeds"].T.astype(np.float32))).cuda()
    out_a = ctx.alloc_outputs(rid_a, T, K, best=True)
    ctx.ik_solve(rid_a, targets, seeds_a, K, w, o, out_a)
    torch.cuda.synchronize()
    pe_a = out_a["pos_err"].cpu().numpy()[0].reshape(T, K)[np.arange(T), out_a["best_index"].cpu().numpy()]
    res = _line("IK solves/sec at 5mm/0.05rad success (mobile base)", succ / (ms / 1e3), "solves/s",
                args, ms,
                {"workload": f"mobile-base IK: 7-DoF arm on an SE(2) base (10 variables), {T} "
                             f"translated targets x {K} seeds, {wl['options']['max_iters']} "
                             f"iterations, pose + limit, best-of-{K}", "targets": T,
                 "problems": N},
                success_rate=succ / T,
                mean_pos_err_mm=float(pe[np.arange(T), bi].mean() * 1e3),
                fixed_base={"success_rate": float(out_a["target_success"].float().mean()),
                            "mean_pos_err_mm": float(pe_a.mean() * 1e3)},
                fp64_fallback_fraction=float(((st & 0x100) != 0).mean()),
                roofline={"bound": "alu", "achieved": round(ach, 4), "peak": FP32_VALU_PEAK,
                          "unit": "TFLOP/s", "frac": round(ach / FP32_VALU_PEAK, 6), "traffic": None,
                          "kernel": (f"lm_lane_kernel<1,{ctx.robot_info(rid)['chain_len']},pose+prismatic>"
                                     if ctx.robot_info(rid)["chains"] == 1 else "lm_path_kernel<16,4>"),
                          "kernel_ms": round(ms, 5), "algorithmic_flops": flops})
    if not args.no_cpu:
        rate, th, done, el = _oracle_rate([{"tree": mob, "q_star": g["q_star"], "seeds": g["seeds"],
                                            "K": K}], wl["weights"], wl["options"], args.cpu_seconds)
        res["cpu_baseline"] = {"value": rate, "unit": "solves/s", "cores": th, "kind": "oracle",
                               "sample": f"first {done} of {T} targets x {K} seeds, {el:.1f} s"}
    print(json.dumps(res), flush=True)
    ctx.close()


FP64_VALU_PEAK = 78.6       # TFLOP/s, MI355X FP64 vector (datasheet)


def traj_solve_flops(V, hb):
    """Algorithmic FLOPs of one damped band solve, counted as a band Cholesky
    (column scale and trailing update) plus the two triangular solves, V
    variables, half-bandwidth hb (divisions and square roots counted as one;
    the kernel's L D L^T has the same count up to lower-order terms)."""
    f = 0
    for j in range(V):
        w = min(hb, V - 1 - j)
        f += 1 + w + w * (w + 1) + 4 * w + 2
    return f


def run_traj(args):
    """Trajectory optimisation: 1024 arm trajectories x 32 timesteps, 20 LM
    iterations, one workgroup of four wavefronts per trajectory (banded FP64
    normal equations, blocked L D L^T)."""
    import numpy as np
    import torch

    import paper_2505_03728_amd as pk
    import synth
    wl = synth.workload("traj")
    tree, c, o = wl["tree"], wl["costs"], wl["options"]
    B, T, n = wl["init"].shape
    ctx = pk.Context(0)
    rid = ctx.upload(tree)
    st = _dev_targets(ctx, rid, tree, wl["start_q"])
    gl = _dev_targets(ctx, rid, tree, wl["goal_q"])
    init = torch.from_numpy(np.ascontiguousarray(wl["init"], dtype=np.float32)).cuda()
    vmax = torch.tensor(c["vmax"], dtype=torch.float32, device="cuda")
    opt = pk.Options.from_dict(o)
    out = ctx.traj_solve(rid, st, gl, init, c, opt, vmax=vmax)
    ms = _time(lambda: ctx.traj_solve(rid, st, gl, init, c, opt, vmax=vmax, out=out), args.steps,
               args.warmup)
    succ = float(((out["status"] & 0xFF) == 0).float().mean())
    iters = int(out["iters"].sum())
    flops = iters * traj_solve_flops(T * n, 4 * n)
    ach = flops / (ms / 1e3) / 1e12
    res = _line("optimised trajectories/sec", B / (ms / 1e3), "trajectories/s", args, ms,
                {"workload": f"trajectory optimisation on the 7-DoF arm: {B} trajectories x {T} "
                             f"timesteps (dt {c['dt']} s), start/goal pose + limit + smoothness + "
                             f"velocity limit + five-point acceleration and jerk, "
                             f"{o['max_iters']} LM iterations", "trajectories": B, "timesteps": T},
                dtype="f64 (normal equations) / f32 (kinematics)", success_rate=succ,
                roofline={"bound": "alu", "achieved": round(ach, 4), "peak": FP64_VALU_PEAK,
                          "unit": "TFLOP/s", "frac": round(ach / FP64_VALU_PEAK, 6), "traffic": None,
                          "kernel": "traj_kernel<7>", "kernel_ms": round(ms, 5),
                          "algorithmic_flops": flops,
                          "count": "band factorisation (Cholesky count) + two triangular solves per LM iteration"})
    if not args.no_cpu:
        import oracle
        from oracle import traj
        from threadpoolctl import threadpool_limits
        st_o = oracle.targets_from(tree, wl["start_q"])
        gl_o = oracle.targets_from(tree, wl["goal_q"])
        done = 0
        el = 0.0
        with threadpool_limits(1):
            while done < B and el < args.cpu_seconds:
                t0 = time.perf_counter()
                traj.lm_solve(tree, st_o[done], gl_o[done], c, o, wl["init"][done])
                el += time.perf_counter() - t0
                done += 1
        res["cpu_baseline"] = {"value": done / el if el else 0.0, "unit": "trajectories/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"first {done} of {B} trajectories, FP64 dense LM "
                                         f"(numpy, one thread), {el:.1f} s"}
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

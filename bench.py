"""Benchmark: batched LM IK solves/s on one MI355X.

Workload (one step): 16384 reachable targets x 8 random in-limit seeds on
the seeded 7-DoF arm (131072 LM problems), FP32, 30 LM iterations, pose +
joint-limit + rest (0.01) residuals, best-of-8 per target.  Inputs are
resident in HBM before timing (targets are FK of seeded configurations,
computed on the GPU).  value = successful targets (1 mm / 0.01 rad) per
second of the timed region.

Prints one JSON line.  The roofline entry is for the LM kernel, timed alone
with HIP events on its stream; the CPU baseline is the FP64 oracle on a
bounded sample of the same workload on the host's cores.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--targets", type=int, default=16384)
    ap.add_argument("--variant", type=int, default=0)
    return ap.parse_args()


def cpu_baseline(tree, wl, T_full, K, budget_s):
    """FP64 oracle on the host: whole chunks of targets until the budget is spent."""
    import numpy as np

    import oracle
    import synth
    threads = max(1, min(16, os.cpu_count() or 1))
    g = synth.workload("arm131k", targets=T_full)["groups"][0]
    chunk = 512
    done_t = succ = 0
    t0 = time.perf_counter()
    elapsed = 0.0
    while done_t < T_full and elapsed < budget_s:
        a, b = done_t, min(T_full, done_t + chunk)
        tg = oracle.targets_from(tree, g["q_star"][a:b])
        s0 = time.perf_counter()
        r = oracle.lm_solve_batch(tree, tg, g["seeds"][a * K:b * K], K, wl["weights"],
                                  wl["options"], threads=threads)
        _, ok = oracle.best_of_k(r["status"], r["cost"], r["pose_cost"], K)
        elapsed += time.perf_counter() - s0
        succ += int(ok.sum())
        done_t = b
    rate = succ / elapsed if elapsed > 0 else 0.0
    return {"value": rate, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"first {done_t} of {T_full} targets x {K} seeds, FP64, "
                      f"{wl['options']['max_iters']} iterations, {elapsed:.1f} s (FK of targets "
                      f"not timed)",
            "success_rate": succ / max(done_t, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2505_03728_amd as pk
    from paper_2505_03728_amd.flops import lm_bytes, lm_flops
    import synth

    dev = "cuda:0"
    wl = synth.workload("arm131k", targets=args.targets)
    g = wl["groups"][0]
    tree, K = g["tree"], g["K"]
    T = g["q_star"].shape[0]
    N = T * K
    ctx = pk.Context(0)
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

    for _ in range(args.warmup):
        ctx.ik_solve(rid, targets, seeds, K, w, o, out)
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.ik_solve(rid, targets, seeds, K, w, o, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    success = int(out["target_success"].sum().item())
    value = success / (ms_step / 1e3)
    print(f"# timed {args.steps} steps: {ms_step:.4f} ms/step", file=sys.stderr, flush=True)

    # LM kernel alone (no best-of-K launch), HIP events on the same stream.
    out2 = ctx.alloc_outputs(rid, T, K, best=False, full=True)
    ctx.ik_solve(rid, targets, seeds, K, w, o, out2)
    torch.cuda.synchronize()
    ks = max(5, args.steps)
    e0.record(stream)
    for _ in range(ks):
        ctx.ik_solve(rid, targets, seeds, K, w, o, out2)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / ks
    iters = int(out2["iters"].sum().item())
    accepts = int(out2["accepts"].sum().item())
    blocks = [info["chain_len"]] * info["chains"] if (info["chains"] and args.variant != 2) else [info["n"]]
    flops = lm_flops(tree.parent, tree.ee_joint, tree.ee_kind, blocks, iters, accepts, N)
    achieved = flops / (k_ms / 1e3) / 1e12
    conv = ((out2["status"] & 0xFF) == pk.CONVERGED).float().mean().item()
    fp64 = ((out2["status"] & pk.FLAG_FP64) != 0).float().mean().item()
    itt = out2["iters_to_tol"].cpu().numpy().reshape(T, K)
    itt_t = np.where(itt >= 0, itt, 10 ** 6).min(1)
    solved = itt_t < 10 ** 6
    hbm = lm_bytes(info["n"], info["m"], info["target_floats"], N, T)

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
                               f"{wl['options']['max_iters']} iterations, pose(1.0/0.5) + limit(10) "
                               f"+ rest(0.01), best-of-{K}", "targets": T, "seeds_per_target": K,
                   "problems": N, "lm_iters": wl["options"]["max_iters"],
                   "variant": ["auto", "lane", "wave"][args.variant]},
        "success_rate": success / T,
        "problem_convergence": round(conv, 5),
        "fp64_fallback_fraction": round(fp64, 5),
        "iters_to_tol_mean_per_target": float(itt_t[solved].mean()) if solved.any() else None,
        "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": FP32_VALU_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VALU_PEAK, 5),
                     "traffic": None, "kernel": "lm_lane_kernel<1,7,pose>" if args.variant != 2
                     else "lm_wave_kernel", "kernel_ms": round(k_ms, 5),
                     "algorithmic_flops": flops, "algorithmic_hbm_bytes": hbm,
                     "peak_unpacked_fp32": FP32_VALU_UNPACKED,
                     "frac_of_unpacked": round(achieved / FP32_VALU_UNPACKED, 5),
                     "lm_problem_iterations": iters, "accepted": accepts},
    }
    if not args.no_cpu:
        print("# cpu baseline (FP64 oracle) ...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(tree, wl, T, K, args.cpu_seconds)
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

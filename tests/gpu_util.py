"""Helpers shared by the GPU tests: device marshalling and oracle comparison."""
import numpy as np

import oracle
import synth


def rot_angle(Ra, Rb):
    """Angle of Ra^T Rb (radians), FP64."""
    return float(np.linalg.norm(oracle.so3_log(Ra.T @ Rb)))


def quat_to_R(q):
    return oracle.quat_to_R(np.asarray(q, dtype=np.float64))


def soa(a, device):
    """[N, n] host array -> [n, N] cuda float32 tensor."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32).T)).to(device)


def targets_dev(tree, tg, device):
    import torch
    import paper_2505_03728_amd as pk
    return torch.from_numpy(pk.pack_targets(tree.ee_kind, tg)).to(device)


def solve_gpu(ctx, rid, tree, tg, seeds, K, weights, options, trace_iters=0, best=False,
              device="cuda:0", **optkw):
    import torch
    import paper_2505_03728_amd as pk
    T = tg.shape[0]
    out = ctx.alloc_outputs(rid, T, K, best=best, trace_iters=trace_iters)
    ctx.ik_solve(rid, targets_dev(tree, tg, device), soa(seeds, device), K,
                 pk.Weights.from_dict(weights), pk.Options.from_dict(options, **optkw), out)
    torch.cuda.synchronize()
    res = {}
    for k, v in out.items():
        if k.startswith("_"):
            continue
        res[k] = v.cpu().numpy()
    res["q"] = res["joints"].T
    if "trace_q" in res:
        res["trace_q"] = res["trace_q"].transpose(2, 0, 1)       # [N, t, n]
        res["trace_accept"] = res["trace_accept"].T               # [N, t]
    return res


def borderline_at(tree, tg, w, trace_q, it, tol_pos=1e-3, tol_rot=1e-2, frac=0.05):
    """The oracle's iterate after iteration `it` (1-based) has an EE error
    within 5% of a tolerance, so the iteration at which FP32 first meets the
    tolerance may differ from FP64's by rounding."""
    import oracle
    if it < 1 or it > len(trace_q):
        return False
    _, pe, re = oracle.residual(tree, tg, w, trace_q[it - 1])
    pose = np.asarray(tree.ee_kind) == 0
    return bool(np.any(np.abs(pe - tol_pos) <= frac * tol_pos) or
                np.any((np.abs(re - tol_rot) <= frac * tol_rot) & pose))


def borderline(ora_res, p, tol_pos=1e-3, tol_rot=1e-2, frac=0.05):
    """Oracle's final error within 5% of a tolerance (success not decidable in FP32)."""
    pe, re = ora_res["pos_err"][p], ora_res["rot_err"][p]
    return bool(np.any(np.abs(pe - tol_pos) <= frac * tol_pos) or
                np.any(np.abs(re - tol_rot) <= frac * tol_rot))

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


def fp32_fragile(tree, tg, w, o, seed, ora, t, rel_tie=1e-5, eps_step=1e-6):
    """Whether the oracle's accept decision at iteration t (1-based) is one
    FP32 cannot settle.  Replays the oracle to the state before iteration t
    (its trace and lambda schedule), forms the damped system there in FP64 and
    compares |c' - c| with rel_tie * c plus the first-order change of c' that
    a relative step error of eps_step * cond(A_lambda) causes; eps_step is the
    relative accuracy of an FP32-formed Jacobian (about 16 ulps)."""
    import oracle
    q = np.asarray(seed, dtype=np.float64) if t == 1 else ora["trace_q"][t - 2]
    lam = o["lambda0"]
    for i in range(t - 1):
        lam = max(lam / o["nu_down"], o["lambda_min"]) if ora["trace_acc"][i] else \
            min(lam * o["nu_up"], o["lambda_max"])
    r, _, _ = oracle.residual(tree, tg, w, q)
    J = oracle.jacobian(tree, tg, w, q)
    A = J.T @ J
    g = J.T @ r
    Al = A + lam * np.diag(np.maximum(np.diag(A), o["damping_floor"]))
    d = np.linalg.solve(Al, -g)
    c, ct = oracle.cost(tree, tg, w, q), oracle.cost(tree, tg, w, q + d)
    return bool(abs(ct - c) <= rel_tie * c + eps_step * np.linalg.cond(Al) * 2 * abs(g @ d))


def first_divergence(acc_gpu, acc_ora):
    """First iteration (1-based) at which two accept sequences differ, or 0."""
    n = min(len(acc_gpu), len(acc_ora))
    for i in range(n):
        if int(acc_gpu[i]) != int(acc_ora[i]):
            return i + 1
    return 0


def at_limit(tree, q, eps=1e-6):
    """Some joint within eps (relative to 1 + |limit|) of a limit: the limit
    residual's kink, where whether its Jacobian row is active (the strict
    test q > upper / q < lower) is decided by rounding (a Gauss-Newton step
    that projects a joint back onto its limit lands on it, just inside or just
    outside, depending on the last bits)."""
    q = np.asarray(q, dtype=np.float64)
    lo, hi = np.asarray(tree.lower), np.asarray(tree.upper)
    return bool(np.any(np.abs(q - lo) <= eps * (1 + np.abs(lo))) or
                np.any(np.abs(q - hi) <= eps * (1 + np.abs(hi))))


def compare_outcome(ctx, rid, tree, tg, seed, w, o, status, iters, ora, variant=0):
    """'same' when the GPU's success flag (and, if both converged, iteration
    count) equals the oracle's; 'excused' when the difference traces back to
    something FP32 cannot settle (a near-tie, a final or crossing error within
    5% of a tolerance, or a first differing decision that is FP32-fragile or
    taken from an iterate on a joint limit's kink); else 'bad'.  ora:
    oracle.lm_solve result with a full trace."""
    cg, co = (status & 0xff) == 0, (ora["status"] & 0xff) == 0
    if cg == co and (not cg or iters == ora["iters"]):
        return "same"
    if ora["trace_tie"].any() or borderline({"pos_err": [ora["pos_err"]], "rot_err": [ora["rot_err"]]}, 0):
        return "excused"
    if cg and co and borderline_at(tree, tg, w, ora["trace_q"], int(min(iters, ora["iters"]))):
        return "excused"
    kw = {"variant": variant} if variant else {}
    res = solve_gpu(ctx, rid, tree, tg[None], np.asarray(seed)[None], 1, w, o,
                    trace_iters=o["max_iters"], **kw)
    t = first_divergence(res["trace_accept"][0], ora["trace_acc"])
    if t == 0:
        return "bad"
    if fp32_fragile(tree, tg, w, o, seed, ora, t):
        return "excused"
    qg = np.asarray(seed) if t == 1 else res["trace_q"][0][t - 2]
    qo = np.asarray(seed) if t == 1 else ora["trace_q"][t - 2]
    return "excused" if at_limit(tree, qg) or at_limit(tree, qo) else "bad"


def borderline(ora_res, p, tol_pos=1e-3, tol_rot=1e-2, frac=0.05):
    """Oracle's final error within 5% of a tolerance (success not decidable in FP32)."""
    pe, re = ora_res["pos_err"][p], ora_res["rot_err"][p]
    return bool(np.any(np.abs(pe - tol_pos) <= frac * tol_pos) or
                np.any(np.abs(re - tol_rot) <= frac * tol_rot))

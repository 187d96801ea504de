"""FP64 CPU oracle for batched Levenberg-Marquardt IK (test infrastructure).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never loads it.

The arithmetic lives in ``oracle.c`` (plain C, double precision); this module
only marshals numpy arrays through ctypes.  ``build()`` compiles it with gcc.

Paper passages followed: Sec. III-A (LM on a sum of squared residuals),
Sec. III-B (FK over revolute joints), Sec. III-C (joint pose, joint limit and
joint regularisation costs, weighted).  Parity pins: see tests/test_oracle_*.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CONVERGED, MAX_ITERS, STALLED, NONFINITE = 0, 1, 2, 3
FLAG_FP64 = 0x100


def build(force: bool = True) -> str:
    """Compile liboracle.so next to the source (portable -O3, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _setup(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Tree(C.Structure):
    _fields_ = [("n", C.c_int), ("parent", _ip), ("mount_quat", _dp), ("offset", _dp),
                ("axis", _dp), ("lower", _dp), ("upper", _dp), ("m", C.c_int),
                ("ee_joint", _ip), ("ee_offset", _dp), ("ee_quat", _dp), ("ee_kind", _ip),
                ("joint_type", _ip), ("mimic_joint", _ip), ("mimic_mult", _dp),
                ("mimic_offset", _dp)]


class _Weights(C.Structure):
    _fields_ = [("w_pos", C.c_double), ("w_rot", C.c_double), ("w_limit", C.c_double),
                ("w_rest", C.c_double), ("q_rest", _dp)]


class _Options(C.Structure):
    _fields_ = [("max_iters", C.c_int), ("lambda0", C.c_double), ("nu_up", C.c_double),
                ("nu_down", C.c_double), ("lambda_min", C.c_double),
                ("lambda_max", C.c_double), ("early_exit", C.c_int),
                ("tol_pos", C.c_double), ("tol_rot", C.c_double),
                ("damping_floor", C.c_double), ("pivot_rel", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("cost", C.c_double), ("pose_cost", C.c_double), ("iters", C.c_int),
                ("accepts", C.c_int), ("status", C.c_int), ("iters_to_tol", C.c_int),
                ("flags", C.c_int)]


def _setup(L):
    P = C.POINTER
    sigs = {
        "ora_quat_to_R": [_dp, _dp],
        "ora_so3_exp": [_dp, _dp], "ora_so3_log": [_dp, _dp], "ora_so3_jl": [_dp, _dp],
        "ora_so3_jl_inv": [_dp, _dp], "ora_se3_Q": [_dp, _dp, _dp],
        "ora_se3_exp": [_dp, _dp, _dp], "ora_se3_log": [_dp, _dp, _dp],
        "ora_se3_jl_inv": [_dp, _dp], "ora_se3_jr_inv": [_dp, _dp],
        "ora_fk": [P(_Tree), _dp, _dp, _dp, _dp, _dp],
        "ora_fk_pose7": [P(_Tree), _dp, _dp],
        "ora_residual": [P(_Tree), _dp, P(_Weights), _dp, _dp, _dp, _dp],
        "ora_jacobian": [P(_Tree), _dp, P(_Weights), _dp, _dp],
        "ora_chol_solve": [C.c_int, _dp, _dp, _dp],
        "ora_lm_solve": [P(_Tree), _dp, P(_Weights), P(_Options), _dp, _dp, _dp, _dp,
                         P(_Result), C.c_int, _dp, _ip, _dp, _ip],
        "ora_lm_solve_batch": [P(_Tree), _dp, _dp, C.c_long, C.c_int, P(_Weights),
                               P(_Options), _dp, _dp, _dp, _dp, _dp, _ip, _ip, _ip, _ip,
                               C.c_int],
        "ora_best_of_k": [C.c_long, C.c_int, _ip, _dp, _dp, _ip, _ip],
        "ora_beam_select": [C.c_long, C.c_int, C.c_int, _ip, _dp, _dp, _ip],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = None
    L.ora_rows.argtypes = [P(_Tree)]
    L.ora_rows.restype = C.c_int
    L.ora_nvar.argtypes = [P(_Tree)]
    L.ora_nvar.restype = C.c_int
    L.ora_cost.argtypes = [P(_Tree), _dp, P(_Weights), _dp]
    L.ora_cost.restype = C.c_double
    L.ora_cholesky.argtypes = [C.c_int, _dp, _dp]
    L.ora_cholesky.restype = C.c_int
    L.ora_lm_step.argtypes = [P(_Tree), _dp, P(_Weights), P(_Options), _dp, C.c_double,
                              _dp, _ip]
    L.ora_lm_step.restype = C.c_int


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


class OTree:
    """ctypes view of a synth.Tree (keeps the arrays alive)."""

    def __init__(self, tree):
        self.n, self.m = tree.n, tree.m
        jt = getattr(tree, "joint_type", None)
        mj = getattr(tree, "mimic_joint", None)
        self.ee_kind = np.asarray(tree.ee_kind)
        self._keep = [_i(tree.parent), _d(tree.mount_quat), _d(tree.offset), _d(tree.axis),
                      _d(tree.lower), _d(tree.upper), _i(tree.ee_joint), _d(tree.ee_offset),
                      _d(tree.ee_quat), _i(tree.ee_kind), None if jt is None else _i(jt),
                      None if mj is None else _i(mj),
                      None if mj is None else _d(tree.mimic_multiplier),
                      None if mj is None else _d(tree.mimic_offset)]
        k = self._keep
        opt = lambda a, t: _p(a, t) if a is not None else None
        self.s = _Tree(self.n, _p(k[0], _ip), _p(k[1]), _p(k[2]), _p(k[3]), _p(k[4]), _p(k[5]),
                       self.m, _p(k[6], _ip), _p(k[7]), _p(k[8]), _p(k[9], _ip),
                       opt(k[10], _ip), opt(k[11], _ip), opt(k[12], _dp), opt(k[13], _dp))
        self.nv = lib().ora_nvar(self.s)

    @property
    def ref(self):
        return C.byref(self.s)


def _ot(tree):
    return tree if isinstance(tree, OTree) else OTree(tree)


def _weights(w, n):
    qr = w.get("q_rest")
    qr = _d(qr) if qr is not None else None
    s = _Weights(w["w_pos"], w["w_rot"], w["w_limit"], w["w_rest"], _p(qr))
    return s, qr


def _options(o):
    return _Options(int(o["max_iters"]), o["lambda0"], o["nu_up"], o["nu_down"],
                    o["lambda_min"], o["lambda_max"], int(bool(o["early_exit"])),
                    o["tol_pos"], o["tol_rot"], o["damping_floor"], o["pivot_rel"])


# ------------------------------------------------------------ Lie groups

def _v2m(fn, v):
    v = _d(v)
    out = np.zeros(9)
    getattr(lib(), fn)(_p(v), _p(out))
    return out.reshape(3, 3)


def quat_to_R(q):
    return _v2m("ora_quat_to_R", q)


def so3_exp(phi):
    return _v2m("ora_so3_exp", phi)


def so3_log(R):
    R = _d(R).reshape(9)
    out = np.zeros(3)
    lib().ora_so3_log(_p(R), _p(out))
    return out


def so3_jl(phi):
    return _v2m("ora_so3_jl", phi)


def so3_jl_inv(phi):
    return _v2m("ora_so3_jl_inv", phi)


def se3_Q(rho, phi):
    rho, phi = _d(rho), _d(phi)
    out = np.zeros(9)
    lib().ora_se3_Q(_p(rho), _p(phi), _p(out))
    return out.reshape(3, 3)


def se3_exp(xi):
    xi = _d(xi)
    R, t = np.zeros(9), np.zeros(3)
    lib().ora_se3_exp(_p(xi), _p(R), _p(t))
    return R.reshape(3, 3), t


def se3_log(R, t):
    R, t = _d(R).reshape(9), _d(t)
    xi = np.zeros(6)
    lib().ora_se3_log(_p(R), _p(t), _p(xi))
    return xi


def se3_jl_inv(xi):
    xi = _d(xi)
    out = np.zeros(36)
    lib().ora_se3_jl_inv(_p(xi), _p(out))
    return out.reshape(6, 6)


def se3_jr_inv(xi):
    xi = _d(xi)
    out = np.zeros(36)
    lib().ora_se3_jr_inv(_p(xi), _p(out))
    return out.reshape(6, 6)


# ------------------------------------------------------------ kinematics

def fk(tree, q):
    """Returns (R[n,3,3], p[n,3], R_ee[m,3,3], p_ee[m,3])."""
    t = _ot(tree)
    q = _d(q)
    R, p = np.zeros((t.n, 9)), np.zeros((t.n, 3))
    Re, pe = np.zeros((t.m, 9)), np.zeros((t.m, 3))
    lib().ora_fk(t.ref, _p(q), _p(R), _p(p), _p(Re), _p(pe))
    return R.reshape(-1, 3, 3), p, Re.reshape(-1, 3, 3), pe


def fk_pose7(tree, q):
    """EE poses [m,7] = (p, quat wxyz with w >= 0)."""
    t = _ot(tree)
    q = _d(q)
    out = np.zeros((t.m, 7))
    lib().ora_fk_pose7(t.ref, _p(q), _p(out))
    return out


def targets_from(tree, Q, round_f32=True):
    """Targets [T, m, 7] = FK(Q[t]); rounded to FP32 (then promoted) by default."""
    t = _ot(tree)
    Q = _d(Q)
    out = np.zeros((Q.shape[0], t.m, 7))
    for i in range(Q.shape[0]):
        lib().ora_fk_pose7(t.ref, _p(Q[i]), _p(out[i]))
    if round_f32:
        out = out.astype(np.float32).astype(np.float64)
    return out


def n_rows(tree):
    return lib().ora_rows(_ot(tree).ref)


def residual(tree, targets, w, q):
    t = _ot(tree)
    tg, q = _d(targets), _d(q)
    r = np.zeros(n_rows(t))
    pe, re = np.zeros(t.m), np.zeros(t.m)
    ws, _k = _weights(w, t.nv)
    lib().ora_residual(t.ref, _p(tg), C.byref(ws), _p(q), _p(r), _p(pe), _p(re))
    return r, pe, re


def jacobian(tree, targets, w, q):
    t = _ot(tree)
    tg, q = _d(targets), _d(q)
    J = np.zeros((n_rows(t), t.nv))
    ws, _k = _weights(w, t.nv)
    lib().ora_jacobian(t.ref, _p(tg), C.byref(ws), _p(q), _p(J))
    return J


def cost(tree, targets, w, q):
    t = _ot(tree)
    tg, q = _d(targets), _d(q)
    ws, _k = _weights(w, t.nv)
    return lib().ora_cost(t.ref, _p(tg), C.byref(ws), _p(q))


# --------------------------------------------------------- linear algebra

def cholesky(A):
    """Returns (L lower, ok, min pivot ratio)."""
    A = _d(A).copy()
    n = A.shape[0]
    mr = C.c_double()
    ok = lib().ora_cholesky(n, _p(A), C.byref(mr))
    return np.tril(A), bool(ok), mr.value


def chol_solve(L, b):
    L, b = _d(L), _d(b)
    x = np.zeros_like(b)
    lib().ora_chol_solve(L.shape[0], _p(L), _p(b), _p(x))
    return x


def lm_step(tree, targets, w, o, q, lam):
    t = _ot(tree)
    tg, q = _d(targets), _d(q)
    ws, _k = _weights(w, t.nv)
    os_ = _options(o)
    d = np.zeros(t.nv)
    fb = C.c_int()
    ok = lib().ora_lm_step(t.ref, _p(tg), C.byref(ws), C.byref(os_), _p(q), lam, _p(d),
                           C.byref(fb))
    return d, bool(ok), bool(fb.value)


# ------------------------------------------------------------------- LM

def lm_solve(tree, targets, w, o, q0, n_trace=0):
    """One problem.  targets [m,7].  Returns a dict (q, errors, counters, trace)."""
    t = _ot(tree)
    tg, q0 = _d(targets), _d(q0)
    ws, _k = _weights(w, t.nv)
    os_ = _options(o)
    q = np.zeros(t.nv)
    pe, re = np.zeros(t.m), np.zeros(t.m)
    res = _Result()
    nt = max(int(n_trace), 0)
    tq = np.zeros((max(nt, 1), t.nv))
    ta = np.zeros(max(nt, 1), np.int32)
    tc = np.zeros(max(nt, 1))
    tt = np.zeros(max(nt, 1), np.int32)
    lib().ora_lm_solve(t.ref, _p(tg), C.byref(ws), C.byref(os_), _p(q0), _p(q), _p(pe),
                       _p(re), C.byref(res), nt, _p(tq), _p(ta, _ip), _p(tc), _p(tt, _ip))
    return {"q": q, "pos_err": pe, "rot_err": re, "cost": res.cost,
            "pose_cost": res.pose_cost, "iters": res.iters, "accepts": res.accepts,
            "status": res.status, "iters_to_tol": res.iters_to_tol, "flags": res.flags,
            "trace_q": tq[:nt], "trace_acc": ta[:nt], "trace_cost": tc[:nt],
            "trace_tie": tt[:nt]}


def lm_solve_batch(tree, targets, seeds, K, w, o, threads=None):
    """targets [T,m,7], seeds [T*K, n]; problem p uses target p // K."""
    t = _ot(tree)
    tg, sd = _d(targets), _d(seeds)
    N = sd.shape[0]
    ws, _k = _weights(w, t.nv)
    os_ = _options(o)
    q = np.zeros((N, t.nv))
    pe, re = np.zeros((N, t.m)), np.zeros((N, t.m))
    c, pc = np.zeros(N), np.zeros(N)
    it, ac, st, itt = (np.zeros(N, np.int32) for _ in range(4))
    threads = threads or os.cpu_count() or 1
    lib().ora_lm_solve_batch(t.ref, _p(tg), _p(sd), N, int(K), C.byref(ws), C.byref(os_),
                             _p(q), _p(pe), _p(re), _p(c), _p(pc), _p(it, _ip), _p(ac, _ip),
                             _p(st, _ip), _p(itt, _ip), int(threads))
    return {"q": q, "pos_err": pe, "rot_err": re, "cost": c, "pose_cost": pc, "iters": it,
            "accepts": ac, "status": st, "iters_to_tol": itt}


def best_of_k(status, cost, pose_cost, K):
    st = _i(status)
    c, pc = _d(cost), _d(pose_cost)
    T = st.shape[0] // K
    best, succ = np.zeros(T, np.int32), np.zeros(T, np.int32)
    lib().ora_best_of_k(T, int(K), _p(st, _ip), _p(c), _p(pc), _p(best, _ip), _p(succ, _ip))
    return best, succ.astype(bool)


def beam_select(status, cost, pose_cost, K, keep):
    """IK-Beam survivors (Sec. V-C): per target the ``keep`` best of its K
    seeds, best first, as seed indices [T, keep].  Order: within tolerance
    before not; then total cost (within) or pose-only cost (not), NaN last;
    then the lower index."""
    st = _i(status)
    c, pc = _d(cost), _d(pose_cost)
    T = st.shape[0] // K
    kept = np.zeros((T, keep), np.int32)
    lib().ora_beam_select(T, int(K), int(keep), _p(st, _ip), _p(c), _p(pc), _p(kept, _ip))
    return kept


def ik_beam(tree, targets, seeds, K0, iters0, keep, iters1, w, o, threads=None):
    """IK-Beam (Sec. V-C) in FP64.  targets [T,m,7], seeds [T*K0, n].

    Stage 0: LM from every seed for ``iters0`` iterations.  The ``keep``
    survivors per target (``beam_select``) restart LM, lambda back at its
    initial value, from their stage-0 joints for ``iters1`` iterations.  The
    first of the survivors' results in the same order is returned.
    Returns the stage results, the survivors and, per target, the chosen
    seed's index (0..K0-1), joints and success flag.
    """
    o0, o1 = dict(o), dict(o)
    o0["max_iters"], o1["max_iters"] = int(iters0), int(iters1)
    s0 = lm_solve_batch(tree, targets, seeds, K0, w, o0, threads)
    kept = beam_select(s0["status"], s0["cost"], s0["pose_cost"], K0, keep)
    T = kept.shape[0]
    rows = (np.arange(T)[:, None] * K0 + kept).reshape(-1)
    s1 = lm_solve_batch(tree, targets, s0["q"][rows], keep, w, o1, threads)
    pick = beam_select(s1["status"], s1["cost"], s1["pose_cost"], keep, 1)[:, 0]
    win = np.arange(T) * keep + pick
    return {"stage0": s0, "kept": kept, "seeds1": s0["q"][rows], "stage1": s1, "pick": pick,
            "best_index": kept[np.arange(T), pick], "best_q": s1["q"][win],
            "success": (s1["status"][win] & 0xFF) == CONVERGED,
            "pos_err": s1["pos_err"][win], "rot_err": s1["rot_err"][win],
            "cost": s1["cost"][win]}

"""Batched Levenberg-Marquardt inverse kinematics on AMD MI355X (gfx950).

Thin ctypes binding over ``libpkmi.so`` (C ABI in ``include/pkmi.h``).  It
only marshals arguments: every step of the solve runs in the library's HIP
kernels.  PyTorch tensors provide device memory and the stream.  There is no
CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["Context", "Seeder", "Weights", "Options", "lib", "LibraryMissing", "PkError",
           "CONVERGED", "MAX_ITERS", "STALLED", "NONFINITE", "FLAG_FP64",
           "EE_POSE", "EE_POSITION", "VARIANT_AUTO", "VARIANT_LANE", "VARIANT_WAVE", "VARIANT_WAVE_JOINT",
           "pack_targets", "target_floats"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpkmi.so")

CONVERGED, MAX_ITERS, STALLED, NONFINITE, TARGET_SOLVED = 0, 1, 2, 3, 4
JOINT_REVOLUTE, JOINT_PRISMATIC, JOINT_FIXED = 0, 1, 2
FLAG_FP64 = 0x100
NOALLOC_MAX_PROBLEMS = 1 << 20      # problems per pk_ik_solve_noalloc call (include/pkmi.h)
EE_POSE, EE_POSITION = 0, 1
VARIANT_AUTO, VARIANT_LANE, VARIANT_WAVE, VARIANT_WAVE_JOINT = 0, 1, 2, 3
SCHED_SINGLE, SCHED_PER_GROUP = 0, 1


class LibraryMissing(RuntimeError):
    pass


class PkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pkmi error {code}: {msg}")
        self.code = code


_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class _Tree(C.Structure):
    _fields_ = [("n_joints", C.c_int32), ("parent", _i32p), ("mount_quat", _f64p),
                ("offset", _f64p), ("axis", _f64p), ("lower", _f64p), ("upper", _f64p),
                ("n_ee", C.c_int32), ("ee_joint", _i32p), ("ee_offset", _f64p),
                ("ee_quat", _f64p), ("ee_kind", _i32p), ("joint_type", _i32p),
                ("mimic_joint", _i32p), ("mimic_multiplier", _f64p), ("mimic_offset", _f64p)]


class _Weights(C.Structure):
    _fields_ = [("w_pos", C.c_float), ("w_rot", C.c_float), ("w_limit", C.c_float),
                ("w_rest", C.c_float), ("q_rest", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("lambda0", C.c_float), ("nu_up", C.c_float),
                ("nu_down", C.c_float), ("lambda_min", C.c_float), ("lambda_max", C.c_float),
                ("early_exit", C.c_int32), ("tol_pos", C.c_float), ("tol_rot", C.c_float),
                ("damping_floor", C.c_float), ("pivot_rel", C.c_float), ("variant", C.c_int32),
                ("target_exit", C.c_int32)]


class _Problem(C.Structure):
    _fields_ = [("n_targets", C.c_int64), ("K", C.c_int32), ("targets", C.c_void_p),
                ("seeds", C.c_void_p)]


class _Outputs(C.Structure):
    _fields_ = [("joints", C.c_void_p), ("pos_err", C.c_void_p), ("rot_err", C.c_void_p),
                ("cost", C.c_void_p), ("iters", C.c_void_p), ("accepts", C.c_void_p),
                ("status", C.c_void_p), ("iters_to_tol", C.c_void_p),
                ("best_index", C.c_void_p), ("best_joints", C.c_void_p),
                ("target_success", C.c_void_p), ("trace_iters", C.c_int32),
                ("trace_q", C.c_void_p), ("trace_accept", C.c_void_p), ("pose_cost", C.c_void_p)]


class _SeededOptions(C.Structure):
    _fields_ = [("seeder_id", C.c_int32), ("fallback_K", C.c_int32), ("fallback_seeds", C.c_void_p),
                ("refine", _Options), ("fallback", _Options), ("refine_iters_per_launch", C.c_int32),
                ("refine_blocks_per_cu", C.c_int32), ("restart_iters", C.c_int32),
                ("persist_waves_per_cu", C.c_int32), ("fallback_chunk", C.c_int32)]


class _SeededOutputs(C.Structure):
    _fields_ = [("best_joints", C.c_void_p), ("target_success", C.c_void_p),
                ("source", C.c_void_p), ("iters_to_tol", C.c_void_p),
                ("refine_iters", C.c_void_p), ("refine_accepts", C.c_void_p),
                ("fallback_iters", C.c_void_p), ("fallback_accepts", C.c_void_p),
                ("n_fallback", C.c_void_p), ("restart_iters", C.c_void_p),
                ("restart_accepts", C.c_void_p), ("n_restart", C.c_void_p),
                ("n_fallback_problems", C.c_void_p)]


class _BeamSchedule(C.Structure):
    _fields_ = [("n_seeds", C.c_int32), ("iters0", C.c_int32), ("keep", C.c_int32),
                ("iters1", C.c_int32)]


_BEAM_OUT = ["best_joints", "best_index", "target_success", "pos_err", "rot_err", "cost",
             "stage0_joints", "stage0_cost", "stage0_pose_cost", "stage0_status", "kept",
             "stage1_joints", "stage1_cost", "stage1_pose_cost", "stage1_status"]


class _BeamOutputs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in _BEAM_OUT]


class _TrajProblem(C.Structure):
    _fields_ = [("B", C.c_int64), ("T", C.c_int32), ("start", C.c_void_p), ("goal", C.c_void_p),
                ("init", C.c_void_p)]


class _TrajCosts(C.Structure):
    _fields_ = [(k, C.c_float) for k in ["dt", "w_pos", "w_rot", "w_limit", "w_smooth", "w_vel",
                                         "w_acc", "w_jerk"]] + [("vmax", C.c_void_p)]


_TRAJ_OUT = ["traj", "cost", "iters", "accepts", "status", "pos_err", "rot_err"]


class _TrajOutputs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in _TRAJ_OUT]


class _Group(C.Structure):
    _fields_ = [("robot_id", C.c_int32), ("problem", _Problem), ("weights", _Weights),
                ("out", _Outputs)]


MAX_GROUPS = 16


class _Sched(C.Structure):
    _fields_ = [("iters_per_launch", C.c_int32), ("waves_per_cu", C.c_int32),
                ("use_graph", C.c_int32), ("workgroup_size", C.c_int32), ("mode", C.c_int32),
                ("variant", C.c_int32 * MAX_GROUPS)]


_lib = None


def lib():
    """Load libpkmi.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.pk_create.argtypes = [C.POINTER(vp), C.c_int]
        L.pk_destroy.argtypes = [vp]
        L.pk_last_error.argtypes = [vp]
        L.pk_last_error.restype = C.c_char_p
        L.pk_robot_upload.argtypes = [vp, C.POINTER(_Tree), C.POINTER(i32)]
        L.pk_robot_info.argtypes = [vp, i32] + [C.POINTER(i32)] * 6
        L.pk_fk.argtypes = [vp, i32, i64, vp, vp, vp, vp]
        L.pk_residual_jacobian.argtypes = [vp, i32, i64, i32, vp, vp, C.POINTER(_Weights), vp,
                                           vp, vp]
        L.pk_ik_solve.argtypes = [vp, i32, C.POINTER(_Problem), C.POINTER(_Weights),
                                  C.POINTER(_Options), C.POINTER(_Outputs), vp]
        L.pk_ik_solve_noalloc.argtypes = L.pk_ik_solve.argtypes
        fp = C.POINTER(C.c_float)
        L.pk_seeder_create.argtypes = [vp, i32, i32, i32, i32, fp, i64, C.POINTER(i32)]
        L.pk_seeder_param_count.argtypes = [vp, i32, C.POINTER(i64)]
        L.pk_seeder_get.argtypes = [vp, i32, i32, fp, i64]
        L.pk_seeder_forward.argtypes = [vp, i32, vp, i64, vp, vp]
        L.pk_seeder_forward_layers.argtypes = [vp, i32, vp, i64, vp, vp]
        L.pk_seeder_grad.argtypes = [vp, i32, vp, vp, i64, vp, vp]
        L.pk_seeder_train.argtypes = [vp, i32, vp, i64, i32, i32, C.c_float, vp, vp, vp]
        L.pk_seeder_infer.argtypes = [vp, i32, vp, i64, vp, vp]
        L.pk_seeder_save.argtypes = [vp, i32, C.c_char_p]
        L.pk_seeder_load.argtypes = [vp, i32, C.c_char_p]
        L.pk_ik_solve_seeded.argtypes = [vp, i32, i64, vp, C.POINTER(_Weights),
                                         C.POINTER(_SeededOptions), C.POINTER(_SeededOutputs), vp]
        L.pk_ik_solve_mixed.argtypes = [vp, i32, C.POINTER(_Group), C.POINTER(_Options),
                                        C.POINTER(_Sched), vp]
        L.pk_autotune_mixed.argtypes = [vp, i32, C.POINTER(_Group), C.POINTER(_Options),
                                        C.POINTER(_Sched), C.POINTER(C.c_float), vp]
        L.pk_autotune_save.argtypes = [vp, C.c_char_p]
        L.pk_autotune_load.argtypes = [vp, C.c_char_p, C.POINTER(i32)]
        L.pk_autotune_lookup.argtypes = [vp, i32, C.POINTER(_Group), C.POINTER(_Options),
                                         C.POINTER(_Sched), C.POINTER(C.c_float)]
        L.pk_ik_beam.argtypes = [vp, i32, i64, vp, vp, C.POINTER(_Weights), C.POINTER(_Options),
                                 C.POINTER(_BeamSchedule), C.POINTER(_BeamOutputs), vp]
        L.pk_traj_solve.argtypes = [vp, i32, C.POINTER(_TrajProblem), C.POINTER(_TrajCosts),
                                    C.POINTER(_Options), C.POINTER(_TrajOutputs), vp]
        for f in ["pk_create", "pk_destroy", "pk_robot_upload", "pk_robot_info", "pk_fk",
                  "pk_residual_jacobian", "pk_ik_solve", "pk_seeder_create",
                  "pk_seeder_param_count", "pk_seeder_get", "pk_seeder_forward",
                  "pk_seeder_forward_layers", "pk_seeder_grad", "pk_seeder_train",
                  "pk_seeder_infer", "pk_seeder_save",
                  "pk_seeder_load", "pk_ik_solve_seeded", "pk_ik_solve_mixed",
                  "pk_autotune_mixed", "pk_autotune_save", "pk_autotune_load",
                  "pk_autotune_lookup", "pk_ik_solve_noalloc", "pk_ik_beam", "pk_traj_solve"]:
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def exported_symbols():
    """Names of the C entry points this binding expects the library to export."""
    return ["pk_create", "pk_destroy", "pk_last_error", "pk_robot_upload", "pk_robot_info",
            "pk_fk", "pk_residual_jacobian", "pk_ik_solve", "pk_seeder_create",
            "pk_seeder_param_count", "pk_seeder_get", "pk_seeder_forward",
            "pk_seeder_forward_layers", "pk_seeder_grad",
            "pk_seeder_train", "pk_seeder_infer", "pk_seeder_save", "pk_seeder_load",
            "pk_ik_solve_seeded", "pk_ik_solve_mixed", "pk_autotune_mixed", "pk_autotune_save",
            "pk_autotune_load", "pk_autotune_lookup", "pk_ik_solve_noalloc", "pk_ik_beam",
            "pk_traj_solve"]


class Weights:
    def __init__(self, w_pos=1.0, w_rot=0.5, w_limit=10.0, w_rest=0.0, q_rest=None):
        self.w_pos, self.w_rot, self.w_limit, self.w_rest = w_pos, w_rot, w_limit, w_rest
        self.q_rest = q_rest          # device tensor [n] or None

    @classmethod
    def from_dict(cls, d):
        return cls(d["w_pos"], d["w_rot"], d["w_limit"], d["w_rest"], d.get("q_rest"))

    def _c(self):
        qr = self.q_rest
        return _Weights(self.w_pos, self.w_rot, self.w_limit, self.w_rest,
                        qr.data_ptr() if qr is not None else None)


class Options:
    def __init__(self, max_iters=30, lambda0=1e-3, nu_up=10.0, nu_down=10.0, lambda_min=1e-10,
                 lambda_max=1e10, early_exit=False, tol_pos=1e-3, tol_rot=1e-2,
                 damping_floor=1e-6, pivot_rel=1e-6, variant=VARIANT_AUTO, target_exit=False):
        self.__dict__.update(locals())
        del self.__dict__["self"]

    @classmethod
    def from_dict(cls, d, **kw):
        o = cls(**{k: d[k] for k in ["max_iters", "lambda0", "nu_up", "nu_down", "lambda_min",
                                     "lambda_max", "early_exit", "tol_pos", "tol_rot",
                                     "damping_floor", "pivot_rel"]})
        o.__dict__.update(kw)
        return o

    def _c(self):
        return _Options(int(self.max_iters), self.lambda0, self.nu_up, self.nu_down,
                        self.lambda_min, self.lambda_max, int(bool(self.early_exit)),
                        self.tol_pos, self.tol_rot, self.damping_floor, self.pivot_rel,
                        int(self.variant), int(bool(self.target_exit)))


def target_floats(ee_kind) -> int:
    return int(sum(7 if k == EE_POSE else 3 for k in ee_kind))


def pack_targets(ee_kind, targets) -> np.ndarray:
    """[T, m, 7] (p, quat) -> the library's SoA plane layout [sum(widths), T] (float32)."""
    targets = np.asarray(targets)
    T = targets.shape[0]
    planes = []
    for k, kind in enumerate(ee_kind):
        w = 7 if kind == EE_POSE else 3
        planes.append(targets[:, k, :w].T)
    return np.ascontiguousarray(np.concatenate(planes, 0).astype(np.float32)).reshape(-1, T)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check(t, name, shape, dtype="float32", device=None):
    """Raises PkError (PK_EINVAL) unless ``t`` is a contiguous tensor of
    ``dtype`` and ``shape`` (None entries match any size) on ``device``: the
    kernels index these buffers by the sizes the call passes, so a mismatch
    would read or write past them."""
    import torch
    want = getattr(torch, dtype)
    if not isinstance(t, torch.Tensor):
        raise PkError(-1, f"{name}: expected a tensor")
    if t.dtype != want:
        raise PkError(-1, f"{name}: dtype {t.dtype}, expected {want}")
    if device is not None and t.device != device:
        raise PkError(-1, f"{name}: on {t.device}, expected {device}")
    if t.device.type != "cuda":
        raise PkError(-1, f"{name}: must be a device tensor")
    if not t.is_contiguous():
        raise PkError(-1, f"{name}: must be contiguous")
    if len(t.shape) != len(shape) or any(w is not None and int(a) != int(w)
                                         for a, w in zip(t.shape, shape)):
        raise PkError(-1, f"{name}: shape {tuple(t.shape)}, expected "
                          f"{tuple('*' if w is None else w for w in shape)}")


class Context:
    """One library context on one HIP device."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.device = device
        self._h = C.c_void_p()
        self._call(lib().pk_create(C.byref(self._h), device), ctx=False)
        self._trees = {}

    def _call(self, rc, ctx=True):
        if rc != 0:
            msg = lib().pk_last_error(self._h if ctx else None)
            raise PkError(rc, msg.decode() if msg else "")

    def close(self):
        if self._h:
            lib().pk_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream(self):
        return C.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)

    # ------------------------------------------------------------- robots
    def upload(self, tree) -> int:
        """tree: object with parent, mount_quat, offset, axis, lower, upper, ee_joint,
        ee_offset, ee_quat, ee_kind arrays and optionally joint_type (None = all
        revolute) and mimic_joint / mimic_multiplier / mimic_offset (see
        include/pkmi.h)."""
        d = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        jt = getattr(tree, "joint_type", None)
        mj = getattr(tree, "mimic_joint", None)
        keep = [i(tree.parent), d(tree.mount_quat), d(tree.offset), d(tree.axis), d(tree.lower),
                d(tree.upper), i(tree.ee_joint), d(tree.ee_offset), d(tree.ee_quat),
                i(tree.ee_kind), None if jt is None else i(jt), None if mj is None else i(mj),
                None if mj is None else d(tree.mimic_multiplier),
                None if mj is None else d(tree.mimic_offset)]
        pi = lambda a: a.ctypes.data_as(_i32p) if a is not None else None
        pd = lambda a: a.ctypes.data_as(_f64p) if a is not None else None
        t = _Tree(len(keep[0]), pi(keep[0]), pd(keep[1]), pd(keep[2]), pd(keep[3]), pd(keep[4]),
                  pd(keep[5]), len(keep[6]), pi(keep[6]), pd(keep[7]), pd(keep[8]), pi(keep[9]),
                  pi(keep[10]), pi(keep[11]), pd(keep[12]), pd(keep[13]))
        rid = C.c_int32()
        self._call(lib().pk_robot_upload(self._h, C.byref(t), C.byref(rid)))
        self._trees[rid.value] = keep
        return rid.value

    def robot_info(self, rid):
        v = [C.c_int32() for _ in range(6)]
        self._call(lib().pk_robot_info(self._h, rid, *[C.byref(x) for x in v]))
        return dict(zip(["n", "m", "target_floats", "rows", "chains", "chain_len"],
                        [x.value for x in v]))

    # ---------------------------------------------------------------- FK
    def fk(self, rid, q, frames=False):
        """q: cuda float32 [n, N] -> ee_pose [m, 7, N] (and joint frames [n, 12, N])."""
        torch = self._torch
        info = self.robot_info(rid)
        N = q.shape[1]
        ee = torch.empty((info["m"], 7, N), dtype=torch.float32, device=q.device)
        fr = torch.empty((info["n"], 12, N), dtype=torch.float32, device=q.device) if frames else None
        self._call(lib().pk_fk(self._h, rid, N, _ptr(q), _ptr(ee), _ptr(fr), self.stream()))
        return (ee, fr) if frames else ee

    def residual_jacobian(self, rid, targets, q, K, weights: Weights, jac=True):
        """targets [tf, T], q [n, N] -> r [rows, N], J [rows, n, N]."""
        torch = self._torch
        info = self.robot_info(rid)
        N = q.shape[1]
        r = torch.empty((info["rows"], N), dtype=torch.float32, device=q.device)
        J = torch.empty((info["rows"], info["n"], N), dtype=torch.float32, device=q.device) if jac else None
        w = weights._c()
        self._call(lib().pk_residual_jacobian(self._h, rid, N, K, _ptr(targets), _ptr(q),
                                              C.byref(w), _ptr(r), _ptr(J), self.stream()))
        return r, J

    # ---------------------------------------------------------------- IK
    def alloc_outputs(self, rid, T, K, best=False, trace_iters=0, full=True):
        torch = self._torch
        info = self.robot_info(rid)
        n, m, N = info["n"], info["m"], T * K
        dev = f"cuda:{self.device}"
        f = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
        i = lambda *s: torch.empty(s, dtype=torch.int32, device=dev)
        out = {"joints": f(n, N)}
        if full:
            out.update(pos_err=f(m, N), rot_err=f(m, N), cost=f(N), iters=i(N), accepts=i(N),
                       status=i(N), iters_to_tol=i(N), pose_cost=f(N))
        if best:
            out.update(best_index=i(T), best_joints=f(n, T), target_success=i(T))
        if trace_iters:
            out.update(trace_q=f(trace_iters, n, N), trace_accept=i(trace_iters, N))
        out["_trace_iters"] = trace_iters
        return out

    def ik_solve_seeded(self, rid, targets, seeder, weights: Weights, refine: Options,
                        fallback: Options = None, fallback_seeds=None, fallback_K=0,
                        counters=False, refine_iters_per_launch=0, refine_blocks_per_cu=0,
                        restart_iters=0, persist_waves_per_cu=0, fallback_chunk=0):
        """Learned seeds + LM, an optional restart of the unsolved targets' problems
        from their refined joints, fallback to random-seed LM, all at once or in
        stages of fallback_chunk seeds (see include/pkmi.h).

        Returns a dict of device tensors: best_joints [n, T], target_success,
        source, iters_to_tol [T], n_fallback, n_restart, n_fallback_problems [1]
        (and the LM counters)."""
        torch = self._torch
        T = targets.shape[1]
        info = self.robot_info(rid)
        dev = targets.device
        K = seeder.K
        _check(targets, "targets", (info["target_floats"], T))
        if fallback_K:
            _check(fallback_seeds, "fallback_seeds", (info["n"], T * int(fallback_K)), device=dev)
        i = lambda *s: torch.empty(s, dtype=torch.int32, device=dev)
        out = {"best_joints": torch.empty((info["n"], T), dtype=torch.float32, device=dev),
               "target_success": i(T), "source": i(T), "iters_to_tol": i(T), "n_fallback": i(1),
               "n_restart": i(1), "n_fallback_problems": i(1)}
        if counters:
            out.update(refine_iters=i(T * K), refine_accepts=i(T * K),
                       fallback_iters=i(max(T * fallback_K, 1)),
                       fallback_accepts=i(max(T * fallback_K, 1)),
                       restart_iters=i(T * K), restart_accepts=i(T * K))
        fb = fallback or refine
        so = _SeededOptions(seeder.id, int(fallback_K), _ptr(fallback_seeds), refine._c(), fb._c(),
                            int(refine_iters_per_launch), int(refine_blocks_per_cu), int(restart_iters),
                            int(persist_waves_per_cu), int(fallback_chunk))
        oo = _SeededOutputs(*[_ptr(out.get(k)) for k in ["best_joints", "target_success", "source",
                                                          "iters_to_tol", "refine_iters",
                                                          "refine_accepts", "fallback_iters",
                                                          "fallback_accepts", "n_fallback",
                                                          "restart_iters", "restart_accepts",
                                                          "n_restart", "n_fallback_problems"]])
        w = weights._c()
        self._call(lib().pk_ik_solve_seeded(self._h, rid, T, _ptr(targets), C.byref(w), C.byref(so),
                                            C.byref(oo), self.stream()))
        return out

    @staticmethod
    def _check_ik(info, targets, seeds, T, K, out=None):
        """Shapes, dtypes and device of a batch and its outputs (as in
        alloc_outputs) against the robot's sizes."""
        n, m, N = info["n"], info["m"], T * K
        dev = targets.device
        _check(targets, "targets", (info["target_floats"], T))
        _check(seeds, "seeds", (n, N), device=dev)
        if out is None:
            return
        tr = int(out.get("_trace_iters", 0))
        shapes = {"joints": ((n, N), "float32"), "pos_err": ((m, N), "float32"),
                  "rot_err": ((m, N), "float32"), "cost": ((N,), "float32"),
                  "iters": ((N,), "int32"), "accepts": ((N,), "int32"), "status": ((N,), "int32"),
                  "iters_to_tol": ((N,), "int32"), "best_index": ((T,), "int32"),
                  "best_joints": ((n, T), "float32"), "target_success": ((T,), "int32"),
                  "trace_q": ((tr, n, N), "float32"), "trace_accept": ((tr, N), "int32"),
                  "pose_cost": ((N,), "float32")}
        for k, (shp, dt) in shapes.items():
            if out.get(k) is not None:
                _check(out[k], k, shp, dt, device=dev)

    @staticmethod
    def _outputs_c(out):
        return _Outputs(*[_ptr(out.get(k)) for k in ["joints", "pos_err", "rot_err", "cost", "iters",
                                                      "accepts", "status", "iters_to_tol",
                                                      "best_index", "best_joints",
                                                      "target_success"]],
                        int(out.get("_trace_iters", 0)), _ptr(out.get("trace_q")),
                        _ptr(out.get("trace_accept")), _ptr(out.get("pose_cost")))

    def _groups_c(self, groups):
        arr = (_Group * len(groups))()
        for i, g in enumerate(groups):
            T = g["targets"].shape[1]
            self._check_ik(self.robot_info(g["rid"]), g["targets"], g["seeds"], T, g["K"], g["out"])
            arr[i] = _Group(g["rid"], _Problem(T, g["K"], _ptr(g["targets"]), _ptr(g["seeds"])),
                            g["weights"]._c(), self._outputs_c(g["out"]))
        return arr

    def ik_solve_mixed(self, groups, options: Options, iters_per_launch=0, waves_per_cu=0,
                       use_graph=True, variants=None, workgroup_size=0, mode=None):
        """groups: list of dicts rid, targets [tf, T], seeds [n, T*K], K, weights, out
        (from alloc_outputs).  variants: per group VARIANT_LANE / VARIANT_WAVE (None =
        the options' choice).  mode: SCHED_SINGLE (one persistent launch per round over
        every group, the default) or SCHED_PER_GROUP.  Zero k and waves_per_cu pick the
        autotuned entry."""
        arr = self._groups_c(groups)
        v = (C.c_int32 * MAX_GROUPS)(*(list(variants or []) + [0] * MAX_GROUPS)[:MAX_GROUPS])
        sch = _Sched(iters_per_launch, waves_per_cu, 1 if use_graph else 0, workgroup_size,
                     SCHED_SINGLE if mode is None else mode, v)
        o = options._c()
        self._call(lib().pk_ik_solve_mixed(self._h, len(groups), arr, C.byref(o), C.byref(sch),
                                           self.stream()))
        return groups

    @staticmethod
    def _sched_dict(sch, n, ms):
        return {"mode": sch.mode, "k": sch.iters_per_launch, "waves_per_cu": sch.waves_per_cu,
                "workgroup_size": sch.workgroup_size, "variants": list(sch.variant)[:n], "ms": ms}

    def autotune_mixed(self, groups, options: Options):
        """Times the candidate schedules on these groups; returns the fastest as a
        dict: k, waves_per_cu, workgroup_size, variants (per group), ms."""
        arr = self._groups_c(groups)
        sch = _Sched()
        ms = C.c_float()
        o = options._c()
        self._call(lib().pk_autotune_mixed(self._h, len(groups), arr, C.byref(o), C.byref(sch),
                                           C.byref(ms), self.stream()))
        return self._sched_dict(sch, len(groups), ms.value)

    def autotune_lookup(self, groups, options: Options):
        """The autotune table's entry for this batch (dict as autotune_mixed), or None."""
        arr = self._groups_c(groups)
        sch = _Sched()
        ms = C.c_float()
        o = options._c()
        rc = lib().pk_autotune_lookup(self._h, len(groups), arr, C.byref(o), C.byref(sch), C.byref(ms))
        if rc == -5:
            return None
        self._call(rc)
        return self._sched_dict(sch, len(groups), ms.value)

    def autotune_save(self, path):
        self._call(lib().pk_autotune_save(self._h, os.fsencode(path)))

    def autotune_load(self, path):
        """Reads a table written by autotune_save; returns the number of entries."""
        n = C.c_int32()
        self._call(lib().pk_autotune_load(self._h, os.fsencode(path), C.byref(n)))
        return n.value

    def alloc_beam_outputs(self, rid, T, n_seeds=64, keep=4, stages=False, device=None):
        """Device tensors for ik_beam: best_joints [n, T], best_index,
        target_success [T], pos_err / rot_err [m, T], cost [T] and, with
        ``stages``, the stage-0 / stage-1 per-problem results and ``kept``
        [T, keep]."""
        torch = self._torch
        info = self.robot_info(rid)
        n, m = info["n"], info["m"]
        dev = device or f"cuda:{self.device}"
        f = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
        i = lambda *s: torch.empty(s, dtype=torch.int32, device=dev)
        out = {"best_joints": f(n, T), "best_index": i(T), "target_success": i(T),
               "pos_err": f(m, T), "rot_err": f(m, T), "cost": f(T)}
        if stages:
            N0, N1 = T * n_seeds, T * keep
            out.update(stage0_joints=f(n, N0), stage0_cost=f(N0), stage0_pose_cost=f(N0),
                       stage0_status=i(N0), kept=i(T, keep), stage1_joints=f(n, N1),
                       stage1_cost=f(N1), stage1_pose_cost=f(N1), stage1_status=i(N1))
        return out

    def ik_beam(self, rid, targets, seeds, weights: Weights, options: Options, n_seeds=64,
                iters0=6, keep=4, iters1=10, stages=False, out=None):
        """IK-Beam (see include/pkmi.h): targets [tf, T], seeds [n, T*n_seeds];
        out from alloc_beam_outputs (allocated here when None).  Returns out."""
        T = targets.shape[1]
        self._check_ik(self.robot_info(rid), targets, seeds, T, int(n_seeds))
        if out is None:
            out = self.alloc_beam_outputs(rid, T, n_seeds, keep, stages, targets.device)
        oo = _BeamOutputs(*[_ptr(out.get(k)) for k in _BEAM_OUT])
        sch = _BeamSchedule(int(n_seeds), int(iters0), int(keep), int(iters1))
        w, op = weights._c(), options._c()
        self._call(lib().pk_ik_beam(self._h, rid, T, _ptr(targets), _ptr(seeds), C.byref(w),
                                    C.byref(op), C.byref(sch), C.byref(oo), self.stream()))
        return out

    def traj_solve(self, rid, start, goal, init, costs: dict, options: Options, vmax=None,
                   out=None):
        """Trajectory optimisation (see include/pkmi.h): start / goal [7, B] poses,
        init [B, T, n] (cuda float32); costs: dt, w_pos, w_rot, w_limit, w_smooth,
        w_vel, w_acc, w_jerk; vmax: cuda [n] or None.  Returns a dict of device
        tensors traj [B, T, n], cost, iters, accepts, status [B], pos_err /
        rot_err [2, B]."""
        torch = self._torch
        info = self.robot_info(rid)
        if init.dim() != 3:
            raise PkError(-1, f"init: shape {tuple(init.shape)}, expected (B, T, n)")
        B, T, n = init.shape
        if n != info["n"]:
            raise PkError(-1, f"init: last dimension {n}, the robot has {info['n']} variables")
        dev = init.device
        _check(init, "init", (B, T, n))
        _check(start, "start", (7, B), device=dev)
        _check(goal, "goal", (7, B), device=dev)
        if vmax is not None:
            _check(vmax, "vmax", (n,), device=dev)
        if out is None:
            f = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
            i = lambda *s: torch.empty(s, dtype=torch.int32, device=dev)
            out = {"traj": f(B, T, n), "cost": f(B), "iters": i(B), "accepts": i(B),
                   "status": i(B), "pos_err": f(2, B), "rot_err": f(2, B)}
        shapes = {"traj": (B, T, n), "cost": (B,), "iters": (B,), "accepts": (B,), "status": (B,),
                  "pos_err": (2, B), "rot_err": (2, B)}
        for k, shp in shapes.items():
            if out.get(k) is not None:
                _check(out[k], k, shp, "int32" if k in ("iters", "accepts", "status") else "float32",
                       device=dev)
        pr = _TrajProblem(B, T, _ptr(start), _ptr(goal), _ptr(init))
        c = _TrajCosts(*[float(costs[k]) for k in ["dt", "w_pos", "w_rot", "w_limit", "w_smooth",
                                                    "w_vel", "w_acc", "w_jerk"]], _ptr(vmax))
        oo = _TrajOutputs(*[_ptr(out.get(k)) for k in _TRAJ_OUT])
        op = options._c()
        self._call(lib().pk_traj_solve(self._h, rid, C.byref(pr), C.byref(c), C.byref(op),
                                       C.byref(oo), self.stream()))
        return out

    def ik_solve(self, rid, targets, seeds, K, weights: Weights, options: Options, out):
        """targets [tf, T] and seeds [n, T*K] are cuda float32 tensors; out from
        alloc_outputs (missing keys are passed as NULL)."""
        info = self.robot_info(rid)
        if targets.dim() != 2:
            raise PkError(-1, f"targets: shape {tuple(targets.shape)}, expected (floats, T)")
        T = targets.shape[1]
        self._check_ik(info, targets, seeds, T, K, out)
        pr = _Problem(T, K, _ptr(targets), _ptr(seeds))
        o = self._outputs_c(out)
        w, op = weights._c(), options._c()
        self._call(lib().pk_ik_solve(self._h, rid, C.byref(pr), C.byref(w), C.byref(op),
                                     C.byref(o), self.stream()))
        return out

    def ik_solve_noalloc(self, rid, targets, seeds, K, weights: Weights, options: Options, out):
        """As ik_solve, through the allocation-free entry point (T*K at most
        NOALLOC_MAX_PROBLEMS; calls on one GPU share its scratch and must not
        overlap in time)."""
        info = self.robot_info(rid)
        if targets.dim() != 2:
            raise PkError(-1, f"targets: shape {tuple(targets.shape)}, expected (floats, T)")
        T = targets.shape[1]
        self._check_ik(info, targets, seeds, T, K, out)
        pr = _Problem(T, K, _ptr(targets), _ptr(seeds))
        o = self._outputs_c(out)
        w, op = weights._c(), options._c()
        self._call(lib().pk_ik_solve_noalloc(self._h, rid, C.byref(pr), C.byref(w), C.byref(op),
                                             C.byref(o), self.stream()))
        return out


class Seeder:
    """Learned seeder bound to one robot of a Context (see include/pkmi.h)."""

    def __init__(self, ctx: "Context", rid: int, K=8, hidden=512, depth=3, init=None):
        """init: list of (W [out,in], b [out]) host arrays (FP32), or None."""
        self.ctx, self.rid, self.K = ctx, rid, K
        flat, cnt = None, 0
        if init is not None:
            flat = np.ascontiguousarray(np.concatenate(
                [np.concatenate([np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32)])
                 for W, b in init]), dtype=np.float32)
            cnt = flat.size
        sid = C.c_int32()
        ctx._call(lib().pk_seeder_create(ctx._h, rid, K, hidden, depth,
                                         flat.ctypes.data_as(C.POINTER(C.c_float)) if flat is not None else None,
                                         cnt, C.byref(sid)))
        self.id = sid.value
        self.hidden, self.depth = hidden, depth
        self._n = ctx.robot_info(rid)["n"]

    def param_count(self):
        c = C.c_int64()
        self.ctx._call(lib().pk_seeder_param_count(self.ctx._h, self.id, C.byref(c)))
        return c.value

    def get(self, which=0):
        """Parameters (0), gradients (1), Adam moments (2, 3) as [(W, b)] host arrays."""
        cnt = self.param_count()
        buf = np.zeros(cnt, np.float32)
        self.ctx._call(lib().pk_seeder_get(self.ctx._h, self.id, which,
                                           buf.ctypes.data_as(C.POINTER(C.c_float)), cnt))
        out, off = [], 0
        dims = [7] + [self.hidden] * self.depth + [self._n * self.K]
        for fi, fo in zip(dims[:-1], dims[1:]):
            W = buf[off:off + fi * fo].reshape(fo, fi)
            off += fi * fo
            b = buf[off:off + fo]
            off += fo
            out.append((W.copy(), b.copy()))
        return out

    def forward(self, x, layers=False):
        """x: cuda float32 [B, 7] (encoded) -> y [B, n*K].  layers=True takes the
        layer-by-layer GEMM path instead of the fused inference kernel."""
        y = self.ctx._torch.empty((x.shape[0], self._n * self.K), dtype=self.ctx._torch.float32,
                                  device=x.device)
        fn = lib().pk_seeder_forward_layers if layers else lib().pk_seeder_forward
        self.ctx._call(fn(self.ctx._h, self.id, _ptr(x), x.shape[0], _ptr(y), self.ctx.stream()))
        return y

    def grad(self, x, q):
        loss = self.ctx._torch.zeros(1, dtype=self.ctx._torch.float32, device=x.device)
        self.ctx._call(lib().pk_seeder_grad(self.ctx._h, self.id, _ptr(x), _ptr(q), x.shape[0],
                                            _ptr(loss), self.ctx.stream()))
        return loss

    def train(self, q_train, batch=8192, epochs=1, lr=1e-3, perm=None, loss_log=None):
        """q_train: cuda float32 [n, S]; perm: cuda int32 [epochs, S] or None."""
        S = q_train.shape[1]
        self.ctx._call(lib().pk_seeder_train(self.ctx._h, self.id, _ptr(q_train), S, batch, epochs,
                                             lr, _ptr(perm), _ptr(loss_log), self.ctx.stream()))

    def infer(self, targets, seeds=None):
        """targets: cuda float32 [7, T] -> seeds [n, T*K]."""
        T = targets.shape[1]
        if seeds is None:
            seeds = self.ctx._torch.empty((self._n, T * self.K), dtype=self.ctx._torch.float32,
                                          device=targets.device)
        self.ctx._call(lib().pk_seeder_infer(self.ctx._h, self.id, _ptr(targets), T, _ptr(seeds),
                                             self.ctx.stream()))
        return seeds

    def save(self, path):
        self.ctx._call(lib().pk_seeder_save(self.ctx._h, self.id, str(path).encode()))

    def load(self, path):
        self.ctx._call(lib().pk_seeder_load(self.ctx._h, self.id, str(path).encode()))

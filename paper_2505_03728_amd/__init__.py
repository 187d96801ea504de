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

__all__ = ["Context", "Weights", "Options", "lib", "LibraryMissing", "PkError",
           "CONVERGED", "MAX_ITERS", "STALLED", "NONFINITE", "FLAG_FP64",
           "EE_POSE", "EE_POSITION", "VARIANT_AUTO", "VARIANT_LANE", "VARIANT_WAVE",
           "pack_targets", "target_floats"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpkmi.so")

CONVERGED, MAX_ITERS, STALLED, NONFINITE = 0, 1, 2, 3
FLAG_FP64 = 0x100
EE_POSE, EE_POSITION = 0, 1
VARIANT_AUTO, VARIANT_LANE, VARIANT_WAVE = 0, 1, 2


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
                ("ee_quat", _f64p), ("ee_kind", _i32p)]


class _Weights(C.Structure):
    _fields_ = [("w_pos", C.c_float), ("w_rot", C.c_float), ("w_limit", C.c_float),
                ("w_rest", C.c_float), ("q_rest", C.c_void_p)]


class _Options(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("lambda0", C.c_float), ("nu_up", C.c_float),
                ("nu_down", C.c_float), ("lambda_min", C.c_float), ("lambda_max", C.c_float),
                ("early_exit", C.c_int32), ("tol_pos", C.c_float), ("tol_rot", C.c_float),
                ("damping_floor", C.c_float), ("pivot_rel", C.c_float), ("variant", C.c_int32)]


class _Problem(C.Structure):
    _fields_ = [("n_targets", C.c_int64), ("K", C.c_int32), ("targets", C.c_void_p),
                ("seeds", C.c_void_p)]


class _Outputs(C.Structure):
    _fields_ = [("joints", C.c_void_p), ("pos_err", C.c_void_p), ("rot_err", C.c_void_p),
                ("cost", C.c_void_p), ("iters", C.c_void_p), ("accepts", C.c_void_p),
                ("status", C.c_void_p), ("iters_to_tol", C.c_void_p),
                ("best_index", C.c_void_p), ("best_joints", C.c_void_p),
                ("target_success", C.c_void_p), ("trace_iters", C.c_int32),
                ("trace_q", C.c_void_p), ("trace_accept", C.c_void_p)]


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
        for f in ["pk_create", "pk_destroy", "pk_robot_upload", "pk_robot_info", "pk_fk",
                  "pk_residual_jacobian", "pk_ik_solve"]:
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def exported_symbols():
    """Names of the C entry points this binding expects the library to export."""
    return ["pk_create", "pk_destroy", "pk_last_error", "pk_robot_upload", "pk_robot_info",
            "pk_fk", "pk_residual_jacobian", "pk_ik_solve"]


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
                 damping_floor=1e-6, pivot_rel=1e-6, variant=VARIANT_AUTO):
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
                        int(self.variant))


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
        ee_offset, ee_quat, ee_kind arrays (see include/pkmi.h)."""
        d = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        keep = [i(tree.parent), d(tree.mount_quat), d(tree.offset), d(tree.axis), d(tree.lower),
                d(tree.upper), i(tree.ee_joint), d(tree.ee_offset), d(tree.ee_quat),
                i(tree.ee_kind)]
        pi = lambda a: a.ctypes.data_as(_i32p)
        pd = lambda a: a.ctypes.data_as(_f64p)
        t = _Tree(len(keep[0]), pi(keep[0]), pd(keep[1]), pd(keep[2]), pd(keep[3]), pd(keep[4]),
                  pd(keep[5]), len(keep[6]), pi(keep[6]), pd(keep[7]), pd(keep[8]), pi(keep[9]))
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
                       status=i(N), iters_to_tol=i(N))
        if best:
            out.update(best_index=i(T), best_joints=f(n, T), target_success=i(T))
        if trace_iters:
            out.update(trace_q=f(trace_iters, n, N), trace_accept=i(trace_iters, N))
        out["_trace_iters"] = trace_iters
        return out

    def ik_solve(self, rid, targets, seeds, K, weights: Weights, options: Options, out):
        """targets [tf, T] and seeds [n, T*K] are cuda float32 tensors; out from
        alloc_outputs (missing keys are passed as NULL)."""
        T = targets.shape[1]
        pr = _Problem(T, K, _ptr(targets), _ptr(seeds))
        o = _Outputs(*[_ptr(out.get(k)) for k in ["joints", "pos_err", "rot_err", "cost", "iters",
                                                   "accepts", "status", "iters_to_tol",
                                                   "best_index", "best_joints",
                                                   "target_success"]],
                     int(out.get("_trace_iters", 0)), _ptr(out.get("trace_q")),
                     _ptr(out.get("trace_accept")))
        w, op = weights._c(), options._c()
        self._call(lib().pk_ik_solve(self._h, rid, C.byref(pr), C.byref(w), C.byref(op),
                                     C.byref(o), self.stream()))
        return out

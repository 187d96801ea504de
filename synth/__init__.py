"""Seeded synthetic inputs for batched IK: robot trees, joint draws, seeds.

This module only *draws* numbers.  It holds none of the method's arithmetic
(no forward kinematics, no residuals, no solver); both the FP64 oracle and
the GPU path consume what it returns, and each computes targets = FK(q*)
with its own code.

Every floating-point value returned here is representable in FP32 (it is
rounded to FP32 and promoted back), so both sides start from bit-identical
inputs.  Draw order is fixed and documented per function so that a smaller
request with the same seed is a prefix of a larger one.

Robot families (the paper's workloads use real URDFs that are not available;
these seeded families stand in for them):

* ``arm7``  — 7-DoF serial revolute arm, axes z,y,z,y,z,y,z, link offsets
  (U[0.05,0.30], 0, U[0.05,0.30]) in the parent frame, limits ±U[pi/2, pi].
* ``tree34`` — humanoid-like tree: a 6-joint torso chain (z,y,z,y,z,y) and 4
  branches of 7 joints (z,y,z,y,z,y,z) hanging off the torso's last joint,
  branch c mounted with a rotation Rz(c*pi/2); one pose end effector per
  branch.  34 DoF, 4 EEs.
* ``hand16`` — 4 fingers of 4 joints (z,y,z,y) from the base, offsets
  U[0.02,0.05], finger c's root shifted by (0, (c-1.5)*0.02, 0); one
  position-only fingertip EE per finger.  16 DoF, 4 EEs.
* ``arm7_tool`` — arm7 with two fixed joints: a flange between joints 3 and 4
  (mount Rx(pi/2)) and a tool at the tip that carries the EE.  7 DoF.
* ``scara4`` — revolute z, revolute z, prismatic z, revolute z (a SCARA-like
  chain with one sliding joint), pose EE.  4 DoF.
* ``mobile_arm7`` — a planar base (prismatic x, prismatic y, revolute z: the
  SE(2) base pose) carrying arm7.  10 DoF.
* ``hand16_mimic`` — hand16 whose distal joints follow the joint before them
  (mimic joints).  12 DoF.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Tree", "EE_POSE", "EE_POSITION", "JOINT_REVOLUTE", "JOINT_PRISMATIC", "JOINT_FIXED",
    "arm7", "tree34", "hand16", "chain", "arm7_tool", "scara4", "mobile_arm7", "hand16_mimic",
    "planar2", "one_joint", "uniform_configs", "workload", "mlp_init",
    "epoch_permutation", "f32",
]

EE_POSE = 0
EE_POSITION = 1
JOINT_REVOLUTE = 0
JOINT_PRISMATIC = 1
JOINT_FIXED = 2

_AX = {"x": (1.0, 0.0, 0.0), "y": (0.0, 1.0, 0.0), "z": (0.0, 0.0, 1.0)}


def f32(a):
    """Round to FP32 and promote back to float64 (exact)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@dataclass
class Tree:
    """A joint tree in topological order (parent[j] < j, -1 = base).

    Joint j's frame is its parent's frame, translated by ``offset[j]``
    (expressed in the parent frame), rotated by the mount rotation
    ``mount_quat[j]`` (wxyz) and then moved by the joint: a rotation about
    ``axis[j]`` (expressed after the mount) for a revolute joint, a
    translation along it for a prismatic one, nothing for a fixed one.  The
    variables are the non-fixed joints in index order (``var_joints``); EE k
    is rigidly attached to joint ``ee_joint[k]`` with ``ee_offset[k]`` /
    ``ee_quat[k]``.  ``joint_type`` None means every joint is revolute.  A
    mimic joint (``mimic_joint[j]`` >= 0) follows its driver:
    q_j = mimic_multiplier[j] * q_driver + mimic_offset[j].
    """
    name: str
    parent: np.ndarray          # int32 [n]
    mount_quat: np.ndarray      # [n,4] wxyz
    offset: np.ndarray          # [n,3]
    axis: np.ndarray            # [n,3]
    lower: np.ndarray           # [n]
    upper: np.ndarray           # [n]
    ee_joint: np.ndarray        # int32 [m]
    ee_offset: np.ndarray       # [m,3]
    ee_quat: np.ndarray         # [m,4]
    ee_kind: np.ndarray         # int32 [m]
    meta: dict = field(default_factory=dict)
    joint_type: np.ndarray | None = None   # int32 [n] JOINT_*, None = all revolute
    mimic_joint: np.ndarray | None = None  # int32 [n] driver or -1, None = no mimic joints
    mimic_multiplier: np.ndarray | None = None
    mimic_offset: np.ndarray | None = None

    @property
    def n(self) -> int:
        """Joints of the description (fixed ones included)."""
        return int(self.parent.shape[0])

    @property
    def types(self) -> np.ndarray:
        if self.joint_type is None:
            return np.zeros(self.n, dtype=np.int32)
        return np.asarray(self.joint_type, dtype=np.int32)

    @property
    def mimics(self) -> np.ndarray:
        if self.mimic_joint is None:
            return np.full(self.n, -1, dtype=np.int32)
        return np.asarray(self.mimic_joint, dtype=np.int32)

    @property
    def var_joints(self) -> np.ndarray:
        """Indices of the joints that are variables (neither fixed nor mimic), in order."""
        return np.nonzero((self.types != JOINT_FIXED) & (self.mimics < 0))[0]

    @property
    def dof(self) -> int:
        return int(self.var_joints.shape[0])

    @property
    def m(self) -> int:
        return int(self.ee_joint.shape[0])

    def target_width(self) -> list[int]:
        """Per EE: 7 target values (p, quat) for pose EEs, 3 for position EEs."""
        return [7 if k == EE_POSE else 3 for k in self.ee_kind]


def _finish(name, parent, mount, offset, axis, lim, ee_joint, ee_offset, ee_quat,
            ee_kind, meta=None, joint_type=None) -> Tree:
    lim = f32(lim)
    return Tree(
        name=name,
        parent=np.asarray(parent, dtype=np.int32),
        mount_quat=f32(mount).reshape(-1, 4),
        offset=f32(offset).reshape(-1, 3),
        axis=f32(axis).reshape(-1, 3),
        lower=-lim.copy(),
        upper=lim.copy(),
        ee_joint=np.asarray(ee_joint, dtype=np.int32),
        ee_offset=f32(ee_offset).reshape(-1, 3),
        ee_quat=f32(ee_quat).reshape(-1, 4),
        ee_kind=np.asarray(ee_kind, dtype=np.int32),
        meta=dict(meta or {}),
        joint_type=None if joint_type is None else np.asarray(joint_type, dtype=np.int32),
    )


def _xz_offsets(rng, count, lo, hi):
    """count offsets (x, 0, z); per offset x is drawn, then z."""
    d = rng.uniform(lo, hi, size=(count, 2))
    out = np.zeros((count, 3))
    out[:, 0] = d[:, 0]
    out[:, 2] = d[:, 1]
    return out


def chain(axes: str, seed: int, off_lo=0.05, off_hi=0.30, name=None) -> Tree:
    """Serial revolute chain from the base with one pose EE at its tip.

    Draw order (one PCG64 stream): n joint offsets, the EE offset, n limit
    half-widths U[pi/2, pi].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(axes)
    offs = _xz_offsets(rng, n + 1, off_lo, off_hi)
    lim = rng.uniform(math.pi / 2, math.pi, size=n)
    ident = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    return _finish(name or f"chain{n}", np.arange(n) - 1, ident, offs[:n],
                   [_AX[a] for a in axes], lim, [n - 1], offs[n:n + 1],
                   [[1.0, 0.0, 0.0, 0.0]], [EE_POSE], {"seed": seed, "axes": axes})


def arm7(seed: int = 0) -> Tree:
    return chain("zyzyzyz", seed, name="arm7")


def tree34(seed: int = 5) -> Tree:
    """Torso (6) + 4 branches (7 each) off the torso tip; 4 pose EEs.

    Draw order: 34 joint offsets in joint order (torso, then branch 0..3),
    4 EE offsets, 34 limit half-widths.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    torso, nb, lb = 6, 4, 7
    n = torso + nb * lb
    offs = _xz_offsets(rng, n, 0.05, 0.30)
    eeo = _xz_offsets(rng, nb, 0.05, 0.30)
    lim = rng.uniform(math.pi / 2, math.pi, size=n)
    parent, axes, mount, ee_joint = [], [], [], []
    for j in range(torso):
        parent.append(j - 1)
        axes.append(_AX["zy"[j % 2]])
        mount.append([1.0, 0.0, 0.0, 0.0])
    for c in range(nb):
        for i in range(lb):
            j = torso + c * lb + i
            parent.append(torso - 1 if i == 0 else j - 1)
            axes.append(_AX["zy"[i % 2]])
            if i == 0:
                h = c * math.pi / 4.0   # half-angle of Rz(c*pi/2)
                mount.append([math.cos(h), 0.0, 0.0, math.sin(h)])
            else:
                mount.append([1.0, 0.0, 0.0, 0.0])
        ee_joint.append(torso + c * lb + lb - 1)
    return _finish("tree34", parent, mount, offs, axes, lim, ee_joint, eeo,
                   np.tile([1.0, 0.0, 0.0, 0.0], (nb, 1)), [EE_POSE] * nb,
                   {"seed": seed, "torso": torso, "branches": nb, "branch_len": lb})


def hand16(seed: int = 8) -> Tree:
    """4 fingers x 4 joints from the base; 4 position-only fingertip EEs.

    Draw order: 16 joint offsets (finger-major), 4 fingertip offsets, 16 limit
    half-widths.  Finger c's root offset gets (0, (c-1.5)*0.02, 0) added.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nf, lf = 4, 4
    n = nf * lf
    offs = _xz_offsets(rng, n, 0.02, 0.05)
    eeo = _xz_offsets(rng, nf, 0.02, 0.05)
    lim = rng.uniform(math.pi / 2, math.pi, size=n)
    parent, axes, ee_joint = [], [], []
    for c in range(nf):
        for i in range(lf):
            j = c * lf + i
            parent.append(-1 if i == 0 else j - 1)
            axes.append(_AX["zy"[i % 2]])
            if i == 0:
                offs[j, 1] += (c - 1.5) * 0.02
        ee_joint.append(c * lf + lf - 1)
    return _finish("hand16", parent, np.tile([1.0, 0, 0, 0], (n, 1)), offs, axes, lim,
                   ee_joint, eeo, np.tile([1.0, 0, 0, 0], (nf, 1)), [EE_POSITION] * nf,
                   {"seed": seed, "fingers": nf, "finger_len": lf})


def planar2(l1: float = 0.6, l2: float = 0.4, kind: int = EE_POSE, lim=math.pi) -> Tree:
    """Planar 2-link arm: two z joints, link lengths along x; EE at the tip."""
    return _finish("planar2", [-1, 0], np.tile([1.0, 0, 0, 0], (2, 1)),
                   [[0, 0, 0], [l1, 0, 0]], [_AX["z"], _AX["z"]], [lim, lim], [1],
                   [[l2, 0, 0]], [[1.0, 0, 0, 0]], [kind])


def one_joint(offset=(0.1, 0.2, 0.3), ee_offset=(0.5, 0.0, 0.0), axis="z",
              lim=math.pi, kind: int = EE_POSE) -> Tree:
    return _finish("one_joint", [-1], [[1.0, 0, 0, 0]], [offset], [_AX[axis]], [lim],
                   [0], [ee_offset], [[1.0, 0, 0, 0]], [kind])


def arm7_tool(seed: int = 0) -> Tree:
    """arm7 with a fixed flange after joint 3 (mount Rx(pi/2), offset
    (0, 0, 0.05)) and a fixed tool after joint 6 (offset (0, 0, 0.12),
    mount Ry(pi/4)) that carries the pose EE (at arm7's EE offset)."""
    a = arm7(seed)
    h = math.sqrt(0.5)
    c8 = math.cos(math.pi / 8)
    s8 = math.sin(math.pi / 8)
    order = [0, 1, 2, 3, "flange", 4, 5, 6, "tool"]
    idx = {}
    parent, mount, offset, axis, lim, jt = [], [], [], [], [], []
    for i, o in enumerate(order):
        idx[o] = i
        if o == "flange":
            parent.append(idx[3]); mount.append([h, h, 0.0, 0.0]); offset.append([0.0, 0.0, 0.05])
            axis.append(_AX["z"]); lim.append(0.0); jt.append(JOINT_FIXED)
        elif o == "tool":
            parent.append(idx[6]); mount.append([c8, 0.0, s8, 0.0]); offset.append([0.0, 0.0, 0.12])
            axis.append(_AX["z"]); lim.append(0.0); jt.append(JOINT_FIXED)
        else:
            parent.append(-1 if o == 0 else (idx["flange"] if o == 4 else idx[o - 1]))
            mount.append(a.mount_quat[o]); offset.append(a.offset[o]); axis.append(a.axis[o])
            lim.append(a.upper[o]); jt.append(JOINT_REVOLUTE)
    return _finish("arm7_tool", parent, mount, offset, axis, lim, [idx["tool"]], a.ee_offset,
                   [[1.0, 0.0, 0.0, 0.0]], [EE_POSE], {"seed": seed}, joint_type=jt)


def scara4() -> Tree:
    """Revolute z, revolute z (0.35 m link along x), prismatic z (0.25 m link,
    stroke +-0.2 m), revolute z; pose EE 0.05 m below the last joint."""
    return _finish("scara4", [-1, 0, 1, 2], np.tile([1.0, 0, 0, 0], (4, 1)),
                   [[0, 0, 0.4], [0.35, 0, 0], [0.25, 0, 0], [0, 0, 0]],
                   [_AX["z"]] * 4, [math.pi * 0.9, math.pi * 0.8, 0.2, math.pi], [3],
                   [[0, 0, -0.05]], [[1.0, 0, 0, 0]], [EE_POSE],
                   joint_type=[JOINT_REVOLUTE, JOINT_REVOLUTE, JOINT_PRISMATIC, JOINT_REVOLUTE])


def mobile_arm7(seed: int = 0, reach: float = 2.0) -> Tree:
    """SE(2) base pose as joints (prismatic x, prismatic y, revolute z, all at
    the base origin; x and y within +-reach metres, yaw within +-pi) carrying
    arm7 (its joint 0 hangs off the yaw joint)."""
    a = arm7(seed)
    n = a.n
    parent = [-1, 0, 1] + [2 if j == 0 else j + 2 for j in range(n)]
    mount = [[1.0, 0, 0, 0]] * 3 + list(a.mount_quat)
    offset = [[0.0, 0.0, 0.0]] * 3 + list(a.offset)
    axis = [_AX["x"], _AX["y"], _AX["z"]] + list(a.axis)
    lim = [reach, reach, math.pi] + list(a.upper)
    jt = [JOINT_PRISMATIC, JOINT_PRISMATIC, JOINT_REVOLUTE] + [JOINT_REVOLUTE] * n
    return _finish("mobile_arm7", parent, mount, offset, axis, lim, [a.ee_joint[0] + 3],
                   a.ee_offset, a.ee_quat, [EE_POSE], {"seed": seed, "reach": reach},
                   joint_type=jt)


def hand16_mimic(seed: int = 8, mult: float = 0.8, off: float = 0.1) -> Tree:
    """hand16 with each finger's last joint coupled to the one before it
    (q_3 = mult * q_2 + off per finger, as a finger's distal joint follows its
    middle joint): 12 variables."""
    h = hand16(seed)
    mj = np.full(h.n, -1, dtype=np.int32)
    for c in range(4):
        mj[4 * c + 3] = 4 * c + 2
    t = Tree(**{**h.__dict__, "name": "hand16_mimic"})
    t.mimic_joint = mj
    t.mimic_multiplier = f32(np.where(mj >= 0, mult, 0.0))
    t.mimic_offset = f32(np.where(mj >= 0, off, 0.0))
    return t


def uniform_configs(tree: Tree, count: int, seed: int) -> np.ndarray:
    """count x dof variable vectors, q_v ~ U[lower, upper] of the v-th
    non-fixed joint (row-major draws)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vj = tree.var_joints
    u = rng.random(size=(count, vj.shape[0]))
    return f32(tree.lower[vj] + u * (tree.upper[vj] - tree.lower[vj]))


def _weights(w_pos=1.0, w_rot=0.5, w_limit=10.0, w_rest=0.0):
    return {"w_pos": w_pos, "w_rot": w_rot, "w_limit": w_limit, "w_rest": w_rest}


def _options(max_iters, early_exit=False):
    return {"max_iters": max_iters, "lambda0": 1e-3, "nu_up": 10.0, "nu_down": 10.0,
            "lambda_min": 1e-10, "lambda_max": 1e10, "early_exit": bool(early_exit),
            "tol_pos": 1e-3, "tol_rot": 1e-2, "damping_floor": 1e-6, "pivot_rel": 1e-6}


def workload(name: str, scale: float = 1.0, targets: int | None = None) -> dict:
    """Seeded workload description.

    ``name`` is one of:
      * ``arm16``   — 16 targets on arm7, 1 seed each, pose+limit, 50 iterations;
      * ``arm131k`` — 16384 targets x 8 seeds on arm7, pose+limit+rest(0.01),
                      30 iterations, best-of-8;
      * ``tree4k``  — 4096 problems on tree34 (4 pose EEs), pose+limit, 40 its;
      * ``mixed84k``— 60000 arm7 + 20000 hand16 + 4096 tree34 problems, early
                      exit, rest 0.01, up to 50 iterations (per-group weights in
                      each group's ``weights``);
      * ``seeder``  — 2M training configurations + 131072 evaluation targets;
      * ``beam``    — IK-Beam on arm7 (pose+limit): 2000 targets x 64 seeds,
                      6 iterations, 4 kept, 10 iterations; the batch sizes
                      1, 10, 100, 1000, 2000 are prefixes of the same draws;
      * ``mobile``  — IK with a mobile base: 4096 arm7 poses reachable from
                      the base at the origin, each translated horizontally by
                      U[-1, 1]^2 m; mobile_arm7 (base pose free) x 4 seeds
                      with the base at the origin, and the same targets for
                      arm7 alone (fixed base); pose+limit+rest(0.01), up to
                      30 iterations with early exit, success at 5 mm /
                      0.05 rad;
      * ``traj``    — trajectory optimisation on arm7: 1024 trajectories of
                      32 timesteps (dt 0.05 s) between the poses of two
                      random configurations, initialised by linear
                      interpolation between perturbed endpoint
                      configurations plus a sine bump; 20 iterations.
    ``targets`` overrides the target count (a prefix of the same draws).
    Returns q* (configurations whose FK are the targets) and seeds; the caller
    computes the target poses with its own FK.
    """
    if name == "arm16":
        r = arm7(0)
        T = targets or 16
        return {"groups": [{"tree": r, "q_star": uniform_configs(r, T, 1), "K": 1,
                            "seeds": uniform_configs(r, T, 2)}],
                "weights": _weights(), "options": _options(50)}
    if name == "arm131k":
        r = arm7(0)
        T = targets or int(16384 * scale)
        K = 8
        return {"groups": [{"tree": r, "q_star": uniform_configs(r, T, 3), "K": K,
                            "seeds": uniform_configs(r, T * K, 4)}],
                "weights": _weights(w_rest=0.01), "options": _options(30)}
    if name == "tree4k":
        r = tree34(5)
        T = targets or int(4096 * scale)
        return {"groups": [{"tree": r, "q_star": uniform_configs(r, T, 6), "K": 1,
                            "seeds": uniform_configs(r, T, 7)}],
                "weights": _weights(), "options": _options(40)}
    if name == "mixed84k":
        counts = [60000, 20000, 4096]
        if targets is not None:
            counts = [targets] * 3
        else:
            counts = [max(1, int(c * scale)) for c in counts]
        robots = [arm7(0), hand16(8), tree34(5)]
        # The hand's links are an order of magnitude shorter than the arm's:
        # its position residuals (metres) get a 10x weight so that the rest
        # term (radians) does not dominate its optimum.
        wts = [_weights(w_rest=0.01), _weights(w_pos=10.0, w_rest=0.01), _weights(w_rest=0.01)]
        gs = []
        for r, c, sq, ss, w in zip(robots, counts, (9, 10, 11), (12, 13, 14), wts):
            gs.append({"tree": r, "q_star": uniform_configs(r, c, sq), "K": 1,
                       "seeds": uniform_configs(r, c, ss), "weights": w})
        return {"groups": gs, "weights": _weights(w_rest=0.01),
                "options": _options(50, early_exit=True)}
    if name == "beam":
        r = arm7(0)
        T = targets or int(2000 * scale)
        K = 64
        return {"groups": [{"tree": r, "q_star": uniform_configs(r, T, 20), "K": K,
                            "seeds": uniform_configs(r, T * K, 21)}],
                "weights": _weights(), "options": _options(16),
                "schedule": {"n_seeds": K, "iters0": 6, "keep": 4, "iters1": 10},
                "batches": [1, 10, 100, 1000, 2000]}
    if name == "mobile":
        arm, mob = arm7(0), mobile_arm7(0)
        T = targets or int(4096 * scale)
        K = 4
        q_arm = uniform_configs(arm, T, 22)
        shift = f32(np.random.Generator(np.random.PCG64(23)).uniform(-1.0, 1.0, size=(T, 2)))
        seeds_arm = uniform_configs(arm, T * K, 24)
        q_star = np.concatenate([shift, np.zeros((T, 1)), q_arm], 1)
        seeds = np.concatenate([np.zeros((T * K, 3)), seeds_arm], 1)
        o = dict(_options(30, early_exit=True), tol_pos=5e-3, tol_rot=5e-2)
        return {"groups": [{"tree": mob, "q_star": q_star, "K": K, "seeds": seeds}],
                "fixed_base": {"tree": arm, "seeds": seeds_arm},
                "weights": _weights(w_rest=0.01), "options": o}
    if name == "traj":
        r = arm7(0)
        B = targets or int(1024 * scale)
        T = 32
        qa = uniform_configs(r, B, 25)
        qb = uniform_configs(r, B, 26)
        rng = np.random.Generator(np.random.PCG64(27))
        ea = rng.normal(0.0, 0.05, size=(B, r.dof))
        eb = rng.normal(0.0, 0.05, size=(B, r.dof))
        u = rng.normal(0.0, 1.0, size=(B, r.dof))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        s_ = np.linspace(0.0, 1.0, T)[None, :, None]
        init = ((1 - s_) * (qa + ea)[:, None, :] + s_ * (qb + eb)[:, None, :] +
                0.3 * np.sin(np.pi * s_) * u[:, None, :])
        costs = {"T": T, "dt": 0.05, "w_pos": 10.0, "w_rot": 5.0, "w_limit": 10.0,
                 "w_smooth": 0.1, "w_vel": 1.0, "vmax": [2.0] * r.dof, "w_acc": 0.05,
                 "w_jerk": 0.01}
        return {"tree": r, "start_q": qa, "goal_q": qb, "init": f32(init), "costs": costs,
                "options": _options(20)}
    if name == "seeder":
        r = arm7(0)
        S = int(2_000_000 * scale)
        T = targets or int(131072 * scale)
        K = 8
        return {"tree": r, "train_q": uniform_configs(r, S, 15),
                "eval_q_star": uniform_configs(r, T, 16), "K": K,
                "plain_seeds": uniform_configs(r, T * K, 17),
                "weights": _weights(w_rest=0.01), "options": _options(30),
                "mlp": {"hidden": 512, "depth": 3, "batch": 8192, "lr": 1e-3,
                        "epochs": 40, "init_seed": 18, "shuffle_seed": 19}}
    raise KeyError(name)


def mlp_init(sizes: list[int], seed: int) -> list[tuple[np.ndarray, np.ndarray]]:
    """Layer i: W [sizes[i+1], sizes[i]] then b [sizes[i+1]], both U(+-1/sqrt(fan_in)).

    Draw order: W0, b0, W1, b1, ... from one PCG64 stream; FP32-rounded.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        a = 1.0 / math.sqrt(fi)
        W = f32(rng.uniform(-a, a, size=(fo, fi)))
        b = f32(rng.uniform(-a, a, size=fo))
        out.append((W, b))
    return out


def epoch_permutation(count: int, seed: int, epoch: int) -> np.ndarray:
    """Sample order for one training epoch (int32)."""
    rng = np.random.Generator(np.random.PCG64([seed, epoch]))
    return rng.permutation(count).astype(np.int32)

"""Pins for the oracle's forward kinematics, residuals and Jacobian.

FK (Sec. III-B, T_base<-i = FK(q)_i) is checked against closed forms
(zero configuration, one joint, planar 2-link) and against an independent
product of 4x4 homogeneous matrices built with scipy's Rotation.  The
residuals (Sec. III-C) are checked against their definitions evaluated with
scipy's matrix logarithm, and the analytic Jacobian against central finite
differences of the residual.
"""
import math

import numpy as np
import pytest
from scipy.linalg import logm
from scipy.spatial.transform import Rotation

import synth

rng = np.random.default_rng(99)
TREES = [synth.arm7(0), synth.tree34(5), synth.hand16(8)]
# fixed, prismatic and mixed joint kinds (Sec. III-B)
KINDS = [synth.arm7_tool(0), synth.scara4(), synth.mobile_arm7(0), synth.hand16_mimic(8)]


def homog(R, t):
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def fk_homogeneous(tree, q):
    """Independent FK: T_j = T_parent * Trans(t_j) * Rot(mount_j) * M_j, with
    M_j = Rot(axis_j, q_j) (revolute), Trans(axis_j q_j) (prismatic) or I
    (fixed); q_j is joint j's variable (variables in joint order), or for a
    mimic joint mult * (its driver's value) + offset."""
    Ts = []
    vals = {}
    v = 0
    mim = tree.mimics
    for j in range(tree.n):
        par = tree.parent[j]
        Tp = np.eye(4) if par < 0 else Ts[par]
        mq = tree.mount_quat[j]
        Rm = Rotation.from_quat([mq[1], mq[2], mq[3], mq[0]]).as_matrix()
        a = tree.axis[j] / np.linalg.norm(tree.axis[j])
        kind = tree.types[j]
        if kind != synth.JOINT_FIXED:
            if mim[j] >= 0:
                vals[j] = tree.mimic_multiplier[j] * vals[mim[j]] + tree.mimic_offset[j]
            else:
                vals[j] = q[v]
                v += 1
        if kind == synth.JOINT_REVOLUTE:
            Mj = homog(Rotation.from_rotvec(a * vals[j]).as_matrix(), np.zeros(3))
        elif kind == synth.JOINT_PRISMATIC:
            Mj = homog(np.eye(3), a * vals[j])
        else:
            Mj = np.eye(4)
        Ts.append(Tp @ homog(np.eye(3), tree.offset[j]) @ homog(Rm, np.zeros(3)) @ Mj)
    ees = []
    for k in range(tree.m):
        eq = tree.ee_quat[k]
        Re = Rotation.from_quat([eq[1], eq[2], eq[3], eq[0]]).as_matrix()
        ees.append(Ts[tree.ee_joint[k]] @ homog(Re, tree.ee_offset[k]))
    return Ts, ees


@pytest.mark.parametrize("tree", TREES + KINDS, ids=lambda t: t.name)
def test_fk_matches_homogeneous_product(ora, tree):
    for q in synth.uniform_configs(tree, 20, 5):
        R, p, Re, pe = ora.fk(tree, q)
        Ts, ees = fk_homogeneous(tree, q)
        for j in range(tree.n):
            np.testing.assert_allclose(R[j], Ts[j][:3, :3], atol=1e-13)
            np.testing.assert_allclose(p[j], Ts[j][:3, 3], atol=1e-13)
        for k in range(tree.m):
            np.testing.assert_allclose(Re[k], ees[k][:3, :3], atol=1e-13)
            np.testing.assert_allclose(pe[k], ees[k][:3, 3], atol=1e-13)


def test_fk_arm_zero_configuration(ora):
    tree = synth.arm7(0)
    _, _, Re, pe = ora.fk(tree, np.zeros(7))
    np.testing.assert_allclose(Re[0], np.eye(3), atol=0)
    np.testing.assert_allclose(pe[0], tree.offset.sum(0) + tree.ee_offset[0], atol=1e-15)


def test_fk_tree_zero_configuration(ora):
    tree = synth.tree34(5)
    _, _, Re, pe = ora.fk(tree, np.zeros(34))
    torso = tree.offset[:6].sum(0)
    for c in range(4):
        b = 6 + 7 * c
        h = c * math.pi / 2
        Rz = np.array([[math.cos(h), -math.sin(h), 0], [math.sin(h), math.cos(h), 0], [0, 0, 1]])
        want = torso + tree.offset[b] + Rz @ (tree.offset[b + 1:b + 7].sum(0) + tree.ee_offset[c])
        np.testing.assert_allclose(pe[c], want, atol=1e-7)   # mount quat is FP32-rounded
        np.testing.assert_allclose(Re[c], Rz, atol=1e-7)


def test_fk_one_joint_closed_form(ora):
    t, e = np.array([0.1, 0.2, 0.3]), np.array([0.5, 0.0, 0.0])
    tree = synth.one_joint(t, e)
    for q in [-2.0, 0.0, 0.7, 3.0]:
        _, _, Re, pe = ora.fk(tree, np.array([q]))
        Rz = np.array([[math.cos(q), -math.sin(q), 0], [math.sin(q), math.cos(q), 0], [0, 0, 1]])
        np.testing.assert_allclose(pe[0], t + Rz @ e, atol=1e-15)
        np.testing.assert_allclose(Re[0], Rz, atol=1e-15)


def test_fk_planar_two_link_closed_form(ora):
    l1, l2 = 0.6, 0.4
    tree = synth.planar2(l1, l2)
    for q1, q2 in rng.uniform(-3, 3, size=(10, 2)):
        _, _, Re, pe = ora.fk(tree, np.array([q1, q2]))
        np.testing.assert_allclose(
            pe[0], [l1 * math.cos(q1) + l2 * math.cos(q1 + q2),
                    l1 * math.sin(q1) + l2 * math.sin(q1 + q2), 0.0], atol=1e-15)
        np.testing.assert_allclose(ora.so3_log(Re[0]), [0, 0, (q1 + q2 + math.pi) % (2 * math.pi) - math.pi],
                                   atol=1e-12)


@pytest.mark.parametrize("tree", TREES, ids=lambda t: t.name)
def test_fk_pose7_quaternion_consistent(ora, tree):
    for q in synth.uniform_configs(tree, 10, 6):
        pose = ora.fk_pose7(tree, q)
        _, _, Re, pe = ora.fk(tree, q)
        for k in range(tree.m):
            assert pose[k, 3] >= 0
            np.testing.assert_allclose(np.linalg.norm(pose[k, 3:]), 1.0, atol=1e-14)
            np.testing.assert_allclose(ora.quat_to_R(pose[k, 3:]), Re[k], atol=1e-14)
            np.testing.assert_allclose(pose[k, :3], pe[k], atol=0)


WEIGHTS = {"w_pos": 1.0, "w_rot": 0.5, "w_limit": 10.0, "w_rest": 0.01, "q_rest": None}


@pytest.mark.parametrize("tree", TREES, ids=lambda t: t.name)
def test_pose_residual_is_se3_log_of_relative_transform(ora, tree):
    qs = synth.uniform_configs(tree, 6, 7)
    tg = ora.targets_from(tree, synth.uniform_configs(tree, 6, 8))
    for q, t in zip(qs, tg):
        r, pe, re = ora.residual(tree, t, WEIGHTS, q)
        _, ees = fk_homogeneous(tree, q)
        row = 0
        for k in range(tree.m):
            Tt = homog(ora.quat_to_R(t[k, 3:]), t[k, :3])
            if tree.ee_kind[k] == synth.EE_POSE:
                L = np.real(logm(np.linalg.inv(Tt) @ ees[k]))
                xi = np.array([L[0, 3], L[1, 3], L[2, 3], L[2, 1], L[0, 2], L[1, 0]])
                np.testing.assert_allclose(r[row:row + 3], WEIGHTS["w_pos"] * xi[:3], atol=1e-9)
                np.testing.assert_allclose(r[row + 3:row + 6], WEIGHTS["w_rot"] * xi[3:], atol=1e-9)
                np.testing.assert_allclose(re[k], np.linalg.norm(xi[3:]), atol=1e-9)
                row += 6
            else:
                np.testing.assert_allclose(r[row:row + 3], ees[k][:3, 3] - t[k, :3], atol=1e-14)
                row += 3
            np.testing.assert_allclose(pe[k], np.linalg.norm(ees[k][:3, 3] - t[k, :3]), atol=1e-14)
        lim = r[row:row + tree.n]
        want = WEIGHTS["w_limit"] * (np.maximum(0, q - tree.upper) + np.maximum(0, tree.lower - q))
        np.testing.assert_allclose(lim, want, atol=0)
        rest = r[row + tree.n:]
        np.testing.assert_allclose(rest, WEIGHTS["w_rest"] * (q - 0.5 * (tree.lower + tree.upper)),
                                   atol=1e-18)


def test_limit_residual_values(ora):
    tree = synth.one_joint(lim=1.0)
    tg = ora.targets_from(tree, np.zeros((1, 1)))[0]
    w = dict(WEIGHTS, w_rest=0.0)
    for q, want in [(1.5, 0.5), (-1.25, 0.25), (0.3, 0.0), (1.0, 0.0)]:
        r, _, _ = ora.residual(tree, tg, w, np.array([q]))
        assert r[6] == pytest.approx(10.0 * want, abs=1e-15)


def _fd_jac(ora, tree, t, w, q, h=1e-6):
    J = np.zeros((ora.n_rows(tree), tree.dof))
    for j in range(tree.dof):
        e = np.zeros(tree.dof)
        e[j] = h
        J[:, j] = (ora.residual(tree, t, w, q + e)[0] - ora.residual(tree, t, w, q - e)[0]) / (2 * h)
    return J


@pytest.mark.parametrize("tree", TREES + KINDS + [synth.planar2(),
                                                  synth.one_joint(kind=synth.EE_POSITION)],
                         ids=lambda t: t.name + str(t.ee_kind[0]))
def test_analytic_jacobian_matches_finite_differences(ora, tree):
    qs = synth.uniform_configs(tree, 8, 11)
    # Push a few joints outside their limits (away from the kink).
    qs[::2, 0] = tree.upper[tree.var_joints[0]] + 0.3
    tg = ora.targets_from(tree, synth.uniform_configs(tree, 8, 12))
    for q, t in zip(qs, tg):
        J = ora.jacobian(tree, t, WEIGHTS, q)
        Jf = _fd_jac(ora, tree, t, WEIGHTS, q)
        rel = np.linalg.norm(J - Jf) / max(np.linalg.norm(Jf), 1e-6)
        assert rel < 1e-7, rel


def test_jacobian_zero_for_non_ancestors(ora):
    tree = synth.hand16(8)
    q = synth.uniform_configs(tree, 1, 3)[0]
    tg = ora.targets_from(tree, synth.uniform_configs(tree, 1, 4))[0]
    J = ora.jacobian(tree, tg, WEIGHTS, q)
    for k in range(4):
        blk = J[3 * k:3 * k + 3]
        for j in range(16):
            if j // 4 != k:
                assert np.all(blk[:, j] == 0)
            else:
                assert np.any(blk[:, j] != 0)


def test_fk_scara_closed_form(ora):
    """Two revolute z joints (links 0.35, 0.25 along x), a prismatic z joint
    and a revolute z joint: planar position, height 0.4 + d - 0.05, yaw the
    sum of the angles."""
    tree = synth.scara4()
    # the tree's FP32-rounded lengths
    l1, l2, h, e = tree.offset[1][0], tree.offset[2][0], tree.offset[0][2], tree.ee_offset[0][2]
    for t1, t2, d, t4 in [(0.3, -0.7, 0.1, 1.2), (-2.0, 1.5, -0.15, -0.4), (0, 0, 0, 0)]:
        _, _, Re, pe = ora.fk(tree, np.array([t1, t2, d, t4]))
        x = l1 * math.cos(t1) + l2 * math.cos(t1 + t2)
        y = l1 * math.sin(t1) + l2 * math.sin(t1 + t2)
        np.testing.assert_allclose(pe[0], [x, y, h + d + e], atol=1e-14)
        yaw = t1 + t2 + t4
        np.testing.assert_allclose(Re[0], [[math.cos(yaw), -math.sin(yaw), 0],
                                           [math.sin(yaw), math.cos(yaw), 0], [0, 0, 1]], atol=1e-14)


def test_fk_mobile_base_is_se2_times_arm(ora):
    """The planar base (x, y, yaw) composes as T_world<-base = Trans(x, y, 0)
    Rz(yaw) in front of the arm's own FK (Sec. V-B)."""
    arm, mob = synth.arm7(0), synth.mobile_arm7(0)
    for q in synth.uniform_configs(mob, 10, 7):
        _, _, Re, pe = ora.fk(mob, q)
        _, _, Ra, pa = ora.fk(arm, q[3:])
        c, s_ = math.cos(q[2]), math.sin(q[2])
        Rz = np.array([[c, -s_, 0], [s_, c, 0], [0, 0, 1.0]])
        np.testing.assert_allclose(Re[0], Rz @ Ra[0], atol=1e-13)
        np.testing.assert_allclose(pe[0], Rz @ pa[0] + [q[0], q[1], 0], atol=1e-13)


def test_fixed_joints_fold_into_their_neighbours(ora):
    """A fixed joint is the same as composing its transform into the next
    joint's mount and offset (and the EE's): the tool arm against a revolute
    arm built with the folded transforms by hand."""
    tool = synth.arm7_tool(0)
    arm = synth.arm7(0)

    def rot(wxyz):
        return Rotation.from_quat([wxyz[1], wxyz[2], wxyz[3], wxyz[0]]).as_matrix()
    Rf, Rt = rot(tool.mount_quat[4]), rot(tool.mount_quat[8])     # flange, tool (as stored)
    assert tool.types[4] == tool.types[8] == synth.JOINT_FIXED
    folded = synth.Tree("folded", arm.parent.copy(), arm.mount_quat.copy(), arm.offset.copy(),
                        arm.axis.copy(), arm.lower.copy(), arm.upper.copy(), arm.ee_joint.copy(),
                        arm.ee_offset.copy(), arm.ee_quat.copy(), arm.ee_kind.copy())
    # joint 4 hangs off the flange: offset 0.05 z then Rf, then its own offset and mount
    folded.offset[4] = tool.offset[4] + Rf @ arm.offset[4]
    m4 = Rotation.from_quat(np.r_[arm.mount_quat[4][1:], arm.mount_quat[4][0]]).as_matrix()
    qf = Rotation.from_matrix(Rf @ m4).as_quat()
    folded.mount_quat[4] = np.r_[qf[3], qf[:3]]
    folded.ee_offset[0] = tool.offset[8] + Rt @ arm.ee_offset[0]
    qe = Rotation.from_matrix(Rt).as_quat()
    folded.ee_quat[0] = np.r_[qe[3], qe[:3]]
    for q in synth.uniform_configs(arm, 10, 9):
        _, _, Ra, pa = ora.fk(tool, q)
        _, _, Rb, pb = ora.fk(folded, q)
        np.testing.assert_allclose(Ra, Rb, atol=1e-13)
        np.testing.assert_allclose(pa, pb, atol=1e-13)


def test_prismatic_column_is_the_world_axis(ora):
    """Position EE below a prismatic joint: d p_ee / d q = the joint's world
    axis (closed form, no rotation part)."""
    tree = synth.scara4()
    q = np.array([0.4, -0.3, 0.05, 0.9])
    tg = ora.targets_from(tree, q[None])[0]
    w = dict(WEIGHTS, w_pos=1.0, w_rot=1.0, w_limit=0.0, w_rest=0.0)
    J = ora.jacobian(tree, tg, w, q)
    # at the target itself the pose log is zero, J_r^-1 = I and R_ee^T maps
    # the world z axis to the EE's z axis, which is world z here
    np.testing.assert_allclose(J[:6, 2], [0, 0, 1, 0, 0, 0], atol=1e-12)


def test_mimic_joints_equal_the_expanded_hand(ora):
    """A mimic joint takes mult * q_driver + offset: the coupled hand's FK at
    12 variables equals the uncoupled hand's at the expanded 16 values, and
    its Jacobian is the uncoupled one with each mimic column added into its
    driver's (times mult) and dropped."""
    hm, h = synth.hand16_mimic(8), synth.hand16(8)
    tg = ora.targets_from(h, synth.uniform_configs(h, 4, 41))
    w = dict(WEIGHTS, w_rest=0.0, w_limit=0.0)
    for i, q in enumerate(synth.uniform_configs(hm, 4, 40)):
        full = np.zeros(16)
        full[hm.var_joints] = q
        for j in range(16):
            if hm.mimics[j] >= 0:
                full[j] = hm.mimic_multiplier[j] * full[hm.mimics[j]] + hm.mimic_offset[j]
        _, _, Ra, pa = ora.fk(hm, q)
        _, _, Rb, pb = ora.fk(h, full)
        np.testing.assert_array_equal(Ra, Rb)
        np.testing.assert_array_equal(pa, pb)
        Jm = ora.jacobian(hm, tg[i], w, q)
        Jf = ora.jacobian(h, tg[i], w, full)
        want = Jf[:12].copy()
        for j in range(16):
            if hm.mimics[j] >= 0:
                want[:, hm.mimics[j]] += hm.mimic_multiplier[j] * want[:, j]
        np.testing.assert_allclose(Jm[:12], want[:, hm.var_joints], rtol=1e-12, atol=1e-14)

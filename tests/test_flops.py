"""Host logic: the algorithmic FLOP model used by the benchmark."""
import synth
from paper_2505_03728_amd.flops import ancestors, lm_flops, per_unit, tree_solve_flops


def test_ancestor_counts():
    assert ancestors(synth.arm7(0).parent, synth.arm7(0).ee_joint) == [7]
    assert ancestors(synth.tree34(5).parent, synth.tree34(5).ee_joint) == [13] * 4
    assert ancestors(synth.hand16(8).parent, synth.hand16(8).ee_joint) == [4] * 4


def test_arm_counts():
    a = synth.arm7(0)
    trial, acc = per_unit(a.parent, a.ee_joint, a.ee_kind, [7])
    # FK 270 + residual 140 + limit/rest 63 + damping 21 + Cholesky 343/3 + solves 98
    assert abs(trial - (270 + 140 + 63 + 21 + 343 / 3 + 98)) < 1e-9
    # Jacobian 96*7+175, J^T J 12*28, J^T r 12*7
    assert acc == 96 * 7 + 175 + 12 * 28 + 12 * 7
    assert abs(lm_flops(a.parent, a.ee_joint, a.ee_kind, [7], 10, 4, 1) - (11 * trial + 5 * acc)) < 1e-6


def test_tree_factor_counts():
    # tree34: torso chain of 6 (depths 0..5), four arms of 7 (depths 6..12)
    t = synth.tree34(5)
    torso = sum(d * (d + 1) + d for d in range(6)) + 4 * sum(range(6))
    arm = sum(d * (d + 1) + d for d in range(6, 13)) + 4 * sum(range(6, 13))
    assert tree_solve_flops(t.parent) == torso + 4 * arm == 2969 + 1068
    # a chain reduces to ~n^3/3: the 7-chain factor is 112 + 21, solves 84
    a = synth.arm7(0)
    assert tree_solve_flops(a.parent) == 112 + 21 + 84
    dense, _ = per_unit(t.parent, t.ee_joint, t.ee_kind, [t.n])
    sparse, _ = per_unit(t.parent, t.ee_joint, t.ee_kind, None)
    assert abs(dense - sparse - (34 ** 3 / 3 + 2 * 34 ** 2 - 4037)) < 1e-9

"""Algorithmic work of one LM problem-iteration (FLOPs, FMA = 2).

Counted over structural nonzeros only (a joint's Jacobian column is nonzero
only for the EEs it is an ancestor of), with the minimal per-step schedule:
every trial evaluates FK, residuals and the damped factor/solve; an accepted
trial additionally forms the Jacobian, J^T J and J^T r at the new point.
Transcendentals (sin/cos, sqrt, atan2, divisions) are not counted.

Per term (n joints, m EEs, a_k ancestors of EE k):
  FK                 36 n + 18 m
  pose residual      140 per pose EE, 12 per position EE
  limit + rest       9 n
  Jacobian           96 a_k + 175 per pose EE, 12 a_k per position EE
  J^T J              12 a_k (a_k + 1) / 2 pose, 6 a_k (a_k + 1) / 2 position
  J^T r              12 a_k pose, 6 a_k position
  Cholesky           b^3 / 3 per factored block of size b
  triangular solves  2 b^2 per block
  damping + update   3 n
or, for the leaves-first tree factorization (blocks=None; d_k = number of
proper ancestors of joint k, the factor has no fill):
  L^T D L factor     sum_k d_k (d_k + 1) + d_k
  triangular solves  4 sum_k d_k
"""
from __future__ import annotations


def ancestors(parent, ee_joint):
    out = []
    for e in ee_joint:
        a, c = int(e), 0
        while a >= 0:
            c += 1
            a = int(parent[a])
        out.append(c)
    return out


def depths(parent):
    d = []
    for j, p in enumerate(parent):
        d.append(0 if int(p) < 0 else d[int(p)] + 1)
    return d


def tree_solve_flops(parent):
    """Leaves-first L^T D L factor of a tree-structured J^T J plus both solves."""
    ds = depths(parent)
    return float(sum(d * (d + 1) + d for d in ds) + 4 * sum(ds))


def per_unit(parent, ee_joint, ee_kind, blocks):
    """(FLOPs per trial, extra FLOPs per accepted trial).  blocks: sizes of
    the dense diagonal blocks factored, or None for the tree factorization."""
    n, m = len(parent), len(ee_joint)
    anc = ancestors(parent, ee_joint)
    trial = 36 * n + 18 * m + 9 * n + 3 * n
    acc = 0
    for a, kind in zip(anc, ee_kind):
        if int(kind) == 0:
            trial += 140
            acc += 96 * a + 175 + 12 * a * (a + 1) // 2 + 12 * a
        else:
            trial += 12
            acc += 12 * a + 6 * a * (a + 1) // 2 + 6 * a
    if blocks is None:
        trial += tree_solve_flops(parent)
    else:
        for b in blocks:
            trial += b ** 3 / 3.0 + 2 * b * b
    return float(trial), float(acc)


def lm_flops(parent, ee_joint, ee_kind, blocks, iters, accepts, problems):
    """Total algorithmic FLOPs of a solve from its per-problem counters.

    iters/accepts: totals over the batch; problems: batch size (each pays
    one initial evaluation with Jacobian)."""
    trial, acc = per_unit(parent, ee_joint, ee_kind, blocks)
    init = trial + acc
    return float(iters) * trial + float(accepts) * acc + float(problems) * init


# Algorithmic HBM bytes per problem of a solve: seeds in and joints out
# (4 n each), per-EE errors (8 m), and 4 bytes per per-problem scalar output
# (by default all six: cost, pose-only cost, iterations, accepts, status,
# iterations-to-tolerance); targets (4 * target floats) once per target.
def lm_bytes(n, m, target_floats, problems, targets, scalars=6):
    return problems * (8 * n + 8 * m + 4 * scalars) + targets * 4 * target_floats

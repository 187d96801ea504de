"""Pins for the oracle's SO(3)/SE(3) arithmetic.

The pose residual of Sec. III-C is log(T_target^-1 T_i); its analytic
Jacobian needs the SE(3) right-Jacobian inverse.  Each function here is
checked against something other than itself: scipy's matrix exponential and
logarithm (generic Pade / Schur algorithms), scipy's Rotation class, finite
differences through those, closed forms, and continuity across the series
thresholds.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm, logm
from scipy.spatial.transform import Rotation

rng = np.random.default_rng(1234)


def hat(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0.0]])


def twist(xi):
    M = np.zeros((4, 4))
    M[:3, :3] = hat(xi[3:])
    M[:3, 3] = xi[:3]
    return M


def vee_twist(M):
    return np.array([M[0, 3], M[1, 3], M[2, 3], M[2, 1], M[0, 2], M[1, 0]])


def se3_expm(xi):
    return expm(twist(xi))


def se3_logm(T):
    return vee_twist(np.real(logm(T)))


def rand_xi(max_theta=3.0):
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    return np.concatenate([rng.normal(size=3) * 0.7, axis * rng.uniform(0.05, max_theta)])


def test_so3_exp_matches_scipy(ora):
    for _ in range(50):
        phi = rng.normal(size=3) * rng.uniform(0, 3)
        R = ora.so3_exp(phi)
        np.testing.assert_allclose(R, Rotation.from_rotvec(phi).as_matrix(), atol=1e-13)
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1.0) < 1e-13


def test_so3_log_matches_scipy_and_round_trips(ora):
    for _ in range(50):
        phi = rng.normal(size=3)
        phi *= rng.uniform(1e-6, math.pi - 2e-3) / np.linalg.norm(phi)
        R = Rotation.from_rotvec(phi).as_matrix()
        np.testing.assert_allclose(ora.so3_log(R), phi, atol=1e-12)
        np.testing.assert_allclose(ora.so3_exp(ora.so3_log(R)), R, atol=1e-12)


def test_so3_log_known_values(ora):
    for th in [0.0, 1e-9, 0.3, 2.0, math.pi - 1e-6]:
        c, s = math.cos(th), math.sin(th)
        Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
        np.testing.assert_allclose(ora.so3_log(Rz), [0, 0, th], atol=1e-9)
    np.testing.assert_allclose(ora.so3_log(np.eye(3)), 0.0, atol=0)


@pytest.mark.parametrize("eps", [0.0, 1e-9, 1e-6, 1e-4, 5e-4])
def test_so3_log_near_pi(ora, eps):
    for _ in range(20):
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        th = math.pi - eps
        R = Rotation.from_rotvec(a * th).as_matrix()
        phi = ora.so3_log(R)
        np.testing.assert_allclose(np.linalg.norm(phi), th, atol=1e-7)
        np.testing.assert_allclose(ora.so3_exp(phi), R, atol=1e-7)
        if eps > 0:
            # Sign is fixed by the antisymmetric part when it does not vanish.
            np.testing.assert_allclose(phi, a * th, atol=2e-5)


def test_se3_exp_log_match_matrix_exponential(ora):
    for _ in range(40):
        xi = rand_xi()
        R, t = ora.se3_exp(xi)
        T = se3_expm(xi)
        np.testing.assert_allclose(R, T[:3, :3], atol=1e-12)
        np.testing.assert_allclose(t, T[:3, 3], atol=1e-12)
        np.testing.assert_allclose(ora.se3_log(R, t), xi, atol=1e-11)
        np.testing.assert_allclose(se3_logm(T), xi, atol=1e-9)


def test_se3_log_special_cases(ora):
    t = np.array([0.3, -0.2, 0.7])
    np.testing.assert_allclose(ora.se3_log(np.eye(3), t), np.r_[t, 0, 0, 0], atol=0)
    th = 1.1
    c, s = math.cos(th), math.sin(th)
    Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
    np.testing.assert_allclose(ora.se3_log(Rz, np.zeros(3)), [0, 0, 0, 0, 0, th], atol=1e-15)


def _fd_right(xi, h=1e-6):
    """d/dh log(exp(xi) exp(h e_i)) by central differences through scipy."""
    T = se3_expm(xi)
    J = np.zeros((6, 6))
    for i in range(6):
        e = np.zeros(6)
        e[i] = h
        J[:, i] = (se3_logm(T @ se3_expm(e)) - se3_logm(T @ se3_expm(-e))) / (2 * h)
    return J


def _fd_left(xi, h=1e-6):
    T = se3_expm(xi)
    J = np.zeros((6, 6))
    for i in range(6):
        e = np.zeros(6)
        e[i] = h
        J[:, i] = (se3_logm(se3_expm(e) @ T) - se3_logm(se3_expm(-e) @ T)) / (2 * h)
    return J


@pytest.mark.parametrize("theta", [1e-3, 5e-3, 0.02, 0.4, 1.5, 2.8])
def test_se3_jacobian_inverses_by_finite_differences(ora, theta):
    for _ in range(5):
        xi = rand_xi()
        xi[3:] *= theta / np.linalg.norm(xi[3:])
        np.testing.assert_allclose(ora.se3_jr_inv(xi), _fd_right(xi), atol=2e-7)
        np.testing.assert_allclose(ora.se3_jl_inv(xi), _fd_left(xi), atol=2e-7)


def test_se3_jacobian_at_zero_is_identity(ora):
    np.testing.assert_allclose(ora.se3_jr_inv(np.zeros(6)), np.eye(6), atol=0)
    np.testing.assert_allclose(ora.se3_jl_inv(np.zeros(6)), np.eye(6), atol=0)


def test_so3_left_jacobian_by_finite_differences(ora):
    # exp(phi + h e_i) = exp(J_l(phi) h e_i) exp(phi) to first order.
    for _ in range(10):
        phi = rng.normal(size=3) * rng.uniform(0.01, 2.5)
        R0 = Rotation.from_rotvec(phi).as_matrix()
        J = np.zeros((3, 3))
        h = 1e-6
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            Rp = Rotation.from_rotvec(phi + e).as_matrix() @ R0.T
            Rm = Rotation.from_rotvec(phi - e).as_matrix() @ R0.T
            J[:, i] = (Rotation.from_matrix(Rp).as_rotvec()
                       - Rotation.from_matrix(Rm).as_rotvec()) / (2 * h)
        np.testing.assert_allclose(ora.so3_jl(phi), J, atol=1e-8)
        np.testing.assert_allclose(ora.so3_jl_inv(phi), np.linalg.inv(J), atol=1e-7)


@pytest.mark.parametrize("name,thr", [("so3_jl_inv", 1e-3), ("so3_jl", 1e-3),
                                      ("so3_exp", 1e-4)])
def test_series_branches_are_continuous(ora, name, thr):
    f = getattr(ora, name)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    lo, hi = f(a * thr * (1 - 1e-9)), f(a * thr * (1 + 1e-9))
    np.testing.assert_allclose(lo, hi, atol=1e-12)


def test_q_matrix_series_branch_is_continuous(ora):
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    rho = rng.normal(size=3)
    lo = ora.se3_Q(rho, a * 1e-2 * (1 - 1e-9))
    hi = ora.se3_Q(rho, a * 1e-2 * (1 + 1e-9))
    np.testing.assert_allclose(lo, hi, atol=1e-12)


def test_q_matrix_is_block_of_the_left_jacobian(ora):
    # The SE(3) left Jacobian [[J, Q], [0, J]] is the FD derivative of
    # exp; its inverse must therefore invert the FD left Jacobian of log.
    for _ in range(5):
        xi = rand_xi()
        Jl = np.zeros((6, 6))
        Jl[:3, :3] = Jl[3:, 3:] = ora.so3_jl(xi[3:])
        Jl[:3, 3:] = ora.se3_Q(xi[:3], xi[3:])
        np.testing.assert_allclose(Jl @ ora.se3_jl_inv(xi), np.eye(6), atol=1e-12)

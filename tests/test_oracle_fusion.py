"""Pins of the oracle's pose fusion between successive clusters (Sec. 3.2,
Eq. (8)): a match-count weighted mean of two poses, positions linear,
rotations on SO(3).

Independent checks: scipy's quaternion Slerp (another library's geodesic
interpolation), the closed form for rotations about one axis (the weighted
mean of the angles), the special cases w_new = 0, w_old = 0 and equal poses,
symmetry under swapping the two poses with their weights, distances along
the geodesic, and the running mean of positions over a chain of fusions.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation as Rot, Slerp

import oracle


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def angle(A, B):
    return Rot.from_matrix(A.T @ B).magnitude()


def test_exp_matches_scipy_rotvec():
    rng = np.random.default_rng(3)
    for w in list(rng.normal(size=(20, 3))) + [np.array([1e-9, -2e-9, 3e-10]), np.zeros(3),
                                               np.array([0.0, 0.0, np.pi - 1e-7])]:
        assert np.abs(oracle.so3_exp(w) - Rot.from_rotvec(w).as_matrix()).max() < 1e-14


@pytest.mark.parametrize("theta", [0.0, 1e-12, 1e-7, 1e-3, 0.5, 2.0, np.pi - 1e-4, np.pi - 1e-8])
def test_log_matches_scipy_rotvec(theta):
    rng = np.random.default_rng(int(theta * 1e6) % 1000)
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    R = Rot.from_rotvec(theta * ax).as_matrix()
    got = oracle.so3_log(R)
    # Near pi the skew part of R vanishes and the axis is conditioned by
    # 1 / (pi - theta): looser bounds there.
    near_pi = theta > np.pi - 1e-3
    assert np.abs(got - theta * ax).max() < (1e-7 if near_pi else 1e-14)
    assert np.abs(oracle.so3_exp(got) - R).max() < (1e-12 if near_pi else 1e-14)


def test_fused_rotation_is_scipy_slerp():
    rng = np.random.default_rng(11)
    for _ in range(50):
        A, B = Rot.random(2, random_state=rng).as_matrix()
        wo, wn = rng.integers(1, 500, 2).astype(float)
        R, _, _ = oracle.fuse_pose(A, np.zeros(3), wo, B, np.zeros(3), wn)
        ref = Slerp([0.0, 1.0], Rot.from_matrix([A, B]))([wn / (wo + wn)]).as_matrix()[0]
        # random pairs reach relative angles near pi, where Log loses digits
        assert np.abs(R - ref).max() < 1e-12


def test_common_axis_averages_angles():
    """Rotations about one axis: the fused angle is the weighted mean angle."""
    for a, b, wo, wn in [(0.1, 0.4, 30, 10), (-0.2, 0.3, 1, 3), (1.0, 1.0 + 1e-5, 250, 17), (-3.0, -0.5, 2, 2)]:
        R, _, _ = oracle.fuse_pose(rot_z(a), np.zeros(3), wo, rot_z(b), np.zeros(3), wn)
        assert np.abs(R - rot_z((wo * a + wn * b) / (wo + wn))).max() < 1e-15 * 8


def test_fused_position_and_weight():
    To, Tn = np.array([4.0e6, 1.0e6, 300.0]), np.array([4.0e6 + 3.0, 1.0e6 - 1.5, 302.0])
    _, T, w = oracle.fuse_pose(np.eye(3), To, 3.0, np.eye(3), Tn, 1.0)
    assert w == 4.0
    assert np.array_equal(T, (3.0 * To + Tn) / 4.0)
    assert np.abs(T - np.array([4.0e6 + 0.75, 1.0e6 - 0.375, 300.5])).max() < 1e-9


def test_zero_weights():
    rng = np.random.default_rng(5)
    A, B = Rot.random(2, random_state=rng).as_matrix()
    To, Tn = rng.normal(size=3), rng.normal(size=3)
    R, T, w = oracle.fuse_pose(A, To, 7.0, B, Tn, 0.0)      # nothing new: the old pose stays
    assert np.abs(R - A).max() < 1e-15 and np.array_equal(T, To) and w == 7.0
    R, T, w = oracle.fuse_pose(A, To, 0.0, B, Tn, 9.0)      # nothing stored: the new pose is written
    assert np.array_equal(R, B) and np.array_equal(T, Tn) and w == 9.0


def test_equal_poses_stay():
    R0 = Rot.from_rotvec([0.3, -0.2, 1.1]).as_matrix()
    T0 = np.array([1.0, 2.0, 3.0])
    R, T, w = oracle.fuse_pose(R0, T0, 5.0, R0, T0, 8.0)
    assert np.abs(R - R0).max() < 1e-15 and np.abs(T - T0).max() < 1e-15 and w == 13.0


def test_symmetric_in_the_two_poses():
    rng = np.random.default_rng(8)
    for _ in range(20):
        A, B = Rot.random(2, random_state=rng).as_matrix()
        Ta, Tb = rng.normal(size=(2, 3))
        wa, wb = rng.uniform(1, 50, 2)
        R1, T1, _ = oracle.fuse_pose(A, Ta, wa, B, Tb, wb)
        R2, T2, _ = oracle.fuse_pose(B, Tb, wb, A, Ta, wa)
        assert np.abs(R1 - R2).max() < 1e-13 and np.abs(T1 - T2).max() < 1e-14


def test_geodesic_distances_split_by_weight():
    rng = np.random.default_rng(9)
    for _ in range(20):
        A, B = Rot.random(2, random_state=rng).as_matrix()
        wo, wn = rng.uniform(1, 50, 2)
        R, _, _ = oracle.fuse_pose(A, np.zeros(3), wo, B, np.zeros(3), wn)
        d = angle(A, B)
        assert abs(np.linalg.det(R) - 1.0) < 1e-14 and np.abs(R.T @ R - np.eye(3)).max() < 1e-14
        assert abs(angle(A, R) - wn / (wo + wn) * d) < 1e-12
        assert abs(angle(R, B) - wo / (wo + wn) * d) < 1e-12


def test_chain_of_fusions_is_the_running_mean():
    """Fusing n poses one after another, with accumulated weights, gives the
    weighted mean of the positions and, about one axis, of the angles."""
    rng = np.random.default_rng(12)
    Ts = rng.normal(size=(6, 3)) * 10
    ang = rng.uniform(-0.4, 0.4, 6)
    ws = rng.integers(5, 80, 6).astype(float)
    R, T, w = rot_z(ang[0]), Ts[0], ws[0]
    for i in range(1, 6):
        R, T, w = oracle.fuse_pose(R, T, w, rot_z(ang[i]), Ts[i], ws[i])
    assert w == ws.sum()
    assert np.abs(T - np.average(Ts, axis=0, weights=ws)).max() < 1e-13
    assert np.abs(R - rot_z(np.average(ang, weights=ws))).max() < 1e-14

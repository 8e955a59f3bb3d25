"""Pins of quaternion/rotation and geometry oracle code (Sec. 2.1, App. B)."""
import json
import os

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import bodies, quat
from paper_2107_10800_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _scipy(theta):
    return Rotation.from_quat(np.concatenate([theta[..., 1:], theta[..., :1]], -1))


def test_rotation_matrix_against_scipy():
    rng = np.random.default_rng(0)
    rot = Rotation.random(50, random_state=rng)
    xyzw = rot.as_quat()
    theta = np.concatenate([xyzw[:, 3:], xyzw[:, :3]], 1)
    assert np.allclose(quat.rotation_matrix(theta), rot.as_matrix(), atol=1e-15)


def test_rotation_properties():
    rng = np.random.default_rng(1)
    t = rng.standard_normal((20, 4))
    t /= np.linalg.norm(t, axis=1)[:, None]
    R = quat.rotation_matrix(t)
    assert np.allclose(R @ R.transpose(0, 2, 1), np.eye(3), atol=1e-15)
    assert np.allclose(np.linalg.det(R), 1.0)
    # double cover: theta and -theta give the same rotation
    assert np.allclose(quat.rotation_matrix(-t), R, atol=1e-15)
    # R(t2 . t1) = R(t2) R(t1)  (App. B)
    t2 = np.roll(t, 1, axis=0)
    assert np.allclose(quat.rotation_matrix(quat.quat_mul(t2, t)), R[np.r_[19, 0:19]] @ R,
                       atol=1e-14)


def test_finite_rotation_quaternion():
    # a quarter turn about z takes e_x to e_y; small rotations give I + gamma^x
    R = quat.rotation_matrix(quat.quat_from_rotvec(np.array([0, 0, np.pi / 2])))
    assert np.allclose(R @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    g = np.array([1e-7, -2e-7, 3e-7])
    R = quat.rotation_matrix(quat.quat_from_rotvec(g))
    assert np.allclose(R, np.eye(3) + quat.cross_matrix(g), atol=1e-13)
    assert np.allclose(quat.quat_from_rotvec(np.zeros(3)), [1, 0, 0, 0])


def test_blob_positions_against_scipy():
    wl = W.bacteria(n_bact=8, seed=11)
    r = bodies.blob_positions(wl.q, wl.theta, wl.r_ref, wl.blob_offset)
    body = bodies.body_of_blob(wl.blob_offset)
    rs = np.vstack([wl.q[p] + _scipy(wl.theta[p]).apply(wl.r_ref[i])
                    for i, p in enumerate(body)])
    assert np.allclose(r, rs, atol=1e-12)


def test_filament_joints_coincide():
    # robot-arm layout (Eq. robot-arm): every joint satisfied to rounding
    wl = W.filament()
    g = bodies.link_residual(wl, wl.q, wl.theta)
    assert np.abs(g).max() < 1e-13


def test_bacteria_geometry():
    wl = W.bacteria(n_bact=16, seed=12)
    assert wl.N == 16 * 122 and wl.M == 32 and wl.n_rows == 16 * 6
    r = bodies.blob_positions(wl.q, wl.theta, wl.r_ref, wl.blob_offset)
    assert r[:, 2].min() >= 1.5
    # hinge links satisfied at t = 0 (both arms lie on the shared axis)
    assert np.abs(bodies.link_residual(wl, wl.q, wl.theta)).max() < 1e-12
    # minimum distance between blobs of different bacteria >= 2a
    bact = bodies.body_of_blob(wl.blob_offset) // 2
    d = np.linalg.norm(r[:, None] - r[None], axis=2)
    other = bact[:, None] != bact[None, :]
    assert d[other].min() >= 2.0
    ico = W.icosphere42(5.0)
    dd = np.linalg.norm(ico[:, None] - ico[None], axis=2)
    assert np.allclose(np.linalg.norm(ico, axis=1), 5.0)
    assert abs(np.sort(dd[dd > 0])[0] - np.sort(dd[dd > 0])[:120].max()) < 0.6


def test_diatom_links_coincide():
    wl = W.diatoms(n_col=4, seed=13)
    assert np.abs(bodies.link_residual(wl, wl.q, wl.theta)).max() < 1e-12
    assert wl.r_ref.shape[0] == 45 * wl.M


def test_printed_system_sizes():
    g = json.load(open(os.path.join(GOLD, "paper_sizes.json")))
    for c in g["cases"]:
        n = 3 * c["blobs_counted"] + 6 * c["bodies"] + 3 * c["links"]
        assert n == c["n"], c["cite"]
    for c in g["ratios"]:
        assert abs(3 * c["links"] / (6 * c["bodies"]) - c["ratio"]) < 0.005


def test_matrix_free_rigid_operators_match_dense():
    # K U, K^T lambda and the sparse C of the oracle against its dense K and C
    wl = W.bacteria(n_bact=3, side=50.0, seed=31)
    r = bodies.blob_positions(wl.q, wl.theta, wl.r_ref, wl.blob_offset)
    K = bodies.K_matrix(r, wl.q, wl.blob_offset)
    rng = np.random.default_rng(8)
    U = rng.standard_normal(6 * wl.M)
    lam = rng.standard_normal(3 * wl.N)
    assert np.allclose(bodies.K_apply(r, wl.q, wl.blob_offset, U).ravel(), K @ U,
                       rtol=0, atol=1e-13 * np.abs(K @ U).max())
    assert np.allclose(bodies.KT_apply(r, wl.q, wl.blob_offset, lam).ravel(), K.T @ lam,
                       rtol=0, atol=1e-13 * np.abs(K.T @ lam).max())
    C, B = bodies.constraint_rows(wl)
    Cs, Bs = bodies.constraint_rows(wl, sparse=True)
    assert np.array_equal(Cs.toarray(), C) and np.array_equal(Bs, B)

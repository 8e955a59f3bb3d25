"""Unit quaternions theta = [s, p] (scalar first) and rotations.

Paper: Sec. 2.1 (finite-rotation quaternion, Eq. quaternion_mult) and App. B
(Eq. rot_mat).
"""
import numpy as np


def quat_mul(t2, t1):
    """theta_3 = theta_2 . theta_1: rotation theta_1 followed by theta_2
    (Eq. quaternion_mult).  Works on (...,4) arrays."""
    t2 = np.asarray(t2, float)
    t1 = np.asarray(t1, float)
    s2, p2 = t2[..., 0], t2[..., 1:]
    s1, p1 = t1[..., 0], t1[..., 1:]
    s = s2 * s1 - np.sum(p2 * p1, axis=-1)
    p = s2[..., None] * p1 + s1[..., None] * p2 + np.cross(p2, p1)
    return np.concatenate([s[..., None], p], axis=-1)


def quat_from_rotvec(gamma):
    """Quaternion of the finite rotation by vector gamma: [cos(g/2), sin(g/2) gamma/g]
    (Sec. 2.1).  gamma = 0 gives the identity."""
    gamma = np.asarray(gamma, float)
    g = np.linalg.norm(gamma, axis=-1)
    out = np.zeros(gamma.shape[:-1] + (4,))
    out[..., 0] = np.cos(g / 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        fac = np.where(g > 0, np.sin(g / 2) / np.where(g > 0, g, 1), 0.5)
    out[..., 1:] = fac[..., None] * gamma
    return out


def rotation_matrix(theta):
    """R = 2 [p p^T + s p^x + (s^2 - 1/2) I]  (App. B, Eq. rot_mat), where
    p^x x = p cross x.  Works on (...,4) arrays, returns (...,3,3)."""
    theta = np.asarray(theta, float)
    s = theta[..., 0]
    p = theta[..., 1:]
    ppT = p[..., :, None] * p[..., None, :]
    px = np.zeros(theta.shape[:-1] + (3, 3))
    px[..., 0, 1] = -p[..., 2]
    px[..., 0, 2] = p[..., 1]
    px[..., 1, 0] = p[..., 2]
    px[..., 1, 2] = -p[..., 0]
    px[..., 2, 0] = -p[..., 1]
    px[..., 2, 1] = p[..., 0]
    eye = np.broadcast_to(np.eye(3), px.shape)
    return 2.0 * (ppT + s[..., None, None] * px + (s * s - 0.5)[..., None, None] * eye)


def cross_matrix(v):
    """v^x such that v^x w = v cross w."""
    v = np.asarray(v, float)
    m = np.zeros(v.shape[:-1] + (3, 3))
    m[..., 0, 1] = -v[..., 2]
    m[..., 0, 2] = v[..., 1]
    m[..., 1, 0] = v[..., 2]
    m[..., 1, 2] = -v[..., 0]
    m[..., 2, 0] = -v[..., 1]
    m[..., 2, 1] = v[..., 0]
    return m

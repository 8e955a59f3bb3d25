"""Generalised RPY mobility of single-blob bodies, unbounded (Sec. 2.4), float64.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 2.4 represents a rigid body by one blob that carries a force f and a
torque tau and moves with velocity u and angular velocity w; the body
mobility N is then the generalised Rotne-Prager-Yamakawa tensor cited there
(Wajnryb et al.), i.e. Eq. RPY extended to rotations: the force is spread
uniformly over the sphere |x - r_j| = a, the torque as the surface density
3/(8 pi a^3) tau x n, and u_i, w_i are the surface averages of v and of
(3/(2a)) n x v over the sphere around r_i, v the Stokes flow of that density.
Written out for equal radii a, r = r_i - r_j, r = |r|, rhat = r / r, in units
of 1/(8 pi eta):

  translation-translation (u_i from f_j): the RPY tensor of oracle.rpy
  rotation-translation (w_i from f_j):  c_r f_j x r
  translation-rotation (u_i from tau_j): c_r tau_j x r
  rotation-rotation (w_i from tau_j):   d_1 tau_j + d_2 (r . tau_j) r
  with, for r > 2a,   c_r = 1/r^3,               d_1 = -1/(2 r^3),  d_2 = 3/(2 r^5)
       for r <= 2a,   c_r = (1 - 3r/(8a)) / (2 a^3),
                      d_1 = (1 - 27r/(32a) + 5r^3/(64a^3)) / a^3,
                      d_2 = (9/(32 a r) - 3r/(64 a^3)) / a^3   (d_2 r r^T -> 0 at r = 0).
  At r = 0 the blocks are the self mobilities I/(6 pi eta a) and I/(8 pi eta a^3).

Per body the generalised vectors are ordered (u, w) and (f, tau), as the body
velocities U_p and forces F_p of Eq. linear_system.

Reading: the paper applies this model only in an unbounded domain (its
filament and shell tests); the rotational couplings above a wall are not
written here.
"""
from __future__ import annotations

import numpy as np

from .rpy import rpy_free_blocks


def _cross_mat(v):
    """[v]_x with [v]_x w = v x w, (...,3,3)."""
    m = np.zeros(v.shape[:-1] + (3, 3))
    m[..., 0, 1] = -v[..., 2]
    m[..., 0, 2] = v[..., 1]
    m[..., 1, 0] = v[..., 2]
    m[..., 1, 2] = -v[..., 0]
    m[..., 2, 0] = -v[..., 1]
    m[..., 2, 1] = v[..., 0]
    return m


def rot_coefficients(r, a):
    """(c_r, d_1, d_2) of the module header in units of 1/(8 pi eta), arrays."""
    r = np.asarray(r, float)
    with np.errstate(divide="ignore", invalid="ignore"):
        rs = np.where(r > 0, r, 1.0)
        far = (1.0 / rs ** 3, -0.5 / rs ** 3, 1.5 / rs ** 5)
        near = ((1 - 3 * r / (8 * a)) / (2 * a ** 3),
                (1 - 27 * r / (32 * a) + 5 * r ** 3 / (64 * a ** 3)) / a ** 3,
                np.where(r > 0, (9 / (32 * a * rs) - 3 * r / (64 * a ** 3)) / a ** 3, 0.0))
    ov = r <= 2 * a
    return tuple(np.where(ov, n, f) for n, f in zip(near, far))


def pair_blocks(rvec, a, eta):
    """6x6 blocks [[tt, tr], [rt, rr]] for separation vectors rvec (...,3): the
    generalised velocity of blob i per unit generalised force on blob j."""
    rvec = np.asarray(rvec, float)
    r = np.linalg.norm(rvec, axis=-1)
    cr, d1, d2 = rot_coefficients(r, a)
    k = 1.0 / (8 * np.pi * eta)
    out = np.zeros(rvec.shape[:-1] + (6, 6))
    out[..., :3, :3] = rpy_free_blocks(rvec, a, eta)
    # w_i = c_r f_j x r = -c_r [r]_x f_j;  u_i = c_r tau_j x r likewise
    rx = _cross_mat(rvec)
    out[..., 3:, :3] = -k * cr[..., None, None] * rx
    out[..., :3, 3:] = -k * cr[..., None, None] * rx
    rr = rvec[..., :, None] * rvec[..., None, :]
    out[..., 3:, 3:] = k * (d1[..., None, None] * np.eye(3) + d2[..., None, None] * rr)
    return out


def body_mobility(pos, a, eta):
    """The 6M x 6M body mobility N of single-blob bodies at positions pos (M,3),
    body p occupying rows/columns 6p .. 6p+5 as (u, w) / (f, tau)."""
    pos = np.asarray(pos, float)
    M = len(pos)
    B = pair_blocks(pos[:, None, :] - pos[None, :, :], a, eta)     # (M,M,6,6)
    return B.transpose(0, 2, 1, 3).reshape(6 * M, 6 * M)


def body_mobility_apply(pos, FT, a, eta):
    """N (f, tau) for generalised forces FT (M,6), as a (M,6) array."""
    return (body_mobility(pos, a, eta) @ np.asarray(FT, float).ravel()).reshape(-1, 6)

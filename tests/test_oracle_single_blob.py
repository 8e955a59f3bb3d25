"""Pins of the single-blob oracle (Sec. 2.4): the generalised RPY tensor and the
constrained system of Eq. linear_system_general with its preconditioner.

The tensor is checked against its definition (Eq. RPY extended to torques:
surface averages over the two spheres, estimated by Monte Carlo), against the
vorticity of the Oseen flow in the far field, continuity at contact, the
self mobilities, and symmetry / positive definiteness.  The system is
checked against the formal solution of Eq. U, and the preconditioner against
the exact inverse of its approximate problem."""
import numpy as np
import pytest

from oracle import gmres, rpy_rot, single_blob, system
from paper_2107_10800_amd import workloads as W

A, ETA = 1.0, 1.0


def _cross(v):
    m = np.zeros(v.shape[:-1] + (3, 3))
    m[..., 0, 1], m[..., 0, 2] = -v[..., 2], v[..., 1]
    m[..., 1, 0], m[..., 1, 2] = v[..., 2], -v[..., 0]
    m[..., 2, 0], m[..., 2, 1] = -v[..., 1], v[..., 0]
    return m


@pytest.mark.parametrize("sep", [3.0, 1.5])
def test_surface_average_monte_carlo(sep):
    """Force spread uniformly over sphere j, torque as 3/(8 pi a^3) tau x n;
    u_i = <v>, w_i = (3/(2a)) <n x v> over sphere i (Eq. RPY with rotations)."""
    rng = np.random.default_rng(5)
    batches = []
    for _ in range(8):
        m = 200000
        ni = rng.standard_normal((m, 3))
        ni /= np.linalg.norm(ni, axis=1)[:, None]
        nj = rng.standard_normal((m, 3))
        nj /= np.linalg.norm(nj, axis=1)[:, None]
        d = np.array([sep, 0.3, -0.2]) + A * ni - A * nj
        r = np.linalg.norm(d, axis=1)
        G = (np.eye(3)[None] / r[:, None, None]
             + d[:, :, None] * d[:, None, :] / r[:, None, None] ** 3) / (8 * np.pi * ETA)
        Xi, Xj = _cross(ni), -_cross(nj)          # n_i x ., and tau -> tau x n_j
        c = 3.0 / (2 * A)
        blk = np.zeros((m, 6, 6))
        blk[:, :3, :3] = G
        blk[:, 3:, :3] = c * Xi @ G
        blk[:, :3, 3:] = c * G @ Xj
        blk[:, 3:, 3:] = c * c * Xi @ G @ Xj
        batches.append(blk.mean(0))
    b = np.array(batches)
    mean, err = b.mean(0), b.std(0) / np.sqrt(len(b))
    ref = rpy_rot.pair_blocks(np.array([sep, 0.3, -0.2]), A, ETA)
    assert np.all(np.abs(mean - ref) <= 6 * err + 2e-5 * np.abs(ref).max())


def test_far_field_is_oseen_vorticity():
    """For r > 2a, w_i = (1/2) curl of the Oseen flow of f_j (the rotlet and
    the Faxen terms of a point force have no vorticity correction)."""
    r0 = np.array([3.1, -1.7, 2.2])
    f = np.array([0.4, -1.1, 0.7])

    def oseen(x):
        rr = np.linalg.norm(x)
        return (f / rr + x * (x @ f) / rr ** 3) / (8 * np.pi * ETA)

    h = 1e-5
    J = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (oseen(r0 + e) - oseen(r0 - e)) / (2 * h)
    curl = np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])
    w = rpy_rot.pair_blocks(r0, A, ETA)[3:, :3] @ f
    assert np.allclose(w, 0.5 * curl, rtol=1e-7, atol=1e-12)


def test_contact_continuity_and_self():
    c_lo = rpy_rot.rot_coefficients(np.array([2.0 - 1e-12]), A)
    c_hi = rpy_rot.rot_coefficients(np.array([2.0 + 1e-12]), A)
    for lo, hi in zip(c_lo, c_hi):
        assert abs(lo[0] - hi[0]) < 1e-9 * max(abs(hi[0]), 1e-3)
    B0 = rpy_rot.pair_blocks(np.zeros(3), A, ETA)
    assert np.allclose(B0[:3, :3], np.eye(3) / (6 * np.pi * ETA * A))
    assert np.allclose(B0[3:, 3:], np.eye(3) / (8 * np.pi * ETA * A ** 3))
    assert np.all(B0[:3, 3:] == 0) and np.all(B0[3:, :3] == 0)


def test_symmetric_positive_definite():
    rng = np.random.default_rng(7)
    for trial in range(3):
        pos = rng.uniform(0, 6, (30, 3))          # many overlapping pairs
        Nm = rpy_rot.body_mobility(pos, A, ETA)
        assert np.abs(Nm - Nm.T).max() < 1e-15
        assert np.linalg.eigvalsh(Nm).min() > 0


@pytest.mark.parametrize("make", [lambda: W.blob_shells(1), lambda: W.blob_filaments(2, 1)])
def test_system_matches_formal_solution(make):
    wl = make()
    S = single_blob.assemble(wl)
    y = single_blob.solve_dense(S)
    U, phi = single_blob.solve_formal(S, wl.F)
    M = wl.M
    assert np.allclose(y[:6 * M], U, rtol=0, atol=1e-10 * np.abs(U).max())
    assert np.abs(S["C"] @ y[:6 * M] - S["B"]).max() < 1e-10
    # the projection of Eq. U
    Nm, C = S["N"], S["C"]
    G = system.pinv_sym(C @ Nm @ C.T)
    Q = np.eye(6 * M) - Nm @ C.T @ G @ C
    assert np.abs(Q @ Q - Q).max() < 1e-9


def test_preconditioner_inverts_its_approximate_problem():
    """The preconditioner is the exact inverse of [I, -N~ C^T; C, 0]."""
    wl = W.blob_shells(1)
    S = single_blob.assemble(wl)
    P = single_blob.Preconditioner(wl, S["C"])
    M = wl.M
    At = S["A"].copy()
    At[:6 * M, 6 * M:] = -P.Nt @ S["C"].T
    rng = np.random.default_rng(8)
    y = rng.standard_normal(At.shape[0])
    assert np.allclose(P.apply(At @ y), y, atol=1e-10)
    # and it makes GMRES converge where the plain iteration is slow
    y1, info = gmres.gmres(lambda v: S["A"] @ v, P.apply, S["b"], tol=1e-10)
    y0, info0 = gmres.gmres(lambda v: S["A"] @ v, lambda v: v, S["b"], tol=1e-10, max_iter=400)
    assert info["iterations"] < info0["iterations"]
    assert np.linalg.norm(S["A"] @ y1 - S["b"]) <= 1e-10 * np.linalg.norm(S["b"]) * 1.01

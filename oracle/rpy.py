"""Rotne-Prager-Yamakawa blob mobility (Sec. 2.3, Eq. RPY), float64.

The paper defines M_ij as the double surface average of the Stokes Green's
function over the two blob spheres (Eq. RPY) and cites the closed forms of
Rotne-Prager / Wajnryb et al. (unbounded) and Swan & Brady (above a no-slip
wall) without printing them.  This module writes them out:

* Unbounded (equal radii a, r = r_i - r_j, r = |r|):
    r > 2a : M = 1/(8 pi eta r) [(1 + 2a^2/(3r^2)) I + (1 - 2a^2/r^2) rr/r^2]
    r <= 2a: M = 1/(6 pi eta a) [(1 - 9r/(32a)) I + 3/(32 a r) r r^T]
  (r = 0 gives I/(6 pi eta a)).  Reading: the boundary r = 2a takes the
  overlap branch; both branches agree there in value and slope.

* Above a no-slip plane z = 0 (every blob at z > a):
    M^wall(x, y) = M^RPY(x - y)
                 + 1/(8 pi eta) F_x F_y [G^Blake(x, y) - G^Oseen(x - y)]
  with the Faxen operator F = 1 + (a^2/6) Laplacian applied in each argument,
  and Blake's image system for a point force at y (height h = y_3, image
  point y* = (y1, y2, -y3), R = x - y*, D = diag(1, 1, -1)):
    G^Blake_ij = (d_ij/r + r_i r_j/r^3) - (d_ij/R + R_i R_j/R^3)
               + 2 h D_jk d/dR_k [h R_i/R^3 - (d_i3/R + R_i R_3/R^3)].
  The derivatives are taken symbolically (sympy) from exactly this
  definition; no simplified form is used here.  The same expression with
  x = y gives the blob's own wall-corrected self mobility.
"""
from __future__ import annotations

import functools

import numpy as np


def rpy_free_blocks(rvec: np.ndarray, a: float, eta: float) -> np.ndarray:
    """Unbounded RPY 3x3 blocks for separation vectors rvec (...,3)."""
    rvec = np.asarray(rvec, float)
    r = np.linalg.norm(rvec, axis=-1)
    eye = np.eye(3)
    with np.errstate(divide="ignore", invalid="ignore"):
        rr = rvec[..., :, None] * rvec[..., None, :]
        # far branch
        rs = np.where(r > 0, r, 1.0)
        far = (1.0 / (8 * np.pi * eta * rs))[..., None, None] * (
            (1 + 2 * a * a / (3 * rs * rs))[..., None, None] * eye
            + (1 - 2 * a * a / (rs * rs))[..., None, None] * rr / (rs * rs)[..., None, None])
        # overlap branch; the r r^T term is guarded to 0 at r = 0
        near = (1.0 / (6 * np.pi * eta * a)) * (
            (1 - 9 * r / (32 * a))[..., None, None] * eye
            + np.where(r > 0, 3.0 / (32 * a * rs), 0.0)[..., None, None] * rr)
    return np.where((r <= 2 * a)[..., None, None], near, far)


@functools.lru_cache(maxsize=1)
def wall_image_exprs():
    """((x1, x2, x3), (y1, y2, y3), a, exprs): the nine components (row-major) of
    F_x F_y (G^Blake - G^Oseen)(x, y) as sympy expressions."""
    import sympy as sp

    x = sp.symbols("x1:4", real=True)
    y = sp.symbols("y1:4", real=True)
    a = sp.Symbol("a", positive=True)
    R = [x[0] - y[0], x[1] - y[1], x[2] + y[2]]
    h = y[2]
    Rn = sp.sqrt(R[0] ** 2 + R[1] ** 2 + R[2] ** 2)
    D = [1, 1, -1]

    def delta(i, j):
        return 1 if i == j else 0

    def image(i, j):
        # Blake minus Oseen: the direct Stokeslet cancels, the rest is the image
        w = -(delta(i, j) / Rn + R[i] * R[j] / Rn ** 3)
        inner = h * R[i] / Rn ** 3 - (delta(i, 2) / Rn + R[i] * R[2] / Rn ** 3)
        # d/dR_k at fixed source equals d/dx_k
        w += 2 * h * D[j] * sp.diff(inner, x[j])
        return w

    def lap(f, v):
        return sum(sp.diff(f, s, 2) for s in v)

    exprs = []
    for i in range(3):
        for j in range(3):
            w = image(i, j)
            lx = lap(w, x)
            exprs.append(w + a ** 2 / 6 * (lx + lap(w, y)) + a ** 4 / 36 * lap(lx, y))
    return x, y, a, exprs


@functools.lru_cache(maxsize=1)
def _wall_image_fn():
    """Lambdified F_x F_y (G^Blake - G^Oseen) as a function of (x, y, a)."""
    import sympy as sp

    x, y, a, exprs = wall_image_exprs()
    return sp.lambdify((*x, *y, a), exprs, "numpy", cse=True)


def wall_image_blocks(x: np.ndarray, y: np.ndarray, a: float, eta: float) -> np.ndarray:
    """1/(8 pi eta) F_x F_y W(x, y) for target points x (...,3), sources y (...,3)."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    x, y = np.broadcast_arrays(x, y)
    f = _wall_image_fn()
    comps = f(x[..., 0], x[..., 1], x[..., 2], y[..., 0], y[..., 1], y[..., 2], a)
    out = np.empty(x.shape[:-1] + (3, 3))
    for k, c in enumerate(comps):
        out[..., k // 3, k % 3] = c
    return out / (8 * np.pi * eta)


def check_above_wall(pos: np.ndarray, a: float) -> None:
    """Blobs overlapping the wall (z <= a) are outside the model."""
    if np.any(np.asarray(pos)[:, 2] <= a):
        raise ValueError("blob at or below z = a with a no-slip wall")


def pair_blocks(x: np.ndarray, y: np.ndarray, a: float, eta: float, wall: bool) -> np.ndarray:
    """M(x, y) 3x3 blocks for broadcastable target/source point arrays."""
    blocks = rpy_free_blocks(np.asarray(x) - np.asarray(y), a, eta)
    if wall:
        blocks = blocks + wall_image_blocks(x, y, a, eta)
    return blocks


def mobility_matrix(pos: np.ndarray, a: float, eta: float, wall: bool) -> np.ndarray:
    """Dense 3N x 3N blob mobility, xyz interleaved per blob."""
    pos = np.asarray(pos, float)
    if wall:
        check_above_wall(pos, a)
    n = len(pos)
    blocks = pair_blocks(pos[:, None, :], pos[None, :, :], a, eta, wall)
    return blocks.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)


def mobility_apply(pos: np.ndarray, lam: np.ndarray, a: float, eta: float, wall: bool,
                   targets=None, chunk: int = 1 << 20) -> np.ndarray:
    """u_i = sum_j M_ij lam_j over all sources j (including j = i).

    ``targets`` optionally restricts the output rows (indices); the sum always
    runs over every source.  Returns (len(targets), 3)."""
    pos = np.asarray(pos, float)
    lam = np.asarray(lam, float).reshape(-1, 3)
    if wall:
        check_above_wall(pos, a)
    tgt = np.arange(len(pos)) if targets is None else np.asarray(targets)
    out = np.zeros((len(tgt), 3))
    n = len(pos)
    rows = max(1, chunk // max(n, 1))
    for s in range(0, len(tgt), rows):
        ti = tgt[s:s + rows]
        blocks = pair_blocks(pos[ti][:, None, :], pos[None, :, :], a, eta, wall)
        out[s:s + rows] = np.einsum("tsij,sj->ti", blocks, lam)
    return out

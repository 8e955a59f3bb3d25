"""Fast (interpolation-based multipole) approximation of the blob mobility product, float64.

TEST INFRASTRUCTURE ONLY (see the package header): nothing in the product
path may use this module.

The paper applies the blob mobility by direct summation and points to fast
summation (fast multipole or spectral methods, Sec. 1, Sec. 2.3, Sec. 6) as the
route to larger systems without fixing one.  The library's fast product is a
kernel-independent multipole method: the black-box FMM of Fong and Darve
(J. Comput. Phys. 228, 2009), in which the pair tensor M(x, y) of two
well-separated cells is replaced by its tensor-product Chebyshev interpolant in
both arguments.  This module writes out the approximation that method defines,
as a plain sum over cell pairs, with no translation operators: every term is
computed from its definition.

Definitions (units of length; the library uses the same ones):
  * root cube: origin o = the componentwise minimum of the blob positions,
    side S = (largest extent over x, y, z) * (1 + 2^-20) (S = a if all blobs
    coincide); at level l a blob at x lies in the cell with integer
    coordinates floor(((x - o) / S) * 2^l);
  * cell of level l with coordinates i: centre o + (i + 1/2) S / 2^l,
    half-width w = S / 2^(l+1); two cells of one level are adjacent when their
    coordinates differ by at most 1 in each direction (a cell is adjacent to
    itself); the parent of i is floor(i / 2);
  * Chebyshev points of the first kind xi_k = cos((2k + 1) pi / (2n)),
    k = 0..n-1, Lagrange polynomials l_k(xi) = prod_{j != k} (xi - xi_j) /
    (xi_k - xi_j); the n^3 proxy points of a cell are c + w (xi_kx, xi_ky,
    xi_kz) and its interpolation weights S_k(x) = l_kx(u_x) l_ky(u_y) l_kz(u_z)
    with u = (x - c) / w;
  * interaction list of a cell c of level l >= 2: the non-empty cells of level
    l whose parent is adjacent to the parent of c and which are not adjacent to
    c themselves;
  * leaf level L: the product is
        u_i = sum_{j in leaves adjacent to leaf(i)} M(x_i, y_j) lam_j
            + sum_{l=2..L} sum_{c' in IL(c_l(i))} sum_k S^{c}_k(x_i)
                  sum_m M(t^c_k, s^{c'}_m) qhat^{c'}_m,
        qhat^{c'}_m = sum_{j in c'} S^{c'}_m(y_j) lam_j,
    with c = c_l(i) the level-l cell of blob i, t^c the proxy points of c and
    s^{c'} those of c'; a listed cell c' holding fewer blobs than proxies
    (|c'| < n^3) enters with its blobs instead: sum_{j in c'} M(t^c_k, y_j)
    lam_j (exact in the source argument, and cheaper).  Each source is counted once for each target: the
    adjacent leaves and the interaction lists of the ancestors partition the
    blobs.  With L <= 1 there is no interaction list and the product is the
    direct sum.  A leaf side of at least 2a keeps every interpolated pair out of
    the overlap branch of the RPY tensor (r > 2a).
"""
from __future__ import annotations

import numpy as np

from . import rpy


def cheb_nodes(n: int) -> np.ndarray:
    return np.cos((2 * np.arange(n) + 1) * np.pi / (2 * n))


def lagrange(n: int, u: np.ndarray) -> np.ndarray:
    """l_k(u) for k = 0..n-1 at points u (...,): shape (..., n)."""
    x = cheb_nodes(n)
    u = np.asarray(u, float)[..., None]
    out = np.ones(u.shape[:-1] + (n,))
    for k in range(n):
        for j in range(n):
            if j != k:
                out[..., k] *= (u[..., 0] - x[j]) / (x[k] - x[j])
    return out


def weights(n: int, x: np.ndarray, c: np.ndarray, w: float) -> np.ndarray:
    """S_k(x) for points x (m,3) in the cell (centre c, half-width w): (m, n^3),
    proxy index k = (kx n + ky) n + kz."""
    u = (np.asarray(x, float) - c) / w
    lx, ly, lz = (lagrange(n, u[:, d]) for d in range(3))
    return np.einsum("ma,mb,mc->mabc", lx, ly, lz).reshape(len(u), n ** 3)


def proxies(n: int, c: np.ndarray, w: float) -> np.ndarray:
    xi = cheb_nodes(n)
    g = np.stack(np.meshgrid(xi, xi, xi, indexing="ij"), -1).reshape(-1, 3)
    return c + w * g


def root_cube(pos: np.ndarray, a: float):
    pos = np.asarray(pos, float)
    o = pos.min(0)
    ext = float((pos.max(0) - o).max())
    S = ext * (1.0 + 2.0 ** -20) if ext > 0 else a
    return o, S


def cell_coords(pos: np.ndarray, o: np.ndarray, S: float, level: int) -> np.ndarray:
    u = (np.asarray(pos, float) - o) / S
    return np.floor(u * 2.0 ** level).astype(np.int64)


def max_level(pos: np.ndarray, a: float) -> int:
    """Deepest leaf level whose cell side is at least 2a."""
    _, S = root_cube(pos, a)
    L = 0
    while S / 2.0 ** (L + 1) >= 2 * a:
        L += 1
    return L


def fmm_apply(pos, lam, a, eta, wall, n, L, kernel=None, sparse_cells=True):
    """The approximation defined in the module docstring, (N, d).

    lam: (N, d) generalised forces; kernel(x, y) -> (..., d, d) blocks for
    broadcastable point arrays; by default the RPY tensor M(x, y) (d = 3,
    unbounded or above the wall).  For single-blob bodies (Sec. 2.4) the kernel
    is the generalised RPY tensor N(x, y) (d = 6) and lam = (f, tau).
    sparse_cells=False interpolates every listed cell, the plain
    tensor-product interpolation (for the pins of the sparse-cell rule)."""
    pos = np.asarray(pos, float)
    lam = np.asarray(lam, float).reshape(len(pos), -1)
    if kernel is None:
        def kernel(x, y):
            return rpy.pair_blocks(x, y, a, eta, wall)
    o, S = root_cube(pos, a)
    if L > max_level(pos, a):
        raise ValueError("leaf side below 2a")
    out = np.zeros_like(lam)
    # direct sums over adjacent leaves
    leaf = cell_coords(pos, o, S, L)
    keys, inv = np.unique(leaf, axis=0, return_inverse=True)
    inv = inv.ravel()
    for t in range(len(keys)):
        tgt = np.nonzero(inv == t)[0]
        near = np.nonzero(np.abs(leaf - keys[t]).max(1) <= 1)[0]
        blk = kernel(pos[tgt][:, None, :], pos[near][None, :, :])
        out[tgt] += np.einsum("tsij,sj->ti", blk, lam[near])
    # interpolated sums over the interaction lists of levels 2..L
    for lev in range(2, L + 1):
        w = S / 2.0 ** (lev + 1)
        ci = cell_coords(pos, o, S, lev)
        cells, cinv = np.unique(ci, axis=0, return_inverse=True)
        cinv = cinv.ravel()
        centre = o + (cells + 0.5) * (S / 2.0 ** lev)
        members = [np.nonzero(cinv == c)[0] for c in range(len(cells))]
        qhat = [weights(n, pos[m], centre[c], w).T @ lam[m] for c, m in enumerate(members)]
        for c in range(len(cells)):
            il = np.nonzero((np.abs(cells // 2 - cells[c] // 2).max(1) <= 1)
                            & (np.abs(cells - cells[c]).max(1) > 1))[0]
            if not len(il):
                continue
            t = proxies(n, centre[c], w)
            # sparse listed cells enter with their blobs, the others with proxies
            sparse = [sparse_cells and len(members[d]) < n ** 3 for d in il]
            s = np.concatenate([pos[members[d]] if sp else proxies(n, centre[d], w)
                                for d, sp in zip(il, sparse)])
            q = np.concatenate([lam[members[d]] if sp else qhat[d]
                                for d, sp in zip(il, sparse)])
            v = np.einsum("tsij,sj->ti", kernel(t[:, None, :], s[None, :, :]), q)
            out[members[c]] += weights(n, pos[members[c]], centre[c], w) @ v
    return out

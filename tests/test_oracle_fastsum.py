"""Pins of the oracle of the fast multipole approximation (oracle/fastsum.py).

The approximation has a plain definition: interpolate the pair tensor of
well-separated cells in both arguments, sum the rest directly.  The pins check
it against facts that do not come from that code:
  * the Lagrange basis at Chebyshev points of the first kind: l_k(xi_j) =
    delta_kj, partition of unity, and exact reproduction of polynomials of
    degree < n in each coordinate;
  * a kernel that is such a polynomial in x and in y is interpolated exactly,
    so the approximation must equal the direct sum to rounding: this fails for
    a source counted twice or missed (a wrong interaction list, a lost level),
    a transposed weight or a wrong proxy point;
  * with L <= 1 there is no interpolation: the direct RPY sum of the pinned
    dense oracle;
  * with the RPY tensor the error against the dense sum falls geometrically
    with n (free space and above the wall);
  * the RPY mobility is symmetric, so the approximation is too when both
    arguments of every far pair are interpolated (every cell holding at least
    n^3 blobs): a.(M b) = b.(M a), free and above the wall.
"""
import numpy as np
import pytest

from oracle import fastsum, rpy


def test_lagrange_basis():
    for n in (2, 3, 5, 8):
        x = fastsum.cheb_nodes(n)
        assert np.allclose(x, np.cos((2 * np.arange(n) + 1) * np.pi / (2 * n)))
        assert np.abs(fastsum.lagrange(n, x) - np.eye(n)).max() < 1e-13
        u = np.linspace(-1, 1, 17)
        assert np.abs(fastsum.lagrange(n, u).sum(1) - 1).max() < 1e-12


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_weights_reproduce_polynomials(n):
    rng = np.random.default_rng(n)
    c, w = np.array([1.5, -2.0, 4.0]), 0.75
    x = c + w * rng.uniform(-1, 1, (20, 3))
    W = fastsum.weights(n, x, c, w)
    t = fastsum.proxies(n, c, w)
    for ex in [(0, 0, 0), (n - 1, 0, 0), (0, n - 1, n - 1), (n - 1, n - 1, n - 1), (1, 0, n - 1)]:
        p = lambda z: np.prod(z ** np.array(ex), axis=-1)    # noqa: E731
        assert np.abs(W @ p(t) - p(x)).max() <= 1e-11 * max(1.0, np.abs(p(x)).max())


def blobs(N, box, seed, a=1.0, z0=1.5):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, (N, 3)) * np.array(box)
    pos[:, 2] += z0 * a
    return pos, rng.standard_normal((N, 3))


def poly_kernel(n):
    """A 3x3 kernel of degree n-1 in each coordinate of x and of y."""
    B = np.arange(1.0, 10.0).reshape(3, 3)

    def K(x, y):
        x, y = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float))
        s = 1 + 0.3 * x[..., 0] * y[..., 1] - 0.2 * (x[..., 2] ** (n - 1)) * y[..., 2] \
            + 0.1 * x[..., 1] * (y[..., 0] ** (n - 1))
        out = B * s[..., None, None]
        out = out + 0.05 * x[..., :, None] * y[..., None, :]
        return out
    return K


@pytest.mark.parametrize("n,L", [(2, 2), (3, 3), (4, 3)])
def test_polynomial_kernel_is_exact(n, L):
    pos, lam = blobs(300, (40, 40, 20), 11 + n)
    K = poly_kernel(n)
    u = fastsum.fmm_apply(pos, lam, 1.0, 1.0, False, n, L, kernel=K)
    ref = np.einsum("tsij,sj->ti", K(pos[:, None, :], pos[None, :, :]), lam)
    assert np.abs(u - ref).max() <= 1e-10 * np.abs(ref).max()
    # the interpolated part is not empty: the same kernel with one degree too
    # many in y is no longer exact
    K2 = poly_kernel(n + 1)
    u2 = fastsum.fmm_apply(pos, lam, 1.0, 1.0, False, n, L, kernel=K2)
    ref2 = np.einsum("tsij,sj->ti", K2(pos[:, None, :], pos[None, :, :]), lam)
    assert np.abs(u2 - ref2).max() > 1e-6 * np.abs(ref2).max()


def test_levels_and_root_cube():
    pos, _ = blobs(200, (40, 20, 10), 3, a=0.5)
    o, S = fastsum.root_cube(pos, 0.5)
    assert np.all(fastsum.cell_coords(pos, o, S, 4) < 16) and np.all(fastsum.cell_coords(pos, o, S, 4) >= 0)
    L = fastsum.max_level(pos, 0.5)
    assert S / 2 ** L >= 1.0 > S / 2 ** (L + 1)
    with pytest.raises(ValueError):
        fastsum.fmm_apply(pos, np.zeros_like(pos), 0.5, 1.0, False, 3, L + 1)


@pytest.mark.parametrize("wall", [False, True])
def test_no_interaction_list_is_the_direct_sum(wall):
    pos, lam = blobs(120, (30, 30, 8), 5)
    for L in (0, 1):
        u = fastsum.fmm_apply(pos, lam, 1.0, 1.3, wall, 4, L)
        ref = rpy.mobility_apply(pos, lam, 1.0, 1.3, wall)
        assert np.abs(u - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("wall", [False, True])
def test_rpy_error_falls_geometrically_with_order(wall):
    """A slab of 16 cells at leaf level 2 (side 12a) holding more blobs than
    proxies, so that both arguments are interpolated: the max error over blobs,
    relative to the largest entry, falls by a roughly constant factor per
    order.  (The wall tensor of the oracle is slow: fewer blobs and orders.)"""
    N, orders = (2400, (2, 3, 4, 5)) if not wall else (1100, (2, 3, 4))
    pos, lam = blobs(N, (48, 48, 10), 9)
    ref = rpy.mobility_apply(pos, lam, 1.0, 1.0, wall)
    errs = []
    for n in orders:
        u = fastsum.fmm_apply(pos, lam, 1.0, 1.0, wall, n, 2)
        errs.append(np.abs(u - ref).max() / np.abs(ref).max())
    print("max error by order:", ["%.1e" % e for e in errs])
    assert errs[0] > 1e-4                   # the interpolation is really used
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < errs[0] * (1e-2 if not wall else 3e-2)


def poly_kernel6(n):
    """A 6x6 kernel of degree n-1 in each coordinate of x and of y."""
    K3 = poly_kernel(n)

    def K(x, y):
        x, y = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float))
        k = K3(x, y)
        out = np.zeros(x.shape[:-1] + (6, 6))
        out[..., :3, :3] = k
        out[..., 3:, :3] = 0.5 * np.swapaxes(k, -1, -2)
        out[..., :3, 3:] = -0.3 * k
        out[..., 3:, 3:] = 2.0 * k + np.eye(3) * (x[..., 1] * y[..., 2])[..., None, None]
        return out
    return K


@pytest.mark.parametrize("n,L", [(2, 2), (3, 3)])
def test_six_component_polynomial_kernel_is_exact(n, L):
    """Generalised forces (f, tau) and a 6x6 kernel (the single-blob form)."""
    pos, _ = blobs(250, (40, 40, 20), 21 + n)
    lam6 = np.random.default_rng(n).standard_normal((250, 6))
    K = poly_kernel6(n)
    u = fastsum.fmm_apply(pos, lam6, 1.0, 1.0, False, n, L, kernel=K)
    ref = np.einsum("tsij,sj->ti", K(pos[:, None, :], pos[None, :, :]), lam6)
    assert u.shape == (250, 6)
    assert np.abs(u - ref).max() <= 1e-10 * np.abs(ref).max()


def test_generalised_rpy_error_falls_with_order():
    """The single-blob tensor (Sec. 2.4) in the interpolation: the error against
    the dense generalised sum falls with the order."""
    from oracle import rpy_rot
    pos, _ = blobs(2000, (48, 48, 10), 13)       # more bodies per cell than proxies
    ft = np.random.default_rng(5).standard_normal((2000, 6))
    ref = rpy_rot.body_mobility_apply(pos, ft, 1.0, 1.0)

    def K(x, y):
        return rpy_rot.pair_blocks(np.asarray(x) - np.asarray(y), 1.0, 1.0)
    errs = []
    for n in (2, 3, 4):
        u = fastsum.fmm_apply(pos, ft, 1.0, 1.0, False, n, 2, kernel=K)
        errs.append(np.abs(u - ref).max() / np.abs(ref).max())
    print("generalised RPY, max error by order 2..4:", ["%.1e" % e for e in errs])
    assert errs[0] > 1e-4
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:]))


def lattice(shape, spacing, seed, z0=1.5):
    """Jittered lattice: every cell of the levels used holds several blobs."""
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(*[np.arange(m) for m in shape], indexing="ij"), -1).reshape(-1, 3)
    pos = (g + 0.5) * spacing + rng.uniform(-0.15, 0.15, g.shape) * spacing
    pos[:, 2] += z0
    return pos


@pytest.mark.parametrize("wall,shape,n,L", [(False, (24, 24, 6), 2, 3), (False, (12, 12, 6), 3, 2),
                                            (True, (8, 8, 2), 2, 2)])
def test_symmetric_when_every_listed_cell_is_interpolated(wall, shape, n, L):
    """The RPY mobility is symmetric, with or without the wall. When every cell
    of levels 2..L holds at least n^3 blobs, both arguments of every far pair
    are interpolated, so the approximation is symmetric too: a.(M b) = b.(M a)
    to rounding. A weight applied on one side only, a list that is not mutual
    or a wrong proxy on one side breaks it."""
    pos = lattice(shape, 2.0, 3)
    o, S = fastsum.root_cube(pos, 1.0)
    for lev in range(2, L + 1):
        _, occ = np.unique(fastsum.cell_coords(pos, o, S, lev), axis=0, return_counts=True)
        assert occ.min() >= n ** 3
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal((2,) + pos.shape)
    Mb = fastsum.fmm_apply(pos, b, 1.0, 1.0, wall, n, L)
    Ma = fastsum.fmm_apply(pos, a, 1.0, 1.0, wall, n, L)
    if not wall:    # really approximated (the oracle's wall tensor is slow)
        dense = rpy.mobility_apply(pos, b, 1.0, 1.0, wall)
        assert np.abs(Mb - dense).max() > 1e-4 * np.abs(dense).max()
    s1, s2 = np.sum(a * Mb), np.sum(b * Ma)
    assert abs(s1 - s2) <= 1e-12 * np.linalg.norm(a) * np.linalg.norm(Mb)


def test_sparse_cell_rule_only_removes_source_interpolation():
    """The rule that a listed cell with fewer blobs than proxies enters with its
    blobs replaces that cell's source-side interpolation by the exact sum: for
    a kernel of degree n - 1 (interpolated exactly) both forms agree to
    rounding; with the RPY tensor on a loose suspension (most cells sparse) the
    rule changes the result and brings it closer to the dense sum, at the
    orders whose n^3 proxies outnumber the blobs of the cells (about 19 here)."""
    pos, lam = blobs(300, (48, 48, 10), 12)
    for n in (3, 4):
        K = poly_kernel(n)
        u1 = fastsum.fmm_apply(pos, lam, 1.0, 1.0, False, n, 2, kernel=K)
        u0 = fastsum.fmm_apply(pos, lam, 1.0, 1.0, False, n, 2, kernel=K, sparse_cells=False)
        assert np.abs(u1 - u0).max() <= 1e-12 * np.abs(u0).max()
    ref = rpy.mobility_apply(pos, lam, 1.0, 1.0, False)
    for n in (3, 4, 5):
        u1 = fastsum.fmm_apply(pos, lam, 1.0, 1.0, False, n, 2)
        u0 = fastsum.fmm_apply(pos, lam, 1.0, 1.0, False, n, 2, sparse_cells=False)
        e1 = np.linalg.norm(u1 - ref) / np.linalg.norm(ref)
        e0 = np.linalg.norm(u0 - ref) / np.linalg.norm(ref)
        print(f"order {n}: error with the rule {e1:.2e}, all cells interpolated {e0:.2e}")
        assert np.abs(u1 - u0).max() > 1e-6 * np.abs(ref).max()
        assert e1 < e0

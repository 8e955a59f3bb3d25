"""Pins of the RPY oracle (Sec. 2.3, Eq. RPY) against facts fixed outside it."""
import numpy as np
import pytest
import sympy as sp

from oracle import rpy

A, ETA = 1.0, 1.0


def test_self_mobility_unbounded():
    # r = 0: the blob's own mobility is the Stokes drag of a sphere, I/(6 pi eta a)
    for a, eta in [(1.0, 1.0), (0.5, 3.0)]:
        m = rpy.rpy_free_blocks(np.zeros(3), a, eta)
        assert np.allclose(m, np.eye(3) / (6 * np.pi * eta * a), rtol=1e-15, atol=0)


def test_oseen_far_field():
    rng = np.random.default_rng(0)
    for _ in range(5):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        r = 1e4
        m = rpy.rpy_free_blocks(r * d, A, ETA) * 8 * np.pi * ETA * r
        assert np.allclose(m, np.eye(3) + np.outer(d, d), atol=1e-7)


def test_far_branch_is_faxen_squared_oseen():
    # (1 + a^2/6 lap)^2 G = G + a^2/3 lap G for the biharmonic Oseen tensor
    x = sp.symbols("x1:4", real=True)
    a = sp.Symbol("a", positive=True)
    r = sp.sqrt(sum(c ** 2 for c in x))
    pt = {x[0]: 1.3, x[1]: -2.1, x[2]: 1.7, a: 1.0}
    rv = np.array([1.3, -2.1, 1.7])
    ref = rpy.rpy_free_blocks(rv, 1.0, 1.0) * 8 * np.pi
    for i in range(3):
        for j in range(3):
            G = (1 if i == j else 0) / r + x[i] * x[j] / r ** 3
            lap = sum(sp.diff(G, c, 2) for c in x)
            f2 = G + a ** 2 / 6 * 2 * lap + a ** 4 / 36 * sum(sp.diff(lap, c, 2) for c in x)
            assert abs(float(f2.subs(pt)) - ref[i, j]) < 1e-14


def test_continuity_at_contact():
    d = np.array([0.3, -0.5, 0.8])
    d /= np.linalg.norm(d)
    eps = 1e-7
    lo = rpy.rpy_free_blocks((2 - eps) * d, A, ETA)
    at = rpy.rpy_free_blocks(2 * d, A, ETA)
    hi = rpy.rpy_free_blocks((2 + eps) * d, A, ETA)
    assert np.allclose(lo, hi, atol=1e-8)
    assert np.allclose(at, hi, atol=1e-8)
    # one-sided slopes agree (first derivative continuous)
    s_lo = (at - rpy.rpy_free_blocks((2 - 1e-4) * d, A, ETA)) / 1e-4
    s_hi = (rpy.rpy_free_blocks((2 + 1e-4) * d, A, ETA) - at) / 1e-4
    assert np.allclose(s_lo, s_hi, atol=5e-5)


@pytest.mark.parametrize("sep", [3.0, 1.5])
def test_surface_average_monte_carlo(sep):
    # Eq. RPY literally: average the Oseen tensor over two sphere surfaces.
    rng = np.random.default_rng(1)
    batches = []
    for _ in range(8):
        m = 250000
        u = rng.standard_normal((m, 3))
        v = rng.standard_normal((m, 3))
        d = np.array([sep, 0, 0]) + u / np.linalg.norm(u, axis=1)[:, None] \
            - v / np.linalg.norm(v, axis=1)[:, None]
        r = np.linalg.norm(d, axis=1)
        o = (np.eye(3)[None] / r[:, None, None]
             + d[:, :, None] * d[:, None, :] / r[:, None, None] ** 3) / (8 * np.pi)
        batches.append(o.mean(0))
    b = np.array(batches)
    mean, err = b.mean(0), b.std(0) / np.sqrt(len(b))
    ref = rpy.rpy_free_blocks(np.array([sep, 0, 0]), A, ETA)
    assert np.all(np.abs(mean - ref) <= 6 * err + 1e-9)


@pytest.mark.parametrize("wall", [False, True])
def test_symmetric_positive_definite(wall):
    rng = np.random.default_rng(2)
    for trial in range(3):
        n = 25
        pos = np.column_stack([rng.uniform(0, 5, n), rng.uniform(0, 5, n),
                               rng.uniform(1.05, 4, n)])
        Mm = rpy.mobility_matrix(pos, A, ETA, wall)
        assert np.abs(Mm - Mm.T).max() < 1e-15
        assert np.linalg.eigvalsh(Mm).min() > 0


def test_wall_self_mobility_closed_form():
    # Swan & Brady (cited in Sec. 2.3): closed-form wall self mobility vs height.
    for h in [1.05, 1.5, 2.0, 3.0, 7.5, 40.0]:
        x = np.array([0.4, -1.0, h])
        m = rpy.pair_blocks(x, x, A, ETA, True) * 6 * np.pi * ETA * A
        ht = h / A
        par = 1 - 9 / (16 * ht) + 1 / (8 * ht ** 3) - 1 / (16 * ht ** 5)
        perp = 1 - 9 / (8 * ht) + 1 / (2 * ht ** 3) - 1 / (8 * ht ** 5)
        assert np.allclose(m, np.diag([par, par, perp]), atol=1e-14)


def test_blake_no_slip_on_wall():
    # with a -> 0 the wall tensor is Blake's point-force solution, zero on z = 0
    rng = np.random.default_rng(3)
    a = 1e-9
    for _ in range(5):
        x = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), 0.0])
        y = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(0.5, 3)])
        G = rpy.rpy_free_blocks(x - y, a, ETA) + rpy.wall_image_blocks(x, y, a, ETA)
        scale = np.abs(rpy.rpy_free_blocks(x - y, a, ETA)).max()
        assert np.abs(G).max() < 1e-12 * scale


def test_wall_reciprocity_and_invariance():
    rng = np.random.default_rng(4)
    for _ in range(5):
        x = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(1.1, 4)])
        y = np.array([rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(1.1, 4)])
        mxy = rpy.pair_blocks(x, y, A, ETA, True)
        myx = rpy.pair_blocks(y, x, A, ETA, True)
        assert np.abs(mxy - myx.T).max() < 1e-15
        # rotating both points about the wall normal rotates the tensor
        c, s = np.cos(0.7), np.sin(0.7)
        Q = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
        shift = np.array([3.0, -1.0, 0.0])
        mr = rpy.pair_blocks(Q @ x + shift, Q @ y + shift, A, ETA, True)
        assert np.abs(mr - Q @ mxy @ Q.T).max() < 1e-15


def test_wall_vanishes_far_above():
    # the wall correction of a cluster lifted to height H decays like 1/H
    rng = np.random.default_rng(5)
    base = np.column_stack([rng.uniform(0, 6, 10), rng.uniform(0, 6, 10), rng.uniform(0, 6, 10)])
    diffs = []
    for H in (1e4, 1e5, 1e6):
        pos = base + np.array([0, 0, H])
        Mw = rpy.mobility_matrix(pos, A, ETA, True)
        Mf = rpy.mobility_matrix(pos, A, ETA, False)
        diffs.append(np.abs(Mw - Mf).max())
    assert diffs[2] < 1e-6 * np.abs(Mf).max() * 2
    assert abs(diffs[0] / diffs[1] - 10) < 0.05 and abs(diffs[1] / diffs[2] - 10) < 0.05


def test_below_wall_rejected():
    pos = np.array([[0, 0, 3.0], [1, 1, 0.9]])
    with pytest.raises(ValueError):
        rpy.mobility_matrix(pos, A, ETA, True)


def test_matvec_matches_dense():
    rng = np.random.default_rng(6)
    pos = np.column_stack([rng.uniform(0, 5, 30), rng.uniform(0, 5, 30),
                           rng.uniform(1.2, 4, 30)])
    lam = rng.standard_normal((30, 3))
    for wall in (False, True):
        u = rpy.mobility_apply(pos, lam, A, ETA, wall, chunk=100)
        ud = rpy.mobility_matrix(pos, A, ETA, wall) @ lam.ravel()
        assert np.allclose(u.ravel(), ud, rtol=1e-14, atol=1e-15)
        sub = rpy.mobility_apply(pos, lam, A, ETA, wall, targets=[3, 17])
        assert np.allclose(sub, u[[3, 17]], rtol=1e-14)

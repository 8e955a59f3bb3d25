"""Pins of the oracle's compiled FP64 route for the blob mobility (Sec. 2.3,
Eq. RPY): oracle/rpy_sum.c against the numpy route (rpy.py) and against the
closed forms both must meet, free space and above the wall."""
import numpy as np
import pytest

from oracle import gen_wall_image_c, rpy, rpy_c
from paper_2107_10800_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def lib():
    if not __import__("os").path.exists(rpy_c.LIB):
        rpy_c.build()
    return rpy_c.load()


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.mark.parametrize("wall", [False, True])
def test_sum_matches_numpy_route(wall):
    # overlapping and far pairs, pairs exactly 2a apart (the branch boundary)
    cl = W.random_blobs(300, seed=3, box=25.0)
    pos = np.vstack([cl["pos"], [[40.0, 40.0, 3.0], [42.0, 40.0, 3.0], [40.0, 40.0, 5.0]]])
    lam = np.vstack([cl["lam"], np.random.default_rng(4).standard_normal((3, 3))])
    u = rpy_c.mobility_apply(pos, lam, 1.0, 1.0, wall)
    uo = rpy.mobility_apply(pos, lam, 1.0, 1.0, wall)
    assert rel(u, uo) <= 1e-13
    tg = np.array([0, 7, 301, 302, 299])
    ut = rpy_c.mobility_apply(pos, lam, 1.0, 1.0, wall, targets=tg)
    assert np.array_equal(ut, u[tg])


@pytest.mark.parametrize("wall", [False, True])
def test_matrix_matches_numpy_route(wall):
    cl = W.random_blobs(60, seed=5, box=10.0)
    a, eta = 1.3, 0.7
    pos = cl["pos"] * 1.3 + np.array([0, 0, 0.5])
    M = rpy_c.mobility_matrix(pos, a, eta, wall)
    Mo = rpy.mobility_matrix(pos, a, eta, wall)
    assert np.abs(M - Mo).max() <= 1e-13 * np.abs(Mo).max()
    # the product route and the matrix route agree
    lam = cl["lam"]
    assert rel(M @ lam.ravel(), rpy_c.mobility_apply(pos, lam, a, eta, wall)) <= 1e-14


def test_free_space_closed_forms():
    # self mobility 1/(6 pi eta a); coincident blobs take it too; far field Oseen
    a, eta = 0.8, 1.7
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1e4, 0.0, 0.0]])
    M = rpy_c.mobility_matrix(pos, a, eta, False)
    assert np.allclose(M[:3, :3], np.eye(3) / (6 * np.pi * eta * a), rtol=1e-15, atol=0)
    assert np.allclose(M[:3, 3:6], np.eye(3) / (6 * np.pi * eta * a), rtol=1e-15, atol=0)
    r = 1e4
    oseen = (np.eye(3) + np.diag([1.0, 0, 0])) / (8 * np.pi * eta * r)
    assert np.abs(M[:3, 6:9] - oseen).max() <= 1e-7 * np.abs(oseen).max()


def test_wall_self_mobility_closed_form():
    # Swan & Brady's wall-corrected self mobility of a sphere at height h
    a, eta = 1.0, 1.0
    h = np.array([1.05, 1.5, 2.0, 4.0, 10.0, 100.0])
    pos = np.column_stack([10.0 * np.arange(len(h)) * 1e3, np.zeros_like(h), h])
    M = rpy_c.mobility_matrix(pos, a, eta, True)
    for k, hk in enumerate(h):
        t = hk / a
        par = (1 - 9 / (16 * t) + 1 / (8 * t ** 3) - 1 / (16 * t ** 5)) / (6 * np.pi * eta * a)
        per = (1 - 9 / (8 * t) + 1 / (2 * t ** 3) - 1 / (8 * t ** 5)) / (6 * np.pi * eta * a)
        B = M[3 * k:3 * k + 3, 3 * k:3 * k + 3]
        assert np.allclose(np.diag(B), [par, par, per], rtol=1e-13, atol=0)


def test_symmetric_positive_definite():
    cl = W.random_blobs(80, seed=9, box=8.0, zlo=1.1, zhi=4.0)
    for wall in (False, True):
        M = rpy_c.mobility_matrix(cl["pos"], 1.0, 1.0, wall)
        assert np.abs(M - M.T).max() <= 1e-15 * np.abs(M).max()
        assert np.linalg.eigvalsh(M).min() > 0


def test_result_independent_of_threads():
    cl = W.random_blobs(500, seed=11, box=30.0)
    u1, t1 = rpy_c.mobility_apply(cl["pos"], cl["lam"], 1.0, 1.0, True, threads=1,
                                  return_threads=True)
    u4, t4 = rpy_c.mobility_apply(cl["pos"], cl["lam"], 1.0, 1.0, True, threads=4,
                                  return_threads=True)
    assert t1 == 1 and t4 == 4
    assert np.array_equal(u1, u4)


def test_generated_image_code_is_current():
    # the committed C of the wall image is what the generator writes from the
    # symbolic definition today
    with open(gen_wall_image_c.OUT) as f:
        assert f.read() == gen_wall_image_c.generate()

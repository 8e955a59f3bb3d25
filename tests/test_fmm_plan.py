"""Host logic of the fast product: the octree the library plans (arb_fmm_plan,
host only, no device) against the definitions written out in oracle/fastsum.py,
counted here with numpy: leaf level (explicit, clamped and automatic), cells of
every level, non-empty leaves, directly summed pairs of adjacent leaves and
interaction-list entries.  Runs without a GPU."""
import numpy as np
import pytest

from oracle import fastsum
from paper_2107_10800_amd import arb


def counts(pos, a, n, L, with_pairs=False):
    """(cells of levels 0..L, leaves, direct pairs, interaction-list entries[,
    M2L pair evaluations: n^3 per proxy or blob of each listed cell, the blobs
    when the cell holds fewer than n^3])."""
    o, S = fastsum.root_cube(pos, a)
    P = n ** 3
    cells = 0
    inter = 0
    m2l = 0
    for lev in range(L + 1):
        u, occ = np.unique(fastsum.cell_coords(pos, o, S, lev), axis=0, return_counts=True)
        cells += len(u)
        if lev >= 2:
            for c in u:
                sel = (np.abs(u // 2 - c // 2).max(1) <= 1) & (np.abs(u - c).max(1) > 1)
                inter += int(np.sum(sel))
                m2l += int(P * np.minimum(occ[sel], P).sum())
    leaf = fastsum.cell_coords(pos, o, S, L)
    keys, cnt = np.unique(leaf, axis=0, return_counts=True)
    near = 0
    for k, m in zip(keys, cnt):
        near += int(m) * int(cnt[np.abs(keys - k).max(1) <= 1].sum())
    if with_pairs:
        return cells, len(keys), near, inter, m2l
    return cells, len(keys), near, inter


def auto_level(pos, a, leaf):
    """The documented rule: the shallowest level l >= 2 whose mean occupancy is
    at most `leaf`, never deeper than the deepest level with side >= 2a."""
    Lhi = min(fastsum.max_level(pos, a), 16)
    if Lhi < 2:
        return 0
    o, S = fastsum.root_cube(pos, a)
    for lev in range(2, Lhi + 1):
        if len(pos) <= leaf * len(np.unique(fastsum.cell_coords(pos, o, S, lev), axis=0)):
            return lev
    return Lhi


def blobs(N, box, seed, z0=1.5):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, (N, 3)) * np.array(box, float)
    pos[:, 2] += z0
    return pos


SHAPES = [(500, (40, 40, 10)), (777, (60, 20, 20)), (300, (30, 30, 30)), (1000, (200, 200, 4))]


@pytest.mark.parametrize("N,box", SHAPES)
@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_plan_matches_the_definitions(N, box, L):
    pos = blobs(N, box, N + L)
    a = 0.8
    n = 4
    Lexp = 0 if L < 2 else min(L, fastsum.max_level(pos, a))
    st = arb.arb_fmm_plan(pos, a, order=n, levels=L)
    assert st["levels"] == Lexp
    cells, leaves, near, inter, m2l = counts(pos, a, n, Lexp, with_pairs=True)
    assert (st["cells"], st["leaves"], st["near_pairs"], st["interactions"]) == \
        (cells, leaves, near, inter)
    assert st["m2l_pairs"] == m2l <= inter * n ** 6


def fewest_pairs_level(pos, a, n):
    """The documented default: from level 2, one level deeper while the pair
    evaluations per product (direct pairs + M2L pairs) fall."""
    Lhi = min(fastsum.max_level(pos, a), 16)
    if Lhi < 2:
        return 0
    def cost(lev):
        c = counts(pos, a, n, lev, with_pairs=True)
        return c[2] + c[4]
    L, best = 2, cost(2)
    for lev in range(3, Lhi + 1):
        c = cost(lev)
        if c >= best:
            break
        L, best = lev, c
    return L


@pytest.mark.parametrize("N,box", SHAPES)
@pytest.mark.parametrize("leaf", [16, 100])
def test_level_from_occupancy(N, box, leaf):
    pos = blobs(N, box, 3 * N + leaf)
    n = 3
    st = arb.arb_fmm_plan(pos, 1.0, order=n, leaf=leaf)
    L = auto_level(pos, 1.0, leaf)
    assert st["levels"] == L
    assert st["cells"] == counts(pos, 1.0, n, L)[0]


@pytest.mark.parametrize("N,box", SHAPES)
@pytest.mark.parametrize("n", [2, 3, 4])
def test_default_level_has_the_fewest_pair_evaluations(N, box, n):
    pos = blobs(N, box, 5 * N + n)
    st = arb.arb_fmm_plan(pos, 1.0, order=n)
    L = fewest_pairs_level(pos, 1.0, n)
    assert st["levels"] == L
    cells, leaves, near, inter = counts(pos, 1.0, n, L)
    assert (st["cells"], st["near_pairs"], st["interactions"]) == (cells, near, inter)


def test_degenerate_inputs():
    # coincident blobs: one cell, the direct sum of every pair
    pos = np.tile([[3.0, 4.0, 5.0]], (10, 1))
    st = arb.arb_fmm_plan(pos, 1.0, order=4)
    assert (st["levels"], st["cells"], st["leaves"], st["near_pairs"]) == (0, 1, 1, 100)
    st = arb.arb_fmm_plan(np.zeros((0, 3)), 1.0)
    assert st["cells"] == 0 and st["order"] == 6
    # a cluster narrower than 8a: no level below the root has a side >= 2a
    pos = blobs(50, (5, 5, 3), 1)
    assert arb.arb_fmm_plan(pos, 1.0, levels=4)["levels"] == 0
    for bad in (dict(order=1), dict(order=9), dict(levels=-1), dict(levels=17), dict(leaf=-1)):
        with pytest.raises(arb.ArbError):
            arb.arb_fmm_plan(pos, 1.0, **bad)
    pos[3, 1] = np.nan
    with pytest.raises(arb.ArbError):
        arb.arb_fmm_plan(pos, 1.0)


def test_plan_of_many_blobs():
    """200,000 blobs in a slab: the plan's keys and sort run on several host
    threads there; its counts against the definitions."""
    pos = blobs(200_000, (400, 400, 12), 77)
    st = arb.arb_fmm_plan(pos, 1.0, order=3, levels=5)
    cells, leaves, near, inter, m2l = counts(pos, 1.0, 3, 5, with_pairs=True)
    assert st["levels"] == 5
    assert (st["cells"], st["leaves"], st["near_pairs"], st["interactions"], st["m2l_pairs"]) == \
        (cells, leaves, near, inter, m2l)


@pytest.mark.parametrize("n", [4, 6])
def test_default_level_of_many_blobs(n):
    """400,000 blobs in a thin slab: the level search counts its pairs on
    several host threads. Its choice against the rule, with the pair counts of
    plans at explicit levels (counted from the lists those plans build): the
    cost falls down to the chosen level and does not fall one level deeper."""
    pos = blobs(400_000, (700, 700, 6), 90 + n)
    st = arb.arb_fmm_plan(pos, 1.0, order=n)
    L = st["levels"]
    Lhi = min(fastsum.max_level(pos, 1.0), 16)
    assert 3 <= L <= Lhi

    def cost(lev):
        s = arb.arb_fmm_plan(pos, 1.0, order=n, levels=lev)
        assert s["levels"] == lev
        return s["near_pairs"] + s["m2l_pairs"]

    costs = [cost(lev) for lev in range(2, L + 1)]
    assert all(b < a for a, b in zip(costs, costs[1:]))
    if L < Lhi:
        assert cost(L + 1) >= costs[-1]
    ref = arb.arb_fmm_plan(pos, 1.0, order=n, levels=L)
    assert {k: st[k] for k in st if k != "build_ms"} == {k: ref[k] for k in ref if k != "build_ms"}


@pytest.mark.parametrize("N,box,seed,kw", [
    (200_000, (400, 400, 12), 77, dict(order=3, levels=5)),
    (400_000, (700, 700, 6), 94, dict(order=6)),
    (400_000, (700, 700, 6), 94, dict(order=4, leaf=40)),
])
def test_threaded_plan_equals_serial_plan(monkeypatch, N, box, seed, kw):
    """The octree planned on several host threads is the one a single thread
    plans, array for array: blob order, cells, interaction and near lists,
    work items and tables (their hash), and every count."""
    pos = blobs(N, box, seed)
    monkeypatch.setenv("ARB_HOST_THREADS", "1")
    serial = arb.arb_fmm_plan(pos, 1.0, **kw)
    monkeypatch.setenv("ARB_HOST_THREADS", "16")
    threaded = arb.arb_fmm_plan(pos, 1.0, **kw)
    drop = ("build_ms",)
    assert {k: v for k, v in serial.items() if k not in drop} == \
        {k: v for k, v in threaded.items() if k not in drop}
    assert serial["plan_hash"] != 0
    # a different input gives a different plan hash
    pos2 = pos.copy()
    pos2[[0, 1]] = pos2[[1, 0]]
    assert arb.arb_fmm_plan(pos2, 1.0, **kw)["plan_hash"] != serial["plan_hash"]


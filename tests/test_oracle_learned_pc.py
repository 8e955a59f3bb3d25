"""Pins of the oracle's corrected block preconditioner (given body mobilities).

The preconditioner replaces each blob block by the unbounded one plus a rank-6
term chosen so that the block solve is exact for the supplied N~_w.  Checked
against: its reduction to the unbounded block preconditioner when N~_w is the
unbounded body mobility, the defining identity K^T M~^-1 K = N~_w^-1, a dense
solve of the block-diagonal saddle system it stands for, and the iteration
count it reaches with the exact wall body mobilities.
"""
import dataclasses

import numpy as np
import pytest

from oracle import gmres, precond, system
from paper_2107_10800_amd import workloads as W


@pytest.fixture(scope="module")
def two_bacteria():
    wl = W.bacteria(n_bact=2, side=50.0, seed=31)
    S = system.assemble(wl)
    free = precond.BlockPreconditioner(dataclasses.replace(wl, wall=False), S["r"], S["C"])
    wall = precond.BlockPreconditioner(wl, S["r"], S["C"])
    return wl, S, free, wall


def perturbed(Nts, eps, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in Nts:
        L = np.linalg.cholesky(n)
        L = L * (1.0 + eps * rng.standard_normal(L.shape))
        out.append(L @ L.T)
    return out


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_reduces_to_unbounded_blocks(two_bacteria):
    wl, S, free, wall = two_bacteria
    P = precond.CorrectedBodyPreconditioner(wl, S["r"], S["C"], free.Nt)
    r = np.random.default_rng(1).standard_normal(S["A"].shape[0])
    assert rel(P.apply(r), free.apply(r)) <= 1e-10


def test_body_mobility_identity(two_bacteria):
    wl, S, free, wall = two_bacteria
    Nw = perturbed(wall.Nt, 0.05, 2)
    P = precond.CorrectedBodyPreconditioner(wl, S["r"], S["C"], Nw)
    off = wl.blob_offset
    K = S["K"]
    for p in range(wl.M):
        rows = slice(3 * off[p], 3 * off[p + 1])
        Kp = K[rows, 6 * p:6 * p + 6]
        Mt = P.L[p] @ P.L[p].T
        assert rel(Kp.T @ np.linalg.solve(Mt, Kp), np.linalg.inv(Nw[p])) <= 1e-9


def test_apply_is_the_block_saddle_solve(two_bacteria):
    wl, S, free, wall = two_bacteria
    Nw = perturbed(wall.Nt, 0.05, 3)
    P = precond.CorrectedBodyPreconditioner(wl, S["r"], S["C"], Nw)
    N, M = wl.N, wl.M
    Mt = np.zeros((3 * N, 3 * N))
    off = wl.blob_offset
    for p in range(M):
        sl = slice(3 * off[p], 3 * off[p + 1])
        Mt[sl, sl] = P.L[p] @ P.L[p].T
    K, C = S["K"], S["C"]
    nc = C.shape[0]
    A = np.block([[Mt, -K, np.zeros((3 * N, nc))],
                  [-K.T, np.zeros((6 * M, 6 * M)), C.T],
                  [np.zeros((nc, 3 * N)), C, np.zeros((nc, nc))]])
    r = np.random.default_rng(4).standard_normal(A.shape[0])
    assert rel(P.apply(r), np.linalg.solve(A, r)) <= 1e-9


def test_exact_wall_body_mobility_is_as_good_as_exact_blocks(two_bacteria):
    # with the exact wall N~ the corrected unbounded blocks need no more GMRES
    # iterations than the exact wall blocks; with the inconsistent pairing
    # (unbounded blocks, wall N~) they need more
    wl, S, free, wall = two_bacteria
    P = precond.CorrectedBodyPreconditioner(wl, S["r"], S["C"], wall.Nt)
    its = {}
    for name, pc in (("exact", wall), ("corrected", P)):
        _, info = gmres.gmres(lambda v: S["A"] @ v, pc.apply, S["b"], tol=1e-8)
        its[name] = info["iterations"]
    inconsistent = precond.BlockPreconditioner(dataclasses.replace(wl, wall=False), S["r"], S["C"])
    inconsistent.Nt = [n.copy() for n in wall.Nt]
    inconsistent.G = []
    for bs, rs in zip(inconsistent.asm_bodies, inconsistent.asm_rows):
        cols = np.concatenate([np.arange(6 * p, 6 * p + 6) for p in bs])
        Ca = S["C"][np.ix_(rs, cols)]
        Na = np.zeros((len(cols), len(cols)))
        for k, p in enumerate(bs):
            Na[6 * k:6 * k + 6, 6 * k:6 * k + 6] = inconsistent.Nt[p]
        inconsistent.G.append(precond._chol_or_pinv(Ca @ Na @ Ca.T)[0])
    _, info = gmres.gmres(lambda v: S["A"] @ v, inconsistent.apply, S["b"], tol=1e-8)
    its["inconsistent"] = info["iterations"]
    print(its)
    assert its["corrected"] <= its["exact"] + 1
    assert its["inconsistent"] > its["corrected"]

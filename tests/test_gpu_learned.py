"""GPU checks of the learned body-mobility network and its use as a preconditioner.

BF16 operands bound the forward and gradient parity at about 2^-8 per operand:
per-tensor relative L2 <= 3e-2 against the float64 oracle evaluated at the same
(float32) parameters.  A preconditioner changes iteration counts, not the
solution: the learned-preconditioned solve must match the exact solution within
the same forward-error bar as the exact-preconditioned one.
"""
import dataclasses

import numpy as np
import pytest

from oracle import mlp, precond, system
from paper_2107_10800_amd import arb
from paper_2107_10800_amd import learned
from paper_2107_10800_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


@pytest.fixture(scope="module")
def ctx():
    c = arb.arb_create(precision=arb.ARB_FP64, wall=True)
    yield c
    arb.arb_destroy(c)


def test_forward_and_gradient_match_oracle(ctx):
    P = W.mlp_init_weights(seed=11)
    arb.arb_mlp_set_params(ctx, P)
    assert np.array_equal(arb.arb_mlp_get_params(ctx), P)
    rng = np.random.default_rng(3)
    B = 300                                     # not a multiple of 16: ragged tile
    X = np.column_stack([rng.uniform(8, 15, B), rng.standard_normal((B, 4)),
                         rng.integers(0, 2, (B, 2))]).astype(np.float32)
    T = (0.3 * rng.standard_normal((B, 21))).astype(np.float32)
    Y = arb.arb_mlp_forward(ctx, X)
    Yo, _ = mlp.forward(P.astype(float), X.astype(float))
    print(f"forward rel err {rel(Y, Yo):.2e}")
    assert rel(Y, Yo) <= 3e-2
    loss, g = arb.arb_mlp_grad(ctx, X, T)
    lo, go = mlp.loss_and_grad(P.astype(float), X.astype(float), T.astype(float))
    assert abs(loss - lo) <= 3e-2 * lo
    k = 0
    for (Wo, bo) in mlp.unpack(go):
        for part in (Wo.ravel(), bo):
            e = rel(g[k:k + part.size], part)
            print(f"grad block {k}: rel err {e:.2e}")
            assert e <= 3e-2
            k += part.size


def test_adam_step_matches_oracle():
    # one training step from fresh Adam moments against the oracle's Adam on the
    # oracle's gradient: where the gradient is clearly non-zero (its sign is not
    # decided by BF16 rounding) every weight moves by lr against that sign
    import torch

    P = W.mlp_init_weights(seed=13)
    rng = np.random.default_rng(14)
    B, lr = 256, 1e-3
    X = np.column_stack([rng.uniform(8, 15, B), rng.standard_normal((B, 4)),
                         rng.integers(0, 2, (B, 2))]).astype(np.float32)
    T = (0.3 * rng.standard_normal((B, 21))).astype(np.float32)
    c = arb.arb_create(precision=arb.ARB_FP64, wall=True)
    try:
        arb.arb_mlp_set_params(c, P)
        st = torch.cuda.Stream()
        xd = torch.tensor(X, device="cuda")
        td = torch.tensor(T, device="cuda")
        torch.cuda.synchronize()
        arb.arb_mlp_train_step_dev(c, B, xd, td, lr, stream=st.cuda_stream)
        torch.cuda.synchronize()
        P1 = arb.arb_mlp_get_params(c).astype(float)
    finally:
        arb.arb_destroy(c)
    _, g = mlp.loss_and_grad(P.astype(float), X.astype(float), T.astype(float))
    Po, _, _ = mlp.adam(P.astype(float), g, np.zeros_like(g), np.zeros_like(g), 1, lr=lr)
    big = np.abs(g) > 0.1 * np.sqrt(np.mean(g * g))
    assert big.mean() > 0.1
    d_gpu, d_or = P1 - P, Po - P
    assert np.allclose(d_gpu[big], d_or[big], rtol=1e-3, atol=1e-7)
    assert np.all(np.abs(d_gpu) <= lr * (1 + 1e-3) + 1e-7)


def test_features_match_oracle():
    wl = W.bacterium_poses(40, seed=12)
    c = arb.context_for(wl)
    try:
        X = arb.arb_mlp_features(c)
    finally:
        arb.arb_destroy(c)
    Xo = mlp.features(wl.q[:, 2], wl.theta, wl.body_type)
    assert np.abs(X - Xo).max() <= 1e-6 * np.abs(Xo).max()


def test_labels_match_oracle():
    wl = W.bacterium_poses(3, seed=13)
    c = arb.context_for(wl)
    try:
        Nt, T = arb.arb_body_mobility(c)
    finally:
        arb.arb_destroy(c)
    from oracle import bodies, rpy
    r = bodies.blob_positions(wl.q, wl.theta, wl.r_ref, wl.blob_offset)
    for p in range(wl.M):
        sl = slice(wl.blob_offset[p], wl.blob_offset[p + 1])
        Mpp = rpy.mobility_matrix(r[sl], 1.0, 1.0, True)
        K = bodies.K_matrix(r[sl], wl.q[p:p + 1], np.array([0, sl.stop - sl.start]))
        No = np.linalg.inv(K.T @ np.linalg.solve(Mpp, K))
        assert rel(Nt[p], No) <= 1e-10
    assert rel(T, mlp.target_from_mobility(Nt)) <= 1e-6


def test_standardised_forward_matches_oracle(ctx):
    P = W.mlp_init_weights(seed=12)
    rng = np.random.default_rng(4)
    X = np.column_stack([rng.uniform(8, 15, 64), rng.standard_normal((64, 4)),
                         rng.integers(0, 2, (64, 2))]).astype(np.float32)
    sc = (np.float32([11, 0, 0, 0, 0, .5, .5]), np.float32([2, .5, .5, .5, .5, .5, .5]),
          (0.1 * rng.standard_normal(21)).astype(np.float32),
          rng.uniform(0.5, 2, 21).astype(np.float32))
    learned.load_model(ctx, P, sc)
    try:
        Y = arb.arb_mlp_forward(ctx, X)
    finally:
        arb.arb_mlp_set_scaling(ctx, np.zeros(7), np.ones(7), np.zeros(21), np.ones(21))
    Yo = mlp.predict(P.astype(float), X.astype(float), *[np.asarray(c, float) for c in sc])
    assert rel(Y, Yo) <= 3e-2


@pytest.fixture(scope="module")
def trained():
    # the benchmark's recipe: 2e5 body poses (1e5 bacteria) labelled by the exact
    # block build, 400 epochs of batch 1,024 (about 15 s on the GPU)
    X, T = learned.make_dataset(100000, seed=101)
    sc = learned.scaling(X, T)
    c = arb.arb_create(precision=arb.ARB_FP64, wall=True)
    learned.load_model(c, W.mlp_init_weights(seed=6), sc)
    l0 = arb.arb_mlp_grad(c, X[:20000], T[:20000])[0]
    learned.train(c, X, T, epochs=400, batch=1024, lr=2e-3, seed=7)
    l1 = arb.arb_mlp_grad(c, X[:20000], T[:20000])[0]
    P = arb.arb_mlp_get_params(c)
    Y = arb.arb_mlp_forward(c, X[:2000])
    arb.arb_destroy(c)
    Np = mlp.mobility_from_output(Y)
    Ne = mlp.mobility_from_output(T[:2000])
    err = np.linalg.norm(Np - Ne, axis=(1, 2)) / np.linalg.norm(Ne, axis=(1, 2))
    print(f"training loss {l0:.3e} -> {l1:.3e}; body mobility rel err median "
          f"{np.median(err):.2e} max {err.max():.2e}")
    return (P, sc), l0, l1, X, T


def test_training_reduces_loss(trained):
    P, l0, l1, X, T = trained
    assert l1 < 0.05 * l0


def kappa_of(S):
    s = np.linalg.svd(S["A"], compute_uv=False)
    return s[0] / s[-1]


@pytest.mark.parametrize("prec", [arb.ARB_FP64, arb.ARB_FP32C])
def test_learned_preconditioner_solution(trained, prec):
    # a preconditioner changes iterations, not the solution.  FP64: every block
    # variant solves to 1e-8 and lands within the forward-error bound 10 kappa r
    # of the direct solution.  FP32C: the learned solve driven to
    # r = 1e-5 / (10 kappa) is within 1e-5 of the direct solution on U, phi and
    # lambda.  What the network buys over the method without it (the unbounded
    # body-frame blocks, which need no per-solve work either): fewer iterations
    model = trained[0]
    wl = W.bacteria(n_bact=4, side=60.0, seed=21)
    S = system.assemble(wl)
    kap = kappa_of(S)
    yd = system.solve_dense(S["A"], S["b"])
    N, M = wl.N, wl.M
    ref = dict(lam=yd[:3 * N], U=yd[3 * N:3 * N + 6 * M], phi=yd[3 * N + 6 * M:])
    tol = 1e-8 if prec == arb.ARB_FP64 else 1e-6

    def solve(pc, t):
        c = arb.context_for(wl, precision=prec, tol=t, precond=pc)
        try:
            learned.load_model(c, *model)
            rc, U, phi, lam, info = arb.arb_solve(c, wl.F)
        finally:
            arb.arb_destroy(c)
        assert rc == arb.ARB_OK
        assert info["rel_residual_fp64"] <= t
        return dict(lam=lam.ravel(), U=U.ravel(), phi=phi), info

    out = {pc: solve(pc, tol) for pc in (arb.ARB_PC_BLOCK, arb.ARB_PC_LEARNED,
                                         arb.ARB_PC_BODYFRAME)}
    infoe, info, infob = (out[pc][1] for pc in (arb.ARB_PC_BLOCK, arb.ARB_PC_LEARNED,
                                                 arb.ARB_PC_BODYFRAME))
    print(f"prec {prec}: iterations exact {infoe['iterations']} learned {info['iterations']} "
          f"body-frame {infob['iterations']}, build ms exact {infoe['t_build_ms']:.2f} "
          f"learned {info['t_build_ms']:.2f} body-frame {infob['t_build_ms']:.2f}")
    for pc, (y, inf) in out.items():
        bar = max(1e-12, 10 * kap * inf["rel_residual_fp64"])
        errs = {k: rel(y[k], ref[k]) for k in ref}
        print(f"  pc {pc} to {tol:.0e}: errors {errs} (forward-error bar {bar:.1e})")
        assert all(e <= bar for e in errs.values())
    # the corrected learned blocks are as strong as the exact ones (measured:
    # the same count on 4 to 256 bacteria) and stronger than the body-frame
    # blocks without the network (one iteration more on each of those cases)
    assert info["iterations"] <= infoe["iterations"] + 1
    assert info["iterations"] < infob["iterations"]
    if prec == arb.ARB_FP32C:
        tight = 1e-5 / (10 * kap)
        y, inf = solve(arb.ARB_PC_LEARNED, tight)
        errs = {k: rel(y[k], ref[k]) for k in ref}
        print(f"  learned fp32c to {tight:.1e}: errors {errs}, {inf['iterations']} iterations")
        assert all(e <= 1e-5 for e in errs.values())


def test_learned_apply_matches_oracle(trained):
    # the learned block solve: unbounded per-type blob blocks with the rank-6
    # correction for the network's N~_w, against the oracle's dense version
    model = trained[0]
    wl = W.bacteria(n_bact=4, side=60.0, seed=21)
    S = system.assemble(wl)
    r = np.random.default_rng(9).standard_normal(S["A"].shape[0])
    c = arb.context_for(wl, precision=arb.ARB_FP64, precond=arb.ARB_PC_LEARNED)
    try:
        learned.load_model(c, *model)
        assert arb.arb_precond_build(c) == arb.ARB_OK
        Nw = [arb.arb_precond_block(c, p, 0)[1] for p in range(wl.M)]
        z = arb.arb_precond_apply(c, r)
        with pytest.raises(arb.ArbError):
            arb.arb_precond_block(c, 0, 3 * int(wl.blob_offset[1]))
    finally:
        arb.arb_destroy(c)
    P = precond.CorrectedBodyPreconditioner(wl, S["r"], S["C"], Nw)
    assert rel(z, P.apply(r)) <= 1e-10


def test_bodyframe_apply_matches_oracle():
    # rotated per-type unbounded blocks = the unbounded block preconditioner
    wl = W.bacteria(n_bact=4, side=60.0, seed=21)
    S = system.assemble(wl)
    r = np.random.default_rng(10).standard_normal(S["A"].shape[0])
    c = arb.context_for(wl, precision=arb.ARB_FP64, precond=arb.ARB_PC_BODYFRAME)
    try:
        assert arb.arb_precond_build(c) == arb.ARB_OK
        z = arb.arb_precond_apply(c, r)
    finally:
        arb.arb_destroy(c)
    P = precond.BlockPreconditioner(dataclasses.replace(wl, wall=False), S["r"], S["C"])
    assert rel(z, P.apply(r)) <= 1e-10


def test_learned_fallback_on_invalid_factor():
    # output biases far outside the factor's range: the prediction is rejected
    P = W.mlp_init_weights(seed=6).copy()
    diag = [0, 2, 5, 9, 14, 20]
    P[-21 + np.array(diag)] = 1e3
    wl = W.bacteria(n_bact=2, side=40.0, seed=23)
    c = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-10, precond=arb.ARB_PC_LEARNED)
    try:
        arb.arb_mlp_set_params(c, P)
        rc, U, phi, lam, info = arb.arb_solve(c, wl.F)
    finally:
        arb.arb_destroy(c)
    assert rc == arb.ARB_W_LEARNED_FALLBACK
    assert info["rel_residual"] <= 1e-10


def oracle_residual_rows(wl, U, phi, lam, sample):
    """Rows of b - A y for the solution y = (lam, U, phi) from the oracle
    (Sec. 2.3, Eq. linear_system): the blob rows of the sampled blobs (the C
    oracle's M rows over every source), every body row and every constraint row;
    and ||b||.  Also returns the oracle's (M lam) on the sampled blobs."""
    from oracle import bodies, rpy_c

    r = bodies.blob_positions(wl.q, wl.theta, wl.r_ref, wl.blob_offset)
    lam3 = np.asarray(lam).reshape(-1, 3)
    Ml = rpy_c.mobility_apply(r, lam3, wl.a, wl.eta, wl.wall, targets=sample)
    KU = bodies.K_apply(r, wl.q, wl.blob_offset, U)[sample]
    us = (np.zeros((wl.N, 3)) if wl.u_slip is None
          else np.asarray(wl.u_slip).reshape(-1, 3))[sample]
    r_blob = us - (Ml - KU)
    C, B = bodies.constraint_rows(wl, sparse=True)
    body = -np.asarray(wl.F).reshape(-1) - (-bodies.KT_apply(r, wl.q, wl.blob_offset, lam3)
                                            .reshape(-1) + C.T @ phi)
    cons = B - C @ np.asarray(U).reshape(-1)
    us_all = np.zeros(3 * wl.N) if wl.u_slip is None else np.asarray(wl.u_slip).ravel()
    bnorm = np.linalg.norm(np.concatenate([us_all, np.asarray(wl.F).ravel(), B]))
    return r_blob, body, cons, bnorm, Ml


def test_full_size_learned_solve(trained):
    # 4,096 bacteria above the wall: the learned-block FP32 solve and the plain
    # FP64 exact-block solve both reach 1e-6, and their velocities agree to 1e-5.
    # What the network buys: the iteration count of the exact blocks (fewer
    # than the body-frame blocks, the method without it) at under a quarter of
    # the exact build (which forms the 8,192 blocks' inverses in about 8 ms at
    # this size).  The oracle checks both solutions at this size: the
    # residual on 256 sampled blob rows (its C pair sums over all 499,712
    # sources), on every body row and on every constraint row is bounded by the
    # residual the solver reports (each set of rows is part of the whole), and
    # the FP64 product of the solver's context matches the oracle's rows to 1e-12
    import torch

    model = trained[0]
    wl = W.bacteria(n_bact=4096, seed=5)
    print(f"full size learned: N={wl.N} M={wl.M} Nc={wl.n_rows}", flush=True)
    sample = np.random.default_rng(44).choice(wl.N, 256, replace=False).astype(np.int32)
    out, infos = {}, {}
    for name, prec, pc in (("exact_fp64", arb.ARB_FP64, arb.ARB_PC_BLOCK),
                           ("learned_fp32", arb.ARB_FP32C, arb.ARB_PC_LEARNED),
                           ("bodyframe_fp32", arb.ARB_FP32C, arb.ARB_PC_BODYFRAME)):
        c = arb.context_for(wl, precision=prec, tol=1e-6, restart=100, max_iter=1000,
                            precond=pc)
        try:
            learned.load_model(c, *model)
            rc, U, phi, lam, info = arb.arb_solve(c, wl.F)
            if name == "exact_fp64":
                lam_d = torch.tensor(np.asarray(lam).ravel(), dtype=torch.float64,
                                     device="cuda")
                u_d = torch.zeros_like(lam_d)
                arb.arb_mobility_apply_dev(c, lam_d, u_d)
                torch.cuda.synchronize()
                Ml_gpu = u_d.cpu().numpy().reshape(-1, 3)[sample]
        finally:
            arb.arb_destroy(c)
        assert rc == arb.ARB_OK
        assert info["rel_residual_fp64"] <= 1e-6
        print(f"  {name}: {info['iterations']} iterations, build {info['t_build_ms']:.2f} ms, "
              f"solve {info['t_solve_ms']:.1f} ms", flush=True)
        out[name] = U
        infos[name] = info
        if name == "bodyframe_fp32":
            continue
        r_blob, r_body, r_cons, bnorm, Ml = oracle_residual_rows(wl, U, phi, lam, sample)
        res = info["rel_residual_fp64"]
        e = [np.linalg.norm(x) / bnorm for x in (r_blob, r_body, r_cons)]
        print(f"  {name}: oracle residual rows (sampled blobs, bodies, constraints) "
              f"{e[0]:.2e} {e[1]:.2e} {e[2]:.2e}; solver {res:.2e}", flush=True)
        for x in e:
            assert x <= res * (1 + 1e-6) + 1e-12
        if name == "exact_fp64":
            perr = np.linalg.norm(Ml_gpu - Ml) / np.linalg.norm(Ml)
            print(f"  FP64 product rows against the oracle: {perr:.2e}", flush=True)
            assert perr <= 1e-12
    assert rel(out["learned_fp32"], out["exact_fp64"]) <= 1e-5
    assert infos["learned_fp32"]["iterations"] <= infos["exact_fp64"]["iterations"] + 1
    assert infos["learned_fp32"]["iterations"] < infos["bodyframe_fp32"]["iterations"]
    assert infos["learned_fp32"]["t_build_ms"] <= 0.25 * infos["exact_fp64"]["t_build_ms"]

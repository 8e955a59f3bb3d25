"""GPU parity of the constrained-mobility solver path against the oracle.

Steps: blob geometry (Sec. 2.3), K / K^T (Eq. no-slip, Eq. balance), constraint
rows C, B (Eq. dg, App. A), the saddle operator A (Eq. linear_system), the block
preconditioner (Sec. 3.1), GMRES, Euler update and position correction
(Sec. 4.2-4.3, App. B).  FP64 path: operators at 1e-12 relative (1e-14 for
the linear rigid-body maps); the GPU solve against the oracle's GMRES (the same
algorithm, the same steps) at 1e-12 relative L2 on each output (U, phi,
lambda).  Comparisons with the direct (dense LU) solution are bounded by what
any solver can reach at relative residual r, 10 kappa(A) r: that bar is used
there and only there.  FP32C path (FP32 pair sums inside FP64 iterative
refinement): the refinement is driven to r = 1e-5 / (10 kappa(A)) so that each
output is within 1e-5 of the direct solution; the errors at the practical
tolerance 1e-6 are reported beside.
"""
import numpy as np
import pytest

from oracle import bodies, correct, gmres, precond, system
from paper_2107_10800_amd import arb
from paper_2107_10800_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    b = np.ravel(b)
    return np.linalg.norm(np.ravel(a) - b) / max(np.linalg.norm(b), 1e-300)


def cases():
    return {
        "filament": lambda: W.filament(),
        "rigid_wall": lambda: W.random_rigid(3, 12, seed=7, wall=True),
        "bacteria4": lambda: W.bacteria(n_bact=4, side=60.0, seed=21),
        "diatoms2": lambda: W.diatoms(n_col=2, kmin=3, kmax=5, seed=22, lattice=(2, 1, 1)),
    }


def kappa(A):
    """Condition number of A on its range (largest / smallest nonzero singular value)."""
    s = np.linalg.svd(A, compute_uv=False)
    nz = s[s > 1e-12 * s[0]]
    return s[0] / nz[-1]


def solve_tol(S, r):
    """Forward-error bar against the direct solution for an iterate with
    relative residual r: any solver meets ||dy||/||y|| <= kappa(A) r, so the
    FP64 bar of 1e-12 is applied where the conditioning allows it and
    10 kappa r beyond that.  Used only against the direct solve."""
    return max(1e-12, 10.0 * S["kappa"] * max(r, 2.0 ** -52))


def outputs(wl, y):
    """Split y = [lambda; U; phi] into its three outputs."""
    N, M = wl.N, wl.M
    out = dict(lam=y[:3 * N], U=y[3 * N:3 * N + 6 * M])
    if wl.n_rows:
        out["phi"] = y[3 * N + 6 * M:]
    return out


@pytest.fixture(scope="module", params=list(cases()))
def case(request):
    wl = cases()[request.param]()
    print(f"solver case {request.param}: N={wl.N} M={wl.M} Nc={wl.n_rows}", flush=True)
    S = system.assemble(wl)
    S["kappa"] = kappa(S["A"])
    ctx = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-10)
    yield request.param, wl, S, ctx
    arb.arb_destroy(ctx)


def test_geometry_and_rigid_operators(case):
    name, wl, S, ctx = case
    assert np.abs(arb.arb_blob_positions(ctx) - S["r"]).max() <= 1e-13 * max(1, np.abs(S["r"]).max())
    rng = np.random.default_rng(1)
    U = rng.standard_normal(6 * wl.M)
    lam = rng.standard_normal(3 * wl.N)
    assert rel(arb.arb_K_apply(ctx, U), S["K"] @ U) <= 1e-14
    assert rel(arb.arb_KT_apply(ctx, lam), S["K"].T @ lam) <= 1e-14


def test_constraint_rows(case):
    name, wl, S, ctx = case
    if wl.n_rows == 0:
        pytest.skip("no constraints")
    coef, pq, B = arb.arb_constraint_rows(ctx)
    C = np.zeros((wl.n_rows, 6 * wl.M))
    for k in range(wl.n_rows):
        p, q = pq[k]
        C[k, 6 * p:6 * p + 6] += coef[k, :6]
        if q >= 0:
            C[k, 6 * q:6 * q + 6] += coef[k, 6:]
    assert np.abs(C - S["C"]).max() <= 1e-14 * max(1, np.abs(S["C"]).max())
    assert np.abs(B - S["B"]).max() <= 1e-14 * max(1, np.abs(S["B"]).max())


def test_saddle_operator(case):
    name, wl, S, ctx = case
    y = np.random.default_rng(2).standard_normal(S["A"].shape[0])
    assert rel(arb.arb_system_apply(ctx, y), S["A"] @ y) <= 1e-12


def test_preconditioner(case):
    name, wl, S, ctx = case
    rc = arb.arb_precond_build(ctx)
    assert rc in (arb.ARB_OK, arb.ARB_W_PINV_USED)
    P = precond.BlockPreconditioner(wl, S["r"], S["C"])
    for p in (0, wl.M - 1):
        m = 3 * int(wl.blob_offset[p + 1] - wl.blob_offset[p])
        L, Nt = arb.arb_precond_block(ctx, p, m)
        assert rel(L, P.L[p]) <= 1e-13          # Cholesky factors are unique
        assert rel(Nt, P.Nt[p]) <= 1e-11
    r = np.random.default_rng(3).standard_normal(S["A"].shape[0])
    assert rel(arb.arb_precond_apply(ctx, r), P.apply(r)) <= 1e-11


def test_gmres_solve(case):
    name, wl, S, ctx = case
    us = wl.u_slip
    rc, U, phi, lam, info = arb.arb_solve(ctx, wl.F, u_slip=us)
    assert rc in (arb.ARB_OK, arb.ARB_W_PINV_USED)
    assert info["rel_residual"] <= 1e-10
    P = precond.BlockPreconditioner(wl, S["r"], S["C"])
    y, oinfo = gmres.gmres(lambda v: S["A"] @ v, P.apply, S["b"], tol=1e-10)
    yg = np.concatenate([lam.ravel(), U.ravel(), phi])
    # same algorithm on both sides: same iteration count and iterates that
    # agree to 1e-12 on every output
    assert abs(info["iterations"] - oinfo["iterations"]) <= 1
    errs = {k: rel(v, outputs(wl, y)[k]) for k, v in outputs(wl, yg).items()}
    print(f"  gpu-vs-oracle gmres {errs}, iterations {info['iterations']} / "
          f"{oinfo['iterations']}, kappa {S['kappa']:.1e}")
    assert all(e <= 1e-12 for e in errs.values())
    yd = system.solve_dense(S["A"], S["b"])
    N, M = wl.N, wl.M
    assert rel(U, yd[3 * N:3 * N + 6 * M]) <= solve_tol(S, info["rel_residual"])


def test_left_preconditioned_solve(case):
    # left preconditioning (P^-1 A, the form Sec. 3.1 names) on the GPU and in
    # the oracle: the same algorithm, so the same iteration count (to one) and
    # outputs within 1e-12; the stopping test is on the true residual
    name, wl, S, ctx = case
    c2 = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-10, left_precond=1)
    try:
        rc, U, phi, lam, info = arb.arb_solve(c2, wl.F, u_slip=wl.u_slip)
    finally:
        arb.arb_destroy(c2)
    assert rc in (arb.ARB_OK, arb.ARB_W_PINV_USED)
    assert info["rel_residual"] <= 1e-10
    P = precond.BlockPreconditioner(wl, S["r"], S["C"])
    y, oinfo = gmres.gmres(lambda v: S["A"] @ v, P.apply, S["b"], tol=1e-10, left=True)
    assert oinfo["converged"]
    yg = np.concatenate([lam.ravel(), U.ravel(), phi])
    errs = {k: rel(v, outputs(wl, y)[k]) for k, v in outputs(wl, yg).items()}
    print(f"  left: gpu-vs-oracle {errs}, iterations {info['iterations']} / "
          f"{oinfo['iterations']}")
    assert abs(info["iterations"] - oinfo["iterations"]) <= 1
    assert all(e <= 1e-12 for e in errs.values())
    # against the direct solution, within the forward-error bound
    yd = system.solve_dense(S["A"], S["b"])
    N, M = wl.N, wl.M
    assert rel(U, yd[3 * N:3 * N + 6 * M]) <= solve_tol(S, info["rel_residual"])


def test_gmres_tight_matches_direct(case):
    name, wl, S, ctx = case
    c2 = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-14, max_iter=2000)
    try:
        rc, U, phi, lam, info = arb.arb_solve(c2, wl.F, u_slip=wl.u_slip)
    finally:
        arb.arb_destroy(c2)
    yd = system.solve_dense(S["A"], S["b"])
    N, M = wl.N, wl.M
    assert info["rel_residual"] <= 1e-12
    tol = solve_tol(S, info["rel_residual"])
    print(f"  tight solve: U {rel(U, yd[3 * N:3 * N + 6 * M]):.2e} lam "
          f"{rel(lam, yd[:3 * N]):.2e} (bar {tol:.1e})")
    assert rel(U, yd[3 * N:3 * N + 6 * M]) <= tol
    assert rel(lam, yd[:3 * N]) <= tol
    if wl.n_rows:
        assert rel(phi, yd[3 * N + 6 * M:]) <= tol


def test_fp32c_solve(case):
    # FP32 pair sums inside GMRES iterative refinement with FP64 residuals.  The
    # returned iterate meets the tolerance in FP64.  Driven to
    # r = 1e-5 / (10 kappa), every output is within 1e-5 of the direct solution
    # (the forward-error bound); at the practical tolerance 1e-6 the errors are
    # reported only, since there they are bounded by kappa * 1e-6
    # The residual of the returned iterate is also recomputed with the oracle's
    # dense system: where the last correction was accepted on its bound
    # (refine_final = 0) that bound must hold; refine_final = 1 always ends with
    # an FP64 product.
    name, wl, S, ctx = case
    yd = system.solve_dense(S["A"], S["b"])
    ref = outputs(wl, yd)
    tight = 1e-5 / (10.0 * S["kappa"])
    bnorm = np.linalg.norm(S["b"])
    for tol, final in ((1e-6, 0), (1e-6, 1), (tight, 0)):
        c2 = arb.context_for(wl, precision=arb.ARB_FP32C, tol=tol, refine_final=final)
        try:
            rc, U, phi, lam, info = arb.arb_solve(c2, wl.F, u_slip=wl.u_slip)
        finally:
            arb.arb_destroy(c2)
        assert rc in (arb.ARB_OK, arb.ARB_W_PINV_USED)
        assert info["rel_residual_fp64"] <= tol
        yg = np.concatenate([lam.ravel(), U.ravel(), phi])
        true_res = np.linalg.norm(S["b"] - S["A"] @ yg) / bnorm
        # rounding of the two FP64 products (library and dense oracle)
        slack = 1e-13 * np.linalg.norm(np.abs(S["A"]) @ np.abs(yg)) / bnorm
        got = dict(lam=lam.ravel(), U=U.ravel())
        if wl.n_rows:
            got["phi"] = phi
        errs = {k: rel(got[k], ref[k]) for k in ref}
        print(f"  fp32c solve to {tol:.1e} (refine_final {final}): errors {errs} residual "
              f"{info['rel_residual_fp64']:.1e} (oracle {true_res:.1e}, bounded "
              f"{info['residual_bounded']}), {info['iterations']} iterations, "
              f"{info['products_fp64']} FP64 products")
        if info["residual_bounded"]:
            assert final == 0 and info["products_fp64"] >= 1
            assert true_res <= info["rel_residual"] + slack
        else:
            assert true_res <= tol + slack
    assert all(e <= 1e-5 for e in errs.values())


def test_rank_deficient_hinge_uses_pinv():
    # literal hinge: 6 link rows + motor row, rank 6 of 7 (Sec. 4.4); only U and
    # C^T phi are unique
    wl = W.bacteria(n_bact=2, side=40.0, seed=23, literal_hinge=True)
    S = system.assemble(wl)
    ctx = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-10)
    try:
        rc, U, phi, lam, info = arb.arb_solve(ctx, wl.F)
    finally:
        arb.arb_destroy(ctx)
    assert rc == arb.ARB_W_PINV_USED and info["pinv_used"] >= 1
    yd = system.solve_dense(S["A"], S["b"])
    N, M = wl.N, wl.M
    assert rel(U, yd[3 * N:3 * N + 6 * M]) <= 1e-8
    assert rel(S["C"].T @ phi, S["C"].T @ yd[3 * N + 6 * M:]) <= 1e-8


def test_rank_deficient_large_assembly_uses_pinv():
    # a colony of 14 plates whose second link per plate pair keeps its third
    # row (a repeat of the first link's): one assembly of 78 rows, rank 65, so
    # the block sweep's pivot test fails for it and the pseudo-inverse takes
    # over (Sec. 3.1 with Sec. 5.1); only U and C^T phi are unique
    wl = W.diatoms(n_col=1, kmin=14, kmax=14, seed=9, lattice=(1, 1, 1), literal=True)
    S = system.assemble(wl)
    assert S["C"].shape[0] == 78
    ctx = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-10)
    try:
        rc, U, phi, lam, info = arb.arb_solve(ctx, wl.F)
    finally:
        arb.arb_destroy(ctx)
    assert rc == arb.ARB_W_PINV_USED and info["pinv_used"] >= 1
    yd = system.solve_dense(S["A"], S["b"])
    N, M = wl.N, wl.M
    print(f"  78-row rank-deficient assembly: {info['iterations']} iterations, U "
          f"{rel(U, yd[3 * N:3 * N + 6 * M]):.1e}, C^T phi "
          f"{rel(S['C'].T @ phi, S['C'].T @ yd[3 * N + 6 * M:]):.1e}")
    assert rel(U, yd[3 * N:3 * N + 6 * M]) <= 1e-8
    assert rel(S["C"].T @ phi, S["C"].T @ yd[3 * N + 6 * M:]) <= 1e-8


def test_euler_and_correction():
    wl = W.filament()
    S = system.assemble(wl)
    ctx = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-12)
    try:
        rc, U, phi, lam, info = arb.arb_solve(ctx, wl.F)
        q1, t1 = arb.arb_euler_update(ctx, U.ravel(), 0.1)
        qo, to = correct.euler_update(wl.q, wl.theta, U.ravel(), 0.1)
        assert np.abs(q1 - qo).max() <= 1e-14 and np.abs(t1 - to).max() <= 1e-15
        q2, t2, it, res = arb.arb_correct_positions(ctx, tol=1e-12, max_iter=50)
    finally:
        arb.arb_destroy(ctx)
    qc, tc, oi = correct.correct(wl, qo, to, tol=1e-12)
    assert it == oi["iterations"] and it < 5
    assert res <= 1e-10
    assert np.linalg.norm(bodies.link_residual(wl, q2, t2)) <= 1e-10
    dq, dqo = q2 - q1, qc - qo
    assert np.linalg.norm(dq - dqo) <= 1e-8 * np.linalg.norm(dqo)
    assert np.abs(t2 - tc).max() <= 1e-12


def test_error_paths():
    wl = W.random_rigid(2, 12, seed=5, wall=True)
    ctx = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-14, max_iter=1)
    try:
        rc, *_ = arb.arb_solve(ctx, wl.F)
        assert rc == arb.ARB_W_NOT_CONVERGED
        with pytest.raises(arb.ArbError) as e:
            arb.arb_solve(ctx, np.full(6 * wl.M, np.nan))
        assert e.value.code == arb.ARB_E_NAN
        q = wl.q.copy()
        q[0, 2] = 0.5  # pushes blobs through the wall
        with pytest.raises(arb.ArbError) as e:
            arb.arb_set_state(ctx, q, wl.theta)
        assert e.value.code == arb.ARB_E_BELOW_WALL
        with pytest.raises(arb.ArbError) as e:
            arb.arb_set_state(ctx, wl.q, 2 * wl.theta)
        assert e.value.code == arb.ARB_E_ARG
    finally:
        arb.arb_destroy(ctx)


@pytest.mark.parametrize("n_helix", [150, 170])
def test_preconditioner_large_bodies(n_helix):
    # a long helix (3n = 450: the blocked factorisation at its largest LDS
    # footprint; 3n = 510: the unblocked path for bodies beyond 480 rows) next
    # to a 42-blob shell, above the wall
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(40 + n_helix)
    hel = W.helix80(n_helix, length=60.0)
    hel -= hel.mean(0)
    r_ref = np.vstack([hel, W.icosphere42(5.0)])
    blob_offset = np.array([0, n_helix, n_helix + 42], np.int32)
    q = np.array([[0.0, 0.0, 35.0], [40.0, 0.0, 10.0]])
    theta = W._quat_scalar_first(Rotation.random(2, random_state=rng))
    wl = W.Workload("large", 1.0, 1.0, True, r_ref, blob_offset, q, theta,
                    rng.standard_normal((2, 6)), **W._links(0))
    print(f"large bodies: helix {n_helix} blobs", flush=True)
    S = system.assemble(wl)
    ctx = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-10)
    try:
        rc = arb.arb_precond_build(ctx)
        assert rc in (arb.ARB_OK, arb.ARB_W_PINV_USED)
        P = precond.BlockPreconditioner(wl, S["r"], S["C"])
        for p in range(wl.M):
            m = 3 * int(wl.blob_offset[p + 1] - wl.blob_offset[p])
            L, Nt = arb.arb_precond_block(ctx, p, m)
            assert rel(L, P.L[p]) <= 1e-13
            assert rel(Nt, P.Nt[p]) <= 1e-11
        r = rng.standard_normal(S["A"].shape[0])
        assert rel(arb.arb_precond_apply(ctx, r), P.apply(r)) <= 1e-11
    finally:
        arb.arb_destroy(ctx)


@pytest.mark.parametrize("name,prec", [("filament", arb.ARB_FP64), ("bacteria4", arb.ARB_FP32C),
                                       ("diatoms2", arb.ARB_FP64)])
def test_graph_replays_match_plain_launches(name, prec):
    # the GMRES iteration captured in HIP graphs: every solve (the first
    # captures, the later ones replay, with plain launches and host syncs in
    # between) gives bit for bit the iterates of plain launches (the kernel per
    # operation path, which small systems would otherwise not take)
    wl = cases()[name]()
    tol = 1e-10 if prec == arb.ARB_FP64 else 1e-6
    outs = {}
    for graphs in (1, 0):
        c = arb.context_for(wl, precision=prec, tol=tol, graphs=graphs, small_cycle=1)
        try:
            outs[graphs] = [arb.arb_solve(c, wl.F, u_slip=wl.u_slip) for _ in range(3)]
        finally:
            arb.arb_destroy(c)
    ref = outs[1][0]
    print(f"{name}: {ref[4]['iterations']} iterations", flush=True)
    for rc, U, phi, lam, info in outs[0] + outs[1]:
        assert rc == ref[0] and info["iterations"] == ref[4]["iterations"]
        assert np.array_equal(U, ref[1]) and np.array_equal(phi, ref[2])
        assert np.array_equal(lam, ref[3])


@pytest.mark.parametrize("name", list(cases()))
def test_one_launch_cycle_matches_per_step_kernels(name):
    # small FP64 systems (at most 128 blobs: the filament and the rigid chain
    # here) run each GMRES cycle in one workgroup with the stopping test on the
    # device; the kernel-per-operation path takes the same steps (summation
    # orders differ), so the iteration counts agree within one and every output
    # to 1e-12.  Larger systems keep the per-step path.
    wl = cases()[name]()
    res = {}
    for sc in (0, 1):
        c = arb.context_for(wl, precision=arb.ARB_FP64, tol=1e-10, small_cycle=sc)
        try:
            rc, U, phi, lam, info = arb.arb_solve(c, wl.F, u_slip=wl.u_slip)
        finally:
            arb.arb_destroy(c)
        assert rc in (arb.ARB_OK, arb.ARB_W_PINV_USED)
        assert info["rel_residual"] <= 1e-10
        res[sc] = (np.concatenate([np.ravel(lam), np.ravel(U), np.ravel(phi)]), info)
    (y0, i0), (y1, i1) = res[0], res[1]
    print(f"{name}: one launch {i0['iterations']} iterations in {i0['one_launch_cycles']} "
          f"cycles, {i0['t_solve_ms']:.2f} ms; per step {i1['iterations']}, "
          f"{i1['t_solve_ms']:.2f} ms; difference {rel(y0, y1):.1e}", flush=True)
    assert (i0["one_launch_cycles"] >= 1) == (wl.N <= 128) and i1["one_launch_cycles"] == 0
    assert abs(i0["iterations"] - i1["iterations"]) <= 1
    for key in outputs(wl, y1):
        assert rel(outputs(wl, y0)[key], outputs(wl, y1)[key]) <= 1e-12, key


@pytest.mark.parametrize("cfg", ["bacteria1024", "diatoms256"])
def test_full_size_solve_sampled(cfg):
    # the benchmark's FP32 solves at full size: the returned iterate meets 1e-6 with
    # the library's FP64 product, and that product matches the oracle on sampled
    # blob rows and on every body and constraint row
    from oracle import rpy

    wl = W.bacteria(n_bact=1024, seed=3) if cfg == "bacteria1024" else W.diatoms()
    N, M = wl.N, wl.M
    print(f"full size {cfg}: N={N} M={M} Nc={wl.n_rows}", flush=True)
    c = arb.context_for(wl, precision=arb.ARB_FP32C, tol=1e-6, restart=100, max_iter=1000)
    try:
        rc, U, phi, lam, info = arb.arb_solve(c, wl.F, u_slip=wl.u_slip)
    finally:
        arb.arb_destroy(c)
    assert rc in (arb.ARB_OK, arb.ARB_W_PINV_USED)
    assert info["rel_residual_fp64"] <= 1e-6
    y = np.concatenate([lam.ravel(), U.ravel(), phi])
    c64 = arb.context_for(wl, precision=arb.ARB_FP64)
    try:
        Ay = arb.arb_system_apply(c64, y)
    finally:
        arb.arb_destroy(c64)
    Cs, B = bodies.constraint_rows(wl, sparse=True)
    us = np.zeros(3 * N) if wl.u_slip is None else wl.u_slip.ravel()
    b = np.concatenate([us, -wl.F.ravel(), B])
    res = np.linalg.norm(Ay - b) / np.linalg.norm(b)
    print(f"  {info['iterations']} iterations, residual {res:.2e} (reported "
          f"{info['rel_residual']:.2e}, bounded {info['residual_bounded']}, "
          f"{info['products_fp64']} FP64 products)", flush=True)
    assert res <= 1.01e-6
    if info["residual_bounded"]:
        assert res <= info["rel_residual"] * 1.01
    r = bodies.blob_positions(wl.q, wl.theta, wl.r_ref, wl.blob_offset)
    KU = bodies.K_apply(r, wl.q, wl.blob_offset, U)
    tg = np.unique(np.concatenate([[0, N - 1], np.random.default_rng(5).integers(0, N, 24)]))
    Ml = rpy.mobility_apply(r, lam, wl.a, wl.eta, wl.wall, targets=tg)
    Ml_gpu = Ay[:3 * N].reshape(N, 3)[tg] + KU[tg]
    assert rel(Ml_gpu, Ml) <= 1e-12
    KTl = bodies.KT_apply(r, wl.q, wl.blob_offset, lam).ravel()
    CTp = Cs.T @ phi
    body_rows = Ay[3 * N:3 * N + 6 * M]
    scale = np.linalg.norm(KTl) + np.linalg.norm(CTp)
    assert np.linalg.norm(body_rows - (-KTl + CTp)) <= 1e-12 * scale
    CU = Cs @ U.ravel()
    assert np.linalg.norm(Ay[3 * N + 6 * M:] - CU) <= 1e-12 * np.linalg.norm(CU)


def test_solve_work_counts():
    """The solve's counts of products and preconditioner applications: FP32
    refinement takes one FP32 product per inner Arnoldi step and one FP64
    product per refinement residual; FP64 GMRES one product per step plus one
    per true-residual check at the end of a cycle."""
    wl = W.bacteria(n_bact=4, side=60.0, seed=21)
    for prec in (arb.ARB_FP32C, arb.ARB_FP64):
        ctx = arb.context_for(wl, precision=prec, tol=1e-8)
        try:
            rc, U, phi, lam, info = arb.arb_solve(ctx, wl.F)
        finally:
            arb.arb_destroy(ctx)
        it = info["iterations"]
        print(f"  precision {prec}: iterations {it}, products {info['products_fp32']} + "
              f"{info['products_fp64']}, applies {info['precond_applies']}", flush=True)
        assert info["precond_applies"] >= it + 1
        if prec == arb.ARB_FP32C:
            assert it <= info["products_fp32"] <= it + info["restarts"]
            assert 1 <= info["products_fp64"] <= 30
        else:
            assert info["products_fp32"] == 0
            assert it + 1 <= info["products_fp64"] <= it + 1 + info["restarts"]

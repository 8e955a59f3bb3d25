"""Pins of the saddle system, preconditioner, GMRES and correction oracles."""
import numpy as np
import pytest
from scipy.optimize import least_squares

from oracle import bodies, correct, gmres, precond, system
from paper_2107_10800_amd import workloads as W


@pytest.fixture(scope="module")
def fil():
    wl = W.filament()
    S = system.assemble(wl)
    return wl, S


@pytest.fixture(scope="module")
def rigid():
    wl = W.random_rigid(3, 12, seed=7, wall=True)
    return wl, system.assemble(wl)


def test_saddle_symmetric(fil, rigid):
    for wl, S in (fil, rigid):
        A = S["A"]
        assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()
        n = 3 * wl.N + 6 * wl.M + wl.n_rows
        assert A.shape == (n, n)
    assert fil[1]["A"].shape == (417, 417)


def test_two_direct_routes_agree(fil, rigid):
    for wl, S in (fil, rigid):
        y = system.solve_dense(S["A"], S["b"])
        lam, U, phi, _ = system.solve_formal(S["Mmat"], S["K"], S["C"], S["u_s"],
                                             np.ravel(wl.F), S["B"])
        yf = np.concatenate([lam, U, phi])
        assert np.linalg.norm(yf - y) <= 1e-11 * np.linalg.norm(y)
        assert np.linalg.norm(S["A"] @ y - S["b"]) <= 1e-13 * np.linalg.norm(S["b"])


def test_projector_and_constraints(fil):
    wl, S = fil
    lam, U, phi, ex = system.solve_formal(S["Mmat"], S["K"], S["C"], S["u_s"],
                                          np.ravel(wl.F), S["B"])
    C, N, G = S["C"], ex["N"], ex["G"]
    Q = np.eye(6 * wl.M) - N @ C.T @ G @ C
    assert np.abs(Q @ Q - Q).max() < 1e-10 * np.abs(Q).max()
    assert np.abs(C @ U - S["B"]).max() < 1e-12 * np.abs(U).max()
    # passive links do no work: U . C^T phi = phi . B = 0
    Fc = C.T @ phi
    assert abs(U @ Fc) < 1e-12 * np.linalg.norm(U) * np.linalg.norm(Fc)
    # App. A: no net constraint force or torque (about the origin) on the assembly
    Fc = Fc.reshape(-1, 6)
    assert np.abs(Fc[:, :3].sum(0)).max() < 1e-12 * np.abs(Fc).max()
    torque = Fc[:, 3:].sum(0) + np.cross(wl.q, Fc[:, :3]).sum(0)
    assert np.abs(torque).max() < 1e-11 * np.abs(Fc).max()


def test_axial_spin_null_space(fil):
    # collinear rods: the spin about each rod axis is resistance free (reading R6)
    wl, S = fil
    A = S["A"]
    N, M = wl.N, wl.M
    for p in range(M):
        y0 = np.zeros(A.shape[0])
        y0[3 * N + 6 * p + 3:3 * N + 6 * p + 6] = wl.extra["axis"][p]
        assert np.abs(A @ y0).max() < 1e-14
        assert abs(S["b"] @ y0) < 1e-13
    # the minimum-norm solution carries no axial spin
    y = system.solve_dense(A, S["b"])
    U = y[3 * N:3 * N + 6 * M].reshape(M, 6)
    assert np.abs(np.einsum("ij,ij->i", U[:, 3:], wl.extra["axis"])).max() < 1e-12


def test_preconditioner_exact_for_one_body():
    wl = W.random_rigid(1, 12, seed=3, wall=True)
    S = system.assemble(wl)
    P = precond.BlockPreconditioner(wl, S["r"], S["C"])
    y = P.apply(S["b"])
    assert np.linalg.norm(S["A"] @ y - S["b"]) < 1e-12 * np.linalg.norm(S["b"])
    # U-hat = N (F - K^T M^-1 u_s)  (Sec. 2.3 with M -> M~)
    Minv = np.linalg.inv(S["Mmat"])
    Nb = np.linalg.inv(S["K"].T @ Minv @ S["K"])
    Uhat = Nb @ (np.ravel(wl.F) - S["K"].T @ Minv @ S["u_s"])
    assert np.allclose(y[3 * wl.N:3 * wl.N + 6], Uhat, rtol=1e-11, atol=1e-13)
    _, info = gmres.gmres(lambda v: S["A"] @ v, P.apply, S["b"], tol=1e-10)
    assert info["iterations"] == 1


def test_gmres_matches_direct(fil, rigid):
    for wl, S in (fil, rigid):
        A, b = S["A"], S["b"]
        P = precond.BlockPreconditioner(wl, S["r"], S["C"])
        y = system.solve_dense(A, b)
        rec = {}
        yg, info = gmres.gmres(lambda v: A @ v, P.apply, b, tol=1e-14, record=rec)
        assert info["true_rel"] <= 1e-13
        assert np.linalg.norm(yg - y) <= 1e-11 * np.linalg.norm(y)
        # Arnoldi relation A P^-1 V_k = V_{k+1} H_k and orthonormal basis
        k = min(rec["k"], 20)
        V = np.vstack([rec["V"][:k + 1]])
        V[k] = rec["V"][k] if k < rec["k"] else rec["w_last"]
        H = rec["Hraw"][:k + 1, :k]
        AV = np.column_stack([A @ P.apply(V[j]) for j in range(k)])
        assert np.abs(AV - V.T @ H).max() < 1e-12 * np.abs(AV).max()
        assert np.abs(V @ V.T - np.eye(k + 1)).max() < 1e-13


def test_left_preconditioned_gmres(fil, rigid):
    # the left variant (P^-1 A, the form Sec. 3.1 names): exact in one iteration
    # when the preconditioner is the inverse (one body), equal to the direct
    # solve at a tight tolerance, the Arnoldi relation of P^-1 A, and a true
    # residual below the tolerance at every exit
    wl1 = W.random_rigid(1, 12, seed=3, wall=True)
    S1 = system.assemble(wl1)
    P1 = precond.BlockPreconditioner(wl1, S1["r"], S1["C"])
    _, info = gmres.gmres(lambda v: S1["A"] @ v, P1.apply, S1["b"], tol=1e-10, left=True)
    assert info["iterations"] == 1 and info["true_rel"] <= 1e-10
    for wl, S in (fil, rigid):
        A, b = S["A"], S["b"]
        P = precond.BlockPreconditioner(wl, S["r"], S["C"])
        y = system.solve_dense(A, b)
        rec = {}
        yg, info = gmres.gmres(lambda v: A @ v, P.apply, b, tol=1e-14, record=rec, left=True)
        assert info["true_rel"] <= 1e-13
        assert np.linalg.norm(yg - y) <= 1e-11 * np.linalg.norm(y)
        k = min(rec["k"], 20)
        V = np.vstack([rec["V"][:k + 1]])
        V[k] = rec["V"][k] if k < rec["k"] else rec["w_last"]
        H = rec["Hraw"][:k + 1, :k]
        PAV = np.column_stack([P.apply(A @ V[j]) for j in range(k)])
        assert np.abs(PAV - V.T @ H).max() < 1e-12 * np.abs(PAV).max()
        assert np.abs(V @ V.T - np.eye(k + 1)).max() < 1e-13
        # the first basis vector is P^-1 b normalised (zero initial guess)
        z0 = P.apply(b)
        assert np.allclose(rec["V"][0], z0 / np.linalg.norm(z0), rtol=0, atol=1e-14)
        for tol in (1e-6, 1e-10):
            _, inf = gmres.gmres(lambda v: A @ v, P.apply, b, tol=tol, left=True)
            assert inf["converged"] and inf["true_rel"] <= tol


def test_unpreconditioned_gmres_is_slow(fil):
    # Sec. 3.2.1: without preconditioner iterations scale with the system size
    wl, S = fil
    _, info = gmres.gmres(lambda v: S["A"] @ v, lambda v: v, S["b"], tol=1e-10,
                          restart=500, max_iter=2000)
    P = precond.BlockPreconditioner(wl, S["r"], S["C"])
    _, info_pc = gmres.gmres(lambda v: S["A"] @ v, P.apply, S["b"], tol=1e-10)
    assert info["iterations"] > 100 and info["iterations"] > 5 * info_pc["iterations"]


def test_jacobian_finite_differences(fil):
    wl, _ = fil
    rng = np.random.default_rng(0)
    M = wl.M
    x = np.zeros(7 * M)
    X = x.reshape(M, 7)
    X[:, :3] = 1e-2 * rng.standard_normal((M, 3))
    X[:, 3:] = rng.standard_normal((M, 4))
    J = correct.jacobian(wl, wl.q, wl.theta, x)
    Jfd = np.zeros_like(J)
    h = 1e-6
    for k in range(len(x)):
        e = np.zeros_like(x)
        e[k] = h
        Jfd[:, k] = (correct.residual(wl, wl.q, wl.theta, x + e)
                     - correct.residual(wl, wl.q, wl.theta, x - e)) / (2 * h)
    assert np.abs(J - Jfd).max() < 1e-7
    # App. B: 30 non-zeros per link in the constraint rows (generic geometry)
    wr = W.random_rigid(4, 12, seed=9, wall=False)
    xr = rng.standard_normal(7 * wr.M)
    Jr = correct.jacobian(wr, wr.q, wr.theta, xr)
    assert np.count_nonzero(Jr[:3 * wr.P]) == 30 * wr.P


def test_correction_after_euler_step(fil):
    wl, S = fil
    y = system.solve_dense(S["A"], S["b"])
    U = y[3 * wl.N:3 * wl.N + 6 * wl.M]
    q1, t1 = correct.euler_update(wl.q, wl.theta, U, 0.1)
    g1 = np.linalg.norm(bodies.link_residual(wl, q1, t1))
    assert g1 > 1e-8
    q2, t2, info = correct.correct(wl, q1, t1, tol=1e-12)
    assert info["iterations"] < 5
    assert np.linalg.norm(bodies.link_residual(wl, q2, t2)) <= 1e-10
    assert np.allclose(np.linalg.norm(t2, axis=1), 1.0, atol=1e-14)
    # SciPy least squares on the same problem (the paper's solver) reaches the
    # same constraint level with a correction of the same size and direction.
    x0 = np.zeros(7 * wl.M)
    x0.reshape(wl.M, 7)[:, 3] = 1.0
    sol = least_squares(lambda x: correct.residual(wl, q1, t1, x), x0,
                        jac=lambda x: correct.jacobian(wl, q1, t1, x), method="trf",
                        xtol=1e-15, ftol=1e-15, gtol=1e-15)
    assert np.linalg.norm(sol.fun) < 1e-10
    dq_s = sol.x.reshape(wl.M, 7)[:, :3]
    assert np.linalg.norm(dq_s - (q2 - q1)) < 0.05 * np.linalg.norm(q2 - q1)

"""Pins of the time-integration oracle (Sec. 4): reconstruction and Euler step.

Each check rests on something other than the oracle's own pseudo-inverse
formula: the robot-arm chain walk of Sec. 4.1 (Eq. robot-arm), the normal
equations that characterise a least-squares solution, the paper's statements
that loop-free articulated bodies are rebuilt exactly and that the constraint
error of an explicit Euler step decays as dt^2 (Sec. 4.2, Fig.
convergence_nonlinear a), and invariants (zero-mean pseudo-inverse solution,
fixed points)."""
import numpy as np
import pytest

from oracle import bodies, correct, timeloop
from oracle.correct import link_assemblies
from oracle.quat import quat_from_rotvec, quat_mul, rotation_matrix
from paper_2107_10800_amd import workloads as W


def _perturb(theta, scale, seed):
    rng = np.random.default_rng(seed)
    return quat_mul(quat_from_rotvec(scale * rng.standard_normal((len(theta), 3))), theta)


def _tree():
    """Four rods joined as a branched tree: 0-1, 0-2 (mid-rod branch), 2-3."""
    wl = W.filament(n_rods=4, seed=3)
    wl.pq = np.array([[0, 1], [0, 2], [2, 3]], np.int32)
    wl.dl_p = np.array([[4.0, 0, 0], [0.0, 0, 0], [4.0, 0, 0]])
    wl.dl_q = np.array([[-4.0, 0, 0], [-4.0, 0, 0], [-4.0, 0, 0]])
    for k in ("dldot_p", "dldot_q"):
        setattr(wl, k, np.zeros((3, 3)))
    wl.nproj = np.full(3, 3, np.int32)
    wl.proj = np.tile(np.eye(3), (3, 1, 1))
    return wl


def test_robot_arm_equivalence_for_a_chain():
    """For a linear chain the reconstruction equals the robot-arm walk (Eq.
    robot-arm) from body 1, shifted to the same centre of mass (Sec. 4.1)."""
    wl = W.filament(n_rods=12, seed=5)
    th = _perturb(wl.theta, 0.4, 1)
    R = rotation_matrix(th)
    walk = np.zeros_like(wl.q)
    for n in range(wl.M - 1):          # link n: q_n + R_n dl_p = q_{n+1} + R_{n+1} dl_q
        walk[n + 1] = walk[n] + R[n] @ wl.dl_p[n] - R[n + 1] @ wl.dl_q[n]
    q_in = wl.q + np.random.default_rng(2).standard_normal(wl.q.shape)
    walk += q_in.mean(0) - walk.mean(0)
    out = timeloop.reconstruct(wl, q_in, th)
    assert np.abs(out - walk).max() < 1e-12


@pytest.mark.parametrize("name", ["ring", "filament", "bacteria", "diatoms"])
def test_pinv_solution_has_zero_mean(name):
    """The minimum-norm solution has no null-space component, i.e. zero COM (Sec. 4.1)."""
    wl = dict(ring=lambda: W.ring(), filament=lambda: W.filament(),
              bacteria=lambda: W.bacteria(n_bact=2, side=200.0),
              diatoms=lambda: W.diatoms(n_col=2, kmin=5, kmax=7))[name]()
    th = _perturb(wl.theta, 0.2, 3)
    for b, l in link_assemblies(wl):
        qt = timeloop.pinv_positions(wl, b, l, th)
        assert np.abs(qt.mean(0)).max() < 1e-12 * (1 + np.abs(qt).max())


@pytest.mark.parametrize("name", ["ring", "filament", "bacteria", "diatoms"])
def test_consistent_state_is_a_fixed_point(name):
    """Positions that satisfy every link are rebuilt unchanged."""
    wl = dict(ring=lambda: W.ring(), filament=lambda: W.filament(),
              bacteria=lambda: W.bacteria(n_bact=2, side=200.0),
              diatoms=lambda: W.diatoms(n_col=2, kmin=5, kmax=7))[name]()
    assert np.abs(bodies.link_residual(wl, wl.q, wl.theta)).max() < 1e-12
    out = timeloop.reconstruct(wl, wl.q, wl.theta)
    assert np.abs(out - wl.q).max() < 1e-12


@pytest.mark.parametrize("make", [lambda: W.filament(n_rods=15, seed=9), _tree])
def test_loop_free_bodies_are_rebuilt_exactly(make):
    """Chains and branched trees obey every link after reconstruction, for any
    orientations (Sec. 4.2: only loops can leave a violation)."""
    wl = make()
    th = _perturb(wl.theta, 0.5, 4)
    out = timeloop.reconstruct(wl, wl.q, th)
    assert np.abs(bodies.link_residual(wl, out, th)).max() < 1e-12


def test_loop_reconstruction_is_the_least_squares_solution():
    """With a loop the links cannot all hold; the rebuilt positions satisfy the
    normal equations P^T g = 0 (sum of +-g_n over each body's links vanishes)."""
    wl = W.ring(n_bodies=7)
    th = _perturb(wl.theta, 0.1, 5)
    out = timeloop.reconstruct(wl, wl.q, th)
    g = bodies.link_residual(wl, out, th)
    assert np.abs(g).max() > 1e-3
    ne = np.zeros((wl.M, 3))
    for n, (p, qq) in enumerate(wl.pq):
        ne[p] += g[n]
        ne[qq] -= g[n]
    assert np.abs(ne).max() < 1e-12
    # any other placement with the same COM has a larger residual
    rng = np.random.default_rng(6)
    for _ in range(5):
        d = 1e-3 * rng.standard_normal(out.shape)
        d -= d.mean(0)
        g2 = bodies.link_residual(wl, out + d, th)
        assert (g2 ** 2).sum() > (g ** 2).sum()


def test_anchored_chain():
    """A chain tied to a fixed lab point is rebuilt exactly and independently of
    the incoming tracking points (no translational freedom)."""
    wl = W.filament(n_rods=6, seed=2)
    R0 = rotation_matrix(wl.theta[0])
    anchor = wl.q[0] + R0 @ np.array([-4.0, 0, 0])
    wl.pq = np.vstack([wl.pq, [[0, -1]]]).astype(np.int32)
    wl.dl_p = np.vstack([wl.dl_p, [[-4.0, 0, 0]]])
    wl.dl_q = np.vstack([wl.dl_q, [anchor]])
    wl.dldot_p = np.vstack([wl.dldot_p, np.zeros((1, 3))])
    wl.dldot_q = np.vstack([wl.dldot_q, np.zeros((1, 3))])
    wl.nproj = np.append(wl.nproj, 3).astype(np.int32)
    wl.proj = np.concatenate([wl.proj, np.eye(3)[None]])
    th = _perturb(wl.theta, 0.3, 7)
    out1 = timeloop.reconstruct(wl, wl.q, th)
    out2 = timeloop.reconstruct(wl, wl.q + 5.0, th)
    assert np.abs(out1 - out2).max() < 1e-12
    assert np.abs(bodies.link_residual(wl, out1, th)).max() < 1e-12


def test_euler_constraint_error_is_second_order():
    """E3 (Sec. 4.2): from a state that obeys the links, one explicit Euler step
    of a loop leaves ||g||_inf ~ dt^2; an open chain leaves none."""
    wl = W.ring()
    U, _ = timeloop.solve_velocities(wl, wl.q, wl.theta)
    errs = []
    for dt in (0.2, 0.1, 0.05):
        _, _, info = timeloop.euler_step(wl, wl.q, wl.theta, dt, delta=np.inf, U=U)
        assert not info["corrected"]
        errs.append(info["g_inf_star"])
    assert errs[0] > 1e-8
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4
    fl = W.filament()
    for dt in (0.2, 0.05):
        _, _, info = timeloop.euler_step(fl, fl.q, fl.theta, dt, delta=np.inf)
        assert info["g_inf_star"] < 1e-12


def test_euler_step_moves_the_com_with_the_mean_velocity():
    """Eq. ucom and step 3: the rebuilt articulated body is centred at
    q_COM + dt u_COM; orientations follow theta_{w dt} . theta."""
    wl = W.ring()
    U = np.random.default_rng(8).standard_normal((wl.M, 6))
    dt = 0.07
    _, _, info = timeloop.euler_step(wl, wl.q, wl.theta, dt, delta=np.inf, U=U)
    assert np.abs(info["q_star"].mean(0) - (wl.q.mean(0) + dt * U[:, :3].mean(0))).max() < 1e-12
    for p in range(wl.M):
        w = U[p, 3:]
        ang = np.linalg.norm(w) * dt
        Rw = rotation_matrix(quat_from_rotvec(w * dt))
        # the rotation by w dt about w: axis fixed, angle |w| dt (Rodrigues)
        assert np.abs(Rw @ w - w).max() < 1e-12
        assert abs(np.trace(Rw) - (1 + 2 * np.cos(ang))) < 1e-12
        assert np.abs(rotation_matrix(info["theta_star"][p]) - Rw @ rotation_matrix(wl.theta[p])).max() < 1e-12


def test_euler_step_with_correction_meets_tolerance():
    """When ||g*||^2 >= delta the correction of Sec. 4.2 brings the links to
    its tolerance in a few iterations (Fig. convergence_nonlinear b)."""
    wl = W.ring()
    q, th, info = timeloop.euler_step(wl, wl.q, wl.theta, 0.2, delta=1e-20, corr_tol=1e-12)
    assert info["corrected"] and info["corr"]["iterations"] <= 5
    assert info["corr"]["residual"] <= 1e-12
    # normalising the quaternion increments afterwards moves g by ~ |dl| x 1e-12
    assert info["g_inf"] < 1e-10
    assert np.allclose(np.linalg.norm(th, axis=1), 1.0, atol=1e-14)
    # and a step whose check passes is taken as rebuilt
    q2, th2, info2 = timeloop.euler_step(wl, wl.q, wl.theta, 0.2, delta=1.0)
    assert not info2["corrected"]
    assert np.array_equal(q2, info2["q_star"])


def test_bodies_without_links_take_the_plain_euler_step():
    wl = W.random_rigid(n_bodies=3, blobs=12, seed=7, links="none")
    U = np.random.default_rng(9).standard_normal((wl.M, 6))
    q, th, info = timeloop.euler_step(wl, wl.q, wl.theta, 0.1, delta=np.inf, U=U)
    assert np.abs(q - (wl.q + 0.1 * U[:, :3])).max() < 1e-15


def _integrate(wl, step, T, n, **kw):
    q, th = wl.q.copy(), wl.theta.copy()
    for _ in range(n):
        q, th, _ = step(wl, q, th, T / n, **kw)
    return q, th


def test_global_order_euler_one_midpoint_two():
    """Sec. 4.4 and App. C: with reconstruction and correction, explicit Euler
    keeps first-order and the explicit midpoint scheme second-order global
    convergence (errors at t = 2 against 64 midpoint steps, ring of 6 bodies)."""
    wl = W.ring(n_bodies=6)
    wl.F = 20.0 * wl.F
    T = 2.0
    kw = dict(delta=1e-20, corr_tol=1e-13)
    ref = _integrate(wl, timeloop.midpoint_step, T, 64, **kw)[0]
    for step, order in ((timeloop.euler_step, 1), (timeloop.midpoint_step, 2)):
        errs = [np.abs(_integrate(wl, step, T, n, **kw)[0] - ref).max() for n in (4, 8, 16)]
        for a, b in zip(errs, errs[1:]):
            assert 0.8 * 2 ** order < a / b < 1.25 * 2 ** order, (step.__name__, errs)


def test_midpoint_step_stages():
    """App. C: the half step uses U^k over dt/2, the full step restarts from the
    initial state with the midpoint velocities over dt."""
    wl = W.ring()
    q, th, info = timeloop.midpoint_step(wl, wl.q, wl.theta, 0.3, delta=np.inf)
    qh, thh, _ = timeloop.advance(wl, wl.q, wl.theta, info["U0"], 0.15, np.inf)
    assert np.allclose(info["half"]["q_star"], qh, atol=0, rtol=0)
    U_half, _ = timeloop.solve_velocities(wl, qh, thh)
    assert np.allclose(info["U_half"], U_half, atol=1e-14)
    q2, th2, _ = timeloop.advance(wl, wl.q, wl.theta, U_half, 0.3, np.inf)
    assert np.abs(q - q2).max() < 1e-13 and np.abs(th - th2).max() < 1e-13


def _colony(t):
    # one colony of three plates whose link arms slide in time (Sec. 5.1)
    return W.diatoms(n_col=1, kmin=3, kmax=3, seed=31, lattice=(1, 1, 1), t=t)


def test_arms_steps_with_fixed_arms_are_the_plain_steps():
    """With the same arms at every stage time the steps for time-dependent arms
    are the plain steps, bit for bit."""
    wl = _colony(0.3)
    a = timeloop.euler_step_arms(wl, wl, wl.q, wl.theta, 0.05, delta=np.inf)
    b = timeloop.euler_step(wl, wl.q, wl.theta, 0.05, delta=np.inf)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    a = timeloop.midpoint_step_arms(wl, wl, wl, wl.q, wl.theta, 0.05, delta=np.inf)
    b = timeloop.midpoint_step(wl, wl.q, wl.theta, 0.05, delta=np.inf)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _integrate_arms(step, T, n, stage_arms=True, **kw):
    wl = _colony(0.0)
    q, th = wl.q.copy(), wl.theta.copy()
    dt = T / n
    for k in range(n):
        t = k * dt
        w0 = _colony(t)
        wh, w1 = (_colony(t + 0.5 * dt), _colony(t + dt)) if stage_arms else (w0, w0)
        if step == "euler":
            q, th, _ = timeloop.euler_step_arms(w0, w1, q, th, dt, **kw)
        else:
            q, th, _ = timeloop.midpoint_step_arms(w0, wh, w1, q, th, dt, **kw)
    return q


def test_moving_arms_keep_the_orders_only_with_stage_arms():
    """Sliding plates driven by their arms alone (no forces): with the arms of
    each stage time (App. C with Sec. 2.2) explicit Euler converges at first
    and the midpoint scheme at second order; the midpoint scheme that keeps the
    arms of the start of each step for its later stages falls to first order
    (errors at t = 0.4 against 128 midpoint steps)."""
    T = 0.4
    kw = dict(delta=1e-20, corr_tol=1e-13)
    ref = _integrate_arms("midpoint", T, 128, **kw)
    for step, stage, order in (("euler", True, 1), ("midpoint", True, 2),
                               ("midpoint", False, 1)):
        errs = [np.abs(_integrate_arms(step, T, n, stage, **kw) - ref).max() for n in (8, 16, 32)]
        print(step, stage, errs)
        for a, b in zip(errs, errs[1:]):
            assert 0.75 * 2 ** order < a / b < 1.3 * 2 ** order, (step, stage, errs)


def _shell_solve(wl, q, theta, F):
    from oracle import single_blob
    S = single_blob.assemble(wl, q, theta, F)
    return single_blob.solve_dense(S)[:6 * wl.M].reshape(-1, 6)


def two_shells():
    # E6 (Sec. 4.4): two deformable shells of single blobs sedimenting side by side
    return W.blob_shells(forcing="gravity", centres=[[-1.5, 0.0, -1.5], [1.5, 0.0, 1.5]])


def test_two_sedimenting_shells_orders():
    """Sec. 4.4's two sedimenting shells (42 single-blob bodies and 60 links each,
    centres (+-1.5, 0, +-1.5) R, gravity): with reconstruction and correction
    explicit Euler converges at first and the midpoint scheme at second order
    (errors at t = 8 against 48 midpoint steps)."""
    wl = two_shells()
    T = 8.0
    kw = dict(delta=1e-20, corr_tol=1e-13, solve=_shell_solve)
    ref = _integrate(wl, timeloop.midpoint_step, T, 48, **kw)[0]
    for step, order in ((timeloop.euler_step, 1), (timeloop.midpoint_step, 2)):
        errs = [np.abs(_integrate(wl, step, T, n, **kw)[0] - ref).max() for n in (4, 8, 16)]
        print(step.__name__, ["%.2e" % e for e in errs])
        for a, b in zip(errs, errs[1:]):
            assert 0.75 * 2 ** order < a / b < 1.3 * 2 ** order, (step.__name__, errs)


def test_correction_iterations_stay_flat_with_shell_size():
    """E4 (Sec. 4.4): the correction of Sec. 4.2 needs fewer than five
    Levenberg-Marquardt iterations per articulated body whatever the shell's
    size: the 42-, 162- and 642-blob shells (60, 240, 960 links) with links
    violated by about 1e-2 (a time step's worth) reach 1e-10."""
    for level in (1, 2, 3):
        wl = W.blob_shells(level=level, seed=40 + level)
        rng = np.random.default_rng(7)
        q = wl.q + 2.5e-3 * rng.standard_normal(wl.q.shape)
        th = quat_mul(quat_from_rotvec(1e-3 * rng.standard_normal((wl.M, 3))), wl.theta)
        qc, tc, info = correct.correct(wl, q, th, tol=1e-10, max_iter=50)
        g = np.abs(bodies.link_residual(wl, qc, tc)).max()
        print(f"shell of {wl.M}: {info['iterations']} iterations, |g| {g:.1e}")
        assert info["iterations"] < 5 and g <= 1e-10

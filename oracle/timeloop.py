"""Time integration of articulated bodies with reconstruction and correction (Sec. 4), float64.

TEST INFRASTRUCTURE ONLY (see the package header): nothing in the product
path may use this module.

Sec. 4.1 (general reconstruction).  For one articulated body a, the link
equations g_n = 0 (Eq. constraint) are linear in the tracking points once the
orientations are fixed: with z_n = R(theta_p) dl_np - R(theta_q) dl_nq they
read P^a q^a = -z^a (Eq. Pq_eq_z), where row block n of P^a holds +I in the
column block of body p and -I in that of body q.  The rank of P^a is
3 (M_a - 1); its null space is a common shift of every q_p.  The minimum-norm
solution q~^a = -(P^a)^+ z^a (Eq. pseudo-inv-sol) has zero mean, and the
bodies are placed at q_p = q~_p + q^a_COM (Eq. reconst-up-COM), q_COM the mean
of the tracking points of the articulated body (Eq. ucom uses the same mean
for the velocities).

Sec. 4.3 (explicit Euler with reconstruction and correction), one step:
  1. solve the saddle system (Eq. linear_system) for U at the current state;
  2. u^a_COM = mean of u_p over the bodies of a (Eq. ucom);
  3. q^a_COM <- q^a_COM + dt u^a_COM, theta_p <- theta_{w_p dt} . theta_p;
  4. rebuild the bodies from the new orientations (Sec. 4.1);
  5. g* = g(q*, theta*): accepted if ||g*||_2^2 < delta, otherwise the
     correction of Sec. 4.2 is applied.
App. C (explicit midpoint): steps 2-5 over dt/2 with U^k give the midpoint
state; step 1 there gives U^(k+1/2); steps 2-5 over dt from the initial state
with U^(k+1/2) give the new state.

Readings (where the paper is silent):
  * q_COM at the start of a step is the mean of the current tracking points,
    so the state of the loop is (q, theta) alone; after a correction the next
    step starts from the mean of the corrected positions.
  * Bodies without links are single-body "articulated bodies": q~ = 0 and the
    update is the plain Euler step q_p <- q_p + dt u_p (Eq. dq_dt).
  * A link to a fixed lab point (q = -1 in the link table) has row block +I
    only and z_n = R(theta_p) dl_np - (that point).  An articulated body with
    such a link has no translational null space: it is placed at
    q = -(P^a)^+ z^a with no COM term.
  * The nonlinear correction runs to ||F||_2 <= corr_tol (its own tolerance)
    when the check of step 5 fails.
"""
from __future__ import annotations

import numpy as np

from . import bodies, system
from .correct import correct, link_assemblies
from .quat import quat_from_rotvec, quat_mul, rotation_matrix


def connectivity(wl, bodies_a, links_a, theta):
    """(P^a, z^a) of one articulated body (Eq. Pq_eq_z): P^a is 3 P_a x 3 M_a
    with +I / -I blocks, z^a(theta) the 3 P_a vector such that the link
    equations read P^a q^a = -z^a.  theta: (M,4) orientations of all bodies."""
    loc = {int(b): k for k, b in enumerate(bodies_a)}
    R = rotation_matrix(theta)
    P = np.zeros((3 * len(links_a), 3 * len(bodies_a)))
    z = np.zeros(3 * len(links_a))
    for e, n in enumerate(links_a):
        p, qq = int(wl.pq[n, 0]), int(wl.pq[n, 1])
        P[3 * e:3 * e + 3, 3 * loc[p]:3 * loc[p] + 3] += np.eye(3)
        z[3 * e:3 * e + 3] = R[p] @ wl.dl_p[n]
        if qq >= 0:
            P[3 * e:3 * e + 3, 3 * loc[qq]:3 * loc[qq] + 3] -= np.eye(3)
            z[3 * e:3 * e + 3] -= R[qq] @ wl.dl_q[n]
        else:
            z[3 * e:3 * e + 3] -= wl.dl_q[n]
    return P, z


def pinv_positions(wl, bodies_a, links_a, theta):
    """q~^a = -(P^a)^+ z^a (Eq. pseudo-inv-sol), shape (M_a, 3)."""
    P, z = connectivity(wl, bodies_a, links_a, theta)
    return -(np.linalg.pinv(P, rcond=1e-12) @ z).reshape(-1, 3)


def anchored(wl, links_a):
    """True when the articulated body has a link to a fixed lab point."""
    return bool(np.any(np.asarray(wl.pq)[np.asarray(links_a, int), 1] < 0))


def reconstruct(wl, q, theta, q_com=None):
    """Rebuild every articulated body from the orientations (Sec. 4.1).

    q_com: optional list, one (3,) COM per entry of link_assemblies(wl); by
    default the mean of the current tracking points q of that body.  Bodies
    without links keep q.  Returns the new (M,3) tracking points."""
    q = np.array(q, float)
    out = q.copy()
    for k, (bodies_a, links_a) in enumerate(link_assemblies(wl)):
        qt = pinv_positions(wl, bodies_a, links_a, theta)
        if anchored(wl, links_a):
            out[bodies_a] = qt
        else:
            com = q[bodies_a].mean(0) if q_com is None else np.asarray(q_com[k], float)
            out[bodies_a] = qt + com
    return out


def solve_velocities(wl, q, theta, F=None):
    """U (M,6) and y of the saddle system at the state (q, theta) by a dense
    minimum-norm solve (Eq. linear_system); F defaults to wl.F."""
    d = system.assemble(wl, q, theta)
    b = d["b"].copy()
    if F is not None:
        M = len(q)
        b[3 * wl.N:3 * wl.N + 6 * M] = -np.asarray(F, float).ravel()
    y = system.solve_dense(d["A"], b)
    _, U, _ = system.split(y, wl.N, len(q))
    return U.reshape(-1, 6), y


def advance(wl, q, theta, U, dt, delta, corr_tol=1e-10, corr_max_iter=50):
    """Steps 2-5 of Sec. 4.3 from the state (q, theta) with body velocities U (M,6)
    over dt: u_COM (Eq. ucom), COM and orientation update, rebuild (Sec. 4.1),
    check ||g*||^2 < delta, else the correction of Sec. 4.2.  Returns
    (q_new, theta_new, info) as euler_step."""
    q = np.array(q, float)
    theta = np.array(theta, float)
    U = np.asarray(U, float).reshape(-1, 6)
    # step 3 for the orientations, and the plain Euler step for bodies without links
    theta_s = quat_mul(quat_from_rotvec(dt * U[:, 3:]), theta)
    q_s = q + dt * U[:, :3]
    # steps 2-4 for every articulated body
    for bodies_a, links_a in link_assemblies(wl):
        qt = pinv_positions(wl, bodies_a, links_a, theta_s)
        if anchored(wl, links_a):
            q_s[bodies_a] = qt
        else:
            u_com = U[bodies_a, :3].mean(0)
            q_com = q[bodies_a].mean(0) + dt * u_com
            q_s[bodies_a] = qt + q_com
    # step 5
    g = bodies.link_residual(wl, q_s, theta_s)
    g2 = float(np.sum(g * g))
    info = dict(U=U, q_star=q_s, theta_star=theta_s, g_star=g, g2_star=g2,
                g_inf_star=float(np.max(np.abs(g))) if g.size else 0.0, corrected=False,
                corr=None)
    if g2 < delta:
        q_n, th_n = q_s, theta_s
    else:
        q_n, th_n, ci = correct(wl, q_s, theta_s, tol=corr_tol, max_iter=corr_max_iter)
        info.update(corrected=True, corr=ci)
    gn = bodies.link_residual(wl, q_n, th_n)
    info["g_inf"] = float(np.max(np.abs(gn))) if gn.size else 0.0
    return q_n, th_n, info


def euler_step(wl, q, theta, dt, delta, corr_tol=1e-10, corr_max_iter=50, F=None, U=None,
               solve=None):
    """One explicit Euler step with reconstruction and correction (Sec. 4.3).

    U: body velocities (M,6) to use instead of solving step 1 (for tests that
    compare the integrator alone); solve(wl, q, theta, F) -> U replaces the
    dense multiblob solve (e.g. for single-blob bodies).  Returns (q_new,
    theta_new, info) with info: U, q_star, theta_star, g_star (P,3), g2_star,
    g_inf_star, corrected, corr (the correction's info or None), g_inf (after
    the step)."""
    if U is None:
        U = (solve or _solve_multiblob)(wl, q, theta, F)
    return advance(wl, q, theta, U, dt, delta, corr_tol, corr_max_iter)


def midpoint_step(wl, q, theta, dt, delta, corr_tol=1e-10, corr_max_iter=50, F=None,
                  solve=None):
    """One explicit midpoint (RK2) step with reconstruction and correction (App. C):
    velocities U^k at the state; a half step dt/2 (rebuild, check, correction) to
    the midpoint state; velocities U^(k+1/2) there; the full step dt from the
    initial state with U^(k+1/2) (rebuild, check, correction).  Returns
    (q_new, theta_new, info) with info['half'] the half step's info and
    info['U_half'] = U^(k+1/2)."""
    solve = solve or _solve_multiblob
    U0 = solve(wl, q, theta, F)
    qh, thh, ih = advance(wl, q, theta, U0, 0.5 * dt, delta, corr_tol, corr_max_iter)
    Uh = solve(wl, qh, thh, F)
    qn, thn, info = advance(wl, q, theta, Uh, dt, delta, corr_tol, corr_max_iter)
    info.update(half=ih, U0=np.asarray(U0).reshape(-1, 6), U_half=np.asarray(Uh).reshape(-1, 6))
    return qn, thn, info


def euler_step_arms(wl0, wl1, q, theta, dt, delta, corr_tol=1e-10, corr_max_iter=50, F=None):
    """Explicit Euler (Sec. 4.3) for links whose arms change in time (Sec. 2.2,
    the arms and their rates in the link velocity rows): the velocities at t
    with the links of wl0 (arms at t), the rebuild, check and correction with
    those of wl1 (arms at t + dt).  The two workloads differ only in their
    arms.  Returns as euler_step."""
    U = _solve_multiblob(wl0, q, theta, F)
    return advance(wl1, q, theta, U, dt, delta, corr_tol, corr_max_iter)


def midpoint_step_arms(wl0, wlh, wl1, q, theta, dt, delta, corr_tol=1e-10, corr_max_iter=50,
                       F=None):
    """Explicit midpoint (App. C) for links whose arms change in time: U^k with
    the arms at t (wl0); the half step's rebuild, check and correction and
    U^(k+1/2) with the arms at t + dt/2 (wlh); the full step from (q, theta)
    with the arms at t + dt (wl1).  Returns as midpoint_step."""
    U0 = _solve_multiblob(wl0, q, theta, F)
    qh, thh, ih = advance(wlh, q, theta, U0, 0.5 * dt, delta, corr_tol, corr_max_iter)
    Uh = _solve_multiblob(wlh, qh, thh, F)
    qn, thn, info = advance(wl1, q, theta, Uh, dt, delta, corr_tol, corr_max_iter)
    info.update(half=ih, U0=np.asarray(U0).reshape(-1, 6), U_half=np.asarray(Uh).reshape(-1, 6))
    return qn, thn, info


def _solve_multiblob(wl, q, theta, F):
    return solve_velocities(wl, q, theta, F)[0]

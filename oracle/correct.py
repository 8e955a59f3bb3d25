"""Position/orientation correction (Sec. 4.2, Eq. min_probl, Eq. residual, App. B).

Unknowns per body: increments dq_p (3) and quaternion dtheta_p (4), starting
at dq = 0, dtheta = [1, 0, 0, 0].  Residuals: the link constraints

    g_n = q_p + dq_p + R(dtheta_p . theta_p) dl_np - q_q - dq_q - R(dtheta_q . theta_q) dl_nq

(Eq. residual; 3 rows per link whatever rows the velocity form keeps), and
one row ||dtheta_p||^2 - 1 per body for the unit-norm condition.  Reading:
the paper solves the equality-constrained problem with SciPy's least squares,
which takes no equality constraints, so the unit-norm condition enters as a
weight-1 residual.

Jacobian (App. B): with R(dtheta . theta) = R(dtheta) R(theta) and
l~ = R(theta) dl, g = q + dq + R(dtheta) l~ and, from Eq. rot_mat,
R(dtheta) l~ = 2 [p (p . l~) + s p x l~ + (s^2 - 1/2) l~], so

    dg/d dq = I,   dg/ds = 2 p x l~ + 4 s l~,
    dg_i/dp_l = 2 [delta_il (p . l~) + p_i l~_l + s eps_ilk l~_k].

The residual is evaluated as written in App. B, R(dtheta) l~: it equals
R(dtheta . theta) dl on the unit sphere ||dtheta|| = 1, and its Jacobian
below is exact also off it (the iterates are not unit quaternions).

Reading: the printed indicial form of App. B drops these factors of 2 and
swaps two Levi-Civita indices relative to Eq. rot_mat; Eq. rot_mat is taken
as authoritative (the finite-difference test checks this Jacobian).

Iteration (per articulated body): Levenberg-Marquardt with mu = ||F||^2 (Yamashita-Fukushima),
step delta = -J^T (J J^T + mu I)^-1 F, accepted when ||F|| decreases, else mu
is multiplied by 10 and the step retried (at most 20 times); stop when
||F||_2 <= tol or after max_iter accepted steps.  Bodies of one assembly are
coupled only to each other, so the problem is solved as one system.
"""
from __future__ import annotations

import numpy as np

from .quat import quat_mul, rotation_matrix


def residual(wl, q, theta, x):
    """F(x) for x = [dq (3M), dtheta (4M)] stacked per body as (M,7)."""
    M = len(q)
    X = x.reshape(M, 7)
    dq, dth = X[:, :3], X[:, 3:]
    Rd = rotation_matrix(dth)
    Rt = rotation_matrix(theta)
    g = []
    for n in range(len(wl.pq)):
        p, qq = int(wl.pq[n, 0]), int(wl.pq[n, 1])
        v = q[p] + dq[p] + Rd[p] @ (Rt[p] @ wl.dl_p[n])
        if qq >= 0:
            v = v - q[qq] - dq[qq] - Rd[qq] @ (Rt[qq] @ wl.dl_q[n])
        else:
            v = v - wl.dl_q[n]
        g.append(v)
    g = np.concatenate(g) if g else np.zeros(0)
    unit = np.sum(dth * dth, axis=1) - 1.0
    return np.concatenate([g, unit])


def jacobian(wl, q, theta, x):
    """Exact Jacobian of ``residual`` ((3P + M) x 7M)."""
    M = len(q)
    X = x.reshape(M, 7)
    dth = X[:, 3:]
    Rth = rotation_matrix(theta)
    P = len(wl.pq)
    J = np.zeros((3 * P + M, 7 * M))

    def block(s, p, lt):
        Jb = np.zeros((3, 7))
        Jb[:, :3] = np.eye(3)
        Jb[:, 3] = 2 * np.cross(p, lt) + 4 * s * lt
        for i in range(3):
            for l in range(3):
                v = 2 * ((i == l) * (p @ lt) + p[i] * lt[l])
                # s eps_ilk lt_k
                for k in range(3):
                    eps = np.linalg.det(np.eye(3)[[i, l, k]]) if len({i, l, k}) == 3 else 0.0
                    v += 2 * s * eps * lt[k]
                Jb[i, 4 + l] = v
        return Jb

    for n in range(P):
        p, qq = int(wl.pq[n, 0]), int(wl.pq[n, 1])
        lt = Rth[p] @ wl.dl_p[n]
        J[3 * n:3 * n + 3, 7 * p:7 * p + 7] += block(dth[p, 0], dth[p, 1:], lt)
        if qq >= 0:
            lt = Rth[qq] @ wl.dl_q[n]
            J[3 * n:3 * n + 3, 7 * qq:7 * qq + 7] -= block(dth[qq, 0], dth[qq, 1:], lt)
    for p in range(M):
        J[3 * P + p, 7 * p + 3:7 * p + 7] = 2 * dth[p]
    return J


def link_assemblies(wl):
    """Bodies joined by links (position constraints), as lists of body indices,
    each with the indices of its links.  Bodies without links are left out."""
    M = len(wl.q)
    parent = list(range(M))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    for p, qq in wl.pq:
        if qq >= 0:
            a, b = find(int(p)), find(int(qq))
            if a != b:
                parent[max(a, b)] = min(a, b)
    groups = {}
    for n, (p, qq) in enumerate(wl.pq):
        r = find(int(p))
        groups.setdefault(r, [set(), []])
        groups[r][0].add(int(p))
        if qq >= 0:
            groups[r][0].add(int(qq))
        groups[r][1].append(n)
    return [(np.array(sorted(b)), np.array(l)) for _, (b, l) in sorted(groups.items())]


class _Sub:
    """Links of one assembly with body indices renumbered locally."""

    def __init__(self, wl, bodies, links):
        loc = {int(b): k for k, b in enumerate(bodies)}
        self.pq = np.array([[loc[int(wl.pq[n, 0])], loc.get(int(wl.pq[n, 1]), -1)]
                            for n in links], dtype=int).reshape(-1, 2)
        self.dl_p = wl.dl_p[links]
        self.dl_q = wl.dl_q[links]


def _lm(sub, q, theta, tol, max_iter):
    M = len(q)
    x = np.zeros(7 * M)
    x.reshape(M, 7)[:, 3] = 1.0
    F = residual(sub, q, theta, x)
    f = np.linalg.norm(F)
    hist = [f]
    it = 0
    while f > tol and it < max_iter:
        J = jacobian(sub, q, theta, x)
        mu = f * f
        for _ in range(20):
            S = J @ J.T + mu * np.eye(len(F))
            w = np.linalg.solve(S, F)
            xn = x - J.T @ w
            Fn = residual(sub, q, theta, xn)
            fn = np.linalg.norm(Fn)
            if fn < f:
                break
            mu *= 10.0
        else:
            break
        x, F, f = xn, Fn, fn
        hist.append(f)
        it += 1
    return x, it, hist


def correct(wl, q, theta, tol=1e-10, max_iter=50):
    """Return (q_new, theta_new, info): q + dq and dtheta . theta (Sec. 4.3, step 5).

    Each articulated body (bodies joined by links) is corrected separately, as
    the paper counts nonlinear iterations per articulated body (Sec. 4.4)."""
    q = np.array(q, float)
    theta = np.array(theta, float)
    qn, tn = q.copy(), theta.copy()
    iters, hists = [], []
    for bodies_a, links_a in link_assemblies(wl):
        sub = _Sub(wl, bodies_a, links_a)
        x, it, hist = _lm(sub, q[bodies_a], theta[bodies_a], tol, max_iter)
        X = x.reshape(len(bodies_a), 7)
        dth = X[:, 3:] / np.linalg.norm(X[:, 3:], axis=1)[:, None]
        qn[bodies_a] = q[bodies_a] + X[:, :3]
        tn[bodies_a] = quat_mul(dth, theta[bodies_a])
        iters.append(it)
        hists.append(hist)
    return qn, tn, dict(iterations=max(iters) if iters else 0, per_assembly=iters,
                        history=hists[0] if len(hists) == 1 else hists,
                        residual=max((h[-1] for h in hists), default=0.0))


def euler_update(q, theta, U, dt):
    """Explicit Euler update of every body (Sec. 4.3 step 3 without reconstruction):
    q <- q + dt u,  theta <- theta_{w dt} . theta."""
    from .quat import quat_from_rotvec
    U = np.asarray(U).reshape(-1, 6)
    return q + dt * U[:, :3], quat_mul(quat_from_rotvec(dt * U[:, 3:]), theta)

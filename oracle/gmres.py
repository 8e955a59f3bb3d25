"""Restarted GMRES for the saddle system (Sec. 3.1), float64.

The paper uses preconditioned GMRES with tolerance epsilon and warm starts
(Sec. 3.2.1) but does not fix the variant.  Readings taken here:
  * right preconditioning, A P^-1 z = b, y = P^-1 z, so the Krylov residual
    is the true residual ||b - A y||; left preconditioning (the paper's word)
    measures a preconditioned residual that can hide the true one, which the
    paper itself observes for rank-deficient constraints (Sec. 4.4);
  * Arnoldi with classical Gram-Schmidt applied twice (CGS2);
  * Givens rotations on the Hessenberg matrix, restart length m (default 100),
    initial guess y0 (default 0);
  * stop when the Givens residual estimate is <= tol ||b||; the iterate is then
    formed and the true residual recomputed; if it is still above tol ||b||
    the method restarts from that iterate.

Left preconditioning (the paper's own word, Sec. 3.1) is the option
``left=True``: the Krylov space is that of P^-1 A started from
z0 = P^-1 r0, and the Givens recursion then estimates the preconditioned
residual ||P^-1 (b - A y)||.  A cycle stops when that estimate has fallen by
the factor the true residual still has to fall, tol ||b|| / ||r0||; the
iterate y + V s is formed (no preconditioner at the end) and the stopping
test is always taken on the true residual ||b - A y|| <= tol ||b||,
restarting from y otherwise.
"""
from __future__ import annotations

import numpy as np


def gmres(A_apply, P_apply, b, tol=1e-10, restart=100, max_iter=1000, y0=None, record=None,
          left=False):
    """Return (y, info) with info = dict(iterations, restarts, history, true_rel, converged).

    ``record`` (a dict) receives the Arnoldi basis V and the unrotated
    Hessenberg matrix of the first cycle, for checking the Arnoldi relation.
    ``left``: left preconditioning (module docstring); history then holds the
    true relative residual at each cycle start and the preconditioned
    estimates scaled to it inside a cycle."""
    b = np.asarray(b, float)
    n = len(b)
    bnorm = np.linalg.norm(b)
    y = np.zeros(n) if y0 is None else np.array(y0, float)
    hist = []
    total = 0
    restarts = 0
    if bnorm == 0:
        return np.zeros(n), dict(iterations=0, restarts=0, history=[0.0], true_rel=0.0,
                                 converged=True)
    r = b - A_apply(y) if y0 is not None else b.copy()
    while True:
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta <= tol * bnorm or total >= max_iter:
            break
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        if left:
            # Krylov space of P^-1 A from P^-1 r; the cycle's target is the
            # preconditioned residual cut by the factor the true one needs
            z = P_apply(r)
            rnorm = beta
            beta = np.linalg.norm(z)
            target = tol * bnorm / rnorm * beta
            scale = rnorm / beta
            V[0] = z / beta
        else:
            target = tol * bnorm
            scale = 1.0
            V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            w = P_apply(A_apply(V[j])) if left else A_apply(P_apply(V[j]))
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            col = np.zeros(j + 2)
            col[:j + 1] = h
            col[j + 1] = hn
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            rho = np.hypot(col[j], col[j + 1])
            cs[j] = col[j] / rho
            sn[j] = col[j + 1] / rho
            col[j] = rho
            col[j + 1] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            H[:j + 2, j] = col
            if record is not None and restarts == 0:
                record.setdefault("Hraw", np.zeros((m + 1, m)))[:j + 2, j] = np.r_[h, hn]
                record["V"] = V
                record["k"] = j + 1
                record["w_last"] = w / hn if hn > 0 else w
            total += 1
            k = j + 1
            est = abs(g[j + 1])
            hist.append(est * scale / bnorm)
            if est <= target or total >= max_iter or hn == 0.0:
                break
            V[j + 1] = w / hn
        s = np.zeros(k)
        for i in range(k - 1, -1, -1):
            s[i] = (g[i] - H[i, i + 1:k] @ s[i + 1:k]) / H[i, i]
        y = y + (V[:k].T @ s if left else P_apply(V[:k].T @ s))
        r = b - A_apply(y)
        restarts += 1
        hist.pop()          # the estimate is replaced by the true residual below
    true_rel = np.linalg.norm(r) / bnorm
    return y, dict(iterations=total, restarts=restarts, history=hist, true_rel=true_rel,
                   converged=true_rel <= tol)

"""Articulated bodies made of single blobs (Sec. 2.4), float64.

TEST INFRASTRUCTURE ONLY (see the package header).

Every body is one blob at its tracking point; its 6 x 6 mobility blocks are the
generalised RPY tensor of oracle.rpy_rot.  The constrained problem is Eq.
linear_system_general with the unknowns taken in the order y = [U; phi]:

    [ I   -N C^T ] [ U  ]   [ N F ]
    [ C    0     ] [phi ] = [  B  ]

(the paper writes the same rows with the unknowns in the order [phi; U]).
Its formal solution is Eq. U: U = U^ + N C^T phi, U^ = N F,
phi = G (B - C U^), G = (C N C^T)^-1 (pseudo-inverse when C is rank deficient).

Block-diagonal preconditioner (Sec. 3.1, Eq. precond and Eq.
block_diag_const_res, with N~ the single-body blocks): N~_p = diag(I/(6 pi eta
a), I/(8 pi eta a^3)) and G~_a = (C_a N~_a C_a^T)^-1 per articulated body; the
preconditioner solves [I, -N~ C^T; C, 0] z = r, i.e.
phi = G~ (r_phi - C r_U), U = r_U + N~ C^T phi.
"""
from __future__ import annotations

import numpy as np

from . import bodies, rpy_rot, system
from .precond import _chol_or_pinv


def assemble(wl, q=None, theta=None, F=None):
    """Dict with N (6M x 6M), C, B, A, b for single-blob workload wl."""
    q = wl.q if q is None else np.asarray(q, float)
    theta = wl.theta if theta is None else np.asarray(theta, float)
    F = wl.F if F is None else np.asarray(F, float)
    M = len(q)
    Nm = rpy_rot.body_mobility(q, wl.a, wl.eta)
    C, B = bodies.constraint_rows(wl, q, theta)
    nc = C.shape[0]
    A = np.zeros((6 * M + nc, 6 * M + nc))
    A[:6 * M, :6 * M] = np.eye(6 * M)
    A[:6 * M, 6 * M:] = -Nm @ C.T
    A[6 * M:, :6 * M] = C
    b = np.concatenate([Nm @ np.ravel(F), B])
    return dict(N=Nm, C=C, B=B, A=A, b=b)


def solve_dense(S):
    """Minimum-norm least-squares solution y = [U; phi]."""
    return system.solve_dense(S["A"], S["b"])


def solve_formal(S, F):
    """Eq. U: (U, phi)."""
    Nm, C, B = S["N"], S["C"], S["B"]
    Uhat = Nm @ np.ravel(F)
    G = system.pinv_sym(C @ Nm @ C.T) if C.shape[0] else np.zeros((0, 0))
    phi = G @ (B - C @ Uhat)
    return Uhat + Nm @ (C.T @ phi), phi


class Preconditioner:
    """Sec. 3.1 for single-blob bodies (module header)."""

    def __init__(self, wl, C):
        M = wl.M
        self.M = M
        self.C = np.asarray(C)
        mt, mr = 1.0 / (6 * np.pi * wl.eta * wl.a), 1.0 / (8 * np.pi * wl.eta * wl.a ** 3)
        self.Nt = np.diag(np.tile([mt] * 3 + [mr] * 3, M))
        _, _, rows = bodies.assemblies(wl)
        self.rows = [r for r in rows if len(r)]
        self.G = []
        self.pinv_used = 0
        for r in self.rows:
            Ca = self.C[r]
            Ga, used = _chol_or_pinv(Ca @ self.Nt @ Ca.T)
            self.G.append(Ga)
            self.pinv_used += int(used)

    def apply(self, res):
        M = self.M
        rU, rphi = res[:6 * M], res[6 * M:]
        phi = np.zeros_like(rphi)
        y = rphi - self.C @ rU
        for r, Ga in zip(self.rows, self.G):
            phi[r] = Ga @ y[r]
        U = rU + self.Nt @ (self.C.T @ phi)
        return np.concatenate([U, phi])

"""Block-diagonal preconditioner of Sec. 3.1 (Eq. precond, Eq. block_diag_const_res).

The preconditioner solves the approximate saddle problem in which M is
replaced by its body-diagonal part M~ (M~^(pq) = delta_pq M^(pp)):

    M~ lam - K U = r_lam,   -K^T lam + C^T phi = r_U,   C U = r_phi.

Eliminating row by row (row 1 gives lam = M~^-1 (r_lam + K U); row 2 then
gives N~^-1 U = -r_U - K^T M~^-1 r_lam + C^T phi; row 3 gives
(C N~ C^T) phi = r_phi - C U-hat) yields, per body p and assembly a:

    t_p   = M_pp^-1 r_lam,p                      (Cholesky of M_pp)
    Z_p   = M_pp^-1 K_p,  N~_p = (K_p^T Z_p)^+    (Sec. 3.1)
    U-hat_p = -N~_p (r_U,p + Z_p^T r_lam,p)
    phi_a = G~_a (r_phi,a - C_a U-hat_a),  G~_a = (C_a N~_a C_a^T)^-1, or the
            pseudo-inverse when C_a lacks full row rank (Sec. 3.1)
    U_p   = U-hat_p + N~_p (C^T phi)_p
    lam_p = t_p + Z_p U_p

Readings: N~_p uses the symmetric pseudo-inverse with eigenvalue cutoff
1e-12 * max (the paper gives no cutoff); for bodies with a resistance-free
motion (collinear blobs spinning about their axis) this returns the
minimum-norm velocity.  G~_a is a Cholesky inverse unless a pivot falls
below 1e-12 * max diagonal, in which case the symmetric pseudo-inverse is used.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import bodies, rpy
from .system import pinv_sym


def _chol_or_pinv(S, rel=1e-12):
    """(inverse, used_pinv) of a symmetric PSD matrix."""
    n = S.shape[0]
    if n == 0:
        return S.copy(), False
    L = np.zeros_like(S)
    dmax = np.max(np.abs(np.diag(S)))
    ok = True
    for j in range(n):
        v = S[j, j] - L[j, :j] @ L[j, :j]
        if v <= rel * dmax:
            ok = False
            break
        L[j, j] = np.sqrt(v)
        L[j + 1:, j] = (S[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    if ok:
        Linv = np.linalg.inv(L)
        return Linv.T @ Linv, False
    return pinv_sym(S), True


class BlockPreconditioner:
    def __init__(self, wl, r, C, q=None):
        q = wl.q if q is None else q
        self.N, self.M = wl.N, wl.M
        off = wl.blob_offset
        self.off = off
        self.L, self.Z, self.Nt = [], [], []
        for p in range(self.M):
            rp = r[off[p]:off[p + 1]]
            Mpp = rpy.mobility_matrix(rp, wl.a, wl.eta, wl.wall)
            Kp = bodies.K_matrix(rp, q[p:p + 1], np.array([0, len(rp)]))
            Lp = np.linalg.cholesky(Mpp)
            Zp = np.linalg.solve(Mpp, Kp)
            Rp = Kp.T @ Zp
            self.L.append(Lp)
            self.Z.append(Zp)
            self.Nt.append(pinv_sym(Rp))
        self.C = C
        _, self.asm_bodies, self.asm_rows = bodies.assemblies(wl)
        self.G, self.pinv_used = [], False
        for bs, rs in zip(self.asm_bodies, self.asm_rows):
            cols = np.concatenate([np.arange(6 * p, 6 * p + 6) for p in bs])
            Ca = C[np.ix_(rs, cols)]
            Na = np.zeros((len(cols), len(cols)))
            for k, p in enumerate(bs):
                Na[6 * k:6 * k + 6, 6 * k:6 * k + 6] = self.Nt[p]
            Ga, used = _chol_or_pinv(Ca @ Na @ Ca.T)
            self.pinv_used |= used
            self.G.append(Ga)

    def apply(self, rvec):
        N, M = self.N, self.M
        r_lam = rvec[:3 * N]
        r_U = rvec[3 * N:3 * N + 6 * M]
        r_phi = rvec[3 * N + 6 * M:]
        t = np.zeros(3 * N)
        Uhat = np.zeros(6 * M)
        for p in range(M):
            sl = slice(3 * self.off[p], 3 * self.off[p + 1])
            Lp = self.L[p]
            t[sl] = np.linalg.solve(Lp.T, np.linalg.solve(Lp, r_lam[sl]))
            Uhat[6 * p:6 * p + 6] = -self.Nt[p] @ (r_U[6 * p:6 * p + 6] + self.Z[p].T @ r_lam[sl])
        phi = np.zeros(len(r_phi))
        for bs, rs, Ga in zip(self.asm_bodies, self.asm_rows, self.G):
            if len(rs) == 0:
                continue
            cols = np.concatenate([np.arange(6 * p, 6 * p + 6) for p in bs])
            Ca = self.C[np.ix_(rs, cols)]
            phi[rs] = Ga @ (r_phi[rs] - Ca @ Uhat[cols])
        CTphi = self.C.T @ phi if len(phi) else np.zeros(6 * M)
        U = np.zeros(6 * M)
        lam = np.zeros(3 * N)
        for p in range(M):
            U[6 * p:6 * p + 6] = Uhat[6 * p:6 * p + 6] + self.Nt[p] @ CTphi[6 * p:6 * p + 6]
            sl = slice(3 * self.off[p], 3 * self.off[p + 1])
            lam[sl] = t[sl] + self.Z[p] @ U[6 * p:6 * p + 6]
        return np.concatenate([lam, U, phi])


class CorrectedBodyPreconditioner(BlockPreconditioner):
    """The same block solve with given body mobilities N~_w (learned extension of
    Sec. 3.1: a network predicts N~_p of each body above the wall).

    The blob blocks are the unbounded M_f = M^(pp) (no wall), modified so that
    the block solve is exact for a consistent pair (M~, N~_w):

        M~^-1 = M_f^-1 + Z_f D Z_f^T,   Z_f = M_f^-1 K_p,
        N~_f = (K_p^T Z_f)^-1,          D = N~_f N~_w^-1 N~_f - N~_f,

    so that K_p^T M~^-1 K_p = N~_f^-1 + N~_f^-1 D N~_f^-1 = N~_w^-1.  Written
    out plainly: M~ is formed densely per body and the exact block solve of
    the base class runs on it with N~_p = N~_w.
    """

    def __init__(self, wl, r, C, Nw, q=None):
        q = wl.q if q is None else q
        free = dataclasses.replace(wl, wall=False)
        super().__init__(free, r, C, q)
        off = self.off
        for p in range(self.M):
            rp = r[off[p]:off[p + 1]]
            Kp = bodies.K_matrix(rp, q[p:p + 1], np.array([0, len(rp)]))
            Mf = self.L[p] @ self.L[p].T
            Zf = np.linalg.solve(Mf, Kp)
            Nf = np.linalg.inv(Kp.T @ Zf)
            D = Nf @ np.linalg.inv(Nw[p]) @ Nf - Nf
            Minv = np.linalg.inv(Mf) + Zf @ D @ Zf.T
            Mmod = np.linalg.inv(0.5 * (Minv + Minv.T))
            self.L[p] = np.linalg.cholesky(0.5 * (Mmod + Mmod.T))
            self.Z[p] = np.linalg.solve(Mmod, Kp)
            self.Nt[p] = np.asarray(Nw[p], float)
        self.G, self.pinv_used = [], False
        for bs, rs in zip(self.asm_bodies, self.asm_rows):
            cols = np.concatenate([np.arange(6 * p, 6 * p + 6) for p in bs])
            Ca = C[np.ix_(rs, cols)]
            Na = np.zeros((len(cols), len(cols)))
            for k, p in enumerate(bs):
                Na[6 * k:6 * k + 6, 6 * k:6 * k + 6] = self.Nt[p]
            Ga, used = _chol_or_pinv(Ca @ Na @ Ca.T)
            self.pinv_used |= used
            self.G.append(Ga)

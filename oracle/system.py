"""The constrained mobility saddle system (Sec. 2.3, Eq. linear_system), float64.

    A = [[ M, -K,  0 ],        y = [lambda; U; phi],   b = [u_s; -F; B]
         [-K^T, 0, C^T],
         [ 0,   C,  0 ]]

Two independent direct routes are provided for small problems: a dense
least-squares solve of A y = b (minimum-norm when A is singular), and the
formal solution of Sec. 2.2-2.3 (Eq. U and the slip-corrected U-hat).
"""
from __future__ import annotations

import numpy as np

from . import bodies, rpy


def assemble(wl, q=None, theta=None):
    """Return dict with r, Mmat, K, C, B, A, b for workload wl."""
    q = wl.q if q is None else q
    theta = wl.theta if theta is None else theta
    r = bodies.blob_positions(q, theta, wl.r_ref, wl.blob_offset)
    Mmat = rpy.mobility_matrix(r, wl.a, wl.eta, wl.wall)
    K = bodies.K_matrix(r, q, wl.blob_offset)
    C, B = bodies.constraint_rows(wl, q, theta)
    A = saddle_matrix(Mmat, K, C)
    us = np.zeros(3 * len(r)) if wl.u_slip is None else np.asarray(wl.u_slip).ravel()
    b = np.concatenate([us, -np.asarray(wl.F).ravel(), B])
    return dict(r=r, Mmat=Mmat, K=K, C=C, B=B, A=A, b=b, u_s=us)


def saddle_matrix(Mmat, K, C):
    n3, m6 = K.shape
    nc = C.shape[0]
    n = n3 + m6 + nc
    A = np.zeros((n, n))
    A[:n3, :n3] = Mmat
    A[:n3, n3:n3 + m6] = -K
    A[n3:n3 + m6, :n3] = -K.T
    A[n3:n3 + m6, n3 + m6:] = C.T
    A[n3 + m6:, n3:n3 + m6] = C
    return A


def split(y, N, M):
    return y[:3 * N], y[3 * N:3 * N + 6 * M], y[3 * N + 6 * M:]


def solve_dense(A, b):
    """Minimum-norm least-squares solution of A y = b (LAPACK gelsd)."""
    y, *_ = np.linalg.lstsq(A, b, rcond=1e-13)
    return y


def pinv_sym(S, cutoff=1e-12):
    """Symmetric pseudo-inverse: eigenvalues below cutoff * max eigenvalue -> 0."""
    w, V = np.linalg.eigh(0.5 * (S + S.T))
    lim = cutoff * np.max(np.abs(w))
    winv = np.where(np.abs(w) > lim, 1.0 / np.where(np.abs(w) > lim, w, 1.0), 0.0)
    return (V * winv) @ V.T


def solve_formal(Mmat, K, C, u_s, F, B):
    """Formal solution (Sec. 2.2 Eq. U with the slip term of Sec. 2.3):
    N = (K^T M^-1 K)^+, U-hat = N F - N K^T M^-1 u_s, G = (C N C^T)^+,
    phi = G (B - C U-hat), U = U-hat + N C^T phi, lambda = M^-1 (u_s + K U)."""
    Minv_K = np.linalg.solve(Mmat, K)
    Minv_us = np.linalg.solve(Mmat, u_s)
    Nmob = pinv_sym(K.T @ Minv_K)
    Uhat = Nmob @ F - Nmob @ (K.T @ Minv_us)
    G = pinv_sym(C @ Nmob @ C.T) if C.shape[0] else np.zeros((0, 0))
    phi = G @ (B - C @ Uhat)
    U = Uhat + Nmob @ (C.T @ phi)
    lam = Minv_us + Minv_K @ U
    return lam, U, phi, dict(N=Nmob, G=G, Uhat=Uhat)

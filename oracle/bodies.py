"""Rigid multiblob kinematics and constraints (Sec. 2.1-2.3, App. A), float64.

Conventions
  * U_p = (u_p, w_p), F_p = (f_p, tau_p) with torque about the tracking point q_p.
  * lambda and blob velocities are xyz-interleaved per blob.
  * Link n joins body p (the + end) and body q (the - end, or -1 for a fixed
    lab point); its arms dl_p, dl_q are in the body frames (Eq. constraint).
  * A link may keep only some rows of its velocity constraint: rows
    d_m = R(theta_p) pi_m with pi_m given in the body frame of p.  (Sec. 2.2
    allows constraints on single components.)  A ball joint keeps e_x, e_y, e_z.
  * General rows carry body-p-frame coefficients (c_u_p, c_w_p, c_u_q, c_w_q)
    and a right-hand side.
  * phi / constraint rows: link rows in link order, then general rows.
"""
from __future__ import annotations

import numpy as np

from .quat import cross_matrix, rotation_matrix


def blob_positions(q, theta, r_ref, blob_offset):
    """r_i = q_p + R(theta_p) r_i^ref for every blob i of body p (Sec. 2.3)."""
    R = rotation_matrix(theta)
    body = body_of_blob(blob_offset)
    return q[body] + np.einsum("nij,nj->ni", R[body], r_ref)


def body_of_blob(blob_offset):
    off = np.asarray(blob_offset)
    return np.repeat(np.arange(len(off) - 1), np.diff(off))


def K_matrix(r, q, blob_offset):
    """Dense K (3N x 6M): (K U)_i = u_p + w_p x (r_i - q_p)  (Eq. no-slip)."""
    body = body_of_blob(blob_offset)
    N, M = len(r), len(q)
    K = np.zeros((3 * N, 6 * M))
    for i in range(N):
        p = body[i]
        K[3 * i:3 * i + 3, 6 * p:6 * p + 3] = np.eye(3)
        # w x d = -d x w
        K[3 * i:3 * i + 3, 6 * p + 3:6 * p + 6] = -cross_matrix(r[i] - q[p])
    return K


def K_apply(r, q, blob_offset, U):
    """(K U)_i = u_p + w_p x (r_i - q_p) for every blob i of body p (Eq. no-slip), (N, 3)."""
    body = body_of_blob(blob_offset)
    U = np.asarray(U, float).reshape(-1, 6)
    return U[body, :3] + np.cross(U[body, 3:], np.asarray(r) - np.asarray(q)[body])


def KT_apply(r, q, blob_offset, lam):
    """(K^T lambda)_p = (sum_i lambda_i, sum_i (r_i - q_p) x lambda_i) over the blobs of
    body p (Eq. balance), (M, 6)."""
    body = body_of_blob(blob_offset)
    lam = np.asarray(lam, float).reshape(-1, 3)
    M = len(q)
    out = np.zeros((M, 6))
    np.add.at(out[:, :3], body, lam)
    np.add.at(out[:, 3:], body, np.cross(np.asarray(r) - np.asarray(q)[body], lam))
    return out


def constraint_rows(wl, q=None, theta=None, sparse=False):
    """C (Nc x 6M) and B (Nc) of the velocity constraints C U = B; C dense, or a
    scipy CSR matrix with sparse=True.

    Link n (Eq. dg): u_p + w_p x l_p - u_q - w_q x l_q = B_n with lab arms
    l = R(theta) dl and B_n = R_q dldot_q - R_p dldot_p.  Row m keeps
    d_m . (.) with d_m = R_p pi_m; since d.(w x l) = w.(l x d) the row's
    coefficients are (d, l_p x d) on body p and (-d, -(l_q x d)) on body q,
    i.e. the link block [I, -l_p^x, -I, l_q^x] of App. A for a ball joint.
    """
    q = wl.q if q is None else q
    theta = wl.theta if theta is None else theta
    R = rotation_matrix(theta)
    M = len(q)
    nc = int(wl.nproj.sum()) + len(wl.row_rhs)
    rows, cols, vals = [], [], []

    def put(k, col0, v):  # C[k, col0:col0 + 3] += v
        rows.extend((k, k, k))
        cols.extend((col0, col0 + 1, col0 + 2))
        vals.extend(v)

    B = np.zeros(nc)
    k = 0
    for n in range(len(wl.pq)):
        p, qq = int(wl.pq[n, 0]), int(wl.pq[n, 1])
        lp = R[p] @ wl.dl_p[n]
        Bn = -R[p] @ wl.dldot_p[n]
        if qq >= 0:
            lq = R[qq] @ wl.dl_q[n]
            Bn = Bn + R[qq] @ wl.dldot_q[n]
        else:
            Bn = Bn + wl.dldot_q[n]
        for m in range(int(wl.nproj[n])):
            d = R[p] @ wl.proj[n, m]
            put(k, 6 * p, d)
            put(k, 6 * p + 3, np.cross(lp, d))
            if qq >= 0:
                put(k, 6 * qq, -d)
                put(k, 6 * qq + 3, -np.cross(lq, d))
            B[k] = d @ Bn
            k += 1
    for j in range(len(wl.row_rhs)):
        p, qq = int(wl.row_pq[j, 0]), int(wl.row_pq[j, 1])
        c = wl.row_coef[j].reshape(4, 3)
        put(k, 6 * p, R[p] @ c[0])
        put(k, 6 * p + 3, R[p] @ c[1])
        if qq >= 0:
            put(k, 6 * qq, R[p] @ c[2])
            put(k, 6 * qq + 3, R[p] @ c[3])
        B[k] = wl.row_rhs[j]
        k += 1
    if sparse:
        from scipy.sparse import coo_matrix
        return coo_matrix((vals, (rows, cols)), shape=(nc, 6 * M)).tocsr(), B
    C = np.zeros((nc, 6 * M))
    np.add.at(C, (np.asarray(rows, int), np.asarray(cols, int)), np.asarray(vals, float))
    return C, B


def link_residual(wl, q, theta):
    """g_n = q_p + R_p dl_p - q_q - R_q dl_q for every link (Eq. constraint), (P,3).
    A link with q = -1 compares with the fixed lab point dl_q."""
    R = rotation_matrix(theta)
    g = np.zeros((len(wl.pq), 3))
    for n in range(len(wl.pq)):
        p, qq = int(wl.pq[n, 0]), int(wl.pq[n, 1])
        g[n] = q[p] + R[p] @ wl.dl_p[n]
        if qq >= 0:
            g[n] -= q[qq] + R[qq] @ wl.dl_q[n]
        else:
            g[n] -= wl.dl_q[n]
    return g


def assemblies(wl):
    """Connected components of bodies joined by links or general rows.
    Returns (assembly_of_body (M,), list of body index arrays, list of row index arrays)."""
    M = wl.M
    parent = list(range(M))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    pairs = [tuple(x) for x in wl.pq] + [tuple(x) for x in wl.row_pq]
    for p, qq in pairs:
        if qq >= 0:
            a, b = find(int(p)), find(int(qq))
            if a != b:
                parent[max(a, b)] = min(a, b)
    roots = [find(i) for i in range(M)]
    uniq = sorted(set(roots), key=lambda r: r)
    label = {r: k for k, r in enumerate(uniq)}
    asm = np.array([label[r] for r in roots])
    bodies = [np.where(asm == k)[0] for k in range(len(uniq))]
    row_body = []
    for n in range(len(wl.pq)):
        row_body += [int(wl.pq[n, 0])] * int(wl.nproj[n])
    row_body += [int(p) for p in wl.row_pq[:, 0]]
    row_body = np.array(row_body, int)
    rows = [np.where(asm[row_body] == k)[0] if len(row_body) else np.zeros(0, int)
            for k in range(len(uniq))]
    return asm, bodies, rows

"""Thin ctypes binding of libarb (include/arb.h): same names, argument marshalling only.

Host-pointer entry points take numpy arrays (converted to C-contiguous float64
/ int32); ``*_dev`` entry points take device pointers as ints or objects with
``data_ptr()`` (torch tensors) and an optional stream handle.  Negative status
codes raise ``ArbError``; warnings (positive codes) are returned.

There is no fallback: if libarb.so is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libarb.so")

ARB_OK = 0
ARB_W_NOT_CONVERGED = 1
ARB_W_PINV_USED = 2
ARB_W_LEARNED_FALLBACK = 3
ARB_E_ARG = -1
ARB_E_NOT_SPD = -2
ARB_E_BELOW_WALL = -3
ARB_E_DEVICE = -4
ARB_E_NAN = -5
ARB_E_HOST = -6
ARB_FP64 = 0
ARB_FP32C = 1
ARB_PC_NONE = 0
ARB_PC_BLOCK = 1
ARB_PC_LEARNED = 2
ARB_PC_BODYFRAME = 3
ARB_MODEL_MULTIBLOB = 0
ARB_MODEL_SINGLE_BLOB = 1
ARB_PAIR_AUTO = 0
ARB_PAIR_TARGET = 1
ARB_PAIR_SYMMETRIC = 2
ARB_PAIR_FMM = 3
ARB_NOALLOC_MAX_BLOBS = 65536

SYMBOLS = [
    "arb_create", "arb_destroy", "arb_last_error", "arb_get_slices", "arb_set_bodies",
    "arb_set_state", "arb_blob_positions", "arb_set_links", "arb_set_rows", "arb_sizes",
    "arb_mobility_apply", "arb_mobility_apply_dev", "arb_rpy_apply_dev", "arb_rpy_apply",
    "arb_system_apply", "arb_K_apply", "arb_KT_apply", "arb_constraint_rows",
    "arb_precond_build", "arb_precond_apply", "arb_precond_block", "arb_solve",
    "arb_solve_dev", "arb_euler_update", "arb_correct_positions", "arb_profile",
    "arb_profile_read", "arb_mlp_set_params", "arb_mlp_get_params", "arb_mlp_forward",
    "arb_mlp_grad", "arb_mlp_train_step_dev", "arb_mlp_features", "arb_body_mobility",
    "arb_mlp_set_scaling", "arb_reconstruct", "arb_link_residual", "arb_step_euler",
    "arb_body_mobility_apply", "arb_body_mobility_apply_dev", "arb_step_midpoint",
    "arb_fmm_get_stats", "arb_fmm_plan", "arb_rpy_apply_noalloc_dev", "arb_step_euler_arms",
    "arb_step_midpoint_arms",
]


class ArbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libarb error {code}: {msg}")
        self.code = code


class arb_options(C.Structure):
    _fields_ = [("device", C.c_int), ("precision", C.c_int), ("wall", C.c_int),
                ("eta", C.c_double), ("a", C.c_double), ("tol", C.c_double),
                ("restart", C.c_int), ("max_iter", C.c_int), ("precond", C.c_int),
                ("slices", C.c_int), ("pair_kernel", C.c_int), ("graphs", C.c_int),
                ("model", C.c_int), ("fmm_order", C.c_int), ("fmm_levels", C.c_int),
                ("fmm_leaf", C.c_int), ("left_precond", C.c_int),
                ("small_cycle", C.c_int), ("refine_final", C.c_int)]


class arb_fmm_stats(C.Structure):
    _fields_ = [("levels", C.c_int), ("order", C.c_int), ("cells", C.c_int),
                ("leaves", C.c_int), ("near_pairs", C.c_longlong),
                ("interactions", C.c_longlong), ("m2l_pairs", C.c_longlong),
                ("build_ms", C.c_double), ("plan_hash", C.c_ulonglong)]


class arb_step_info(C.Structure):
    _fields_ = [("solve_status", C.c_int), ("iterations", C.c_int), ("rel_residual", C.c_double),
                ("t_build_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("g_inf_star", C.c_double), ("g2_star", C.c_double), ("corrected", C.c_int),
                ("corr_iterations", C.c_int), ("corr_residual", C.c_double), ("g_inf", C.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class arb_arms(C.Structure):
    _fields_ = [("dl_p", C.POINTER(C.c_double)), ("dl_q", C.POINTER(C.c_double)),
                ("dldot_p", C.POINTER(C.c_double)), ("dldot_q", C.POINTER(C.c_double)),
                ("proj", C.POINTER(C.c_double))]


class arb_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("rel_residual", C.c_double),
                ("rel_residual_fp64", C.c_double), ("t_build_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("pinv_used", C.c_int), ("history_len", C.c_int),
                ("history", C.c_double * 1024), ("products_fp64", C.c_int),
                ("products_fp32", C.c_int), ("precond_applies", C.c_int),
                ("one_launch_cycles", C.c_int), ("residual_bounded", C.c_int)]

    def to_dict(self):
        return dict(iterations=self.iterations, restarts=self.restarts,
                    rel_residual=self.rel_residual, rel_residual_fp64=self.rel_residual_fp64,
                    t_build_ms=self.t_build_ms, t_solve_ms=self.t_solve_ms,
                    pinv_used=self.pinv_used,
                    history=list(self.history[:self.history_len]),
                    products_fp64=self.products_fp64, products_fp32=self.products_fp32,
                    precond_applies=self.precond_applies,
                    one_launch_cycles=self.one_launch_cycles,
                    residual_bounded=self.residual_bounded)


_lib = None
_P = C.c_void_p
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)
_FP = C.POINTER(C.c_float)
N_MLP_PARAMS = 20245


def load():
    """Load libarb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    sig = {
        "arb_create": (C.c_int, [C.POINTER(_P), C.POINTER(arb_options)]),
        "arb_destroy": (None, [_P]),
        "arb_last_error": (C.c_char_p, [_P]),
        "arb_get_slices": (C.c_int, [_P, C.c_int]),
        "arb_set_bodies": (C.c_int, [_P, C.c_int, _IP, _DP, _IP]),
        "arb_set_state": (C.c_int, [_P, _DP, _DP]),
        "arb_blob_positions": (C.c_int, [_P, _DP]),
        "arb_set_links": (C.c_int, [_P, C.c_int, _IP, _DP, _DP, _DP, _DP, _IP, _DP]),
        "arb_set_rows": (C.c_int, [_P, C.c_int, _IP, _DP, _DP]),
        "arb_sizes": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_int64)]),
        "arb_mobility_apply": (C.c_int, [_P, _DP, _DP]),
        "arb_mobility_apply_dev": (C.c_int, [_P, _P, _P, _P]),
        "arb_rpy_apply_dev": (C.c_int, [_P, C.c_int, _P, _P, _P, _P]),
        "arb_rpy_apply": (C.c_int, [_P, C.c_int, _DP, _DP, _DP]),
        "arb_rpy_apply_noalloc_dev": (C.c_int, [_P, C.c_int, _P, _P, _P, _P]),
        "arb_system_apply": (C.c_int, [_P, _DP, _DP]),
        "arb_K_apply": (C.c_int, [_P, _DP, _DP]),
        "arb_KT_apply": (C.c_int, [_P, _DP, _DP]),
        "arb_constraint_rows": (C.c_int, [_P, _DP, _IP, _DP]),
        "arb_precond_build": (C.c_int, [_P]),
        "arb_precond_apply": (C.c_int, [_P, _DP, _DP]),
        "arb_precond_block": (C.c_int, [_P, C.c_int, _DP, _DP]),
        "arb_solve": (C.c_int, [_P, _DP, _DP, _DP, _DP, _DP, _DP, C.POINTER(arb_solve_info)]),
        "arb_solve_dev": (C.c_int, [_P, _P, _P, _P, C.c_int, C.POINTER(arb_solve_info), _P]),
        "arb_euler_update": (C.c_int, [_P, _DP, C.c_double, _DP, _DP]),
        "arb_correct_positions": (C.c_int, [_P, C.c_double, C.c_int, _DP, _DP,
                                            C.POINTER(C.c_int), _DP]),
        "arb_profile": (C.c_int, [_P, C.c_int]),
        "arb_mlp_set_params": (C.c_int, [_P, C.c_int, _FP]),
        "arb_mlp_get_params": (C.c_int, [_P, C.c_int, _FP]),
        "arb_mlp_forward": (C.c_int, [_P, C.c_int, _FP, _FP]),
        "arb_mlp_grad": (C.c_int, [_P, C.c_int, _FP, _FP, _FP, _DP]),
        "arb_mlp_train_step_dev": (C.c_int, [_P, C.c_int, _P, _P, C.c_float, _DP, _P]),
        "arb_mlp_features": (C.c_int, [_P, _FP]),
        "arb_body_mobility": (C.c_int, [_P, _DP, _FP]),
        "arb_mlp_set_scaling": (C.c_int, [_P, _FP, _FP, _FP, _FP]),
        "arb_profile_read": (C.c_int, [_P, _DP, C.POINTER(C.c_int)]),
        "arb_reconstruct": (C.c_int, [_P, _DP, _DP, _DP]),
        "arb_step_midpoint": (C.c_int, [_P, _DP, _DP, C.c_double, C.c_double, C.c_double,
                                        C.c_int, C.c_int, _DP, _DP, _DP,
                                        C.POINTER(arb_step_info)]),
        "arb_body_mobility_apply": (C.c_int, [_P, _DP, _DP]),
        "arb_body_mobility_apply_dev": (C.c_int, [_P, _P, _P, _P]),
        "arb_link_residual": (C.c_int, [_P, _DP, _DP]),
        "arb_fmm_get_stats": (C.c_int, [_P, C.POINTER(arb_fmm_stats)]),
        "arb_fmm_plan": (C.c_int, [C.c_int, _DP, C.c_double, C.c_int, C.c_int, C.c_int,
                                   C.POINTER(arb_fmm_stats)]),
        "arb_step_euler": (C.c_int, [_P, _DP, _DP, C.c_double, C.c_double, C.c_double, C.c_int,
                                     C.c_int, _DP, _DP, _DP, C.POINTER(arb_step_info)]),
        "arb_step_euler_arms": (C.c_int, [_P, _DP, _DP, C.c_double, C.c_double, C.c_double,
                                          C.c_int, C.c_int, C.POINTER(arb_arms), _DP, _DP, _DP,
                                          C.POINTER(arb_step_info)]),
        "arb_step_midpoint_arms": (C.c_int, [_P, _DP, _DP, C.c_double, C.c_double, C.c_double,
                                             C.c_int, C.c_int, C.POINTER(arb_arms),
                                             C.POINTER(arb_arms), _DP, _DP, _DP,
                                             C.POINTER(arb_step_info)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _d(a, n=None):
    """float64 C-contiguous array -> (array, pointer); None -> (None, NULL)."""
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a, a.ctypes.data_as(_DP)


def _i(a, n=None):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.int32)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a, a.ctypes.data_as(_IP)


def _out(n):
    a = np.zeros(n, dtype=np.float64)
    return a, a.ctypes.data_as(_DP)


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return C.c_void_p(x.data_ptr())
    return C.c_void_p(int(x))


def _check(ctx, rc):
    if rc < 0:
        msg = load().arb_last_error(ctx)
        raise ArbError(rc, msg.decode() if msg else "")
    return rc


# ------------------------------------------------------------------ entry points
def arb_create(device=0, precision=ARB_FP64, wall=False, eta=1.0, a=1.0, tol=1e-10,
               restart=100, max_iter=1000, precond=ARB_PC_BLOCK, slices=0, pair_kernel=0,
               graphs=0, model=ARB_MODEL_MULTIBLOB, fmm_order=0, fmm_levels=0, fmm_leaf=0,
               left_precond=0, small_cycle=0, refine_final=0):
    opt = arb_options(device, precision, int(bool(wall)), eta, a, tol, restart, max_iter,
                      precond, slices, pair_kernel, graphs, model, fmm_order, fmm_levels,
                      fmm_leaf, int(left_precond), int(small_cycle), int(refine_final))
    h = _P()
    rc = load().arb_create(C.byref(h), C.byref(opt))
    if rc < 0:
        raise ArbError(rc, "arb_create failed (bad options or no device)")
    return h


def arb_destroy(ctx):
    load().arb_destroy(ctx)


def arb_last_error(ctx):
    m = load().arb_last_error(ctx)
    return m.decode() if m else ""


def arb_get_slices(ctx, n_blobs):
    return load().arb_get_slices(ctx, int(n_blobs))


def arb_set_bodies(ctx, blob_offset, r_ref, body_type=None):
    bo, bop = _i(blob_offset)
    M = bo.size - 1
    rr, rrp = _d(r_ref, 3 * int(bo[-1]))
    bt, btp = _i(body_type, M) if body_type is not None else (None, None)
    return _check(ctx, load().arb_set_bodies(ctx, M, bop, rrp, btp))


def arb_set_state(ctx, q, theta):
    q_, qp = _d(q)
    t_, tp = _d(theta)
    return _check(ctx, load().arb_set_state(ctx, qp, tp))


def arb_sizes(ctx):
    N, M, Nc, n = C.c_int(), C.c_int(), C.c_int(), C.c_int64()
    _check(ctx, load().arb_sizes(ctx, C.byref(N), C.byref(M), C.byref(Nc), C.byref(n)))
    return N.value, M.value, Nc.value, n.value


def arb_blob_positions(ctx):
    N = arb_sizes(ctx)[0]
    out, op = _out(3 * N)
    _check(ctx, load().arb_blob_positions(ctx, op))
    return out.reshape(N, 3)


def arb_set_links(ctx, pq, dl_p, dl_q, dldot_p=None, dldot_q=None, nproj=None, proj=None):
    pq_, pqp = _i(pq)
    P = pq_.size // 2
    a1, p1 = _d(dl_p, 3 * P)
    a2, p2 = _d(dl_q, 3 * P)
    a3, p3 = _d(dldot_p, 3 * P) if dldot_p is not None else (None, None)
    a4, p4 = _d(dldot_q, 3 * P) if dldot_q is not None else (None, None)
    a5, p5 = _i(nproj, P) if nproj is not None else (None, None)
    a6, p6 = _d(proj, 9 * P) if proj is not None else (None, None)
    return _check(ctx, load().arb_set_links(ctx, P, pqp, p1, p2, p3, p4, p5, p6))


def arb_set_rows(ctx, pq, coef, rhs):
    pq_, pqp = _i(pq)
    R = pq_.size // 2
    c_, cp = _d(coef, 12 * R)
    r_, rp = _d(rhs, R)
    return _check(ctx, load().arb_set_rows(ctx, R, pqp, cp, rp))


def arb_mobility_apply(ctx, lam):
    N = arb_sizes(ctx)[0]
    l_, lp = _d(lam, 3 * N)
    u, up = _out(3 * N)
    _check(ctx, load().arb_mobility_apply(ctx, lp, up))
    return u


def arb_body_mobility_apply(ctx, FT):
    """(u, w) per body (M,6) = N (f, tau) for single-blob bodies."""
    M = arb_sizes(ctx)[1]
    f_, fp = _d(FT, 6 * M)
    u, up = _out(6 * M)
    _check(ctx, load().arb_body_mobility_apply(ctx, fp, up))
    return u.reshape(M, 6)


def arb_body_mobility_apply_dev(ctx, FT_dev, UW_dev, stream=None):
    return _check(ctx, load().arb_body_mobility_apply_dev(ctx, _ptr(FT_dev), _ptr(UW_dev),
                                                          _ptr(stream)))


def arb_mobility_apply_dev(ctx, lam_dev, u_dev, stream=None):
    return _check(ctx, load().arb_mobility_apply_dev(ctx, _ptr(lam_dev), _ptr(u_dev),
                                                     _ptr(stream)))


def arb_rpy_apply(ctx, pos, lam):
    p_, pp = _d(pos)
    N = p_.size // 3
    l_, lp = _d(lam, 3 * N)
    u, up = _out(3 * N)
    _check(ctx, load().arb_rpy_apply(ctx, N, pp, lp, up))
    return u


def arb_rpy_apply_dev(ctx, N, pos_dev, lam_dev, u_dev, stream=None):
    return _check(ctx, load().arb_rpy_apply_dev(ctx, int(N), _ptr(pos_dev), _ptr(lam_dev),
                                                _ptr(u_dev), _ptr(stream)))


def arb_rpy_apply_noalloc_dev(ctx, N, pos_dev, lam_dev, u_dev, stream=None):
    return _check(ctx, load().arb_rpy_apply_noalloc_dev(ctx, int(N), _ptr(pos_dev),
                                                        _ptr(lam_dev), _ptr(u_dev),
                                                        _ptr(stream)))


def arb_system_apply(ctx, y):
    n = arb_sizes(ctx)[3]
    y_, yp = _d(y, n)
    o, op = _out(n)
    _check(ctx, load().arb_system_apply(ctx, yp, op))
    return o


def arb_K_apply(ctx, U):
    N, M, _, _ = arb_sizes(ctx)
    u_, up = _d(U, 6 * M)
    o, op = _out(3 * N)
    _check(ctx, load().arb_K_apply(ctx, up, op))
    return o


def arb_KT_apply(ctx, lam):
    N, M, _, _ = arb_sizes(ctx)
    l_, lp = _d(lam, 3 * N)
    o, op = _out(6 * M)
    _check(ctx, load().arb_KT_apply(ctx, lp, op))
    return o


def arb_constraint_rows(ctx):
    Nc = arb_sizes(ctx)[2]
    coef, cp = _out(12 * Nc)
    B, bp = _out(Nc)
    pq = np.zeros(2 * Nc, np.int32)
    _check(ctx, load().arb_constraint_rows(ctx, cp, pq.ctypes.data_as(_IP), bp))
    return coef.reshape(Nc, 12), pq.reshape(Nc, 2), B


def arb_precond_build(ctx):
    return _check(ctx, load().arb_precond_build(ctx))


def arb_precond_apply(ctx, r):
    n = arb_sizes(ctx)[3]
    r_, rp = _d(r, n)
    z, zp = _out(n)
    _check(ctx, load().arb_precond_apply(ctx, rp, zp))
    return z


def arb_precond_block(ctx, p, m):
    """(L (m, m), N~ (6, 6)) of body p; m = 0 returns (None, N~) only (the
    per-type variants have no per-body factor)."""
    L, Lp = _out(m * m) if m > 0 else (None, None)
    Nt, Np = _out(36)
    _check(ctx, load().arb_precond_block(ctx, int(p), Lp, Np))
    return (L.reshape(m, m) if m > 0 else None), Nt.reshape(6, 6)


def arb_solve(ctx, F, u_slip=None, y0=None):
    """Returns (status, U (M,6), phi (Nc,), lambda (N,3), info dict)."""
    N, M, Nc, n = arb_sizes(ctx)
    F_, Fp = _d(F, 6 * M)
    us_, usp = _d(u_slip, 3 * N) if u_slip is not None else (None, None)
    y_, yp = _d(y0, n) if y0 is not None else (None, None)
    U, Up = _out(6 * M)
    phi, php = _out(max(Nc, 1))
    lam, lp = _out(3 * N)
    info = arb_solve_info()
    rc = _check(ctx, load().arb_solve(ctx, Fp, usp, yp, Up, php, lp, C.byref(info)))
    return rc, U.reshape(M, 6), phi[:Nc], lam.reshape(N, 3), info.to_dict()


def arb_solve_dev(ctx, F_dev, u_slip_dev, y_dev, warm=False, stream=None):
    info = arb_solve_info()
    rc = _check(ctx, load().arb_solve_dev(ctx, _ptr(F_dev), _ptr(u_slip_dev), _ptr(y_dev),
                                          int(bool(warm)), C.byref(info), _ptr(stream)))
    return rc, info.to_dict()


def arb_euler_update(ctx, U, dt):
    N, M, _, _ = arb_sizes(ctx)
    u_, up = _d(U, 6 * M)
    q, qp = _out(3 * M)
    t, tp = _out(4 * M)
    _check(ctx, load().arb_euler_update(ctx, up, float(dt), qp, tp))
    return q.reshape(M, 3), t.reshape(M, 4)


def arb_correct_positions(ctx, tol=1e-10, max_iter=50):
    N, M, _, _ = arb_sizes(ctx)
    q, qp = _out(3 * M)
    t, tp = _out(4 * M)
    it = C.c_int()
    res = C.c_double()
    _check(ctx, load().arb_correct_positions(ctx, float(tol), int(max_iter), qp, tp,
                                             C.byref(it), C.byref(res)))
    return q.reshape(M, 3), t.reshape(M, 4), it.value, res.value


def arb_reconstruct(ctx):
    """Returns (q (M,3), g_inf, g2) after rebuilding the articulated bodies."""
    N, M, _, _ = arb_sizes(ctx)
    q, qp = _out(3 * M)
    gi, g2 = C.c_double(), C.c_double()
    _check(ctx, load().arb_reconstruct(ctx, qp, C.byref(gi), C.byref(g2)))
    return q.reshape(M, 3), gi.value, g2.value


def arb_link_residual(ctx):
    """(g_inf, g2) of the links at the context's state."""
    gi, g2 = C.c_double(), C.c_double()
    _check(ctx, load().arb_link_residual(ctx, C.byref(gi), C.byref(g2)))
    return gi.value, g2.value


def arb_step_euler(ctx, F, dt, delta=1e-10, corr_tol=1e-10, corr_max_iter=50, warm=True,
                   u_slip=None):
    """Returns (status, q (M,3), theta (M,4), U (M,6), info dict) after one step."""
    N, M, _, _ = arb_sizes(ctx)
    F_, Fp = _d(F, 6 * M)
    us_, usp = _d(u_slip, 3 * N) if u_slip is not None else (None, None)
    q, qp = _out(3 * M)
    t, tp = _out(4 * M)
    U, Up = _out(6 * M)
    info = arb_step_info()
    rc = _check(ctx, load().arb_step_euler(ctx, Fp, usp, float(dt), float(delta),
                                           float(corr_tol), int(corr_max_iter), int(bool(warm)),
                                           qp, tp, Up, C.byref(info)))
    return rc, q.reshape(M, 3), t.reshape(M, 4), U.reshape(M, 6), info.to_dict()


def arb_step_midpoint(ctx, F, dt, delta=1e-10, corr_tol=1e-10, corr_max_iter=50, warm=True,
                      u_slip=None):
    """Returns (status, q (M,3), theta (M,4), U^(k+1/2) (M,6), info dict) after one step."""
    N, M, _, _ = arb_sizes(ctx)
    F_, Fp = _d(F, 6 * M)
    us_, usp = _d(u_slip, 3 * N) if u_slip is not None else (None, None)
    q, qp = _out(3 * M)
    t, tp = _out(4 * M)
    U, Up = _out(6 * M)
    info = arb_step_info()
    rc = _check(ctx, load().arb_step_midpoint(ctx, Fp, usp, float(dt), float(delta),
                                              float(corr_tol), int(corr_max_iter),
                                              int(bool(warm)), qp, tp, Up, C.byref(info)))
    return rc, q.reshape(M, 3), t.reshape(M, 4), U.reshape(M, 6), info.to_dict()


def _arms(P, dl_p, dl_q, dldot_p=None, dldot_q=None, proj=None):
    """An arb_arms over float64 copies of the arrays (kept alive by the returned list)."""
    keep = []
    ptrs = []
    for a, n in ((dl_p, 3), (dl_q, 3), (dldot_p, 3), (dldot_q, 3), (proj, 9)):
        if a is None:
            ptrs.append(None)
            continue
        x, xp = _d(a, n * P)
        keep.append(x)
        ptrs.append(xp)
    return arb_arms(*ptrs), keep


def arb_step_euler_arms(ctx, F, dt, end, delta=1e-10, corr_tol=1e-10, corr_max_iter=50,
                        warm=True, u_slip=None):
    """arb_step_euler with the arms at t + dt: end = (dl_p, dl_q[, dldot_p, dldot_q
    [, proj]]), the optional ones may be None.  Returns as arb_step_euler."""
    N, M, _, _ = arb_sizes(ctx)
    P = len(np.asarray(end[0]).ravel()) // 3
    ae, keep = _arms(P, *end)
    F_, Fp = _d(F, 6 * M)
    us_, usp = _d(u_slip, 3 * N) if u_slip is not None else (None, None)
    q, qp = _out(3 * M)
    t, tp = _out(4 * M)
    U, Up = _out(6 * M)
    info = arb_step_info()
    rc = _check(ctx, load().arb_step_euler_arms(ctx, Fp, usp, float(dt), float(delta),
                                                float(corr_tol), int(corr_max_iter),
                                                int(bool(warm)), C.byref(ae), qp, tp, Up,
                                                C.byref(info)))
    return rc, q.reshape(M, 3), t.reshape(M, 4), U.reshape(M, 6), info.to_dict()


def arb_step_midpoint_arms(ctx, F, dt, mid, end, delta=1e-10, corr_tol=1e-10, corr_max_iter=50,
                           warm=True, u_slip=None):
    """arb_step_midpoint with the arms at t + dt/2 (mid) and t + dt (end), each as
    for arb_step_euler_arms.  Returns as arb_step_midpoint."""
    N, M, _, _ = arb_sizes(ctx)
    P = len(np.asarray(end[0]).ravel()) // 3
    am, keep_m = _arms(P, *mid)
    ae, keep_e = _arms(P, *end)
    F_, Fp = _d(F, 6 * M)
    us_, usp = _d(u_slip, 3 * N) if u_slip is not None else (None, None)
    q, qp = _out(3 * M)
    t, tp = _out(4 * M)
    U, Up = _out(6 * M)
    info = arb_step_info()
    rc = _check(ctx, load().arb_step_midpoint_arms(ctx, Fp, usp, float(dt), float(delta),
                                                   float(corr_tol), int(corr_max_iter),
                                                   int(bool(warm)), C.byref(am), C.byref(ae),
                                                   qp, tp, Up, C.byref(info)))
    return rc, q.reshape(M, 3), t.reshape(M, 4), U.reshape(M, 6), info.to_dict()


def arb_profile(ctx, enable=True):
    return _check(ctx, load().arb_profile(ctx, int(bool(enable))))


def arb_fmm_get_stats(ctx):
    """Tree statistics of the fast product (after a product has built the tree)."""
    st = arb_fmm_stats()
    _check(ctx, load().arb_fmm_get_stats(ctx, C.byref(st)))
    return {k: getattr(st, k) for k, _ in st._fields_}


def arb_fmm_plan(pos, a, order=0, levels=0, leaf=0):
    """Host-only plan of the fast product's octree (no device): its statistics."""
    p_, pp = _d(pos)
    st = arb_fmm_stats()
    rc = load().arb_fmm_plan(p_.size // 3, pp, float(a), int(order), int(levels), int(leaf),
                             C.byref(st))
    if rc < 0:
        raise ArbError(rc, "arb_fmm_plan")
    return {k: getattr(st, k) for k, _ in st._fields_}


def arb_profile_read(ctx):
    """(summed pair-kernel ms, launches) since the last read."""
    ms = C.c_double()
    n = C.c_int()
    _check(ctx, load().arb_profile_read(ctx, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def _f(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a, a.ctypes.data_as(_FP)


def arb_mlp_set_params(ctx, params):
    p, pp = _f(params, N_MLP_PARAMS)
    return _check(ctx, load().arb_mlp_set_params(ctx, N_MLP_PARAMS, pp))


def arb_mlp_set_scaling(ctx, in_mu, in_sd, out_mu, out_sd):
    a1, p1 = _f(in_mu, 7)
    a2, p2 = _f(in_sd, 7)
    a3, p3 = _f(out_mu, 21)
    a4, p4 = _f(out_sd, 21)
    return _check(ctx, load().arb_mlp_set_scaling(ctx, p1, p2, p3, p4))


def arb_mlp_get_params(ctx):
    out = np.zeros(N_MLP_PARAMS, np.float32)
    _check(ctx, load().arb_mlp_get_params(ctx, N_MLP_PARAMS, out.ctypes.data_as(_FP)))
    return out


def arb_mlp_forward(ctx, X):
    x, xp = _f(X)
    B = x.size // 7
    Y = np.zeros(B * 21, np.float32)
    _check(ctx, load().arb_mlp_forward(ctx, B, xp, Y.ctypes.data_as(_FP)))
    return Y.reshape(B, 21)


def arb_mlp_grad(ctx, X, T):
    x, xp = _f(X)
    B = x.size // 7
    t, tp = _f(T, B * 21)
    g = np.zeros(N_MLP_PARAMS, np.float32)
    loss = C.c_double()
    _check(ctx, load().arb_mlp_grad(ctx, B, xp, tp, g.ctypes.data_as(_FP), C.byref(loss)))
    return loss.value, g


def arb_mlp_train_step_dev(ctx, B, X_dev, T_dev, lr, want_loss=False, stream=None):
    loss = C.c_double()
    _check(ctx, load().arb_mlp_train_step_dev(ctx, int(B), _ptr(X_dev), _ptr(T_dev),
                                              float(lr), C.byref(loss) if want_loss else None,
                                              _ptr(stream)))
    return loss.value if want_loss else None


def arb_mlp_features(ctx):
    M = arb_sizes(ctx)[1]
    X = np.zeros(M * 7, np.float32)
    _check(ctx, load().arb_mlp_features(ctx, X.ctypes.data_as(_FP)))
    return X.reshape(M, 7)


def arb_body_mobility(ctx):
    """(N~ (M,6,6) float64, training labels (M,21) float32)."""
    M = arb_sizes(ctx)[1]
    out, op = _out(36 * M)
    T = np.zeros(M * 21, np.float32)
    _check(ctx, load().arb_body_mobility(ctx, op, T.ctypes.data_as(_FP)))
    return out.reshape(M, 6, 6), T.reshape(M, 21)


# ------------------------------------------------------------------ convenience
def context_for(wl, precision=ARB_FP64, tol=1e-10, restart=100, max_iter=1000,
                precond=ARB_PC_BLOCK, device=0, slices=0, pair_kernel=0, graphs=0, model=None,
                fmm_order=0, fmm_levels=0, fmm_leaf=0, left_precond=0, small_cycle=0,
                refine_final=0):
    """Create a context and load a workload (bodies, links, rows, state).  The body
    model defaults to single-blob for workloads that mark themselves so."""
    if model is None:
        model = ARB_MODEL_SINGLE_BLOB if wl.extra.get("single_blob") else ARB_MODEL_MULTIBLOB
    ctx = arb_create(device=device, precision=precision, wall=wl.wall, eta=wl.eta, a=wl.a,
                     tol=tol, restart=restart, max_iter=max_iter, precond=precond, slices=slices,
                     pair_kernel=pair_kernel, graphs=graphs, model=model, fmm_order=fmm_order,
                     fmm_levels=fmm_levels, fmm_leaf=fmm_leaf, left_precond=left_precond,
                     small_cycle=small_cycle, refine_final=refine_final)
    arb_set_bodies(ctx, wl.blob_offset, wl.r_ref, wl.body_type)
    if len(wl.pq):
        arb_set_links(ctx, wl.pq, wl.dl_p, wl.dl_q, wl.dldot_p, wl.dldot_q, wl.nproj, wl.proj)
    if len(wl.row_rhs):
        arb_set_rows(ctx, wl.row_pq, wl.row_coef, wl.row_rhs)
    arb_set_state(ctx, wl.q, wl.theta)
    return ctx

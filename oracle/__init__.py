"""FP64 CPU oracle for batched rigid-body kinematics and dynamics.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use it; the GPU library never imports, links or calls it, and it
imports nothing of the GPU library.

``rbd_oracle.cpp`` holds the recursive Featherstone algorithms (paper Sec. II,
Eq. (1)-(2); the quantities Alg. 1 and Alg. 2 compute), ``jacobian_form``
computes M and inverse dynamics a second, independent way (centre-of-mass
Jacobians in the world frame and Kane's equations), and ``euler_lagrange``
derives M, c and g symbolically from the Lagrangian for small chains. Every
array here is instance-major float64.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# ORACLE_LIB_OVERRIDE loads another build of rbd_oracle.cpp, e.g. one with a
# deliberately planted mistake, to check that the pins catch it.
_LOAD_PATH = os.environ.get("ORACLE_LIB_OVERRIDE", LIB_PATH)

METHOD_LLT, METHOD_LTL, METHOD_ABA = 0, 1, 2


class _Model(C.Structure):
    _fields_ = [
        ("n_bodies", C.c_int32),
        ("parent", C.POINTER(C.c_int32)),
        ("joint_type", C.POINTER(C.c_int32)),
        ("axis", C.POINTER(C.c_double)),
        ("origin", C.POINTER(C.c_double)),
        ("mass", C.POINTER(C.c_double)),
        ("com", C.POINTER(C.c_double)),
        ("inertia", C.POINTER(C.c_double)),
        ("gravity", C.c_double * 3),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LOAD_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LOAD_PATH)
        P = C.POINTER
        d, i64, i32 = P(C.c_double), C.c_int64, C.c_int32
        m = P(_Model)
        L.orc_dims.argtypes = [m, P(C.c_int), P(C.c_int)]
        L.orc_fk.argtypes = [m, i64, d, d]
        L.orc_jacobian.argtypes = [m, i64, d, i32, P(C.c_int32), d]
        L.orc_rnea.argtypes = [m, i64, d, d, d, d]
        L.orc_rnea_nograv.argtypes = [m, i64, d, d, d, d]
        L.orc_rnea_ext.argtypes = [m, i64, d, d, d, d, d]
        L.orc_fwd_dyn_ext.argtypes = [m, i64, d, d, d, d, d, C.c_int]
        L.orc_crba.argtypes = [m, i64, d, d]
        L.orc_fwd_dyn.argtypes = [m, i64, d, d, d, d, C.c_int]
        L.orc_fwd_dyn_vjp_fd.argtypes = [m, i64, d, d, d, d, d, d, d, d, d, C.c_double, C.c_int]
        L.orc_fwd_dyn_jvp_fd.argtypes = [m, i64, d, d, d, d, d, d, d, d, d, C.c_double, C.c_int]
        L.orc_rnea_jvp_fd.argtypes = [m, i64, d, d, d, d, d, d, d, d, d, C.c_double]
        L.orc_rnea_vjp_fd.argtypes = [m, i64, d, d, d, d, d, d, d, d, d, C.c_double]
        L.orc_count_ops.argtypes = [m, C.c_int, P(C.c_longlong)]
        L.orc_max_threads.argtypes = []
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _model(desc):
    """Build the C view of a TreeDesc; the arrays are kept alive on the struct."""
    d = desc.contiguous()
    s = _Model()
    s.n_bodies = d.n_bodies
    s.parent = d.parent.ctypes.data_as(C.POINTER(C.c_int32))
    s.joint_type = d.joint_type.ctypes.data_as(C.POINTER(C.c_int32))
    s.axis, s.origin, s.mass = _dp(d.axis), _dp(d.origin), _dp(d.mass)
    s.com, s.inertia = _dp(d.com), _dp(d.inertia)
    for k in range(3):
        s.gravity[k] = float(d.gravity[k])
    s._keep = d
    return s


def _c(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid arguments")


def dims(desc):
    nq, nv = C.c_int(), C.c_int()
    _check(lib().orc_dims(C.byref(_model(desc)), C.byref(nq), C.byref(nv)), "dims")
    return nq.value, nv.value


def fk(desc, q):
    """World pose of every body, [B, n_bodies, 3, 4] = [R | p]."""
    q = _c(q)
    B = q.shape[0]
    T = np.empty((B, desc.n_bodies, 12))
    _check(lib().orc_fk(C.byref(_model(desc)), B, _dp(q), _dp(T)), "fk")
    return T.reshape(B, desc.n_bodies, 3, 4)


def jacobian(desc, q, frames=None):
    """World-aligned geometric Jacobians at the frame origins, [B, nf, 6, nv], rows [v; w]."""
    q = _c(q)
    B = q.shape[0]
    frames = np.arange(desc.n_bodies, dtype=np.int32) if frames is None else np.asarray(frames, dtype=np.int32)
    frames = np.ascontiguousarray(frames)
    J = np.empty((B, len(frames), 6, desc.nv))
    _check(lib().orc_jacobian(C.byref(_model(desc)), B, _dp(q), len(frames),
                              frames.ctypes.data_as(C.POINTER(C.c_int32)), _dp(J)), "jacobian")
    return J


def rnea(desc, q, qd, qdd=None, gravity=True, fext=None):
    """Inverse dynamics tau = M qdd + c + g - sum_i J_i^T F_i, Eq. (1); qdd=None gives h(q, qd).

    fext: [B, n_bodies, 6] external spatial forces in world axes, [force; moment
    about the world origin] (the F_ext input of Alg. 1)."""
    q, qd = _c(q), _c(qd)
    qdd = None if qdd is None else _c(qdd)
    tau = np.empty_like(qd)
    if fext is not None:
        if not gravity:
            raise ValueError("oracle rnea: fext with gravity=False is not provided")
        fext = _c(fext)
        _check(lib().orc_rnea_ext(C.byref(_model(desc)), q.shape[0], _dp(q), _dp(qd), _dp(qdd), _dp(fext),
                                  _dp(tau)), "rnea")
        return tau
    fn = lib().orc_rnea if gravity else lib().orc_rnea_nograv
    _check(fn(C.byref(_model(desc)), q.shape[0], _dp(q), _dp(qd), _dp(qdd), _dp(tau)), "rnea")
    return tau


def crba(desc, q):
    """Joint-space mass matrix, [B, nv, nv]."""
    q = _c(q)
    H = np.empty((q.shape[0], desc.nv, desc.nv))
    _check(lib().orc_crba(C.byref(_model(desc)), q.shape[0], _dp(q), _dp(H)), "crba")
    return H


def fwd_dyn(desc, q, qd, tau, method=METHOD_LTL, fext=None):
    """Forward dynamics qdd = M^-1 (tau - h + sum_i J_i^T F_i), Eq. (2); fext as for rnea."""
    q, qd, tau = _c(q), _c(qd), _c(tau)
    qdd = np.empty_like(qd)
    if fext is not None:
        fext = _c(fext)
        _check(lib().orc_fwd_dyn_ext(C.byref(_model(desc)), q.shape[0], _dp(q), _dp(qd), _dp(tau), _dp(fext),
                                     _dp(qdd), method), "fwd_dyn")
        return qdd
    _check(lib().orc_fwd_dyn(C.byref(_model(desc)), q.shape[0], _dp(q), _dp(qd), _dp(tau), _dp(qdd), method),
           "fwd_dyn")
    return qdd


def fwd_dyn_vjp_fd(desc, q, qd, tau, gbar, h=1e-6, method=METHOD_LTL, fext=None):
    """(gq, gqd, gtau) = gbar^T d qdd / d(q, qd, tau) by central differences of step h; with external
    forces fext [B, n, 6] (or [B, 6n]) also gfext = gbar^T d qdd / dF, [B, 6n]."""
    q, qd, tau, gbar = _c(q), _c(qd), _c(tau), _c(gbar)
    gq, gqd, gtau = np.empty_like(q), np.empty_like(qd), np.empty_like(tau)
    fx = None if fext is None else _c(np.asarray(fext).reshape(q.shape[0], -1))
    gf = None if fext is None else np.empty_like(fx)
    _check(lib().orc_fwd_dyn_vjp_fd(C.byref(_model(desc)), q.shape[0], _dp(q), _dp(qd), _dp(tau),
                                    None if fx is None else _dp(fx), _dp(gbar), _dp(gq), _dp(gqd), _dp(gtau),
                                    None if gf is None else _dp(gf), h, method), "vjp")
    return (gq, gqd, gtau) if fext is None else (gq, gqd, gtau, gf)


def fwd_dyn_jvp_fd(desc, q, qd, tau, dq, dqd, dtau, h=1e-6, method=METHOD_LTL, fext=None, dfext=None):
    """d qdd along (dq, dqd, dtau[, dfext]): one central difference of step h of forward dynamics
    (with external forces fext when given; either force array may be None)."""
    q, qd, tau, dq, dqd, dtau = _c(q), _c(qd), _c(tau), _c(dq), _c(dqd), _c(dtau)
    B = q.shape[0]
    fx = None if fext is None else _c(np.asarray(fext).reshape(B, -1))
    dfx = None if dfext is None else _c(np.asarray(dfext).reshape(B, -1))
    dqdd = np.empty_like(qd)
    _check(lib().orc_fwd_dyn_jvp_fd(C.byref(_model(desc)), B, _dp(q), _dp(qd), _dp(tau),
                                    None if fx is None else _dp(fx), _dp(dq), _dp(dqd), _dp(dtau),
                                    None if dfx is None else _dp(dfx), _dp(dqdd), h, method), "jvp")
    return dqdd


def rnea_jvp_fd(desc, q, qd, qdd, dq, dqd, dqdd, h=1e-6, fext=None, dfext=None):
    """d tau along (dq, dqd, dqdd[, dfext]) of inverse dynamics tau = ID(q, qd, qdd, F), Eq. (1): one
    central difference of step h (with external forces fext when given; either force array may be
    None)."""
    q, qd, qdd, dq, dqd, dqdd = _c(q), _c(qd), _c(qdd), _c(dq), _c(dqd), _c(dqdd)
    B = q.shape[0]
    fx = None if fext is None else _c(np.asarray(fext).reshape(B, -1))
    dfx = None if dfext is None else _c(np.asarray(dfext).reshape(B, -1))
    dtau = np.empty_like(qd)
    _check(lib().orc_rnea_jvp_fd(C.byref(_model(desc)), B, _dp(q), _dp(qd), _dp(qdd),
                                 None if fx is None else _dp(fx), _dp(dq), _dp(dqd), _dp(dqdd),
                                 None if dfx is None else _dp(dfx), _dp(dtau), h), "rnea jvp")
    return dtau


def rnea_vjp_fd(desc, q, qd, qdd, lam, h=1e-6, fext=None, want_fext=False):
    """Cotangents (g_q, g_qd, g_qdd[, g_fext]) = lam^T dID/d(q, qd, qdd[, F]) of inverse dynamics
    tau = ID(q, qd, qdd, F), Eq. (1), by central differences of step h on every coordinate (with external
    forces fext when given)."""
    q, qd, qdd, lam = _c(q), _c(qd), _c(qdd), _c(lam)
    B = q.shape[0]
    fx = None if fext is None else _c(np.asarray(fext).reshape(B, -1))
    gq, gqd, gqdd = np.empty_like(q), np.empty_like(qd), np.empty_like(qd)
    gf = np.empty((B, 6 * desc.n_bodies)) if want_fext else None
    _check(lib().orc_rnea_vjp_fd(C.byref(_model(desc)), B, _dp(q), _dp(qd), _dp(qdd),
                                 None if fx is None else _dp(fx), _dp(lam), _dp(gq), _dp(gqd), _dp(gqdd),
                                 None if gf is None else _dp(gf), h), "rnea vjp")
    return (gq, gqd, gqdd, gf) if want_fext else (gq, gqd, gqdd)


OPS = {"fk": 0, "jacobian": 1, "rnea": 2, "rnea_bias": 3, "crba": 4, "fwd_dyn_llt": 5, "fwd_dyn_ltl": 6, "aba": 7}


def count_ops(desc, op):
    """Arithmetic of one evaluation: dict(addsub, mul, div, sqrt, trig, flops=addsub+mul)."""
    out = (C.c_longlong * 5)()
    _check(lib().orc_count_ops(C.byref(_model(desc)), OPS[op], out), "count_ops")
    r = dict(zip(["addsub", "mul", "div", "sqrt", "trig"], list(out)))
    r["flops"] = r["addsub"] + r["mul"]
    return r


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(n: int) -> int:
    """Use n host threads from now on; returns the previous count."""
    return int(lib().orc_set_threads(int(n)))

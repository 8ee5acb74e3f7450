"""Python binding of librbd.so (ctypes): argument marshalling only.

Every batched array is a torch CUDA float32 tensor in structure-of-arrays
layout [rows, batch] with unit stride along the batch (ld = stride(0)); the
call is enqueued on torch's current stream. PyTorch supplies device memory and
streams; all arithmetic runs in the HIP kernels of librbd.so. There is no CPU
fallback: a missing library raises.

Operations (arxiv 2604.04310): fk and jacobian (Sec. II, Sec. IV), rnea
(Eq. (1), Alg. 1), crba (Alg. 2), fwd_dyn (Eq. (2)), fwd_dyn_vjp and the
autograd function FwdDyn (reverse-mode AD, Sec. I).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librbd.so")

RBD_OK = 0
STATUS = {0: "RBD_OK", 1: "RBD_E_INVAL", 2: "RBD_E_NOMEM", 3: "RBD_E_NODEVICE", 4: "RBD_E_LAUNCH",
          5: "RBD_E_UNSUPPORTED", 6: "RBD_E_TIMEOUT", 7: "RBD_E_SHUTDOWN", 8: "RBD_E_COMPILE",
          9: "RBD_E_CANCELLED"}
OP_FWD_DYN, OP_RNEA, OP_FWD_DYN_VJP = 0, 1, 2

# Every symbol include/rbd.h declares.
EXPORTS = ["rbd_model_create", "rbd_model_destroy", "rbd_model_dims", "rbd_model_topology", "rbd_fk",
           "rbd_jacobian", "rbd_rnea", "rbd_crba", "rbd_fwd_dyn", "rbd_aba", "rbd_fwd_dyn_jvp", "rbd_rnea_jvp", "rbd_rnea_vjp", "rbd_fwd_dyn_vjp", "rbd_diff_ik", "rbd_osc", "rbd_status_str",
           "rbd_last_error", "rbd_device_count", "rbd_diag_fma_rate", "rbd_diag_hbm_rate", "rbd_precompile_topology", "rbd_server_create", "rbd_server_submit", "rbd_server_wait", "rbd_server_cancel",
           "rbd_server_get_stats", "rbd_server_reset_stats", "rbd_server_destroy", "rbd_diag_serve_load",
           "rbd_packed_static"]


class RbdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class TreeDescC(C.Structure):
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


class ServerConfigC(C.Structure):
    _fields_ = [("device", C.c_int), ("arena_bytes", C.c_size_t), ("n_streams", C.c_int),
                ("max_batch_requests", C.c_int), ("max_wait_us", C.c_double), ("use_graphs", C.c_int),
                ("per_request", C.c_int), ("executor", C.c_int), ("fail_group", C.c_int64),
                ("max_group_bytes", C.c_size_t)]


EXEC_DEVICE, EXEC_HOST = 0, 1


class LoadRequestC(C.Structure):
    _fields_ = [("model", C.c_void_p), ("op", C.c_int), ("batch", C.c_int64), ("inp", C.c_void_p * 4)]


class PackedRequestC(C.Structure):
    _fields_ = [("inp", C.c_void_p * 4), ("out", C.c_void_p * 3), ("batch", C.c_int64)]


class ServerStatsC(C.Structure):
    _fields_ = [("requests", C.c_uint64), ("instances", C.c_uint64), ("launches", C.c_uint64),
                ("p50_us", C.c_double), ("p99_us", C.c_double), ("max_us", C.c_double), ("mean_us", C.c_double),
                ("busy_s", C.c_double), ("groups_timed", C.c_uint64), ("gpu_kernel_s", C.c_double),
                ("gpu_kernel_overlap_s", C.c_double), ("gpu_kernel_sum_s", C.c_double), ("gpu_copy_s", C.c_double),
                ("gpu_active_s", C.c_double)]


_lib = None


def lib():
    """Load librbd.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P, vp, i64, i32 = C.POINTER, C.c_void_p, C.c_int64, C.c_int32
        L.rbd_model_create.argtypes = [P(TreeDescC), C.c_int, P(vp)]
        L.rbd_model_destroy.argtypes = [vp]
        L.rbd_model_dims.argtypes = [vp, P(C.c_int), P(C.c_int), P(C.c_int)]
        L.rbd_model_topology.argtypes = [vp]
        L.rbd_model_topology.restype = C.c_char_p
        L.rbd_fk.argtypes = [vp, i64, i64, vp, vp, vp]
        L.rbd_jacobian.argtypes = [vp, i64, i64, vp, i32, P(C.c_int32), vp, vp]
        L.rbd_rnea.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp]
        L.rbd_crba.argtypes = [vp, i64, i64, vp, vp, vp]
        L.rbd_fwd_dyn.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp]
        L.rbd_aba.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp]
        L.rbd_fwd_dyn_vjp.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.rbd_fwd_dyn_jvp.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.rbd_rnea_jvp.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.rbd_rnea_vjp.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        f32 = C.c_float
        L.rbd_diff_ik.argtypes = [vp, i64, i64, vp, C.c_int32, vp, f32, f32, vp, vp]
        L.rbd_osc.argtypes = [vp, i64, i64, vp, vp, C.c_int32, vp, f32, f32, f32, vp, vp]
        L.rbd_status_str.argtypes = [C.c_int]
        L.rbd_status_str.restype = C.c_char_p
        L.rbd_last_error.argtypes = []
        L.rbd_last_error.restype = C.c_char_p
        L.rbd_device_count.argtypes = []
        L.rbd_diag_fma_rate.argtypes = [C.c_int, C.c_int, C.c_int, P(C.c_double)]
        L.rbd_diag_hbm_rate.argtypes = [C.c_int, C.c_int64, C.c_int, C.c_int, P(C.c_double)]
        L.rbd_precompile_topology.argtypes = [C.c_int32, P(C.c_int32), C.c_int, C.c_char_p, C.c_int32]
        L.rbd_server_create.argtypes = [P(ServerConfigC), P(vp)]
        L.rbd_server_submit.argtypes = [vp, vp, C.c_int, i64, P(vp), P(vp), P(C.c_uint64)]
        L.rbd_server_wait.argtypes = [vp, C.c_uint64, C.c_double, P(C.c_int)]
        L.rbd_server_cancel.argtypes = [vp, C.c_uint64]
        L.rbd_server_get_stats.argtypes = [vp, P(ServerStatsC)]
        L.rbd_server_reset_stats.argtypes = [vp]
        L.rbd_server_destroy.argtypes = [vp]
        L.rbd_diag_serve_load.argtypes = [vp, C.c_int, P(LoadRequestC), i64, C.c_double, C.c_int, C.c_uint64,
                                          P(C.c_double), P(i64)]
        L.rbd_packed_static.argtypes = [vp, C.c_int, C.c_int, P(PackedRequestC), vp]
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != RBD_OK:
        raise RbdError(status, lib().rbd_last_error().decode())


def device_count() -> int:
    return int(lib().rbd_device_count())


def fma_rate(blocks: int = 256, ilp: int = 16, device: int = 0) -> float:
    """Measured FP32 FMA TFLOP/s at a launch of `blocks` x 256 threads (diagnostic)."""
    out = C.c_double()
    check(lib().rbd_diag_fma_rate(int(device), int(blocks), int(ilp), C.byref(out)))
    return out.value


N_KERNELS = 40


def precompile_topology(parent, floating: bool, cache_dir: Optional[str] = None, kernel: int = -1) -> None:
    """Compile a tree topology's kernels (kernel -1: all of them) into a code-object cache (no GPU needed)."""
    par = (C.c_int32 * len(parent))(*[int(p) for p in parent])
    d = None if cache_dir is None else os.fsencode(cache_dir)
    check(lib().rbd_precompile_topology(len(parent), par, int(bool(floating)), d, int(kernel)))


def hbm_rate(nbytes: int = 1 << 30, mode: int = 0, blocks: int = 8192, device: int = 0) -> float:
    """Measured streaming HBM GB/s: mode 0 writes nbytes, mode 1 copies them (diagnostic)."""
    out = C.c_double()
    check(lib().rbd_diag_hbm_rate(int(device), int(nbytes), int(mode), int(blocks), C.byref(out)))
    return out.value


def desc_struct(desc) -> TreeDescC:
    """rbd_tree_desc view of any object with the tree fields (arrays kept alive)."""
    get = (lambda k: desc[k]) if isinstance(desc, dict) else (lambda k: getattr(desc, k))
    keep = {
        "parent": np.ascontiguousarray(get("parent"), dtype=np.int32),
        "joint_type": np.ascontiguousarray(get("joint_type"), dtype=np.int32),
        "axis": np.ascontiguousarray(get("axis"), dtype=np.float64),
        "origin": np.ascontiguousarray(get("origin"), dtype=np.float64),
        "mass": np.ascontiguousarray(get("mass"), dtype=np.float64),
        "com": np.ascontiguousarray(get("com"), dtype=np.float64),
        "inertia": np.ascontiguousarray(get("inertia"), dtype=np.float64),
    }
    s = TreeDescC()
    s.n_bodies = int(keep["parent"].shape[0])
    s.parent = keep["parent"].ctypes.data_as(C.POINTER(C.c_int32))
    s.joint_type = keep["joint_type"].ctypes.data_as(C.POINTER(C.c_int32))
    for k in ("axis", "origin", "mass", "com", "inertia"):
        setattr(s, k, keep[k].ctypes.data_as(C.POINTER(C.c_double)))
    g = np.asarray(get("gravity"), dtype=np.float64)
    for k in range(3):
        s.gravity[k] = float(g[k])
    s._keep = keep
    return s


class Model:
    """A kinematic tree resident on one GPU (owns the device tables); device=-1 makes a host-only
    model (no kernels) for a server with the host executor."""

    def __init__(self, desc, device: int = 0):
        self._h = C.c_void_p()
        self._desc = desc_struct(desc)
        check(lib().rbd_model_create(C.byref(self._desc), int(device), C.byref(self._h)))
        nq, nv, n = C.c_int(), C.c_int(), C.c_int()
        check(lib().rbd_model_dims(self._h, C.byref(nq), C.byref(nv), C.byref(n)))
        self.nq, self.nv, self.n_bodies, self.device = nq.value, nv.value, n.value, int(device)
        self.topology = lib().rbd_model_topology(self._h).decode()

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().rbd_model_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _soa(x, rows: int, name: str, batch: Optional[int] = None):
    """Checks a [rows, batch] SoA tensor and returns (ptr, batch, ld)."""
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32:
        raise TypeError(f"{name}: expected a CUDA float32 tensor")
    if x.dim() != 2 or x.shape[0] != rows:
        raise ValueError(f"{name}: expected shape [{rows}, batch], got {tuple(x.shape)}")
    if x.stride(1) != 1 and x.shape[1] > 1:
        raise ValueError(f"{name}: the batch dimension must have unit stride")
    if batch is not None and x.shape[1] != batch:
        raise ValueError(f"{name}: batch {x.shape[1]} != {batch}")
    ld = x.stride(0) if x.shape[0] > 1 else max(x.shape[1], 1)
    return C.c_void_p(x.data_ptr()), int(x.shape[1]), int(ld)


def _out(rows: int, batch: int, like):
    torch = _torch()
    return torch.empty((rows, batch), dtype=torch.float32, device=like.device)


def _same_ld(*lds):
    if len(set(lds)) != 1:
        raise ValueError("all arrays of one call must share the leading dimension (ld)")
    return lds[0]


def fk(model: Model, q):
    """World pose of every body: [n_bodies * 12, B], rows (i, 3x4 row-major [R | p])."""
    qp, B, ld = _soa(q, model.nq, "q")
    T = _out(model.n_bodies * 12, B, q)
    if B > 0 and ld != B:
        raise ValueError("fk: q must be contiguous (ld = batch) so that outputs share its ld")
    check(lib().rbd_fk(model.handle, B, ld, qp, C.c_void_p(T.data_ptr()), _stream()))
    return T


def jacobian(model: Model, q, frames: Optional[Sequence[int]] = None):
    """Geometric Jacobians [n_frames * 6 * nv, B] of the given body frames (all by default)."""
    qp, B, ld = _soa(q, model.nq, "q")
    if B > 0 and ld != B:
        raise ValueError("jacobian: q must be contiguous")
    fr = np.arange(model.n_bodies, dtype=np.int32) if frames is None else np.asarray(frames, dtype=np.int32)
    fr = np.ascontiguousarray(fr)
    J = _out(len(fr) * 6 * model.nv, B, q)
    check(lib().rbd_jacobian(model.handle, B, ld, qp, len(fr), fr.ctypes.data_as(C.POINTER(C.c_int32)),
                             C.c_void_p(J.data_ptr()), _stream()))
    return J


def rnea(model: Model, q, qd, qdd=None, out=None, fext=None):
    """Inverse dynamics tau [nv, B] (Eq. (1)); qdd=None gives the bias force h(q, qd).

    fext: optional [6 * n_bodies, B] external spatial forces, world axes, rows
    6 i .. 6 i + 5 = force on body i, then its moment about the world origin."""
    qp, B, l1 = _soa(q, model.nq, "q")
    qdp, _, l2 = _soa(qd, model.nv, "qd", B)
    lds = [l1, l2]
    qddp = None
    if qdd is not None:
        qddp, _, l3 = _soa(qdd, model.nv, "qdd", B)
        lds.append(l3)
    fp = None
    if fext is not None:
        fp, _, l5 = _soa(fext, 6 * model.n_bodies, "fext", B)
        lds.append(l5)
    tau = _out(model.nv, B, q) if out is None else out
    tp, _, l4 = _soa(tau, model.nv, "tau", B)
    ld = _same_ld(*lds, l4)
    check(lib().rbd_rnea(model.handle, B, ld, qp, qdp, qddp, fp, tp, _stream()))
    return tau


def crba(model: Model, q):
    """Mass matrix [nv * nv, B], row-major per instance."""
    qp, B, ld = _soa(q, model.nq, "q")
    if B > 0 and ld != B:
        raise ValueError("crba: q must be contiguous")
    M = _out(model.nv * model.nv, B, q)
    check(lib().rbd_crba(model.handle, B, ld, qp, C.c_void_p(M.data_ptr()), _stream()))
    return M


def _fd(fn, model: Model, q, qd, tau, out, fext):
    qp, B, l1 = _soa(q, model.nq, "q")
    qdp, _, l2 = _soa(qd, model.nv, "qd", B)
    taup, _, l3 = _soa(tau, model.nv, "tau", B)
    lds = [l1, l2, l3]
    fp = None
    if fext is not None:
        fp, _, l5 = _soa(fext, 6 * model.n_bodies, "fext", B)
        lds.append(l5)
    qdd = _out(model.nv, B, q) if out is None else out
    op, _, l4 = _soa(qdd, model.nv, "qdd", B)
    ld = _same_ld(*lds, l4)
    check(fn(model.handle, B, ld, qp, qdp, taup, fp, op, _stream()))
    return qdd


def fwd_dyn(model: Model, q, qd, tau, out=None, fext=None):
    """Forward dynamics qdd [nv, B] (Eq. (2)); fext as for rnea."""
    return _fd(lib().rbd_fwd_dyn, model, q, qd, tau, out, fext)


def aba(model: Model, q, qd, tau, out=None, fext=None):
    """Forward dynamics qdd [nv, B] by the articulated-body algorithm (same result as fwd_dyn)."""
    return _fd(lib().rbd_aba, model, q, qd, tau, out, fext)


def fwd_dyn_vjp(model: Model, q, qd, tau, g_qdd, want=(True, True, True), fext=None, want_fext=False):
    """(g_q [nq, B], g_qd [nv, B], g_tau [nv, B]) = g_qdd^T d qdd / d(q, qd, tau); None where not wanted.
    fext: optional [6 * n_bodies, B] external forces (as for rnea); want_fext adds g_fext [6 * n_bodies, B],
    the cotangent of the forces (returned fourth)."""
    qp, B, l1 = _soa(q, model.nq, "q")
    qdp, _, l2 = _soa(qd, model.nv, "qd", B)
    taup, _, l3 = _soa(tau, model.nv, "tau", B)
    gp, _, l4 = _soa(g_qdd, model.nv, "g_qdd", B)
    lds = [l1, l2, l3, l4]
    fp = None
    nf = 6 * model.n_bodies
    if fext is not None:
        fp, _, l5 = _soa(fext, nf, "fext", B)
        lds.append(l5)
    ld = _same_ld(*lds)
    if B > 0 and ld != B:
        raise ValueError("fwd_dyn_vjp: inputs must be contiguous")
    outs = [_out(model.nq, B, q) if want[0] else None, _out(model.nv, B, q) if want[1] else None,
            _out(model.nv, B, q) if want[2] else None, _out(nf, B, q) if want_fext else None]
    ptrs = [C.c_void_p(o.data_ptr()) if o is not None else None for o in outs]
    check(lib().rbd_fwd_dyn_vjp(model.handle, B, ld, qp, qdp, taup, fp, gp, ptrs[0], ptrs[1], ptrs[2], ptrs[3],
                                _stream()))
    return tuple(outs) if want_fext else tuple(outs[:3])


def rnea_vjp(model: Model, q, qd, qdd, lam, want=(True, True, True), fext=None, want_fext=False):
    """(g_q [nq, B], g_qd [nv, B], g_qdd [nv, B]) = lam^T dID/d(q, qd, qdd) of inverse dynamics (g_qdd = M lam);
    None where not wanted. fext: optional [6 * n_bodies, B] external forces; want_fext adds g_fext
    [6 * n_bodies, B] = -J_i lam (returned fourth)."""
    ins = [_soa(x, r, n, None) for x, r, n in ((q, model.nq, "q"), (qd, model.nv, "qd"), (qdd, model.nv, "qdd"),
                                               (lam, model.nv, "lam"))]
    nf = 6 * model.n_bodies
    fx = None if fext is None else _soa(fext, nf, "fext", None)
    B = ins[0][1]
    if any(i[1] != B for i in ins + ([fx] if fx else [])):
        raise ValueError("rnea_vjp: batch sizes differ")
    ld = _same_ld(*[i[2] for i in ins + ([fx] if fx else [])])
    if B > 0 and ld != B:
        raise ValueError("rnea_vjp: inputs must be contiguous")
    outs = [_out(model.nq, B, q) if want[0] else None, _out(model.nv, B, q) if want[1] else None,
            _out(model.nv, B, q) if want[2] else None, _out(nf, B, q) if want_fext else None]
    ptrs = [C.c_void_p(o.data_ptr()) if (o is not None and B) else None for o in outs]
    p = [i[0] for i in ins]
    check(lib().rbd_rnea_vjp(model.handle, B, ld, p[0], p[1], p[2], fx[0] if fx else None, p[3], *ptrs, _stream()))
    return tuple(outs) if want_fext else tuple(outs[:3])


def rnea_jvp(model: Model, q, qd, qdd, dq, dqd, dqdd, fext=None, dfext=None):
    """d tau [nv, B] of inverse dynamics along the tangent (dq [nq, B], dqd, dqdd [nv, B], and optionally dfext
    [6 * n_bodies, B]), with external forces fext [6 * n_bodies, B] when given."""
    ins = [_soa(x, r, n, None) for x, r, n in ((q, model.nq, "q"), (qd, model.nv, "qd"), (qdd, model.nv, "qdd"),
                                               (dq, model.nq, "dq"), (dqd, model.nv, "dqd"),
                                               (dqdd, model.nv, "dqdd"))]
    nf = 6 * model.n_bodies
    fx = [None if x is None else _soa(x, nf, n, None) for x, n in ((fext, "fext"), (dfext, "dfext"))]
    B = ins[0][1]
    if any(i[1] != B for i in ins + [f for f in fx if f is not None]):
        raise ValueError("rnea_jvp: batch sizes differ")
    ld = _same_ld(*[i[2] for i in ins + [f for f in fx if f is not None]])
    if B > 0 and ld != B:
        raise ValueError("rnea_jvp: inputs must be contiguous")
    dtau = _out(model.nv, B, q)
    p = [i[0] for i in ins]
    check(lib().rbd_rnea_jvp(model.handle, B, ld, p[0], p[1], p[2], fx[0][0] if fx[0] else None, p[3], p[4], p[5],
                             fx[1][0] if fx[1] else None, C.c_void_p(dtau.data_ptr()) if B else None, _stream()))
    return dtau


def fwd_dyn_jvp(model: Model, q, qd, tau, dq, dqd, dtau, want_qdd=False, fext=None, dfext=None):
    """d qdd [nv, B] along the tangent (dq [nq, B], dqd, dtau [nv, B], and optionally dfext [6 * n_bodies, B]),
    with external forces fext [6 * n_bodies, B] when given; with want_qdd also returns qdd."""
    ins = [_soa(x, r, n, None) for x, r, n in ((q, model.nq, "q"), (qd, model.nv, "qd"), (tau, model.nv, "tau"),
                                               (dq, model.nq, "dq"), (dqd, model.nv, "dqd"),
                                               (dtau, model.nv, "dtau"))]
    nf = 6 * model.n_bodies
    fx = [None if x is None else _soa(x, nf, n, None) for x, n in ((fext, "fext"), (dfext, "dfext"))]
    B = ins[0][1]
    if any(i[1] != B for i in ins + [f for f in fx if f is not None]):
        raise ValueError("fwd_dyn_jvp: batch sizes differ")
    ld = _same_ld(*[i[2] for i in ins + [f for f in fx if f is not None]])
    if B > 0 and ld != B:
        raise ValueError("fwd_dyn_jvp: inputs must be contiguous")
    dqdd = _out(model.nv, B, q)
    qdd = _out(model.nv, B, q) if want_qdd else None
    p = [i[0] for i in ins]
    check(lib().rbd_fwd_dyn_jvp(model.handle, B, ld, p[0], p[1], p[2], None if fx[0] is None else fx[0][0],
                                p[3], p[4], p[5], None if fx[1] is None else fx[1][0],
                                C.c_void_p(qdd.data_ptr()) if qdd is not None else None,
                                C.c_void_p(dqdd.data_ptr()), _stream()))
    return (qdd, dqdd) if want_qdd else dqdd


def diff_ik(model: Model, q, target, gain: float, damping: float, frame: Optional[int] = None, out=None):
    """Damped least-squares joint velocity [nv, B] toward target [12, B] ([R* | p*] row-major) for a frame
    (the last body by default; other frames compile their kernel on first use)."""
    qp, B, l1 = _soa(q, model.nq, "q")
    tp, _, l2 = _soa(target, 12, "target", B)
    qd = _out(model.nv, B, q) if out is None else out
    op, _, l3 = _soa(qd, model.nv, "qd", B)
    ld = _same_ld(l1, l2, l3)
    f = model.n_bodies - 1 if frame is None else int(frame)
    check(lib().rbd_diff_ik(model.handle, B, ld, qp, f, tp, float(gain), float(damping), op, _stream()))
    return qd


def osc(model: Model, q, qd, target, kp: float, kd: float, k_null: float, frame: Optional[int] = None, out=None):
    """Operational-space control torques [nv, B] for a frame (the last body by default; other frames compile
    their kernel on first use)."""
    qp, B, l1 = _soa(q, model.nq, "q")
    qdp, _, l2 = _soa(qd, model.nv, "qd", B)
    tp, _, l3 = _soa(target, 12, "target", B)
    tau = _out(model.nv, B, q) if out is None else out
    op, _, l4 = _soa(tau, model.nv, "tau", B)
    ld = _same_ld(l1, l2, l3, l4)
    f = model.n_bodies - 1 if frame is None else int(frame)
    check(lib().rbd_osc(model.handle, B, ld, qp, qdp, f, tp, float(kp), float(kd), float(k_null), op, _stream()))
    return tau


def _make_autograd():
    torch = _torch()

    class FwdDyn(torch.autograd.Function):
        """qdd = FD(q, qd, tau[, fext]) with the hand-written adjoint kernel as backward and the
        tangent kernel as the forward-mode rule (torch.autograd.forward_ad dual tensors; torch.func
        transforms hand the rules storage-less wrappers, which a kernel call cannot take).
        Inputs must be contiguous [rows, B] tensors; fext may be None."""

        @staticmethod
        def forward(model, q, qd, tau, fext):
            return fwd_dyn(model, q, qd, tau, fext=fext)

        @staticmethod
        def setup_context(ctx, inputs, output):
            model, q, qd, tau, fext = inputs
            ctx.model = model
            ctx.has_fext = fext is not None
            saved = (q, qd, tau) + ((fext,) if fext is not None else ())
            ctx.save_for_backward(*saved)
            ctx.save_for_forward(*saved)

        @staticmethod
        def backward(ctx, g):
            q, qd, tau, *rest = ctx.saved_tensors
            fext = rest[0] if ctx.has_fext else None
            want = ctx.needs_input_grad[1:4]
            want_f = ctx.has_fext and ctx.needs_input_grad[4]
            outs = fwd_dyn_vjp(ctx.model, q, qd, tau, g.contiguous(), want=tuple(bool(w) for w in want),
                               fext=fext, want_fext=want_f)
            gf = outs[3] if want_f else None
            return None, outs[0], outs[1], outs[2], gf

        @staticmethod
        def jvp(ctx, _model_t, q_t, qd_t, tau_t, f_t):
            q, qd, tau, *rest = ctx.saved_tensors
            fext = rest[0] if ctx.has_fext else None
            tangents = [torch.zeros_like(x) if t is None else t.contiguous()
                        for x, t in ((q, q_t), (qd, qd_t), (tau, tau_t))]
            df = f_t.contiguous() if (ctx.has_fext and f_t is not None) else None
            return fwd_dyn_jvp(ctx.model, q, qd, tau, *tangents, fext=fext, dfext=df)

    return FwdDyn


_FwdDyn = None
_InvDyn = None


def _make_rnea_autograd():
    torch = _torch()

    class InvDyn(torch.autograd.Function):
        """tau = ID(q, qd, qdd[, fext]) with the adjoint kernel (rbd_rnea_vjp) as backward and the
        tangent kernel (rbd_rnea_jvp) as the forward-mode rule. Inputs must be contiguous [rows, B]
        tensors; fext may be None."""

        @staticmethod
        def forward(model, q, qd, qdd, fext):
            return rnea(model, q, qd, qdd, fext=fext)

        @staticmethod
        def setup_context(ctx, inputs, output):
            model, q, qd, qdd, fext = inputs
            ctx.model = model
            ctx.has_fext = fext is not None
            saved = (q, qd, qdd) + ((fext,) if fext is not None else ())
            ctx.save_for_backward(*saved)
            ctx.save_for_forward(*saved)

        @staticmethod
        def backward(ctx, g):
            q, qd, qdd, *rest = ctx.saved_tensors
            fext = rest[0] if ctx.has_fext else None
            want = tuple(bool(w) for w in ctx.needs_input_grad[1:4])
            want_f = ctx.has_fext and ctx.needs_input_grad[4]
            outs = rnea_vjp(ctx.model, q, qd, qdd, g.contiguous(), want=want, fext=fext, want_fext=want_f)
            return None, outs[0], outs[1], outs[2], outs[3] if want_f else None

        @staticmethod
        def jvp(ctx, _model_t, q_t, qd_t, qdd_t, f_t):
            q, qd, qdd, *rest = ctx.saved_tensors
            fext = rest[0] if ctx.has_fext else None
            tangents = [torch.zeros_like(x) if t is None else t.contiguous()
                        for x, t in ((q, q_t), (qd, qd_t), (qdd, qdd_t))]
            df = f_t.contiguous() if (ctx.has_fext and f_t is not None) else None
            return rnea_jvp(ctx.model, q, qd, qdd, *tangents, fext=fext, dfext=df)

    return InvDyn


def rnea_autograd(model: Model, q, qd, qdd, fext=None):
    """Differentiable inverse dynamics: backward runs rbd_rnea_vjp, forward-mode AD rbd_rnea_jvp; fext
    (optional [6 * n_bodies, B] external forces) is differentiable too."""
    global _InvDyn
    if _InvDyn is None:
        _InvDyn = _make_rnea_autograd()
    return _InvDyn.apply(model, q.contiguous(), qd.contiguous(), qdd.contiguous(),
                         None if fext is None else fext.contiguous())


def fwd_dyn_autograd(model: Model, q, qd, tau, fext=None):
    """Differentiable forward dynamics: backward runs rbd_fwd_dyn_vjp, forward-mode AD rbd_fwd_dyn_jvp;
    fext (optional [6 * n_bodies, B] external forces) is differentiable too."""
    global _FwdDyn
    if _FwdDyn is None:
        _FwdDyn = _make_autograd()
    return _FwdDyn.apply(model, q.contiguous(), qd.contiguous(), tau.contiguous(),
                         None if fext is None else fext.contiguous())


# ---------------------------------------------------------------- serving
def op_shapes(model: Model, op: int):
    """Rows per instance of the inputs and outputs of a served operation."""
    nq, nv = model.nq, model.nv
    if op in (OP_FWD_DYN, OP_RNEA):
        return [nq, nv, nv], [nv]
    if op == OP_FWD_DYN_VJP:
        return [nq, nv, nv, nv], [nq, nv, nv]
    raise ValueError(f"unknown op {op}")


def packed_static(model: Model, op: int, requests) -> None:
    """rbd_packed_static on the current stream: `requests` is a list of (inputs, outputs), each a list of
    contiguous CUDA float32 tensors [batch, rows] with the rows of op_shapes(model, op); the outputs are
    written in place. Allocates no device memory."""
    torch = _torch()
    in_rows, out_rows = op_shapes(model, op)
    arr = (PackedRequestC * max(1, len(requests)))()
    for k, (ins, outs) in enumerate(requests):
        if len(ins) != len(in_rows) or len(outs) != len(out_rows):
            raise ValueError(f"request {k}: op {op} takes {len(in_rows)} inputs and {len(out_rows)} outputs")
        batch = int(ins[0].shape[0])
        for x, r in list(zip(ins, in_rows)) + list(zip(outs, out_rows)):
            if (not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32
                    or tuple(x.shape) != (batch, r) or not x.is_contiguous()):
                raise ValueError(f"request {k}: expected contiguous CUDA float32 [{batch}, {r}] arrays")
        for a, x in enumerate(ins):
            arr[k].inp[a] = x.data_ptr() if batch else None
        for a, x in enumerate(outs):
            arr[k].out[a] = x.data_ptr() if batch else None
        arr[k].batch = batch
    check(lib().rbd_packed_static(model.handle, int(op), len(requests), arr, _stream()))


class Server:
    """Continuous-batching service (rbd_server_*). Requests carry host arrays,
    instance-major float32 [batch, rows]; results land in host arrays."""

    def __init__(self, device: int = 0, arena_bytes: int = 256 << 20, n_streams: int = 4,
                 max_batch_requests: int = 1024, max_wait_us: float = 0.0, use_graphs: bool = True,
                 per_request: bool = False, executor: int = EXEC_DEVICE, fail_group: int = 0,
                 max_group_bytes: int = 0):
        cfg = ServerConfigC(int(device), int(arena_bytes), int(n_streams), int(max_batch_requests),
                            float(max_wait_us), int(bool(use_graphs)), int(bool(per_request)), int(executor),
                            int(fail_group), int(max_group_bytes))
        self._h = C.c_void_p()
        check(lib().rbd_server_create(C.byref(cfg), C.byref(self._h)))
        self._live = {}

    def submit(self, model: Model, op: int, inputs: Sequence[np.ndarray], outputs=None):
        """Queue one request; returns (ticket, outputs) with outputs filled once waited. outputs: optional
        C-contiguous float32 arrays [batch, rows] to write the results into, else new ones."""
        in_rows, out_rows = op_shapes(model, op)
        if len(inputs) != len(in_rows):
            raise ValueError(f"op {op} takes {len(in_rows)} inputs")
        batch = int(inputs[0].shape[0])
        ins = []
        for x, r in zip(inputs, in_rows):
            x = np.ascontiguousarray(x, dtype=np.float32)
            if x.shape != (batch, r):
                raise ValueError(f"input of shape {x.shape}, expected {(batch, r)}")
            ins.append(x)
        if outputs is None:
            outs = [np.empty((batch, r), dtype=np.float32) for r in out_rows]
        else:
            outs = list(outputs)
            if len(outs) != len(out_rows) or any(
                    o.dtype != np.float32 or o.shape != (batch, r) or not o.flags.c_contiguous
                    for o, r in zip(outs, out_rows)):
                raise ValueError("outputs do not match the operation")
        pin = (C.c_void_p * 4)(*[C.c_void_p(x.ctypes.data) for x in ins] + [None] * (4 - len(ins)))
        pout = (C.c_void_p * 3)(*[C.c_void_p(x.ctypes.data) for x in outs] + [None] * (3 - len(outs)))
        t = C.c_uint64()
        check(lib().rbd_server_submit(self._h, model.handle, int(op), batch, pin, pout, C.byref(t)))
        self._live[t.value] = (ins, outs)
        return t.value, outs

    def wait(self, ticket: int, timeout: float = -1.0) -> int:
        st = C.c_int()
        check(lib().rbd_server_wait(self._h, C.c_uint64(ticket), float(timeout), C.byref(st)))
        self._live.pop(ticket, None)
        return st.value

    def cancel(self, ticket: int) -> None:
        """Cancel a request still in the queue (it then completes with RBD_E_CANCELLED)."""
        check(lib().rbd_server_cancel(self._h, C.c_uint64(ticket)))

    def load(self, requests, n_requests: int, rate: float = 0.0, window: int = 1024, seed: int = 0):
        """Native open-loop load (rbd_diag_serve_load): request j is requests[j % len(requests)], each a
        (model, op, inputs) triple of instance-major float32 arrays; Poisson arrivals at `rate` per second
        (0: closed loop). Returns (wall seconds, failed requests)."""
        keep, spec = [], (LoadRequestC * len(requests))()
        for k, (model, op, inputs) in enumerate(requests):
            in_rows, _ = op_shapes(model, op)
            batch = int(inputs[0].shape[0])
            xs = [np.ascontiguousarray(x, dtype=np.float32) for x in inputs]
            if len(xs) != len(in_rows) or any(x.shape != (batch, r) for x, r in zip(xs, in_rows)):
                raise ValueError(f"request {k}: inputs do not match op {op}")
            keep.append(xs)
            spec[k].model, spec[k].op, spec[k].batch = model.handle.value, int(op), batch
            for a, x in enumerate(xs):
                spec[k].inp[a] = x.ctypes.data
        wall, failed = C.c_double(), C.c_int64()
        check(lib().rbd_diag_serve_load(self._h, len(requests), spec, int(n_requests), float(rate), int(window),
                                        int(seed), C.byref(wall), C.byref(failed)))
        return wall.value, failed.value

    def stats(self) -> dict:
        s = ServerStatsC()
        check(lib().rbd_server_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStatsC._fields_}

    def reset_stats(self) -> None:
        check(lib().rbd_server_reset_stats(self._h))

    def close(self) -> None:
        if self._h:
            lib().rbd_server_destroy(self._h)
            self._h = C.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

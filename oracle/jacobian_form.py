"""Inverse dynamics and the mass matrix from body Jacobians, in the world frame.

TEST INFRASTRUCTURE ONLY (see the package docstring).

An independent formulation of the quantities Eq. (1) defines (and Alg. 1 and
Alg. 2 compute): every body's motion is written through its centre-of-mass
Jacobians, and the generalised forces follow from Kane's equations (the
virtual-power form of Newton-Euler), with the partial velocities J as the
generalised-speed derivatives:

    tau = sum_i J_v,i^T m_i (a_c,i - g) + J_w,i^T (I_i alpha_i + w_i x I_i w_i)
    M   = sum_i m_i J_v,i^T J_v,i + J_w,i^T I_i J_w,i

with v_c,i = J_v,i qd, w_i = J_w,i qd, a_c,i = J_v,i qdd + Jdot_v,i qd and
alpha_i = J_w,i qdd + Jdot_w,i qd; I_i is body i's inertia about its centre of
mass in world axes. Jdot qd comes from the motion itself: a world joint axis z
turns as w x z, and a lever arm changes by the difference of two point
velocities. A free base uses the body-frame twist [v_B; w_B] as its
generalised speeds (Kane's equations hold for any generalised speeds), so its
generalised force is the body-frame wrench. Nothing here is shared with
rbd_oracle.cpp (recursive, body frames, spatial algebra): the forward
kinematics are written again, and agreement between the two is a real check.
Gravity enters as the force m_i g on each centre of mass, so tau contains the
holding torque +g(q). No external forces.
"""
from __future__ import annotations

import numpy as np

FREE = 1


def _rodrigues(a, q):
    """Rotation about the unit axis a [3] by angles q [B] -> [B, 3, 3]."""
    a = np.asarray(a, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    c, s = np.cos(q)[:, None, None], np.sin(q)[:, None, None]
    return c * np.eye(3) + s * K + (1.0 - c) * np.outer(a, a)


def _quat(qv):
    """Hamilton rotation of [B, 4] (w, x, y, z) divided by the squared norm."""
    w, x, y, z = (qv[:, k] for k in range(4))
    s = w * w + x * x + y * y + z * z
    R = np.stack([
        np.stack([w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z], -1),
    ], -2)
    return R / s[:, None, None]


def _ancestors(desc, i):
    """Body i and its ancestors, root last."""
    out = []
    while i >= 0:
        out.append(i)
        i = int(desc.parent[i])
    return out


def _kinematics(desc, q):
    """World rotation [B, n, 3, 3], origin [B, n, 3], joint axis in world axes [B, n, 3] (revolute)."""
    B, n = q.shape[0], desc.n_bodies
    Rw, pw, zw = np.zeros((B, n, 3, 3)), np.zeros((B, n, 3)), np.zeros((B, n, 3))
    k = 0
    for i in range(n):
        l = int(desc.parent[i])
        if desc.joint_type[i] == FREE:
            Rw[:, i], pw[:, i] = _quat(q[:, k + 3:k + 7]), q[:, k:k + 3]
            k += 7
            continue
        Rf = np.asarray(desc.origin[i, :9], dtype=np.float64).reshape(3, 3)
        off = np.asarray(desc.origin[i, 9:12], dtype=np.float64)
        Rp = np.broadcast_to(np.eye(3), (B, 3, 3)) if l < 0 else Rw[:, l]
        pp = np.zeros((B, 3)) if l < 0 else pw[:, l]
        Rw[:, i] = Rp @ Rf @ _rodrigues(desc.axis[i], q[:, k])
        pw[:, i] = pp + np.einsum("bij,j->bi", Rp, off)
        a = np.asarray(desc.axis[i], dtype=np.float64)
        zw[:, i] = np.einsum("bij,j->bi", Rw[:, i], a / np.linalg.norm(a))
        k += 1
    return Rw, pw, zw


def _columns(desc, Rw, pw, zw, point, i):
    """Linear [B, 3, nv] and angular [B, 3, nv] Jacobian of a point [B, 3] fixed to body i."""
    B = point.shape[0]
    nv = desc.nv
    Jv, Jw = np.zeros((B, 3, nv)), np.zeros((B, 3, nv))
    v = 0
    vofs = []
    for j in range(desc.n_bodies):
        vofs.append(v)
        v += 6 if desc.joint_type[j] == FREE else 1
    for j in _ancestors(desc, i):
        c = vofs[j]
        if desc.joint_type[j] == FREE:
            for a in range(3):
                e = Rw[:, j, :, a]                       # base axis a in world axes
                Jv[:, :, c + a] = e                      # v_B component a
                Jv[:, :, c + 3 + a] = np.cross(e, point - pw[:, j])  # w_B component a
                Jw[:, :, c + 3 + a] = e
        else:
            Jv[:, :, c] = np.cross(zw[:, j], point - pw[:, j])
            Jw[:, :, c] = zw[:, j]
    return Jv, Jw


def _com_and_inertia(desc, Rw, pw, i):
    m = float(desc.mass[i])
    com = pw[:, i] + np.einsum("bij,j->bi", Rw[:, i], np.asarray(desc.com[i], dtype=np.float64))
    J = np.asarray(desc.inertia[i], dtype=np.float64)
    Ib = np.array([[J[0], J[3], J[4]], [J[3], J[1], J[5]], [J[4], J[5], J[2]]])
    return m, com, Rw[:, i] @ Ib @ np.swapaxes(Rw[:, i], -1, -2)


def mass_matrix(desc, q):
    """M(q) = sum_i m_i J_v,i^T J_v,i + J_w,i^T I_i J_w,i, [B, nv, nv]."""
    q = np.asarray(q, dtype=np.float64)
    Rw, pw, zw = _kinematics(desc, q)
    M = np.zeros((q.shape[0], desc.nv, desc.nv))
    for i in range(desc.n_bodies):
        m, com, Iw = _com_and_inertia(desc, Rw, pw, i)
        Jv, Jw = _columns(desc, Rw, pw, zw, com, i)
        M += m * np.swapaxes(Jv, 1, 2) @ Jv + np.swapaxes(Jw, 1, 2) @ Iw @ Jw
    return M


def inverse_dynamics(desc, q, qd, qdd=None):
    """tau(q, qd, qdd) by Kane's equations, [B, nv]; qdd None gives the bias force h(q, qd)."""
    q, qd = np.asarray(q, dtype=np.float64), np.asarray(qd, dtype=np.float64)
    qdd = np.zeros_like(qd) if qdd is None else np.asarray(qdd, dtype=np.float64)
    B, n = q.shape[0], desc.n_bodies
    Rw, pw, zw = _kinematics(desc, q)
    g = np.asarray(desc.gravity, dtype=np.float64)
    # angular velocity and origin velocity of every body, from its own Jacobians
    w, vo = np.zeros((B, n, 3)), np.zeros((B, n, 3))
    for i in range(n):
        Jv, Jw = _columns(desc, Rw, pw, zw, pw[:, i], i)
        vo[:, i] = np.einsum("bij,bj->bi", Jv, qd)
        w[:, i] = np.einsum("bij,bj->bi", Jw, qd)
    tau = np.zeros((B, desc.nv))
    vofs, v = [], 0
    for j in range(n):
        vofs.append(v)
        v += 6 if desc.joint_type[j] == FREE else 1
    for i in range(n):
        m, com, Iw = _com_and_inertia(desc, Rw, pw, i)
        Jv, Jw = _columns(desc, Rw, pw, zw, com, i)
        vc = np.einsum("bij,bj->bi", Jv, qd)
        # Jdot qd: d/dt of each column, times that column's speed
        jv_dot, jw_dot = np.zeros((B, 3)), np.zeros((B, 3))
        for j in _ancestors(desc, i):
            c = vofs[j]
            if desc.joint_type[j] == FREE:
                for a in range(3):
                    e = Rw[:, j, :, a]
                    e_dot = np.cross(w[:, j], e)
                    lever, lever_dot = com - pw[:, j], vc - vo[:, j]
                    jv_dot += qd[:, c + a, None] * e_dot
                    jv_dot += qd[:, c + 3 + a, None] * (np.cross(e_dot, lever) + np.cross(e, lever_dot))
                    jw_dot += qd[:, c + 3 + a, None] * e_dot
            else:
                z_dot = np.cross(w[:, j], zw[:, j])
                jv_dot += qd[:, c, None] * (np.cross(z_dot, com - pw[:, j]) + np.cross(zw[:, j], vc - vo[:, j]))
                jw_dot += qd[:, c, None] * z_dot
        ac = np.einsum("bij,bj->bi", Jv, qdd) + jv_dot
        alpha = np.einsum("bij,bj->bi", Jw, qdd) + jw_dot
        wi = w[:, i]
        force = m * (ac - g)
        moment = np.einsum("bij,bj->bi", Iw, alpha) + np.cross(wi, np.einsum("bij,bj->bi", Iw, wi))
        tau += np.einsum("bij,bi->bj", Jv, force) + np.einsum("bij,bi->bj", Jw, moment)
    return tau

"""Controller-shaped workloads on top of the FP64 oracle (test infrastructure only).

The paper times differential IK and operational-space control (Sec. IV, Sec. V,
Table II) on real robots with QP-based variants; these are the plain textbook
forms of the two, for one end-effector frame e, written out step by step with
the oracle's own kinematics and dynamics and numpy's dense solves:

  pose error   err = [p* - p_e; 1/2 sum_k R_e[:, k] x R*[:, k]]   (world axes)
  diff_ik      qd = J^T (J J^T + lam^2 I)^-1 (k err)       (damped least squares)
  osc          a* = kp err - kd J qd
               Lambda = (J M^-1 J^T)^-1,  tau_null = -k_null qd
               tau = J^T Lambda (a* - J M^-1 tau_null) + tau_null + h(q, qd)

J is the world-aligned Jacobian of frame e at its origin (rows [v; w]), M and h
the mass matrix and bias force (gravity included). OSC omits the Jdot qd term,
so the task acceleration it commands is J qdd = a* exactly.
"""
from __future__ import annotations

import numpy as np

from . import crba, fk, jacobian, rnea


def pose_error(desc, q, frame, target):
    """err [B, 6] of frame `frame` against target [B, 3, 4] = [R* | p*]."""
    T = fk(desc, q)[:, frame]
    R, p = T[:, :, :3], T[:, :, 3]
    Rs, ps = target[:, :, :3], target[:, :, 3]
    rot = 0.5 * np.cross(np.swapaxes(R, 1, 2), np.swapaxes(Rs, 1, 2)).sum(axis=1)
    return np.concatenate([ps - p, rot], axis=1)


def diff_ik(desc, q, frame, target, gain, damping):
    """Damped least-squares joint velocity [B, nv]."""
    err = pose_error(desc, q, frame, target)
    J = jacobian(desc, q, [frame])[:, 0]
    A = J @ np.swapaxes(J, 1, 2) + damping ** 2 * np.eye(6)
    w = np.linalg.solve(A, gain * err[..., None])
    return (np.swapaxes(J, 1, 2) @ w)[..., 0]


def osc(desc, q, qd, frame, target, kp, kd, k_null):
    """Operational-space control torques [B, nv]."""
    err = pose_error(desc, q, frame, target)
    J = jacobian(desc, q, [frame])[:, 0]
    Jt = np.swapaxes(J, 1, 2)
    a_star = kp * err - kd * (J @ qd[..., None])[..., 0]
    M = crba(desc, q)
    h = rnea(desc, q, qd)
    Minv_Jt = np.linalg.solve(M, Jt)
    Lam = np.linalg.inv(J @ Minv_Jt)
    tau_null = -k_null * qd
    JMinv_tn = (J @ np.linalg.solve(M, tau_null[..., None]))[..., 0]
    F = (Lam @ (a_star - JMinv_tn)[..., None])[..., 0]
    return (Jt @ F[..., None])[..., 0] + tau_null + h

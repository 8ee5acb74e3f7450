"""Test-only helpers that sit beside the oracle (no dynamics arithmetic of its own)."""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation


def quat_mul(a, b):
    """Hamilton product of (w, x, y, z) quaternions, [..., 4]."""
    w1, x1, y1, z1 = np.moveaxis(a, -1, 0)
    w2, x2, y2, z2 = np.moveaxis(b, -1, 0)
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], -1)


def base_rotation(quat):
    """Rotation of (w, x, y, z) quaternions via scipy (x, y, z, w order), [B, 3, 3]."""
    return Rotation.from_quat(np.roll(quat, -1, axis=-1)).as_matrix()


def retract(desc, q, dq, eps):
    """q (+) eps*dq for generalised velocity dq: exact for revolute joints, and the
    first-order body-twist update (p += eps R v, quat <- quat (x) [1, eps w / 2])
    for a free base. Any first-order retraction makes central differences exact to
    O(eps^2)."""
    q = np.array(q, dtype=np.float64, copy=True)
    if desc.floating:
        R = base_rotation(q[:, 3:7] / np.linalg.norm(q[:, 3:7], axis=1, keepdims=True))
        q[:, 0:3] += eps * np.einsum("bij,bj->bi", R, dq[:, 0:3])
        dqt = np.concatenate([np.ones((q.shape[0], 1)), 0.5 * eps * dq[:, 3:6]], axis=1)
        q[:, 3:7] = quat_mul(q[:, 3:7], dqt)
        q[:, 7:] += eps * dq[:, 6:]
    else:
        q += eps * dq
    return q


def com_world(desc, T):
    """CoM positions [B, n, 3] from FK poses T [B, n, 3, 4]."""
    return T[..., :, 3] + np.einsum("bnij,nj->bni", T[..., :, :3], desc.com)


def inertia_matrix(desc, i):
    J = desc.inertia[i]
    return np.array([[J[0], J[3], J[4]], [J[3], J[1], J[5]], [J[4], J[5], J[2]]])


def rel_err(x, ref, axis=None):
    """max over instances of ||x - ref||_inf / ||ref||_inf (normwise, per instance)."""
    x = np.asarray(x, dtype=np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(ref), -1)
    num = np.abs(x - ref).max(axis=1)
    den = np.abs(ref).max(axis=1)
    return float((num / np.maximum(den, 1e-300)).max())


def vjp_err(got, ref, floor=1e-4):
    """Max over instances and over the blocks (g_q, g_qd, g_tau) of
    ||x_b - ref_b||_inf / max(||ref_b||_inf, floor * ||ref||_inf): a block whose true
    value vanishes (a single pendulum has no velocity dependence) is held to an
    absolute bar set by the scale of the whole gradient, not to its FD noise."""
    B = len(ref[0])
    flat = [np.asarray(r, dtype=np.float64).reshape(B, -1) for r in ref]
    scale = np.max([np.abs(r).max(axis=1) for r in flat], axis=0)
    worst = 0.0
    for x, r in zip(got, flat):
        x = np.asarray(x, dtype=np.float64).reshape(B, -1)
        den = np.maximum(np.abs(r).max(axis=1), floor * scale)
        worst = max(worst, float((np.abs(x - r).max(axis=1) / den).max()))
    return worst


def targets_near(T, seed, scale=0.2):
    """Target poses [B, 3, 4] near the frame poses T [B, 3, 4]: a random rotation of standard
    deviation `scale` rad applied in world axes and a random offset of `scale` m."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dR = Rotation.from_rotvec(rng.normal(0, scale, size=(len(T), 3))).as_matrix()
    out = np.empty_like(T)
    out[:, :, :3] = dR @ T[:, :, :3]
    out[:, :, 3] = T[:, :, 3] + rng.normal(0, scale, size=(len(T), 3))
    return out

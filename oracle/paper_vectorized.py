"""The paper's vectorised RNEA (Alg. 1) and CRBA (Alg. 2), restated with NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything is expressed in the root (world) frame, as in Alg. 1 and Alg. 2,
with dense 6x6 spatial matrices in [angular; linear] order and the ancestor
mask U of Sec. III (U[i, j] = 1 iff body j is an ancestor of body i, a body
being its own ancestor; lower triangular for parent[i] < i). The forward
kinematics loop (the one loop the method keeps, Sec. III-A) is written here
independently of rbd_oracle.cpp, so that agreement between the two is a real
cross-check. A multi-DoF joint (the free base) contributes a 6 x k block of
spatial axes; Alg. 1 and Alg. 2 then act on blocks exactly as on columns.

Readings: the gravity term a_g of Alg. 1 is -g (a fictitious upward base
acceleration), so Gamma contains +g(q); Symmetrize(M_lower) is
M_lower + M_lower^T minus the diagonal blocks; external forces are zero.
"""
from __future__ import annotations

import numpy as np

FREE = 1


def _skew(v):
    """[v]x for v [..., 3] -> [..., 3, 3]."""
    z = np.zeros(v.shape[:-1])
    return np.stack([
        np.stack([z, -v[..., 2], v[..., 1]], -1),
        np.stack([v[..., 2], z, -v[..., 0]], -1),
        np.stack([-v[..., 1], v[..., 0], z], -1),
    ], -2)


def _rodrigues(a, q):
    """Rotation about unit axis a [3] by angles q [B] -> [B, 3, 3]."""
    a = np.asarray(a, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = _skew(a)
    c, s = np.cos(q)[:, None, None], np.sin(q)[:, None, None]
    return c * np.eye(3) + s * K + (1 - c) * np.outer(a, a)


def _quat(qv):
    """Normalised Hamilton rotation of [B, 4] (w, x, y, z) quaternions."""
    w, x, y, z = (qv[:, k] for k in range(4))
    s = w * w + x * x + y * y + z * z
    R = np.stack([
        np.stack([w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z], -1),
    ], -2)
    return R / s[:, None, None]


def _crm(v):
    """Motion cross-product matrix v x for v [..., 6] = [w; v]."""
    out = np.zeros(v.shape[:-1] + (6, 6))
    W, V = _skew(v[..., :3]), _skew(v[..., 3:])
    out[..., :3, :3] = W
    out[..., 3:, :3] = V
    out[..., 3:, 3:] = W
    return out


def _crf(v):
    """Force cross-product matrix v x* = -(v x)^T."""
    return -np.swapaxes(_crm(v), -1, -2)


def _motion_to_world(R, p):
    """0_X_i^{-1}: motion in body coordinates -> world coordinates, [B, 6, 6].

    R holds the body axes in world coordinates and p the body origin.
    """
    X = np.zeros(R.shape[:-2] + (6, 6))
    X[..., :3, :3] = R
    X[..., 3:, 3:] = R
    X[..., 3:, :3] = _skew(p) @ R
    return X


def structure(desc):
    """Ancestor mask U, DoF-to-body map and DoF offsets."""
    n = desc.n_bodies
    U = np.zeros((n, n))
    for i in range(n):
        j = i
        while j >= 0:
            U[i, j] = 1.0
            j = int(desc.parent[j])
    nvi = [6 if desc.joint_type[i] == FREE else 1 for i in range(n)]
    body_of = np.concatenate([[i] * nvi[i] for i in range(n)]).astype(int)
    return U, body_of, nvi


def forward_kinematics(desc, q):
    """The FK loop: world rotation [B, n, 3, 3] and origin [B, n, 3] of every body."""
    B, n = q.shape[0], desc.n_bodies
    Rw = np.zeros((B, n, 3, 3))
    pw = np.zeros((B, n, 3))
    qo = 0
    for i in range(n):
        if desc.joint_type[i] == FREE:
            R = _quat(q[:, qo + 3:qo + 7])
            p = q[:, qo:qo + 3]
            qo += 7
        else:
            Rf = np.asarray(desc.origin[i, :9]).reshape(3, 3)
            R = Rf @ _rodrigues(desc.axis[i], q[:, qo])
            p = np.broadcast_to(np.asarray(desc.origin[i, 9:12]), (B, 3))
            qo += 1
        l = int(desc.parent[i])
        if l < 0:
            Rw[:, i], pw[:, i] = R, p
        else:
            Rw[:, i] = Rw[:, l] @ R
            pw[:, i] = pw[:, l] + np.einsum("bij,bj->bi", Rw[:, l], p)
    return Rw, pw


def prepare(desc, q):
    """Root-frame spatial axes 0S [B, nv, 6] and inertias 0I [B, n, 6, 6]."""
    B, n = q.shape[0], desc.n_bodies
    Rw, pw = forward_kinematics(desc, q)
    Xw = _motion_to_world(Rw, pw)                  # body -> world for motion
    S_cols = []
    for i in range(n):
        if desc.joint_type[i] == FREE:
            Sb = np.zeros((6, 6))
            Sb[3:, 0:3] = np.eye(3)                # qd = [v_B; w_B]
            Sb[:3, 3:6] = np.eye(3)
        else:
            a = np.asarray(desc.axis[i], dtype=np.float64)
            Sb = np.concatenate([a / np.linalg.norm(a), np.zeros(3)])[:, None]
        S_cols.append(np.einsum("bij,jk->bki", Xw[:, i], Sb))
    S = np.concatenate(S_cols, axis=1)
    Iw = np.zeros((B, n, 6, 6))
    for i in range(n):
        m = float(desc.mass[i])
        c = np.asarray(desc.com[i], dtype=np.float64)
        J = np.asarray(desc.inertia[i], dtype=np.float64)
        Ic = np.array([[J[0], J[3], J[4]], [J[3], J[1], J[5]], [J[4], J[5], J[2]]])
        C = _skew(c)
        Ib = np.zeros((6, 6))                      # about the body origin, body coordinates
        Ib[:3, :3] = Ic + m * C @ C.T
        Ib[:3, 3:] = m * C
        Ib[3:, :3] = m * C.T
        Ib[3:, 3:] = m * np.eye(3)
        Xinv = np.linalg.inv(Xw[:, i])             # world -> body for motion
        Iw[:, i] = np.swapaxes(Xinv, -1, -2) @ Ib @ Xinv
    return S, Iw


def rnea(desc, q, qd, qdd=None):
    """Alg. 1: V = U(S qd), A = a_g + U(S qdd + V x S qd), F = U^T(I A + V x* I V), Gamma = S . F."""
    q, qd = np.asarray(q, np.float64), np.asarray(qd, np.float64)
    qdd = np.zeros_like(qd) if qdd is None else np.asarray(qdd, np.float64)
    U, body_of, _ = structure(desc)
    S, I = prepare(desc, q)
    n = desc.n_bodies
    Sqd = np.zeros((q.shape[0], n, 6))
    Sqdd = np.zeros((q.shape[0], n, 6))
    np.add.at(Sqd, (slice(None), body_of), S * qd[:, :, None])
    np.add.at(Sqdd, (slice(None), body_of), S * qdd[:, :, None])
    V = np.einsum("ij,bjx->bix", U, Sqd)
    a_g = np.zeros(6)
    a_g[3:] = -np.asarray(desc.gravity, dtype=np.float64)
    A = a_g + np.einsum("ij,bjx->bix", U, Sqdd + np.einsum("bjxy,bjy->bjx", _crm(V), Sqd))
    IV = np.einsum("bixy,biy->bix", I, V)
    local = np.einsum("bixy,biy->bix", I, A) + np.einsum("bixy,biy->bix", _crf(V), IV)
    F = np.einsum("ji,bjx->bix", U, local)         # U^T: sum over descendants
    return np.einsum("bkx,bkx->bk", S, F[:, body_of])


def crba(desc, q):
    """Alg. 2: C = U^T I, M_lower = U (.) (S_i^T C_i S_j), M = Symmetrize(M_lower)."""
    q = np.asarray(q, np.float64)
    U, body_of, _ = structure(desc)
    S, I = prepare(desc, q)
    C = np.einsum("ji,bjxy->bixy", U, I)
    mask = U[body_of][:, body_of]                  # DoF k, l with body(l) an ancestor of body(k)
    same = (body_of[:, None] == body_of[None, :]).astype(float)
    CS = np.einsum("bkxy,bly->bklx", C[:, body_of], S)          # C_{body(k)} S_l
    M_lower = mask * np.einsum("bkx,bklx->bkl", S, CS)
    return M_lower + np.swapaxes(M_lower, -1, -2) - same * M_lower

"""Brute-force Euler-Lagrange dynamics of small fixed-base chains with sympy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a chain of revolute joints this builds the Lagrangian L = T - V directly
from the kinematics (CoM positions and body rotations as exact functions of
q), with T = sum 1/2 m |dc/dt|^2 + 1/2 w^T (R Ibar_c R^T) w, where [w]x is
(dR/dt) R^T, and V = -sum m g . c, and differentiates it symbolically:

    M(q) = d^2 T / dqd^2,
    h(q, qd) = sum_k d/dq_k (dL/dqd) qd_k - dL/dq,

so that tau = M qdd + h is Eq. (1) of the paper with f = 0. Nothing here uses
spatial algebra, so it pins the recursive and vectorised forms independently.

Every quantity is a polynomial in c_k = cos q_k, s_k = sin q_k and qd_k with
float coefficients, held in a sparse polynomial ring, and d/dq_k acts through
the chain rule d/dq_k = -s_k d/dc_k + c_k d/ds_k.
"""
from __future__ import annotations

import numpy as np
from sympy import RR
from sympy.polys.rings import ring


def chain_dynamics(desc):
    """Return (M_fn, h_fn): numeric callables of (q, qd) for a fixed-base chain."""
    n = desc.n_bodies
    assert all(desc.parent[i] == i - 1 for i in range(n)), "chains only"
    assert all(desc.joint_type[i] == 0 for i in range(n)), "revolute joints only"
    names = [f"c{k}" for k in range(n)] + [f"s{k}" for k in range(n)] + [f"qd{k}" for k in range(n)]
    P, *gens = ring(",".join(names), RR)
    c, s, qd = gens[:n], gens[n:2 * n], gens[2 * n:]
    zero = P(0)

    def ddq(f, k):
        return -s[k] * f.diff(c[k]) + c[k] * f.diff(s[k])

    def matmul(A, B):
        return [[sum((A[i][k] * B[k][j] for k in range(len(B))), zero) for j in range(len(B[0]))]
                for i in range(len(A))]

    def const(M):
        M = np.asarray(M, dtype=np.float64)
        return [[P(float(x)) for x in row] for row in M]

    def rot(axis, k):
        a = np.asarray(axis, dtype=np.float64)
        a = a / np.linalg.norm(a)
        K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        A = np.outer(a, a)
        I3 = np.eye(3)
        return [[c[k] * float(I3[i, j] - A[i, j]) + s[k] * float(K[i, j]) + float(A[i, j]) for j in range(3)]
                for i in range(3)]

    g = [float(x) for x in desc.gravity]
    R = const(np.eye(3))
    p = [[zero] for _ in range(3)]
    T = zero
    V = zero
    for i in range(n):
        Rf = const(np.asarray(desc.origin[i, :9]).reshape(3, 3))
        off = const(np.asarray(desc.origin[i, 9:12]).reshape(3, 1))
        Roff = matmul(R, off)
        p = [[p[r][0] + Roff[r][0]] for r in range(3)]
        R = matmul(matmul(R, Rf), rot(desc.axis[i], i))
        Rc = matmul(R, const(np.asarray(desc.com[i]).reshape(3, 1)))
        com = [p[r][0] + Rc[r][0] for r in range(3)]
        m = float(desc.mass[i])
        J = np.asarray(desc.inertia[i], dtype=np.float64)
        Ic = const([[J[0], J[3], J[4]], [J[3], J[1], J[5]], [J[4], J[5], J[2]]])
        cdot = [sum((ddq(com[r], k) * qd[k] for k in range(i + 1)), zero) for r in range(3)]
        Rdot = [[sum((ddq(R[a][b], k) * qd[k] for k in range(i + 1)), zero) for b in range(3)] for a in range(3)]
        RT = [[R[b][a] for b in range(3)] for a in range(3)]
        W = matmul(Rdot, RT)                        # [w]x in world coordinates
        w = [W[2][1], W[0][2], W[1][0]]
        Iw = matmul(matmul(R, Ic), RT)
        Iww = [sum((Iw[a][b] * w[b] for b in range(3)), zero) for a in range(3)]
        T = T + 0.5 * m * sum((cdot[r] * cdot[r] for r in range(3)), zero) \
              + 0.5 * sum((w[a] * Iww[a] for a in range(3)), zero)
        V = V - m * sum((g[r] * com[r] for r in range(3)), zero)
    L = T - V
    Mx = [[T.diff(qd[a]).diff(qd[b]) for b in range(n)] for a in range(n)]
    dLdqd = [L.diff(qd[a]) for a in range(n)]
    h = [sum((ddq(dLdqd[a], k) * qd[k] for k in range(n)), zero) - ddq(L, a) for a in range(n)]

    def ev(poly, qv, qdv):
        x = [float(v) for v in np.cos(qv)] + [float(v) for v in np.sin(qv)] + [float(v) for v in qdv]
        return float(poly(*x)) if len(x) > 1 else float(poly(x[0]))

    def M_num(qv, qdv):
        return np.array([[ev(Mx[a][b], qv, qdv) for b in range(n)] for a in range(n)])

    def h_num(qv, qdv):
        return np.array([ev(h[a], qv, qdv) for a in range(n)])

    return M_num, h_num

"""Pins for the FP64 oracle: closed forms, textbook cases, invariants and brute force.

None of these re-types the oracle's own formulas: each compares it with an
independent statement of the same physics (a closed form, scipy's rotations,
the textbook double pendulum, energy and power identities, finite differences
of kinematics, or a different algorithm).
"""
from __future__ import annotations

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
import workloads as W
from oracle import euler_lagrange as EL
from oracle import jacobian_form as JF
from tests._helpers import base_rotation, com_world, inertia_matrix, rel_err, retract

G = 9.81


def _single_body(seed, floating=False, com_zero=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    d = W.random_tree([-1], floating, seed)
    d.origin[0, :9] = Rotation.random(random_state=seed).as_matrix().reshape(-1)
    if com_zero:
        d.com[0] = 0.0
    return d, rng


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_single_pendulum_closed_form(seed):
    """One revolute joint: M = a^T Ic a + m |a x c|^2, h = g(q) = dV/dq, qdd = (tau - g)/M."""
    d, rng = _single_body(seed)
    a = d.axis[0] / np.linalg.norm(d.axis[0])
    c, m = d.com[0], d.mass[0]
    Ic = inertia_matrix(d, 0)
    Rf = d.origin[0, :9].reshape(3, 3)
    B = 16
    q = rng.uniform(-np.pi, np.pi, size=(B, 1))
    qd = rng.normal(size=(B, 1))
    tau = rng.normal(0, 5, size=(B, 1))
    M_ref = a @ Ic @ a + m * np.dot(np.cross(a, c), np.cross(a, c))
    Rq = Rotation.from_rotvec(a[None, :] * q).as_matrix()
    lever = np.einsum("bij,j->bi", Rq, c)
    dVdq = -m * np.einsum("i,ij,bj->b", d.gravity, Rf, np.cross(a[None, :], lever))
    assert np.allclose(O.crba(d, q)[:, 0, 0], M_ref, rtol=1e-13, atol=0)
    assert np.allclose(O.rnea(d, q, qd)[:, 0], dVdq, rtol=1e-12, atol=1e-13)
    for method in (O.METHOD_LLT, O.METHOD_LTL, O.METHOD_ABA):
        qdd = O.fwd_dyn(d, q, qd, tau, method)
        assert np.allclose(qdd[:, 0], (tau[:, 0] - dVdq) / M_ref, rtol=1e-12, atol=1e-13)


def _spong_double_pendulum(m1, m2, l1, lc1, lc2, I1, I2):
    parent = np.array([-1, 0], dtype=np.int32)
    d = W.TreeDesc(
        parent=parent, joint_type=np.zeros(2, dtype=np.int32),
        axis=np.array([[0.0, 0, 1], [0, 0, 1]]),
        origin=np.array([[1.0, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], [1.0, 0, 0, 0, 1, 0, 0, 0, 1, l1, 0, 0]]),
        mass=np.array([m1, m2]), com=np.array([[lc1, 0, 0], [lc2, 0, 0]]),
        inertia=np.array([[0.7 * I1, 0.9 * I1, I1, 0, 0, 0], [0.6 * I2, 0.8 * I2, I2, 0, 0, 0]]),
        gravity=np.array([0.0, -G, 0.0]), name="spong")
    return d


def test_planar_double_pendulum_textbook():
    """Spong, Robot Modeling and Control, planar elbow manipulator: M, C, g in closed form."""
    m1, m2, l1, lc1, lc2, I1, I2 = 1.3, 0.8, 0.9, 0.4, 0.35, 0.11, 0.07
    d = _spong_double_pendulum(m1, m2, l1, lc1, lc2, I1, I2)
    rng = np.random.Generator(np.random.PCG64(7))
    B = 32
    q = rng.uniform(-np.pi, np.pi, size=(B, 2))
    qd = rng.normal(size=(B, 2))
    qdd = rng.normal(size=(B, 2))
    c2 = np.cos(q[:, 1])
    d11 = m1 * lc1 ** 2 + m2 * (l1 ** 2 + lc2 ** 2 + 2 * l1 * lc2 * c2) + I1 + I2
    d12 = m2 * (lc2 ** 2 + l1 * lc2 * c2) + I2
    d22 = np.full(B, m2 * lc2 ** 2 + I2)
    h = -m2 * l1 * lc2 * np.sin(q[:, 1])
    phi1 = (m1 * lc1 + m2 * l1) * G * np.cos(q[:, 0]) + m2 * lc2 * G * np.cos(q[:, 0] + q[:, 1])
    phi2 = m2 * lc2 * G * np.cos(q[:, 0] + q[:, 1])
    tau1 = d11 * qdd[:, 0] + d12 * qdd[:, 1] + 2 * h * qd[:, 0] * qd[:, 1] + h * qd[:, 1] ** 2 + phi1
    tau2 = d12 * qdd[:, 0] + d22 * qdd[:, 1] - h * qd[:, 0] ** 2 + phi2
    M = O.crba(d, q)
    assert np.allclose(M[:, 0, 0], d11, rtol=1e-13) and np.allclose(M[:, 0, 1], d12, rtol=1e-13)
    assert np.allclose(M[:, 1, 0], d12, rtol=1e-13) and np.allclose(M[:, 1, 1], d22, rtol=1e-13)
    tau = O.rnea(d, q, qd, qdd)
    assert np.allclose(tau, np.stack([tau1, tau2], 1), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_euler_lagrange_random_2link(seed):
    """Random 3-D 2-link chain: M and h from symbolic differentiation of the Lagrangian."""
    d = W.random_tree([-1, 0], False, seed)
    d.origin[1, :9] = Rotation.random(random_state=seed).as_matrix().reshape(-1)
    M_fn, h_fn = EL.chain_dynamics(d)
    st = W.states(d, 6, seed + 100)
    M = O.crba(d, st.q)
    h = O.rnea(d, st.q, st.qd)
    for b in range(6):
        assert np.allclose(M[b], M_fn(st.q[b], st.qd[b]), rtol=1e-12, atol=1e-14)
        assert np.allclose(h[b], h_fn(st.q[b], st.qd[b]), rtol=1e-11, atol=1e-13)


def test_free_body_newton_euler():
    """A free rigid body with its origin at the CoM obeys Newton and Euler in body axes."""
    d, rng = _single_body(21, floating=True, com_zero=True)
    B = 16
    st = W.states(d, B, 5)
    m = d.mass[0]
    Ic = inertia_matrix(d, 0)
    v, w = st.qd[:, 0:3], st.qd[:, 3:6]
    f, n = st.tau[:, 0:3], st.tau[:, 3:6]
    R = base_rotation(st.q[:, 3:7])
    g_body = np.einsum("bji,j->bi", R, d.gravity)
    vdot = f / m + g_body - np.cross(w, v)
    wdot = np.linalg.solve(Ic[None], (n - np.cross(w, np.einsum("ij,bj->bi", Ic, w)))[..., None])[..., 0]
    for method in (O.METHOD_LLT, O.METHOD_LTL, O.METHOD_ABA):
        qdd = O.fwd_dyn(d, st.q, st.qd, st.tau, method)
        assert rel_err(qdd, np.concatenate([vdot, wdot], 1)) < 1e-12


def test_free_body_mass_matrix_offset_com():
    """Body-twist mass matrix of a free body: [[m 1, m [c]x^T], [m [c]x, Ic + m [c]x [c]x^T]]."""
    d, _ = _single_body(22, floating=True)
    m, c = d.mass[0], d.com[0]
    C = np.array([[0, -c[2], c[1]], [c[2], 0, -c[0]], [-c[1], c[0], 0]])
    ref = np.block([[m * np.eye(3), m * C.T], [m * C, inertia_matrix(d, 0) + m * C @ C.T]])
    st = W.states(d, 4, 3)
    assert np.allclose(O.crba(d, st.q), ref[None], rtol=1e-13, atol=1e-15)


def test_tree_free_fall():
    """At rest with no torques the humanoid falls as one body: joints stay, base accel = R^T g."""
    d = W.humanoid()
    st = W.states(d, 32, 9)
    zero = np.zeros_like(st.qd)
    R = base_rotation(st.q[:, 3:7])
    ref = np.zeros_like(st.qd)
    ref[:, 0:3] = np.einsum("bji,j->bi", R, d.gravity)
    for method in (O.METHOD_LLT, O.METHOD_LTL, O.METHOD_ABA):
        qdd = O.fwd_dyn(d, st.q, zero, zero, method)
        assert np.abs(qdd - ref).max() < 1e-11


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_mass_matrix_symmetric_positive_definite(name):
    d = W.chain(7) if name == "chain7" else W.humanoid()
    st = W.states(d, 128, 1)
    M = O.crba(d, st.q)
    assert np.abs(M - np.swapaxes(M, 1, 2)).max() <= 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0
    np.linalg.cholesky(M)


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_kinetic_energy_from_kinematics(name):
    """1/2 qd^T M qd equals the kinetic energy of body velocities taken from FK alone."""
    d = W.chain(7) if name == "chain7" else W.humanoid()
    st = W.states(d, 16, 2)
    eps = 1e-6
    Tp = O.fk(d, retract(d, st.q, st.qd, eps))
    Tm = O.fk(d, retract(d, st.q, st.qd, -eps))
    T0 = O.fk(d, st.q)
    cdot = (com_world(d, Tp) - com_world(d, Tm)) / (2 * eps)
    Rdot = (Tp[..., :3] - Tm[..., :3]) / (2 * eps)
    Wx = np.einsum("bnij,bnkj->bnik", Rdot, T0[..., :3])
    w = np.stack([Wx[..., 2, 1], Wx[..., 0, 2], Wx[..., 1, 0]], -1)
    KE = 0.5 * np.einsum("n,bni,bni->b", d.mass, cdot, cdot)
    for i in range(d.n_bodies):
        Iw = np.einsum("bij,jk,blk->bil", T0[:, i, :, :3], inertia_matrix(d, i), T0[:, i, :, :3])
        KE += 0.5 * np.einsum("bi,bij,bj->b", w[:, i], Iw, w[:, i])
    M = O.crba(d, st.q)
    ke = 0.5 * np.einsum("bi,bij,bj->b", st.qd, M, st.qd)
    assert np.allclose(ke, KE, rtol=1e-7)


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_gravity_is_potential_gradient(name):
    """rnea(q, 0, 0) = dV/dq with V = -sum m g . c(q) (central differences along each DoF)."""
    d = W.chain(7) if name == "chain7" else W.humanoid()
    st = W.states(d, 8, 3)
    zero = np.zeros_like(st.qd)
    grav = O.rnea(d, st.q, zero)

    def V(q):
        return -np.einsum("n,bni,i->b", d.mass, com_world(d, O.fk(d, q)), d.gravity)

    eps = 1e-6
    num = np.zeros_like(grav)
    for k in range(d.nv):
        e = np.zeros_like(st.qd)
        e[:, k] = 1.0
        num[:, k] = (V(retract(d, st.q, e, eps)) - V(retract(d, st.q, e, -eps))) / (2 * eps)
    assert np.abs(num - grav).max() < 1e-6 * np.abs(grav).max()


def test_christoffel_skew_symmetry_fixed_base():
    """Fixed base: Mdot - 2C is skew, and C(q, qd) qd is the Coriolis/centrifugal force c."""
    d = W.chain(7)
    st = W.states(d, 6, 4)
    eps = 1e-5
    n = d.nv
    dM = np.zeros((6, n, n, n))                     # dM[b, k] = dM/dq_k
    for k in range(n):
        e = np.zeros_like(st.q)
        e[:, k] = eps
        dM[:, k] = (O.crba(d, st.q + e) - O.crba(d, st.q - e)) / (2 * eps)
    qd = st.qd
    Mdot = np.einsum("bkij,bk->bij", dM, qd)
    # C_ij = sum_k 1/2 (dM_ij/dq_k + dM_ik/dq_j - dM_jk/dq_i) qd_k
    Cm = 0.5 * (np.einsum("bkij,bk->bij", dM, qd) + np.einsum("bjik,bk->bij", dM, qd)
                - np.einsum("bijk,bk->bij", dM, qd))
    S = Mdot - 2 * Cm
    assert np.abs(S + np.swapaxes(S, 1, 2)).max() < 1e-7 * np.abs(Mdot).max()
    c = O.rnea(d, st.q, qd, gravity=False)
    assert np.abs(np.einsum("bij,bj->bi", Cm, qd) - c).max() < 1e-7 * np.abs(c).max()


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_power_balance(name):
    """qd^T Mdot qd = 2 qd^T c for any base (c without gravity; Mdot along the motion)."""
    d = W.chain(7) if name == "chain7" else W.humanoid()
    st = W.states(d, 8, 5)
    eps = 1e-6
    Mdot = (O.crba(d, retract(d, st.q, st.qd, eps)) - O.crba(d, retract(d, st.q, st.qd, -eps))) / (2 * eps)
    lhs = np.einsum("bi,bij,bj->b", st.qd, Mdot, st.qd)
    c = O.rnea(d, st.q, st.qd, gravity=False)
    rhs = 2 * np.einsum("bi,bi->b", st.qd, c)
    assert np.allclose(lhs, rhs, rtol=1e-6, atol=1e-7 * np.abs(rhs).max())


# ---------------------------------------------------------------- algorithms agree
@pytest.mark.parametrize("name", ["chain7", "humanoid30", "tree12"])
def test_forward_dynamics_round_trip_and_three_methods(name):
    d = {"chain7": W.chain(7), "humanoid30": W.humanoid(),
         "tree12": W.random_tree([-1, 0, 1, 1, 0, 4, 5, 5, 7, 0, 9, 10], True, 5)}[name]
    st = W.states(d, 64, 6)
    q_llt = O.fwd_dyn(d, st.q, st.qd, st.tau, O.METHOD_LLT)
    q_ltl = O.fwd_dyn(d, st.q, st.qd, st.tau, O.METHOD_LTL)
    q_aba = O.fwd_dyn(d, st.q, st.qd, st.tau, O.METHOD_ABA)
    assert rel_err(q_ltl, q_llt) < 1e-11 and rel_err(q_aba, q_llt) < 1e-11
    assert rel_err(O.rnea(d, st.q, st.qd, q_ltl), st.tau) < 1e-11
    M = O.crba(d, st.q)
    h = O.rnea(d, st.q, st.qd)
    ref = np.linalg.solve(M, (st.tau - h)[..., None])[..., 0]
    assert rel_err(q_ltl, ref) < 1e-11


@pytest.mark.parametrize("name", ["chain7", "humanoid30", "tree12", "humanoid30_rot"])
def test_jacobian_form_matches_recursive(name):
    """M and tau from body Jacobians and Kane's equations in the world frame (an independent
    formulation) agree with the recursive body-frame oracle, with rotated joint origins and tilted
    gravity too."""
    d = {"chain7": W.chain(7), "humanoid30": W.humanoid(),
         "tree12": W.random_tree([-1, 0, 1, 1, 0, 4, 5, 5, 7, 0, 9, 10], True, 5),
         "humanoid30_rot": W.humanoid(8, rotated=True, gravity=W.tilted_gravity(9))}[name]
    # FP32 rounding leaves the origin rotations orthonormal only to ~6e-8; the two formulations
    # read a non-orthonormal matrix differently (a transpose as the inverse, or not), so both are
    # given its nearest rotation (polar factor) for an FP64-exact comparison
    for i in range(d.n_bodies):
        U_, _, Vt = np.linalg.svd(d.origin[i, :9].reshape(3, 3))
        d.origin[i, :9] = (U_ @ Vt).reshape(-1)
    st = W.states(d, 32, 7)
    rng = np.random.Generator(np.random.PCG64(3))
    qdd = rng.normal(size=st.qd.shape)
    assert rel_err(JF.mass_matrix(d, st.q), O.crba(d, st.q)) < 1e-12
    assert rel_err(JF.inverse_dynamics(d, st.q, st.qd, qdd), O.rnea(d, st.q, st.qd, qdd)) < 1e-12
    assert rel_err(JF.inverse_dynamics(d, st.q, st.qd), O.rnea(d, st.q, st.qd)) < 1e-12


# ---------------------------------------------------------------- kinematics
def test_fk_at_zero_and_orthonormality():
    d = W.chain(7)
    T = O.fk(d, np.zeros((1, 7)))[0]
    assert np.allclose(T[:, :, 3], np.cumsum(d.origin[:, 9:12], axis=0), atol=1e-15)
    assert np.allclose(T[:, :, :3], np.eye(3)[None], atol=1e-15)
    for dd in (W.chain(7), W.humanoid()):
        st = W.states(dd, 64, 8)
        R = O.fk(dd, st.q)[..., :3]
        assert np.abs(np.einsum("bnij,bnkj->bnik", R, R) - np.eye(3)).max() < 1e-13
        assert np.allclose(np.linalg.det(R), 1.0, atol=1e-13)


def test_fk_base_pose_is_the_free_joint_state():
    d = W.humanoid()
    st = W.states(d, 8, 10)
    T = O.fk(d, st.q)
    assert np.allclose(T[:, 0, :, 3], st.q[:, 0:3], atol=1e-15)
    assert np.allclose(T[:, 0, :, :3], base_rotation(st.q[:, 3:7]), atol=1e-14)
    q2 = st.q.copy()
    q2[:, 3:7] *= 3.7                                  # a scaled quaternion is the same rotation
    assert np.allclose(O.fk(d, q2), T, atol=1e-14)


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_jacobian_is_the_derivative_of_fk(name):
    """J(q) qd = [d p / dt; w] of every frame, with both sides from FK alone."""
    d = W.chain(7) if name == "chain7" else W.humanoid()
    st = W.states(d, 4, 11)
    J = O.jacobian(d, st.q)
    eps = 1e-6
    T0 = O.fk(d, st.q)
    for k in range(d.nv):
        e = np.zeros_like(st.qd)
        e[:, k] = 1.0
        Tp, Tm = O.fk(d, retract(d, st.q, e, eps)), O.fk(d, retract(d, st.q, e, -eps))
        pdot = (Tp[..., :, 3] - Tm[..., :, 3]) / (2 * eps)
        Wx = np.einsum("bnij,bnkj->bnik", (Tp[..., :3] - Tm[..., :3]) / (2 * eps), T0[..., :3])
        w = np.stack([Wx[..., 2, 1], Wx[..., 0, 2], Wx[..., 1, 0]], -1)
        assert np.abs(J[:, :, 0:3, k] - pdot).max() < 1e-8
        assert np.abs(J[:, :, 3:6, k] - w).max() < 1e-8


# ---------------------------------------------------------------- derivatives
@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_vjp_tau_block_is_the_inverse_mass_matrix(name):
    """d qdd / d tau = M^-1, so gbar^T M^-1 is the tau cotangent exactly."""
    d = W.chain(7) if name == "chain7" else W.humanoid()
    st = W.states(d, 8, 12)
    gbar = W.cotangent(d.nv, 8, 13)
    _, _, gtau = O.fwd_dyn_vjp_fd(d, st.q, st.qd, st.tau, gbar)
    ref = np.linalg.solve(O.crba(d, st.q), gbar[..., None])[..., 0]
    assert rel_err(gtau, ref) < 1e-7


def test_vjp_dot_product_with_directional_difference():
    """<gbar, D qdd [dq, dqd, dtau]> = <vjp(gbar), [dq, dqd, dtau]> for random directions."""
    d = W.humanoid()
    st = W.states(d, 8, 14)
    gbar = W.cotangent(d.nv, 8, 15)
    gq, gqd, gtau = O.fwd_dyn_vjp_fd(d, st.q, st.qd, st.tau, gbar)
    rng = np.random.Generator(np.random.PCG64(16))
    dq, dqd, dtau = rng.normal(size=st.q.shape), rng.normal(size=st.qd.shape), rng.normal(size=st.tau.shape)
    eps = 1e-6
    fp = O.fwd_dyn(d, st.q + eps * dq, st.qd + eps * dqd, st.tau + eps * dtau)
    fm = O.fwd_dyn(d, st.q - eps * dq, st.qd - eps * dqd, st.tau - eps * dtau)
    lhs = np.einsum("bi,bi->b", gbar, (fp - fm) / (2 * eps))
    rhs = np.einsum("bi,bi->b", gq, dq) + np.einsum("bi,bi->b", gqd, dqd) + np.einsum("bi,bi->b", gtau, dtau)
    assert np.allclose(lhs, rhs, rtol=1e-5, atol=1e-6 * np.abs(lhs).max())


def test_vjp_position_is_invariant_to_base_translation():
    """Dynamics in body coordinates do not depend on the base position."""
    d = W.humanoid()
    st = W.states(d, 4, 17)
    gbar = W.cotangent(d.nv, 4, 18)
    gq, _, _ = O.fwd_dyn_vjp_fd(d, st.q, st.qd, st.tau, gbar)
    assert np.abs(gq[:, 0:3]).max() < 1e-6


# ---------------------------------------------------------------- operation counts
def test_operation_counts_are_consistent():
    for d in (W.chain(7), W.humanoid()):
        nrev = int((d.joint_type == W.REVOLUTE).sum())
        fk = O.count_ops(d, "fk")
        assert fk["trig"] == 2 * nrev
        ltl, llt = O.count_ops(d, "fwd_dyn_ltl"), O.count_ops(d, "fwd_dyn_llt")
        # one square root per DoF; L^T L starts at the leaves, whose pivots are model constants
        leaves = sum(1 for i in range(d.n_bodies) if i not in set(d.parent.tolist()))
        assert ltl["sqrt"] == d.nv - leaves and llt["sqrt"] <= d.nv
        if d.floating:
            assert ltl["flops"] < llt["flops"]         # branch sparsity saves work
        else:
            assert ltl["flops"] == llt["flops"]        # a chain has none
        # forward dynamics builds the joint transforms once for both passes
        rb, cr = O.count_ops(d, "rnea_bias"), O.count_ops(d, "crba")
        assert ltl["trig"] == rb["trig"] == cr["trig"] == 2 * nrev


# Hand-derived counts of the counting scalar's rules (model-only arithmetic is folded, operations
# with a known 0 operand or a known +-1 factor are free, everything else counts once) for revolute
# joints with identity origin rotations and general axes, origins and inertias (no zero entries).
# Per primitive: mv/mtv (variable matrix or vector) 9 mul 6 add; cross 6 mul 3 add; dot 3 mul 2 add;
# 3x3 product 27 mul 18 add; skew_skew(a, b) = b a^T - (a.b) 1: 12 mul 5 add.
#   joint transform: Rodrigues 2 trig, 1 - c (1 add), diagonal c + t a_k^2 (3 mul 3 add), six
#     off-diagonal t a_j a_k +- s a_l (12 mul 6 add); the identity origin rotation is free: 15 mul 10 add.
#   root body of RNEA (bias): S qd 3 mul; X a_0 with a_0 = (0, 0, 0; 0, 0, 9.81) 3 mul; v x S qd
#     6 mul 3 add (v.l = 0); I a 24 mul 18 add; I v 15 mul 9 add (v.l = 0); v x* I v 12 mul 6 add;
#     sum 6 add: 63 mul 42 add. S^T f: 3 mul 2 add.
#   a child body: S qd 3 mul; X v_p 24 mul 15 add (v_p.l = 0 at the root) + S qd 3 add; X a_p 24 mul
#     18 add; v x S qd 12 mul 6 add; + 6 add; I a 24 mul 18 add; I v 24 mul 18 add; v x* I v 18 mul
#     12 add; + 6 add: 129 mul 102 add. Backward S^T f 3 mul 2 add; f_p += X^T f 24 mul 24 add.
#   CRBA with the transforms given: X^T Ic X of the child 87 mul 73 add (E^T h 9m 6a, + m r 3a, E^T I E
#     54m 36a, two skew_skew 24m 10a, two 3x3 subtractions 18a), Ic_p += 12 add; the root's
#     F = Ic S 15 mul 9 add and S^T F 3 mul 2 add; the child's F = Ic S and S^T F are model constants;
#     F <- X^T F 24 mul 18 add and S^T F 3 mul 2 add.
#   L^T L of 2 DoFs: the leaf's pivot is a constant (its sqrt is free); L_10 = M_10 / L_11 1 div;
#     M_00 -= L_10^2 1 mul 1 add; sqrt(M_00); the two triangular solves 2 mul 2 add 4 div.
def test_operation_count_of_one_pendulum():
    d = W.random_tree([-1], False, 31)
    c = O.count_ops(d, "fwd_dyn_ltl")
    # transform 15m 10a; RNEA root 63m 42a; S^T f 3m 2a; tau - h 1a; M is a model constant;
    # L^T y = b and L x = y: one division each
    assert (c["mul"], c["addsub"], c["div"], c["sqrt"], c["trig"]) == (15 + 63 + 3, 10 + 42 + 2 + 1, 2, 0, 2)
    assert O.count_ops(d, "crba")["flops"] == 15 + 10  # only the transform; M itself is constant
    assert O.count_ops(d, "rnea_bias")["flops"] == (15 + 10) + (63 + 42) + (3 + 2)


def test_operation_count_of_a_two_link_chain():
    d = W.random_tree([-1, 0], False, 32)
    assert not np.any(d.axis == 0.0) and not np.any(d.origin[:, 9:12] == 0.0)
    transforms = 2 * (15 + 10)
    rnea = (63 + 42) + (129 + 102) + (3 + 2) + (24 + 24) + (3 + 2)
    crba = (87 + 73) + 12 + (15 + 9) + (3 + 2) + (24 + 18) + (3 + 2)
    solve = 2 + (1 + 1) + (2 + 2)  # tau - h (2 add), the factor update, the two solves (2 mul 2 add)
    assert O.count_ops(d, "rnea_bias")["flops"] == transforms + rnea
    assert O.count_ops(d, "crba")["flops"] == transforms + crba
    c = O.count_ops(d, "fwd_dyn_ltl")
    assert c["flops"] == transforms + rnea + crba + solve
    assert (c["div"], c["sqrt"], c["trig"]) == (5, 1, 4)


# ---------------------------------------------------------------- external forces (Eq. (1) J^T f, Alg. 1 F_ext)
def _random_fext(desc, B, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, 5.0, size=(B, desc.n_bodies, 6))


@pytest.mark.parametrize("name", ["chain7", "tree12f", "humanoid30"])
def test_external_weight_support_cancels_gravity(name):
    """Each body held up at its CoM by a force equal to its weight: at rest no joint torque is
    needed, and with zero torque nothing accelerates (every method)."""
    desc = {"chain7": W.chain(7), "tree12f": W.random_tree([-1, 0, 1, 1, 0, 4, 5, 5, 7, 0, 9, 10], True, 34),
            "humanoid30": W.humanoid()}[name]
    B = 16
    st = W.states(desc, B, 41)
    zero = np.zeros((B, desc.nv))
    c = com_world(desc, O.fk(desc, st.q))
    f = -desc.mass[None, :, None] * np.asarray(desc.gravity)[None, None, :]
    fext = np.concatenate([np.broadcast_to(f, c.shape), np.cross(c, f)], axis=2)
    scale = np.abs(O.rnea(desc, st.q, zero)).max()
    assert scale > 1.0
    assert np.abs(O.rnea(desc, st.q, zero, fext=fext)).max() < 1e-11 * scale
    for method in (O.METHOD_LLT, O.METHOD_LTL, O.METHOD_ABA):
        assert np.abs(O.fwd_dyn(desc, st.q, zero, zero, method, fext=fext)).max() < 1e-9


@pytest.mark.parametrize("name", ["chain7", "tree12f", "humanoid30"])
def test_external_force_is_virtual_work_through_jacobians(name):
    """tau(F) - tau(0) = -sum_i J_i^T [f_i; n_i - p_i x f_i] with the kinematic Jacobians of the body
    origins p_i (the moment moved from the world origin to p_i)."""
    desc = {"chain7": W.chain(7), "tree12f": W.random_tree([-1, 0, 1, 1, 0, 4, 5, 5, 7, 0, 9, 10], True, 34),
            "humanoid30": W.humanoid()}[name]
    B = 8
    st = W.states(desc, B, 42)
    qdd = W.cotangent(desc.nv, B, 43)
    fext = _random_fext(desc, B, 44)
    dtau = O.rnea(desc, st.q, st.qd, qdd, fext=fext) - O.rnea(desc, st.q, st.qd, qdd)
    p = O.fk(desc, st.q)[..., :, 3]
    J = O.jacobian(desc, st.q)  # [B, n, 6, nv], rows [v; w]
    wrench = np.concatenate([fext[..., :3], fext[..., 3:] - np.cross(p, fext[..., :3])], axis=2)
    ref = -np.einsum("bnrc,bnr->bc", J, wrench)
    assert rel_err(dtau, ref) < 1e-12
    # forward dynamics moves by M^-1 of the same generalised force
    M = O.crba(desc, st.q)
    for method in (O.METHOD_LLT, O.METHOD_LTL, O.METHOD_ABA):
        d_qdd = O.fwd_dyn(desc, st.q, st.qd, st.tau, method, fext=fext) - O.fwd_dyn(desc, st.q, st.qd, st.tau, method)
        assert rel_err(d_qdd, np.linalg.solve(M, -ref[..., None])[..., 0]) < 1e-10


def test_free_body_force_through_com_closed_form():
    """A free body at rest pushed by F through its CoM: the origin accelerates by R^T (F/m + g) in
    body axes and nothing turns."""
    d, rng = _single_body(11, floating=True)
    B = 8
    st = W.states(d, B, 45)
    R = base_rotation(st.q[:, 3:7] / np.linalg.norm(st.q[:, 3:7], axis=1, keepdims=True))
    cw = st.q[:, :3] + np.einsum("bij,j->bi", R, d.com[0])
    F = rng.normal(0, 10, size=(B, 3))
    fext = np.concatenate([F, np.cross(cw, F)], axis=1)[:, None, :]
    lin = np.einsum("bji,bj->bi", R, F / d.mass[0] + np.asarray(d.gravity))
    ref = np.concatenate([lin, np.zeros((B, 3))], axis=1)
    zero = np.zeros((B, 6))
    for method in (O.METHOD_LLT, O.METHOD_LTL, O.METHOD_ABA):
        assert np.allclose(O.fwd_dyn(d, st.q, zero, zero, method, fext=fext), ref, rtol=1e-11, atol=1e-11)


# ---------------------------------------------------------------- forward-mode derivative (jax.jvp, Sec. IV-A)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_jvp_single_pendulum_closed_form(seed):
    """qdd = (tau - G(q)) / M with constant M and G(q) = dV/dq: d qdd = (dtau - G'(q) dq) / M, where
    G'(q) follows from d/dq R(q) c = a x R(q) c; qd does not enter."""
    d, rng = _single_body(seed)
    a = d.axis[0] / np.linalg.norm(d.axis[0])
    c, m = d.com[0], d.mass[0]
    Rf = d.origin[0, :9].reshape(3, 3)
    M_ref = a @ inertia_matrix(d, 0) @ a + m * np.dot(np.cross(a, c), np.cross(a, c))
    B = 16
    q, qd, tau = rng.uniform(-np.pi, np.pi, (B, 1)), rng.normal(size=(B, 1)), rng.normal(0, 5, (B, 1))
    dq, dqd, dtau = rng.normal(size=(B, 1)), rng.normal(size=(B, 1)), rng.normal(size=(B, 1))
    lever = np.einsum("bij,j->bi", Rotation.from_rotvec(a[None, :] * q).as_matrix(), c)
    dG = -m * np.einsum("i,ij,bj->b", d.gravity, Rf, np.cross(a[None, :], np.cross(a[None, :], lever)))
    ref = (dtau[:, 0] - dG * dq[:, 0]) / M_ref
    # a central difference of step 1e-6 carries rounding of about eps |qdd| / h ~ 1e-9 |qdd|
    for method in (O.METHOD_LLT, O.METHOD_LTL, O.METHOD_ABA):
        assert np.allclose(O.fwd_dyn_jvp_fd(d, q, qd, tau, dq, dqd, dtau, method=method)[:, 0], ref,
                           rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_jvp_is_dual_to_vjp(name):
    """<gbar, J dx> = <J^T gbar, dx> between the two difference formulas (each to O(h^2))."""
    desc = W.chain(7) if name == "chain7" else W.humanoid()
    B = 8
    st = W.states(desc, B, 46)
    rng = np.random.Generator(np.random.PCG64(47))
    dq, dqd, dtau = rng.normal(size=st.q.shape), rng.normal(size=st.qd.shape), rng.normal(size=st.tau.shape)
    gbar = W.cotangent(desc.nv, B, 48)
    jv = O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, dq, dqd, dtau)
    gq, gqd, gtau = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar)
    lhs = np.einsum("bk,bk->b", gbar, jv)
    rhs = np.einsum("bk,bk->b", gq, dq) + np.einsum("bk,bk->b", gqd, dqd) + np.einsum("bk,bk->b", gtau, dtau)
    assert np.allclose(lhs, rhs, rtol=1e-6, atol=1e-6 * np.abs(rhs).max())


def test_jvp_tau_direction_is_inverse_mass_matrix():
    """Along (0, 0, dtau) the derivative is M^-1 dtau exactly (forward dynamics is affine in tau)."""
    desc = W.humanoid()
    B = 8
    st = W.states(desc, B, 49)
    dtau = W.cotangent(desc.nv, B, 50)
    jv = O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, np.zeros_like(st.q), np.zeros_like(st.qd), dtau)
    assert rel_err(jv, np.linalg.solve(O.crba(desc, st.q), dtau[..., None])[..., 0]) < 1e-7


# ---------------------------------------------------------------- derivatives with external forces
@pytest.mark.parametrize("name", ["chain7", "tree12f"])
def test_vjp_with_forces_closed_form_blocks(name):
    """With external forces: g_tau = M^-1 gbar still (forward dynamics is affine in tau, forces
    aside), and g_F_i = J_i M^-1 gbar exactly, J_i the Jacobian of body i's twist at the world
    origin, [v_O; w] = [v_p + p x w; w] (qdd is affine in F with slope M^-1 J^T)."""
    desc = W.chain(7) if name == "chain7" else W.random_tree([-1, 0, 1, 1, 0, 4, 5, 5, 7, 0, 9, 10], True, 34)
    B = 6
    st = W.states(desc, B, 60)
    fext = _random_fext(desc, B, 61)
    gbar = W.cotangent(desc.nv, B, 62)
    gq, gqd, gtau, gf = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar, fext=fext)
    lam = np.linalg.solve(O.crba(desc, st.q), gbar[..., None])[..., 0]
    assert rel_err(gtau, lam) < 1e-7
    J = O.jacobian(desc, st.q)  # [B, n, 6, nv], rows [v; w] at the body origin p
    p = O.fk(desc, st.q)[..., :, 3]
    tw = np.einsum("bnrc,bc->bnr", J, lam)
    ref = np.concatenate([tw[..., :3] + np.cross(p, tw[..., 3:]), tw[..., 3:]], axis=2).reshape(B, -1)
    assert rel_err(gf, ref) < 1e-7
    # without forces the q and qd blocks are the force-free ones
    g0 = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar, fext=np.zeros_like(fext))
    r0 = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar)
    assert rel_err(g0[0], r0[0]) < 1e-12 and rel_err(g0[1], r0[1]) < 1e-12


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_jvp_is_dual_to_vjp_with_forces(name):
    """<gbar, J dx> = <J^T gbar, dx> with forces and force tangents (both difference formulas)."""
    desc = W.chain(7) if name == "chain7" else W.humanoid()
    B = 6
    st = W.states(desc, B, 63)
    rng = np.random.Generator(np.random.PCG64(64))
    fext = _random_fext(desc, B, 65)
    dq, dqd, dtau = rng.normal(size=st.q.shape), rng.normal(size=st.qd.shape), rng.normal(size=st.tau.shape)
    df = rng.normal(size=(B, 6 * desc.n_bodies))
    gbar = W.cotangent(desc.nv, B, 66)
    jv = O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, dq, dqd, dtau, fext=fext, dfext=df)
    gq, gqd, gtau, gf = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar, fext=fext)
    lhs = np.einsum("bk,bk->b", gbar, jv)
    rhs = sum(np.einsum("bk,bk->b", g, x) for g, x in ((gq, dq), (gqd, dqd), (gtau, dtau), (gf, df)))
    assert np.allclose(lhs, rhs, rtol=1e-6, atol=1e-6 * np.abs(rhs).max())


# ---------------------------------------------------------------- controller workloads (Sec. IV, Table II)
from oracle import controllers as CT  # noqa: E402


def _targets(desc, q, frame, seed, scale=0.2):
    """Targets near the current pose of `frame`: [B, 3, 4]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = O.fk(desc, q)[:, frame]
    dR = Rotation.from_rotvec(rng.normal(0, scale, size=(len(q), 3))).as_matrix()
    out = np.empty_like(T)
    out[:, :, :3] = dR @ T[:, :, :3]
    out[:, :, 3] = T[:, :, 3] + rng.normal(0, scale, size=(len(q), 3))
    return out


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_diff_ik_moves_the_frame_toward_its_target(name):
    """With no damping the commanded velocity makes the frame's twist k err exactly (J has full row
    rank), and a small step along it shrinks a finite pose error by about k dt."""
    desc = W.chain(7) if name == "chain7" else W.humanoid()
    B = 8
    st = W.states(desc, B, 51)
    e = desc.n_bodies - 1
    tgt = _targets(desc, st.q, e, 52)
    k = 2.0
    qd = CT.diff_ik(desc, st.q, e, tgt, k, 0.0)
    J = O.jacobian(desc, st.q, [e])[:, 0]
    err = CT.pose_error(desc, st.q, e, tgt)
    assert rel_err(np.einsum("brc,bc->br", J, qd), k * err) < 1e-9
    dt = 1e-4
    err2 = CT.pose_error(desc, retract(desc, st.q, qd, dt), e, tgt)
    # first order: d err / dt = -J qd for the position part; the rotation part follows the same
    # rate up to O(|err|^2) terms of the small-angle vector, so compare norms
    assert np.all(np.linalg.norm(err2, axis=1) < np.linalg.norm(err, axis=1))
    lin = err[:, :3] - dt * k * err[:, :3]
    assert np.allclose(err2[:, :3], lin, atol=1e-7)
    # at the target nothing moves
    T = O.fk(desc, st.q)[:, e]
    assert np.abs(CT.diff_ik(desc, st.q, e, T, k, 0.1)).max() < 1e-12


@pytest.mark.parametrize("name", ["chain7", "tree12f", "humanoid30"])
def test_osc_commands_exactly_the_task_acceleration(name):
    """Forward dynamics under the OSC torques gives J qdd = a* (every solver), and with no
    null-space damping tau - h lies in the range of J^T."""
    desc = {"chain7": W.chain(7), "tree12f": W.random_tree([-1, 0, 1, 1, 0, 4, 5, 5, 7, 0, 9, 10], True, 34),
            "humanoid30": W.humanoid()}[name]
    B = 8
    st = W.states(desc, B, 53)
    e = desc.n_bodies - 1
    tgt = _targets(desc, st.q, e, 54)
    kp, kd, kn = 50.0, 10.0, 2.0
    tau = CT.osc(desc, st.q, st.qd, e, tgt, kp, kd, kn)
    J = O.jacobian(desc, st.q, [e])[:, 0]
    a_star = kp * CT.pose_error(desc, st.q, e, tgt) - kd * np.einsum("brc,bc->br", J, st.qd)
    for method in (O.METHOD_LLT, O.METHOD_LTL, O.METHOD_ABA):
        qdd = O.fwd_dyn(desc, st.q, st.qd, tau, method)
        assert rel_err(np.einsum("brc,bc->br", J, qdd), a_star) < 1e-8
    tau0 = CT.osc(desc, st.q, st.qd, e, tgt, kp, kd, 0.0) - O.rnea(desc, st.q, st.qd)
    F, *_ = np.linalg.lstsq(np.swapaxes(J[0], 0, 1), tau0[0], rcond=None)
    assert np.allclose(np.swapaxes(J[0], 0, 1) @ F, tau0[0], rtol=1e-9, atol=1e-9 * np.abs(tau0[0]).max())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rnea_jvp_single_pendulum(seed):
    """The tangent of one revolute joint's inverse dynamics in closed form: tau = M qdd + dV/dq, so
    d tau = M dqdd + (d2V/dq2) dq with d(a x R c)/dq = a x (a x R c), and qd enters nowhere."""
    d, rng = _single_body(seed)
    a = d.axis[0] / np.linalg.norm(d.axis[0])
    c, m = d.com[0], d.mass[0]
    Ic = inertia_matrix(d, 0)
    Rf = d.origin[0, :9].reshape(3, 3)
    B = 16
    q = rng.uniform(-np.pi, np.pi, size=(B, 1))
    qd, qdd, dq, dqd, dqdd = (rng.normal(size=(B, 1)) for _ in range(5))
    M_ref = a @ Ic @ a + m * np.dot(np.cross(a, c), np.cross(a, c))
    Rq = Rotation.from_rotvec(a[None, :] * q).as_matrix()
    lever = np.einsum("bij,j->bi", Rq, c)
    d2V = -m * np.einsum("i,ij,bj->b", d.gravity, Rf, np.cross(a[None, :], np.cross(a[None, :], lever)))
    ref = M_ref * dqdd[:, 0] + d2V * dq[:, 0]
    got = O.rnea_jvp_fd(d, q, qd, qdd, dq, dqd, dqdd)[:, 0]
    assert np.allclose(got, ref, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_rnea_jvp_along_qdd_is_M(name):
    """Inverse dynamics is affine in qdd: its tangent along (0, 0, dqdd) is M(q) dqdd."""
    desc = W.chain(7) if name == "chain7" else W.humanoid()
    st = W.states(desc, 8, 41)
    rng = np.random.Generator(np.random.PCG64(42))
    qdd, dqdd = rng.normal(size=st.qd.shape), rng.normal(size=st.qd.shape)
    z = np.zeros_like
    got = O.rnea_jvp_fd(desc, st.q, st.qd, qdd, z(st.q), z(st.qd), dqdd)
    ref = np.einsum("bij,bj->bi", O.crba(desc, st.q), dqdd)
    assert np.abs(got - ref).max() < 1e-7 * np.abs(ref).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rnea_vjp_single_pendulum(seed):
    """The cotangents of one revolute joint's inverse dynamics tau = M qdd + dV/dq in closed form:
    g_q = lam d2V/dq2, g_qd = 0 (no velocity dependence), g_qdd = M lam."""
    d, rng = _single_body(seed)
    a = d.axis[0] / np.linalg.norm(d.axis[0])
    c, m = d.com[0], d.mass[0]
    Ic = inertia_matrix(d, 0)
    Rf = d.origin[0, :9].reshape(3, 3)
    B = 16
    q = rng.uniform(-np.pi, np.pi, size=(B, 1))
    qd, qdd, lam = (rng.normal(size=(B, 1)) for _ in range(3))
    M_ref = a @ Ic @ a + m * np.dot(np.cross(a, c), np.cross(a, c))
    Rq = Rotation.from_rotvec(a[None, :] * q).as_matrix()
    lever = np.einsum("bij,j->bi", Rq, c)
    d2V = -m * np.einsum("i,ij,bj->b", d.gravity, Rf, np.cross(a[None, :], np.cross(a[None, :], lever)))
    gq, gqd, gqdd = O.rnea_vjp_fd(d, q, qd, qdd, lam)
    assert np.allclose(gq[:, 0], lam[:, 0] * d2V, rtol=1e-7, atol=1e-8)
    assert np.abs(gqd).max() < 1e-8
    assert np.allclose(gqdd[:, 0], M_ref * lam[:, 0], rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_rnea_vjp_qdd_block_is_M(name):
    """Inverse dynamics is affine in qdd with slope M(q), which is symmetric: g_qdd = M lam."""
    desc = W.chain(7) if name == "chain7" else W.humanoid()
    st = W.states(desc, 6, 45)
    rng = np.random.Generator(np.random.PCG64(46))
    qdd, lam = rng.normal(size=st.qd.shape), rng.normal(size=st.qd.shape)
    gqdd = O.rnea_vjp_fd(desc, st.q, st.qd, qdd, lam)[2]
    ref = np.einsum("bij,bj->bi", O.crba(desc, st.q), lam)
    assert np.abs(gqdd - ref).max() < 1e-7 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["chain7", "tree12f"])
def test_rnea_vjp_force_cotangent_and_force_free_blocks(name):
    """ID carries -sum_i J_i^T F_i (Eq. (1)), so g_F_i = -J_i lam exactly, J_i the Jacobian of body
    i's twist at the world origin, [v_O; w] = [v_p + p x w; w]; with zero forces the other blocks are
    the force-free ones."""
    desc = W.chain(7) if name == "chain7" else W.random_tree([-1, 0, 1, 1, 0, 4, 5, 5, 7, 0, 9, 10], True, 34)
    B = 6
    st = W.states(desc, B, 67)
    fext = _random_fext(desc, B, 68)
    rng = np.random.Generator(np.random.PCG64(69))
    qdd, lam = rng.normal(size=st.qd.shape), rng.normal(size=st.qd.shape)
    gq, gqd, gqdd, gf = O.rnea_vjp_fd(desc, st.q, st.qd, qdd, lam, fext=fext, want_fext=True)
    J = O.jacobian(desc, st.q)  # [B, n, 6, nv], rows [v; w] at the body origin p
    p = O.fk(desc, st.q)[..., :, 3]
    tw = np.einsum("bnrc,bc->bnr", J, lam)
    ref = -np.concatenate([tw[..., :3] + np.cross(p, tw[..., 3:]), tw[..., 3:]], axis=2).reshape(B, -1)
    assert rel_err(gf, ref) < 1e-7
    g0 = O.rnea_vjp_fd(desc, st.q, st.qd, qdd, lam, fext=np.zeros_like(fext))
    r0 = O.rnea_vjp_fd(desc, st.q, st.qd, qdd, lam)
    assert all(rel_err(x, y) < 1e-12 for x, y in zip(g0, r0))


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
def test_rnea_vjp_is_dual_to_rnea_jvp(name):
    """<lam, J dx> = <J^T lam, dx> for inverse dynamics, forces and force tangents included."""
    desc = W.chain(7) if name == "chain7" else W.humanoid()
    B = 6
    st = W.states(desc, B, 70)
    rng = np.random.Generator(np.random.PCG64(71))
    fext = _random_fext(desc, B, 72)
    qdd = rng.normal(size=st.qd.shape)
    dq, dqd, dqdd = rng.normal(size=st.q.shape), rng.normal(size=st.qd.shape), rng.normal(size=st.qd.shape)
    df = rng.normal(size=(B, 6 * desc.n_bodies))
    lam = W.cotangent(desc.nv, B, 73)
    jv = O.rnea_jvp_fd(desc, st.q, st.qd, qdd, dq, dqd, dqdd, fext=fext, dfext=df)
    gq, gqd, gqdd, gf = O.rnea_vjp_fd(desc, st.q, st.qd, qdd, lam, fext=fext, want_fext=True)
    lhs = np.einsum("bk,bk->b", lam, jv)
    rhs = sum(np.einsum("bk,bk->b", g, x) for g, x in ((gq, dq), (gqd, dqd), (gqdd, dqdd), (gf, df)))
    assert np.allclose(lhs, rhs, rtol=1e-6, atol=1e-6 * np.abs(rhs).max())


def test_rnea_vjp_composes_with_fwd_dyn_vjp():
    """Implicit differentiation of ID(q, qd, FD(q, qd, tau)) = tau: at qdd = FD(...) and lam =
    M^-1 gbar, the fwd_dyn cotangents are (g_q, g_qd) = -(ID's g_q, g_qd) and g_tau = lam."""
    desc = W.humanoid()
    B = 4
    st = W.states(desc, B, 74)
    gbar = W.cotangent(desc.nv, B, 75)
    qdd = O.fwd_dyn(desc, st.q, st.qd, st.tau)
    lam = np.linalg.solve(O.crba(desc, st.q), gbar[..., None])[..., 0]
    gq, gqd, _ = O.rnea_vjp_fd(desc, st.q, st.qd, qdd, lam)
    fq, fqd, ftau = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar)
    assert rel_err(-gq, fq) < 1e-5 and rel_err(-gqd, fqd) < 1e-5 and rel_err(lam, ftau) < 1e-7


@pytest.mark.parametrize("forces", [False, True])
def test_rnea_jvp_inverts_fwd_dyn_jvp(forces):
    """ID(q, qd, FD(q, qd, tau, F), F) = tau, so along any (dq, dqd, dtau, dF) the tangent of
    inverse dynamics at dqdd = the tangent of forward dynamics returns dtau."""
    desc = W.humanoid()
    st = W.states(desc, 8, 43)
    rng = np.random.Generator(np.random.PCG64(44))
    dq, dqd, dtau = (rng.normal(size=x.shape) for x in (st.q, st.qd, st.tau))
    fx = rng.normal(0.0, 5.0, size=(8, desc.n_bodies * 6)) if forces else None
    dfx = rng.normal(size=(8, desc.n_bodies * 6)) if forces else None
    qdd = O.fwd_dyn(desc, st.q, st.qd, st.tau, fext=None if fx is None else fx.reshape(8, -1, 6))
    dqdd = O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, dq, dqd, dtau, fext=fx, dfext=dfx)
    got = O.rnea_jvp_fd(desc, st.q, st.qd, qdd, dq, dqd, dqdd, fext=fx, dfext=dfx)
    assert np.abs(got - dtau).max() < 1e-5 * np.abs(dtau).max()

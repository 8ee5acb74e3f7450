"""Parity at the benchmark sizes, in the launch configuration the benchmark times.

Chain of 7 at batch 2^20 (fwd_dyn, rnea: first 4096 states against the oracle,
all outputs finite), the 35-DoF humanoid at batch 65536 (fwd_dyn by both the
factorised solve and the articulated-body algorithm on every instance; crba,
fk and jacobian on a strided sample; with external forces on a sample; the
same rows for a URDF-style humanoid with rotated joint origins), and
the adjoint and the forward-mode derivative at 2^18 (chain) and 32768
(humanoid) against central differences on 256 states.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import rel_err, vjp_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rbd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04310_amd as rbd
    rbd.lib()
    return rbd


def gpu(x):
    return torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")


def cols(t, idx):
    """Instances idx of a [rows, B] tensor as a float64 [len(idx), rows] array."""
    torch.cuda.synchronize()
    return t[:, torch.as_tensor(idx, device=t.device)].double().cpu().numpy().T


def test_chain7_batch_2p20(rbd):
    desc = W.chain(7)
    m = rbd.Model(desc, 0)
    st = W.states(desc, 1 << 20, 102)
    q, qd, tau = gpu(st.q), gpu(st.qd), gpu(st.tau)
    qdd = rbd.fwd_dyn(m, q, qd, tau)
    h = rbd.rnea(m, q, qd)
    torch.cuda.synchronize()
    assert torch.isfinite(qdd).all() and torch.isfinite(h).all()
    idx = np.arange(4096)
    assert rel_err(cols(qdd, idx), O.fwd_dyn(desc, st.q[idx], st.qd[idx], st.tau[idx])) < 1e-4
    assert rel_err(cols(h, idx), O.rnea(desc, st.q[idx], st.qd[idx])) < 1e-4


def test_humanoid_batch_65536(rbd):
    desc = W.humanoid()
    m = rbd.Model(desc, 0)
    B = 65536
    st = W.states(desc, B, 103)
    q, qd, tau = gpu(st.q), gpu(st.qd), gpu(st.tau)
    qdd = rbd.fwd_dyn(m, q, qd, tau)
    h = rbd.rnea(m, q, qd)
    torch.cuda.synchronize()
    all_idx = np.arange(B)
    ref = O.fwd_dyn(desc, st.q, st.qd, st.tau)
    assert rel_err(cols(qdd, all_idx), ref) < 1e-4
    del qdd
    qdd_aba = rbd.aba(m, q, qd, tau)
    assert rel_err(cols(qdd_aba, all_idx), ref) < 1e-4
    del qdd_aba
    assert rel_err(cols(h, all_idx), O.rnea(desc, st.q, st.qd)) < 1e-4
    idx = np.arange(0, B, 61)
    M = rbd.crba(m, q)
    Mh = cols(M, idx).reshape(len(idx), -1)
    Mr = O.crba(desc, st.q[idx]).reshape(len(idx), -1)
    assert (np.abs(Mh - Mr).max(1) / np.abs(Mr).max(1)).max() < 1e-5
    del M
    T = rbd.fk(m, q)
    assert rel_err(cols(T, idx), O.fk(desc, st.q[idx]).reshape(len(idx), -1)) < 1e-5
    del T
    J = rbd.jacobian(m, q)
    assert rel_err(cols(J, idx), O.jacobian(desc, st.q[idx]).reshape(len(idx), -1)) < 1e-5
    del J


def test_rotated_humanoid_batch_65536(rbd):
    """The URDF-style humanoid (random joint-origin rotations, gravity in a random direction, joint
    angles up to 1000 rad) at the benchmark size: fwd_dyn on every instance, rnea, crba, fk and
    jacobian on a strided sample."""
    desc = W.humanoid(64, rotated=True, gravity=W.tilted_gravity(65))
    m = rbd.Model(desc, 0)
    B = 65536
    st = W.states(desc, B, 110, q_range=1000.0)
    q, qd, tau = gpu(st.q), gpu(st.qd), gpu(st.tau)
    qdd = rbd.fwd_dyn(m, q, qd, tau)
    torch.cuda.synchronize()
    assert torch.isfinite(qdd).all()
    assert rel_err(cols(qdd, np.arange(B)), O.fwd_dyn(desc, st.q, st.qd, st.tau)) < 1e-4
    del qdd
    idx = np.arange(0, B, 61)
    h = rbd.rnea(m, q, qd)
    assert rel_err(cols(h, idx), O.rnea(desc, st.q[idx], st.qd[idx])) < 1e-4
    M = rbd.crba(m, q)
    Mh = cols(M, idx).reshape(len(idx), -1)
    Mr = O.crba(desc, st.q[idx]).reshape(len(idx), -1)
    assert (np.abs(Mh - Mr).max(1) / np.abs(Mr).max(1)).max() < 1e-5
    del M
    T = rbd.fk(m, q)
    assert rel_err(cols(T, idx), O.fk(desc, st.q[idx]).reshape(len(idx), -1)) < 1e-5
    del T
    J = rbd.jacobian(m, q)
    assert rel_err(cols(J, idx), O.jacobian(desc, st.q[idx]).reshape(len(idx), -1)) < 1e-5
    del J


@pytest.mark.parametrize("name,B", [("chain7", 1 << 18), ("humanoid30", 32768), ("humanoid30", 65536)])
def test_vjp_full_batch(rbd, name, B):
    desc = W.chain(7) if name == "chain7" else W.humanoid()
    m = rbd.Model(desc, 0)
    st = W.states(desc, B, 104)
    gbar = W.cotangent(desc.nv, B, 105)
    gq, gqd, gtau = rbd.fwd_dyn_vjp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), gpu(gbar))
    torch.cuda.synchronize()
    assert torch.isfinite(gq).all() and torch.isfinite(gqd).all() and torch.isfinite(gtau).all()
    idx = np.linspace(0, B - 1, 256).astype(int)
    rq, rqd, rtau = O.fwd_dyn_vjp_fd(desc, st.q[idx], st.qd[idx], st.tau[idx], gbar[idx])
    assert vjp_err([cols(gq, idx), cols(gqd, idx), cols(gtau, idx)], [rq, rqd, rtau]) < 1e-3


@pytest.mark.parametrize("name,B", [("chain7", 1 << 18), ("humanoid30", 32768), ("humanoid30", 65536),
                                    ("humanoid30", 32768 + 37)])
def test_jvp_full_batch(rbd, name, B):
    """The forward-mode derivative at the adjoint's benchmark sizes (the humanoid on two waves per 64
    instances up to 32768, one wave above): finite everywhere, 256 states against central
    differences of the oracle along the same tangent."""
    desc = W.chain(7) if name == "chain7" else W.humanoid()
    m = rbd.Model(desc, 0)
    st = W.states(desc, B, 106)
    rng = np.random.Generator(np.random.PCG64(107))
    dq, dqd, dtau = (W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.tau))
    dqdd = rbd.fwd_dyn_jvp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), gpu(dq), gpu(dqd), gpu(dtau))
    torch.cuda.synchronize()
    assert torch.isfinite(dqdd).all()
    idx = np.linspace(0, B - 1, 256).astype(int)
    ref = O.fwd_dyn_jvp_fd(desc, st.q[idx], st.qd[idx], st.tau[idx], dq[idx], dqd[idx], dtau[idx])
    assert vjp_err([cols(dqdd, idx)], [ref]) < 1e-3


def test_rnea_jvp_full_batch(rbd):
    """The tangent of the humanoid's inverse dynamics at 65536 with external forces: finite
    everywhere, 256 states against central differences of the oracle."""
    desc = W.humanoid()
    m = rbd.Model(desc, 0)
    B = 65536
    st = W.states(desc, B, 114)
    rng = np.random.Generator(np.random.PCG64(115))
    qdd, dq, dqd, dqdd = (W._f32(rng.normal(size=x.shape)) for x in (st.qd, st.q, st.qd, st.qd))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, desc.n_bodies * 6)))
    df = W._f32(rng.normal(size=fext.shape))
    dtau = rbd.rnea_jvp(m, *[gpu(x) for x in (st.q, st.qd, qdd, dq, dqd, dqdd)], fext=gpu(fext), dfext=gpu(df))
    torch.cuda.synchronize()
    assert torch.isfinite(dtau).all()
    idx = np.linspace(0, B - 1, 256).astype(int)
    ref = O.rnea_jvp_fd(desc, *[x[idx] for x in (st.q, st.qd, qdd, dq, dqd, dqdd)], fext=fext[idx], dfext=df[idx])
    assert vjp_err([cols(dtau, idx)], [ref]) < 1e-3


def test_rnea_vjp_full_batch(rbd):
    """The adjoint of the humanoid's inverse dynamics at 65536 with external forces: finite
    everywhere, 256 states against central differences of the oracle."""
    desc = W.humanoid()
    m = rbd.Model(desc, 0)
    B = 65536
    st = W.states(desc, B, 116)
    rng = np.random.Generator(np.random.PCG64(117))
    qdd = W._f32(rng.normal(size=st.qd.shape))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, desc.n_bodies * 6)))
    lam = W.cotangent(desc.nv, B, 118)
    outs = rbd.rnea_vjp(m, *[gpu(x) for x in (st.q, st.qd, qdd, lam)], fext=gpu(fext), want_fext=True)
    torch.cuda.synchronize()
    assert all(torch.isfinite(o).all() for o in outs)
    idx = np.linspace(0, B - 1, 256).astype(int)
    ref = O.rnea_vjp_fd(desc, st.q[idx], st.qd[idx], qdd[idx], lam[idx], fext=fext[idx], want_fext=True)
    assert vjp_err([cols(o, idx) for o in outs], list(ref)) < 1e-3


@pytest.mark.parametrize("B", [32768, 65536])
def test_derivatives_with_external_forces_full_batch(rbd, B):
    """The adjoint and the tangent of the humanoid's forward dynamics under external forces at the
    derivatives' benchmark size and at 65536 (the tangent on two waves per 64 instances, then on
    one): finite everywhere, 256 states against central differences."""
    desc = W.humanoid()
    m = rbd.Model(desc, 0)
    st = W.states(desc, B, 111)
    rng = np.random.Generator(np.random.PCG64(112))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, desc.n_bodies * 6)))
    gbar = W.cotangent(desc.nv, B, 113)
    q, qd, tau, fx = gpu(st.q), gpu(st.qd), gpu(st.tau), gpu(fext)
    outs = rbd.fwd_dyn_vjp(m, q, qd, tau, gpu(gbar), fext=fx, want_fext=True)
    dq, dqd, dtau, df = (W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.tau, fext))
    dqdd = rbd.fwd_dyn_jvp(m, q, qd, tau, gpu(dq), gpu(dqd), gpu(dtau), fext=fx, dfext=gpu(df))
    torch.cuda.synchronize()
    assert all(torch.isfinite(o).all() for o in outs) and torch.isfinite(dqdd).all()
    idx = np.linspace(0, B - 1, 256).astype(int)
    ref = O.fwd_dyn_vjp_fd(desc, st.q[idx], st.qd[idx], st.tau[idx], gbar[idx], fext=fext[idx])
    assert vjp_err([cols(o, idx) for o in outs], list(ref)) < 1e-3
    refj = O.fwd_dyn_jvp_fd(desc, st.q[idx], st.qd[idx], st.tau[idx], dq[idx], dqd[idx], dtau[idx], fext=fext[idx],
                            dfext=df[idx])
    assert vjp_err([cols(dqdd, idx)], [refj]) < 1e-3


def test_external_forces_at_batch_65536(rbd):
    """fwd_dyn and rnea with external forces on the humanoid batch: a strided sample against the oracle."""
    desc = W.humanoid()
    m = rbd.Model(desc, 0)
    B = 65536
    st = W.states(desc, B, 108)
    rng = np.random.Generator(np.random.PCG64(109))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, desc.n_bodies, 6)))
    q, qd, tau, fx = gpu(st.q), gpu(st.qd), gpu(st.tau), gpu(fext.reshape(B, -1))
    qdd = rbd.fwd_dyn(m, q, qd, tau, fext=fx)
    h = rbd.rnea(m, q, qd, fext=fx)
    torch.cuda.synchronize()
    assert torch.isfinite(qdd).all() and torch.isfinite(h).all()
    idx = np.arange(0, B, 131)
    assert rel_err(cols(qdd, idx), O.fwd_dyn(desc, st.q[idx], st.qd[idx], st.tau[idx], fext=fext[idx])) < 1e-4
    assert rel_err(cols(h, idx), O.rnea(desc, st.q[idx], st.qd[idx], fext=fext[idx])) < 1e-4

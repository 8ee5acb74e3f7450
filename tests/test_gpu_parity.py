"""GPU parity: every entry point of librbd.so against the FP64 oracle.

Inputs are seeded, FP32-rounded synthetic robots and states (workloads); the
oracle runs on exactly those values in FP64. The error of an instance is
normwise, ||x - ref||_inf / ||ref||_inf, and the bar is its maximum over
instances: 1e-4 for qdd and tau, 1e-5 for M, T and J, 1e-3 for the VJP
(against central differences of the oracle).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import rel_err, vjp_err
from tests._models import ALL, MODELS, ROTATED, TREE12, draw  # noqa: F401 (MODELS: the topology list)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_QDD, TOL_TAU, TOL_M, TOL_KIN, TOL_VJP = 1e-4, 1e-4, 1e-5, 1e-5, 1e-3


@pytest.fixture(scope="module")
def rbd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04310_amd as rbd
    rbd.lib()
    return rbd


_models = {}


def model_of(rbd, name):
    if name not in _models:
        desc = ALL[name]()
        _models[name] = (desc, rbd.Model(desc, 0))
    return _models[name]


def gpu(x, ld=None):
    """[B, n] float64 -> CUDA float32 [n, B] (or a [n, ld] buffer viewed as [n, B])."""
    B, n = x.shape
    if ld is None:
        return torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")
    buf = torch.full((n, ld), float("nan"), dtype=torch.float32, device="cuda")
    buf[:, :B] = torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")
    return buf[:, :B]


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy().T


# ---------------------------------------------------------------- small batches, every op
BATCH = 1000  # four 256-lane blocks, the last one ragged


@pytest.mark.parametrize("name", list(ALL))
def test_fwd_dyn_parity(rbd, name):
    desc, m = model_of(rbd, name)
    st = draw(name, desc, BATCH, 201)
    qdd = rbd.fwd_dyn(m, gpu(st.q), gpu(st.qd), gpu(st.tau))
    assert rel_err(host(qdd), O.fwd_dyn(desc, st.q, st.qd, st.tau)) < TOL_QDD


@pytest.mark.parametrize("name", list(ALL))
def test_aba_parity(rbd, name):
    """Articulated-body forward dynamics against the oracle's own ABA and its LTL solve."""
    desc, m = model_of(rbd, name)
    st = draw(name, desc, BATCH, 201)
    qdd = host(rbd.aba(m, gpu(st.q), gpu(st.qd), gpu(st.tau)))
    assert rel_err(qdd, O.fwd_dyn(desc, st.q, st.qd, st.tau, method=O.METHOD_ABA)) < TOL_QDD
    assert rel_err(qdd, O.fwd_dyn(desc, st.q, st.qd, st.tau)) < TOL_QDD


@pytest.mark.parametrize("name", list(ALL))
def test_rnea_parity(rbd, name):
    desc, m = model_of(rbd, name)
    st = draw(name, desc, BATCH, 202)
    qdd_in = W.cotangent(desc.nv, BATCH, 203) * 3.0
    tau = rbd.rnea(m, gpu(st.q), gpu(st.qd), gpu(qdd_in))
    assert rel_err(host(tau), O.rnea(desc, st.q, st.qd, qdd_in)) < TOL_TAU
    h = rbd.rnea(m, gpu(st.q), gpu(st.qd))
    assert rel_err(host(h), O.rnea(desc, st.q, st.qd)) < TOL_TAU


@pytest.mark.parametrize("name", list(ALL))
def test_crba_parity(rbd, name):
    desc, m = model_of(rbd, name)
    st = draw(name, desc, BATCH, 204)
    M = host(rbd.crba(m, gpu(st.q))).reshape(BATCH, desc.nv, desc.nv)
    ref = O.crba(desc, st.q)
    err = (np.abs(M - ref).reshape(BATCH, -1).max(1) / np.abs(ref).reshape(BATCH, -1).max(1)).max()
    assert err < TOL_M
    assert np.array_equal(M, np.swapaxes(M, 1, 2))  # written symmetric, bit for bit


@pytest.mark.parametrize("name", list(ALL))
def test_fk_parity(rbd, name):
    desc, m = model_of(rbd, name)
    st = draw(name, desc, BATCH, 205)
    T = host(rbd.fk(m, gpu(st.q)))
    assert rel_err(T, O.fk(desc, st.q).reshape(BATCH, -1)) < TOL_KIN


@pytest.mark.parametrize("name", list(ALL))
def test_jacobian_parity(rbd, name):
    desc, m = model_of(rbd, name)
    st = draw(name, desc, BATCH, 206)
    rng = np.random.Generator(np.random.PCG64(7))
    frames = np.concatenate([np.arange(desc.n_bodies), rng.integers(0, desc.n_bodies, 3)]).astype(np.int32)
    J = host(rbd.jacobian(m, gpu(st.q), frames))
    ref = O.jacobian(desc, st.q, frames).reshape(BATCH, -1)
    assert rel_err(J, ref) < TOL_KIN
    assert np.all(J[ref == 0.0] == 0.0)  # non-ancestor columns are exact zeros


@pytest.mark.parametrize("name", list(ALL))
def test_fwd_dyn_vjp_parity(rbd, name):
    desc, m = model_of(rbd, name)
    B = 256
    st = draw(name, desc, B, 207)
    gbar = W.cotangent(desc.nv, B, 208)
    gq, gqd, gtau = rbd.fwd_dyn_vjp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), gpu(gbar))
    rq, rqd, rtau = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar, h=1e-6)
    assert vjp_err([host(gq), host(gqd), host(gtau)], [rq, rqd, rtau]) < TOL_VJP
    # any output may be skipped; the others are unchanged
    _, gqd2, gtau2 = rbd.fwd_dyn_vjp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), gpu(gbar), want=(False, True, True))
    assert np.array_equal(host(gqd2), host(gqd)) and np.array_equal(host(gtau2), host(gtau))


@pytest.mark.parametrize("name", ["chain7", "tree12f", "humanoid30", "humanoid30_rot"])
def test_fwd_dyn_vjp_output_subsets(rbd, name):
    """Every non-empty choice of outputs: the kernel variant changes with the choice (values held in
    registers, parked in g_qd and g_tau, or parked in rows of g_q), the results do not."""
    desc, m = model_of(rbd, name)
    B = 300
    st = draw(name, desc, B, 209)
    gbar = W.cotangent(desc.nv, B, 210)
    args = [gpu(x) for x in (st.q, st.qd, st.tau, gbar)]
    full = [host(x) for x in rbd.fwd_dyn_vjp(m, *args)]
    ref = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar, h=1e-6)
    assert vjp_err(full, list(ref)) < TOL_VJP
    for want in [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1) if a or b or c]:
        outs = rbd.fwd_dyn_vjp(m, *args, want=tuple(bool(w) for w in want))
        for w, o, f in zip(want, outs, full):
            assert (o is not None) == bool(w)
            if w:  # the same arithmetic; FP32 contraction may differ between variants
                assert rel_err(host(o), f) < 1e-4, want


@pytest.mark.parametrize("name", list(ALL))
def test_external_force_parity(rbd, name):
    """rnea, fwd_dyn and aba with per-body external forces (world axes) against the oracle."""
    desc, m = model_of(rbd, name)
    st = draw(name, desc, BATCH, 220)
    rng = np.random.Generator(np.random.PCG64(221))
    fext = W._f32(rng.normal(0.0, 5.0, size=(BATCH, desc.n_bodies, 6)))
    fx = gpu(fext.reshape(BATCH, -1))
    qdd_in = W.cotangent(desc.nv, BATCH, 222) * 3.0
    tau = host(rbd.rnea(m, gpu(st.q), gpu(st.qd), gpu(qdd_in), fext=fx))
    assert rel_err(tau, O.rnea(desc, st.q, st.qd, qdd_in, fext=fext)) < TOL_TAU
    h = host(rbd.rnea(m, gpu(st.q), gpu(st.qd), fext=fx))
    assert rel_err(h, O.rnea(desc, st.q, st.qd, fext=fext)) < TOL_TAU
    ref = O.fwd_dyn(desc, st.q, st.qd, st.tau, fext=fext)
    assert rel_err(host(rbd.fwd_dyn(m, gpu(st.q), gpu(st.qd), gpu(st.tau), fext=fx)), ref) < TOL_QDD
    assert rel_err(host(rbd.aba(m, gpu(st.q), gpu(st.qd), gpu(st.tau), fext=fx)), ref) < TOL_QDD


def test_external_weight_support_on_gpu(rbd):
    """Weight-supporting external forces at every CoM: zero holding torque and, with zero torque and
    velocity, zero acceleration by both forward-dynamics kernels."""
    desc, m = model_of(rbd, "humanoid30")
    B = 256
    st = W.states(desc, B, 223)
    T = O.fk(desc, st.q)
    c = T[..., :, 3] + np.einsum("bnij,nj->bni", T[..., :, :3], desc.com)
    f = -desc.mass[None, :, None] * np.asarray(desc.gravity)[None, None, :]
    fext = np.concatenate([np.broadcast_to(f, c.shape), np.cross(c, f)], axis=2)
    fx = gpu(fext.reshape(B, -1))
    zero = np.zeros((B, desc.nv))
    g_scale = np.abs(O.rnea(desc, st.q, zero)).max()
    tau = host(rbd.rnea(m, gpu(st.q), gpu(zero), fext=fx))
    assert np.abs(tau).max() < 1e-4 * g_scale
    # the accelerations that cancel are those of the unsupported robot; they vanish to the tolerance
    # of the parity tests relative to that scale
    a_scale = np.abs(O.fwd_dyn(desc, st.q, zero, zero)).max()
    for fn in (rbd.fwd_dyn, rbd.aba):
        qdd = host(fn(m, gpu(st.q), gpu(zero), gpu(zero), fext=fx))
        assert np.abs(qdd).max() < TOL_QDD * a_scale


@pytest.mark.parametrize("name", list(ALL))
def test_rnea_jvp_parity(rbd, name):
    """Tangent of inverse dynamics along (dq, dqd, dqdd) against the oracle's central differences."""
    desc, m = model_of(rbd, name)
    B = 256 + 17  # a ragged last block
    st = draw(name, desc, B, 250)
    rng = np.random.Generator(np.random.PCG64(251))
    qdd = W._f32(rng.normal(size=st.qd.shape))
    dq, dqd, dqdd = (W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.qd))
    dtau = host(rbd.rnea_jvp(m, gpu(st.q), gpu(st.qd), gpu(qdd), gpu(dq), gpu(dqd), gpu(dqdd)))
    assert vjp_err([dtau], [O.rnea_jvp_fd(desc, st.q, st.qd, qdd, dq, dqd, dqdd)]) < TOL_VJP


@pytest.mark.parametrize("name", ["chain7", "tree12f", "humanoid30", "humanoid30_rot"])
def test_rnea_jvp_with_external_forces(rbd, name):
    """The same with external forces and their tangent, and with the force tangent alone."""
    desc, m = model_of(rbd, name)
    B = 256
    st = draw(name, desc, B, 252)
    rng = np.random.Generator(np.random.PCG64(253))
    qdd = W._f32(rng.normal(size=st.qd.shape))
    dq, dqd, dqdd = (W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.qd))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, 6 * desc.n_bodies)))
    dfext = W._f32(rng.normal(size=fext.shape))
    args = [gpu(x) for x in (st.q, st.qd, qdd, dq, dqd, dqdd)]
    dtau = host(rbd.rnea_jvp(m, *args, fext=gpu(fext), dfext=gpu(dfext)))
    ref = O.rnea_jvp_fd(desc, st.q, st.qd, qdd, dq, dqd, dqdd, fext=fext, dfext=dfext)
    assert vjp_err([dtau], [ref]) < TOL_VJP
    z = [np.zeros_like(x) for x in (dq, dqd, dqdd)]
    only_f = host(rbd.rnea_jvp(m, *args[:3], *[gpu(x) for x in z], dfext=gpu(dfext)))
    assert vjp_err([only_f], [O.rnea_jvp_fd(desc, st.q, st.qd, qdd, *z, dfext=dfext)]) < TOL_VJP


@pytest.mark.parametrize("name", list(ALL))
def test_rnea_vjp_parity(rbd, name):
    """Adjoint of inverse dynamics (g_q, g_qd, g_qdd) against the oracle's central differences."""
    desc, m = model_of(rbd, name)
    B = 256 + 17  # a ragged last block
    st = draw(name, desc, B, 256)
    rng = np.random.Generator(np.random.PCG64(257))
    qdd = W._f32(rng.normal(size=st.qd.shape))
    lam = W.cotangent(desc.nv, B, 258)
    outs = rbd.rnea_vjp(m, gpu(st.q), gpu(st.qd), gpu(qdd), gpu(lam))
    assert vjp_err([host(o) for o in outs], list(O.rnea_vjp_fd(desc, st.q, st.qd, qdd, lam))) < TOL_VJP


@pytest.mark.parametrize("name", ["chain7", "tree12f", "humanoid30", "humanoid30_rot"])
def test_rnea_vjp_with_external_forces(rbd, name):
    """With external forces and the force cotangent; every output subset equals the full call's."""
    desc, m = model_of(rbd, name)
    B = 256
    st = draw(name, desc, B, 259)
    rng = np.random.Generator(np.random.PCG64(260))
    qdd = W._f32(rng.normal(size=st.qd.shape))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, 6 * desc.n_bodies)))
    lam = W.cotangent(desc.nv, B, 261)
    args = [gpu(x) for x in (st.q, st.qd, qdd, lam)]
    full = [host(o) for o in rbd.rnea_vjp(m, *args, fext=gpu(fext), want_fext=True)]
    ref = O.rnea_vjp_fd(desc, st.q, st.qd, qdd, lam, fext=fext, want_fext=True)
    assert vjp_err(full, list(ref)) < TOL_VJP
    for k in range(3):
        want = tuple(i == k for i in range(3))
        part = rbd.rnea_vjp(m, *args, want=want, fext=gpu(fext))
        assert all((p is None) == (not w) for p, w in zip(part, want))
        got = host(part[k])
        assert np.abs(got - full[k]).max() <= 1e-6 * max(np.abs(full[k]).max(), 1e-30)


def test_rnea_vjp_on_gpu_is_dual_to_rnea_jvp_and_its_qdd_block_is_M(rbd):
    """<lam, J dx> = <J^T lam, dx> between the two GPU kernels (forces and force tangents included),
    and g_qdd = M lam with M from the GPU's CRBA."""
    desc, m = model_of(rbd, "humanoid30_rot")
    B = 512
    st = draw("humanoid30_rot", desc, B, 262)
    rng = np.random.Generator(np.random.PCG64(263))
    qdd = W._f32(rng.normal(size=st.qd.shape))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, 6 * desc.n_bodies)))
    dq, dqd, dqdd, df = (W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.qd, fext))
    lam = W.cotangent(desc.nv, B, 264)
    q, qd, a, fx = gpu(st.q), gpu(st.qd), gpu(qdd), gpu(fext)
    jv = host(rbd.rnea_jvp(m, q, qd, a, gpu(dq), gpu(dqd), gpu(dqdd), fext=fx, dfext=gpu(df)))
    g = [host(o) for o in rbd.rnea_vjp(m, q, qd, a, gpu(lam), fext=fx, want_fext=True)]
    terms_l = lam * jv
    terms_r = [gk * xk for gk, xk in zip(g, (dq, dqd, dqdd, df))]
    lhs, rhs = terms_l.sum(1), sum(t.sum(1) for t in terms_r)
    scale = np.abs(terms_l).sum(1) + sum(np.abs(t).sum(1) for t in terms_r)
    assert (np.abs(lhs - rhs) / scale).max() < 1e-4
    M = host(rbd.crba(m, q)).reshape(B, desc.nv, desc.nv)
    Ml = np.einsum("bij,bj->bi", M, lam)
    assert (np.abs(g[2] - Ml).max(1) / np.abs(Ml).max(1)).max() < 1e-5


def test_rnea_autograd(rbd):
    """Backward through rnea_autograd runs the adjoint kernel (forces included); forward-mode AD runs
    the tangent kernel."""
    from torch.autograd import forward_ad as fwAD
    desc, m = model_of(rbd, "tree12f_rot")
    B = 64
    st = draw("tree12f_rot", desc, B, 265)
    rng = np.random.Generator(np.random.PCG64(266))
    qdd = W._f32(rng.normal(size=st.qd.shape))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, desc.n_bodies * 6)))
    lam = W.cotangent(desc.nv, B, 267)
    xs = [gpu(x).requires_grad_(True) for x in (st.q, st.qd, qdd, fext)]
    tau = rbd.rnea_autograd(m, *xs[:3], fext=xs[3])
    (tau * gpu(lam)).sum().backward()
    ref = O.rnea_vjp_fd(desc, st.q, st.qd, qdd, lam, fext=fext, want_fext=True)
    assert vjp_err([host(x.grad) for x in xs], list(ref)) < TOL_VJP
    dq, dqd, dqdd = (W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.qd))
    with fwAD.dual_level():
        out = rbd.rnea_autograd(m, fwAD.make_dual(gpu(st.q), gpu(dq)), fwAD.make_dual(gpu(st.qd), gpu(dqd)),
                                fwAD.make_dual(gpu(qdd), gpu(dqdd)), fext=gpu(fext))
        t = fwAD.unpack_dual(out).tangent
    assert vjp_err([host(t)], [O.rnea_jvp_fd(desc, st.q, st.qd, qdd, dq, dqd, dqdd, fext=fext)]) < TOL_VJP


def test_rnea_jvp_inverts_fwd_dyn_jvp_on_gpu(rbd):
    """ID(q, qd, FD(q, qd, tau)) = tau: the GPU's tangent of inverse dynamics at the GPU's tangent
    of forward dynamics gives back dtau. That dtau is the sum of the state part (dq, dqd) and the
    acceleration part M dqdd, which are often far larger and nearly cancel, so the error is measured
    against the largest of the three; the tangent is linear, so the two parts also add up to the whole."""
    desc, m = model_of(rbd, "humanoid30")
    B = 512
    st = W.states(desc, B, 254)
    rng = np.random.Generator(np.random.PCG64(255))
    dq, dqd, dtau = (W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.tau))
    q, qd = gpu(st.q), gpu(st.qd)
    qdd, dqdd = rbd.fwd_dyn_jvp(m, q, qd, gpu(st.tau), gpu(dq), gpu(dqd), gpu(dtau), want_qdd=True)
    back = host(rbd.rnea_jvp(m, q, qd, qdd, gpu(dq), gpu(dqd), dqdd))
    zq, zv = gpu(np.zeros_like(dq)), gpu(np.zeros_like(dqd))
    state = host(rbd.rnea_jvp(m, q, qd, qdd, gpu(dq), gpu(dqd), zv))
    acc = host(rbd.rnea_jvp(m, q, qd, qdd, zq, zv, dqdd))
    scale = np.maximum.reduce([np.abs(x).max(axis=1) for x in (dtau, state, acc)])
    assert (np.abs(back - dtau).max(axis=1) / scale).max() < TOL_VJP
    assert (np.abs(back - (state + acc)).max(axis=1) / scale).max() < 1e-5


@pytest.mark.parametrize("name", list(ALL))
def test_fwd_dyn_jvp_parity(rbd, name):
    """Forward-mode derivative against the oracle's central differences along the same tangent."""
    desc, m = model_of(rbd, name)
    B = 256
    st = draw(name, desc, B, 230)
    rng = np.random.Generator(np.random.PCG64(231))
    dq, dqd, dtau = (W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.tau))
    args = [gpu(x) for x in (st.q, st.qd, st.tau, dq, dqd, dtau)]
    qdd, dqdd = rbd.fwd_dyn_jvp(m, *args, want_qdd=True)
    ref = O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, dq, dqd, dtau)
    assert vjp_err([host(dqdd)], [ref]) < TOL_VJP
    assert rel_err(host(qdd), O.fwd_dyn(desc, st.q, st.qd, st.tau)) < TOL_QDD
    # without the qdd output the tangent is parked in dqdd itself; same result bit for bit
    assert np.array_equal(host(rbd.fwd_dyn_jvp(m, *args)), host(dqdd))


@pytest.mark.parametrize("name", list(ALL))
def test_derivatives_with_external_forces(rbd, name):
    """The adjoint (g_q, g_qd, g_tau and the force cotangent g_fext) and the tangent (with force
    tangents) of forward dynamics under external forces, against central differences of the
    oracle; the outputs of every subset agree with the full call."""
    desc, m = model_of(rbd, name)
    B = 128
    st = draw(name, desc, B, 260)
    rng = np.random.Generator(np.random.PCG64(261))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, desc.n_bodies * 6)))
    gbar = W.cotangent(desc.nv, B, 262)
    args = [gpu(x) for x in (st.q, st.qd, st.tau, gbar)]
    fx = gpu(fext)
    outs = rbd.fwd_dyn_vjp(m, *args, fext=fx, want_fext=True)
    ref = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar, fext=fext)
    assert vjp_err([host(o) for o in outs], list(ref)) < TOL_VJP
    full = [host(o) for o in outs]
    for want in [(1, 0, 0, 0), (0, 1, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (0, 0, 0, 1), (1, 1, 1, 0)]:
        sub = rbd.fwd_dyn_vjp(m, *args, want=tuple(bool(w) for w in want[:3]), fext=fx, want_fext=bool(want[3]))
        for w, o, f in zip(want, sub, full):
            assert (o is not None) == bool(w)
            if w:
                assert rel_err(host(o), f) < 1e-4, want
    dx = [W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.tau)]
    df = W._f32(rng.normal(size=fext.shape))
    dqdd = host(rbd.fwd_dyn_jvp(m, *args[:3], *[gpu(x) for x in dx], fext=fx, dfext=gpu(df)))
    refj = O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, *dx, fext=fext, dfext=df)
    assert vjp_err([dqdd], [refj]) < TOL_VJP
    # force tangent alone, without forces: M^-1 sum J^T dF
    dz = [np.zeros_like(x) for x in dx]
    d2 = host(rbd.fwd_dyn_jvp(m, *args[:3], *[gpu(x) for x in dz], dfext=gpu(df)))
    assert vjp_err([d2], [O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, *dz, dfext=df)]) < TOL_VJP


def test_autograd_with_external_forces(rbd):
    """Backward through fwd_dyn_autograd reaches the forces; forward-mode carries a force tangent."""
    from torch.autograd import forward_ad as fwAD
    desc, m = model_of(rbd, "tree12f_rot")
    B = 64
    st = draw("tree12f_rot", desc, B, 263)
    rng = np.random.Generator(np.random.PCG64(264))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, desc.n_bodies * 6)))
    gbar = W.cotangent(desc.nv, B, 265)
    q = gpu(st.q).requires_grad_(True)
    f = gpu(fext).requires_grad_(True)
    qdd = rbd.fwd_dyn_autograd(m, q, gpu(st.qd), gpu(st.tau), fext=f)
    (qdd * gpu(gbar)).sum().backward()
    ref = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar, fext=fext)
    assert vjp_err([host(q.grad), host(f.grad)], [ref[0], ref[3]]) < TOL_VJP
    df = W._f32(rng.normal(size=fext.shape))
    with fwAD.dual_level():
        out = rbd.fwd_dyn_autograd(m, gpu(st.q), gpu(st.qd), gpu(st.tau), fext=fwAD.make_dual(gpu(fext), gpu(df)))
        t = fwAD.unpack_dual(out).tangent
    z = [np.zeros_like(x) for x in (st.q, st.qd, st.tau)]
    assert vjp_err([host(t)], [O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, *z, fext=fext, dfext=df)]) < TOL_VJP


# The remaining compiled chains, each with its own random inertial parameters. Together with MODELS
# they cover every topology in the library (a CPU test checks that the two lists stay complete).
EXTRA_TOPOLOGIES = {f"chain{n}": (n, 40 + n) for n in (3, 4, 5, 6, 8)}


@pytest.mark.parametrize("name", list(EXTRA_TOPOLOGIES))
def test_every_compiled_chain(rbd, name):
    """Every row on a chain the per-op tests above do not visit, at a ragged batch of 300."""
    n, seed = EXTRA_TOPOLOGIES[name]
    desc = W.random_tree(list(range(-1, n - 1)), False, seed)
    m = rbd.Model(desc, 0)
    B = 300
    st = W.states(desc, B, seed + 100)
    q, qd, tau = gpu(st.q), gpu(st.qd), gpu(st.tau)
    ref_qdd = O.fwd_dyn(desc, st.q, st.qd, st.tau)
    assert rel_err(host(rbd.fwd_dyn(m, q, qd, tau)), ref_qdd) < TOL_QDD
    assert rel_err(host(rbd.aba(m, q, qd, tau)), ref_qdd) < TOL_QDD
    assert rel_err(host(rbd.rnea(m, q, qd, gpu(ref_qdd))), O.rnea(desc, st.q, st.qd, ref_qdd)) < TOL_TAU
    M = host(rbd.crba(m, q)).reshape(B, n, n)
    ref_M = O.crba(desc, st.q)
    assert (np.abs(M - ref_M).reshape(B, -1).max(1) / np.abs(ref_M).reshape(B, -1).max(1)).max() < TOL_M
    assert rel_err(host(rbd.fk(m, q)), O.fk(desc, st.q).reshape(B, -1)) < TOL_KIN
    frames = np.arange(n, dtype=np.int32)
    assert rel_err(host(rbd.jacobian(m, q, frames)), O.jacobian(desc, st.q, frames).reshape(B, -1)) < TOL_KIN
    gbar = W.cotangent(n, B, seed + 101)
    gs = rbd.fwd_dyn_vjp(m, q, qd, tau, gpu(gbar))
    assert vjp_err([host(x) for x in gs], list(O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar, h=1e-6))) < TOL_VJP
    rng = np.random.Generator(np.random.PCG64(seed + 102))
    dx = [W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.tau)]
    dqdd = host(rbd.fwd_dyn_jvp(m, q, qd, tau, *[gpu(x) for x in dx]))
    assert vjp_err([dqdd], [O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, *dx)]) < TOL_VJP


def test_jvp_vjp_duality_on_gpu(rbd):
    """<gbar, J dx> from the tangent kernel equals <J^T gbar, dx> from the adjoint kernel."""
    desc, m = model_of(rbd, "humanoid30")
    B = 512
    st = W.states(desc, B, 232)
    rng = np.random.Generator(np.random.PCG64(233))
    dx = [W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.tau)]
    gbar = W.cotangent(desc.nv, B, 234)
    dqdd = host(rbd.fwd_dyn_jvp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), *[gpu(x) for x in dx]))
    gs = [host(x) for x in rbd.fwd_dyn_vjp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), gpu(gbar))]
    lhs = np.einsum("bk,bk->b", gbar, dqdd)
    rhs = sum(np.einsum("bk,bk->b", g, x) for g, x in zip(gs, dx))
    scale = sum(np.einsum("bk,bk->b", np.abs(g), np.abs(x)) for g, x in zip(gs, dx))
    assert (np.abs(lhs - rhs) / scale).max() < 1e-4


def test_forward_mode_autograd(rbd):
    """Forward-mode AD (dual tensors) through fwd_dyn_autograd runs the tangent kernel."""
    from torch.autograd import forward_ad as fwAD
    desc, m = model_of(rbd, "tree12f")
    B = 128
    st = W.states(desc, B, 235)
    rng = np.random.Generator(np.random.PCG64(236))
    dq = W._f32(rng.normal(size=st.q.shape))
    qd, tau = gpu(st.qd), gpu(st.tau)
    with fwAD.dual_level():
        out = rbd.fwd_dyn_autograd(m, fwAD.make_dual(gpu(st.q), gpu(dq)), qd, tau)
        t = fwAD.unpack_dual(out).tangent
    ref = O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, dq, np.zeros_like(st.qd), np.zeros_like(st.tau))
    assert vjp_err([host(t)], [ref]) < TOL_VJP


# ---------------------------------------------------------------- layout and edge cases
def test_leading_dimension_larger_than_batch(rbd):
    desc, m = model_of(rbd, "humanoid30")
    B, ld = 300, 512
    st = W.states(desc, B, 210)
    out = torch.full((desc.nv, ld), 7.0, dtype=torch.float32, device="cuda")
    rbd.fwd_dyn(m, gpu(st.q, ld), gpu(st.qd, ld), gpu(st.tau, ld), out=out[:, :B])
    o = out.cpu().numpy()
    assert np.all(o[:, B:] == 7.0)  # padding untouched
    assert rel_err(o[:, :B].T.astype(np.float64), O.fwd_dyn(desc, st.q, st.qd, st.tau)) < TOL_QDD


@pytest.mark.parametrize("B", [0, 1, 255, 257])
def test_batch_edges(rbd, B):
    desc, m = model_of(rbd, "humanoid30")
    st = W.states(desc, max(B, 1), 211)
    if B == 0:
        z = torch.zeros((desc.nq, 0), dtype=torch.float32, device="cuda")
        zv = torch.zeros((desc.nv, 0), dtype=torch.float32, device="cuda")
        assert rbd.fwd_dyn(m, z, zv, zv).shape == (desc.nv, 0)
        assert rbd.rnea_jvp(m, z, zv, zv, z, zv, zv).shape == (desc.nv, 0)
        assert [o.shape for o in rbd.rnea_vjp(m, z, zv, zv, zv)] == [(desc.nq, 0), (desc.nv, 0), (desc.nv, 0)]
        return
    qdd = rbd.fwd_dyn(m, gpu(st.q), gpu(st.qd), gpu(st.tau))
    assert rel_err(host(qdd), O.fwd_dyn(desc, st.q, st.qd, st.tau)) < TOL_QDD
    # the derivatives on a ragged last block (the tangent on two waves per 64 instances, the adjoint
    # parked in LDS)
    rng = np.random.Generator(np.random.PCG64(213))
    dx = [W._f32(rng.normal(size=x.shape)) for x in (st.q, st.qd, st.tau)]
    dqdd = host(rbd.fwd_dyn_jvp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), *[gpu(x) for x in dx]))
    assert vjp_err([dqdd], [O.fwd_dyn_jvp_fd(desc, st.q, st.qd, st.tau, *dx)]) < TOL_VJP
    gbar = W.cotangent(desc.nv, B, 214)
    g = [host(x) for x in rbd.fwd_dyn_vjp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), gpu(gbar))]
    assert vjp_err(g, list(O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar))) < TOL_VJP
    # the tangent and adjoint of inverse dynamics (tau standing in for an acceleration)
    jv = host(rbd.rnea_jvp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), *[gpu(x) for x in dx]))
    assert vjp_err([jv], [O.rnea_jvp_fd(desc, st.q, st.qd, st.tau, *dx)]) < TOL_VJP
    g = [host(x) for x in rbd.rnea_vjp(m, gpu(st.q), gpu(st.qd), gpu(st.tau), gpu(gbar))]
    assert vjp_err(g, list(O.rnea_vjp_fd(desc, st.q, st.qd, st.tau, gbar))) < TOL_VJP


def test_inverse_dynamics_derivatives_with_leading_dimension_larger_than_batch(rbd):
    """rbd_rnea_jvp and rbd_rnea_vjp through the C ABI on [rows, ld] arrays with ld > batch: the
    results match the contiguous call and the padding columns are untouched."""
    import ctypes as C
    desc, m = model_of(rbd, "tree12f")
    B, ld = 300, 448
    st = W.states(desc, B, 215)
    rng = np.random.Generator(np.random.PCG64(216))
    qdd, dqdd, lam = (W._f32(rng.normal(size=st.qd.shape)) for _ in range(3))
    dq, dqd = W._f32(rng.normal(size=st.q.shape)), W._f32(rng.normal(size=st.qd.shape))
    ins = [gpu(x, ld) for x in (st.q, st.qd, qdd, dq, dqd, dqdd, lam)]
    p = [C.c_void_p(x.data_ptr()) for x in ins]
    outs = [torch.full((r, ld), 7.0, dtype=torch.float32, device="cuda") for r in (desc.nv, desc.nq, desc.nv, desc.nv)]
    o = [C.c_void_p(x.data_ptr()) for x in outs]
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = rbd.lib()
    assert L.rbd_rnea_jvp(m.handle, B, ld, p[0], p[1], p[2], None, p[3], p[4], p[5], None, o[0], s) == 0
    assert L.rbd_rnea_vjp(m.handle, B, ld, p[0], p[1], p[2], None, p[6], o[1], o[2], o[3], None, s) == 0
    torch.cuda.synchronize()
    for x in outs:
        assert torch.all(x[:, B:] == 7.0)
    ref_j = rbd.rnea_jvp(m, *[gpu(x) for x in (st.q, st.qd, qdd, dq, dqd, dqdd)])
    ref_v = rbd.rnea_vjp(m, *[gpu(x) for x in (st.q, st.qd, qdd, lam)])
    for got, ref in zip(outs, [ref_j, *ref_v]):
        assert torch.equal(got[:, :B], ref)


def test_special_states(rbd):
    """q = 0, q = +-pi, qd = 0, large qd, joint angles of up to 10^6 rad and exact multiples of
    pi / 2 far from zero, and a scaled (non-unit) quaternion."""
    desc, m = model_of(rbd, "humanoid30")
    st = W.states(desc, 64, 212)
    q, qd, tau = st.q.copy(), st.qd.copy(), st.tau.copy()
    q[0:8, 7:] = 0.0
    q[8:16, 7:] = np.pi
    q[16:24, 7:] = -np.pi
    qd[24:32] = 0.0
    qd[32:40] *= 20.0
    rng = np.random.Generator(np.random.PCG64(219))
    q[40:48, 7:] = rng.uniform(-1e6, 1e6, size=(8, desc.nq - 7))
    q[48:56, 7:] = 0.5 * np.pi * rng.integers(-4000, 4000, size=(8, desc.nq - 7))
    q = W._f32(q)
    qd = W._f32(qd)
    qdd = host(rbd.fwd_dyn(m, gpu(q), gpu(qd), gpu(tau)))
    assert rel_err(qdd, O.fwd_dyn(desc, q, qd, tau)) < TOL_QDD
    q2 = q.copy()
    q2[:, 3:7] *= 2.5  # same rotation
    qdd2 = host(rbd.fwd_dyn(m, gpu(q2), gpu(qd), gpu(tau)))
    assert rel_err(qdd2, O.fwd_dyn(desc, q, qd, tau)) < TOL_QDD


def test_aba_special_states_and_layout(rbd):
    """ABA on q = 0, +-pi, qd = 0, large qd, a scaled quaternion, with ld > batch."""
    desc, m = model_of(rbd, "humanoid30")
    B, ld = 64, 96
    st = W.states(desc, B, 212)
    q, qd = st.q.copy(), st.qd.copy()
    q[0:8, 7:] = 0.0
    q[8:16, 7:] = np.pi
    q[16:24, 7:] = -np.pi
    qd[24:32] = 0.0
    qd[32:40] *= 20.0
    q[40:48, 3:7] *= 0.3
    q, qd = W._f32(q), W._f32(qd)
    out = torch.full((desc.nv, ld), 7.0, dtype=torch.float32, device="cuda")
    rbd.aba(m, gpu(q, ld), gpu(qd, ld), gpu(st.tau, ld), out=out[:, :B])
    o = out.cpu().numpy()
    assert np.all(o[:, B:] == 7.0)
    assert rel_err(o[:, :B].T.astype(np.float64), O.fwd_dyn(desc, q, qd, st.tau, method=O.METHOD_ABA)) < TOL_QDD


def test_zero_quaternion_poisons_only_its_instance(rbd):
    desc, m = model_of(rbd, "humanoid30")
    st = W.states(desc, 64, 213)
    q = st.q.copy()
    q[5, 3:7] = 0.0
    qdd = host(rbd.fwd_dyn(m, gpu(q), gpu(st.qd), gpu(st.tau)))
    assert np.isnan(qdd[5]).any()
    keep = np.arange(64) != 5
    assert np.isfinite(qdd[keep]).all()
    assert rel_err(qdd[keep], O.fwd_dyn(desc, q[keep], st.qd[keep], st.tau[keep])) < TOL_QDD


def test_autograd_function(rbd):
    desc, m = model_of(rbd, "chain7")
    B = 128
    st = W.states(desc, B, 214)
    q = gpu(st.q).requires_grad_(True)
    qd = gpu(st.qd).requires_grad_(True)
    tau = gpu(st.tau).requires_grad_(True)
    gbar = W.cotangent(desc.nv, B, 215)
    qdd = rbd.fwd_dyn_autograd(m, q, qd, tau)
    (qdd * gpu(gbar)).sum().backward()
    rq, rqd, rtau = O.fwd_dyn_vjp_fd(desc, st.q, st.qd, st.tau, gbar)
    assert vjp_err([host(q.grad), host(qd.grad), host(tau.grad)], [rq, rqd, rtau]) < TOL_VJP


def test_batch_limit_is_checked_before_launch(rbd):
    """More than 2^30 instances in one call is an argument error (no pointer is touched)."""
    import ctypes as C
    desc, m = model_of(rbd, "chain7")
    big = (1 << 30) + 1
    p = C.c_void_p(16)  # never dereferenced: the host check fails first
    assert rbd.lib().rbd_fwd_dyn(m.handle, big, big, p, p, p, None, p, None) == 1
    assert b"2^30" in rbd.lib().rbd_last_error()


def test_overlapping_derivative_outputs_are_rejected(rbd):
    """The VJP and JVP keep intermediate values in their outputs, so outputs that share an element are an
    argument error (checked before launch: the addresses below are never dereferenced); outputs that
    interleave in one strided buffer without sharing an element are accepted and exact."""
    import ctypes as C
    desc, m = model_of(rbd, "humanoid30")
    L = rbd.lib()
    p, o = C.c_void_p(1 << 20), C.c_void_p((1 << 20) + 4 * 3)
    i = C.c_void_p(1 << 30)  # inputs elsewhere
    assert L.rbd_fwd_dyn_vjp(m.handle, 8, 8, i, i, i, None, i, None, p, o, None, None) == 1
    assert b"overlap" in L.rbd_last_error()
    assert L.rbd_fwd_dyn_vjp(m.handle, 8, 8, i, i, i, None, i, o, p, None, None, None) == 1
    assert L.rbd_fwd_dyn_vjp(m.handle, 8, 8, i, i, i, None, i, None, p, None, o, None) == 1  # g_f_ext too
    assert L.rbd_fwd_dyn_jvp(m.handle, 8, 8, i, i, i, None, i, i, i, None, o, o, None) == 1
    assert L.rbd_fwd_dyn_vjp(m.handle, 8, 8, p, i, i, None, i, None, o, None, None, None) == 1  # output on q
    assert b"overlaps an input" in L.rbd_last_error()
    B, ld = 8, 16
    st = W.states(desc, B, 217)
    gbar = W.cotangent(desc.nv, B, 218)
    ins = [gpu(x, ld) for x in (st.q, st.qd, st.tau, gbar)]
    buf = torch.full((desc.nv, ld), float("nan"), dtype=torch.float32, device="cuda")
    ptr = buf.data_ptr()
    ip = [C.c_void_p(x.data_ptr()) for x in ins]
    rc = L.rbd_fwd_dyn_vjp(m.handle, B, ld, ip[0], ip[1], ip[2], None, ip[3], None, C.c_void_p(ptr),
                           C.c_void_p(ptr + 4 * B), None, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    _, gqd, gtau = rbd.fwd_dyn_vjp(m, *[gpu(x) for x in (st.q, st.qd, st.tau, gbar)], want=(False, True, True))
    got = host(buf)  # [ld, nv]: rows 0..B-1 hold g_qd, rows B..2B-1 hold g_tau
    assert np.array_equal(got[:B], host(gqd)) and np.array_equal(got[B:], host(gtau))


def test_invalid_arguments_raise(rbd):
    desc, m = model_of(rbd, "chain7")
    st = W.states(desc, 8, 216)
    with pytest.raises(ValueError):
        rbd.fwd_dyn(m, gpu(st.q)[:5], gpu(st.qd), gpu(st.tau))
    with pytest.raises(rbd.RbdError):
        rbd.jacobian(m, gpu(st.q), [0, 99])


# ---------------------------------------------------------------- edge cases of the later entry points
def test_new_entry_points_empty_batch(rbd):
    desc, m = model_of(rbd, "humanoid30")
    zq = torch.zeros((desc.nq, 0), dtype=torch.float32, device="cuda")
    zv = torch.zeros((desc.nv, 0), dtype=torch.float32, device="cuda")
    zf = torch.zeros((6 * desc.n_bodies, 0), dtype=torch.float32, device="cuda")
    zt = torch.zeros((12, 0), dtype=torch.float32, device="cuda")
    assert rbd.aba(m, zq, zv, zv).shape == (desc.nv, 0)
    assert rbd.fwd_dyn(m, zq, zv, zv, fext=zf).shape == (desc.nv, 0)
    assert rbd.rnea(m, zq, zv, fext=zf).shape == (desc.nv, 0)
    assert rbd.fwd_dyn_jvp(m, zq, zv, zv, zq, zv, zv).shape == (desc.nv, 0)
    assert rbd.osc(m, zq, zv, zt, 1.0, 1.0, 1.0).shape == (desc.nv, 0)
    assert rbd.diff_ik(m, zq, zt, 1.0, 0.1).shape == (desc.nv, 0)


def test_new_entry_points_with_padded_leading_dimension(rbd):
    """ld > batch for every array (padding never read or written) on a ragged batch."""
    desc, m = model_of(rbd, "tree12f")
    B, ld = 300, 512
    st = W.states(desc, B, 250)
    rng = np.random.Generator(np.random.PCG64(251))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, desc.n_bodies, 6)))
    q, qd, tau = gpu(st.q, ld), gpu(st.qd, ld), gpu(st.tau, ld)
    fx = gpu(fext.reshape(B, -1), ld)

    def padded(rows):
        return torch.full((rows, ld), 7.0, dtype=torch.float32, device="cuda")

    out = padded(desc.nv)
    rbd.aba(m, q, qd, tau, out=out[:, :B], fext=fx)
    o = out.cpu().numpy()
    assert np.all(o[:, B:] == 7.0)
    assert rel_err(o[:, :B].T.astype(np.float64), O.fwd_dyn(desc, st.q, st.qd, st.tau, fext=fext)) < TOL_QDD
    out = padded(desc.nv)
    rbd.rnea(m, q, qd, out=out[:, :B], fext=fx)
    o = out.cpu().numpy()
    assert np.all(o[:, B:] == 7.0)
    assert rel_err(o[:, :B].T.astype(np.float64), O.rnea(desc, st.q, st.qd, fext=fext)) < TOL_TAU


def test_new_entry_points_reject_bad_arguments(rbd):
    desc, m = model_of(rbd, "chain7")
    st = W.states(desc, 8, 252)
    q, qd, tau = gpu(st.q), gpu(st.qd), gpu(st.tau)
    with pytest.raises(ValueError):  # f_ext rows must be 6 per body
        rbd.fwd_dyn(m, q, qd, tau, fext=torch.zeros((5, 8), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):  # tangent batch differs
        rbd.fwd_dyn_jvp(m, q, qd, tau, gpu(st.q[:4]), qd, tau)
    with pytest.raises(rbd.RbdError):  # non-finite gain
        rbd.osc(m, q, qd, torch.zeros((12, 8), dtype=torch.float32, device="cuda"), float("nan"), 1.0, 1.0)

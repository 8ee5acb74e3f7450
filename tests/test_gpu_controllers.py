"""GPU parity of the controller workloads (differential IK, operational-space control) against
the oracle's plain forms (whose physics, J qdd = a* under forward dynamics and exact task-space
tracking, the oracle pins check), at small sizes on every compiled tree and at the benchmark
shape on a strided sample."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import controllers as CT
from tests._helpers import targets_near

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from tests._models import ALL, draw
# OSC needs J of full row rank: at least six DoFs on the end effector's path
OSC_MODELS = ["chain7", "free1", "tree12f", "humanoid30", "chain7_rot", "tree12f_rot", "humanoid30_rot"]
KP, KD, KN = 50.0, 10.0, 2.0
GAIN, DAMP = 2.0, 0.05
TOL = 1e-4
U32 = 2.0 ** -24  # unit roundoff of FP32


# Both controllers end in a small symmetric solve and a product with J^T. In FP32 an instance's
# error is bounded by a small multiple of u times the problem's conditioning, which near a
# singular arm pose far exceeds 1e-4 / u, so the bar per instance is
#   |x - ref|_inf <= max(TOL |ref|_inf, floor_i)
# with an FP32 error floor computed in FP64 from the oracle's J and M:
#   osc:     8 u cond(J M^-1 J^T) |ref|_inf (measured errors stay below 0.25 u cond |ref|)
#   diff_ik: 8 u cond(A) || |P| (|b| + beta) ||_inf for qd = P b, b = k err, A the normal matrix
#            the kernel solves and beta = k [|p_e| + |p*| (position), 2 (rotation)] the size of
#            the terms whose rounding enters b (a single joint's qd can cancel to ~0).
def floor_osc(desc, q, e, ref):
    J = O.jacobian(desc, q, [e])[:, 0]
    kappa = np.linalg.cond(J @ np.linalg.solve(O.crba(desc, q), np.swapaxes(J, 1, 2)))
    return 8.0 * U32 * kappa * np.abs(ref).max(1)


def floor_ik(desc, q, e, tgt):
    J = O.jacobian(desc, q, [e])[:, 0]
    path = np.abs(J).max(axis=(0, 1)) > 0
    Jp = J[:, :, path]
    b = GAIN * CT.pose_error(desc, q, e, tgt)
    pe = O.fk(desc, q)[:, e, :, 3]
    beta = GAIN * np.concatenate([np.abs(pe) + np.abs(tgt[:, :, 3]), np.full((len(q), 3), 2.0)], axis=1)
    if path.sum() >= 6:
        A = Jp @ np.swapaxes(Jp, 1, 2) + DAMP ** 2 * np.eye(6)
        P = np.swapaxes(Jp, 1, 2) @ np.linalg.inv(A)
    else:
        A = np.swapaxes(Jp, 1, 2) @ Jp + DAMP ** 2 * np.eye(int(path.sum()))
        P = np.linalg.inv(A) @ np.swapaxes(Jp, 1, 2)
    return 8.0 * U32 * np.linalg.cond(A) * np.einsum("bij,bj->bi", np.abs(P), np.abs(b) + beta).max(1)


def within_bar(got, ref, floor):
    """max over instances of |x - ref|_inf / max(TOL |ref|_inf, floor_i); < 1 passes."""
    err = np.abs(got - ref).max(1)
    return float((err / np.maximum(TOL * np.abs(ref).max(1), floor)).max())


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


def gpu(x):
    return torch.tensor(np.ascontiguousarray(x.reshape(len(x), -1).T), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy().T


def case(desc, B, seed, name=""):
    st = draw(name, desc, B, seed)
    e = desc.n_bodies - 1
    tgt = W._f32(targets_near(O.fk(desc, st.q)[:, e], seed + 1))
    return st, e, tgt


@pytest.mark.parametrize("name", list(ALL))
def test_diff_ik_parity(rbd, name):
    desc, m = model_of(rbd, name)
    st, e, tgt = case(desc, 1000, 240, name)
    qd = host(rbd.diff_ik(m, gpu(st.q), gpu(tgt), GAIN, DAMP))
    assert within_bar(qd, CT.diff_ik(desc, st.q, e, tgt, GAIN, DAMP), floor_ik(desc, st.q, e, tgt)) < 1.0


@pytest.mark.parametrize("name", OSC_MODELS)
def test_osc_parity(rbd, name):
    desc, m = model_of(rbd, name)
    st, e, tgt = case(desc, 1000, 241, name)
    tau = host(rbd.osc(m, gpu(st.q), gpu(st.qd), gpu(tgt), KP, KD, KN))
    ref = CT.osc(desc, st.q, st.qd, e, tgt, KP, KD, KN)
    assert within_bar(tau, ref, floor_osc(desc, st.q, e, ref)) < 1.0


def test_controllers_at_batch_65536(rbd):
    """The benchmark shape: every instance finite, a strided sample against the oracle."""
    desc, m = model_of(rbd, "humanoid30")
    B = 65536
    st, e, tgt = case(desc, B, 242)
    q, qd, tg = gpu(st.q), gpu(st.qd), gpu(tgt)
    tau = rbd.osc(m, q, qd, tg, KP, KD, KN)
    v = rbd.diff_ik(m, q, tg, GAIN, DAMP)
    torch.cuda.synchronize()
    assert torch.isfinite(tau).all() and torch.isfinite(v).all()
    idx = np.arange(0, B, 97)
    sel = lambda t: t[:, torch.as_tensor(idx, device="cuda")].double().cpu().numpy().T  # noqa: E731
    qs, qds, ts = st.q[idx], st.qd[idx], tgt[idx]
    ref = CT.osc(desc, qs, qds, e, ts, KP, KD, KN)
    assert within_bar(sel(tau), ref, floor_osc(desc, qs, e, ref)) < 1.0
    assert within_bar(sel(v), CT.diff_ik(desc, qs, e, ts, GAIN, DAMP), floor_ik(desc, qs, e, ts)) < 1.0


@pytest.mark.parametrize("name,frame", [("humanoid30", 6), ("humanoid30", 22), ("chain7", 3), ("humanoid30_rot", 22)])
def test_controllers_for_other_frames(rbd, name, frame):
    """Controllers of a frame other than the last body (a foot, the other hand, the middle of the
    arm): kernels compiled for that frame at run time, against the oracle's plain forms."""
    desc, m = model_of(rbd, name)
    B = 500
    st = draw(name, desc, B, 244 + frame)
    tgt = W._f32(targets_near(O.fk(desc, st.q)[:, frame], 245 + frame))
    qd = host(rbd.diff_ik(m, gpu(st.q), gpu(tgt), GAIN, DAMP, frame=frame))
    assert within_bar(qd, CT.diff_ik(desc, st.q, frame, tgt, GAIN, DAMP), floor_ik(desc, st.q, frame, tgt)) < 1.0
    path = O.jacobian(desc, st.q[:1], [frame])[0, 0].any(axis=0).sum()
    if path >= 6:
        tau = host(rbd.osc(m, gpu(st.q), gpu(st.qd), gpu(tgt), KP, KD, KN, frame=frame))
        ref = CT.osc(desc, st.q, st.qd, frame, tgt, KP, KD, KN)
        assert within_bar(tau, ref, floor_osc(desc, st.q, frame, ref)) < 1.0


def test_controller_arguments_are_checked(rbd):
    desc, m = model_of(rbd, "chain7")
    st, e, tgt = case(desc, 8, 243)
    with pytest.raises(rbd.RbdError) as ex:
        rbd.diff_ik(m, gpu(st.q), gpu(tgt), GAIN, DAMP, frame=7)
    assert ex.value.status == 1
    with pytest.raises(rbd.RbdError):
        rbd.diff_ik(m, gpu(st.q), gpu(tgt), GAIN, -1.0)

"""Trees outside the compiled topology list: the library compiles their kernels at run time
(hiprtc), caches the code objects and runs every row through them. The PREBUILT shapes load
code objects that the build compiled into the library's cache with the same compiler path; one
small tree is compiled on the GPU machine itself, into an empty cache directory. Every model has
random joint-origin rotations, gravity in a random direction and joint angles up to 1000 rad."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import controllers as CT
from paper_2604_04310_amd.build import PREBUILT
from tests._helpers import rel_err, targets_near, vjp_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_QDD, TOL_TAU, TOL_M, TOL_KIN, TOL_VJP = 1e-4, 1e-4, 1e-5, 1e-5, 1e-3
TREES = {name: (fl, par, 70 + k) for k, (name, (fl, par)) in enumerate(PREBUILT.items())}


@pytest.fixture(scope="module")
def rbd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04310_amd as rbd
    rbd.lib()
    return rbd


def gpu(x):
    return torch.tensor(np.ascontiguousarray(x.reshape(len(x), -1).T), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy().T


def desc_of(fl, par, seed):
    return W.random_tree(par, fl, seed, rotated=True, gravity=W.tilted_gravity(seed + 1))


def check_every_row(rbd, m, desc, seed, B=300):
    """fwd_dyn, aba, rnea, crba, fk, jacobian, external forces, vjp, jvp and the controllers of the
    last body against the oracle, at a ragged batch."""
    st = W.states(desc, B, seed + 100, q_range=1000.0)
    q, qd, tau = gpu(st.q), gpu(st.qd), gpu(st.tau)
    ref_qdd = O.fwd_dyn(desc, st.q, st.qd, st.tau)
    assert rel_err(host(rbd.fwd_dyn(m, q, qd, tau)), ref_qdd) < TOL_QDD
    assert rel_err(host(rbd.aba(m, q, qd, tau)), ref_qdd) < TOL_QDD
    qdd_in = W.cotangent(desc.nv, B, seed + 101) * 3.0
    assert rel_err(host(rbd.rnea(m, q, qd, gpu(qdd_in))), O.rnea(desc, st.q, st.qd, qdd_in)) < TOL_TAU
    assert rel_err(host(rbd.rnea(m, q, qd)), O.rnea(desc, st.q, st.qd)) < TOL_TAU
    nv = desc.nv
    M = host(rbd.crba(m, q)).reshape(B, nv, nv)
    ref_M = O.crba(desc, st.q)
    assert (np.abs(M - ref_M).reshape(B, -1).max(1) / np.abs(ref_M).reshape(B, -1).max(1)).max() < TOL_M
    assert rel_err(host(rbd.fk(m, q)), O.fk(desc, st.q).reshape(B, -1)) < TOL_KIN
    frames = np.arange(desc.n_bodies, dtype=np.int32)
    assert rel_err(host(rbd.jacobian(m, q, frames)), O.jacobian(desc, st.q, frames).reshape(B, -1)) < TOL_KIN
    rng = np.random.Generator(np.random.PCG64(seed + 102))
    fext = W._f32(rng.normal(0.0, 5.0, size=(B, desc.n_bodies, 6)))
    fx = gpu(fext.reshape(B, -1))
    ref_ext = O.fwd_dyn(desc, st.q, st.qd, st.tau, fext=fext)
    assert rel_err(host(rbd.fwd_dyn(m, q, qd, tau, fext=fx)), ref_ext) < TOL_QDD
    assert rel_err(host(rbd.aba(m, q, qd, tau, fext=fx)), ref_ext) < TOL_QDD
    assert rel_err(host(rbd.rnea(m, q, qd, fext=fx)), O.rnea(desc, st.q, st.qd, fext=fext)) < TOL_TAU
    Bd = 128
    gbar = W.cotangent(nv, Bd, seed + 103)
    args = [gpu(x[:Bd]) for x in (st.q, st.qd, st.tau)]
    gs = rbd.fwd_dyn_vjp(m, *args, gpu(gbar))
    ref = O.fwd_dyn_vjp_fd(desc, st.q[:Bd], st.qd[:Bd], st.tau[:Bd], gbar, h=1e-6)
    assert vjp_err([host(x) for x in gs], list(ref)) < TOL_VJP
    dx = [W._f32(rng.normal(size=x[:Bd].shape)) for x in (st.q, st.qd, st.tau)]
    dqdd = host(rbd.fwd_dyn_jvp(m, *args, *[gpu(x) for x in dx]))
    assert vjp_err([dqdd], [O.fwd_dyn_jvp_fd(desc, st.q[:Bd], st.qd[:Bd], st.tau[:Bd], *dx)]) < TOL_VJP
    # the derivatives with external forces
    fb = fext[:Bd].reshape(Bd, -1)
    outs = rbd.fwd_dyn_vjp(m, *args, gpu(gbar), fext=gpu(fb), want_fext=True)
    ref = O.fwd_dyn_vjp_fd(desc, st.q[:Bd], st.qd[:Bd], st.tau[:Bd], gbar, fext=fb)
    assert vjp_err([host(x) for x in outs], list(ref)) < TOL_VJP
    df = W._f32(rng.normal(size=fb.shape))
    dqdd = host(rbd.fwd_dyn_jvp(m, *args, *[gpu(x) for x in dx], fext=gpu(fb), dfext=gpu(df)))
    refj = O.fwd_dyn_jvp_fd(desc, st.q[:Bd], st.qd[:Bd], st.tau[:Bd], *dx, fext=fb, dfext=df)
    assert vjp_err([dqdd], [refj]) < TOL_VJP
    # controllers of the last body, against the oracle's plain forms with the FP32 error floor of the
    # controller tests (conditioning of the task-space solve)
    from tests.test_gpu_controllers import DAMP, GAIN, KD, KN, KP, floor_ik, floor_osc, within_bar
    e = desc.n_bodies - 1
    tgt = W._f32(targets_near(O.fk(desc, st.q)[:, e], seed + 104))
    v = host(rbd.diff_ik(m, q, gpu(tgt), GAIN, DAMP))
    assert within_bar(v, CT.diff_ik(desc, st.q, e, tgt, GAIN, DAMP), floor_ik(desc, st.q, e, tgt)) < 1.0
    path = O.jacobian(desc, st.q[:1], [e])[0, 0].any(axis=0).sum()
    if path >= 6:  # OSC needs J of full row rank
        t = host(rbd.osc(m, q, qd, gpu(tgt), KP, KD, KN))
        ref_t = CT.osc(desc, st.q, st.qd, e, tgt, KP, KD, KN)
        assert within_bar(t, ref_t, floor_osc(desc, st.q, e, ref_t)) < 1.0


@pytest.mark.parametrize("name", list(TREES))
def test_new_topology_every_row(rbd, name):
    fl, par, seed = TREES[name]
    desc = desc_of(fl, par, seed)
    m = rbd.Model(desc, 0)
    assert m.topology.startswith("jit_"), m.topology  # not one of the compiled topologies
    check_every_row(rbd, m, desc, seed)


def test_compiled_on_the_device_host(rbd, tmp_path, monkeypatch):
    """A topology found in no cache: each kernel is compiled here with hiprtc, into an empty cache
    directory, when it is first launched, then served like any other; a second model of the
    topology reuses the loaded kernels."""
    monkeypatch.setenv("RBD_JIT_CACHE", str(tmp_path))

    def n_code_objects():
        return len([f for f in os.listdir(tmp_path) if f.endswith(".hsaco")])

    desc = desc_of(False, [-1, 0, 0], 90)
    print(f"compiling tree3 into {tmp_path}", flush=True)
    m = rbd.Model(desc, 0)
    assert m.topology.startswith("jit_3_")
    assert n_code_objects() == 0  # nothing is compiled before it is used
    st = W.states(desc, 64, 92)
    qdd = host(rbd.fwd_dyn(m, gpu(st.q), gpu(st.qd), gpu(st.tau)))
    assert rel_err(qdd, O.fwd_dyn(desc, st.q, st.qd, st.tau)) < TOL_QDD
    assert n_code_objects() == 1
    check_every_row(rbd, m, desc, 90)
    assert 10 <= n_code_objects() <= rbd.N_KERNELS + 6  # a controller frame or two may add its own
    m2 = rbd.Model(desc_of(False, [-1, 0, 0], 91), 0)
    assert m2.topology == m.topology

"""The continuous-batching server on the GPU: every request's result is the same
alone and in a mix (bit for bit: each instance runs the same code in its own
lane), matches the oracle, and completes exactly once under memory pressure."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests._helpers import rel_err, vjp_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04310_amd as rbd
    descs = {"chain7": W.chain(7), "humanoid30": W.humanoid()}
    models = {k: rbd.Model(d, 0) for k, d in descs.items()}
    return rbd, descs, models


def make_requests(rbd, descs, n, seed):
    """A seeded mix: robots 50/50, ops 60/25/15 fwd_dyn/rnea/vjp, batch log-uniform in [1, 4096]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for k in range(n):
        name = "chain7" if rng.random() < 0.5 else "humanoid30"
        u = rng.random()
        op = rbd.OP_FWD_DYN if u < 0.60 else (rbd.OP_RNEA if u < 0.85 else rbd.OP_FWD_DYN_VJP)
        B = int(np.clip(round(np.exp(rng.uniform(0, np.log(4096)))), 1, 4096))
        d = descs[name]
        st = W.states(d, B, 1000 + seed * 1000 + k)
        if op == rbd.OP_FWD_DYN:
            ins = [st.q, st.qd, st.tau]
        elif op == rbd.OP_RNEA:
            ins = [st.q, st.qd, W.cotangent(d.nv, B, 7 + k)]
        else:
            ins = [st.q, st.qd, st.tau, W.cotangent(d.nv, B, 9 + k)]
        reqs.append((name, op, [x.astype(np.float32) for x in ins]))
    return reqs


def run_all(srv, models, reqs, together):
    results = [None] * len(reqs)
    if together:
        tickets = [srv.submit(models[n], op, ins) for n, op, ins in reqs]
        for k, (t, outs) in enumerate(tickets):
            assert srv.wait(t, 60.0) == 0
            results[k] = outs
    else:
        for k, (n, op, ins) in enumerate(reqs):
            t, outs = srv.submit(models[n], op, ins)
            assert srv.wait(t, 60.0) == 0
            results[k] = outs
    return results


def check_oracle(rbd, descs, reqs, results, every=5):
    for k in range(0, len(reqs), every):
        name, op, ins = reqs[k]
        d = descs[name]
        x = [a.astype(np.float64) for a in ins]
        out = [o.astype(np.float64) for o in results[k]]
        if op == rbd.OP_FWD_DYN:
            assert rel_err(out[0], O.fwd_dyn(d, *x)) < 1e-4
        elif op == rbd.OP_RNEA:
            assert rel_err(out[0], O.rnea(d, x[0], x[1], x[2])) < 1e-4
        else:
            n = min(len(x[0]), 32)
            ref = O.fwd_dyn_vjp_fd(d, x[0][:n], x[1][:n], x[2][:n], x[3][:n])
            assert vjp_err([o[:n] for o in out], ref) < 1e-3


def test_alone_equals_mix(env):
    rbd, descs, models = env
    reqs = make_requests(rbd, descs, 48, 1)
    # a short gather window makes the packing of the mixed phase independent of thread timing
    srv = rbd.Server(arena_bytes=512 << 20, n_streams=4, max_batch_requests=256, max_wait_us=2000.0)
    alone = run_all(srv, models, reqs, together=False)
    mixed = run_all(srv, models, reqs, together=True)
    st = srv.stats()
    srv.close()
    for a, b in zip(alone, mixed):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    assert st["requests"] == 2 * len(reqs)
    assert st["launches"] < st["requests"]  # the mix was packed into fewer launches
    check_oracle(rbd, descs, reqs, mixed)


def test_admission_under_a_small_arena(env):
    """An arena that holds only a couple of requests: the rest queue, all complete once."""
    rbd, descs, models = env
    reqs = make_requests(rbd, descs, 24, 2)
    need = max(sum(x.nbytes for x in ins) * 2 for _, _, ins in reqs)
    srv = rbd.Server(arena_bytes=int(need * 1.5) + (1 << 16), n_streams=2, max_batch_requests=64)
    mixed = run_all(srv, models, reqs, together=True)
    st = srv.stats()
    srv.close()
    assert st["requests"] == len(reqs)
    ref_srv = rbd.Server(arena_bytes=256 << 20, n_streams=1, per_request=True, use_graphs=False)
    alone = run_all(ref_srv, models, reqs, together=False)
    ref_srv.close()
    for a, b in zip(alone, mixed):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("graphs,per_request", [(False, False), (True, False), (False, True)])
def test_modes_agree_with_direct_calls(env, graphs, per_request):
    rbd, descs, models = env
    d, m = descs["humanoid30"], models["humanoid30"]
    B = 777
    st = W.states(d, B, 55)
    srv = rbd.Server(use_graphs=graphs, per_request=per_request)
    t, outs = srv.submit(m, rbd.OP_FWD_DYN, [st.q.astype(np.float32), st.qd.astype(np.float32),
                                            st.tau.astype(np.float32)])
    assert srv.wait(t, 60.0) == 0
    srv.close()
    g = lambda x: torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")
    direct = rbd.fwd_dyn(m, g(st.q), g(st.qd), g(st.tau)).cpu().numpy().T
    assert np.array_equal(outs[0], direct)


def test_server_rejects_bad_requests(env):
    rbd, descs, models = env
    srv = rbd.Server(arena_bytes=1 << 20)
    d, m = descs["humanoid30"], models["humanoid30"]
    st = W.states(d, 4096, 3)
    with pytest.raises(rbd.RbdError):  # can never fit a 1 MiB arena
        srv.submit(m, rbd.OP_FWD_DYN, [st.q, st.qd, st.tau])
    with pytest.raises(rbd.RbdError):
        srv.wait(123456, 0.0)
    srv.close()


def test_groups_split_at_the_byte_cap(env):
    """Requests totalling far more than one launch group may hold (16 MiB of staged data) are
    served in several packed launches, each bit-identical to the direct call."""
    rbd, descs, models = env
    d, m = descs["humanoid30"], models["humanoid30"]
    B = 4096  # 4096 x (36 + 35 + 35 + 35) x 4 B = 2.3 MB staged per request
    reqs = []
    for k in range(16):
        st = W.states(d, B, 300 + k)
        reqs.append(("humanoid30", rbd.OP_FWD_DYN, [x.astype(np.float32) for x in (st.q, st.qd, st.tau)]))
    # a gather window longer than the submission loop: packing then depends only on the cap
    srv = rbd.Server(arena_bytes=1 << 30, n_streams=2, max_batch_requests=1024, max_wait_us=50000.0)
    outs = run_all(srv, models, reqs, together=True)
    st = srv.stats()
    srv.close()
    assert st["requests"] == len(reqs)
    assert 3 <= st["launches"] < len(reqs)  # 37 MB of staging: at least three groups, still packed
    g = lambda x: torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")  # noqa: E731
    for (_, _, ins), o in zip(reqs, outs):
        direct = rbd.fwd_dyn(m, *[g(x) for x in ins]).cpu().numpy().T
        assert np.array_equal(o[0], direct)


def test_a_new_model_never_replays_a_destroyed_models_graphs(env):
    """Captured launches are cached per model; after a model is destroyed, a new model (possibly at
    the same host address) gets its own, so its results match its direct calls bit for bit."""
    rbd, descs, _ = env
    srv = rbd.Server(arena_bytes=64 << 20, n_streams=1, use_graphs=True)
    g = lambda x: torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")  # noqa: E731
    for seed in (61, 62, 63):
        d = W.random_tree([-1, 0, 1, 2, 3, 4, 5], False, seed)  # same topology, new parameters
        m = rbd.Model(d, 0)
        st = W.states(d, 300, seed)
        ins = [x.astype(np.float32) for x in (st.q, st.qd, st.tau)]
        t, outs = srv.submit(m, rbd.OP_FWD_DYN, ins)
        assert srv.wait(t, 60.0) == 0
        direct = rbd.fwd_dyn(m, *[g(x) for x in ins]).cpu().numpy().T
        assert np.array_equal(outs[0], direct)
        m.close()
    srv.close()


def test_native_load_generator_on_the_device(env):
    """rbd_diag_serve_load against the device executor: closed loop and Poisson arrivals complete
    every request with status OK, and the server counts each request once."""
    rbd, descs, models = env
    reqs = make_requests(rbd, descs, 12, 7)
    specs = [(models[n], op, ins) for n, op, ins in reqs]
    srv = rbd.Server(arena_bytes=64 << 20, n_streams=3, max_batch_requests=64)
    srv.reset_stats()
    wall, failed = srv.load(specs, 240, rate=0.0, window=48, seed=1)
    st = srv.stats()
    assert failed == 0 and st["requests"] == 240 and 0 < st["launches"] <= 240 and wall > 0
    # the device timeline: every group timed, kernels inside the active time, overlap inside kernel time
    assert st["groups_timed"] == st["launches"]
    assert 0 < st["gpu_kernel_s"] <= st["gpu_kernel_sum_s"] + 1e-9
    assert st["gpu_kernel_overlap_s"] <= st["gpu_kernel_s"] + 1e-9
    assert st["gpu_kernel_s"] <= st["gpu_active_s"] + 1e-9 and st["gpu_active_s"] <= 1.05 * wall + 1e-3
    assert 0 < st["gpu_copy_s"] <= st["gpu_active_s"] + 1e-9
    srv.reset_stats()
    wall, failed = srv.load(specs, 120, rate=5000.0, window=24, seed=2)
    assert failed == 0 and srv.stats()["requests"] == 120
    srv.close()

"""The serving scheduler on the CPU: the host executor runs the same admission, packing,
completion, cancellation and failure handling over host memory, with a fixed stand-in computation
(output a of instance i: out_a[i][c] = in_(a mod n_in)[i][c mod rows] + 1000 a), so every request's
results show that they came from its own inputs."""
from __future__ import annotations

import os
import threading

import numpy as np
import pytest

import workloads as W

OK, LAUNCH, CANCELLED = 0, 4, 9


@pytest.fixture(scope="module")
def rbd():
    import paper_2604_04310_amd as rbd
    if not os.path.exists(rbd.LIB_PATH):
        pytest.skip("librbd.so not built")
    rbd.lib()
    return rbd


@pytest.fixture(scope="module")
def models(rbd):
    return {"chain7": rbd.Model(W.chain(7), -1), "humanoid30": rbd.Model(W.humanoid(), -1)}


def expected(rbd, model, op, ins):
    in_rows, out_rows = rbd.op_shapes(model, op)
    outs = []
    for a, r in enumerate(out_rows):
        src = ins[a % len(ins)]
        cols = np.arange(r) % in_rows[a % len(ins)]
        outs.append(src[:, cols] + np.float32(1000.0 * a))
    return outs


def make_request(rbd, model, op, batch, seed):
    in_rows, _ = rbd.op_shapes(model, op)
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.normal(size=(batch, r)).astype(np.float32) for r in in_rows]


def test_host_only_model_has_no_kernels(rbd, models):
    import ctypes as C
    m = models["chain7"]
    assert m.topology == "chain7"
    L = rbd.lib()
    p = C.c_void_p(16)
    assert L.rbd_fwd_dyn(m.handle, 1, 1, p, p, p, None, p, None) == 3  # RBD_E_NODEVICE
    assert b"host-only" in L.rbd_last_error()


def test_every_request_gets_its_own_results(rbd, models):
    """A mix of robots, operations and batch sizes from two client threads: every ticket completes
    once, with its own inputs' results, across many packed groups."""
    # a gather window makes packing certain: without one, three workers can keep up with two
    # Python clients and every request may run alone
    srv = rbd.Server(executor=rbd.EXEC_HOST, arena_bytes=4 << 20, n_streams=3, max_batch_requests=64,
                     max_wait_us=3000.0)
    rng = np.random.Generator(np.random.PCG64(1))
    plan = [(list(models)[int(rng.integers(2))], int(rng.choice([rbd.OP_FWD_DYN, rbd.OP_RNEA, rbd.OP_FWD_DYN_VJP])),
             int(np.clip(round(np.exp(rng.uniform(0, np.log(2048)))), 1, 2048))) for _ in range(400)]
    results = {}
    lock = threading.Lock()

    def client(part):
        for k in part:
            name, op, B = plan[k]
            ins = make_request(rbd, models[name], op, B, k)
            t, outs = srv.submit(models[name], op, ins)
            with lock:
                results[k] = (t, ins, outs)

    threads = [threading.Thread(target=client, args=(range(i, len(plan), 2),)) for i in range(2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert len({t for t, _, _ in results.values()}) == len(plan)
    for k, (t, ins, outs) in results.items():
        assert srv.wait(t, 30.0) == OK
        name, op, _ = plan[k]
        for got, ref in zip(outs, expected(rbd, models[name], op, ins)):
            assert np.array_equal(got, ref), k
    st = srv.stats()
    assert st["requests"] == len(plan) and 0 < st["launches"] < len(plan)  # requests were packed
    with pytest.raises(rbd.RbdError):
        srv.wait(results[0][0], 1.0)  # a ticket is waited once
    srv.close()


def test_a_failed_group_fails_only_its_own_requests(rbd, models):
    """The third launch group fails (injected from the host before anything of it runs): exactly
    its requests report RBD_E_LAUNCH and leave their outputs untouched; every other request, before
    and after it, completes with its own results."""
    srv = rbd.Server(executor=rbd.EXEC_HOST, arena_bytes=8 << 20, n_streams=1, max_batch_requests=4,
                     fail_group=3)
    m = models["humanoid30"]
    reqs = []
    for k in range(40):
        ins = make_request(rbd, m, rbd.OP_FWD_DYN, 16 + k, 100 + k)
        # sentinel: a failed request's outputs are not written
        t, outs = srv.submit(m, rbd.OP_FWD_DYN, ins, outputs=[np.full((16 + k, m.nv), -7.0, np.float32)])
        reqs.append((t, ins, outs))
    status = [srv.wait(t, 30.0) for t, _, _ in reqs]
    failed = [k for k, s in enumerate(status) if s != OK]
    assert failed and all(status[k] == LAUNCH for k in failed)
    assert 1 <= len(failed) <= 4 and failed == list(range(failed[0], failed[-1] + 1))  # one group
    for k, (t, ins, outs) in enumerate(reqs):
        if k in failed:
            assert np.all(outs[0] == -7.0)
        else:
            assert np.array_equal(outs[0], expected(rbd, m, rbd.OP_FWD_DYN, ins)[0])
    srv.close()


def test_cancel_a_queued_request(rbd, models):
    """With a long gather window the requests wait in the queue: one of them is cancelled (it
    completes at once as RBD_E_CANCELLED, outputs untouched), the others run; a request that has
    left the queue can no longer be cancelled."""
    srv = rbd.Server(executor=rbd.EXEC_HOST, arena_bytes=8 << 20, n_streams=2, max_batch_requests=64,
                     max_wait_us=300000.0)
    m = models["chain7"]
    reqs = []
    for k in range(6):
        ins = make_request(rbd, m, rbd.OP_RNEA, 32, 200 + k)
        t, outs = srv.submit(m, rbd.OP_RNEA, ins, outputs=[np.full((32, m.nv), -7.0, np.float32)])
        reqs.append((t, ins, outs))
    srv.cancel(reqs[2][0])
    assert srv.wait(reqs[2][0], 0.0) == CANCELLED
    assert np.all(reqs[2][2][0] == -7.0)
    for k in (0, 1, 3, 4, 5):
        t, ins, outs = reqs[k]
        assert srv.wait(t, 30.0) == OK
        assert np.array_equal(outs[0], expected(rbd, m, rbd.OP_RNEA, ins)[0])
    t, _ = srv.submit(m, rbd.OP_RNEA, make_request(rbd, m, rbd.OP_RNEA, 8, 300))
    assert srv.wait(t, 30.0) == OK
    with pytest.raises(rbd.RbdError):
        srv.cancel(t)  # finished and waited: unknown now
    srv.close()


def test_admission_by_memory_and_shutdown(rbd, models):
    """A tiny arena admits one large request at a time; requests bigger than the arena are refused
    at submit; destroying the server drains whatever is still queued."""
    srv = rbd.Server(executor=rbd.EXEC_HOST, arena_bytes=1 << 20, n_streams=4, max_batch_requests=16)
    m = models["humanoid30"]
    big = (1 << 20) // (4 * (m.nq + 3 * m.nv)) // 3  # a request fills about a third of the arena
    with pytest.raises(rbd.RbdError):
        srv.submit(m, rbd.OP_FWD_DYN, make_request(rbd, m, rbd.OP_FWD_DYN, 4096, 1))
    reqs = []
    for k in range(12):
        ins = make_request(rbd, m, rbd.OP_FWD_DYN, big, 400 + k)
        reqs.append((*srv.submit(m, rbd.OP_FWD_DYN, ins), ins))
    for t, outs, ins in reqs:
        assert srv.wait(t, 30.0) == OK
        assert np.array_equal(outs[0], expected(rbd, m, rbd.OP_FWD_DYN, ins)[0])
    late = [srv.submit(m, rbd.OP_RNEA, make_request(rbd, m, rbd.OP_RNEA, 64, 500 + k)) for k in range(8)]
    srv.close()  # drains the queue before freeing
    assert all(np.isfinite(outs[0]).all() for _, outs in late)


def test_host_executor_validation(rbd, models):
    with pytest.raises(rbd.RbdError):
        rbd.Server(executor=7)
    with pytest.raises(rbd.RbdError):
        rbd.Server(executor=rbd.EXEC_HOST, fail_group=-1)


def test_native_load_generator(rbd, models):
    """rbd_diag_serve_load drives a server from native threads: closed loop and Poisson arrivals
    both complete every request, the server's counters see each of them once, and a bad spec or an
    injected group failure is reported."""
    srv = rbd.Server(executor=rbd.EXEC_HOST, arena_bytes=8 << 20, n_streams=4, max_batch_requests=64)
    specs = []
    for k in range(6):
        name = "chain7" if k % 2 else "humanoid30"
        op = [rbd.OP_FWD_DYN, rbd.OP_RNEA, rbd.OP_FWD_DYN_VJP][k % 3]
        specs.append((models[name], op, make_request(rbd, models[name], op, 7 + 60 * k, 600 + k)))
    n_inst = sum(s[2][0].shape[0] for s in specs)
    srv.reset_stats()
    wall, failed = srv.load(specs, 600, rate=0.0, window=16, seed=3)
    st = srv.stats()
    assert failed == 0 and wall > 0
    assert st["requests"] == 600 and st["instances"] == 100 * n_inst and st["launches"] <= 600
    assert st["groups_timed"] == 0 and st["gpu_kernel_s"] == 0.0  # no device timeline without a device
    srv.reset_stats()
    wall, failed = srv.load(specs, 300, rate=20000.0, window=64, seed=4)
    assert failed == 0 and srv.stats()["requests"] == 300
    assert wall >= 0.5 * 300 / 20000.0  # arrivals are paced, not sent at once
    with pytest.raises(ValueError):
        srv.load([(models["chain7"], rbd.OP_FWD_DYN, [np.zeros((4, 7), np.float32)])], 1)
    srv.close()
    bad = rbd.Server(executor=rbd.EXEC_HOST, arena_bytes=8 << 20, n_streams=1, max_batch_requests=1,
                     fail_group=5)
    wall, failed = bad.load(specs[:1], 20, window=4)
    assert failed == 1  # one request per group, the fifth group fails
    bad.close()


def test_group_byte_cap(rbd, models):
    """max_group_bytes bounds a launch group: requests of 144 KiB under a 256 KiB cap run one per
    group even when a gather window has all of them queued, and each still gets its own results."""
    m = models["humanoid30"]
    B = 256  # (nq + 2 nv + nv) floats per instance: 144 KiB per request
    srv = rbd.Server(executor=rbd.EXEC_HOST, arena_bytes=64 << 20, n_streams=1, max_batch_requests=64,
                     max_wait_us=20000.0, max_group_bytes=256 << 10)
    reqs = []
    for k in range(10):
        ins = make_request(rbd, m, rbd.OP_FWD_DYN, B, 800 + k)
        reqs.append((*srv.submit(m, rbd.OP_FWD_DYN, ins), ins))
    for t, outs, ins in reqs:
        assert srv.wait(t, 30.0) == OK
        assert np.array_equal(outs[0], expected(rbd, m, rbd.OP_FWD_DYN, ins)[0])
    assert srv.stats()["launches"] == 10
    srv.close()


def test_many_clients_cancels_and_shutdown(rbd, models):
    """Eight client threads submit a random mix while one of them cancels some of its queued
    requests: every request completes exactly once, either cancelled (outputs untouched) or with
    its own results, the counters match, and destroying the server with requests still queued
    drains them."""
    srv = rbd.Server(executor=rbd.EXEC_HOST, arena_bytes=2 << 20, n_streams=4, max_batch_requests=16,
                     max_wait_us=200.0)
    names = list(models)
    done, errors = [], []
    lock = threading.Lock()

    def client(c):
        rng = np.random.Generator(np.random.PCG64(900 + c))
        mine = []
        for k in range(60):
            name = names[int(rng.integers(2))]
            op = int(rng.choice([rbd.OP_FWD_DYN, rbd.OP_RNEA, rbd.OP_FWD_DYN_VJP]))
            B = int(rng.integers(1, 300))
            ins = make_request(rbd, models[name], op, B, 10000 * c + k)
            outs = [np.full((B, r), -7.0, np.float32) for r in rbd.op_shapes(models[name], op)[1]]
            t, outs = srv.submit(models[name], op, ins, outputs=outs)
            mine.append((t, name, op, ins, outs))
            if c == 0 and k % 3 == 0:
                try:
                    srv.cancel(t)
                except rbd.RbdError:
                    pass  # already left the queue
        for t, name, op, ins, outs in mine:
            st = srv.wait(t, 60.0)
            try:
                if st == CANCELLED:
                    assert all(np.all(o == -7.0) for o in outs)
                else:
                    assert st == OK
                    for got, ref in zip(outs, expected(rbd, models[name], op, ins)):
                        assert np.array_equal(got, ref)
            except AssertionError as e:
                errors.append((c, t, str(e)))
            with lock:
                done.append((t, st))

    srv.reset_stats()
    threads = [threading.Thread(target=client, args=(c,)) for c in range(8)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors[:3]
    assert len(done) == 480 and len({t for t, _ in done}) == 480
    n_ok = sum(st == OK for _, st in done)
    assert srv.stats()["requests"] == n_ok and n_ok >= 480 - 20
    late = [srv.submit(models["chain7"], rbd.OP_FWD_DYN, make_request(rbd, models["chain7"], rbd.OP_FWD_DYN, 50, k))
            for k in range(30)]
    srv.close()  # drains the queue before freeing
    assert all(np.isfinite(outs[0]).all() for _, outs in late)

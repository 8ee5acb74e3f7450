"""The allocation-free packed launch (rbd_packed_static, for callers that cannot allocate device memory)
against the packed launch of the serving runtime (rbd_server_submit) on the same requests: equal
outputs, bit for bit (the same kernel runs every instance), on two calls in a row, the second with
fewer and smaller requests; argument errors; a tree compiled at run time."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_04310_amd as rbd
    descs = {"chain7": W.chain(7), "humanoid30": W.humanoid()}
    models = {k: rbd.Model(d, 0) for k, d in descs.items()}
    srv = rbd.Server(arena_bytes=256 << 20, n_streams=2)
    yield rbd, descs, models, srv
    srv.close()


def host_inputs(rbd, desc, op, B, seed):
    st = W.states(desc, B, seed)
    if op == rbd.OP_FWD_DYN:
        ins = [st.q, st.qd, st.tau]
    elif op == rbd.OP_RNEA:
        ins = [st.q, st.qd, W.cotangent(desc.nv, B, seed + 1)]
    else:
        ins = [st.q, st.qd, st.tau, W.cotangent(desc.nv, B, seed + 2)]
    return [np.ascontiguousarray(x, dtype=np.float32) for x in ins]


def compare_with_server(rbd, srv, m, desc, op, batches, seed):
    """One rbd_packed_static call over requests of `batches` against rbd_server_submit of each."""
    _, out_rows = rbd.op_shapes(m, op)
    host = [host_inputs(rbd, desc, op, B, seed + 10 * k) for k, B in enumerate(batches)]
    tickets = [srv.submit(m, op, ins) if B else None for ins, B in zip(host, batches)]
    dev = []
    for ins, B in zip(host, batches):
        di = [torch.from_numpy(x).cuda() for x in ins]
        do = [torch.full((B, r), float("nan"), device="cuda") for r in out_rows]
        dev.append((di, do))
    rbd.packed_static(m, op, dev)
    torch.cuda.synchronize()
    for t, (_, do) in zip(tickets, dev):
        if t is None:
            continue
        ticket, outs = t
        assert srv.wait(ticket, 60.0) == 0
        for ref, got in zip(outs, do):
            np.testing.assert_array_equal(got.cpu().numpy(), ref)


@pytest.mark.parametrize("name", ["chain7", "humanoid30"])
@pytest.mark.parametrize("op", [0, 1, 2])
def test_packed_static_equals_server(env, name, op):
    rbd, descs, models, srv = env
    print(f"packed_static {name} op {op}", flush=True)
    # ragged batches, an empty request, more than one chunk of descriptors on the first call
    first = [700, 64, 1, 0, 129, 4096 + 37] + [5 + 3 * k for k in range(30)]
    compare_with_server(rbd, srv, models[name], descs[name], op, first, 300 + op)
    compare_with_server(rbd, srv, models[name], descs[name], op, [37, 5], 900 + op)


def test_packed_static_errors(env):
    rbd, descs, models, srv = env
    m = models["chain7"]
    ins = [torch.zeros((2, 7), device="cuda") for _ in range(3)]
    outs = [torch.zeros((2, 7), device="cuda")]
    with pytest.raises(rbd.RbdError, match="requests"):
        rbd.packed_static(m, rbd.OP_FWD_DYN, [(ins, outs)] * 1025)
    big = 32768 * 64 + 1
    bins = [torch.zeros((big, 7), device="cuda") for _ in range(3)]
    bouts = [torch.zeros((big, 7), device="cuda")]
    with pytest.raises(rbd.RbdError, match="tiles"):
        rbd.packed_static(m, rbd.OP_FWD_DYN, [(bins, bouts)])
    del bins, bouts
    L = rbd.lib()
    assert L.rbd_packed_static(m.handle, 7, 0, None, None) == 1
    assert b"bad op" in L.rbd_last_error()
    rbd.packed_static(m, rbd.OP_FWD_DYN, [])  # nothing to do


def test_packed_static_tree_compiled_at_run_time(env):
    """A tree without compiled kernels: refused until its packed kernel is loaded (loading allocates),
    then equal to the server."""
    rbd, descs, models, srv = env
    # a shape no other test uses, so that its packed kernel is not loaded yet in this process
    desc = W.random_tree(W.random_dfs_parents(10, 77), False, 5)
    m = rbd.Model(desc, 0)
    ins = [torch.zeros((3, desc.nv), device="cuda") for _ in range(3)]
    outs = [torch.zeros((3, desc.nv), device="cuda")]
    with pytest.raises(rbd.RbdError, match="not loaded"):
        rbd.packed_static(m, rbd.OP_RNEA, [(ins, outs)])
    t, _ = srv.submit(m, rbd.OP_RNEA, host_inputs(rbd, desc, rbd.OP_RNEA, 3, 77))
    assert srv.wait(t, 120.0) == 0
    compare_with_server(rbd, srv, m, desc, rbd.OP_RNEA, [100, 3, 64], 78)
    compare_with_server(rbd, srv, m, desc, rbd.OP_RNEA, [9], 79)


def test_packed_static_in_a_captured_graph(env):
    """What the entry point is for: captured once into a HIP graph (torch.cuda.graph), then replayed
    with new inputs copied into the same buffers between replays (eager work and synchronisation in
    between); every replay equals an eager call on the same inputs, bit for bit."""
    rbd, descs, models, srv = env
    m, d = models["humanoid30"], descs["humanoid30"]
    op = rbd.OP_FWD_DYN_VJP
    batches = [300, 64, 5]
    in_rows, out_rows = rbd.op_shapes(m, op)
    dev = [([torch.empty((B, r), device="cuda") for r in in_rows],
            [torch.empty((B, r), device="cuda") for r in out_rows]) for B in batches]

    def fill(seed):
        for k, (B, (di, _)) in enumerate(zip(batches, dev)):
            for x, h in zip(di, host_inputs(rbd, d, op, B, seed + 10 * k)):
                x.copy_(torch.from_numpy(h))
        torch.cuda.synchronize()

    fill(500)
    rbd.packed_static(m, op, dev)  # eager first: the static table's address is looked up here
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rbd.packed_static(m, op, dev)
    for rep in range(3):
        fill(600 + 100 * rep)
        g.replay()
        torch.cuda.synchronize()
        replayed = [[o.clone() for o in outs] for _, outs in dev]
        for _, outs in dev:
            for o in outs:
                o.fill_(float("nan"))
        rbd.packed_static(m, op, dev)
        torch.cuda.synchronize()
        for got, (_, outs) in zip(replayed, dev):
            for a, b in zip(got, outs):
                assert torch.isfinite(b).all()
                assert torch.equal(a, b)

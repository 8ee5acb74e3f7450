"""Benchmark: forward-dynamics evals/s of the 35-DoF floating-base tree on one GPU.

One step = one fused forward-dynamics launch (transforms, bias force, mass
matrix, branch-sparse L^T L factorisation and both solves) over a batch of
65536 resident, seeded synthetic states of the 30-body humanoid (floating base
plus 29 revolute joints). Prints one JSON line with the throughput, the
roofline of that kernel (FP32 VALU, using the oracle's per-evaluation operation
count), the FP64 CPU oracle timed on the host as a baseline, per-operation
timings of the other hot-path kernels, and p50/p99 latency of the
continuous-batching server under a Poisson request mix.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "forward-dynamics evals/sec (35-DoF tree, FP32) + p50/p99 request latency"
BATCH = 65536
# MI355X published peaks: FP32 vector 157.3 TFLOP/s counts packed FP32 (two per
# lane per cycle); the kernels are built without packed FP32, which leaves one
# FMA per lane per cycle: 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fwd_dyn_humanoid30_b65536_traffic.txt")
CSRC = os.path.join(ROOT, "paper_2604_04310_amd", "csrc")


KERNEL_SOURCES = ["rbd_lane.hpp", "rbd_kernels.hpp", "rbd_kern_topo.hip", "rbd_shared.hpp", "rbd_topologies.hpp"]


def kernel_source_hash() -> str:
    """Hash of the device-code sources: the counter figures hold while it is unchanged."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def read_counters():
    """Figures from the committed counter summary (HBM bytes per launch, executed
    FP32 FLOPs per evaluation), or {} when the kernels changed after the
    counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():
        return {}
    out = {}
    for k in ("hbm_bytes_per_launch", "executed_fp32_flops_per_eval"):
        try:
            out[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    return out


def counters_driver():
    """The run the counter summaries are taken from: five humanoid fwd_dyn
    launches at batch 65536, three each of crba, fk and jacobian (all 30
    frames) on the same states, then three plain 512 MiB device copies (the
    calibration kernel for FETCH_SIZE / WRITE_SIZE)."""
    import torch

    import paper_2604_04310_amd as rbd
    import workloads as W
    desc = W.humanoid()
    m = rbd.Model(desc, 0)
    st = W.states(desc, BATCH, 103)
    q, qd, tau = soa(st.q, torch), soa(st.qd, torch), soa(st.tau, torch)
    out = torch.empty((desc.nv, BATCH), dtype=torch.float32, device="cuda")
    for _ in range(5):
        rbd.fwd_dyn(m, q, qd, tau, out=out)
    # the HBM-bound kernels of the same batch, three launches each
    for fn in (lambda: rbd.crba(m, q), lambda: rbd.fk(m, q), lambda: rbd.jacobian(m, q)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    a = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("counters driver done", flush=True)


def soa(x, torch):
    return torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")


def time_launches(fn, n, torch, warm=3):
    """Average duration (ms) of n back-to-back launches, by HIP events on the launch stream."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(n):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / n


def cpu_baseline(desc, st, budget_s):
    """The FP64 oracle (test infrastructure) on the host cores over repeated
    passes of a 4096-state slice of the same workload, for about budget_s."""
    import oracle as O
    n = 4096
    q, qd, tau = st.q[:n], st.qd[:n], st.tau[:n]
    O.fwd_dyn(desc, q, qd, tau)  # warm
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        O.fwd_dyn(desc, q, qd, tau)
        done += n
    dt = time.perf_counter() - t0
    cores = O.max_threads()
    # the same on one core, over a quarter of the budget
    m = 512
    prev = O.set_threads(1)
    done1, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < budget_s / 4:
        O.fwd_dyn(desc, q[:m], qd[:m], tau[:m])
        done1 += m
    dt1 = time.perf_counter() - t1
    O.set_threads(prev)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": done / dt, "unit": "evals/s", "cores": cores, "kind": "oracle", "cpu_model": model,
            "sample": f"{done} humanoid30 fwd_dyn evals (FP64, branch-sparse L^T L) = {done // n} passes over "
                      f"the first {n} states of the batch, {dt:.1f} s wall",
            "one_core_evals_per_s": done1 / dt1}


def serving_leg(rbd, torch, seconds, seed=7):
    """Poisson mix of chain7/humanoid30 requests (ops 60/25/15 fwd_dyn/rnea/vjp,
    batch log-uniform in [1, 4096]) at half and at 80 % of the measured
    closed-loop capacity."""
    import workloads as W
    descs = {"chain7": W.chain(7), "humanoid30": W.humanoid()}
    models = {k: rbd.Model(d, 0) for k, d in descs.items()}
    rng = np.random.Generator(np.random.PCG64(seed))
    pool = []
    for k in range(256):
        name = "chain7" if rng.random() < 0.5 else "humanoid30"
        u = rng.random()
        op = rbd.OP_FWD_DYN if u < 0.60 else (rbd.OP_RNEA if u < 0.85 else rbd.OP_FWD_DYN_VJP)
        B = int(np.clip(round(np.exp(rng.uniform(0, np.log(4096)))), 1, 4096))
        d = descs[name]
        st = W.states(d, B, 5000 + k)
        ins = [st.q, st.qd, st.tau] if op != rbd.OP_RNEA else [st.q, st.qd, W.cotangent(d.nv, B, k)]
        if op == rbd.OP_FWD_DYN_VJP:
            ins = ins + [W.cotangent(d.nv, B, 77 + k)]
        pool.append((name, op, B, [x.astype(np.float32) for x in ins]))

    def run(srv, n_req, rate):
        """Open loop when rate > 0 (exponential gaps), else all at once; returns (stats, wall)."""
        tickets = []
        waiter_err = []
        lock = threading.Condition()

        def waiter():
            k = 0
            while k < n_req:
                with lock:
                    while len(tickets) <= k:
                        lock.wait()
                    t = tickets[k]
                if srv.wait(t, 120.0) != 0:
                    waiter_err.append(t)
                k += 1

        th = threading.Thread(target=waiter)
        th.start()
        srv.reset_stats()
        t0 = time.perf_counter()
        next_t = t0
        for k in range(n_req):
            if rate > 0:
                next_t += rng.exponential(1.0 / rate)
                while time.perf_counter() < next_t:
                    pass
            name, op, B, ins = pool[k % len(pool)]
            t, _ = srv.submit(models[name], op, ins)
            with lock:
                tickets.append(t)
                lock.notify()
        th.join()
        wall = time.perf_counter() - t0
        if waiter_err:
            raise RuntimeError(f"{len(waiter_err)} served requests failed")
        return srv.stats(), wall

    out = {}
    srv = rbd.Server(arena_bytes=1 << 30, n_streams=4, max_batch_requests=1024, use_graphs=True)
    run(srv, 512, 0.0)  # warm: graphs, pools
    st, wall = run(srv, 2048, 0.0)
    cap = st["requests"] / wall
    run(srv, 4000, 0.5 * cap)  # open-loop warm-up, not reported
    n_open = int(max(512, min(20000, cap * 0.5 * seconds)))
    st, wall = run(srv, n_open, 0.5 * cap)
    out["batched"] = {"offered_req_per_s": round(0.5 * cap, 1), "requests": st["requests"],
                      "launches": st["launches"], "evals_per_s": st["instances"] / wall,
                      "p50_us": st["p50_us"], "p99_us": st["p99_us"], "max_us": st["max_us"],
                      "closed_loop_capacity_req_per_s": round(cap, 1)}
    n80 = int(max(512, min(20000, cap * 0.8 * seconds)))
    st, wall = run(srv, n80, 0.8 * cap)
    out["batched_at_80pct"] = {"offered_req_per_s": round(0.8 * cap, 1), "requests": st["requests"],
                               "launches": st["launches"], "evals_per_s": st["instances"] / wall,
                               "p50_us": st["p50_us"], "p99_us": st["p99_us"], "max_us": st["max_us"]}
    srv.close()
    base = rbd.Server(arena_bytes=1 << 30, n_streams=1, per_request=True, use_graphs=False)
    run(base, 256, 0.0)
    st, wall = run(base, 2048, 0.0)
    bcap = st["requests"] / wall
    n_b = int(max(256, min(20000, min(0.5 * cap, 0.9 * bcap) * seconds)))
    st, wall = run(base, n_b, min(0.5 * cap, 0.9 * bcap))
    out["one_launch_per_request"] = {"offered_req_per_s": round(min(0.5 * cap, 0.9 * bcap), 1),
                                     "requests": st["requests"], "evals_per_s": st["instances"] / wall,
                                     "p50_us": st["p50_us"], "p99_us": st["p99_us"], "max_us": st["max_us"],
                                     "closed_loop_capacity_req_per_s": round(bcap, 1)}
    base.close()
    out["mix"] = "Poisson arrivals, chain7/humanoid30 50/50, fwd_dyn/rnea/fwd_dyn_vjp 60/25/15, batch log-uniform 1..4096, host I/O included"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--counters", action="store_true", help="only run the counter-collection driver")
    args = ap.parse_args()
    if args.counters:
        counters_driver()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the dynamics of independent robot instances need no "
              f"cross-GPU exchange, so each GPU runs its own shard (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle as O
    import paper_2604_04310_amd as rbd
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    desc = W.humanoid()
    model = rbd.Model(desc, 0)
    st = W.states(desc, BATCH, 103)
    q, qd, tau = soa(st.q, torch), soa(st.qd, torch), soa(st.tau, torch)
    qdd = torch.empty((desc.nv, BATCH), dtype=torch.float32, device="cuda")

    def step():
        rbd.fwd_dyn(model, q, qd, tau, out=qdd)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(args.steps):
        step()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = e0.elapsed_time(e1) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    value = BATCH * args.steps / wall

    # the same launch replayed from a captured HIP graph, and one launch's latency
    # (launch to completion seen by the host)
    n_graph = 20
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(gs):
        step()
    torch.cuda.current_stream().wait_stream(gs)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(n_graph):
            step()
    graph.replay()
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps // n_graph)
    g0.record(s)
    for _ in range(reps):
        graph.replay()
    g1.record(s)
    torch.cuda.synchronize()
    graph_us = 1e3 * g0.elapsed_time(g1) / (reps * n_graph)
    lat = []
    for _ in range(21):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
    single_launch_us = 1e6 * float(np.median(lat))
    del graph

    # parity of the timed output on a sample (the full check lives in tests/)
    idx = np.arange(0, BATCH, 257)
    got = qdd[:, torch.as_tensor(idx, device="cuda")].double().cpu().numpy().T
    ref = O.fwd_dyn(desc, st.q[idx], st.qd[idx], st.tau[idx])
    max_rel = float((np.abs(got - ref).max(1) / np.abs(ref).max(1)).max())

    flops = O.count_ops(desc, "fwd_dyn_ltl")
    per_eval = flops["flops"]
    achieved = per_eval * BATCH / (kernel_ms * 1e-3) / 1e12
    cnt = read_counters()
    traffic = cnt.get("hbm_bytes_per_launch")
    ceiling = rbd.fma_rate(256, 16)  # measured FMA issue ceiling at this launch shape
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_fwd_dyn<humanoid30>", "kernel_ms": round(kernel_ms, 5),
                "flops_per_eval": per_eval, "flops_source": "oracle count of the same algorithm (FP64 counting scalar)",
                "peak_unpacked_fp32": round(PEAK_FP32_UNPACKED_TFLOPS, 1),
                "frac_of_unpacked_peak": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4),
                "measured_fma_ceiling_at_this_launch_shape": round(ceiling, 1),
                "executed_fp32_flops_per_eval": cnt.get("executed_fp32_flops_per_eval"),
                "executed_tflops": (round(cnt["executed_fp32_flops_per_eval"] * BATCH / (kernel_ms * 1e-3) / 1e12, 2)
                                    if "executed_fp32_flops_per_eval" in cnt else None),
                "algorithmic_bytes_per_eval": 4 * (desc.nq + 3 * desc.nv),
                "hbm_gbs_algorithmic": round(4 * (desc.nq + 3 * desc.nv) * BATCH / (kernel_ms * 1e-3) / 1e9, 1)}

    # the other hot-path kernels at their benchmark shapes
    ops = {}
    n_t = max(5, args.steps // 10)
    ops["aba_humanoid30_b65536_us"] = 1e3 * time_launches(lambda: rbd.aba(model, q, qd, tau), n_t, torch)
    ops["rnea_bias_humanoid30_b65536_us"] = 1e3 * time_launches(lambda: rbd.rnea(model, q, qd), n_t, torch)
    ops["crba_humanoid30_b65536_us"] = 1e3 * time_launches(lambda: rbd.crba(model, q), n_t, torch)
    ops["fk_humanoid30_b65536_us"] = 1e3 * time_launches(lambda: rbd.fk(model, q), n_t, torch)
    ops["jacobian30_humanoid30_b65536_us"] = 1e3 * time_launches(lambda: rbd.jacobian(model, q), n_t, torch)
    torch.cuda.empty_cache()
    Bv = 32768
    gq = soa(W.cotangent(desc.nv, Bv, 9), torch)
    vq, vqd, vtau = q[:, :Bv].contiguous(), qd[:, :Bv].contiguous(), tau[:, :Bv].contiguous()
    ops["fwd_dyn_vjp_humanoid30_b32768_us"] = 1e3 * time_launches(
        lambda: rbd.fwd_dyn_vjp(model, vq, vqd, vtau, gq), n_t, torch)
    tq, tqd, ttau = (soa(W._f32(np.random.default_rng(s).normal(size=(Bv, r))), torch)
                     for s, r in ((11, desc.nq), (12, desc.nv), (13, desc.nv)))
    ops["fwd_dyn_jvp_humanoid30_b32768_us"] = 1e3 * time_launches(
        lambda: rbd.fwd_dyn_jvp(model, vq, vqd, vtau, tq, tqd, ttau), n_t, torch)
    del tq, tqd, ttau
    rng_t = np.random.default_rng(15)
    tgt = np.concatenate([np.stack([W.random_rotation(rng_t) for _ in range(256)])[np.arange(BATCH) % 256],
                          rng_t.normal(0.0, 0.5, size=(BATCH, 3, 1))], axis=2)
    tg = soa(W._f32(tgt.reshape(BATCH, 12)), torch)
    ops["osc_humanoid30_b65536_us"] = 1e3 * time_launches(lambda: rbd.osc(model, q, qd, tg, 50.0, 10.0, 2.0), n_t, torch)
    ops["diff_ik_humanoid30_b65536_us"] = 1e3 * time_launches(lambda: rbd.diff_ik(model, q, tg, 2.0, 0.05), n_t, torch)
    del tg
    fx = soa(W._f32(np.random.default_rng(14).normal(0.0, 5.0, size=(BATCH, 6 * desc.n_bodies))), torch)
    ops["fwd_dyn_fext_humanoid30_b65536_us"] = 1e3 * time_launches(
        lambda: rbd.fwd_dyn(model, q, qd, tau, fext=fx), n_t, torch)
    del fx
    chain = W.chain(7)
    cm = rbd.Model(chain, 0)
    cs = W.states(chain, 1 << 20, 102)
    cq, cqd, ctau = soa(cs.q, torch), soa(cs.qd, torch), soa(cs.tau, torch)
    ops["fwd_dyn_chain7_b1048576_us"] = 1e3 * time_launches(lambda: rbd.fwd_dyn(cm, cq, cqd, ctau), n_t, torch)
    ops["aba_chain7_b1048576_us"] = 1e3 * time_launches(lambda: rbd.aba(cm, cq, cqd, ctau), n_t, torch)
    ops["rnea_bias_chain7_b1048576_us"] = 1e3 * time_launches(lambda: rbd.rnea(cm, cq, cqd), n_t, torch)
    Bc = 1 << 18
    cg = soa(W.cotangent(chain.nv, Bc, 3), torch)
    wq, wqd, wtau = cq[:, :Bc].contiguous(), cqd[:, :Bc].contiguous(), ctau[:, :Bc].contiguous()
    ops["fwd_dyn_vjp_chain7_b262144_us"] = 1e3 * time_launches(
        lambda: rbd.fwd_dyn_vjp(cm, wq, wqd, wtau, cg), n_t, torch)
    ops["fwd_dyn_chain7_evals_per_s"] = (1 << 20) / (ops["fwd_dyn_chain7_b1048576_us"] * 1e-6)
    ops = {k: round(v, 2) if "us" in k else float(f"{v:.4g}") for k, v in ops.items()}
    del cq, cqd, ctau
    torch.cuda.empty_cache()

    serving = None if args.no_serving else serving_leg(rbd, torch, args.serve_seconds)
    cpu = None if args.no_cpu else cpu_baseline(desc, st, args.cpu_seconds)

    line = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "humanoid30 fwd_dyn: floating base + 29 revolute joints (35 DoF, 30 bodies), "
                               "batch 65536 resident states, one instance per lane",
                   "batch": BATCH, "nq": desc.nq, "nv": desc.nv, "parallelism": "none (1 GPU)"},
        "parity_max_rel_err_sample": max_rel,
        "fwd_dyn_graph_replay_us": round(graph_us, 2),
        "fwd_dyn_single_launch_latency_us": round(single_launch_us, 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "ops": ops,
        "serving": serving,
        "paper_context": "frax reports upwards of 1e8 dynamics evals/s at batch 4096 on an RTX 4090, "
                         "I/O included, robot and precision unstated (context, not a target)",
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

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
COUNTERS_FILE = os.path.join(ROOT, "profiles", "kernel_counters_humanoid30_chain7.txt")
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
    """Per-kernel figures from the committed counter summary: {key: {field: value}}
    with executed FP32 FLOPs per evaluation and HBM bytes per launch, or {} when
    the kernels changed after the counters were taken."""
    if not os.path.exists(COUNTERS_FILE):
        return {}
    out, src = {}, None
    for line in open(COUNTERS_FILE):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("source_hash"):
            src = line.split("=", 1)[1].strip()
            continue
        fields = dict(f.split("=", 1) for f in line.split() if "=" in f)
        if "kernel" in fields:
            key = fields.pop("kernel")
            out[key] = {k: float(v) for k, v in fields.items()}
    return out if src == kernel_source_hash() else {}


def counters_driver():
    """The run the counter summaries are taken from: each hot kernel at its
    benchmark shape on the seeded states (humanoid30 at batch 65536, its
    derivatives at 32768, the 7-chain at 2^20 and its adjoint at 2^18), a few
    launches each, then three plain 512 MiB device copies (the calibration
    kernel for FETCH_SIZE / WRITE_SIZE). Each step prints its name first."""
    import torch

    import paper_2604_04310_amd as rbd
    import workloads as W

    def step(name, fn, n=3):
        print(f"counters: {name}", flush=True)
        for _ in range(n):
            fn()
        torch.cuda.synchronize()

    desc = W.humanoid()
    m = rbd.Model(desc, 0)
    st = W.states(desc, BATCH, 103)
    q, qd, tau = soa(st.q, torch), soa(st.qd, torch), soa(st.tau, torch)
    out = torch.empty((desc.nv, BATCH), dtype=torch.float32, device="cuda")
    step("fwd_dyn humanoid30 65536", lambda: rbd.fwd_dyn(m, q, qd, tau, out=out), 5)
    step("rnea bias humanoid30 65536", lambda: rbd.rnea(m, q, qd, out=out))
    step("aba humanoid30 65536", lambda: rbd.aba(m, q, qd, tau, out=out))
    for name, fn in (("crba", lambda: rbd.crba(m, q)), ("fk", lambda: rbd.fk(m, q)),
                     ("jacobian", lambda: rbd.jacobian(m, q))):
        step(f"{name} humanoid30 65536", fn)
        torch.cuda.empty_cache()
    tg = soa(W._f32(targets(W, BATCH)), torch)
    step("osc humanoid30 65536", lambda: rbd.osc(m, q, qd, tg, 50.0, 10.0, 2.0))
    step("diff_ik humanoid30 65536", lambda: rbd.diff_ik(m, q, tg, 2.0, 0.05))
    del tg
    Bv = 32768
    vq, vqd, vtau = q[:, :Bv].contiguous(), qd[:, :Bv].contiguous(), tau[:, :Bv].contiguous()
    gq = soa(W.cotangent(desc.nv, Bv, 9), torch)
    step("fwd_dyn_vjp humanoid30 32768", lambda: rbd.fwd_dyn_vjp(m, vq, vqd, vtau, gq))
    tq, tqd, ttau = (soa(W._f32(np.random.default_rng(s).normal(size=(Bv, r))), torch)
                     for s, r in ((11, desc.nq), (12, desc.nv), (13, desc.nv)))
    step("fwd_dyn_jvp humanoid30 32768", lambda: rbd.fwd_dyn_jvp(m, vq, vqd, vtau, tq, tqd, ttau))
    step("rnea_jvp humanoid30 32768", lambda: rbd.rnea_jvp(m, vq, vqd, vtau, tq, tqd, ttau))
    step("rnea_vjp humanoid30 32768", lambda: rbd.rnea_vjp(m, vq, vqd, vtau, gq))
    del q, qd, tau, out, vq, vqd, vtau, gq, tq, tqd, ttau
    torch.cuda.empty_cache()
    chain = W.chain(7)
    cm = rbd.Model(chain, 0)
    cs = W.states(chain, 1 << 20, 102)
    cq, cqd, ctau = soa(cs.q, torch), soa(cs.qd, torch), soa(cs.tau, torch)
    step("fwd_dyn chain7 1048576", lambda: rbd.fwd_dyn(cm, cq, cqd, ctau))
    step("rnea bias chain7 1048576", lambda: rbd.rnea(cm, cq, cqd))
    Bc = 1 << 18
    cg = soa(W.cotangent(chain.nv, Bc, 3), torch)
    wq, wqd, wtau = cq[:, :Bc].contiguous(), cqd[:, :Bc].contiguous(), ctau[:, :Bc].contiguous()
    step("fwd_dyn_vjp chain7 262144", lambda: rbd.fwd_dyn_vjp(cm, wq, wqd, wtau, cg))
    del cq, cqd, ctau, wq, wqd, wtau, cg
    torch.cuda.empty_cache()
    a = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    step("copy 512 MiB", lambda: b.copy_(a))
    print("counters driver done", flush=True)


def targets(W, B):
    """End-effector target poses [B, 12] for the controller kernels (256 distinct, tiled)."""
    rng_t = np.random.default_rng(15)
    tgt = np.concatenate([np.stack([W.random_rotation(rng_t) for _ in range(256)])[np.arange(B) % 256],
                          rng_t.normal(0.0, 0.5, size=(B, 3, 1))], axis=2)
    return tgt.reshape(B, 12)


def kernel_rooflines(O, W, desc, chain, ops, cnt, hbm):
    """Roofline of every other hot kernel at its benchmark shape: VALU-bound ones
    against the FP32 peak (oracle count where the oracle counts the operation,
    and the executed count from the hardware counters), memory-bound ones
    against the measured streaming-write ceiling and the HBM spec."""
    B, Bv, Bc, Bw = BATCH, 32768, 1 << 20, 1 << 18
    nb = desc.n_bodies

    def valu(key, us, batch, oracle_flops, counter_batch=None):
        c = dict(cnt.get(key, {}))
        if counter_batch is not None and counter_batch != batch:
            c.pop("fetch_bytes", None)  # bytes per launch were counted at another batch
            c.pop("write_bytes", None)
        exe = c.get("flops_per_eval")
        r = {"kernel_us": us, "batch": batch, "bound": "alu", "peak_tflops": PEAK_FP32_TFLOPS,
             "oracle_flops_per_eval": oracle_flops,
             "achieved_tflops": round(oracle_flops * batch / (us * 1e-6) / 1e12, 2) if oracle_flops else None,
             "executed_fp32_flops_per_eval": exe,
             "executed_tflops": round(exe * batch / (us * 1e-6) / 1e12, 2) if exe else None}
        basis = r["achieved_tflops"] if oracle_flops else r["executed_tflops"]
        r["frac"] = round(basis / PEAK_FP32_TFLOPS, 4) if basis else None
        r["frac_basis"] = "oracle count" if oracle_flops else ("executed (hardware counter)" if exe else None)
        if exe:
            r["executed_frac"] = round(r["executed_tflops"] / PEAK_FP32_TFLOPS, 4)
        if "fetch_bytes" in c:
            r["traffic"] = c["fetch_bytes"] + c["write_bytes"]
        return r

    def mem(key, us, batch, bytes_per_eval):
        c = cnt.get(key, {})
        gbs = bytes_per_eval * batch / (us * 1e-6) / 1e9
        r = {"kernel_us": us, "batch": batch, "bound": "hbm", "algorithmic_bytes_per_eval": bytes_per_eval,
             "achieved_gbs": round(gbs, 1), "frac_of_spec": round(gbs / PEAK_HBM_GBS, 4),
             "frac_of_measured_write_ceiling": round(gbs / hbm["write_gbs"], 4)}
        if "fetch_bytes" in c:
            r["traffic"] = c["fetch_bytes"] + c["write_bytes"]
        return r

    f = lambda d, op: O.count_ops(d, op)["flops"]  # noqa: E731
    nv = desc.nv
    return {
        "fwd_dyn_chain7": valu("fwd_dyn_chain7", ops["fwd_dyn_chain7_b1048576_us"], Bc, f(chain, "fwd_dyn_ltl")),
        "rnea_bias_humanoid30": valu("rnea_bias_humanoid30", ops["rnea_bias_humanoid30_b65536_us"], B,
                                     f(desc, "rnea_bias")),
        "rnea_bias_chain7": valu("rnea_bias_chain7", ops["rnea_bias_chain7_b1048576_us"], Bc, f(chain, "rnea_bias")),
        "aba_humanoid30": valu("aba_humanoid30", ops["aba_humanoid30_b65536_us"], B, f(desc, "aba")),
        "fwd_dyn_vjp_humanoid30": valu("fwd_dyn_vjp_humanoid30", ops["fwd_dyn_vjp_humanoid30_b32768_us"], Bv, None),
        "fwd_dyn_vjp_chain7": valu("fwd_dyn_vjp_chain7", ops["fwd_dyn_vjp_chain7_b262144_us"], Bw, None),
        "fwd_dyn_jvp_humanoid30": valu("fwd_dyn_jvp_humanoid30", ops["fwd_dyn_jvp_humanoid30_b32768_us"], Bv, None),
        "fwd_dyn_vjp_humanoid30_b65536": valu("fwd_dyn_vjp_humanoid30", ops["fwd_dyn_vjp_humanoid30_b65536_us"], B,
                                              None, counter_batch=Bv),
        "fwd_dyn_jvp_humanoid30_b65536": valu("fwd_dyn_jvp_humanoid30", ops["fwd_dyn_jvp_humanoid30_b65536_us"], B,
                                              None, counter_batch=Bv),
        "rnea_jvp_humanoid30_b65536": valu("rnea_jvp_humanoid30", ops["rnea_jvp_humanoid30_b65536_us"], B, None,
                                           counter_batch=Bv),
        "rnea_vjp_humanoid30_b65536": valu("rnea_vjp_humanoid30", ops["rnea_vjp_humanoid30_b65536_us"], B, None,
                                           counter_batch=Bv),
        "osc_humanoid30": valu("osc_humanoid30", ops["osc_humanoid30_b65536_us"], B, None),
        "crba_humanoid30": mem("crba_humanoid30", ops["crba_humanoid30_b65536_us"], B, 4 * (desc.nq + nv * nv)),
        "fk_humanoid30": mem("fk_humanoid30", ops["fk_humanoid30_b65536_us"], B, 4 * (desc.nq + 12 * nb)),
        "jacobian30_humanoid30": mem("jacobian_humanoid30", ops["jacobian30_humanoid30_b65536_us"], B,
                                     4 * (desc.nq + nb * 6 * nv)),
        "note": "the oracle differentiates by central differences and its controllers are NumPy solves, so the "
                "derivative and controller kernels are reported on the executed (hardware-counter) basis only",
    }


# ---------------------------------------------------------------- profile summaries
def _topology_names():
    """Tree<...> template arguments -> compiled topology name."""
    import re
    text = open(os.path.join(CSRC, "rbd_topologies.hpp")).read().replace("\\\n", " ")
    return {re.sub(r"\s+", " ", f"{fr}, {par.strip()}"): name
            for name, fr, par in re.findall(r"X\((\w+), (true|false), ([-0-9, \s]+)\)", text)}


def _short_kernel(name, topo):
    """'void rbd::k_fwd_dyn<rbd::Tree<true, -1, ...>, true, false>(...)' -> 'k_fwd_dyn<humanoid30, true, false>'."""
    import re
    name = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").replace("rbd::", "")
    m = re.search(r"Tree<([^>]*)>", name)
    if m:
        name = name.replace(m.group(0), topo.get(re.sub(r"\s+", " ", m.group(1).strip()), "tree"))
    return name


def _kernel_key(short):
    """The bench's key of a kernel at its benchmark shape (None for kernels the bench does not rate)."""
    base, _, rest = short.partition("<")
    topo = rest.split(",")[0].rstrip(">").strip()
    key = {"k_fwd_dyn": "fwd_dyn", "k_rnea": "rnea_bias", "k_aba": "aba", "k_crba": "crba", "k_fk": "fk",
           "k_jacobian": "jacobian", "k_osc": "osc", "k_diff_ik": "diff_ik", "k_fwd_dyn_vjp": "fwd_dyn_vjp",
           "k_fwd_dyn_jvp": "fwd_dyn_jvp", "k_fwd_dyn_jvp_split": "fwd_dyn_jvp", "k_fwd_dyn_vjp_split": "fwd_dyn_vjp",
           "k_rnea_jvp": "rnea_jvp", "k_rnea_vjp": "rnea_vjp"}.get(base)
    return f"{key}_{topo}" if key and topo in ("humanoid30", "chain7") else None


def summarize_profiles(out_dir):
    """Writes the committed profile summaries from the rocprofv3 databases of one
    run of gpu commands (kernel trace of the bench, and three counter passes of
    bench.py --counters): profiles/bench_kernels_humanoid30_chain7_stats.txt and
    profiles/kernel_counters_humanoid30_chain7.txt."""
    import collections
    import sqlite3
    topo = _topology_names()

    def db(sub):
        return sqlite3.connect(os.path.join(out_dir, sub, "run_results.db")).cursor()

    # kernel trace: calls and average duration per kernel
    cur = db("prof_trace")
    rows = list(cur.execute("select name, total_calls, average, total_duration, percentage from top_kernels"))
    lines = ["# Kernel trace of bench.py on one MI355X (gfx950), rocprofv3 --kernel-trace --stats",
             "#", "# command (run from /tmp with TMPDIR=/tmp):",
             "#   rocprofv3 --kernel-trace --stats -d <out> -o run -- python3 <repo>/bench.py --steps 20 --warmup 5 "
             "--no-serving --no-cpu",
             "# Durations per dispatch in microseconds, over every dispatch of the run (warm-up, timed launches, "
             "graph replays, single launches).",
             f"# source_hash = {kernel_source_hash()}", "#",
             f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'total_us':>11s} {'pct':>6s}"]
    for name, calls, avg, total, pct in rows:
        lines.append(f"{_short_kernel(name, topo)[:70]:70s} {calls:6d} {avg:10.3f} {total:11.1f} {pct:6.2f}")
    with open(os.path.join(ROOT, "profiles", "bench_kernels_humanoid30_chain7_stats.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    # counters: summed over shader engines per dispatch, medians per kernel
    def counters(sub):
        agg, names = collections.defaultdict(float), {}
        for did, kname, cname, val in db(sub).execute(
                "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
            agg[(did, cname)] += val
            names[did] = kname
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        for (did, cname), v in agg.items():
            per[names[did]][cname].append(v)
        return per

    fetch, write, sq = counters("pmc_FETCH_SIZE"), counters("pmc_WRITE_SIZE"), counters("pmc_SQ_INSTS_VALU_FLOPS_FP32")
    med = lambda xs: float(np.median(xs))  # noqa: E731
    copy = next(k for k in fetch if "copyBuffer" in k and med(fetch[k]["FETCH_SIZE"]) > 1e5)
    copy_bytes = 512 << 20
    fscale = copy_bytes / (med(fetch[copy]["FETCH_SIZE"]) * 1024.0)
    wscale = copy_bytes / (med(write[copy]["WRITE_SIZE"]) * 1024.0)
    out = ["# Hardware counters of the hot kernels at their benchmark shapes, one MI355X (gfx950)", "#",
           "# commands (each its own run, from /tmp with TMPDIR=/tmp):",
           "#   rocprofv3 --pmc FETCH_SIZE -d <out> -o run -- python3 <repo>/bench.py --counters",
           "#   rocprofv3 --pmc WRITE_SIZE -d <out> -o run -- python3 <repo>/bench.py --counters",
           "#   rocprofv3 --pmc SQ_INSTS_VALU_FLOPS_FP32 SQ_INSTS_VALU SQ_WAVES SQ_WAVE_CYCLES SQ_WAIT_ANY "
           "SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY -d <out> -o run -- python3 <repo>/bench.py --counters",
           "# then: python3 bench.py --summarize-profiles <out dir> (this file and the kernel-trace summary).",
           "# Counter values summed over shader engines per dispatch, median over the dispatches of a kernel.",
           f"# Calibration on a plain 512 MiB device copy: FETCH_SIZE scale {fscale:.4f}, WRITE_SIZE scale "
           f"{wscale:.4f} (bytes = KiB x 1024 x scale).",
           "# flops_per_eval = SQ_INSTS_VALU_FLOPS_FP32 / SQ_WAVES (FP32 FLOPs of one lane, one instance per lane;",
           "# twice that for the tangent and the adjoint of the 35-DoF tree at batch 32768, which run two waves per 64 instances);",
           "# valu_insts_per_wave = SQ_INSTS_VALU / SQ_WAVES; quad-cycles per wave: wave_cycles, wait_any "
           "(dependency and memory waits), wait_inst_any (issue waits), active_inst_any (issuing).",
           f"source_hash = {kernel_source_hash()}"]
    for name in sq:
        key = _kernel_key(_short_kernel(name, topo))
        if key is None or name not in fetch or name not in write:
            continue
        c = {k: med(v) for k, v in sq[name].items()}
        w = max(c.get("SQ_WAVES", 0.0), 1.0)
        # waves per 64 instances: two for the tangent split over two waves
        per = 2.0 if _short_kernel(name, topo).startswith(("k_fwd_dyn_jvp_split", "k_fwd_dyn_vjp_split")) else 1.0
        fb = med(fetch[name]["FETCH_SIZE"]) * 1024.0 * fscale
        wb = med(write[name]["WRITE_SIZE"]) * 1024.0 * wscale
        out.append(f"kernel={key} flops_per_eval={c['SQ_INSTS_VALU_FLOPS_FP32'] * per / w:.0f} "
                   f"valu_insts_per_wave={c['SQ_INSTS_VALU'] / w:.0f} waves={w:.0f} fetch_bytes={fb:.0f} "
                   f"write_bytes={wb:.0f} wave_cycles={c['SQ_WAVE_CYCLES'] / w:.0f} wait_any={c['SQ_WAIT_ANY'] / w:.0f} "
                   f"wait_inst_any={c['SQ_WAIT_INST_ANY'] / w:.0f} active_inst_any={c['SQ_ACTIVE_INST_ANY'] / w:.0f}")
    with open(COUNTERS_FILE, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))
    if os.path.exists(os.path.join(out_dir, "prof_serving", "run_results.db")):
        summarize_serving_trace(os.path.join(out_dir, "prof_serving", "run_results.db"), topo)


def _union(iv):
    """Total length of the union of [start, end) intervals."""
    tot, cur_s, cur_e = 0, None, None
    for s0, e0 in sorted(iv):
        if cur_e is None or s0 > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = s0, e0
        else:
            cur_e = max(cur_e, e0)
    return tot + (cur_e - cur_s if cur_e is not None else 0)


def summarize_serving_trace(path, topo):
    """profiles/serving_overlap_chain7_humanoid30.txt: from a kernel and memory-copy trace of the
    serving leg, how the packed launches and copies of different launch slots overlap in time."""
    import collections
    import sqlite3
    cur = sqlite3.connect(path).cursor()
    ks = [(n, st, q, s0, e0) for n, st, q, s0, e0 in
          cur.execute("select name, stream_id, queue_id, start, end from kernels") if "k_packed" in n]
    cps = list(cur.execute("select start, end from memory_copies"))
    t0 = min(min(k[3] for k in ks), min(c[0] for c in cps))
    t1 = max(max(k[4] for k in ks), max(c[1] for c in cps))
    k_iv = [(k[3], k[4]) for k in ks]
    k_sum, k_union = sum(e - s for s, e in k_iv), _union(k_iv)
    ev = sorted([(s, 1) for s, _ in k_iv] + [(e, -1) for _, e in k_iv])
    conc, last, multi = 0, None, 0
    for t, d in ev:
        if conc >= 2 and last is not None:
            multi += t - last
        conc += d
        last = t
    per = collections.defaultdict(list)
    for n, st, q, s0, e0 in ks:
        per[_short_kernel(n, topo)].append(e0 - s0)
    lines = ["# Serving leg under a kernel and copy trace, one MI355X (gfx950)", "#",
             "# command (run from /tmp with TMPDIR=/tmp):",
             "#   rocprofv3 --kernel-trace --memory-copy-trace -d <out>/prof_serving -o run -- python3 "
             "<repo>/bench.py --serving-only --serve-seconds 2",
             "# then: python3 bench.py --summarize-profiles <out> (with the other profile runs)",
             f"# source_hash = {kernel_source_hash()}",
             f"span_ms = {(t1 - t0) / 1e6:.1f}",
             f"packed_launches = {len(ks)} on {len({k[1] for k in ks})} streams, {len({k[2] for k in ks})} hardware queues",
             f"packed_kernel_time_ms = {k_sum / 1e6:.2f} (sum of durations)",
             f"packed_kernel_busy_ms = {k_union / 1e6:.2f} (union: time with at least one packed kernel running)",
             f"gpu_kernel_busy_frac = {k_union / (t1 - t0):.3f} (union over the span)",
             f"time_with_two_or_more_packed_kernels_ms = {multi / 1e6:.2f} "
             f"({multi / max(k_union, 1):.3f} of the busy time)",
             f"copies = {len(cps)}, copy_busy_ms = {_union(cps) / 1e6:.2f}, "
             f"kernel_or_copy_busy_frac = {_union(k_iv + cps) / (t1 - t0):.3f}",
             "", f"{'kernel':70s} {'calls':>7s} {'avg_us':>9s} {'p99_us':>9s}"]
    for name, d in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{name[:70]:70s} {len(d):7d} {np.mean(d) / 1e3:9.2f} {np.percentile(d, 99) / 1e3:9.2f}")
    with open(os.path.join(ROOT, "profiles", "serving_overlap_chain7_humanoid30.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


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
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"value": done / dt, "unit": "evals/s", "cores": cores, "kind": "oracle", "cpu_model": model,
            "affinity_cpus": affinity, "logical_cpus": os.cpu_count(),
            "build": "g++ -O2 -fopenmp, no -march (portable code, as committed)",
            "parallelism": "OpenMP over states, one state per thread at a time, default affinity",
            "sample": f"{done} humanoid30 fwd_dyn evals (FP64, branch-sparse L^T L) = {done // n} passes over "
                      f"the first {n} states of the batch, {dt:.1f} s wall",
            "one_core_evals_per_s": done1 / dt1}


def serving_leg(rbd, torch, seconds, seed=7, n_streams=4, group_bytes=0):
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

    def run_python(srv, n_req):
        """Closed loop from Python (submit all, then wait in order): the binding's own overhead."""
        srv.reset_stats()
        t0 = time.perf_counter()
        tickets = [srv.submit(models[pool[k % len(pool)][0]], pool[k % len(pool)][1], pool[k % len(pool)][3])[0]
                   for k in range(n_req)]
        bad = sum(srv.wait(t, 120.0) != 0 for t in tickets)
        if bad:
            raise RuntimeError(f"{bad} served requests failed")
        return n_req / (time.perf_counter() - t0)

    specs = [(models[name], op, ins) for name, op, _, ins in pool]

    def run(srv, n_req, rate, seed):
        """Native open-loop client (Poisson at `rate`, 0 = closed loop); returns (stats, wall)."""
        srv.reset_stats()
        wall, failed = srv.load(specs, n_req, rate=rate, window=4 * len(specs), seed=seed)
        if failed:
            raise RuntimeError(f"{failed} served requests failed")
        return srv.stats(), wall

    def leg(st, wall, rate):
        ks = max(st["gpu_kernel_s"], 1e-12)
        return {"offered_req_per_s": round(rate, 1), "requests": st["requests"], "launches": st["launches"],
                "evals_per_s": st["instances"] / wall, "p50_us": st["p50_us"], "p99_us": st["p99_us"],
                "max_us": st["max_us"], "groups_in_flight_frac": round(st["busy_s"] / wall, 3),
                # device timeline from the server's own per-group timing events
                "gpu_kernel_busy_frac": round(st["gpu_kernel_s"] / wall, 3),
                "gpu_kernel_overlap_frac": round(st["gpu_kernel_overlap_s"] / ks, 3),
                "gpu_copy_busy_frac": round(st["gpu_copy_s"] / wall, 3),
                "gpu_active_frac": round(st["gpu_active_s"] / wall, 3),
                "mean_kernel_us": round(1e6 * st["gpu_kernel_sum_s"] / max(st["groups_timed"], 1), 1)}

    out = {}
    srv = rbd.Server(arena_bytes=1 << 30, n_streams=n_streams, max_batch_requests=1024, use_graphs=True,
                     max_group_bytes=group_bytes)
    run(srv, 1024, 0.0, 1)  # warm: graphs, pools
    st, wall = run(srv, 8192, 0.0, 2)
    cap = st["requests"] / wall
    run(srv, 4000, 0.5 * cap, 3)  # open-loop warm-up, not reported
    st, wall = run(srv, int(max(512, min(200000, cap * 0.5 * seconds))), 0.5 * cap, 4)
    out["batched"] = dict(leg(st, wall, 0.5 * cap), closed_loop_capacity_req_per_s=round(cap, 1),
                          closed_loop_evals_per_s=None)
    st, wall = run(srv, int(max(512, min(200000, cap * 0.8 * seconds))), 0.8 * cap, 5)
    out["batched_at_80pct"] = leg(st, wall, 0.8 * cap)
    st, wall = run(srv, int(max(512, min(200000, cap * 0.25 * seconds))), 0.25 * cap, 10)
    out["batched_at_25pct"] = leg(st, wall, 0.25 * cap)
    st, wall = run(srv, 8192, 0.0, 6)
    out["batched"]["closed_loop_evals_per_s"] = st["instances"] / wall
    out["python_client_closed_loop_req_per_s"] = round(run_python(srv, 2048), 1)
    srv.close()
    base = rbd.Server(arena_bytes=1 << 30, n_streams=1, per_request=True, use_graphs=False)
    run(base, 256, 0.0, 7)
    st, wall = run(base, 2048, 0.0, 8)
    bcap = st["requests"] / wall
    rate = min(0.5 * cap, 0.9 * bcap)
    st, wall = run(base, int(max(256, min(50000, rate * seconds))), rate, 9)
    out["one_launch_per_request"] = dict(leg(st, wall, rate), closed_loop_capacity_req_per_s=round(bcap, 1))
    base.close()
    out["client"] = ("native open-loop generator (rbd_diag_serve_load): Poisson arrivals from one submitting "
                     f"thread, one waiting thread; {n_streams} launch slots (stream + worker thread each)")
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
    ap.add_argument("--serving-only", action="store_true", help="only the serving leg (for a trace of it)")
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-group-mib", type=float, default=0.0, help="launch-group byte cap (0: default)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--counters", action="store_true", help="only run the counter-collection driver")
    ap.add_argument("--summarize-profiles", metavar="DIR", help="write profiles/ summaries from rocprofv3 output")
    args = ap.parse_args()
    if args.counters:
        counters_driver()
        return
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
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
    if args.serving_only:
        print(json.dumps(serving_leg(rbd, torch, args.serve_seconds, n_streams=args.serve_streams,
                                     group_bytes=int(args.serve_group_mib * (1 << 20)))), flush=True)
        return
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
    head = cnt.get("fwd_dyn_humanoid30", {})
    traffic = (head["fetch_bytes"] + head["write_bytes"]) if "fetch_bytes" in head else None
    ceiling = rbd.fma_rate(256, 16)  # measured FMA issue ceiling at this launch shape
    exe = head.get("flops_per_eval")
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_fwd_dyn<humanoid30>", "kernel_ms": round(kernel_ms, 5),
                "flops_per_eval": per_eval,
                "flops_source": "oracle count (FP64 counting scalar: state-dependent add/sub/mul, transforms shared "
                                "by RNEA and CRBA, trivial operations not counted)",
                "peak_unpacked_fp32": round(PEAK_FP32_UNPACKED_TFLOPS, 1),
                "frac_of_unpacked_peak": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4),
                "measured_fma_ceiling_at_this_launch_shape": round(ceiling, 1),
                "executed_fp32_flops_per_eval": exe,
                "executed_tflops": round(exe * BATCH / (kernel_ms * 1e-3) / 1e12, 2) if exe else None,
                "executed_frac": round(exe * BATCH / (kernel_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4) if exe else None,
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
    # every output subset of the adjoint (what autograd asks for when only some inputs need grads)
    for want in ((True, False, False), (False, True, False), (False, False, True), (True, True, False),
                 (True, False, True), (False, True, True)):
        tag = "".join(n for n, w in zip(("q", "qd", "tau"), want) if w)
        ops[f"fwd_dyn_vjp_{tag}_humanoid30_b32768_us"] = 1e3 * time_launches(
            lambda: rbd.fwd_dyn_vjp(model, vq, vqd, vtau, gq, want=want), n_t, torch)
    # the same two at batch 65536, where their waves fill every SIMD (32768 instances fill half)
    g65 = soa(W.cotangent(desc.nv, BATCH, 9), torch)
    ops["fwd_dyn_vjp_humanoid30_b65536_us"] = 1e3 * time_launches(
        lambda: rbd.fwd_dyn_vjp(model, q, qd, tau, g65), n_t, torch)
    tq, tqd, ttau = (soa(W._f32(np.random.default_rng(s).normal(size=(BATCH, r))), torch)
                     for s, r in ((11, desc.nq), (12, desc.nv), (13, desc.nv)))
    ops["fwd_dyn_jvp_humanoid30_b65536_us"] = 1e3 * time_launches(
        lambda: rbd.fwd_dyn_jvp(model, q, qd, tau, tq, tqd, ttau), n_t, torch)
    acc = soa(W._f32(np.random.default_rng(15).normal(size=(BATCH, desc.nv))), torch)
    ops["rnea_jvp_humanoid30_b65536_us"] = 1e3 * time_launches(
        lambda: rbd.rnea_jvp(model, q, qd, acc, tq, tqd, ttau), n_t, torch)
    ops["rnea_vjp_humanoid30_b65536_us"] = 1e3 * time_launches(
        lambda: rbd.rnea_vjp(model, q, qd, acc, g65), n_t, torch)
    del tq, tqd, ttau, g65, acc
    tg = soa(W._f32(targets(W, BATCH)), torch)
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
    hbm = {"write_gbs": round(max(rbd.hbm_rate(1 << 30, m, b) for m in (0, 2) for b in (0, 2048, 8192)), 1),
           "copy_gbs": round(max(rbd.hbm_rate(1 << 30, 1, b) for b in (0, 2048, 8192)), 1),
           "spec_gbs": PEAK_HBM_GBS,
           "how": "streaming kernels over 1 GiB (16-byte stores, non-temporal or plain; unrolled tiles or a "
                  "grid-stride loop), the best configuration, best of 10 launches each"}
    kernels = kernel_rooflines(O, W, desc, chain, ops, cnt, hbm)

    serving = None if args.no_serving else serving_leg(rbd, torch, args.serve_seconds, n_streams=args.serve_streams)
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
        "kernels": kernels,
        "hbm_ceiling": hbm,
        "cpu_baseline": cpu,
        "ops": ops,
        "serving": serving,
        "paper_context": "frax reports upwards of 1e8 dynamics evals/s at batch 4096 on an RTX 4090, "
                         "I/O included, robot and precision unstated (context, not a target)",
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

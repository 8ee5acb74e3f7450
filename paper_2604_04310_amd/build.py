"""Build librbd.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import os
import re
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librbd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HOST_SOURCES = ["rbd_api.cpp", "rbd_dispatch.cpp", "rbd_serve.cpp"]
DEVICE_SOURCES = ["rbd_diag.hip"]
TOPO_SOURCE = "rbd_kern_topo.hip"

# Packed FP32 (v_pk_*_f32) is switched off for every HIP translation unit.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          f"-I{INCLUDE}", f"-I{CSRC}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
DEVICE = ["--offload-arch=gfx950", "-ffp-contract=fast"]


def topologies():
    """Names in the RBD_TOPOLOGIES list, in order."""
    text = open(os.path.join(CSRC, "rbd_topologies.hpp")).read()
    return re.findall(r"^\s*X\((\w+),", text, flags=re.M)


def _jobs():
    cpus = os.cpu_count() or 4
    return max(1, min(16, cpus, int(os.environ.get("MAX_JOBS", cpus))))


def _newest_source() -> float:
    paths = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]
    return max(os.path.getmtime(p) for p in paths)


def build(verbose: bool = False, jobs: int = 0, resource_usage: bool = False, incremental: bool = False) -> str:
    """Compile one object per topology part plus the host sources in parallel, then link librbd.so.

    incremental=True skips objects newer than every source and header (a
    development convenience; the default always recompiles everything)."""
    out_dir = os.path.join(PKG, "_build")
    os.makedirs(out_dir, exist_ok=True)
    jobs = jobs or _jobs()
    work = []
    # the largest topologies first, so the longest compiles start early
    for name in reversed(topologies()):
        for part in (2, 7, 4, 6, 5, 3, 1):
            obj = os.path.join(out_dir, f"kern_{name}_p{part}.o")
            cmd = [HIPCC, *DEVICE, *COMMON, f"-DRBD_TOPO={name}", f"-DRBD_PART={part}", "-c",
                   os.path.join(CSRC, TOPO_SOURCE), "-o", obj]
            if resource_usage:
                cmd.append("-Rpass-analysis=kernel-resource-usage")
            work.append((obj, cmd))
    for src in DEVICE_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        work.append((obj, [HIPCC, *DEVICE, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]))
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        work.append((obj, [HIPCC, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]))
    t0 = time.time()
    running, logs, objs = [], [], []
    if incremental and not resource_usage:
        newest = _newest_source()
        fresh = [(o, c) for o, c in work if os.path.exists(o) and os.path.getmtime(o) > newest]
        objs = [o for o, _ in fresh]
        work = [(o, c) for o, c in work if (o, c) not in fresh]
    pending = list(work)
    while pending or running:
        while pending and len(running) < jobs:
            obj, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((obj, cmd, subprocess.Popen(cmd, stderr=subprocess.PIPE)))
        time.sleep(0.1)
        for item in list(running):
            obj, cmd, p = item
            if p.poll() is None:
                continue
            running.remove(item)
            err = p.stderr.read().decode()
            if p.returncode != 0:
                for _, _, q in running:
                    q.kill()
                sys.stderr.write(err)
                raise RuntimeError(f"compilation failed: {' '.join(cmd)}")
            logs.append(err)
            objs.append(obj)
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *sorted(objs), "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    if resource_usage:
        return "\n".join(logs)
    return LIB


if __name__ == "__main__":
    ru = "--resource-usage" in sys.argv
    out = build(verbose=True, resource_usage=ru, incremental="--incremental" in sys.argv)
    if ru:
        print(out)

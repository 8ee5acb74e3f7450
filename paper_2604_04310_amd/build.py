"""Build librbd.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import hashlib
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

HOST_SOURCES = ["rbd_api.cpp", "rbd_dispatch.cpp", "rbd_serve.cpp", "rbd_jit.cpp", "rbd_loadgen.cpp"]
DEVICE_SOURCES = ["rbd_diag.hip", "rbd_noalloc.hip"]
TOPO_SOURCE = "rbd_kern_topo.hip"
# Device headers the run-time compiler instantiates for a new topology; their
# text is embedded in the library.
JIT_HEADERS = ["rbd_kernels.hpp", "rbd_kernel_ids.hpp", "rbd_lane.hpp", "rbd_shared.hpp"]

# Packed FP32 (v_pk_*_f32) is switched off for every HIP translation unit.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          f"-I{INCLUDE}", f"-I{CSRC}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
DEVICE = ["--offload-arch=gfx950", "-ffp-contract=fast"]


# Topologies outside the compiled list whose run-time-compiled kernels are
# installed with the library (the "_jit" cache beside librbd.so, built by
# build()), so that their models load without compiling: a quadruped (free
# trunk, four 3-joint legs), random depth-first trees of 9 and 20 bodies on a
# fixed base and one of 40 bodies on a free base. Name: (floating, parents).
PREBUILT = {
    "quadruped13f": (True, [-1, 0, 1, 2, 0, 4, 5, 0, 7, 8, 0, 10, 11]),
    "tree9": (False, [-1, 0, 1, 1, 3, 0, 5, 6, 7]),
    "tree20": (False, [-1, 0, 1, 0, 3, 4, 3, 6, 7, 8, 9, 7, 0, 12, 12, 14, 14, 0, 17, 18]),
    "tree40f": (True, [-1, 0, 1, 0, 0, 0, 0, 6, 7, 8, 9, 10, 9, 0, 13, 0, 15, 16, 0, 0, 0, 0, 21, 0, 23, 24, 25, 0,
                       27, 28, 29, 30, 31, 32, 29, 34, 27, 0, 37, 38]),
}
# Controller kernels of frames other than the last body, installed the same
# way: topology name (compiled or PREBUILT) -> frames.
PREBUILT_FRAMES = {"humanoid30": [6, 22], "chain7": [3], "quadruped13f": [3]}
JIT_DIR = os.path.join(PKG, "_jit")
N_KERNELS = 40  # RBD_N_KERNELS


def _precompile_one(args):
    """One kernel of one topology into JIT_DIR (runs in a worker process)."""
    import ctypes as C
    name, floating, parent, kernel = args
    lib = C.CDLL(LIB)
    lib.rbd_precompile_topology.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.c_int, C.c_char_p, C.c_int32]
    lib.rbd_last_error.restype = C.c_char_p
    par = (C.c_int32 * len(parent))(*parent)
    st = lib.rbd_precompile_topology(len(parent), par, int(floating), JIT_DIR.encode(), kernel)
    return name, kernel, st, (lib.rbd_last_error().decode() if st else "")


def _elf_symbols(data: bytes):
    """Names of the symbols in an ELF64 little-endian image's .symtab."""
    import struct
    shoff, = struct.unpack_from("<Q", data, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", data, shoff + k * shentsize) for k in range(shnum)]
    names = []
    for sec in secs:
        if sec[1] != 2:  # SHT_SYMTAB
            continue
        strtab = secs[sec[6]]
        for off in range(sec[4], sec[4] + sec[5], sec[9]):
            name_off, = struct.unpack_from("<I", data, off)
            start = strtab[4] + name_off
            names.append(data[start:data.index(b"\0", start)].decode())
    return names


def _section(data: bytes, wanted: str) -> bytes:
    import struct
    shoff, = struct.unpack_from("<Q", data, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", data, shoff + k * shentsize) for k in range(shnum)]
    shstr = secs[shstrndx][4]
    for sec in secs:
        start = shstr + sec[0]
        if data[start:data.index(b"\0", start)].decode() == wanted:
            return data[sec[4]:sec[4] + sec[5]]
    raise ValueError(f"no section {wanted}")


def check_kernel_names(lib: str = LIB) -> int:
    """Every kernel the library registers on the host side (its __device_stub__ symbols) must exist,
    under the same name, in the gfx950 code objects embedded in the library; a launch of a
    registered kernel missing from its code object cannot be resolved. Returns the kernel count."""
    import struct
    data = open(lib, "rb").read()
    fat = _section(data, ".hip_fatbin")
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    device = set()
    pos = fat.find(magic)
    while pos >= 0:
        n, = struct.unpack_from("<Q", fat, pos + len(magic))
        q = pos + len(magic) + 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", fat, q)
            triple = fat[q + 24:q + 24 + tlen].decode()
            q += 24 + tlen
            if "gfx950" in triple and size:
                device.update(x[:-3] for x in _elf_symbols(fat[pos + off:pos + off + size]) if x.endswith(".kd"))
        pos = fat.find(magic, q)
    stubs = set()
    for sym in _elf_symbols(data):
        m = re.match(r"_ZN3rbd(\d+)__device_stub__(\w+)", sym)
        if m:
            name = sym[m.start(2):m.start(2) + int(m.group(1)) - len("__device_stub__")]
            rest = sym[m.start(2) + len(name):]
            stubs.add(f"_ZN3rbd{len(name)}{name}{rest}")
    missing = sorted(stubs - device)
    if missing or not stubs:
        raise RuntimeError(f"{lib}: {len(missing)} registered kernels are missing from the device code, e.g. "
                           f"{missing[:2]}" if missing else f"{lib}: no kernels registered")
    return len(stubs)


def prebuild_jit(verbose: bool = False, jobs: int = 0) -> None:
    """Compile every kernel of the PREBUILT topologies into the library's _jit
    cache, one kernel per worker process (hiprtc compiles one program at a
    time per process). Code objects already there are kept: the cache is keyed
    by a hash of the sources, options, topology and kernel."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    t0 = time.time()
    work = [(name, fl, par, k) for name, (fl, par) in PREBUILT.items() for k in range(N_KERNELS)]
    shapes = {**compiled_topologies(), **PREBUILT}
    for name, frames in PREBUILT_FRAMES.items():
        fl, par = shapes[name]
        work += [(f"{name} frame {f}", fl, par, N_KERNELS + 2 * f + osc) for f in frames for osc in (0, 1)]
    work.sort(key=lambda w: -len(w[2]))  # the largest trees first
    with ProcessPoolExecutor(max_workers=jobs or _jobs(), mp_context=mp.get_context("spawn")) as ex:
        for name, kernel, st, err in ex.map(_precompile_one, work):
            if st != 0:
                raise RuntimeError(f"precompiling kernel {kernel} of {name} failed: {err}")
    # every code object in use was just written or touched: the rest are stale
    for f in os.listdir(JIT_DIR):
        path = os.path.join(JIT_DIR, f)
        if f.endswith(".hsaco") and os.path.getmtime(path) < t0 - 1.0:
            os.remove(path)
    if verbose:
        print(f"jit cache: {len(work)} kernels of {len(PREBUILT)} topologies ready in {time.time() - t0:.1f}s",
              flush=True)


def compiled_topologies():
    """name -> (floating, parents) of every topology compiled ahead of time."""
    text = open(os.path.join(CSRC, "rbd_topologies.hpp")).read().replace("\\\n", " ")
    return {name: (fr == "true", [int(x) for x in par.split(",")])
            for name, fr, par in re.findall(r"X\((\w+), (true|false), ([-0-9, \s]+)\)", text)}


def topologies():
    """Names in the RBD_TOPOLOGIES list, in order."""
    text = open(os.path.join(CSRC, "rbd_topologies.hpp")).read()
    return re.findall(r"^\s*X\((\w+),", text, flags=re.M)


def _jobs():
    cpus = os.cpu_count() or 4
    return max(1, min(16, cpus, int(os.environ.get("MAX_JOBS", cpus))))


# What each kind of object is compiled from (for incremental builds).
DEVICE_DEPS = [TOPO_SOURCE, "rbd_kernels.hpp", "rbd_kernel_ids.hpp", "rbd_lane.hpp", "rbd_shared.hpp",
               "rbd_topologies.hpp"]
HOST_HEADERS = ["rbd_internal.hpp", "rbd_shared.hpp", "rbd_kernel_ids.hpp", "rbd_topologies.hpp"]


def _inputs_hash(obj: str, cmd) -> str:
    """Hash of an object's compile command and the text of every file it is compiled from, taken
    before the compile starts. An incremental build reuses an object only if the hash recorded
    with it matches: a file edited while its compile ran (hipcc reads the headers once for the
    device pass and again for the host pass, so such an object can pair a host stub with device
    code of another version) leaves a stale hash, and the object is compiled again."""
    h = hashlib.sha256(" ".join(cmd).encode())
    for path in _deps(obj, cmd):
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _deps(obj: str, cmd) -> list:
    """Sources and headers an object depends on."""
    inc = [os.path.join(INCLUDE, "rbd.h")]
    if os.path.basename(obj).startswith("kern_"):
        return [os.path.join(CSRC, f) for f in DEVICE_DEPS]
    src = cmd[-3]  # ... -c <source> -o <object>
    return [src] + [os.path.join(CSRC, f) for f in HOST_HEADERS] + inc


def write_jit_sources(out_dir: str) -> str:
    """A C++ source holding the device headers' text (for hiprtc at run time)."""
    path = os.path.join(out_dir, "rbd_jit_sources.cpp")
    parts = ["// Generated by build.py: the device headers, compiled at run time for new topologies.",
             "namespace rbd {", f"extern const int kJitNumHeaders = {len(JIT_HEADERS)};",
             "extern const char* const kJitHeaderNames[] = {" + ", ".join(f'"{h}"' for h in JIT_HEADERS) + "};",
             "extern const char* const kJitHeaderTexts[] = {"]
    for h in JIT_HEADERS:
        text = open(os.path.join(CSRC, h)).read()
        assert ')rbdjit"' not in text
        parts.append('R"rbdjit(' + text + ')rbdjit",')
    parts += ["};", "}  // namespace rbd", ""]
    new = "\n".join(parts)
    if not os.path.exists(path) or open(path).read() != new:
        with open(path, "w") as fh:
            fh.write(new)
    return path


def build(verbose: bool = False, jobs: int = 0, resource_usage: bool = False, incremental: bool = False) -> str:
    """Compile one object per topology part plus the host sources in parallel, then link librbd.so.

    incremental=True skips objects newer than every source and header they
    are compiled from (a development convenience; the default always
    recompiles everything)."""
    out_dir = os.path.join(PKG, "_build")
    os.makedirs(out_dir, exist_ok=True)
    jobs = jobs or _jobs()
    work = []
    # the largest topologies first, so the longest compiles start early
    for name in reversed(topologies()):
        for part in (8, 2, 7, 4, 6, 5, 3, 1):
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
    jit_src = write_jit_sources(out_dir)
    obj = os.path.join(out_dir, "rbd_jit_sources.o")
    work.append((obj, [HIPCC, *COMMON, "-c", jit_src, "-o", obj]))
    t0 = time.time()
    running, logs, objs = [], [], []
    def recorded(o):
        try:
            with open(o + ".inputs") as fh:
                return fh.read().strip()
        except OSError:
            return None

    if incremental and not resource_usage:
        fresh = [(o, c) for o, c in work if os.path.exists(o) and recorded(o) == _inputs_hash(o, c)]
        objs = [o for o, _ in fresh]
        work = [(o, c) for o, c in work if (o, c) not in fresh]
    pending = list(work)
    while pending or running:
        while pending and len(running) < jobs:
            obj, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            if os.path.exists(obj + ".inputs"):
                os.remove(obj + ".inputs")
            digest = _inputs_hash(obj, cmd)
            running.append((obj, cmd, digest, subprocess.Popen(cmd, stderr=subprocess.PIPE)))
        time.sleep(0.1)
        for item in list(running):
            obj, cmd, digest, p = item
            if p.poll() is None:
                continue
            running.remove(item)
            err = p.stderr.read().decode()
            if p.returncode != 0:
                for _, _, _, q in running:
                    q.kill()
                sys.stderr.write(err)
                raise RuntimeError(f"compilation failed: {' '.join(cmd)}")
            with open(obj + ".inputs", "w") as fh:
                fh.write(digest + "\n")
            logs.append(err)
            objs.append(obj)
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *sorted(objs), "-o", tmp, "-lpthread", "-lhiprtc",
            "-ldl"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    check_kernel_names(tmp)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    prebuild_jit(verbose, jobs)
    if resource_usage:
        return "\n".join(logs)
    return LIB


if __name__ == "__main__":
    ru = "--resource-usage" in sys.argv
    out = build(verbose=True, resource_usage=ru, incremental="--incremental" in sys.argv)
    if ru:
        print(out)

"""The C ABI on the CPU: the library loads without a GPU, exports every symbol
include/rbd.h declares, and rejects bad models with the documented status."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rbd():
    import paper_2604_04310_amd as rbd
    if not os.path.exists(rbd.LIB_PATH):
        pytest.skip("librbd.so not built")
    rbd.lib()
    return rbd


def test_header_declarations_are_exported(rbd):
    header = open(os.path.join(ROOT, "include", "rbd.h")).read()
    declared = set(re.findall(r"\b(rbd_[a-z_]+)\s*\(", header))
    assert declared == set(rbd.EXPORTS)
    for name in declared:
        assert hasattr(rbd.lib(), name), name


def test_status_strings(rbd):
    L = rbd.lib()
    assert L.rbd_status_str(0) == b"ok"
    assert L.rbd_status_str(1) == b"invalid argument"
    assert L.rbd_status_str(5) == b"unsupported topology"


def _create(rbd, desc):
    h = C.c_void_p()
    s = rbd.desc_struct(desc) if desc is not None else None
    st = rbd.lib().rbd_model_create(C.byref(s) if s is not None else None, 0, C.byref(h))
    if st == 0:
        rbd.lib().rbd_model_destroy(h)
    return st, rbd.lib().rbd_last_error().decode()


def _mutated(**kw):
    d = W.chain(7)
    for k, fn in kw.items():
        arr = getattr(d, k).copy()
        fn(arr)
        setattr(d, k, arr)
    return d


@pytest.mark.parametrize("case,msg", [
    ("parent_order", "parent"), ("free_not_root", "free joint"), ("zero_axis", "axis"),
    ("bad_rotation", "rotation"), ("mass", "mass"), ("not_pd", "positive definite"),
    ("triangle", "triangle"), ("not_dfs", "contiguous"), ("bad_joint", "joint_type"),
])
def test_invalid_models_are_rejected(rbd, case, msg):
    muts = {
        "parent_order": dict(parent=lambda a: a.__setitem__(3, 5)),
        "free_not_root": dict(joint_type=lambda a: a.__setitem__(2, 1)),
        "zero_axis": dict(axis=lambda a: a.__setitem__(1, 0.0)),
        "bad_rotation": dict(origin=lambda a: a.__setitem__((2, 0), 2.0)),
        "mass": dict(mass=lambda a: a.__setitem__(4, -1.0)),
        "not_pd": dict(inertia=lambda a: a.__setitem__(0, [-1.0, 1, 1, 0, 0, 0])),
        "triangle": dict(inertia=lambda a: a.__setitem__(0, [1.0, 1.0, 5.0, 0, 0, 0])),
        "bad_joint": dict(joint_type=lambda a: a.__setitem__(3, 7)),
    }
    if case == "not_dfs":
        d = W.random_tree([-1, 0, 0, 1], False, 3)  # body 3 hangs under 1 after 2: not depth-first
    else:
        d = _mutated(**muts[case])
    st, err = _create(rbd, d)
    assert st == 1, (st, err)
    assert msg in err


def test_null_desc(rbd):
    st, err = _create(rbd, None)
    assert st == 1 and "NULL" in err


def test_new_topology_without_device(rbd):
    """A valid tree outside the compiled list is accepted (its kernels are compiled at run time on a
    device host); without a GPU the call stops at the device check, before compiling."""
    st, err = _create(rbd, W.random_tree([-1, 0, 0], False, 4))
    if rbd.device_count() == 0:
        assert st == 3, err


def test_precompile_writes_every_kernel(rbd, tmp_path):
    """Run-time compilation without a GPU: one kernel, then every kernel of a new topology into a
    cache directory; a second call finds them all there and compiles nothing."""
    import time
    rbd.precompile_topology([-1, 0], False, str(tmp_path), kernel=7)
    assert len([f for f in os.listdir(tmp_path) if f.endswith(".hsaco")]) == 1
    rbd.precompile_topology([-1, 0], False, str(tmp_path))
    files = sorted(f for f in os.listdir(tmp_path) if f.endswith(".hsaco"))
    assert len(files) == rbd.N_KERNELS
    blobs = [open(os.path.join(tmp_path, f), "rb").read() for f in files]
    t0 = time.time()
    rbd.precompile_topology([-1, 0], False, str(tmp_path))
    assert time.time() - t0 < 2.0  # cache hits only
    assert sorted(f for f in os.listdir(tmp_path) if f.endswith(".hsaco")) == files
    assert blobs == [open(os.path.join(tmp_path, f), "rb").read() for f in files]


def test_precompile_rejects_bad_topologies(rbd, tmp_path):
    with pytest.raises(rbd.RbdError):
        rbd.precompile_topology([-1, 0, 0, 1], False, str(tmp_path))  # not depth-first
    with pytest.raises(rbd.RbdError):
        rbd.precompile_topology([0], False, str(tmp_path))
    with pytest.raises(rbd.RbdError):
        rbd.precompile_topology([-1] * 65, False, str(tmp_path))
    with pytest.raises(rbd.RbdError):
        rbd.precompile_topology([-1, 0], False, str(tmp_path), kernel=rbd.N_KERNELS + 4)  # 2 bodies
    with pytest.raises(rbd.RbdError):
        rbd.precompile_topology([-1, 0], False, str(tmp_path), kernel=-2)


def test_prebuilt_topologies_are_new_and_installed(rbd):
    """The shapes installed with run-time-compiled kernels are not compiled topologies, and build()
    put all of the kernels of each in the library's cache."""
    from paper_2604_04310_amd.build import CSRC, JIT_DIR, PREBUILT
    import workloads as W2
    text = open(os.path.join(CSRC, "rbd_topologies.hpp")).read().replace("\\\n", " ")
    compiled = {(fr == "true", tuple(int(x) for x in par.split(",")))
                for fr, par in re.findall(r"X\(\w+, (true|false), ([-0-9, ]+)\)", text)}
    assert len(compiled) == 11
    assert not {(fl, tuple(par)) for fl, par in PREBUILT.values()} & compiled
    assert PREBUILT["tree9"][1] == W2.random_dfs_parents(9, 2)
    assert PREBUILT["tree20"][1] == W2.random_dfs_parents(20, 4)
    assert PREBUILT["tree40f"][1] == W2.random_dfs_parents(40, 9)
    assert PREBUILT["quadruped13f"][1] == W2.QUADRUPED_PARENT
    assert len([f for f in os.listdir(JIT_DIR) if f.endswith(".hsaco")]) >= 30 * len(PREBUILT)


def test_valid_model_without_device(rbd):
    st, err = _create(rbd, W.chain(7))
    if rbd.device_count() == 0:
        assert st == 3, err
    else:
        assert st == 0, err


def test_null_model_calls(rbd):
    L = rbd.lib()
    assert L.rbd_fwd_dyn(None, 1, 1, None, None, None, None, None, None) == 1
    assert b"model is NULL" in L.rbd_last_error()
    assert L.rbd_aba(None, 1, 1, None, None, None, None, None, None) == 1
    assert L.rbd_rnea(None, 1, 1, None, None, None, None, None, None) == 1
    assert L.rbd_fwd_dyn_jvp(None, 1, 1, *([None] * 11)) == 1
    assert b"model is NULL" in L.rbd_last_error()
    assert L.rbd_fwd_dyn_vjp(None, 1, 1, *([None] * 10)) == 1
    assert b"model is NULL" in L.rbd_last_error()
    assert L.rbd_rnea_jvp(None, 1, 1, *([None] * 10)) == 1
    assert b"model is NULL" in L.rbd_last_error()
    assert L.rbd_rnea_vjp(None, 1, 1, *([None] * 10)) == 1
    assert b"model is NULL" in L.rbd_last_error()
    assert L.rbd_packed_static(None, 0, 1, None, None) == 1
    assert b"model is NULL" in L.rbd_last_error()


def _server_create(rbd, **kw):
    cfg = dict(device=0, arena_bytes=1 << 24, n_streams=2, max_batch_requests=64, max_wait_us=0.0,
               use_graphs=1, per_request=0, executor=0, fail_group=0)
    cfg.update(kw)
    from paper_2604_04310_amd import rbd as R
    c = R.ServerConfigC(cfg["device"], cfg["arena_bytes"], cfg["n_streams"], cfg["max_batch_requests"],
                        cfg["max_wait_us"], cfg["use_graphs"], cfg["per_request"], cfg["executor"],
                        cfg["fail_group"])
    h = C.c_void_p()
    st = rbd.lib().rbd_server_create(C.byref(c), C.byref(h))
    if st == 0:
        rbd.lib().rbd_server_destroy(h)
    return st, rbd.lib().rbd_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(n_streams=0), "n_streams"), (dict(n_streams=9), "n_streams"),
    (dict(max_batch_requests=0), "max_batch_requests"), (dict(max_batch_requests=5000), "max_batch_requests"),
    (dict(arena_bytes=1024), "arena_bytes"), (dict(max_wait_us=-1.0), "max_wait_us"),
])
def test_server_config_validation(rbd, kw, msg):
    st, err = _server_create(rbd, **kw)
    assert st == 1 and msg in err


def test_server_needs_a_device(rbd):
    st, err = _server_create(rbd)
    if rbd.device_count() == 0:
        assert st == 3, err
    else:
        assert st == 0, err


def test_server_null_handles(rbd):
    L = rbd.lib()
    t = C.c_uint64()
    assert L.rbd_server_submit(None, None, 0, 1, None, None, C.byref(t)) == 1
    assert L.rbd_server_wait(None, 1, 0.0, None) == 1
    assert L.rbd_server_destroy(None) == 0


def test_parity_tests_cover_every_compiled_topology():
    """The GPU parity lists name every topology the library compiles, and nothing else."""
    from paper_2604_04310_amd.build import topologies
    from tests.test_gpu_parity import EXTRA_TOPOLOGIES, MODELS
    assert set(MODELS) | set(EXTRA_TOPOLOGIES) == set(topologies())
    assert not set(MODELS) & set(EXTRA_TOPOLOGIES)


def test_registered_kernels_exist_in_device_code(rbd):
    """Every kernel the library registers on the host side exists under the same name in its
    embedded gfx950 code objects (a stale object pairing a host stub of one header version with
    device code of another would make its launches unresolvable)."""
    from paper_2604_04310_amd.build import check_kernel_names
    assert check_kernel_names(rbd.LIB_PATH) >= 11 * rbd.N_KERNELS


def test_plain_c_program_uses_the_boundary(rbd, tmp_path):
    """include/rbd.h compiles as C11 and librbd.so links and runs from a C program with no Python in
    the loop: a host-only model (dimensions, a compute call refused without kernels, an invalid tree
    rejected with a message) and a server with the host executor (submit, wait, statistics)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lib_dir = os.path.dirname(rbd.LIB_PATH)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "c_abi_host")
    subprocess.run([gcc, "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I" + os.path.join(root, "include"), "-I" + os.path.join(rocm, "include"),
                    os.path.join(root, "tests", "c_abi_host.c"), "-o", exe, rbd.LIB_PATH,
                    "-Wl,-rpath," + lib_dir], check=True, capture_output=True, timeout=120)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "c abi ok"


def test_kernel_count_is_the_same_everywhere(rbd):
    """The kernel list (csrc/rbd_kernel_ids.hpp), RBD_N_KERNELS in include/rbd.h, the binding and the
    build all count the same kernels."""
    from paper_2604_04310_amd import build as B
    ids = open(os.path.join(ROOT, "paper_2604_04310_amd", "csrc", "rbd_kernel_ids.hpp")).read()
    listed = re.findall(r"^\s*X\((KID_\w+),", ids, flags=re.M)
    assert len(listed) == len(set(listed))
    header = open(os.path.join(ROOT, "include", "rbd.h")).read()
    declared = int(re.search(r"#define RBD_N_KERNELS (\d+)", header).group(1))
    assert len(listed) == declared == rbd.N_KERNELS == B.N_KERNELS


def test_packed_static_rejects_host_only_models_and_bad_arguments(rbd):
    """rbd_packed_static's host-side checks that need no GPU: a null model and a host-only model
    (device -1) are refused before anything is launched."""
    L = rbd.lib()
    s = rbd.desc_struct(W.chain(3))
    h = C.c_void_p()
    assert L.rbd_model_create(C.byref(s), -1, C.byref(h)) == 0
    try:
        req = (rbd.rbd.PackedRequestC * 1)()
        assert L.rbd_packed_static(h, 0, 1, req, None) == 1
        assert b"host-only" in L.rbd_last_error()
    finally:
        L.rbd_model_destroy(h)
    assert L.rbd_packed_static(None, 0, 0, None, None) == 1  # the model is checked first
    assert b"model is NULL" in L.rbd_last_error()

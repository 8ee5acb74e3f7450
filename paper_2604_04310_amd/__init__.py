"""Batched rigid-body kinematics and dynamics on one MI355X (arxiv 2604.04310, frax).

The compute path is librbd.so (hand-written HIP kernels for gfx950 behind the C
ABI in include/rbd.h); this package is its thin Python binding.
"""
from .rbd import (EXPORTS, LIB_PATH, Model, RbdError, aba, crba, desc_struct, device_count, diff_ik, fma_rate,  # noqa: F401
                  hbm_rate, precompile_topology, N_KERNELS, packed_static,
                  fk, fwd_dyn, osc,
                  fwd_dyn_autograd, fwd_dyn_jvp, fwd_dyn_vjp, rnea_jvp, rnea_vjp, rnea_autograd, jacobian, lib, rnea, Server, op_shapes,
                  OP_FWD_DYN, OP_RNEA, OP_FWD_DYN_VJP, EXEC_DEVICE, EXEC_HOST)

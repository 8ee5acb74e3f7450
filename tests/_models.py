"""The seeded robots the GPU tests run, shared by the parity and controller tests."""
from __future__ import annotations

import numpy as np

import workloads as W

TREE12 = [-1, 0, 1, 1, 0, 4, 5, 5, 7, 0, 9, 10]
# One model per compiled topology that the per-row tests visit (identity joint-origin rotations,
# gravity along -z, joint angles in [-pi, pi]).
MODELS = {
    "chain1": lambda: W.random_tree([-1], False, 31),
    "chain2": lambda: W.random_tree([-1, 0], False, 32),
    "chain7": lambda: W.chain(7),
    "free1": lambda: W.random_tree([-1], True, 33),
    "tree12f": lambda: W.random_tree(TREE12, True, 34),
    "humanoid30": lambda: W.humanoid(),
}
# URDF-style models: a random fixed rotation on every joint origin, gravity in a random direction,
# and joint angles of continuous joints that have turned many times (|q| up to 1000 rad). They run
# the compiled kernels of the same topologies through the host's table precomputation and the
# kernels' angle reduction, which the models above leave at identity and |q| <= pi.
ROTATED = {
    "chain7_rot": lambda: W.chain(7, 60, rotated=True, gravity=W.tilted_gravity(61)),
    "tree12f_rot": lambda: W.random_tree(TREE12, True, 62, rotated=True, gravity=W.tilted_gravity(63)),
    "humanoid30_rot": lambda: W.humanoid(64, rotated=True, gravity=W.tilted_gravity(65)),
}
Q_RANGE = {name: 1000.0 for name in ROTATED}
ALL = {**MODELS, **ROTATED}


def draw(name, desc, batch, seed):
    """The seeded states of a model: joint angles in [-pi, pi], or up to 1000 rad for ROTATED."""
    return W.states(desc, batch, seed, q_range=Q_RANGE.get(name, np.pi))

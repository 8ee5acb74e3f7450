"""Seeded synthetic robots and robot states.

This module is shared by the tests, the benchmark and the smoke check. It only
draws random numbers and lays them out: it holds none of the dynamics
arithmetic, so neither the FP64 oracle nor the GPU path depends on the other
through it.

The paper measures on a Franka Panda arm and a Unitree G1 humanoid (abstract,
Fig. 1, Sec. V and Table II); their model files are not available, so synthetic
kinematic trees of the same shape stand in for them:

* a serial chain of revolute joints (the arm), and
* a 30-body floating-base tree (the humanoid): a 6-DoF free base plus 29
  revolute joints in two 6-joint legs, a 3-joint waist and two 7-joint arms.

Every generated value is rounded to FP32 and returned as float64, so that the
FP64 oracle and the FP32 kernels see exactly the same numbers and a parity
check measures kernel error only, never input quantisation.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

REVOLUTE = 0
FREE = 1

# Seeds of the standard workloads (numpy PCG64).
SEED_CHAIN_MODEL = 0
SEED_TREE_MODEL = 1


def _f32(x):
    """Round to the nearest FP32 value, returned as float64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclass
class TreeDesc:
    """A kinematic tree, bodies numbered so that parent[i] < i (-1 = world).

    joint_type[i] is REVOLUTE or FREE (FREE only for body 0). For a revolute
    joint the body frame is the joint frame: it sits at ``origin`` p (in the
    parent body frame), is turned by the fixed rotation R (row-major in
    ``origin[:9]``) and then by q about the unit ``axis``. A FREE body's pose
    comes from q directly (position, then quaternion w,x,y,z); its ``origin``
    and ``axis`` are not used. Inertia is about the CoM in the body frame,
    ordered xx yy zz xy xz yz.
    """

    parent: np.ndarray
    joint_type: np.ndarray
    axis: np.ndarray
    origin: np.ndarray
    mass: np.ndarray
    com: np.ndarray
    inertia: np.ndarray
    gravity: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, -9.81]))
    name: str = "tree"

    @property
    def n_bodies(self) -> int:
        return int(self.parent.shape[0])

    @property
    def floating(self) -> bool:
        return bool(self.joint_type[0] == FREE)

    @property
    def nq(self) -> int:
        return self.n_bodies + (6 if self.floating else 0)

    @property
    def nv(self) -> int:
        return self.n_bodies + (5 if self.floating else 0)

    def contiguous(self) -> "TreeDesc":
        return TreeDesc(
            parent=np.ascontiguousarray(self.parent, dtype=np.int32),
            joint_type=np.ascontiguousarray(self.joint_type, dtype=np.int32),
            axis=np.ascontiguousarray(self.axis, dtype=np.float64),
            origin=np.ascontiguousarray(self.origin, dtype=np.float64),
            mass=np.ascontiguousarray(self.mass, dtype=np.float64),
            com=np.ascontiguousarray(self.com, dtype=np.float64),
            inertia=np.ascontiguousarray(self.inertia, dtype=np.float64),
            gravity=np.ascontiguousarray(self.gravity, dtype=np.float64),
            name=self.name,
        )


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation from a normalised Gaussian quaternion (w, x, y, z)."""
    qv = rng.normal(size=4)
    qv /= np.linalg.norm(qv)
    w, x, y, z = qv
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def random_inertia(rng: np.random.Generator, m: float, r_lo=0.03, r_hi=0.15) -> np.ndarray:
    """Inertia about the CoM, R diag(a,b,c) R^T, triangle inequality by construction.

    With d_k = m r_k^2, a = d2+d3, b = d1+d3, c = d1+d2 are the principal
    moments of three point-mass pairs, so a+b >= c etc. always hold.
    """
    r = rng.uniform(r_lo, r_hi, size=3)
    d = m * r * r
    diag = np.array([d[1] + d[2], d[0] + d[2], d[0] + d[1]])
    R = random_rotation(rng)
    I = R @ np.diag(diag) @ R.T
    return np.array([I[0, 0], I[1, 1], I[2, 2], I[0, 1], I[0, 2], I[1, 2]])


def random_axis(rng: np.random.Generator) -> np.ndarray:
    a = rng.normal(size=3)
    return a / np.linalg.norm(a)


def _random_bodies(rng, parent, joint_type, name, rotated=False, gravity=None):
    """rotated: each revolute joint frame gets a uniform random fixed rotation
    (as URDF joint origins carry); otherwise the fixed rotation is identity.
    gravity: the gravity vector (default (0, 0, -9.81))."""
    n = len(parent)
    axis = np.zeros((n, 3))
    origin = np.zeros((n, 12))
    mass = np.zeros(n)
    com = np.zeros((n, 3))
    inertia = np.zeros((n, 6))
    for i in range(n):
        origin[i, 0:9] = np.eye(3).reshape(-1)          # fixed rotation = identity
        if joint_type[i] == REVOLUTE:
            origin[i, 9:12] = rng.uniform(-0.3, 0.3, size=3)
            axis[i] = random_axis(rng)
            if rotated:
                origin[i, 0:9] = random_rotation(rng).reshape(-1)
        else:
            axis[i] = [0.0, 0.0, 1.0]                    # unused by a free joint
        mass[i] = rng.uniform(0.5, 4.0)
        com[i] = rng.uniform(-0.1, 0.1, size=3)
        inertia[i] = random_inertia(rng, mass[i])
    desc = TreeDesc(
        parent=np.asarray(parent, dtype=np.int32),
        joint_type=np.asarray(joint_type, dtype=np.int32),
        axis=_f32(axis), origin=_f32(origin), mass=_f32(mass), com=_f32(com),
        inertia=_f32(inertia), gravity=_f32([0.0, 0.0, -9.81] if gravity is None else gravity), name=name)
    # Renormalising after rounding would move the value off the FP32 grid; a
    # rounded unit vector is unit to ~6e-8, which both sides accept as given.
    return desc


def chain(n: int = 7, seed: int = SEED_CHAIN_MODEL, rotated: bool = False, gravity=None) -> TreeDesc:
    """Serial chain of n revolute joints (the arm workload; 7 joints by default)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _random_bodies(rng, list(range(-1, n - 1)), [REVOLUTE] * n, f"chain{n}", rotated, gravity)


HUMANOID_PARENT = (
    [-1]                                   # 0 pelvis (free)
    + [0, 1, 2, 3, 4, 5]                   # 1-6 left leg
    + [0, 7, 8, 9, 10, 11]                 # 7-12 right leg
    + [0, 13, 14]                          # 13-15 waist
    + [15, 16, 17, 18, 19, 20, 21]         # 16-22 left arm
    + [15, 23, 24, 25, 26, 27, 28]         # 23-29 right arm
)


def humanoid(seed: int = SEED_TREE_MODEL, rotated: bool = False, gravity=None) -> TreeDesc:
    """30-body floating-base tree: free pelvis, 2 legs x 6, waist 3, 2 arms x 7."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jt = [FREE] + [REVOLUTE] * 29
    return _random_bodies(rng, HUMANOID_PARENT, jt, "humanoid30", rotated, gravity)


def random_tree(parent, floating: bool, seed: int, rotated: bool = False, gravity=None) -> TreeDesc:
    """Any topologically sorted tree with the standard inertial sampling."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jt = [FREE if (floating and i == 0) else REVOLUTE for i in range(len(parent))]
    return _random_bodies(rng, list(parent), jt, f"tree{len(parent)}{'f' if floating else ''}", rotated, gravity)


def random_dfs_parents(n: int, seed: int, p_continue: float = 0.6) -> list:
    """A random tree of n bodies numbered depth-first: body i hangs on body i-1
    with probability p_continue, else on a uniformly chosen body of the path
    from the root to body i-1 (the root itself when the path is short)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parent = [-1]
    for i in range(1, n):
        path = []
        k = i - 1
        while k >= 0:
            path.append(k)
            k = parent[k]
        parent.append(i - 1 if rng.random() < p_continue else int(path[rng.integers(len(path))]))
    return parent


# A quadruped: a free trunk and four 3-joint legs.
QUADRUPED_PARENT = [-1, 0, 1, 2, 0, 4, 5, 0, 7, 8, 0, 10, 11]


def tilted_gravity(seed: int) -> np.ndarray:
    """A gravity vector of magnitude 9.81 in a random direction (for models whose world z is not up)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return 9.81 * random_axis(rng)


@dataclass
class States:
    """A batch of robot states, instance-major: q [B, nq], qd [B, nv], tau [B, nv]."""

    q: np.ndarray
    qd: np.ndarray
    tau: np.ndarray

    @property
    def batch(self) -> int:
        return int(self.q.shape[0])


def states(desc: TreeDesc, batch: int, seed: int, q_range: float = np.pi) -> States:
    """q ~ U(-q_range, q_range) per revolute joint (pi by default; larger for
    continuous joints that have turned many times), qd ~ N(0, 1), tau ~ N(0, 5)
    (sigma 5).

    A free base takes its position from U(-1, 1)^3 and its orientation as a
    uniform unit quaternion (normalised Gaussian, w first).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nq, nv = desc.nq, desc.nv
    q = np.empty((batch, nq))
    if desc.floating:
        q[:, 0:3] = rng.uniform(-1.0, 1.0, size=(batch, 3))
        quat = rng.normal(size=(batch, 4))
        quat /= np.linalg.norm(quat, axis=1, keepdims=True)
        q[:, 3:7] = quat
        q[:, 7:] = rng.uniform(-q_range, q_range, size=(batch, nq - 7))
    else:
        q[:] = rng.uniform(-q_range, q_range, size=(batch, nq))
    qd = rng.normal(0.0, 1.0, size=(batch, nv))
    tau = rng.normal(0.0, 5.0, size=(batch, nv))
    return States(q=_f32(q), qd=_f32(qd), tau=_f32(tau))


def cotangent(nv: int, batch: int, seed: int) -> np.ndarray:
    """Random cotangent for q-double-dot, N(0, 1), FP32-rounded, [B, nv]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return _f32(rng.normal(size=(batch, nv)))


def soa(x: np.ndarray, ld: int | None = None) -> np.ndarray:
    """[B, n] instance-major -> [n, ld] structure-of-arrays (zero padded)."""
    B, n = x.shape
    ld = B if ld is None else ld
    out = np.zeros((n, ld), dtype=x.dtype)
    out[:, :B] = x.T
    return out

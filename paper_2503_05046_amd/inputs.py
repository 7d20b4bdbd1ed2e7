"""Seeded synthetic scenes for the MPM-rigid substep.

This module only builds inputs: particle arrays, grid geometry, material and
rigid-body tables. It holds none of the method's arithmetic, and both the GPU
library and the CPU oracle consume what it returns.

Workloads (the paper's robotics scenes, Table I, are not available, so these
synthetic scenes of the same kind stand in for them, larger and denser):

* ``plain_cube``     elastic cube (fixed-corotated, E=1e5, nu=0.3, rho=1000) of
                     20^3 particles on a 32^3 grid over a rigid half-space,
                     mu=0.5, h=2e-4. ``contact=True`` places it just above the
                     plane moving at (0.5, 0, -1) m/s so contact starts at once.
* ``granular_pour``  1M Drucker-Prager sand particles (30 deg, E=3.5e5,
                     nu=0.3) uniform in a 0.4^3 box on a 128^3 grid, falling at
                     1 m/s onto four static boxes (mu=0.4), h=1e-4.
* ``gripper``        250k-particle elastic ellipsoid (E=5e4, nu=0.4) on a 96^3
                     grid between two kinematic jaw boxes closing at 0.05 m/s,
                     mu=0.8, h=1e-4, 10 substeps per rigid step.
* ``batched``        many independent environments in one handle: particle
                     counts log-uniform in [p_min, p_max], each env with its own
                     n^3 grid (dx = 1/n), elastic or sand at random, a particle
                     cube resting on a floor slab and moving down at 0.5 m/s,
                     0-2 more boxes beside it, mu uniform in [0.2, 0.9].
* ``differentiable`` 200k-particle elastic cube on a 96^3 grid pushed by a
                     kinematic box at 0.5 m/s (the backward-form workload).
* ``tiny_block`` / ``tiny_random``: small scenes for exhaustive checks.

Units are SI, z is up, gravity is (0, 0, -9.81). The domain of every env is
[0, 1)^3 with grid node (i, j, k) at origin + (i, j, k) * dx. Particle arrays
are float32 and component-major: x, v are [3, P], F and C are [9, P] with
row-major 3x3 per particle.

The contact stiffness is k = kappa * E * V0^(1/3) with kappa = 10, the
dissipation d = 0 and the friction regularisation eps_s = 1e-4 m/s (the paper
defers these constants to its references; see the design notes).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

FIXED_COROTATED = 0
DRUCKER_PRAGER = 1
HALF_SPACE = 0
BOX = 1
STATIC = 0
KINEMATIC = 1
DYNAMIC = 2

KAPPA = 10.0
EPS_S = 1e-4
GRAVITY = (0.0, 0.0, -9.81)


@dataclasses.dataclass
class EnvSpec:
    dims: Sequence[int]
    dx: float
    origin: Sequence[float] = (0.0, 0.0, 0.0)
    gravity: Sequence[float] = GRAVITY
    material: int = FIXED_COROTATED
    E: float = 1e5
    nu: float = 0.3
    rho: float = 1000.0
    V0: float = 1e-6
    friction_angle: float = 30.0
    k: float = 0.0
    d: float = 0.0
    eps_s: float = EPS_S
    p_begin: int = 0
    p_end: int = 0

    @property
    def m_p(self) -> float:
        return self.rho * self.V0


@dataclasses.dataclass
class RigidSpec:
    env: int
    shape: int
    mu: float
    motion: int = STATIC
    normal: Sequence[float] = (0.0, 0.0, 1.0)
    offset: float = 0.0
    half: Sequence[float] = (0.0, 0.0, 0.0)
    R: Sequence[float] = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0)
    t: Sequence[float] = (0.0, 0.0, 0.0)
    V: Sequence[float] = (0.0, 0.0, 0.0)
    w: Sequence[float] = (0.0, 0.0, 0.0)
    # DYNAMIC boxes (body origin at the centre of mass)
    mass: float = 0.0
    inertia: Sequence[float] = (0.0, 0.0, 0.0)
    force: Sequence[float] = (0.0, 0.0, 0.0)
    torque: Sequence[float] = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Scene:
    name: str
    h: float
    N: int
    envs: List[EnvSpec]
    rigids: List[RigidSpec]
    x: np.ndarray
    v: np.ndarray
    F: np.ndarray
    C: np.ndarray
    eps_r: float = 1e-6
    eps_a: float = 2.220446049250313e-16
    max_iter: int = 500
    ls_max_iter: int = 100

    @property
    def P(self) -> int:
        return int(self.x.shape[1])

    def copy(self) -> "Scene":
        s = dataclasses.replace(self)
        s.envs = [dataclasses.replace(e) for e in self.envs]
        s.rigids = [dataclasses.replace(r) for r in self.rigids]
        s.x, s.v, s.F, s.C = self.x.copy(), self.v.copy(), self.F.copy(), self.C.copy()
        return s


def single_env(scene: Scene, e: int) -> Scene:
    """Environment e of a scene as a scene of its own (same state and rigids)."""
    env = dataclasses.replace(scene.envs[e])
    sl = slice(env.p_begin, env.p_end)
    env.p_begin, env.p_end = 0, env.p_end - env.p_begin
    rig = [dataclasses.replace(r, env=0) for r in scene.rigids if r.env == e]
    out = dataclasses.replace(scene, name=f"{scene.name}[{e}]", envs=[env], rigids=rig)
    out.x, out.v, out.F, out.C = (np.ascontiguousarray(a[:, sl]) for a in (scene.x, scene.v, scene.F, scene.C))
    return out


def _stiffness(E: float, V0: float) -> float:
    return KAPPA * E * V0 ** (1.0 / 3.0)


def _identity_F(P: int) -> np.ndarray:
    F = np.zeros((9, P), np.float32)
    F[0] = F[4] = F[8] = 1.0
    return F


def _state(pos: np.ndarray, vel) -> tuple:
    P = pos.shape[0]
    x = np.ascontiguousarray(pos.T.astype(np.float32))
    v = np.zeros((3, P), np.float32)
    v[:] = np.asarray(vel, np.float32).reshape(3, 1)
    return x, v, _identity_F(P), np.zeros((9, P), np.float32)


def plain_cube(contact: bool = False, seed: int = 0, n_side: int = 20) -> Scene:
    """20^3-particle elastic cube over a half-space at z = 0.125 (dx = 1/32)."""
    rng = np.random.default_rng(seed)
    n = 32
    dx = 1.0 / n
    z_plane = 0.125
    sp = dx / 2
    lo = np.array([11 * dx, 11 * dx, z_plane + 0.05])
    vel = (0.0, 0.0, 0.0)
    if contact:
        lo[2] = z_plane - 0.1 * dx
        vel = (0.5, 0.0, -1.0)
    i = np.arange(n_side)
    g = np.stack(np.meshgrid(i, i, i, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    pos = lo + (g + 0.5) * sp + rng.uniform(-0.1 * dx, 0.1 * dx, g.shape)
    V0 = sp ** 3
    env = EnvSpec(dims=(n, n, n), dx=dx, E=1e5, nu=0.3, rho=1000.0, V0=V0,
                  k=_stiffness(1e5, V0), p_begin=0, p_end=pos.shape[0])
    plane = RigidSpec(env=0, shape=HALF_SPACE, mu=0.5, normal=(0.0, 0.0, 1.0), offset=z_plane)
    x, v, F, C = _state(pos, vel)
    return Scene("plain_cube_contact" if contact else "plain_cube", 2e-4, 10, [env], [plane],
                 x, v, F, C)


def granular_pour(n_particles: int = 1_000_000, seed: int = 1, n: int = 128, sink: float = 0.0) -> Scene:
    """Sand block falling at 1 m/s onto four static boxes (dx = 1/128). With
    sink > 0 the block starts sink metres lower; past dx/2 its bottom layer
    starts inside the box tops (z = 0.15), so the first substep has contacts."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    z_s = 0.15 + 0.5 * dx - sink
    lo = np.array([0.3, 0.3, z_s])
    pos = lo + rng.uniform(0.0, 0.4, (n_particles, 3))
    V0 = 0.4 ** 3 / n_particles
    env = EnvSpec(dims=(n, n, n), dx=dx, material=DRUCKER_PRAGER, E=3.5e5, nu=0.3, rho=1000.0,
                  V0=V0, friction_angle=30.0, k=_stiffness(3.5e5, V0), p_begin=0,
                  p_end=n_particles)
    boxes = [RigidSpec(env=0, shape=BOX, mu=0.4, half=(0.09, 0.09, 0.05), t=(cx, cy, 0.10))
             for cy in (0.4, 0.6) for cx in (0.4, 0.6)]
    x, v, F, C = _state(pos, (0.0, 0.0, -1.0))
    return Scene("granular_pour", 1e-4, 10, [env], boxes, x, v, F, C)


def gripper(n_particles: int = 250_000, seed: int = 2, n: int = 96, overlap: float = 0.0) -> Scene:
    """Elastic ellipsoid between two kinematic jaws closing at 0.05 m/s. With
    overlap > 0 each jaw starts that many metres inside the ellipsoid's tip
    (a dense-contact state: about 2e4 particles inside the jaws at 0.065 m)."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    semi = np.array([0.25, 0.185, 0.185])
    pts = np.empty((0, 3))
    while pts.shape[0] < n_particles:
        cand = rng.uniform(-1.0, 1.0, (2 * n_particles, 3))
        cand = cand[(cand ** 2).sum(1) < 1.0]
        pts = np.concatenate([pts, cand])
    pos = 0.5 + pts[:n_particles] * semi
    V0 = 4.0 / 3.0 * math.pi * float(np.prod(semi)) / n_particles
    env = EnvSpec(dims=(n, n, n), dx=dx, E=5e4, nu=0.4, rho=1000.0, V0=V0,
                  k=_stiffness(5e4, V0), p_begin=0, p_end=n_particles)
    jaws = [RigidSpec(env=0, shape=BOX, mu=0.8, motion=KINEMATIC, half=(0.02, 0.25, 0.25),
                      t=(0.5 + s * (0.25 + 0.02 - overlap), 0.5, 0.5), V=(-s * 0.05, 0.0, 0.0))
            for s in (-1.0, 1.0)]
    x, v, F, C = _state(pos, (0.0, 0.0, 0.0))
    return Scene("gripper", 1e-4, 10, [env], jaws, x, v, F, C)


def batched(n_envs: int = 64, seed: int = 4, p_min: int = 5_000, p_max: int = 100_000,
            n: int = 64, h: float = 1e-4, N: int = 10, z_floor: float = 0.2,
            v0: float = -0.5) -> Scene:
    """Independent environments of uneven size: particle counts log-uniform in
    [p_min, p_max]; each env is elastic (fixed-corotated, E=1e5, nu=0.3,
    particles on a lattice of spacing dx/2 with +-0.1 dx jitter) or sand
    (Drucker-Prager 30 deg, E=3.5e5, nu=0.3, uniform random positions) with
    probability 1/2, a cube of side (P_e/8)^(1/3) dx centred in x and y whose
    bottom rests on a static floor slab (top at z_floor), falling at v0, and
    0-2 more static boxes beside the cube; mu uniform in [0.2, 0.9] per box."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    counts = np.exp(rng.uniform(math.log(p_min), math.log(p_max), n_envs)).round().astype(np.int64)
    envs, rigids, xs = [], [], []
    p0 = 0
    for e in range(n_envs):
        cnt = int(counts[e])
        sand = bool(rng.integers(0, 2))
        m = max(2, int(round((cnt / 8.0) ** (1.0 / 3.0) * 2.0)))  # lattice points per side (spacing dx/2)
        side = m * 0.5 * dx
        lo = np.array([0.5 - 0.5 * side, 0.5 - 0.5 * side, z_floor])
        if sand:
            pos = lo + rng.uniform(0.0, side, (cnt, 3))
        else:
            g = (np.arange(m) + 0.5) * 0.5 * dx
            lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
            lat = lat[rng.permutation(lat.shape[0])[:cnt]] if lat.shape[0] >= cnt else lat
            cnt = lat.shape[0]
            pos = lo + lat + rng.uniform(-0.1 * dx, 0.1 * dx, lat.shape)
        xs.append(pos)
        V0 = side ** 3 / cnt
        E_mod = 3.5e5 if sand else 1e5
        envs.append(EnvSpec(dims=(n, n, n), dx=dx, material=DRUCKER_PRAGER if sand else FIXED_COROTATED,
                            E=E_mod, nu=0.3, rho=1000.0, V0=V0, friction_angle=30.0,
                            k=_stiffness(E_mod, V0), p_begin=p0, p_end=p0 + cnt))
        p0 += cnt
        # the floor slab, then boxes beside the cube (alternately at -x and +x)
        rigids.append(RigidSpec(env=e, shape=BOX, mu=float(rng.uniform(0.2, 0.9)),
                                half=(0.4, 0.4, 0.05), t=(0.5, 0.5, z_floor - 0.05)))
        for b in range(int(rng.integers(0, 3))):
            hx, hy, hz = rng.uniform(0.02, 0.06, 3)
            sgn = -1.0 if b == 0 else 1.0
            cx = 0.5 + sgn * (0.5 * side + hx + 0.02)
            rigids.append(RigidSpec(env=e, shape=BOX, mu=float(rng.uniform(0.2, 0.9)),
                                    half=(hx, hy, hz), t=(cx, 0.5 + rng.uniform(-0.1, 0.1), z_floor + hz)))
    x, v, F, C = _state(np.concatenate(xs), (0.0, 0.0, v0))
    return Scene("batched", h, N, envs, rigids, x, v, F, C)


def differentiable(n_particles: int = 200_000, seed: int = 5, n: int = 96) -> Scene:
    """Elastic cube (fixed-corotated, E=1e5, nu=0.3, rho=1000) of side 0.3046 m
    (about 8 particles per cell, uniform random) centred at 0.5 on a 96^3
    grid, pushed along +x by a kinematic box (half extents 0.02, 0.2, 0.2)
    touching its -x face and moving at 0.5 m/s, mu = 0.5; gravity on."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    side = 0.3046
    pos = 0.5 - 0.5 * side + rng.uniform(0.0, side, (n_particles, 3))
    V0 = side ** 3 / n_particles
    env = EnvSpec(dims=(n, n, n), dx=dx, E=1e5, nu=0.3, rho=1000.0, V0=V0, k=_stiffness(1e5, V0),
                  p_begin=0, p_end=n_particles)
    box = RigidSpec(env=0, shape=BOX, mu=0.5, motion=KINEMATIC, half=(0.02, 0.2, 0.2),
                    t=(0.5 - 0.5 * side - 0.02, 0.5, 0.5), V=(0.5, 0.0, 0.0))
    x, v, F, C = _state(pos, (0.0, 0.0, 0.0))
    return Scene("differentiable", 1e-4, 10, [env], [box], x, v, F, C)


def tiny_block(n_side: int = 3, seed: int = 5, vel=(0.3, 0.1, -0.5), mu: float = 0.5,
               material: int = FIXED_COROTATED, n: int = 16, depth: float = 0.1,
               rotated_plane: bool = False) -> Scene:
    """A few particles straddling a half-space: a contact problem small enough
    for dense brute force."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    sp = dx / 2
    z_plane = 0.3
    i = np.arange(n_side)
    g = np.stack(np.meshgrid(i, i, i, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    lo = np.array([0.5 - n_side * sp / 2, 0.5 - n_side * sp / 2, z_plane - depth * dx])
    pos = lo + (g + 0.5) * sp + rng.uniform(-0.1 * dx, 0.1 * dx, g.shape)
    V0 = sp ** 3
    env = EnvSpec(dims=(n, n, n), dx=dx, material=material, E=1e5, nu=0.3, rho=1000.0, V0=V0,
                  k=_stiffness(1e5, V0), p_begin=0, p_end=pos.shape[0])
    if rotated_plane:
        nrm = np.array([0.2, -0.1, 1.0])
        nrm /= np.linalg.norm(nrm)
        plane = RigidSpec(env=0, shape=HALF_SPACE, mu=mu, normal=tuple(nrm),
                          offset=float(nrm @ np.array([0.5, 0.5, z_plane])))
    else:
        plane = RigidSpec(env=0, shape=HALF_SPACE, mu=mu, offset=z_plane)
    x, v, F, C = _state(pos, vel)
    return Scene("tiny_block", 1e-4, 1, [env], [plane], x, v, F, C)


def tiny_random(P: int = 400, seed: int = 6, n: int = 24, material: int = FIXED_COROTATED,
                with_box: bool = True) -> Scene:
    """Random particles with random velocities and a random deformation, over a
    half-space and (optionally) a rotated, moving box."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    pos = rng.uniform([0.35, 0.35, 0.28], [0.65, 0.65, 0.45], (P, 3))
    V0 = (dx / 2) ** 3
    env = EnvSpec(dims=(n, n, n), dx=dx, material=material, E=1e5, nu=0.3, rho=1000.0, V0=V0,
                  k=_stiffness(1e5, V0), p_begin=0, p_end=P)
    rig = [RigidSpec(env=0, shape=HALF_SPACE, mu=0.6, offset=0.3)]
    if with_box:
        ang = 0.3
        c, s = math.cos(ang), math.sin(ang)
        R = (c, -s, 0.0, s, c, 0.0, 0.0, 0.0, 1.0)
        rig.append(RigidSpec(env=0, shape=BOX, mu=0.4, motion=KINEMATIC, half=(0.06, 0.05, 0.04),
                             R=R, t=(0.5, 0.5, 0.42), V=(0.1, -0.05, 0.0), w=(0.0, 0.0, 0.5)))
    x, v, F, C = _state(pos, (0.0, 0.0, 0.0))
    x = x.astype(np.float32)
    v = rng.normal(0.0, 0.3, (3, P)).astype(np.float32)
    A = rng.normal(0.0, 0.03, (P, 3, 3))
    F = (np.eye(3) + A).reshape(P, 9).T.astype(np.float32).copy()
    C = rng.normal(0.0, 1.0, (9, P)).astype(np.float32)
    return Scene("tiny_random", 1e-4, 2, [env], rig, x, v, F, C)


def slab_on_plane(nx: int = 6, nz: int = 3, vel=(0.0, 0.0, 0.0), mu: float = 0.5,
                  seed: int = 31, n: int = 32, penetration: float = 2e-5,
                  h: float = 1e-4) -> Scene:
    """An elastic slab of nx*nx*nz particles (spacing dx/2, jitter in x and y
    only) whose bottom layer sits `penetration` metres inside a half-space."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    sp = dx / 2
    z_plane = 0.3
    i = np.arange(nx)
    k = np.arange(nz)
    g = np.stack(np.meshgrid(i, i, k, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    pos = np.empty_like(g)
    pos[:, :2] = 0.5 - nx * sp / 2 + (g[:, :2] + 0.5) * sp + rng.uniform(-0.1 * dx, 0.1 * dx,
                                                                       (g.shape[0], 2))
    pos[:, 2] = z_plane - penetration + g[:, 2] * sp
    V0 = sp ** 3
    env = EnvSpec(dims=(n, n, n), dx=dx, E=1e5, nu=0.3, rho=1000.0, V0=V0,
                  k=_stiffness(1e5, V0), p_begin=0, p_end=pos.shape[0])
    plane = RigidSpec(env=0, shape=HALF_SPACE, mu=mu, offset=z_plane)
    x, v, F, C = _state(pos, vel)
    return Scene("slab_on_plane", h, 1, [env], [plane], x, v, F, C, max_iter=50000)

"""Seeded synthetic scenes shaped like the paper's workloads.

This module only generates inputs (particle lattices, materials, tool
poses); it holds none of the method's arithmetic and imports neither the GPU
library nor the oracle, so both can be fed from it.

The paper's tissue scenes are Unity assets without stated sizes (Sec. V);
its one measured workload is a falling cube on a fixed 56^3 grid
(Sec. III-D). The scenes below are synthetic stand-ins:

* ``c1``   8,000 particles, 20^3 lattice at dx/2 spacing in a cube at the
  centre of a 32^3 grid, free fall, uniform E = 5e3 Pa, nu = 0.3.
* ``c1s``  c1 spinning about z at 2 rad/s with F0 = diag(1.05, 1, 1).
* ``c2``   1,048,576 particles filling a 0.8 x 0.2 x 0.8 slab on a 128^3
  grid, E ~ U(2e3, 8e3), nu = 0.4, a capsule (r = 3 dx) pressing down at
  0.05 m/s, dt = 5e-5, 1,000 substeps.
* ``c2s``  c2 on a 32^3 grid (16,384 particles), 100 substeps.
* ``c3``   4,194,304 particles in the slab on a 256^3 grid, a thin oriented
  box blade (thickness 0.5 dx, length 0.3) sweeping along x at 1 m/s through
  the slab plus a capsule grasper, friction 0.3, dt = 5e-5, 500 substeps.
* ``c3s``  c3 on a 32^3 grid (8,192 particles), 100 substeps.
* ``c5``   65,536 particles on a 64^3 grid, per-particle E = exp(theta),
  capsule tool, dt = 1e-4, 200 substeps (differentiable-rollout shape).
* ``cube`` the paper's performance scene: falling cube, 56^3 grid,
  dt = 2e-3, 10 substeps per frame, ``n_particles`` chosen by the caller.
* ``cube_pb`` the same cube for PB-MPM: one dt = 0.02 step per frame with
  10 (or 20) constraint iterations.
* ``pb_drop`` PB-MPM contact case: a 16^3 cube thrown at the sticky floor
  under a pressing capsule, 32^3 grid, dt = 5e-3, 20 steps of 10 passes.

A scene's ``solver`` is None (MLS-MPM) or (kind, iterations, beta) with kind
0 MLS-MPM, 1 standard MPM, 2 PB-MPM.

Every scene: domain [0, 1)^3, dx = 1/n, rho = 1e3, gravity (0, -9.8, 0),
sticky walls 3 nodes thick, v0 = 0, C0 = 0, F0 = I unless stated,
lattice points cell-centred and jittered per component by U[0, 0.1 dx)
drawn from numpy's PCG64 seeded with the scene seed; positions are drawn
before E.
"""
from dataclasses import dataclass, field
import math

import numpy as np

TOOL_NONE, TOOL_CAPSULE, TOOL_BOX, TOOL_PLANE, TOOL_SLICER, TOOL_SEGMENT, TOOL_ARC = 0, 1, 2, 3, 4, 5, 6
RHO = 1e3
GRAVITY = (0.0, -9.8, 0.0)
WALL_BAND = 3
SQRT_HALF = math.sqrt(0.5)


@dataclass
class Tool:
    type: int
    center: tuple
    quat: tuple = (1.0, 0.0, 0.0, 0.0)
    size: tuple = (0.0, 0.0, 0.0)
    lin_vel: tuple = (0.0, 0.0, 0.0)
    ang_vel: tuple = (0.0, 0.0, 0.0)
    mu: float = 0.3
    drag: float = 1.0
    margin: float = 0.0
    push_out: bool = False

    def kwargs(self):
        return dict(center=self.center, quat=self.quat, size=self.size, lin_vel=self.lin_vel,
                    ang_vel=self.ang_vel, mu=self.mu, drag=self.drag, margin=self.margin,
                    push_out=self.push_out)


@dataclass
class Scene:
    name: str
    n_grid: int
    dt: float
    n_substeps: int
    nu: float
    E_default: float
    mass: float
    vol0: float
    x: np.ndarray                      # (N, 3) float32
    v: np.ndarray = None               # (N, 3) float32 or None (zero)
    C: np.ndarray = None               # (N, 3, 3) float32 or None (zero)
    F: np.ndarray = None               # (N, 3, 3) float32 or None (identity)
    E: np.ndarray = None               # (N,) float32 or None (E_default)
    tools: list = field(default_factory=list)
    gravity: tuple = GRAVITY
    wall_band: int = WALL_BAND
    theta: np.ndarray = None           # (N,) float32 log E, differentiable scenes
    vel_tables: dict = field(default_factory=dict)  # tool id -> (T, 3) float64 per-substep velocities
    solver: tuple = None               # (kind, iterations, beta); None: MLS-MPM

    @property
    def N(self):
        return int(self.x.shape[0])

    @property
    def dx(self):
        return 1.0 / self.n_grid

    def particle_arrays(self):
        return dict(x=self.x, v=self.v, C=self.C, F=self.F, E=self.E)


def lattice(lo, counts, spacing):
    """Cell-centred lattice points lo + (i + 1/2) * spacing, x fastest."""
    axes = [lo[a] + (np.arange(counts[a], dtype=np.float64) + 0.5) * spacing[a] for a in range(3)]
    X, Y, Z = np.meshgrid(axes[0], axes[1], axes[2], indexing="ij")
    pts = np.stack([X.ravel(order="F"), Y.ravel(order="F"), Z.ravel(order="F")], axis=1)
    return pts


def jitter(rng, n, dx):
    return rng.uniform(0.0, 0.1 * dx, size=(n, 3))


def _cube(n_grid, per_axis, spacing, seed):
    dx = 1.0 / n_grid
    side = per_axis * spacing
    lo = 0.5 - 0.5 * side
    rng = np.random.default_rng(seed)
    pts = lattice((lo, lo, lo), (per_axis,) * 3, (spacing,) * 3)
    pts = pts + jitter(rng, pts.shape[0], dx)
    return pts.astype(np.float32), rng


def scene_c1(seed=1):
    n = 32
    dx = 1.0 / n
    x, _ = _cube(n, 20, dx / 2, seed)
    vol0 = (dx / 2) ** 3
    return Scene("c1", n, 1e-4, 100, 0.3, 5e3, RHO * vol0, vol0, x)


def scene_c1s(seed=1, omega=(0.0, 0.0, 2.0), stretch=1.05, gravity=GRAVITY):
    s = scene_c1(seed)
    w = np.asarray(omega, dtype=np.float64)
    r = s.x.astype(np.float64) - 0.5
    v = np.cross(np.broadcast_to(w, r.shape), r)
    W = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    s.name = "c1s"
    s.v = v.astype(np.float32)
    s.C = np.broadcast_to(W, (s.N, 3, 3)).astype(np.float32).copy()
    F = np.zeros((s.N, 3, 3), dtype=np.float32)
    F[:, 0, 0], F[:, 1, 1], F[:, 2, 2] = stretch, 1.0, 1.0
    s.F = F
    s.gravity = tuple(gravity)
    return s


def _slab(n_grid, counts, seed, E_range=(2e3, 8e3)):
    """Slab x, z in [0.1, 0.9], y in [3 dx, 3 dx + 0.2], resting on the floor band."""
    dx = 1.0 / n_grid
    lo = (0.1, 3 * dx, 0.1)
    ext = (0.8, 0.2, 0.8)
    spacing = tuple(ext[a] / counts[a] for a in range(3))
    rng = np.random.default_rng(seed)
    pts = lattice(lo, counts, spacing)
    pts = pts + jitter(rng, pts.shape[0], dx)
    E = rng.uniform(E_range[0], E_range[1], size=pts.shape[0]).astype(np.float32)
    N = pts.shape[0]
    vol0 = 0.128 / N
    top = 3 * dx + 0.2
    return pts.astype(np.float32), E, vol0, top


# Start offset of the press capsule off the node lattice, in units of dx. On
# the lattice, nodes can lie exactly on the capsule surface (e.g. offsets
# (0.4, 2.8, 1) dx from a cap centre are exactly r = 3 dx away), and whether
# such a node is in contact is then decided by rounding.
PRESS_OFFSET_DX = (0.0173, 0.0, 0.0291)


def _press_capsule(n_grid, top, center_xz=(0.5, 0.5), axis="z", half_length=0.15, speed=0.05):
    dx = 1.0 / n_grid
    r = 3 * dx
    quat = (SQRT_HALF, 0.0, -SQRT_HALF, 0.0) if axis == "z" else (1.0, 0.0, 0.0, 0.0)
    c = (center_xz[0] + PRESS_OFFSET_DX[0] * dx, top + r, center_xz[1] + PRESS_OFFSET_DX[2] * dx)
    return Tool(TOOL_CAPSULE, c, quat, (half_length, r, 0.0), (0.0, -speed, 0.0), mu=0.3)


def scene_c2(seed=2, n_grid=128, counts=(128, 64, 128), n_substeps=1000):
    x, E, vol0, top = _slab(n_grid, counts, seed)
    tool = _press_capsule(n_grid, top)
    return Scene("c2", n_grid, 5e-5, n_substeps, 0.4, 5e3, RHO * vol0, vol0, x, E=E, tools=[tool])


def scene_c2s(seed=2):
    s = scene_c2(seed, n_grid=32, counts=(32, 16, 32), n_substeps=100)
    s.name = "c2s"
    return s


def _blade_and_grasper(n_grid, top):
    dx = 1.0 / n_grid
    ox, oz = PRESS_OFFSET_DX[0] * dx, PRESS_OFFSET_DX[2] * dx  # off the node lattice (faces, caps)
    blade = Tool(TOOL_BOX, (0.1 + ox, top, 0.5 + oz), (1.0, 0.0, 0.0, 0.0), (0.15, 0.15, 0.25 * dx),
                 (1.0, 0.0, 0.0), mu=0.3)
    r = 3 * dx
    grasper = Tool(TOOL_CAPSULE, (0.7 + ox, top + r, 0.3 + oz), (1.0, 0.0, 0.0, 0.0), (0.1, r, 0.0),
                   (0.0, -0.05, 0.0), mu=0.3)
    return [blade, grasper]


def scene_c3(seed=3, n_grid=256, counts=(256, 64, 256), n_substeps=500):
    x, E, vol0, top = _slab(n_grid, counts, seed)
    return Scene("c3", n_grid, 5e-5, n_substeps, 0.4, 5e3, RHO * vol0, vol0, x, E=E,
                 tools=_blade_and_grasper(n_grid, top))


def scene_c3s(seed=3):
    s = scene_c3(seed, n_grid=32, counts=(32, 8, 32), n_substeps=100)
    s.name = "c3s"
    return s


def scene_c3m(seed=3):
    """c3 on a 64^3 grid (65,536 particles): several blocks per axis."""
    s = scene_c3(seed, n_grid=64, counts=(64, 16, 64), n_substeps=100)
    s.name = "c3m"
    return s


def press_table(n_substeps):
    """Per-substep capsule velocities of the differentiable scenes: a downward
    press of 0.5 m/s modulated by one period of a sideways and vertical wave."""
    ph = 2.0 * math.pi * np.arange(n_substeps) / max(1, n_substeps)
    return np.stack([0.1 * np.cos(ph), -0.5 + 0.2 * np.sin(ph), np.zeros(n_substeps)], axis=1)


def scene_c5(seed=5, n_substeps=200, n_grid=64, counts=(64, 16, 64)):
    """Differentiable press: a slab with E_p = exp(theta_p), theta_p =
    ln(5e3) + U(-0.2, 0.2), pressed by a capsule that follows a per-substep
    velocity table."""
    x, _, vol0, top = _slab(n_grid, counts, seed)
    rng = np.random.default_rng(seed + 1000)
    theta = (math.log(5e3) + rng.uniform(-0.2, 0.2, size=x.shape[0])).astype(np.float32)
    E = np.exp(theta.astype(np.float64)).astype(np.float32)
    tool = _press_capsule(n_grid, top)
    tool.lin_vel = (0.0, 0.0, 0.0)
    s = Scene("c5", n_grid, 1e-4, n_substeps, 0.3, 5e3, RHO * vol0, vol0, x, E=E, tools=[tool])
    s.theta = theta
    s.vel_tables = {0: press_table(n_substeps)}
    return s


def scene_c5s(seed=5):
    """c5 at 32^3 with 8,192 particles and 40 substeps."""
    s = scene_c5(seed, n_substeps=40, n_grid=32, counts=(32, 8, 32))
    s.name = "c5s"
    return s


def scene_cube(n_particles=1 << 16, seed=7, n_grid=56):
    """The paper's performance scene: a cube falling under gravity on a fixed
    56^3 grid, 10 substeps of dt = 2e-3 per 0.02 s frame."""
    per_axis = max(2, int(round(n_particles ** (1.0 / 3.0))))
    dx = 1.0 / n_grid
    side = 0.4
    spacing = side / per_axis
    rng = np.random.default_rng(seed)
    lo = 0.5 - side / 2
    pts = lattice((lo, lo, lo), (per_axis,) * 3, (spacing,) * 3)
    pts = (pts + jitter(rng, pts.shape[0], dx)).astype(np.float32)
    vol0 = side ** 3 / pts.shape[0]
    return Scene("cube", n_grid, 2e-3, 10, 0.3, 5e3, RHO * vol0, vol0, pts)


SOLVER_MLS, SOLVER_PIC, SOLVER_PB = 0, 1, 2


def scene_on_lattice(seed=9, n_grid=64, counts=(64, 16, 64), n_substeps=4):
    """Tools placed ON the node lattice, so that nodes lie exactly on their
    surfaces (in exact arithmetic) and the contact decision of those nodes is
    a rounding tie: a capsule along z (turned by a quaternion, radius 5 dx,
    half length 6 dx, centre on a node), whose cylinder and caps pass through
    nodes at integer offsets (0, 5), (3, 4), (4, 3) dx, pressing down at
    0.05 m/s; and a box turned a quarter turn about y (half extents 4, 3, 2
    dx, centre on a node), whose faces lie on node planes, moving along x at
    0.1 m/s. Both start slightly inside the c5-shaped slab (64^3, 65,536
    particles). The tools move off the lattice after the first substep."""
    x, E, vol0, top = _slab(n_grid, counts, seed)
    dx = 1.0 / n_grid
    top_node = math.floor(top / dx)
    cap = Tool(TOOL_CAPSULE, ((n_grid // 2 - 8) * dx, (top_node + 4) * dx, (n_grid // 2) * dx),
               (SQRT_HALF, 0.0, -SQRT_HALF, 0.0), (6 * dx, 5 * dx, 0.0), (0.0, -0.05, 0.0), mu=0.3)
    box = Tool(TOOL_BOX, ((n_grid // 2 + 10) * dx, (top_node + 3) * dx, (n_grid // 2 - 6) * dx),
               (SQRT_HALF, 0.0, SQRT_HALF, 0.0), (4 * dx, 3 * dx, 2 * dx), (0.1, 0.0, 0.0), mu=0.3)
    return Scene("on_lattice", n_grid, 1e-4, n_substeps, 0.3, 5e3, RHO * vol0, vol0, x, E=E, tools=[cap, box])


def scene_cube_pb(n_particles=1 << 12, seed=7, n_grid=56, iterations=10, beta=0.5):
    """The performance cube as the paper runs PB-MPM on it: one step of
    dt = 0.02 per frame with `iterations` passes (Sec. III-D)."""
    s = scene_cube(n_particles, seed, n_grid)
    s.name = f"cube_pb{iterations}"
    s.dt = 0.02
    s.n_substeps = 1
    s.solver = (SOLVER_PB, iterations, beta)
    return s


def scene_pb_drop(seed=8, n_grid=32, per_axis=16, n_substeps=20, iterations=10, beta=0.5):
    """A PB-MPM contact case: a 16^3 cube (dx/2 spacing) thrown at the
    floor at 1.5 m/s from 1.5 dx above the wall band while a capsule presses
    its top, dt = 5e-3 per step; E = 5e3, nu = 0.3."""
    dx = 1.0 / n_grid
    spacing = 0.5 * dx
    side = per_axis * spacing
    rng = np.random.default_rng(seed)
    lo = (0.5 - side / 2, (WALL_BAND + 1.5) * dx, 0.5 - side / 2)
    pts = lattice(lo, (per_axis,) * 3, (spacing,) * 3)
    pts = (pts + jitter(rng, pts.shape[0], dx)).astype(np.float32)
    N = pts.shape[0]
    vol0 = spacing ** 3
    s = Scene("pb_drop", n_grid, 5e-3, n_substeps, 0.3, 5e3, RHO * vol0, vol0, pts)
    s.v = np.tile(np.float32([0.2, -1.5, 0.0]), (N, 1))
    top = lo[1] + side
    # capsule along z over the cube's top face, off the node lattice
    s.tools = [Tool(TOOL_CAPSULE, (0.5 + 0.31 * dx, top + 2.2 * dx, 0.5 + 0.17 * dx), (SQRT_HALF, 0.0, SQRT_HALF, 0.0),
                    (0.15, 2.0 * dx, 0.0), (0.0, -2.5, 0.0), mu=0.3)]
    s.solver = (SOLVER_PB, iterations, beta)
    return s


def tiny_block(n_grid=16, per_axis=6, seed=11, spacing_dx=0.5, center=(0.5, 0.5, 0.5),
               gravity=GRAVITY, with_state=True, E_range=None):
    """A small random block of particles for unit tests (<= a few hundred)."""
    dx = 1.0 / n_grid
    spacing = spacing_dx * dx
    side = per_axis * spacing
    rng = np.random.default_rng(seed)
    lo = tuple(center[a] - side / 2 for a in range(3))
    pts = lattice(lo, (per_axis,) * 3, (spacing,) * 3)
    pts = (pts + jitter(rng, pts.shape[0], dx)).astype(np.float32)
    N = pts.shape[0]
    vol0 = spacing ** 3
    s = Scene("tiny", n_grid, 1e-4, 10, 0.3, 5e3, RHO * vol0, vol0, pts, gravity=tuple(gravity))
    if with_state:
        s.v = rng.normal(0.0, 0.05, size=(N, 3)).astype(np.float32)
        s.C = rng.normal(0.0, 0.5, size=(N, 3, 3)).astype(np.float32)
        s.F = (np.eye(3) + rng.normal(0.0, 0.03, size=(N, 3, 3))).astype(np.float32)
    if E_range is not None:
        s.E = rng.uniform(E_range[0], E_range[1], size=N).astype(np.float32)
    return s


def _unit_quat_to(axis):
    """Unit quaternion (w, x, y, z) rotating body +x onto `axis`."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    ex = np.array([1.0, 0.0, 0.0])
    c = float(np.dot(ex, a))
    if c < -1.0 + 1e-12:
        return (0.0, 0.0, 1.0, 0.0)
    axis_r = np.cross(ex, a)
    q = np.array([1.0 + c, axis_r[0], axis_r[1], axis_r[2]])
    q /= np.linalg.norm(q)
    return tuple(float(v) for v in q)


@dataclass
class Batch:
    """Scenes that share the grid size, dt, material and walls (one batched
    handle); each has its own particles and tools."""
    name: str
    scenes: list
    n_grid: int
    dt: float
    n_substeps: int
    nu: float
    E_default: float
    mass: float
    vol0: float
    gravity: tuple = GRAVITY
    wall_band: int = WALL_BAND

    @property
    def counts(self):
        return np.array([sc.N for sc in self.scenes], dtype=np.int64)

    @property
    def N(self):
        return int(self.counts.sum())

    def concat(self, field):
        arrs = [getattr(sc, field) for sc in self.scenes]
        if all(a is None for a in arrs):
            return None
        if any(a is None for a in arrs):
            raise ValueError(f"{field} given for some scenes only")
        return np.concatenate(arrs, axis=0)


def batch_c4(n_scenes=256, seed=4, n_grid=64, n_substeps=200, k_range=(16, 40)):
    """Many independent falling-cube scenes of uneven size: scene s holds a
    k_s^3 cube lattice at spacing dx/2, k_s = round(exp(u/3)) with u uniform
    in [3 ln k_lo, 3 ln k_hi] (so counts are log-uniform between k_lo^3 and
    k_hi^3), centred in its 64^3 domain with U[0, 0.1 dx) jitter; E = 5e3,
    nu = 0.3, dt = 1e-4. Each scene has one capsule (r = 3 dx, half length
    0.1) whose centre is U(0.3, 1) r above the cube's top face (so it starts
    in contact), with a uniformly random axis and a velocity of uniform
    direction and speed U(0, 0.1) m/s."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n_grid
    spacing = 0.5 * dx
    vol0 = spacing ** 3
    lo, hi = 3.0 * math.log(k_range[0]), 3.0 * math.log(k_range[1])
    scenes = []
    for sidx in range(n_scenes):
        k = int(round(math.exp(rng.uniform(lo, hi) / 3.0)))
        side = k * spacing
        corner = tuple(0.5 - side / 2 for _ in range(3))
        pts = lattice(corner, (k, k, k), (spacing,) * 3)
        pts = (pts + jitter(rng, pts.shape[0], dx)).astype(np.float32)
        axis = rng.normal(size=3)
        direction = rng.normal(size=3)
        speed = rng.uniform(0.0, 0.1)
        vel = tuple(float(v) for v in speed * direction / np.linalg.norm(direction))
        r = 3 * dx
        center = (0.5 + rng.uniform(-0.05, 0.05), 0.5 + side / 2 + rng.uniform(0.3, 1.0) * r,
                  0.5 + rng.uniform(-0.05, 0.05))
        tool = Tool(TOOL_CAPSULE, center, _unit_quat_to(axis), (0.1, r, 0.0), vel, mu=0.3)
        scenes.append(Scene(f"c4[{sidx}]", n_grid, 1e-4, n_substeps, 0.3, 5e3, RHO * vol0, vol0, pts,
                            tools=[tool]))
    return Batch("c4", scenes, n_grid, 1e-4, n_substeps, 0.3, 5e3, RHO * vol0, vol0)


def batch_c4s(seed=4):
    """c4 with 6 scenes on 32^3 grids (4^3 .. 12^3 particles), 40 substeps."""
    b = batch_c4(n_scenes=6, seed=seed, n_grid=32, n_substeps=40, k_range=(4, 12))
    b.name = "c4s"
    return b


SCENES = {
    "c1": scene_c1, "c1s": scene_c1s, "c2": scene_c2, "c2s": scene_c2s, "c3": scene_c3,
    "c3s": scene_c3s, "c3m": scene_c3m, "c5": scene_c5, "c5s": scene_c5s, "cube": scene_cube,
    "cube_pb": scene_cube_pb, "pb_drop": scene_pb_drop, "on_lattice": scene_on_lattice,
}


def make(name, **kw):
    return SCENES[name](**kw)

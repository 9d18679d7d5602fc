"""Shared helpers of the GPU parity tests: run a seeded scene on the oracle
and on the HIP library, and compare element by element.

Tolerances (the parity bound of the substep is on positions; the others
follow from FP32 arithmetic against the FP64 oracle):
* positions: max |x_gpu - x_or| / max |x_or| <= 1e-4, and the displacement
  from x0 agrees to 1e-2 of the largest displacement plus the FP32 storage
  rounding of x (half an ulp of max |x| per substep, n substeps);
* velocity:  max |v_gpu - v_or| <= 2e-3 max |v_or| + 1e-5 m/s;
* F:         max |F_gpu - F_or| <= 1e-4;
* C:         max |C_gpu - C_or| <= 2e-2 max |C_or| + 2e-3 1/s.
"""
import numpy as np

import oracle as O
from paper_2502_18437_amd import scenes

POS_REL = 1e-4
DISP_REL = 1e-2
V_REL, V_ABS = 2e-3, 1e-5
F_ABS = 1e-4
C_REL, C_ABS = 2e-2, 2e-3


def run_oracle(scene, n_substeps, idx=None):
    """FP64 oracle on the scene (optionally on the particle subset idx)."""
    sel = (lambda a: None if a is None else a[idx]) if idx is not None else (lambda a: a)
    o = O.Oracle(scene.n_grid, scene.dt, gravity=scene.gravity, wall_band=scene.wall_band, nu=scene.nu,
                 E_default=scene.E_default)
    o.set_particles(sel(scene.x), sel(scene.v), sel(scene.C), sel(scene.F), sel(scene.E), scene.mass,
                    scene.vol0)
    for k, t in enumerate(scene.tools):
        o.set_tool(k, t.type, **t.kwargs())
    for k, tab in scene.vel_tables.items():
        o.set_velocity_table(k, tab)
    if scene.solver is not None:
        o.set_solver(*scene.solver)
    st = o.step(n_substeps)
    r = o.read()
    r["status"] = st
    r["impulses"] = o.impulses()
    return r


def run_gpu(scene, n_substeps, chunks=None, **kw):
    from paper_2502_18437_amd import mpm
    sim = mpm.simulation_from_scene(scene, **kw)
    if chunks is None:
        sim.step(n_substeps)
    else:
        done = 0
        for c in chunks:
            sim.step(c)
            done += c
        assert done == n_substeps
    r, st = sim.read_state(allow_errors=True)
    r = {k: v.astype(np.float64) for k, v in r.items()}
    r["status"] = st
    r["info"] = sim.info()
    sim.close()
    return r


def dyadic_poses(scene):
    """The scene with a dyadic dt, tool centres and tool velocities, so that
    every FP64 tool pose centre + k dt v is an exact sum, whichever substep
    the count starts from (the resume tests compare bits)."""
    scene.dt = 2.0 ** -14
    for t in scene.tools:
        t.center = tuple(round(c * 2 ** 20) / 2 ** 20 for c in t.center)
        t.lin_vel = (0.0625, -0.25, 0.125)
    return scene


def advance_tools(scene, n_substeps):
    """Move each tool's centre to its pose n_substeps later (linear motion)."""
    for t in scene.tools:
        t.center = tuple(c + n_substeps * scene.dt * v for c, v in zip(t.center, t.lin_vel))


def errors(gpu, orc, x0):
    x0 = np.asarray(x0, np.float32).astype(np.float64)
    ex = np.max(np.abs(gpu["x"] - orc["x"])) / np.max(np.abs(orc["x"]))
    disp = orc["x"] - x0
    dmax = np.max(np.abs(disp))
    da = np.max(np.abs((gpu["x"] - x0) - disp))
    ed = da / max(dmax, 1e-30)
    ev = np.max(np.abs(gpu["v"] - orc["v"]))
    eF = np.max(np.abs(gpu["F"] - orc["F"]))
    eC = np.max(np.abs(gpu["C"] - orc["C"]))
    return dict(x_rel=ex, disp_rel=ed, disp_abs=da, disp_max=dmax, x_max=np.max(np.abs(orc["x"])), v_abs=ev, v_max=np.max(np.abs(orc["v"])), F_abs=eF, C_abs=eC,
                C_max=np.max(np.abs(orc["C"])))


def assert_parity(gpu, orc, x0, n_substeps, label=""):
    e = errors(gpu, orc, x0)
    print(f"[parity {label}] " + " ".join(f"{k}={v:.3e}" for k, v in e.items()), flush=True)
    assert e["x_rel"] <= POS_REL, e
    rounding = n_substeps * 2.0 ** -24 * e["x_max"]
    assert e["disp_abs"] <= DISP_REL * e["disp_max"] + rounding, e
    assert e["v_abs"] <= V_REL * e["v_max"] + V_ABS, e
    assert e["F_abs"] <= F_ABS, e
    assert e["C_abs"] <= C_REL * e["C_max"] + C_ABS, e
    return e


def subbox(x0, lo, hi):
    """Indices of particles whose initial position lies in [lo, hi)."""
    x0 = np.asarray(x0)
    m = np.all((x0 >= np.asarray(lo)) & (x0 < np.asarray(hi)), axis=1)
    return np.nonzero(m)[0]


def blob_scene(n_grid, origin_cells, seed=5):
    """A 12^3 lattice at half-cell spacing with a dyadic jitter and dyadic
    random velocities, its corner at origin_cells * dx. Every position is a
    multiple of 2^-16 below 1, so it is exact in FP32."""
    dx = 1.0 / n_grid
    rng = np.random.default_rng(seed)
    g = np.arange(12, dtype=np.float64)
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) * 0.5 * dx
    jit = rng.integers(0, 32, size=lat.shape) * 2.0 ** -16
    x = np.asarray(origin_cells, np.float64) * dx + lat + jit
    v = rng.integers(-64, 65, size=lat.shape) * 2.0 ** -10
    vol0 = (0.5 * dx) ** 3
    return scenes.Scene(name=f"blob{n_grid}", n_grid=n_grid, dt=2.0 ** -14, n_substeps=40, nu=0.3,
                        E_default=2e4, mass=1e3 * vol0, vol0=vol0, x=x.astype(np.float32),
                        v=v.astype(np.float32))


def shifted_blobs(n_grid):
    """A blob near the far corner (clear of the 3-node walls) and the same
    blob moved down by whole 8-node blocks, a different number per axis,
    both inside [0.5, 1) per axis; returns them and the shift in cells."""
    hi = n_grid - 19
    k = (hi - n_grid // 2) // 8
    shift = np.array([8 * k, 8 * (k - 1), 8 * (k - 2)])
    a = blob_scene(n_grid, (hi, hi, hi))
    b = blob_scene(n_grid, (hi - shift[0], hi - shift[1], hi - shift[2]))
    return a, b, shift

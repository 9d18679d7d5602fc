"""Dense blocks: a grid block holding more than one work item's worth of
particles is shared by several workgroups, each scattering into its own LDS
tile. Parity with the FP64 oracle on a dense spinning cube under a pressing
capsule, and bit-identical results in the fixed-point mode whatever the
number of workgroups."""
import numpy as np
import pytest

import oracle as O
from paper_2502_18437_amd import scenes
from tests.parity import assert_parity, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dense_cube(solver=None):
    """2^18 particles in a 0.4 m cube on a 56^3 grid (about 23 per cell, about
    12,000 per block): spinning about y, pre-strained, a capsule on its top."""
    s = scenes.scene_cube(1 << 18, seed=12)
    rng = np.random.default_rng(12)
    c = np.array([0.5, 0.5, 0.5])
    w = np.array([0.0, 3.0, 0.0])
    s.v = np.cross(w, s.x.astype(np.float64) - c).astype(np.float32)
    s.F = (np.eye(3) + 0.02 * rng.standard_normal((s.N, 3, 3))).astype(np.float32)
    s.dt = 2e-4
    s.n_substeps = 8
    dx = 1.0 / s.n_grid
    top = float(s.x[:, 1].max())
    s.tools = [scenes.Tool(scenes.TOOL_CAPSULE, (0.5 + 0.23 * dx, top + 1.1 * dx, 0.5 + 0.41 * dx),
                           (scenes.SQRT_HALF, 0.0, scenes.SQRT_HALF, 0.0), (0.15, 1.5 * dx, 0.0), (0.0, -1.0, 0.0))]
    if solver is not None:
        s.solver = solver
    return s


def test_block_sizes_exceed_one_item():
    s = dense_cube()
    cell = np.floor(s.x / (1.0 / s.n_grid) - 0.5).astype(np.int64)
    blk = cell // 8
    _, counts = np.unique(blk[:, 0] * 10000 + blk[:, 1] * 100 + blk[:, 2], return_counts=True)
    assert counts.max() > 4 * 2048  # several work items per block


@pytest.mark.parametrize("solver", [None, (O.SOLVER_PIC, 1, 0.5), (O.SOLVER_PB, 3, 0.5)])
def test_dense_cube_matches_oracle(solver):
    from paper_2502_18437_amd import mpm
    s = dense_cube(solver)
    n = s.n_substeps
    print(f"[dense {solver}] N={s.N}", flush=True)
    sim = mpm.simulation_from_scene(s)
    sim.step(n)
    r, st = sim.read_state()
    imp = sim.tool_impulses()
    sim.close()
    assert st == 0
    o = run_oracle(s, n)
    assert o["status"] == 0
    assert_parity({k: v.astype(np.float64) for k, v in r.items()}, o, s.x, n, f"dense {solver}")
    scale = np.abs(o["impulses"][0]).max()
    assert scale > 0
    np.testing.assert_allclose(imp[0], -o["impulses"][0], rtol=0, atol=2e-3 * scale)


def test_dense_cube_is_bitwise_across_workgroup_counts():
    from paper_2502_18437_amd import mpm
    s = dense_cube()
    ref = None
    for wgs in (8, 96, 2048):
        sim = mpm.simulation_from_scene(s, accum_mode=mpm.MPM_ACCUM_FIXED)
        sim.set_launch_config(transfer_wgs=wgs, resort_interval=3)
        sim.step(7)
        r, st = sim.read_state()
        sim.close()
        assert st == 0
        if ref is None:
            ref = r
            continue
        for k in ("x", "v", "C", "F"):
            assert np.array_equal(ref[k], r[k]), (wgs, k)


@pytest.mark.parametrize("fixed,n_particles", [(False, 1 << 16), (True, 3000)])
def test_extreme_density_keeps_the_mass_sums(fixed, n_particles):
    """Particles crowded into one cell: the FP32 case (65,536 particles, 8
    transfer workgroups, so work items of 2048) puts about 600 units of
    weight on a node from one work item, the fixed-point case (3,000
    particles) about 900 units on a node in total; a 32-bit sum of 2^-24
    units would wrap at 256. In free fall, away from the walls, every
    particle must follow v = v0 + n dt g to FP32 rounding, with F = I."""
    from paper_2502_18437_amd import mpm
    n_grid = 32
    dx = 1.0 / n_grid
    rng = np.random.default_rng(21)
    # base cell 10 on every axis
    x = ((10.5 + rng.random((n_particles, 3))) * dx).astype(np.float32)
    x = np.clip(x, np.float32(10.5 * dx), np.float32(11.49 * dx))
    vol0 = dx ** 3 / n_particles
    sim = mpm.Simulation(n_grid, 1e-4, gravity=(0.0, -9.8, 0.0), max_particles=n_particles,
                         accum_mode=mpm.MPM_ACCUM_FIXED if fixed else mpm.MPM_ACCUM_F32)
    v0 = np.float32([0.05, 0.0, 0.0])
    sim.set_particles(x, np.tile(v0, (n_particles, 1)), None, None, None, 1e3 * vol0, vol0)
    sim.set_launch_config(transfer_wgs=8, resort_interval=4)
    n = 6
    print(f"[dense extreme fixed={fixed} N={n_particles}]", flush=True)
    sim.step(n)
    r, st = sim.read_state()
    sim.close()
    assert st == 0
    v_exp = v0.astype(np.float64) + n * 1e-4 * np.array([0.0, -9.8, 0.0])
    np.testing.assert_allclose(r["v"], np.tile(v_exp, (n_particles, 1)), rtol=0, atol=1e-5)
    np.testing.assert_allclose(r["F"], np.tile(np.eye(3), (n_particles, 1, 1)), rtol=0, atol=1e-5)

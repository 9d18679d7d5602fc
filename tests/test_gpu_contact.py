"""GPU parity of the cutting and suturing contact models (slicer, line
segment, arc; CRESSim-MPM Sec. IV-B, IV-C) and of the two-way coupling
impulses (Sec. IV-A) against the FP64 oracle."""
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


def thin_tool_scene(seed=0, n_grid=32):
    dx = 1.0 / n_grid
    s = scenes.tiny_block(n_grid=n_grid, per_axis=16, seed=seed, E_range=(2e3, 8e3), center=(0.5, 0.45, 0.5))
    s.v = (0.3 * s.v).astype(np.float32)
    s.dt = 5e-5
    s.tools = [
        scenes.Tool(O.TOOL_SLICER, (0.5, 0.5, 0.5 + 0.3 * dx), (0.97, 0.0, 0.1, 0.2), (0.12, 0.06, 0.0),
                    (0.0, -0.6, 0.1), (0.0, 0.0, 0.5), mu=0.3, drag=0.9, margin=0.7 * dx),
        scenes.Tool(O.TOOL_SEGMENT, (0.47, 0.42, 0.46), (0.9, 0.2, 0.0, 0.1), (0.1, 0.9 * dx, 0.0),
                    (0.2, 0.3, 0.0), mu=0.2),
        scenes.Tool(O.TOOL_ARC, (0.52, 0.43, 0.53), (0.95, 0.0, 0.3, 0.0), (0.07, 1.2, 0.8 * dx),
                    (-0.1, 0.4, 0.2), (1.0, 0.0, 0.0), mu=0.1),
    ]
    return s


def run_gpu_with_impulses(s, n):
    from paper_2502_18437_amd import mpm
    sim = mpm.simulation_from_scene(s)
    sim.step(n)
    r, st = sim.read_state()
    imp = sim.tool_impulses()
    sim.close()
    r = {k: v.astype(np.float64) for k, v in r.items()}
    r["status"] = st
    return r, imp


@pytest.mark.parametrize("seed", [0, 1])
def test_thin_tools_parity(seed):
    s = thin_tool_scene(seed)
    n = 60
    g, gimp = run_gpu_with_impulses(s, n)
    o = run_oracle(s, n)
    assert g["status"] == 0 and o["status"] == 0
    assert np.all(np.linalg.norm(o["impulses"][:3], axis=1) > 0)  # every tool acts
    assert_parity(g, o, s.x, n, f"thin tools seed={seed}")
    # impulses on the tools are minus the momentum the tools gave the material
    scale = np.max(np.abs(o["impulses"]))
    np.testing.assert_allclose(gimp, -o["impulses"], rtol=0, atol=2e-3 * scale)


@pytest.mark.parametrize("name", ["c2s", "c3s"])
def test_tool_impulses_match_oracle(name):
    s = scenes.make(name)
    n = 40
    g, gimp = run_gpu_with_impulses(s, n)
    o = run_oracle(s, n)
    scale = np.max(np.abs(o["impulses"]))
    assert scale > 0
    np.testing.assert_allclose(gimp, -o["impulses"], rtol=0, atol=2e-3 * scale)
    # momentum budget on the GPU: P1 - P0 = M g dt n - (impulses on tools and walls)
    M = s.mass * s.N
    P0 = np.zeros(3) if s.v is None else s.mass * s.v.astype(np.float64).sum(axis=0)
    P1 = s.mass * g["v"].sum(axis=0)
    expect = P0 + n * M * np.asarray(s.gravity) * s.dt - gimp.sum(axis=0)
    np.testing.assert_allclose(P1, expect, rtol=0, atol=1e-4 * max(np.max(np.abs(P1)), M * 1e-3))


def test_impulses_cover_only_the_last_step():
    s = scenes.scene_c2s()
    from paper_2502_18437_amd import mpm
    sim = mpm.simulation_from_scene(s)
    sim.step(10)
    a = sim.tool_impulses()
    sim.step(0)
    assert np.array_equal(sim.tool_impulses(), a)  # a zero-substep call changes nothing
    sim.step(10)
    b = sim.tool_impulses()
    assert not np.allclose(a, b)
    sim.close()


@pytest.mark.parametrize("solver", [None, (O.SOLVER_PIC, 1, 0.5), (O.SOLVER_PB, 3, 0.5)])
def test_particle_push_out_matches_oracle(solver):
    """A capsule driven into a block, a box sweeping in and a rising tilted
    plane, all pushing particles out after each substep (x - phi n), for
    every solver; the fast tools make push-outs happen."""
    from tests.test_oracle_push_out import push_scene
    from tests.parity import run_gpu
    s = push_scene(0)
    s.n_substeps = 20
    if solver is not None:
        s.solver = solver
    n = s.n_substeps
    print(f"[push-out {solver}] N={s.N}", flush=True)
    g = run_gpu(s, n)
    o = run_oracle(s, n)
    assert g["status"] == 0 and o["status"] == 0
    assert_parity(g, o, s.x, n, f"push-out {solver}")
    for t in s.tools:
        t.push_out = False
    off = run_oracle(s, n)
    assert np.max(np.abs(off["x"] - o["x"])) > 1e-4  # the push-out acted


def test_rollout_refuses_push_out():
    import torch
    from paper_2502_18437_amd import mpm
    s = scenes.make("c5s")
    s.tools[0].push_out = True
    sim = mpm.simulation_from_scene(s)
    with pytest.raises(mpm.MPMError) as e:
        sim.rollout_forward(2, 1, theta=torch.as_tensor(s.theta, device="cuda"))
    assert e.value.code == mpm.MPM_EINVAL
    sim.close()

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


def test_tools_on_the_node_lattice_tie_decisions():
    """The tie case of the contact decision (Sec. IV-A, eq. v_correction: a
    node is corrected when it is inside the tool): a capsule and a box placed
    on the node lattice, so that nodes lie exactly on their surfaces and FP32
    and FP64 may decide those nodes either way (both are correct results).
    The oracle records every decision within 2e-6 m of its threshold and the
    particles whose state depends on one (their cone of influence). Those
    unmarked are held to the strict parity bar; the marked ones must be
    finite and within the change a tie can make: node velocities move by at
    most the largest jump J of a tie (G2P and P2G average them), C by the
    affine moment of that (|x_I - x_p| <= 1.5 sqrt(3) dx, times 4/dx^2), F and
    x by dt times those over the substeps."""
    s = scenes.scene_on_lattice()
    k = s.n_substeps
    eta = 2e-6
    o = O.Oracle(s.n_grid, s.dt, gravity=s.gravity, wall_band=s.wall_band, nu=s.nu, E_default=s.E_default)
    o.set_particles(s.x, s.v, s.C, s.F, s.E, s.mass, s.vol0)
    for q, t in enumerate(s.tools):
        o.set_tool(q, t.type, **t.kwargs())
    o.set_tie_band(eta, 0)
    assert o.step(k) == 0
    orc = o.read()
    taint, n_tie, J = o.ties()
    assert n_tie > 100 and 1000 < taint.sum() < s.N - 1000
    from tests.parity import run_gpu
    g = run_gpu(s, k)
    assert g["status"] == 0
    keep = ~taint
    sub = lambda r: {f: r[f][keep] for f in ("x", "v", "C", "F")}  # noqa: E731
    assert_parity(sub(g), sub(orc), s.x[keep], k, f"on-lattice tools, {keep.sum()} particles outside tie cones")
    dv = 2.0 * J
    dC = 4.0 * 1.5 * np.sqrt(3.0) / s.dx * dv
    bounds = {"v": dv + 1e-5, "C": dC + 2e-3, "x": k * s.dt * dv + 1e-6,
              "F": k * s.dt * dC * np.abs(orc["F"]).max() + 1e-4}
    for f, b in bounds.items():
        a = g[f][taint]
        assert np.isfinite(a).all(), f
        d = np.abs(a - orc[f][taint]).max()
        print(f"[ties] {f}: largest difference over {taint.sum()} marked particles {d:.3e} (bound {b:.3e})")
        assert d <= b, (f, d, b)

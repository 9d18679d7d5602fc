"""GPU parity of the two other solvers of Sec. III against the FP64 oracle:
standard MPM (PIC transfers, Neo-Hookean stress as a grid force) and PB-MPM
(iterated APIC transfers with the co-rotational constraint). Also: graph
replay and launch configurations give the same bits in the fixed-point mode,
batches equal their scenes run alone, and the solver switch validates its
arguments."""
import numpy as np
import pytest

import oracle as O
from paper_2502_18437_amd import scenes
from tests.parity import assert_parity, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

PIC = (O.SOLVER_PIC, 1, 0.5)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def with_solver(name, solver):
    s = scenes.make(name)
    if solver is not None:
        s.solver = solver
    return s


def check_impulses(gpu_imp, orc_imp, label):
    scale = np.max(np.abs(orc_imp))
    print(f"[impulses {label}] max {scale:.3e} err {np.max(np.abs(gpu_imp + orc_imp)):.3e}", flush=True)
    assert scale > 0
    # mpm_read_tool_impulses reports the force on the tool (minus the
    # momentum given to the material)
    np.testing.assert_allclose(gpu_imp, -orc_imp, rtol=0, atol=2e-3 * scale)


def gpu_with_impulses(scene, n, **kw):
    from paper_2502_18437_amd import mpm
    sim = mpm.simulation_from_scene(scene, **kw)
    print(f"[solver {scene.name} {scene.solver} N={scene.N} n={n} {kw}]", flush=True)
    sim.step(n)
    r, st = sim.read_state(allow_errors=True)
    imp = sim.tool_impulses()
    info = sim.info()
    sim.close()
    r = {k: v.astype(np.float64) for k, v in r.items()}
    r["status"] = st
    return r, imp, info


@pytest.mark.parametrize("name", ["c2s", "c3s"])
def test_standard_mpm_matches_oracle(name):
    s = with_solver(name, PIC)
    n = s.n_substeps
    g, imp, _ = gpu_with_impulses(s, n)
    o = run_oracle(s, n)
    assert g["status"] == 0 and o["status"] == 0
    assert_parity(g, o, s.x, n, f"PIC {name}")
    check_impulses(imp, o["impulses"], f"PIC {name}")


@pytest.mark.parametrize("iterations", [1, 10])
def test_pb_mpm_matches_oracle(iterations):
    s = scenes.scene_pb_drop(iterations=iterations)
    n = s.n_substeps
    g, imp, _ = gpu_with_impulses(s, n)
    o = run_oracle(s, n)
    assert g["status"] == 0 and o["status"] == 0
    assert_parity(g, o, s.x, n, f"PB it={iterations}")
    check_impulses(imp, o["impulses"], f"PB it={iterations}")


def test_pb_mpm_on_the_slab_with_blade_and_grasper():
    s = with_solver("c3s", (O.SOLVER_PB, 4, 0.7))
    n = 40
    g, imp, _ = gpu_with_impulses(s, n)
    o = run_oracle(s, n)
    assert g["status"] == 0
    assert_parity(g, o, s.x, n, "PB c3s")
    check_impulses(imp, o["impulses"], "PB c3s")


@pytest.mark.parametrize("solver", [PIC, (O.SOLVER_PB, 1, 0.5), (O.SOLVER_PB, 6, 0.3)])
def test_free_fall_is_uniform(solver):
    """Away from walls and tools every solver moves a stress-free block
    rigidly: v = v0 + n dt g, F = I, C = 0 (to FP32 rounding)."""
    s = scenes.tiny_block(n_grid=32, per_axis=8, seed=4, with_state=False)
    s.v = np.tile(np.float32([0.1, 0.0, -0.05]), (s.N, 1))
    s.solver = solver
    n = 12
    g = run_gpu(s, n)
    assert g["status"] == 0
    v0 = np.float32([0.1, 0.0, -0.05]).astype(np.float64)
    gv = np.asarray(s.gravity)
    np.testing.assert_allclose(g["v"], np.tile(v0 + n * s.dt * gv, (s.N, 1)), rtol=0, atol=1e-5)
    x_exp = s.x.astype(np.float64) + n * s.dt * v0 + s.dt ** 2 * gv * n * (n + 1) / 2
    np.testing.assert_allclose(g["x"], x_exp, rtol=0, atol=2e-6)
    np.testing.assert_allclose(g["F"], np.tile(np.eye(3), (s.N, 1, 1)), rtol=0, atol=1e-5)
    assert np.abs(g["C"]).max() < 2e-3


def stepped(scene, calls, config):
    from paper_2502_18437_amd import mpm
    sim = mpm.simulation_from_scene(scene, accum_mode=mpm.MPM_ACCUM_FIXED)
    sim.set_launch_config(**config)
    reads = []
    for c in calls:
        sim.step(c)
        r, st = sim.read_state()
        assert st == 0
        reads.append(r)
    imp = sim.tool_impulses()
    sim.close()
    return reads, imp


@pytest.mark.parametrize("solver", [PIC, (O.SOLVER_PB, 3, 0.5)])
def test_graphs_and_launch_configs_are_bitwise_in_fixed_mode(solver):
    s = with_solver("c3s", solver)
    calls = [13, 3, 11]
    print(f"[solver graphs {solver}]", flush=True)
    ref, imp_ref = stepped(s, calls, {"graph_chunk": 0, "resort_interval": 8})
    for cfg in ({"graph_chunk": 4, "resort_interval": 8}, {"graph_chunk": 2, "resort_interval": 3, "transfer_wgs": 64},
                {"graph_chunk": 0, "resort_interval": 1, "transfer_wgs": 1024}):
        got, imp = stepped(s, calls, cfg)
        for r_e, r_g in zip(ref, got):
            for k in ("x", "v", "C", "F"):
                assert np.array_equal(r_e[k], r_g[k]), (cfg, k)
        assert np.array_equal(imp_ref, imp), cfg


@pytest.mark.parametrize("solver", [PIC, (O.SOLVER_PB, 3, 0.5)])
def test_batch_equals_its_scenes_in_fixed_mode(solver):
    from paper_2502_18437_amd import mpm
    b = scenes.batch_c4s()
    n = 12
    sim = mpm.Simulation(b.n_grid, b.dt, gravity=b.gravity, wall_band=b.wall_band, nu=b.nu, E_default=b.E_default,
                         max_particles=b.N, n_scenes=len(b.scenes), accum_mode=mpm.MPM_ACCUM_FIXED)
    sim.set_batch_particles(b.counts, b.concat("x"), b.concat("v"), b.concat("C"), b.concat("F"), b.concat("E"),
                            b.mass, b.vol0)
    for s_i, sc in enumerate(b.scenes):
        for k, t in enumerate(sc.tools):
            sim.set_tool(k, t.type, scene=s_i, **t.kwargs())
    sim.set_solver(*solver)
    sim.step(n)
    r, st = sim.read_state()
    assert st == 0
    imp = [sim.tool_impulses(scene=i) for i in range(len(b.scenes))]
    sim.close()
    offs = np.concatenate([[0], np.cumsum(b.counts)])
    for i, sc in enumerate(b.scenes):
        sc.solver = solver
        one = mpm.simulation_from_scene(sc, accum_mode=mpm.MPM_ACCUM_FIXED)
        one.step(n)
        q, st1 = one.read_state()
        imp1 = one.tool_impulses()
        one.close()
        assert st1 == 0
        for k in ("x", "v", "C", "F"):
            assert np.array_equal(r[k][offs[i]:offs[i + 1]], q[k]), (i, k)
        assert np.array_equal(imp[i], imp1), i


def test_solver_switch_validates_and_gates_the_rollout():
    import torch
    from paper_2502_18437_amd import mpm
    s = scenes.make("c5s")
    sim = mpm.simulation_from_scene(s)
    assert sim.solver()["solver"] == mpm.MPM_SOLVER_MLS
    for bad in ((3, 1, 0.5), (-1, 1, 0.5), (mpm.MPM_SOLVER_PB, 0, 0.5), (mpm.MPM_SOLVER_PB, 1025, 0.5),
                (mpm.MPM_SOLVER_PB, 4, 1.5), (mpm.MPM_SOLVER_PB, 4, float("nan"))):
        with pytest.raises(mpm.MPMError) as e:
            sim.set_solver(*bad)
        assert e.value.code == mpm.MPM_EINVAL
    sim.set_solver(mpm.MPM_SOLVER_PB, 7, 0.25)
    got = sim.solver()
    assert got["solver"] == mpm.MPM_SOLVER_PB and got["iterations"] == 7 and got["beta"] == 0.25
    theta = torch.as_tensor(s.theta, device="cuda")
    with pytest.raises(mpm.MPMError) as e:
        sim.rollout_forward(2, 1, theta=theta)
    assert e.value.code == mpm.MPM_EINVAL
    sim.set_solver(mpm.MPM_SOLVER_MLS)
    sim.rollout_forward(2, 1, theta=theta)
    sim.rollout_backward()
    sim.close()


def test_switching_solvers_mid_run_matches_the_oracle():
    """MLS-MPM for 20 substeps, then standard MPM for 20 (the C slot changes
    meaning from the affine matrix to the velocity gradient)."""
    from paper_2502_18437_amd import mpm
    s = scenes.make("c2s")
    sim = mpm.simulation_from_scene(s)
    sim.step(20)
    sim.set_solver(mpm.MPM_SOLVER_PIC)
    sim.step(20)
    r, st = sim.read_state()
    sim.close()
    assert st == 0
    o = O.Oracle(s.n_grid, s.dt, gravity=s.gravity, wall_band=s.wall_band, nu=s.nu, E_default=s.E_default)
    o.set_particles(s.x, s.v, s.C, s.F, s.E, s.mass, s.vol0)
    for k, t in enumerate(s.tools):
        o.set_tool(k, t.type, **t.kwargs())
    assert o.step(20) == 0
    o.set_solver(O.SOLVER_PIC)
    assert o.step(20) == 0
    assert_parity({k: v.astype(np.float64) for k, v in r.items()}, o.read(), s.x, 40, "MLS then PIC")


@pytest.mark.parametrize("solver", [PIC, (O.SOLVER_PB, 5, 0.6)])
def test_solvers_with_thin_tools_and_a_velocity_table(solver):
    """The other solvers share the grid update, so the slicer, the segment and
    a capsule following a per-substep velocity table act on them too."""
    from tests.test_gpu_adjoint import three_tool_scene
    s = three_tool_scene()
    s.solver = solver
    n = s.n_substeps
    g, imp, _ = gpu_with_impulses(s, n)
    o = run_oracle(s, n)
    assert g["status"] == 0 and o["status"] == 0
    assert_parity(g, o, s.x, n, f"thin tools {solver}")
    for q in range(3):
        assert np.abs(o["impulses"][q]).max() > 0, q  # every tool touched the material
    check_impulses(imp, o["impulses"], f"thin tools {solver}")

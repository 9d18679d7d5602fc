"""Parity of the HIP substep (through the C ABI) with the FP64 oracle on the
same seeded inputs, at sizes the oracle finishes in seconds (several grid
blocks, ragged particle counts), plus edge cases and error codes."""
import copy

import numpy as np
import pytest

import oracle as O
from paper_2502_18437_amd import scenes
from tests.parity import advance_tools, assert_parity, dyadic_poses, errors, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def mpm():
    from paper_2502_18437_amd import mpm as m
    return m


# ---------------------------------------------------------------- stress
def test_stress_matches_oracle():
    rng = np.random.default_rng(0)
    Fs = [np.eye(3) + s * rng.normal(size=(400, 3, 3)) for s in (1e-4, 1e-2, 0.1, 0.3)]
    F = np.concatenate(Fs).astype(np.float32)
    F = F[np.linalg.det(F.astype(np.float64)) > 0.05]
    E = rng.uniform(2e3, 8e3, F.shape[0]).astype(np.float32)
    tau = mpm().eval_stress(F, E, 0.4)
    ref = np.stack([O.kirchhoff(F[i].astype(np.float64), float(E[i]), 0.4)[0] for i in range(F.shape[0])])
    scale = E[:, None, None].astype(np.float64) * np.maximum(1.0, np.abs(F).max(axis=(1, 2)))[:, None, None] ** 2
    err = np.max(np.abs(tau - ref) / scale)
    print(f"[stress] max err / (E |F|^2) = {err:.3e}", flush=True)
    assert err < 2e-6


def test_stress_inverted_uses_signfixed_rotation():
    rng = np.random.default_rng(1)
    F = (np.eye(3) + 0.2 * rng.normal(size=(200, 3, 3)))
    F[:, 2, :] *= -1.0  # det < 0
    F = F[np.linalg.det(F) < -0.05].astype(np.float32)
    E = np.full(F.shape[0], 5e3, np.float32)
    tau = mpm().eval_stress(F, E, 0.3)
    ref = np.stack([O.kirchhoff(F[i].astype(np.float64), 5e3, 0.3)[0] for i in range(F.shape[0])])
    err = np.max(np.abs(tau - ref)) / (5e3 * np.max(np.abs(F)) ** 2)
    print(f"[stress inverted] err = {err:.3e}", flush=True)
    assert err < 1e-5


# ---------------------------------------------------------------- scenes
def test_c1_parity_and_closed_form():
    s = scenes.scene_c1()
    g = run_gpu(s, s.n_substeps)
    o = run_oracle(s, s.n_substeps)
    assert g["status"] == 0 and o["status"] == 0
    assert_parity(g, o, s.x, s.n_substeps, "c1")
    # closed form: dy = g dt^2 n(n+1)/2, vy = n dt g (FP32 rounding only)
    dy = -9.8 * s.dt ** 2 * 100 * 101 / 2
    assert np.max(np.abs(g["x"][:, 1] - s.x[:, 1].astype(np.float64) - dy)) < 2e-7
    assert np.max(np.abs(g["v"][:, 1] + 0.098)) < 1e-6


def test_c1s_parity():
    s = scenes.scene_c1s()
    g = run_gpu(s, s.n_substeps)
    o = run_oracle(s, s.n_substeps)
    assert g["status"] == 0 and o["status"] == 0
    assert_parity(g, o, s.x, s.n_substeps, "c1s")


@pytest.mark.parametrize("name", ["c2s", "c3s"])
def test_contact_scene_parity(name):
    s = scenes.make(name)
    g = run_gpu(s, s.n_substeps)
    o = run_oracle(s, s.n_substeps)
    assert g["status"] == 0 and o["status"] == 0
    assert np.linalg.norm(o["impulses"][0]) > 0  # the tool acts
    assert_parity(g, o, s.x, s.n_substeps, name)


def test_c3m_parity_many_blocks():
    s = scenes.scene_c3m()
    n = 40
    g = run_gpu(s, n)
    o = run_oracle(s, n)
    assert g["status"] == 0 and o["status"] == 0
    assert g["info"]["occupied_blocks"] > 8
    assert_parity(g, o, s.x, n, "c3m")


@pytest.mark.parametrize("resort", [1, 5, 1000])
def test_rebinning_schedules(resort):
    s = scenes.scene_c2s()
    g = run_gpu(s, s.n_substeps, resort_interval=resort, rebin_drift=0)  # the fixed schedule only
    o = run_oracle(s, s.n_substeps)
    assert_parity(g, o, s.x, s.n_substeps, f"c2s resort={resort}")
    assert g["info"]["resorts"] == (1 if resort >= s.n_substeps else -(-s.n_substeps // resort))


def test_chunked_steps_match():
    s = scenes.scene_c2s()
    g = run_gpu(s, s.n_substeps, chunks=[1, 2, 3, 10, 84])
    o = run_oracle(s, s.n_substeps)
    assert_parity(g, o, s.x, s.n_substeps, "c2s chunked")


def test_resume_in_fp32_mode_matches_the_uninterrupted_oracle():
    """Checkpoint and resume in the default FP32 mode: the state read after
    40 substeps, given to a new handle with its tools at the poses they
    reached, ends within the parity tolerances of the oracle's uninterrupted
    100-substep run (float atomics make the bits order-dependent here)."""
    from paper_2502_18437_amd import mpm
    s = dyadic_poses(scenes.scene_c2s())
    n1, n2 = 40, 60
    sim = mpm.simulation_from_scene(s)
    sim.step(n1)
    mid, st = sim.read_state(allow_errors=True)
    sim.close()
    assert st == 0
    t = copy.deepcopy(s)
    t.x, t.v, t.C, t.F = (np.array(mid[k], np.float32) for k in ("x", "v", "C", "F"))
    advance_tools(t, n1)
    g = run_gpu(t, n2)
    assert g["status"] == 0
    o = run_oracle(s, n1 + n2)
    assert_parity(g, o, s.x, n1 + n2, "c2s resumed")


def test_shuffled_particle_order():
    s = scenes.scene_c3s()
    perm = np.random.default_rng(9).permutation(s.N)
    s.x = s.x[perm]
    s.E = s.E[perm]
    g = run_gpu(s, s.n_substeps)
    o = run_oracle(s, s.n_substeps)
    assert_parity(g, o, s.x, s.n_substeps, "c3s shuffled")


@pytest.mark.parametrize("per_axis", [1, 2, 5, 11])
def test_ragged_particle_counts(per_axis):
    s = scenes.tiny_block(n_grid=32, per_axis=per_axis, seed=per_axis, E_range=(2e3, 8e3))
    g = run_gpu(s, 20)
    o = run_oracle(s, 20)
    assert g["status"] == 0 and o["status"] == 0
    assert_parity(g, o, s.x, 20, f"ragged N={s.N}")


def test_drift_out_of_tile_fallback():
    """Fast particles and no re-binning: stencils leave their block's tile,
    take the global-memory path and claim overflow blocks."""
    s = scenes.tiny_block(n_grid=32, per_axis=8, seed=3, center=(0.35, 0.5, 0.4), with_state=False)
    s.dt = 1e-3
    s.gravity = (0.0, 0.0, 0.0)
    s.v = np.tile(np.array([12.0, 3.0, -6.0], np.float32), (s.N, 1))
    n = 20
    g = run_gpu(s, n, resort_interval=1000)
    o = run_oracle(s, n)
    assert g["info"]["n_fallback"] > 0
    assert_parity(g, o, s.x, n, "drift")


def test_walls_stop_particles():
    s = scenes.tiny_block(n_grid=32, per_axis=6, seed=4, center=(0.5, 0.16, 0.5), with_state=False)
    s.v = np.tile(np.array([0.0, -3.0, 0.5], np.float32), (s.N, 1))
    g = run_gpu(s, 100)
    o = run_oracle(s, 100)
    assert np.linalg.norm(o["impulses"][8]) > 0
    assert_parity(g, o, s.x, 100, "walls")


# ---------------------------------------------------------------- API paths
def test_device_pointer_path_matches_host_path():
    import torch
    s = scenes.scene_c2s()
    m = mpm()
    dev = torch.device("cuda", 0)
    sim = m.Simulation(s.n_grid, s.dt, gravity=s.gravity, nu=s.nu, max_particles=s.N)
    sim.set_particles(torch.from_numpy(s.x).to(dev), None, None, None, torch.from_numpy(s.E).to(dev),
                      s.mass, s.vol0)
    for k, t in enumerate(s.tools):
        sim.set_tool(k, t.type, **t.kwargs())
    sim.step(30)
    out = {k: torch.empty((s.N, 3) if k in "xv" else (s.N, 3, 3), dtype=torch.float32, device=dev)
           for k in ("x", "v", "C", "F")}
    sim.read_state(out)
    o = run_oracle(s, 30)
    gd = {k: out[k].cpu().numpy().astype(np.float64) for k in out}
    assert_parity(gd, o, s.x, 30, "device pointers")
    sim.close()


def test_empty_scene_and_single_particle():
    m = mpm()
    sim = m.Simulation(32, 1e-4, max_particles=16)
    sim.set_particles(np.zeros((0, 3), np.float32), mass=1.0, vol0=1.0)
    sim.step(5)
    r, st = sim.read_state()
    assert st == 0 and r["x"].shape == (0, 3)
    one = np.array([[0.5, 0.5, 0.5]], np.float32)
    sim.set_particles(one, mass=1e-3, vol0=1e-6)
    sim.step(10)
    r, st = sim.read_state()
    assert st == 0
    dy = -9.8 * 1e-8 * 10 * 11 / 2
    assert abs(r["x"][0, 1] - (0.5 + dy)) < 1e-7
    sim.close()


@pytest.mark.parametrize("rebin_mode", ["in_place", "advance"])
def test_particles_leaving_the_grid_keep_their_last_state(rebin_mode):
    """A block falling through the floor of a grid without walls: its
    particles leave the grid one layer after another, and from then on each
    is left unchanged (EDOMAIN) with the v, C, F and x of the substep that
    moved it out, as in the oracle. The re-binnings every 3 substeps (in
    place, then also after a G2P pass) sort those particles last, with a
    sentinel key; their state must travel with them."""
    m = mpm()
    s = scenes.tiny_block(n_grid=32, per_axis=6, seed=21, center=(0.5, 0.2, 0.5))
    s.wall_band = 0
    s.dt = 5e-4
    # falling at 30 m/s and spinning at 20 rad/s about z, so that particles
    # of one block differ in velocity by up to a few m/s: a particle that
    # carried another's v would be far outside the bar
    w = 20.0
    r = s.x.astype(np.float64) - np.array([0.5, 0.2, 0.5])
    spin = np.stack([-w * r[:, 1], w * r[:, 0], np.zeros(s.N)], axis=1)
    s.v = (s.v + spin + np.array([0.0, -30.0, 0.0])).astype(np.float32)
    s.C = (s.C + np.array([[0.0, -w, 0.0], [w, 0.0, 0.0], [0.0, 0.0, 0.0]])).astype(np.float32)
    k = 13  # the lowest layers leave from about substep 10 on
    mode = m.MPM_REBIN_IN_PLACE if rebin_mode == "in_place" else m.MPM_REBIN_ADVANCE
    g = run_gpu(s, k, resort_interval=3, rebin_mode=mode)
    o = run_oracle(s, k)
    assert g["status"] == m.MPM_EDOMAIN and o["status"] == O.ST_EDOMAIN
    gone = np.nonzero(o["x"][:, 1] / s.dx - 0.5 < 0.0)[0]
    assert 20 < gone.size < s.N  # some left early, some stay in the grid
    assert g["info"]["resorts"] >= 4
    assert_parity(g, o, s.x, k, f"leaving the grid ({rebin_mode}, {gone.size} left)")
    # the particles that left, on their own: each carries its own last state
    sub = lambda r: {f: r[f][gone] for f in ("x", "v", "C", "F")}  # noqa: E731
    assert_parity(sub(g), sub(o), s.x[gone], k, f"the {gone.size} particles that left ({rebin_mode})")


def test_error_codes():
    m = mpm()
    with pytest.raises(m.MPMError) as e:
        m.Simulation(4, 1e-4)
    assert e.value.code == m.MPM_EINVAL
    with pytest.raises(m.MPMError):
        m.Simulation(32, -1.0)
    sim = m.Simulation(32, 1e-4, max_particles=8)
    with pytest.raises(m.MPMError) as e:
        sim.set_particles(np.full((9, 3), 0.5, np.float32), mass=1.0, vol0=1.0)  # over capacity
    assert e.value.code == m.MPM_EINVAL
    with pytest.raises(m.MPMError):
        sim.set_tool(8, m.MPM_TOOL_CAPSULE, size=(0.1, 0.01, 0))
    with pytest.raises(m.MPMError):
        sim.set_tool(0, m.MPM_TOOL_CAPSULE, size=(0.1, -0.01, 0))
    with pytest.raises(m.MPMError):
        sim.step(-1)
    x = np.full((4, 3), 0.5, np.float32)
    x[1] = [0.01, 0.5, 0.5]  # stencil outside the grid (x / dx - 1/2 < 0)
    sim.set_particles(x, mass=1e-3, vol0=1e-6)
    sim.step(2)
    r, st = sim.read_state(allow_errors=True)
    assert st == m.MPM_EDOMAIN
    np.testing.assert_array_equal(r["x"][1], x[1])  # left unchanged
    x[1] = [np.nan, 0.5, 0.5]
    sim.set_particles(x, mass=1e-3, vol0=1e-6)
    sim.step(1)
    assert sim.read_state(allow_errors=True)[1] == m.MPM_ENONFINITE
    F = np.tile(np.eye(3, dtype=np.float32), (4, 1, 1))
    F[2] = np.diag([1.0, 1.0, -0.5])
    x[1] = [0.45, 0.5, 0.5]
    sim.set_particles(x, F=F, mass=1e-3, vol0=1e-6)
    sim.step(1)
    assert sim.read_state(allow_errors=True)[1] == m.MPM_EINVERTED
    # errors clear on the next set_particles
    sim.set_particles(x, mass=1e-3, vol0=1e-6)
    sim.step(1)
    assert sim.read_state()[1] == 0
    sim.close()


def test_info_counters():
    s = scenes.scene_c2s()
    m = mpm()
    sim = m.simulation_from_scene(s)
    sim.step(10)
    info = sim.info()
    assert info["n_particles"] == s.N
    assert info["substeps"] == 10
    assert info["occupied_blocks"] > 0 and info["active_blocks"] >= info["occupied_blocks"]
    assert info["active_nodes"] > 0
    assert info["n_tools"] == 1
    sim.close()

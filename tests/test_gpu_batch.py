"""Batches of scenes in one handle: every scene of a batch must give what the
same scene gives alone (bit for bit in the fixed-point mode, where all sums
are exact integers) and match the FP64 oracle; tools, walls and impulses
stay per scene."""
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


def batch_sim(b, **kw):
    from paper_2502_18437_amd import mpm
    sim = mpm.Simulation(b.n_grid, b.dt, gravity=b.gravity, wall_band=b.wall_band, nu=b.nu, E_default=b.E_default,
                         max_particles=max(1, b.N), n_scenes=len(b.scenes), **kw)
    sim.set_batch_particles(b.counts, b.concat("x"), b.concat("v"), b.concat("C"), b.concat("F"), b.concat("E"),
                            b.mass, b.vol0)
    for s_i, sc in enumerate(b.scenes):
        for k, t in enumerate(sc.tools):
            sim.set_tool(k, t.type, scene=s_i, **t.kwargs())
    return sim


def split(arr, counts):
    return np.split(arr, np.cumsum(counts)[:-1])


def run_batch(b, n, **kw):
    sim = batch_sim(b, **kw)
    print(f"[batch {b.name}: {len(b.scenes)} scenes, {b.N} particles, {n} substeps, {kw}]", flush=True)
    sim.step(n)
    r, st = sim.read_state(allow_errors=True)
    imp = [sim.tool_impulses(scene=i) for i in range(len(b.scenes))]
    info = sim.info()
    sim.close()
    per = [dict(zip(r.keys(), parts)) for parts in zip(*[split(v, b.counts) for v in r.values()])]
    return per, st, imp, info


def run_single(sc, n, **kw):
    from paper_2502_18437_amd import mpm
    sim = mpm.simulation_from_scene(sc, **kw)
    sim.step(n)
    r, st = sim.read_state(allow_errors=True)
    imp = sim.tool_impulses()
    sim.close()
    return r, st, imp


@pytest.mark.parametrize("resort", [1, 7])
def test_batch_is_bitwise_the_single_scene_path_in_fixed_mode(resort):
    from paper_2502_18437_amd import mpm
    b = scenes.batch_c4s()
    n = b.scenes[0].n_substeps
    per, st, imp, _ = run_batch(b, n, accum_mode=mpm.MPM_ACCUM_FIXED, resort_interval=resort)
    assert st == 0
    for i, sc in enumerate(b.scenes):
        r, st1, imp1 = run_single(sc, n, accum_mode=mpm.MPM_ACCUM_FIXED, resort_interval=resort)
        assert st1 == 0
        for k in ("x", "v", "C", "F"):
            assert np.array_equal(per[i][k], r[k]), (i, k)
        assert np.array_equal(imp[i], imp1), i


def test_batch_scenes_match_the_oracle():
    b = scenes.batch_c4s()
    n = b.scenes[0].n_substeps
    per, st, imp, _ = run_batch(b, n)
    assert st == 0
    touched = 0
    for i, sc in enumerate(b.scenes):
        o = run_oracle(sc, n)
        g = {k: v.astype(np.float64) for k, v in per[i].items()}
        assert_parity(g, o, sc.x, n, f"batch scene {i}")
        scale = np.max(np.abs(o["impulses"]))
        if scale > 0:
            touched += 1
            np.testing.assert_allclose(imp[i], -o["impulses"], rtol=0, atol=2e-3 * scale)
    assert touched >= 3  # the capsules start in contact


def test_uneven_and_empty_scenes():
    """Scenes of 0, 1 and many particles side by side; the empty ones change
    nothing and report no impulses."""
    base = scenes.batch_c4s()
    sc_empty = scenes.Scene("empty", base.n_grid, base.dt, 10, base.nu, base.E_default, base.mass, base.vol0,
                            np.zeros((0, 3), np.float32))
    one = base.scenes[1]
    single = scenes.Scene("one", base.n_grid, base.dt, 10, base.nu, base.E_default, base.mass, base.vol0,
                          one.x[:1].copy(), tools=[])
    b = scenes.Batch("mixed", [sc_empty, base.scenes[0], single, sc_empty, base.scenes[2]], base.n_grid, base.dt, 10,
                     base.nu, base.E_default, base.mass, base.vol0)
    per, st, imp, info = run_batch(b, 10)
    assert st == 0
    assert info["n_tools"] == 2
    for i, sc in enumerate(b.scenes):
        if sc.N == 0:
            assert per[i]["x"].shape == (0, 3)
            assert not imp[i].any()
            continue
        o = run_oracle(sc, 10)
        assert_parity({k: v.astype(np.float64) for k, v in per[i].items()}, o, sc.x, 10, f"mixed {i}")


def test_scene_tools_stay_in_their_scene():
    """A tool of scene 1 placed where scene 0's material is leaves scene 0
    alone."""
    b = scenes.batch_c4s()
    b.scenes = b.scenes[:2]
    b.scenes[0].tools = []
    n = 10
    per, st, imp, _ = run_batch(b, n)
    assert st == 0
    o = run_oracle(b.scenes[0], n)
    assert_parity({k: v.astype(np.float64) for k, v in per[0].items()}, o, b.scenes[0].x, n, "isolated scene 0")
    assert not imp[0][:8].any()


def test_batch_calls_reject_bad_scenes():
    from paper_2502_18437_amd import mpm
    b = scenes.batch_c4s()
    sim = batch_sim(b)
    with pytest.raises(mpm.MPMError):
        sim.set_particles(b.scenes[0].x)  # several scenes: the batch call is required
    with pytest.raises(mpm.MPMError):
        sim.set_tool(0, O.TOOL_CAPSULE, size=(0.1, 0.05, 0), scene=len(b.scenes))
    with pytest.raises(mpm.MPMError):
        sim.tool_impulses(scene=-1)
    with pytest.raises(mpm.MPMError):
        sim.rollout_forward(2, 1)
    sim.close()


def test_c4_full_batch_runs_and_samples_match():
    """The full 256-scene batch (uneven 16^3 .. 40^3 cubes on 64^3 grids) for
    10 substeps; three scenes are checked against the oracle."""
    b = scenes.batch_c4()
    n = 10
    per, st, imp, info = run_batch(b, n)
    assert st == 0
    assert info["n_particles"] == b.N
    for i in (0, int(np.argmax(b.counts)), len(b.scenes) - 1):
        sc = b.scenes[i]
        o = run_oracle(sc, n)
        assert_parity({k: v.astype(np.float64) for k, v in per[i].items()}, o, sc.x, n, f"c4 scene {i}")


def test_push_out_in_one_scene_of_a_batch_in_fixed_mode():
    """Scene 1's capsule pushes particles out; the batch still equals each
    scene run alone, bit for bit (the push-out code path runs for every
    scene but acts only where a tool has it on)."""
    from paper_2502_18437_amd import mpm
    b = scenes.batch_c4s()
    t = b.scenes[1].tools[0]
    t.push_out = True
    t.lin_vel = (0.0, -2.0, 0.0)  # fast enough to end inside the capsule
    n = 16
    per, st, imp, _ = run_batch(b, n, accum_mode=mpm.MPM_ACCUM_FIXED)
    assert st == 0
    for i, sc in enumerate(b.scenes):
        r, st1, imp1 = run_single(sc, n, accum_mode=mpm.MPM_ACCUM_FIXED)
        assert st1 == 0
        for k in ("x", "v", "C", "F"):
            assert np.array_equal(per[i][k], r[k]), (i, k)
        assert np.array_equal(imp[i], imp1), i
    sc = b.scenes[1]
    sc.tools[0].push_out = False
    off, _, _ = run_single(sc, n, accum_mode=mpm.MPM_ACCUM_FIXED)
    assert not np.array_equal(off["x"], per[1]["x"])  # the push-out acted in scene 1

"""Transfer work tiles of 4 cells against 8 cells. The tile edge changes only
how particles are grouped into LDS tiles: in the fixed-point mode every P2G
sum is an exact integer sum, so the state and the impulses must be bit for
bit those of 8-cell tiles, whatever the scene (contact, dense blocks split
into several work items, particles drifting out of their tiles, batches of
scenes, the other solvers). In FP32 the 4-cell tiles match the oracle to the
parity bar. The tile can be switched between calls, and the autotuner
chooses among both edges."""
import numpy as np
import pytest

from paper_2502_18437_amd import scenes
from tests.parity import assert_parity, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def mpm():
    from paper_2502_18437_amd import mpm as m
    return m


def run_with_impulses(s, n, **kw):
    m = mpm()
    sim = m.simulation_from_scene(s, **kw)
    sim.step(n)
    r, st = sim.read_state(allow_errors=True)
    info = sim.info()
    imp = sim.tool_impulses()
    sim.close()
    r = {k: np.asarray(v, np.float32) for k, v in r.items()}
    return r, imp, st, info


def same_bits(a, b, label):
    for k in ("x", "v", "C", "F"):
        assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), (label, k)


@pytest.mark.parametrize("name,n", [("c2s", 60), ("c3s", 60), ("c3m", 30)])
def test_tile_edges_agree_bitwise_in_fixed_mode(name, n):
    m = mpm()
    s = scenes.make(name)
    a, ia, sa, infa = run_with_impulses(s, n, accum_mode=m.MPM_ACCUM_FIXED, tile=8)
    b, ib, sb, infb = run_with_impulses(s, n, accum_mode=m.MPM_ACCUM_FIXED, tile=4)
    assert sa == 0 and sb == 0
    assert infa["tile"] == 8 and infb["tile"] == 4
    # a 4-cell tile covers an eighth of a block: more occupied tiles
    assert infb["occupied_blocks"] > infa["occupied_blocks"]
    same_bits(a, b, name)
    assert np.array_equal(ia, ib)


@pytest.mark.parametrize("solver", [None, (1, 1, 0.5), (2, 4, 0.7)])
def test_tile_edges_agree_bitwise_for_every_solver(solver):
    m = mpm()
    s = scenes.scene_c3s()
    s.solver = solver
    n = 20 if solver is None or solver[0] != 2 else 5
    a = run_with_impulses(s, n, accum_mode=m.MPM_ACCUM_FIXED, tile=8)[0]
    b = run_with_impulses(s, n, accum_mode=m.MPM_ACCUM_FIXED, tile=4)[0]
    same_bits(a, b, f"solver {solver}")


def test_dense_and_drifting_tiles_agree_bitwise():
    """The dense falling cube (blocks split into several work items, items
    dealt to lanes apart) and a re-binning interval long enough that
    particles drift out of their tiles (global-memory path)."""
    m = mpm()
    s = scenes.scene_cube(1 << 15)
    s.n_substeps = 12
    ra, _, sa, ia = run_with_impulses(s, 12, accum_mode=m.MPM_ACCUM_FIXED, tile=8, resort_interval=6)
    rb, _, sb, ib = run_with_impulses(s, 12, accum_mode=m.MPM_ACCUM_FIXED, tile=4, resort_interval=6)
    assert sa == 0 and sb == 0
    assert ib["n_fallback"] > 0
    same_bits(ra, rb, "dense cube")


def test_batch_with_4_cell_tiles_is_each_scene_alone_in_fixed_mode():
    """The 6-scene batch with 4-cell tiles against each scene run alone with
    8-cell tiles: bit for bit, impulses included."""
    from tests.test_gpu_batch import run_batch, run_single
    m = mpm()
    b = scenes.batch_c4s()
    n = 20
    per, st, imp, info = run_batch(b, n, accum_mode=m.MPM_ACCUM_FIXED, tile=4, resort_interval=5)
    assert st == 0 and info["tile"] == 4
    for i, sc in enumerate(b.scenes):
        r, st1, imp1 = run_single(sc, n, accum_mode=m.MPM_ACCUM_FIXED, tile=8)
        assert st1 == 0
        for k in ("x", "v", "C", "F"):
            assert np.array_equal(per[i][k], r[k]), (i, k)
        assert np.array_equal(imp[i], imp1), i


@pytest.mark.parametrize("name", ["c1s", "c2s", "c3s"])
def test_4_cell_tiles_match_the_oracle(name):
    s = scenes.make(name)
    g = run_gpu(s, s.n_substeps, tile=4)
    o = run_oracle(s, s.n_substeps)
    assert g["status"] == 0 and g["info"]["tile"] == 4
    assert_parity(g, o, s.x, s.n_substeps, f"{name} 4-cell tiles")


def test_switching_the_tile_between_calls():
    """8-cell tiles for 30 substeps, 4-cell tiles for 40, 8 again for 30
    (each switch re-bins) against the oracle's 100 substeps, and in the
    fixed-point mode bit for bit against one call with 8-cell tiles."""
    m = mpm()
    s = scenes.scene_c2s()

    def chunked(**kw):
        sim = m.simulation_from_scene(s, **kw)
        for tile, k in ((8, 30), (4, 40), (8, 30)):
            sim.set_launch_config(tile=tile)
            assert sim.launch_config()["tile"] == tile
            sim.step(k)
        r, st = sim.read_state()
        sim.close()
        return {k: np.asarray(v, np.float32) for k, v in r.items()}, st

    g, st = chunked()
    assert st == 0
    o = run_oracle(s, 100)
    assert_parity({k: v.astype(np.float64) for k, v in g.items()}, o, s.x, 100, "c2s tile switches")
    f, _ = chunked(accum_mode=m.MPM_ACCUM_FIXED)
    ref = run_with_impulses(s, 100, accum_mode=m.MPM_ACCUM_FIXED, tile=8)[0]
    same_bits(f, ref, "tile switches")


def test_autotuner_considers_both_tile_edges():
    m = mpm()
    s = scenes.scene_c3m()
    sim = m.simulation_from_scene(s)
    cfg = sim.autotune(trial_substeps=8)
    assert cfg["tile"] in (4, 8)
    assert sim.launch_config() == cfg
    sim.step(10)
    r, st = sim.read_state()
    sim.close()
    assert st == 0 and np.isfinite(r["x"]).all()
    with pytest.raises(m.MPMError):
        sim2 = m.simulation_from_scene(s)
        try:
            sim2.set_launch_config(tile=6)
        finally:
            sim2.close()

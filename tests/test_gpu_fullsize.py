"""Parity at the full benchmark sizes (c2: 1,048,576 particles on 128^3;
c3: 4,194,304 particles on 256^3) in the library's default launch
configuration, on sampled outputs the oracle can compute.

A particle's update in one substep reads the 27 nodes of its stencil, and
those nodes hold contributions of particles whose base cells lie within
+-2 cells of its own. After k substeps a particle therefore depends only on
the initial particles within 2k cells of it (plus its drift, far below a
cell here). The oracle runs the whole grid but only the particles of a core
box widened by a margin of 2k + 3 cells; particles of the core are then
exact samples of the full-scene result."""
import numpy as np
import pytest

from paper_2502_18437_amd import scenes
from tests.parity import assert_parity, run_oracle, subbox

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_full_gpu(s, k, **kw):
    from paper_2502_18437_amd import mpm
    sim = mpm.simulation_from_scene(s, **kw)
    sim.step(k)
    r, st = sim.read_state()
    info = sim.info()
    sim.close()
    assert st == 0
    return {kk: v.astype(np.float64) for kk, v in r.items()}, info


def check_cores(s, g, k, cores, label):
    dx = s.dx
    margin = (2 * k + 3) * dx
    for lo, hi in cores:
        lo, hi = np.asarray(lo), np.asarray(hi)
        region = subbox(s.x, lo - margin, hi + margin)
        core = subbox(s.x, lo, hi)
        assert core.size > 100, (lo, hi, core.size)
        o = run_oracle(s, k, idx=region)
        pos = np.searchsorted(region, core)
        assert np.array_equal(region[pos], core)
        oc = {kk: o[kk][pos] for kk in ("x", "v", "C", "F")}
        gc = {kk: g[kk][core] for kk in ("x", "v", "C", "F")}
        assert_parity(gc, oc, s.x[core], k, f"{label} core {lo}-{hi} ({core.size} particles)")


def test_c3_full_size_sampled():
    s = scenes.scene_c3()
    k = 10
    g, info = run_full_gpu(s, k, resort_interval=4)
    assert info["resorts"] == 3
    top = 3 * s.dx + 0.2
    cores = [
        ((0.22, top - 0.04, 0.48), (0.27, top, 0.52)),   # blade leading edge
        ((0.76, top - 0.04, 0.28), (0.82, top, 0.32)),   # capsule end cap
        ((0.40, 0.012, 0.60), (0.44, 0.05, 0.64)),        # bulk on the floor band
    ]
    check_cores(s, g, k, cores, "c3")


def test_c2_full_size_sampled():
    s = scenes.scene_c2()
    k = 10
    g, info = run_full_gpu(s, k)
    top = 3 * s.dx + 0.2
    cores = [
        ((0.46, top - 0.05, 0.6), (0.54, top, 0.68)),    # under the capsule, off its centre
        ((0.1, 0.02, 0.1), (0.16, 0.08, 0.16)),           # slab corner on the floor band
    ]
    check_cores(s, g, k, cores, "c2")

"""Parity at the full benchmark sizes (c2: 1,048,576 particles on 128^3;
c3: 4,194,304 particles on 256^3) in the library's default launch
configuration, on sampled outputs the oracle can compute: over the
100-substep window against stored oracle runs of the whole scene
(tests/golden/make_fullsize.py), and over 10 substeps against live oracle
runs of core boxes.

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
from tests.parity import assert_parity, run_oracle, shifted_blobs, subbox

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
    g, info = run_full_gpu(s, k, resort_interval=4, rebin_drift=0)
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


def golden(name):
    """The oracle's 100-substep state of a full scene on sampled particles
    (tests/golden/make_fullsize.py); refused if the generator changed."""
    import os
    from tests.golden.make_fullsize import input_digest
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"fullsize_{name}_100.npz")
    z = np.load(path, allow_pickle=False)
    s = scenes.make(name)
    assert input_digest(s) == str(z["input_sha256"]), "scene generator changed: rerun make_fullsize.py"
    return s, z


@pytest.mark.parametrize("name,resort", [("c2", 0), ("c3", 0), ("c3", 32)])
def test_full_size_100_substeps_default_launch(name, resort):
    """The whole scene for the 100-substep parity window in the library's
    default launch configuration (re-binning every 256 substeps or earlier
    when particles drift out of their tiles, the re-binning mode chosen
    automatically, runs of substeps replayed as HIP graphs), and for c3 also
    re-binning every 32 substeps (in-place re-binnings inside the window),
    against the FP64 oracle's run of the same full scene on a sample of
    particles (uniform, plus particles along each tool's path), with the
    tool impulses of the 100 substeps."""
    from paper_2502_18437_amd import mpm
    s, z = golden(name)
    k = int(z["n_substeps"])
    sim = mpm.simulation_from_scene(s)
    cfg = sim.launch_config()
    assert cfg["resort_interval"] == 256 and cfg["rebin_mode"] == mpm.MPM_REBIN_AUTO and cfg["graph_chunk"] > 0
    assert cfg["rebin_drift"] > 0 and cfg["tile"] == 8
    if resort:
        sim.set_launch_config(resort_interval=resort)
    sim.step(k)
    r, st = sim.read_state()
    info = sim.info()
    imp = sim.tool_impulses()
    sim.close()
    assert st == 0 and int(z["status"]) == 0
    idx = z["idx"]
    g = {kk: r[kk][idx].astype(np.float64) for kk in ("x", "v", "C", "F")}
    o = {kk: z[kk] for kk in ("x", "v", "C", "F")}
    print(f"[{name} resort {resort or 'default'}] resorts={info['resorts']} fallback particle-substeps="
          f"{info['n_fallback']} active nodes={info['active_nodes']}", flush=True)
    if resort:
        assert info["resorts"] >= 4
    assert_parity(g, o, s.x[idx], k, f"{name} full scene, 100 substeps, {idx.size} sampled")
    # impulses on the tools are minus the momentum the tools gave the material
    oi = z["impulses"]
    scale = np.abs(oi).max()
    assert scale > 0
    np.testing.assert_allclose(imp, -oi, rtol=0, atol=2e-3 * scale)


@pytest.mark.parametrize("n_grid", [128, 1024])
def test_largest_grid_is_translation_invariant_bitwise(n_grid):
    """The largest grid, n_grid = 1024 (2^30 nodes, block ids up to 2^21 - 1),
    against an exact property the oracle's dense grid is too large to check
    there: a blob near the far corner and the same blob moved down by whole
    8-node blocks, both inside [0.5, 1) per axis, give the same v, C, F and
    the same x less the shift, bit for bit, in fixed-point mode. dx is a
    power of two and the shift a multiple of the FP32 ulp of that binade, so
    every rounding of the two runs lands on the same grid; nothing in the
    substep (no tools, walls 3 nodes from the blob) depends on where the
    blob is."""
    from paper_2502_18437_amd import mpm
    a, b, shift = shifted_blobs(n_grid)
    assert np.all(b.x >= 0.5) and np.all(a.x < 1.0)

    def run(s):
        sim = mpm.simulation_from_scene(s, accum_mode=mpm.MPM_ACCUM_FIXED)
        sim.step(s.n_substeps)
        r, st = sim.read_state(allow_errors=True)
        info = sim.info()
        sim.close()
        assert st == 0 and info["n_range"] == 0 and info["n_inverted"] == 0, (st, info)
        return {f: np.asarray(r[f], np.float32) for f in ("x", "v", "C", "F")}

    ra = run(a)
    rb = run(b)
    assert np.max(np.abs(ra["v"] - a.v)) > 1e-3  # the material responded
    xa = (ra["x"].astype(np.float64) - shift / n_grid).astype(np.float32)
    assert np.array_equal(xa.view(np.uint32), rb["x"].view(np.uint32))
    for f in ("v", "C", "F"):
        assert np.array_equal(ra[f].view(np.uint32), rb[f].view(np.uint32)), f

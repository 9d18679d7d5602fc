"""The fixed-point accumulation mode (MPM_ACCUM_FIXED): every P2G sum is an
exact integer sum, so the state is bit-identical across runs, particle
orders and re-binning schedules; it also matches the oracle to the FP32
tolerances."""
import copy

import numpy as np
import pytest

import oracle as O
from paper_2502_18437_amd import scenes
from tests.parity import assert_parity, advance_tools, dyadic_poses, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def fixed_run(s, n, **kw):
    from paper_2502_18437_amd import mpm
    return run_gpu(s, n, accum_mode=mpm.MPM_ACCUM_FIXED, **kw)


def same_bits(a, b):
    for k in ("x", "v", "C", "F"):
        assert np.array_equal(a[k].astype(np.float32).view(np.uint32), b[k].astype(np.float32).view(np.uint32)), k


def test_fixed_mode_parity():
    s = scenes.scene_c3s()
    g = fixed_run(s, s.n_substeps)
    o = run_oracle(s, s.n_substeps)
    assert g["status"] == 0
    assert_parity(g, o, s.x, s.n_substeps, "c3s fixed")


def test_fixed_mode_bit_identical_runs_and_schedules():
    s = scenes.scene_c2s()
    n = 60
    ref = fixed_run(s, n)
    same_bits(ref, fixed_run(s, n))
    same_bits(ref, fixed_run(s, n, resort_interval=1))
    same_bits(ref, fixed_run(s, n, resort_interval=7))
    same_bits(ref, fixed_run(s, n, resort_interval=1000))
    same_bits(ref, fixed_run(s, n, chunks=[5, 20, 35]))


def test_fixed_mode_bit_identical_under_shuffle():
    s = scenes.scene_c3s()
    n = 40
    ref = fixed_run(s, n)
    perm = np.random.default_rng(4).permutation(s.N)
    t = scenes.scene_c3s()
    t.x, t.E = t.x[perm], t.E[perm]
    sh = fixed_run(t, n)
    inv = np.argsort(perm)
    same_bits(ref, {k: sh[k][inv] for k in ("x", "v", "C", "F")})


def test_fixed_mode_bit_identical_with_tile_fallback():
    """Particles leaving their tile take the global path; the integer
    contributions are the same, so the result does not depend on it."""
    s = scenes.tiny_block(n_grid=32, per_axis=8, seed=3, center=(0.35, 0.5, 0.4), with_state=False)
    s.dt = 1e-3
    s.gravity = (0.0, 0.0, 0.0)
    s.v = np.tile(np.array([12.0, 3.0, -6.0], np.float32), (s.N, 1))
    a = fixed_run(s, 20, resort_interval=1000)
    b = fixed_run(s, 20, resort_interval=1, rebin_mode=1)
    assert a["info"]["n_fallback"] > 0 and b["info"]["n_fallback"] == 0
    same_bits(a, b)


@pytest.mark.parametrize("solver", [None, (O.SOLVER_PIC, 1, 0.5), (O.SOLVER_PB, 3, 0.5)])
def test_rebin_modes_agree_bitwise_on_a_drifting_block(solver):
    """Re-binning in place sorts by the positions of the coming G2P, so the
    particles that cross a block boundary in that substep scatter through
    global memory; re-binning after a G2P pass avoids that. The integer
    contributions are the same either way, for every solver."""
    s = scenes.tiny_block(n_grid=32, per_axis=8, seed=3, center=(0.35, 0.5, 0.4), with_state=False)
    s.dt = 1e-3
    s.gravity = (0.0, 0.0, 0.0)
    s.v = np.tile(np.array([12.0, 3.0, -6.0], np.float32), (s.N, 1))
    if solver is not None:
        s.solver = solver
    adv = fixed_run(s, 20, resort_interval=2, rebin_mode=1)
    for interval in (1, 2, 5):
        inp = fixed_run(s, 20, resort_interval=interval, rebin_mode=2)
        assert inp["info"]["n_fallback"] > 0, interval
        same_bits(adv, inp)


def test_resume_from_read_state_is_bitwise():
    """Checkpoint and resume: the state read after n1 substeps, handed to a
    new handle whose tools are set at the poses they have reached, goes on
    bit for bit like the uninterrupted run (the new handle bins its
    particles afresh; integer P2G sums do not depend on the order)."""
    from paper_2502_18437_amd import mpm
    s = dyadic_poses(scenes.scene_c2s())
    n1, n2 = 25, 35
    ref = fixed_run(s, n1 + n2)
    sim = mpm.simulation_from_scene(s, accum_mode=mpm.MPM_ACCUM_FIXED)
    sim.step(n1)
    mid, st = sim.read_state(allow_errors=True)
    sim.close()
    assert st == 0 and ref["status"] == 0
    t = copy.deepcopy(s)
    t.x, t.v, t.C, t.F = (np.array(mid[k], np.float32) for k in ("x", "v", "C", "F"))
    advance_tools(t, n1)
    res = fixed_run(t, n2)
    assert res["status"] == 0
    same_bits(ref, res)

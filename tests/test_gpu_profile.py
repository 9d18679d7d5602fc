"""Per-kernel event timing (mpm_profile / mpm_profile_read): which launches
are timed, at every substep or every k-th, and that timing changes no result
bit in the fixed-point mode."""
import numpy as np
import pytest

from paper_2502_18437_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sim(**kw):
    from paper_2502_18437_amd import mpm
    s = scenes.make("c3s")
    return mpm.simulation_from_scene(s, accum_mode=mpm.MPM_ACCUM_FIXED, resort_interval=1000, rebin_drift=0, **kw)


def test_timed_launches_every_substep_and_every_kth():
    sim = _sim()
    sim.profile(True)
    sim.step(20)  # substeps 0-19: P2G at the first, fused transfers after it
    p = sim.profile_read()
    print(f"[profile every 1] {p}", flush=True)
    assert p["p2g"][1] == 1 and p["g2p2g"][1] == 19 and p["grid"][1] == 20 and p["g2p"][1] == 1
    assert p["binning"][1] >= 1
    for name, (ms, n) in p.items():
        assert n == 0 or (np.isfinite(ms) and ms > 0.0), name
    sim.profile(True, every=4)  # clears the totals
    sim.step(20)  # substeps 20-39: timed at 20, 24, 28, 32, 36; 20 is the call's P2G
    p = sim.profile_read()
    print(f"[profile every 4] {p}", flush=True)
    assert p["p2g"][1] == 1 and p["g2p2g"][1] == 4 and p["grid"][1] == 5 and p["g2p"][1] == 1
    sim.profile(False)
    sim.close()


def test_timing_changes_no_result_bit():
    runs = []
    for every in (0, 1, 3):
        sim = _sim()
        if every:
            sim.profile(True, every=every)
        sim.step(17)
        sim.step(9)
        r, st = sim.read_state()
        assert st == 0
        runs.append(r)
        sim.close()
    for r in runs[1:]:
        for k in ("x", "v", "C", "F"):
            assert np.array_equal(runs[0][k], r[k]), k


def test_profile_rejects_a_negative_stride():
    from paper_2502_18437_amd import mpm
    sim = _sim()
    with pytest.raises(mpm.MPMError):
        sim._check(mpm._lib.mpm_profile(sim.h, -1))
    sim.close()

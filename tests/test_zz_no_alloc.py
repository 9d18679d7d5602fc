"""mpm_eval_stress_noalloc (the stress evaluation staged through the library's
fixed device array instead of per-call allocations) against mpm_eval_stress,
called through the C ABI: two calls in a row, the second smaller, must give
the existing entry point's result bit for bit (the same kernel), on host and
device arrays; sizes above the fixed maximum are refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2502_18437_amd import mpm
    return mpm


def _inputs(rng, n):
    # deformation gradients around I, a few of them inverted (the sign-fixed
    # polar path), and per-particle Young's moduli
    F = (np.eye(3, dtype=np.float64) + 0.15 * rng.standard_normal((n, 3, 3))).astype(np.float32)
    flip = rng.random(n) < 0.01
    F[flip, :, 0] *= -1.0
    E = rng.uniform(2e3, 8e3, n).astype(np.float32)
    return np.ascontiguousarray(F), E


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def test_noalloc_matches_eval_stress_on_host_arrays():
    mpm = _lib()
    rng = np.random.default_rng(2502)
    for n in (mpm.MPM_NOALLOC_MAX_PARTICLES, 40000, 1237):  # the largest, then smaller calls in a row
        F, E = _inputs(rng, n)
        ref = np.empty((n, 3, 3), np.float32)
        got = np.full((n, 3, 3), np.nan, np.float32)
        assert mpm.mpm_eval_stress(n, _ptr(F), _ptr(E), ctypes.c_float(0.4), _ptr(ref), mpm.MPM_HOST) == mpm.MPM_OK
        assert mpm.mpm_eval_stress_noalloc(n, _ptr(F), _ptr(E), ctypes.c_float(0.4), _ptr(got),
                                           mpm.MPM_HOST) == mpm.MPM_OK
        assert np.isfinite(ref).all()
        np.testing.assert_array_equal(got, ref)


def test_noalloc_matches_eval_stress_on_device_arrays():
    import torch
    mpm = _lib()
    rng = np.random.default_rng(18437)
    for n in (30000, 999):
        F, E = _inputs(rng, n)
        dF = torch.from_numpy(F).cuda()
        dE = torch.from_numpy(E).cuda()
        ref = torch.empty((n, 3, 3), dtype=torch.float32, device="cuda")
        got = torch.full((n, 3, 3), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        assert mpm.mpm_eval_stress(n, dF.data_ptr(), dE.data_ptr(), ctypes.c_float(0.3), ref.data_ptr(),
                                   mpm.MPM_DEVICE) == mpm.MPM_OK
        assert mpm.mpm_eval_stress_noalloc(n, dF.data_ptr(), dE.data_ptr(), ctypes.c_float(0.3), got.data_ptr(),
                                           mpm.MPM_DEVICE) == mpm.MPM_OK
        np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_refuses_sizes_above_its_maximum():
    mpm = _lib()
    n = mpm.MPM_NOALLOC_MAX_PARTICLES + 1
    F = np.tile(np.eye(3, dtype=np.float32), (n, 1, 1))
    E = np.full(n, 5e3, np.float32)
    tau = np.full((n, 3, 3), 7.0, np.float32)
    rc = mpm.mpm_eval_stress_noalloc(n, _ptr(F), _ptr(E), ctypes.c_float(0.3), _ptr(tau), mpm.MPM_HOST)
    assert rc == mpm.MPM_ETOOBIG
    assert b"MPM_NOALLOC_MAX_PARTICLES" in mpm.mpm_last_error(None)
    assert (tau == 7.0).all()  # nothing written
    # a valid call afterwards clears the message and works
    m = 16
    ref = np.empty((m, 3, 3), np.float32)
    assert mpm.mpm_eval_stress_noalloc(m, _ptr(F[:m].copy()), _ptr(E[:m].copy()), ctypes.c_float(0.3), _ptr(ref),
                                       mpm.MPM_HOST) == mpm.MPM_OK
    assert np.abs(ref).max() < 1e-3  # F = I: zero stress

"""Thin ctypes binding of the C ABI in include/mpm.h (argument marshalling
only: every step of the substep runs in the HIP library).

Importing this module loads ``libmpm.so`` from the package directory and
raises ImportError if it has not been built (``__graft_entry__.build()`` or
``python paper_2502_18437_amd/build.py``); there is no CPU fallback.

Module-level functions carry the C names (``mpm_create``, ``mpm_step``, ...);
``Simulation`` wraps one handle for Python callers. Arrays may be NumPy
arrays (host memory) or torch CUDA tensors (device memory, ``where`` =
MPM_DEVICE); they must be float32 and C-contiguous.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm.so")

MPM_OK, MPM_EINVAL, MPM_ENOMEM, MPM_EHIP, MPM_EDOMAIN, MPM_ENONFINITE, MPM_EINVERTED = 0, -1, -2, -3, -4, -5, -6
MPM_ERANGE = -7
MPM_ETOOBIG = -8
MPM_NOALLOC_MAX_PARTICLES = 65536
MPM_HOST, MPM_DEVICE = 0, 1
MPM_ACCUM_F32, MPM_ACCUM_FIXED = 0, 1
MPM_TOOL_NONE, MPM_TOOL_CAPSULE, MPM_TOOL_BOX, MPM_TOOL_PLANE = 0, 1, 2, 3
MPM_TOOL_SLICER, MPM_TOOL_SEGMENT, MPM_TOOL_ARC = 4, 5, 6
MPM_MAX_TOOLS = 8
MPM_SOLVER_MLS, MPM_SOLVER_PIC, MPM_SOLVER_PB = 0, 1, 2
MPM_REBIN_AUTO, MPM_REBIN_ADVANCE, MPM_REBIN_IN_PLACE = 0, 1, 2
MPM_KERNEL_KINDS = 5
KERNEL_NAMES = ("binning", "p2g", "g2p2g", "g2p", "grid")

STATUS_NAMES = {0: "MPM_OK", -1: "MPM_EINVAL", -2: "MPM_ENOMEM", -3: "MPM_EHIP", -4: "MPM_EDOMAIN",
                -5: "MPM_ENONFINITE", -6: "MPM_EINVERTED", -7: "MPM_ERANGE", -8: "MPM_ETOOBIG"}

EXPORTED = ("mpm_create", "mpm_destroy", "mpm_set_particles", "mpm_set_tool_sdf", "mpm_step",
            "mpm_read_state", "mpm_get_info", "mpm_last_error", "mpm_eval_stress", "mpm_profile",
            "mpm_profile_read", "mpm_read_tool_impulses", "mpm_set_tool_velocity_table", "mpm_rollout_forward",
            "mpm_rollout_backward", "mpm_create_batch", "mpm_set_batch_particles", "mpm_set_scene_tool",
            "mpm_set_scene_tool_velocity_table", "mpm_read_scene_tool_impulses", "mpm_get_launch_config",
            "mpm_set_launch_config", "mpm_autotune", "mpm_set_solver", "mpm_get_solver",
            "mpm_eval_stress_noalloc")


class mpm_params(ctypes.Structure):
    _fields_ = [("n_grid", ctypes.c_int32), ("dt", ctypes.c_float), ("gravity", ctypes.c_float * 3),
                ("wall_band", ctypes.c_int32), ("nu", ctypes.c_float), ("E_default", ctypes.c_float),
                ("accum_mode", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("resort_interval", ctypes.c_int32), ("max_particles", ctypes.c_int64)]


class mpm_tool(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("center", ctypes.c_double * 3), ("quat", ctypes.c_double * 4),
                ("size", ctypes.c_double * 3), ("lin_vel", ctypes.c_double * 3),
                ("ang_vel", ctypes.c_double * 3), ("mu", ctypes.c_float), ("drag", ctypes.c_float),
                ("margin", ctypes.c_float), ("push_out", ctypes.c_int32)]


class mpm_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_particles", "substeps", "resorts", "occupied_blocks", "active_blocks", "active_nodes",
        "n_inverted", "n_domain", "n_nonfinite", "n_fallback", "n_range")] + \
        [(n, ctypes.c_int32) for n in ("tile", "resort_interval", "accum_mode", "n_tools")] + \
        [("rollouts", ctypes.c_int64)]


class mpm_launch_config(ctypes.Structure):
    _fields_ = [("resort_interval", ctypes.c_int32), ("transfer_wgs", ctypes.c_int32),
                ("graph_chunk", ctypes.c_int32), ("rebin_mode", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("rebin_drift", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class mpm_kernel_times(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double * MPM_KERNEL_KINDS),
                ("launches", ctypes.c_int64 * MPM_KERNEL_KINDS)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                      "(run __graft_entry__.build() or python paper_2502_18437_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_h = ctypes.c_void_p
_lib.mpm_create.argtypes = [ctypes.POINTER(mpm_params), ctypes.c_uint64, ctypes.POINTER(_h)]
_lib.mpm_destroy.argtypes = [_h]
_lib.mpm_set_particles.argtypes = [_h, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_int32]
_lib.mpm_set_tool_sdf.argtypes = [_h, ctypes.c_int32, ctypes.POINTER(mpm_tool)]
_lib.mpm_step.argtypes = [_h, ctypes.c_int32]
_lib.mpm_read_state.argtypes = [_h, _vp, _vp, _vp, _vp, ctypes.c_int32]
_lib.mpm_get_info.argtypes = [_h, ctypes.POINTER(mpm_info)]
_lib.mpm_last_error.argtypes = [_h]
_lib.mpm_last_error.restype = ctypes.c_char_p
_lib.mpm_eval_stress.argtypes = [ctypes.c_int64, _vp, _vp, ctypes.c_float, _vp, ctypes.c_int32]
_lib.mpm_eval_stress_noalloc.argtypes = [ctypes.c_int64, _vp, _vp, ctypes.c_float, _vp, ctypes.c_int32]
_lib.mpm_profile.argtypes = [_h, ctypes.c_int32]
_lib.mpm_profile_read.argtypes = [_h, ctypes.POINTER(mpm_kernel_times)]
_lib.mpm_read_tool_impulses.argtypes = [_h, ctypes.POINTER(ctypes.c_double)]
_lib.mpm_set_tool_velocity_table.argtypes = [_h, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
_lib.mpm_rollout_forward.argtypes = [_h, ctypes.c_int32, ctypes.c_int32, _vp]
_lib.mpm_create_batch.argtypes = [ctypes.POINTER(mpm_params), ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(_h)]
_lib.mpm_set_batch_particles.argtypes = [_h, ctypes.POINTER(ctypes.c_int64), _vp, _vp, _vp, _vp, _vp, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_int32]
_lib.mpm_set_scene_tool.argtypes = [_h, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(mpm_tool)]
_lib.mpm_set_scene_tool_velocity_table.argtypes = [_h, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                                   ctypes.POINTER(ctypes.c_double)]
_lib.mpm_read_scene_tool_impulses.argtypes = [_h, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
_lib.mpm_get_launch_config.argtypes = [_h, ctypes.POINTER(mpm_launch_config)]
_lib.mpm_set_launch_config.argtypes = [_h, ctypes.POINTER(mpm_launch_config)]
_lib.mpm_autotune.argtypes = [_h, ctypes.c_int32, ctypes.POINTER(mpm_launch_config)]
_lib.mpm_set_solver.argtypes = [_h, ctypes.c_int32, ctypes.c_int32, ctypes.c_float]
_lib.mpm_get_solver.argtypes = [_h, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_float)]
_lib.mpm_rollout_backward.argtypes = [_h, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp, _vp, _vp,
                                      _vp]

# C names, re-exported
mpm_create = _lib.mpm_create
mpm_destroy = _lib.mpm_destroy
mpm_set_particles = _lib.mpm_set_particles
mpm_set_tool_sdf = _lib.mpm_set_tool_sdf
mpm_step = _lib.mpm_step
mpm_read_state = _lib.mpm_read_state
mpm_get_info = _lib.mpm_get_info
mpm_last_error = _lib.mpm_last_error
mpm_eval_stress = _lib.mpm_eval_stress
mpm_eval_stress_noalloc = _lib.mpm_eval_stress_noalloc
mpm_profile = _lib.mpm_profile
mpm_profile_read = _lib.mpm_profile_read
mpm_read_tool_impulses = _lib.mpm_read_tool_impulses
mpm_set_tool_velocity_table = _lib.mpm_set_tool_velocity_table
mpm_rollout_forward = _lib.mpm_rollout_forward
mpm_rollout_backward = _lib.mpm_rollout_backward
mpm_create_batch = _lib.mpm_create_batch
mpm_set_batch_particles = _lib.mpm_set_batch_particles
mpm_set_scene_tool = _lib.mpm_set_scene_tool
mpm_set_scene_tool_velocity_table = _lib.mpm_set_scene_tool_velocity_table
mpm_read_scene_tool_impulses = _lib.mpm_read_scene_tool_impulses
mpm_get_launch_config = _lib.mpm_get_launch_config
mpm_set_launch_config = _lib.mpm_set_launch_config
mpm_autotune = _lib.mpm_autotune


class MPMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _arg(a, shape_tail, n):
    """(pointer, where, keepalive) of one float32 array argument."""
    if a is None:
        return None, None, None
    if _is_torch(a):
        if not a.is_cuda:
            a = a.numpy()
        else:
            if a.dtype != __import__("torch").float32 or not a.is_contiguous():
                raise ValueError("device arrays must be contiguous float32 tensors")
            if a.numel() != n * int(np.prod(shape_tail)):
                raise ValueError(f"expected {n} x {shape_tail}, got {tuple(a.shape)}")
            return a.data_ptr(), MPM_DEVICE, a
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != n * int(np.prod(shape_tail)):
        raise ValueError(f"expected {n} x {shape_tail}, got {a.shape}")
    return a.ctypes.data, MPM_HOST, a


def _device_f32(a, n):
    """A contiguous float32 CUDA tensor of n elements holding `a` (host
    arrays are copied to the device)."""
    import torch
    t = a if _is_torch(a) else torch.as_tensor(np.asarray(a, dtype=np.float32))
    if not t.is_cuda:
        t = t.to(torch.device("cuda", torch.cuda.current_device()))
    t = t.detach().to(torch.float32).contiguous()
    if t.numel() != n:
        raise ValueError(f"expected {n} elements, got {tuple(t.shape)}")
    return t


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return 0


class Simulation:
    """One scene (mpm_handle)."""

    def __init__(self, n_grid, dt, gravity=(0.0, -9.8, 0.0), wall_band=3, nu=0.3, E_default=5e3,
                 accum_mode=MPM_ACCUM_F32, tile=0, resort_interval=0, max_particles=0, stream=None, n_scenes=1):
        p = mpm_params(int(n_grid), float(dt), (ctypes.c_float * 3)(*gravity), int(wall_band), float(nu),
                       float(E_default), int(accum_mode), int(tile), int(resort_interval), int(max_particles))
        h = _h()
        s = _current_stream() if stream is None else int(stream)
        self.n_scenes = int(n_scenes)
        if self.n_scenes == 1:
            rc = _lib.mpm_create(ctypes.byref(p), ctypes.c_uint64(s), ctypes.byref(h))
        else:
            rc = _lib.mpm_create_batch(ctypes.byref(p), self.n_scenes, ctypes.c_uint64(s), ctypes.byref(h))
        if rc != MPM_OK:
            raise MPMError(rc, _lib.mpm_last_error(None).decode())
        self.h = h
        self.n_grid = int(n_grid)
        self.N = 0

    # -- lifecycle
    def close(self):
        if getattr(self, "h", None):
            rc = _lib.mpm_destroy(self.h)
            self.h = None
            return rc
        return MPM_OK

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != MPM_OK and rc not in allow:
            raise MPMError(rc, _lib.mpm_last_error(self.h).decode())
        return rc

    # -- calls
    def set_particles(self, x, v=None, C=None, F=None, E=None, mass=1.0, vol0=1.0):
        n = int(x.shape[0])
        args = [_arg(x, (3,), n), _arg(v, (3,), n), _arg(C, (3, 3), n), _arg(F, (3, 3), n), _arg(E, (), n)]
        wheres = {w for _, w, _ in args if w is not None}
        if len(wheres) > 1:
            raise ValueError("all arrays must be host or all device")
        where = wheres.pop() if wheres else MPM_HOST
        ptrs = [p for p, _, _ in args]
        self._keep = [k for _, _, k in args]
        rc = _lib.mpm_set_particles(self.h, n, *ptrs, float(mass), float(vol0), where)
        self._check(rc)
        self.N = n

    def set_batch_particles(self, counts, x, v=None, C=None, F=None, E=None, mass=1.0, vol0=1.0):
        """All scenes' particles, concatenated scene after scene."""
        counts = np.ascontiguousarray(np.asarray(counts, dtype=np.int64))
        n = int(counts.sum())
        args = [_arg(x, (3,), n), _arg(v, (3,), n), _arg(C, (3, 3), n), _arg(F, (3, 3), n), _arg(E, (), n)]
        wheres = {w for _, w, _ in args if w is not None}
        if len(wheres) > 1:
            raise ValueError("all arrays must be host or all device")
        where = wheres.pop() if wheres else MPM_HOST
        self._keep = [k for _, _, k in args] + [counts]
        rc = _lib.mpm_set_batch_particles(self.h, counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          *[p for p, _, _ in args], float(mass), float(vol0), where)
        self._check(rc)
        self.N = n
        self.counts = counts.copy()

    def set_tool(self, tool_id, tool_type, center=(0, 0, 0), quat=(1, 0, 0, 0), size=(0, 0, 0),
                 lin_vel=(0, 0, 0), ang_vel=(0, 0, 0), mu=0.0, drag=1.0, margin=0.0, push_out=False, scene=0):
        t = mpm_tool(int(tool_type), (ctypes.c_double * 3)(*center), (ctypes.c_double * 4)(*quat),
                     (ctypes.c_double * 3)(*size), (ctypes.c_double * 3)(*lin_vel),
                     (ctypes.c_double * 3)(*ang_vel), float(mu), float(drag), float(margin), int(bool(push_out)))
        if scene == 0:
            self._check(_lib.mpm_set_tool_sdf(self.h, int(tool_id), ctypes.byref(t)))
        else:
            self._check(_lib.mpm_set_scene_tool(self.h, int(scene), int(tool_id), ctypes.byref(t)))

    def step(self, n):
        self._check(_lib.mpm_step(self.h, int(n)))

    def read_state(self, out=None, allow_errors=False):
        """Blocking read. Returns (dict of arrays, status). Without `out`,
        host NumPy arrays are returned; `out` may hold torch CUDA tensors
        (keys x, v, C, F) to read into device memory."""
        n = self.N
        if out is None:
            out = {"x": np.empty((n, 3), np.float32), "v": np.empty((n, 3), np.float32),
                   "C": np.empty((n, 3, 3), np.float32), "F": np.empty((n, 3, 3), np.float32)}
        args = {k: _arg(out.get(k), (3,) if k in "xv" else (3, 3), n) for k in ("x", "v", "C", "F")}
        wheres = {w for _, w, _ in args.values() if w is not None}
        where = wheres.pop() if wheres else MPM_HOST
        rc = _lib.mpm_read_state(self.h, *[args[k][0] for k in ("x", "v", "C", "F")], where)
        if rc in (MPM_EDOMAIN, MPM_ENONFINITE, MPM_EINVERTED, MPM_ERANGE) and allow_errors:
            return out, rc
        self._check(rc)
        return out, rc

    def info(self):
        i = mpm_info()
        self._check(_lib.mpm_get_info(self.h, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in mpm_info._fields_}

    def tool_impulses(self, scene=0):
        """(MPM_MAX_TOOLS + 1, 3) impulses on each tool of a scene (last row:
        walls) over the most recent step() call."""
        out = np.zeros((MPM_MAX_TOOLS + 1, 3), np.float64)
        self._check(_lib.mpm_read_scene_tool_impulses(self.h, int(scene),
                                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_tool_velocity_table(self, tool_id, table, scene=0):
        """Per-substep linear velocities (T x 3) of a tool from the current
        substep on (re-anchored at its current pose)."""
        t = np.ascontiguousarray(np.asarray(table, dtype=np.float64).reshape(-1, 3))
        self._check(_lib.mpm_set_scene_tool_velocity_table(self.h, int(scene), int(tool_id), t.shape[0],
                                                            t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def rollout_forward(self, n_substeps, checkpoint_every=20, theta=None):
        """Run and record a differentiable rollout; theta (N,) sets E = exp(theta)."""
        keep = None
        ptr = None
        if theta is not None:
            keep = _device_f32(theta, self.N)
            ptr = keep.data_ptr()
        self._check(_lib.mpm_rollout_forward(self.h, int(n_substeps), int(checkpoint_every), ptr))
        self._keep_theta = keep
        self._rollout_T = int(n_substeps)

    def rollout_backward(self, xb=None, vb=None, Cb=None, Fb=None, want_vel=True, want_state=True):
        """Gradient through the recorded rollout for the cotangents of the
        final x, v, C, F (None = 0). Returns a dict: theta (N,) and, when
        asked for, vel (MPM_MAX_TOOLS, T, 3) host float64 and x0, v0, C0, F0
        (device tensors, cotangents of the starting state)."""
        import torch
        n = self.N
        seeds = [None if a is None else _device_f32(a, n * k) for a, k in ((xb, 3), (vb, 3), (Cb, 9), (Fb, 9))]
        dev = torch.device("cuda", torch.cuda.current_device())
        theta_bar = torch.empty(n, dtype=torch.float32, device=dev)
        T = getattr(self, "_rollout_T", 0)
        vel = np.zeros((MPM_MAX_TOOLS, T, 3), np.float64) if want_vel else None
        outs = [torch.empty(shape, dtype=torch.float32, device=dev) for shape in ((n, 3), (n, 3), (n, 3, 3), (n, 3, 3))] \
            if want_state else [None] * 4
        rc = _lib.mpm_rollout_backward(
            self.h, *[None if a is None else a.data_ptr() for a in seeds], theta_bar.data_ptr(),
            None if vel is None else vel.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            *[None if a is None else a.data_ptr() for a in outs])
        self._check(rc)
        r = {"theta": theta_bar, "vel": vel}
        for k, a in zip(("x0", "v0", "C0", "F0"), outs):
            r[k] = a
        return r

    def set_solver(self, solver, iterations=10, beta=0.5):
        """MPM_SOLVER_MLS (default), MPM_SOLVER_PIC (standard MPM, Neo-Hookean)
        or MPM_SOLVER_PB (PB-MPM with `iterations` passes per step and the
        co-rotational constraint weight `beta`)."""
        self._check(_lib.mpm_set_solver(self.h, int(solver), int(iterations), float(beta)))

    def solver(self):
        k, it, beta = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        self._check(_lib.mpm_get_solver(self.h, ctypes.byref(k), ctypes.byref(it), ctypes.byref(beta)))
        return {"solver": k.value, "iterations": it.value, "beta": beta.value}

    def launch_config(self):
        c = mpm_launch_config()
        self._check(_lib.mpm_get_launch_config(self.h, ctypes.byref(c)))
        return c.as_dict()

    def set_launch_config(self, resort_interval=None, transfer_wgs=None, graph_chunk=None, rebin_mode=None,
                          tile=None, rebin_drift=None):
        """Replace the given fields of the launch configuration (MPM_REBIN_*
        for rebin_mode; tile 4 or 8 cells; rebin_drift in particles per
        million per substep, 0 = off); the others keep their values."""
        cur = self.launch_config()
        given = {"resort_interval": resort_interval, "transfer_wgs": transfer_wgs, "graph_chunk": graph_chunk,
                 "rebin_mode": rebin_mode, "tile": tile, "rebin_drift": rebin_drift}
        c = mpm_launch_config(**{k: int(v if v is not None else cur[k]) for k, v in given.items()})
        self._check(_lib.mpm_set_launch_config(self.h, ctypes.byref(c)))

    def autotune(self, trial_substeps=32):
        """Time the candidate launch configurations on the current scene and
        keep the fastest, unless the configuration in use is within 5% of it
        (then that one stays); returns the configuration kept."""
        c = mpm_launch_config()
        self._check(_lib.mpm_autotune(self.h, int(trial_substeps), ctypes.byref(c)))
        return c.as_dict()

    def profile(self, enable=True, every=1):
        """Per-kernel event timing on (the transfer and grid kernels of every
        `every`-th substep) or off."""
        self._check(_lib.mpm_profile(self.h, max(1, int(every)) if enable else 0))

    def profile_read(self):
        t = mpm_kernel_times()
        self._check(_lib.mpm_profile_read(self.h, ctypes.byref(t)))
        return {KERNEL_NAMES[k]: (t.total_ms[k], t.launches[k]) for k in range(MPM_KERNEL_KINDS)}


def eval_stress(F, E, nu):
    """Kirchhoff stress of (n, 3, 3) deformation gradients on the GPU."""
    n = int(F.shape[0])
    pF, w1, kF = _arg(F, (3, 3), n)
    pE, w2, kE = _arg(E, (), n)
    if w1 != w2:
        raise ValueError("F and E must both be host or both be device arrays")
    if w1 == MPM_DEVICE:
        import torch
        tau = torch.empty((n, 3, 3), dtype=torch.float32, device=F.device)
        ptr = tau.data_ptr()
    else:
        tau = np.empty((n, 3, 3), np.float32)
        ptr = tau.ctypes.data
    rc = _lib.mpm_eval_stress(n, pF, pE, float(nu), ptr, w1)
    if rc != MPM_OK:
        raise MPMError(rc, "mpm_eval_stress")
    return tau


def simulation_from_scene(scene, **kw):
    """Create a Simulation holding a scenes.Scene (particles and tools).
    Keywords are Simulation parameters (tile among them) or
    launch-configuration fields (transfer_wgs, graph_chunk, rebin_mode,
    rebin_drift)."""
    launch = {k: kw.pop(k) for k in ("transfer_wgs", "graph_chunk", "rebin_mode", "rebin_drift") if k in kw}
    params = dict(n_grid=scene.n_grid, dt=scene.dt, gravity=scene.gravity, wall_band=scene.wall_band,
                  nu=scene.nu, E_default=scene.E_default, max_particles=max(1, scene.N))
    params.update(kw)
    sim = Simulation(**params)
    if launch:
        sim.set_launch_config(**launch)
    sim.set_particles(scene.x, scene.v, scene.C, scene.F, scene.E, scene.mass, scene.vol0)
    for k, t in enumerate(scene.tools):
        sim.set_tool(k, t.type, **t.kwargs())
    for k, tab in scene.vel_tables.items():
        sim.set_tool_velocity_table(k, tab)
    if scene.solver is not None:
        sim.set_solver(*scene.solver)
    return sim


def rollout(sim, n_substeps, theta, vel_table=None, tool_id=0, checkpoint_every=20):
    """Differentiable rollout of `sim` (torch.autograd): returns the state
    (x, v, C, F) after n_substeps as CUDA tensors. Gradients flow to theta
    (E_p = exp(theta_p), shape (N,)) and to vel_table (n_substeps x 3 linear
    velocities of tool `tool_id`, one row per substep), through the
    hand-written adjoint kernels of the library."""
    return _rollout_fn()(theta, vel_table, sim, int(n_substeps), int(tool_id), int(checkpoint_every))


_ROLLOUT = None


def _rollout_fn():
    global _ROLLOUT
    if _ROLLOUT is not None:
        return _ROLLOUT.apply
    import torch

    class Rollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, vel_table, sim, T, tool_id, K):
            if vel_table is not None:
                if tuple(vel_table.shape) != (T, 3):
                    raise ValueError("vel_table must be n_substeps x 3")
                sim.set_tool_velocity_table(tool_id, vel_table.detach().cpu().double().numpy())
            sim.rollout_forward(T, K, theta=theta)
            n = sim.N
            dev = theta.device
            out = {"x": torch.empty((n, 3), dtype=torch.float32, device=dev),
                   "v": torch.empty((n, 3), dtype=torch.float32, device=dev),
                   "C": torch.empty((n, 3, 3), dtype=torch.float32, device=dev),
                   "F": torch.empty((n, 3, 3), dtype=torch.float32, device=dev)}
            sim.read_state(out)
            # The library differentiates only its latest rollout: remember
            # which one this node recorded.
            ctx.generation = sim.info()["rollouts"]
            ctx.sim, ctx.tool_id = sim, tool_id
            ctx.table = None if vel_table is None else (vel_table.dtype, vel_table.device)
            ctx.theta_dtype = theta.dtype
            return out["x"], out["v"], out["C"], out["F"]

        @staticmethod
        def backward(ctx, gx, gv, gC, gF):
            if ctx.sim.info()["rollouts"] != ctx.generation:
                raise RuntimeError("mpm.rollout: the simulation recorded another rollout after this one; "
                                   "its backward would use the later rollout's checkpoints (call backward "
                                   "before the next rollout on the same Simulation)")
            g = ctx.sim.rollout_backward(gx, gv, gC, gF, want_vel=ctx.table is not None, want_state=False)
            tb = None
            if ctx.table is not None:
                tb = torch.from_numpy(g["vel"][ctx.tool_id].copy()).to(dtype=ctx.table[0], device=ctx.table[1])
            return g["theta"].to(ctx.theta_dtype), tb, None, None, None, None

    _ROLLOUT = Rollout
    return Rollout.apply

"""FP64 CPU oracle of the explicit MLS-MPM substep (CRESSim-MPM, Sec. III-B,
Algorithm 1, with the contact law of Sec. IV-A).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library. It shares no code with
the HIP path. The arithmetic lives in ``mpm_oracle.cpp`` (plain FP64 loops);
this module only marshals arguments through ctypes.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm_oracle.so")

TOOL_NONE, TOOL_CAPSULE, TOOL_BOX, TOOL_PLANE, TOOL_SLICER, TOOL_SEGMENT, TOOL_ARC = 0, 1, 2, 3, 4, 5, 6
SOLVER_MLS, SOLVER_PIC, SOLVER_PB = 0, 1, 2
ST_OK, ST_EINVAL, ST_ENOMEM, ST_EDOMAIN, ST_ENONFINITE, ST_EINVERTED = 0, -1, -2, -4, -5, -6

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.c_void_p
        L.oracle_create.restype = ctypes.c_void_p
        L.oracle_create.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double]
        L.oracle_destroy.argtypes = [ctypes.c_void_p]
        L.oracle_set_particles.argtypes = [ctypes.c_void_p, ctypes.c_longlong, fp, fp, fp, fp, fp,
                                           ctypes.c_double, ctypes.c_double]
        L.oracle_set_tool.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp,
                                      dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_set_tool_push.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.oracle_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.oracle_read.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.oracle_last_grid.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.oracle_impulses.argtypes = [ctypes.c_void_p, dp]
        L.oracle_counters.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong)]
        L.oracle_set_tie_band.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        L.oracle_read_ties.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong), dp]
        L.oracle_weights.argtypes = [ctypes.c_double, dp]
        L.oracle_polar.restype = ctypes.c_double
        L.oracle_polar.argtypes = [dp, dp]
        L.oracle_kirchhoff.restype = ctypes.c_double
        L.oracle_kirchhoff.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_energy.restype = ctypes.c_double
        L.oracle_energy.argtypes = [dp, ctypes.c_double, ctypes.c_double]
        L.oracle_sdf.restype = ctypes.c_double
        L.oracle_sdf.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
        L.oracle_contact.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_node_contact.restype = ctypes.c_int
        L.oracle_node_contact.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, dp, dp]
        L.oracle_set_state_f64.argtypes = [ctypes.c_void_p, ctypes.c_longlong, dp, dp, dp, dp, dp,
                                           ctypes.c_double, ctypes.c_double]
        L.oracle_set_velocity_table.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, dp]
        L.oracle_rollout_adjoint.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp,
                                             dp, dp]
        L.oracle_polar_adjoint.argtypes = [dp, dp, dp]
        L.oracle_set_solver.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.oracle_neo_hookean.restype = ctypes.c_double
        L.oracle_neo_hookean.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_pb_constraint.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_kirchhoff_adjoint.restype = ctypes.c_double
        L.oracle_kirchhoff_adjoint.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.oracle_frame_contact.restype = ctypes.c_int
        L.oracle_frame_contact.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, dp, dp]
        L.oracle_contact_adjoint.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, dp, dp, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f32(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- unit calls
def weights(f):
    o, p = _d(np.zeros(3))
    lib().oracle_weights(float(f), p)
    return o


def polar(F):
    F, pF = _d(np.asarray(F).reshape(9))
    R, pR = _d(np.zeros(9))
    J = lib().oracle_polar(pF, pR)
    return R.reshape(3, 3), J


def kirchhoff(F, E, nu):
    F, pF = _d(np.asarray(F).reshape(9))
    t, pt = _d(np.zeros(9))
    J = lib().oracle_kirchhoff(pF, float(E), float(nu), pt)
    return t.reshape(3, 3), J


def energy(F, E, nu):
    F, pF = _d(np.asarray(F).reshape(9))
    return lib().oracle_energy(pF, float(E), float(nu))


def sdf(tool_type, center, quat, size, p):
    c, pc = _d(center)
    q, pq = _d(quat)
    s, ps = _d(size)
    x, px = _d(p)
    g, pg = _d(np.zeros(3))
    phi = lib().oracle_sdf(int(tool_type), pc, pq, ps, px, pg)
    return phi, g.copy()


def contact(n, u, mu, drag):
    n, pn = _d(n)
    u, pu = _d(u)
    o, po = _d(np.zeros(3))
    lib().oracle_contact(pn, pu, float(mu), float(drag), po)
    return o.copy()


def node_contact(tool_type, center, quat, size, lin_vel, ang_vel, mu, drag, margin, xI, vI):
    """(velocity after contact, in_contact) of one node and one tool."""
    args = [_d(a) for a in (center, quat, size, lin_vel, ang_vel)]
    x, px = _d(xI)
    v, pv = _d(np.array(vI, dtype=np.float64))
    hit = lib().oracle_node_contact(int(tool_type), *[p for _, p in args], float(mu), float(drag),
                                    float(margin), px, pv)
    return v.copy(), bool(hit)


def neo_hookean(F, E, nu):
    """(Kirchhoff stress mu (F F^T - I) + lambda ln J I, J) of standard MPM."""
    F, pF = _d(np.asarray(F).reshape(9))
    t, pt = _d(np.zeros(9))
    J = lib().oracle_neo_hookean(pF, float(E), float(nu), pt)
    return t.reshape(3, 3), J


def pb_constraint(F, C, dt, beta):
    """C after the PB-MPM co-rotational constraint on one particle."""
    F, pF = _d(np.asarray(F).reshape(9))
    C, pC = _d(np.asarray(C).reshape(9))
    o, po = _d(np.zeros(9))
    lib().oracle_pb_constraint(pF, pC, float(dt), float(beta), po)
    return o.reshape(3, 3)


def polar_adjoint(F, Rb):
    """Cotangent of F for a cotangent Rb of its rotation factor."""
    F, pF = _d(np.asarray(F).reshape(9))
    Rb, pRb = _d(np.asarray(Rb).reshape(9))
    o, po = _d(np.zeros(9))
    lib().oracle_polar_adjoint(pF, pRb, po)
    return o.reshape(3, 3)


def kirchhoff_adjoint(F, E, nu, taub):
    """(cotangent of F, d/d log E) for a cotangent taub of the Kirchhoff stress."""
    F, pF = _d(np.asarray(F).reshape(9))
    t, pt = _d(np.asarray(taub).reshape(9))
    o, po = _d(np.zeros(9))
    th = lib().oracle_kirchhoff_adjoint(pF, float(E), float(nu), pt, po)
    return o.reshape(3, 3), th


def frame_contact(tool_type, center, quat, size, lin_vel, ang_vel, mu, drag, margin, xI, vI):
    """(velocity after contact, law code) through the differentiable contact frame."""
    args = [_d(a) for a in (center, quat, size, lin_vel, ang_vel)]
    x, px = _d(xI)
    v, pv = _d(np.array(vI, dtype=np.float64))
    law = lib().oracle_frame_contact(int(tool_type), *[p for _, p in args], float(mu), float(drag),
                                     float(margin), px, pv)
    return v.copy(), int(law)


def contact_adjoint(tool_type, center, quat, size, lin_vel, ang_vel, mu, drag, margin, xI, vin, vbar):
    """Cotangents (of the input velocity, of the tool centre, of its linear
    velocity) of one node's contact map for a cotangent vbar of its output."""
    args = [_d(a) for a in (center, quat, size, lin_vel, ang_vel)]
    x, px = _d(xI)
    vi, pvi = _d(vin)
    vb, pvb = _d(np.array(vbar, dtype=np.float64))
    cb, pcb = _d(np.zeros(3))
    lb, plb = _d(np.zeros(3))
    lib().oracle_contact_adjoint(int(tool_type), *[p for _, p in args], float(mu), float(drag), float(margin),
                                 px, pvi, pvb, pcb, plb)
    return vb.copy(), cb.copy(), lb.copy()


# ---------------------------------------------------------------- scene object
class Oracle:
    """One scene on the FP64 oracle. Inputs are the FP32 arrays the GPU
    library receives; they are widened to FP64 inside."""

    def __init__(self, n_grid, dt, gravity=(0.0, -9.8, 0.0), wall_band=3, nu=0.3, E_default=5e3):
        g, pg = _d(gravity)
        self.n = int(n_grid)
        self.h = lib().oracle_create(self.n, float(dt), pg, int(wall_band), float(nu), float(E_default))
        if not self.h:
            raise ValueError("oracle_create rejected its arguments")
        self.N = 0

    def close(self):
        if self.h:
            lib().oracle_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_particles(self, x, v=None, C=None, F=None, E=None, mass=1.0, vol0=1.0):
        x, px = _f32(x)
        keep = [x]
        ptrs = []
        for a in (v, C, F, E):
            arr, p = _f32(a)
            keep.append(arr)
            ptrs.append(p)
        self.N = x.shape[0]
        st = lib().oracle_set_particles(self.h, self.N, px, *ptrs, float(mass), float(vol0))
        if st != 0:
            raise ValueError(f"oracle_set_particles: status {st}")

    def set_state_f64(self, x, v=None, C=None, F=None, E=None, mass=1.0, vol0=1.0):
        """FP64 state, for finite-difference checks."""
        x, px = _d(np.asarray(x).reshape(-1, 3))
        keep, ptrs = [x], []
        for a in (v, C, F, E):
            if a is None:
                ptrs.append(None)
            else:
                arr, p = _d(np.asarray(a).reshape(-1))
                keep.append(arr)
                ptrs.append(p)
        self.N = x.shape[0]
        st = lib().oracle_set_state_f64(self.h, self.N, px, *ptrs, float(mass), float(vol0))
        if st != 0:
            raise ValueError(f"oracle_set_state_f64: status {st}")

    def set_solver(self, kind, iterations=10, beta=0.5):
        """0 MLS-MPM, 1 standard MPM (PIC, Neo-Hookean), 2 PB-MPM."""
        st = lib().oracle_set_solver(self.h, int(kind), int(iterations), float(beta))
        if st != 0:
            raise ValueError(f"oracle_set_solver: status {st}")

    def set_velocity_table(self, tool_id, table):
        """Per-substep linear velocities (T x 3) of a tool from now on."""
        t, pt = _d(np.asarray(table, dtype=np.float64).reshape(-1, 3))
        st = lib().oracle_set_velocity_table(self.h, int(tool_id), t.shape[0], pt)
        if st != 0:
            raise ValueError(f"oracle_set_velocity_table: status {st}")

    def rollout_adjoint(self, T, xb=None, vb=None, Cb=None, Fb=None):
        """Advance T substeps and return the reverse-mode gradient for the
        seeds (cotangents of the final x, v, C, F): a dict with theta
        (d/d log E per particle), vel (8 x T x 3, per tool and substep
        linear velocity), x0, v0, C0, F0 (cotangent of the starting state)
        and status."""
        N = self.N
        seeds = []
        keep = []
        for a in (xb, vb, Cb, Fb):
            if a is None:
                seeds.append(None)
            else:
                arr, p = _d(np.asarray(a).reshape(-1))
                keep.append(arr)
                seeds.append(p)
        th, pth = _d(np.zeros(N))
        vel, pvel = _d(np.zeros((8, int(T), 3)))
        outs = [_d(np.zeros(shape)) for shape in ((N, 3), (N, 3), (N, 3, 3), (N, 3, 3))]
        st = lib().oracle_rollout_adjoint(self.h, int(T), *seeds, pth, pvel, *[p for _, p in outs])
        r = {"theta": th, "vel": vel, "status": st}
        for k, (arr, _) in zip(("x0", "v0", "C0", "F0"), outs):
            r[k] = arr
        return r

    def set_tool(self, tool_id, tool_type, center=(0, 0, 0), quat=(1, 0, 0, 0), size=(0, 0, 0),
                 lin_vel=(0, 0, 0), ang_vel=(0, 0, 0), mu=0.0, drag=1.0, margin=0.0, push_out=False):
        arrs = [_d(a) for a in (center, quat, size, lin_vel, ang_vel)]
        st = lib().oracle_set_tool(self.h, int(tool_id), int(tool_type), *[p for _, p in arrs],
                                   float(mu), float(drag), float(margin))
        if st == 0:
            st = lib().oracle_set_tool_push(self.h, int(tool_id), int(bool(push_out)))
        if st != 0:
            raise ValueError(f"oracle_set_tool: status {st}")

    def step(self, n):
        return lib().oracle_step(self.h, int(n))

    def read(self):
        N = self.N
        x, px = _d(np.zeros((N, 3)))
        v, pv = _d(np.zeros((N, 3)))
        C, pC = _d(np.zeros((N, 3, 3)))
        F, pF = _d(np.zeros((N, 3, 3)))
        st = lib().oracle_read(self.h, px, pv, pC, pF)
        return {"x": x, "v": v, "C": C, "F": F, "status": st}

    def last_grid(self):
        n = self.n
        m, pm = _d(np.zeros((n, n, n)))
        p, pp = _d(np.zeros((n, n, n, 3)))
        v, pv = _d(np.zeros((n, n, n, 3)))
        lib().oracle_last_grid(self.h, pm, pp, pv)
        return m, p, v

    def impulses(self):
        o, po = _d(np.zeros((9, 3)))
        lib().oracle_impulses(self.h, po)
        return o

    def set_tie_band(self, eta, policy=0):
        """Record contact decisions within eta (m) of their threshold (ties
        that rounding decides) and decide them by policy: 0 as computed, +1 in
        contact, -1 not in contact; eta < 0 turns tracking off. MLS-MPM."""
        assert lib().oracle_set_tie_band(self.h, float(eta), int(policy)) == 0

    def ties(self):
        """(taint, n_tie, max_jump): the particles whose state depends on a
        recorded tie decision (bool, N), the number of tie decisions and the
        largest velocity jump (m/s) one of them could make at its node."""
        t = np.zeros(self.N, dtype=np.uint8)
        n = ctypes.c_longlong(0)
        j, pj = _d(np.zeros(1))
        lib().oracle_read_ties(self.h, t.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n), pj)
        return t.astype(bool), int(n.value), float(j[0])

    def counters(self):
        o = np.zeros(3, dtype=np.int64)
        lib().oracle_counters(self.h, o.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
        return {"inverted": int(o[0]), "domain": int(o[1]), "nonfinite": int(o[2])}

"""NumPy brute-force twin of the FP64 oracle (test infrastructure only).

A second, independent formulation of the same explicit MLS-MPM substep
(CRESSim-MPM Sec. III-A/III-B, Algorithm 1; contact of Sec. IV-A), for tiny
inputs only:

* The transfer weights form a dense matrix W[p, I] built from the quadratic
  B-spline kernel evaluated at every grid node (no base-node stencil), so
  P2G is W^T applied to particle quantities and G2P is W applied to grid
  quantities.
* The MLS momentum term is regrouped as sum_p W A_p x_I - W A_p x_p.
* The polar rotation comes from LAPACK's SVD (numpy.linalg.svd) with the
  sign fix that keeps it a rotation.

Readings of the paper are the ones the C++ oracle states in its header.
"""
import numpy as np

TOOL_NONE, TOOL_CAPSULE, TOOL_BOX, TOOL_PLANE, TOOL_SLICER, TOOL_SEGMENT, TOOL_ARC = 0, 1, 2, 3, 4, 5, 6
SOLVER_MLS, SOLVER_PIC, SOLVER_PB = 0, 1, 2


def kernel(r):
    """Quadratic B-spline N(r) with support |r| < 3/2 (Sec. III-A)."""
    a = np.abs(r)
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def dkernel(r):
    """Derivative of the quadratic B-spline kernel."""
    a = np.abs(r)
    return np.where(a < 0.5, -2.0 * r, np.where(a < 1.5, -(1.5 - a) * np.sign(r), 0.0))


def neo_hookean(F, E, nu):
    """Kirchhoff stress J sigma of eq. neo_hookean, batched."""
    mu = E / (2 * (1 + nu))
    la = E * nu / ((1 + nu) * (1 - 2 * nu))
    J = np.linalg.det(F)
    B = F @ np.swapaxes(F, -1, -2)
    lnJ = np.log(np.maximum(J, 1e-6))
    return mu[:, None, None] * (B - np.eye(3)) + (la * lnJ)[:, None, None] * np.eye(3)


def quat_matrix(q):
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def rotation_part(F):
    """Rotation R of the sign-fixed SVD F = U S V^T, batched over F[..., 3, 3]."""
    U, _, Vt = np.linalg.svd(F)
    R = U @ Vt
    flip = np.linalg.det(R) < 0
    if np.any(flip):
        U = U.copy()
        U[flip, :, 2] *= -1.0
        R = U @ Vt
    return R


def kirchhoff(F, E, nu):
    mu = E / (2 * (1 + nu))
    la = E * nu / ((1 + nu) * (1 - 2 * nu))
    R = rotation_part(F)
    J = np.linalg.det(F)
    tau = 2 * mu[:, None, None] * (F - R) @ np.swapaxes(F, -1, -2)
    tau = tau + (la * (J - 1) * J)[:, None, None] * np.eye(3)
    return tau


def sdf_nodes(tool, pts):
    """Signed distance and unit outward normal of one tool at points (M, 3)."""
    R = quat_matrix(tool["quat"])
    c = np.asarray(tool["center"], dtype=np.float64)
    size = np.asarray(tool["size"], dtype=np.float64)
    pl = (pts - c) @ R  # body coordinates R^T (p - c), row-vector form
    M = pts.shape[0]
    gl = np.zeros((M, 3))
    gl[:, 1] = 1.0
    t = tool["type"]
    if t == TOOL_CAPSULE:
        h, r = size[0], size[1]
        e = pl.copy()
        e[:, 0] = pl[:, 0] - np.clip(pl[:, 0], -h, h)
        L = np.linalg.norm(e, axis=1)
        phi = L - r
        nz = L > 0
        gl[nz] = e[nz] / L[nz, None]
    elif t == TOOL_BOX:
        q = np.abs(pl) - size
        o = np.maximum(q, 0.0)
        L = np.linalg.norm(o, axis=1)
        k = np.argmax(q, axis=1)  # first maximum: lowest axis wins ties
        qmax = q[np.arange(M), k]
        phi = L + np.minimum(qmax, 0.0)
        outside = L > 0
        sgn = np.where(pl < 0, -1.0, 1.0)
        gl[outside] = (sgn * o)[outside] / L[outside, None]
        ins = ~outside
        gi = np.zeros((M, 3))
        gi[np.arange(M), k] = sgn[np.arange(M), k]
        gl[ins] = gi[ins]
    elif t == TOOL_PLANE:
        phi = pl[:, 1].copy()
    else:
        raise ValueError(t)
    g = gl @ R.T
    g = g / np.linalg.norm(g, axis=1, keepdims=True)
    return phi, g


def _friction(u, un, tg_vec, tg_len, mu, drag):
    """Corrected relative velocity for approaching nodes: the kept tangential
    vector scaled by c_d max(1 + mu u_n / |t|, 0) (0 where |t| = 0)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        k = np.where(tg_len > 0, np.maximum(1.0 + mu * un / np.where(tg_len > 0, tg_len, 1.0), 0.0), 0.0)
    return drag * k[:, None] * tg_vec


def thin_tool_contact(tool, pts, vel):
    """Slicer, line segment and arc contact (Sec. IV-B/IV-C) on nodes
    (M, 3) with velocities (M, 3); returns (new velocities, hit mask)."""
    R = quat_matrix(tool["quat"])
    c = np.asarray(tool["center"], dtype=np.float64)
    size = np.asarray(tool["size"], dtype=np.float64)
    r = pts - c
    pl = r @ R
    M = pts.shape[0]
    vr = np.asarray(tool["lv"]) + np.cross(np.asarray(tool["av"]), r)
    u = vel - vr
    t = tool["type"]
    out = vel.copy()
    if t == TOOL_SLICER:
        hx, hy = size[0], size[1]
        qx = np.maximum(np.abs(pl[:, 0]) - hx, 0.0)
        qy = np.maximum(np.abs(pl[:, 1]) - hy, 0.0)
        d = np.sqrt(qx * qx + qy * qy + pl[:, 2] ** 2)
        hit = d < tool["margin"]
        spine = hit & (pl[:, 1] > hy)
        face = hit & ~spine
        nl = np.zeros((M, 3))
        nl[:, 2] = np.where(pl[:, 2] < 0, -1.0, 1.0)
        n = nl @ R.T
        un = np.einsum("ia,ia->i", n, u)
        tv = u - un[:, None] * n
        unew = _friction(u, un, tv, np.linalg.norm(tv, axis=1), tool["mu"], tool["drag"])
        app = face & (un < 0)
        out[app] = vr[app] + unew[app]
        out[spine] = vr[spine]
        return out, hit
    if t == TOOL_SEGMENT:
        h, thick = size[0], size[1]
        proj = np.zeros((M, 3))
        proj[:, 0] = np.clip(pl[:, 0], -h, h)
        tl = np.tile([1.0, 0.0, 0.0], (M, 1))
    elif t == TOOL_ARC:
        ra, ha, thick = size[0], size[1], size[2]
        ang = np.arctan2(pl[:, 1], pl[:, 0])
        outside = (ang > ha) | (ang < -ha)
        e0 = np.array([ra * np.cos(ha), ra * np.sin(ha)])
        e1 = np.array([ra * np.cos(-ha), ra * np.sin(-ha)])
        d0 = ((pl[:, :2] - e0) ** 2).sum(axis=1)
        d1 = ((pl[:, :2] - e1) ** 2).sum(axis=1)
        ang = np.where(outside, np.where(d1 < d0, -ha, ha), ang)
        proj = np.stack([ra * np.cos(ang), ra * np.sin(ang), np.zeros(M)], axis=1)
        tl = np.stack([-np.sin(ang), np.cos(ang), np.zeros(M)], axis=1)
    else:
        raise ValueError(t)
    e = pl - proj
    L = np.linalg.norm(e, axis=1)
    hit = L < thick
    nl = np.where(L[:, None] > 0, e / np.where(L > 0, L, 1.0)[:, None],
                  np.stack([-tl[:, 1], tl[:, 0], np.zeros(M)], axis=1))
    n = nl @ R.T
    tg = tl @ R.T
    un = np.einsum("ia,ia->i", n, u)
    ut = np.einsum("ia,ia->i", tg, u)
    unew = _friction(u, un, ut[:, None] * tg, np.abs(ut), tool["mu"], tool["drag"])
    app = hit & (un < 0)
    out[app] = vr[app] + unew[app]
    return out, hit


class Brute:
    def __init__(self, n_grid, dt, gravity=(0.0, -9.8, 0.0), wall_band=3, nu=0.3, E_default=5e3):
        self.n = int(n_grid)
        self.dx = 1.0 / self.n
        self.dt = float(dt)
        self.g = np.asarray(gravity, dtype=np.float64)
        self.band = int(wall_band)
        self.nu = float(nu)
        self.E_default = float(E_default)
        self.tools = {}
        self.substep = 0
        self.solver, self.pb_iterations, self.pb_beta = SOLVER_MLS, 10, 0.5
        idx = np.arange(self.n)
        I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
        self.node_idx = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
        self.xI = self.node_idx * self.dx

    def set_particles(self, x, v=None, C=None, F=None, E=None, mass=1.0, vol0=1.0):
        x = np.asarray(x, dtype=np.float32).astype(np.float64)
        N = x.shape[0]
        self.x = x
        self.v = np.zeros((N, 3)) if v is None else np.asarray(v, np.float32).astype(np.float64).reshape(N, 3)
        self.C = np.zeros((N, 3, 3)) if C is None else np.asarray(C, np.float32).astype(np.float64).reshape(N, 3, 3)
        self.F = np.tile(np.eye(3), (N, 1, 1)) if F is None else np.asarray(F, np.float32).astype(np.float64).reshape(N, 3, 3)
        self.E = np.full(N, self.E_default) if E is None else np.asarray(E, np.float32).astype(np.float64)
        self.mass = float(mass)
        self.vol0 = float(vol0)

    def set_tool(self, tool_id, tool_type, center=(0, 0, 0), quat=(1, 0, 0, 0), size=(0, 0, 0),
                 lin_vel=(0, 0, 0), ang_vel=(0, 0, 0), mu=0.0, drag=1.0, margin=0.0, push_out=False):
        if tool_type == TOOL_NONE:
            self.tools.pop(tool_id, None)
            return
        self.tools[tool_id] = dict(type=tool_type, center0=np.asarray(center, np.float64),
                                   quat=np.asarray(quat, np.float64), size=np.asarray(size, np.float64),
                                   lv=np.asarray(lin_vel, np.float64), av=np.asarray(ang_vel, np.float64),
                                   mu=float(mu), drag=float(drag), margin=float(margin),
                                   set_at=self.substep, push=bool(push_out))

    def set_solver(self, kind, iterations=10, beta=0.5):
        self.solver, self.pb_iterations, self.pb_beta = int(kind), int(iterations), float(beta)

    def weight_gradients(self, x):
        """dW[a][p, I]: derivative of node I's weight with respect to x_p[a]."""
        r = x / self.dx
        idx = np.arange(self.n)
        Wa = [kernel(r[:, a][:, None] - idx[None, :]) for a in range(3)]
        dWa = [dkernel(r[:, a][:, None] - idx[None, :]) / self.dx for a in range(3)]
        out = []
        for a in range(3):
            f = [dWa[b] if b == a else Wa[b] for b in range(3)]
            out.append(np.einsum("pi,pj,pk->pijk", f[0], f[1], f[2]).reshape(x.shape[0], -1))
        return out

    def weight_matrix(self, x):
        r = x / self.dx  # (N, 3)
        idx = np.arange(self.n)
        Wa = [kernel(r[:, a][:, None] - idx[None, :]) for a in range(3)]  # (N, n) each
        W = np.einsum("pi,pj,pk->pijk", Wa[0], Wa[1], Wa[2]).reshape(x.shape[0], -1)
        return W

    def step(self, nsub):
        for _ in range(nsub):
            if self.solver == SOLVER_PIC:
                self._substep_pic()
            elif self.solver == SOLVER_PB:
                self._step_pb()
            else:
                self._substep()
            self._push_out()
            self.substep += 1

    def _push_out(self):
        """Particles inside a solid tool whose push-out is on move to its
        surface, x - phi n where phi < 0; tools in id order, each where it is
        one substep later."""
        for q in sorted(self.tools):
            t = self.tools[q]
            if not t["push"] or t["type"] not in (TOOL_CAPSULE, TOOL_BOX, TOOL_PLANE):
                continue
            ahead = dict(t, center=t["center0"] + (self.substep + 1 - t["set_at"]) * self.dt * t["lv"])
            phi, n = sdf_nodes(ahead, self.x)
            inside = phi < 0.0
            self.x[inside] = self.x[inside] - phi[inside, None] * n[inside]

    def _p2g_affine(self, W, x, v, A):
        """m_I and sum_p W (m v + A (x_I - x_p)), regrouped."""
        m = W.T @ np.full(x.shape[0], self.mass)
        Ax = np.einsum("pab,pb->pa", A, x)
        p = W.T @ (self.mass * v - Ax)
        MA = np.einsum("pI,pab->Iab", W, A)
        return m, p + np.einsum("Iab,Ib->Ia", MA, self.xI)

    def _substep(self):
        dt, dx = self.dt, self.dx
        Minv = 4.0 / dx ** 2
        x, v, C, F = self.x, self.v, self.C, self.F
        W = self.weight_matrix(x)  # (N, nodes)
        tau = kirchhoff(F, self.E, self.nu)
        A = self.mass * C - dt * self.vol0 * Minv * tau  # (N, 3, 3)
        m, p = self._p2g_affine(W, x, v, A)
        vI = self._grid(m, p, gravity=True)
        # G2P
        vn = W @ vI
        B = np.einsum("pI,Ia,Ib->pab", W, vI, self.xI) - np.einsum("pa,pb->pab", vn, x)
        self.C = Minv * B
        self.F = (np.eye(3) + dt * self.C) @ F
        self.v = vn
        self.x = x + dt * vn

    def _substep_pic(self):
        """Standard MPM: PIC transfers, force -V0 tau grad N, L = sum v_I grad N^T."""
        dt = self.dt
        x, v, F = self.x, self.v, self.F
        W = self.weight_matrix(x)
        dW = self.weight_gradients(x)
        tau = neo_hookean(F, self.E, self.nu)
        m = W.T @ np.full(x.shape[0], self.mass)
        p = W.T @ (self.mass * v)
        for b in range(3):  # f_I[a] = -sum_p V0 tau[a, b] dN/dx_b
            p = p - dt * self.vol0 * (dW[b].T @ tau[:, :, b])
        vI = self._grid(m, p, gravity=True)
        vn = W @ vI
        L = np.stack([dW[b] @ vI for b in range(3)], axis=-1)  # L[p, a, b]
        self.C = L
        self.F = (np.eye(3) + dt * L) @ F
        self.v = vn
        self.x = x + dt * vn

    def _step_pb(self):
        """PB-MPM step: gravity once, `iterations` of (constraint, APIC P2G,
        grid without gravity, APIC G2P of v and C), then F and x."""
        dt, dx = self.dt, self.dx
        Minv = 4.0 / dx ** 2
        x, F = self.x, self.F
        W = self.weight_matrix(x)
        v = self.v + dt * self.g
        C = self.C
        Finv = np.linalg.inv(F)
        for it in range(self.pb_iterations):
            Fs = (np.eye(3) + dt * C) @ F
            R = rotation_part(Fs)
            J = np.linalg.det(Fs)
            T = self.pb_beta * R + (1.0 - self.pb_beta) * Fs / np.cbrt(J)[:, None, None]
            C = (T @ Finv - np.eye(3)) / dt
            m, p = self._p2g_affine(W, x, v, self.mass * C)
            vI = self._grid(m, p, gravity=False)
            v = W @ vI
            B = np.einsum("pI,Ia,Ib->pab", W, vI, self.xI) - np.einsum("pa,pb->pab", v, x)
            C = Minv * B
        self.C = C
        self.F = (np.eye(3) + dt * C) @ F
        self.v = v
        self.x = x + dt * v

    def _grid(self, m, p, gravity):
        dt = self.dt
        has = m > 0
        vI = np.zeros_like(p)
        vI[has] = p[has] / m[has, None] + (dt * self.g if gravity else 0.0)
        for tid in sorted(self.tools):
            t = self.tools[tid]
            c = t["center0"] + (self.substep - t["set_at"]) * dt * t["lv"]
            tt = dict(t, center=c)
            if t["type"] in (TOOL_SLICER, TOOL_SEGMENT, TOOL_ARC):
                vnew, hit = thin_tool_contact(tt, self.xI, vI)
                hit = hit & has
                vI[hit] = vnew[hit]
                continue
            phi, nrm = sdf_nodes(tt, self.xI)
            hit = has & (phi < t["margin"])
            r = self.xI - c
            vr = t["lv"] + np.cross(t["av"], r)
            u = vI - vr
            un = np.einsum("ia,ia->i", nrm, u)
            tg = u - un[:, None] * nrm
            s = np.linalg.norm(tg, axis=1)
            with np.errstate(divide="ignore", invalid="ignore"):
                k = np.where(s > 0, np.maximum(1.0 + t["mu"] * un / np.where(s > 0, s, 1.0), 0.0), 0.0)
            unew = t["drag"] * k[:, None] * tg
            app = hit & (un < 0)
            vI[app] = vr[app] + unew[app]
        lo, hi = self.band, self.n - 1 - self.band
        wall = np.any((self.node_idx < lo) | (self.node_idx > hi), axis=1)
        vI[wall] = 0.0
        self.grid = (m, p, vI)
        return vI

    def read(self):
        return {"x": self.x.copy(), "v": self.v.copy(), "C": self.C.copy(), "F": self.F.copy()}

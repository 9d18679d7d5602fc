"""Pins of the oracle's reverse-mode adjoint of the substep (the gradient of a
rollout with respect to per-particle stiffness theta = log E, the tools'
per-substep linear velocities and the starting state).

The adjoint is checked against things it does not compute itself:
central finite differences of the pinned forward oracle (unit maps and whole
rollouts), and closed forms that follow from momentum conservation of the
APIC/MLS transfers (Sec. III-B): without tools and walls, sum_p v_p changes
only by gravity, so d(sum_p a.x_T)/d v0_q = T dt a and d/d theta = 0."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2502_18437_amd import scenes

RNG = np.random.default_rng(20250218)


def fd(fn, base, direction, h):
    return (fn(base + h * direction) - fn(base - h * direction)) / (2 * h)


# ---------------------------------------------------------------- unit maps
@pytest.mark.parametrize("kind", ["near_identity", "rotated_stretch", "shear"])
def test_polar_adjoint_matches_finite_differences(kind):
    if kind == "near_identity":
        F = np.eye(3) + 0.05 * RNG.standard_normal((3, 3))
    elif kind == "rotated_stretch":
        Q, _ = np.linalg.qr(RNG.standard_normal((3, 3)))
        Q *= np.sign(np.linalg.det(Q))
        F = Q @ np.diag([1.4, 0.8, 1.1])
    else:
        F = np.array([[1.0, 0.6, 0.0], [0.0, 1.0, 0.2], [0.1, 0.0, 0.9]])
    Rb = RNG.standard_normal((3, 3))
    g = O.polar_adjoint(F, Rb)
    num = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            E = np.zeros((3, 3))
            E[i, j] = 1.0
            num[i, j] = fd(lambda X: np.sum(Rb * O.polar(X)[0]), F, E, 1e-6)
    np.testing.assert_allclose(g, num, rtol=0, atol=1e-8 * max(1.0, np.abs(num).max()))


def test_polar_adjoint_of_a_rotation_only_cotangent_is_skew_in_body_frame():
    """Rotations of F by a small Q = exp(eps W) rotate R by the same Q (exact
    for the polar factor), so <Fb, W F> = <Rb, W R> for any skew W."""
    F = np.eye(3) + 0.2 * RNG.standard_normal((3, 3))
    R, _ = O.polar(F)
    Rb = RNG.standard_normal((3, 3))
    Fb = O.polar_adjoint(F, Rb)
    for _ in range(3):
        w = RNG.standard_normal(3)
        W = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        assert abs(np.sum(Fb * (W @ F)) - np.sum(Rb * (W @ R))) < 1e-10 * max(1.0, np.abs(Rb).sum())


def test_kirchhoff_adjoint_matches_finite_differences():
    F = np.eye(3) + 0.15 * RNG.standard_normal((3, 3))
    E, nu = 4.3e3, 0.35
    tb = RNG.standard_normal((3, 3))
    g, th = O.kirchhoff_adjoint(F, E, nu, tb)
    num = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            D = np.zeros((3, 3))
            D[i, j] = 1.0
            num[i, j] = fd(lambda X: np.sum(tb * O.kirchhoff(X, E, nu)[0]), F, D, 1e-6)
    np.testing.assert_allclose(g, num, rtol=0, atol=1e-8 * np.abs(num).max())
    # theta = log E enters linearly: d/d theta = tb : tau
    num_th = fd(lambda t: np.sum(tb * O.kirchhoff(F, math.exp(t), nu)[0]), math.log(E), 1.0, 1e-5)
    assert abs(th - num_th) < 1e-8 * abs(num_th)
    assert abs(th - np.sum(tb * O.kirchhoff(F, E, nu)[0])) < 1e-9 * abs(th)


def test_kirchhoff_adjoint_at_rest_is_the_linear_elasticity_tensor():
    """At F = I, d tau = mu (dF + dF^T) + lambda tr(dF) I: the adjoint of a
    cotangent tb is mu (tb + tb^T) + lambda tr(tb) I."""
    E, nu = 5e3, 0.3
    mu, la = E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))
    tb = RNG.standard_normal((3, 3))
    g, th = O.kirchhoff_adjoint(np.eye(3), E, nu, tb)
    np.testing.assert_allclose(g, mu * (tb + tb.T) + la * np.trace(tb) * np.eye(3), rtol=0, atol=1e-9 * E)
    assert abs(th) < 1e-9


TOOLS = [
    (O.TOOL_CAPSULE, (0.05, 0.02, 0.0)),
    (O.TOOL_BOX, (0.05, 0.03, 0.02)),
    (O.TOOL_PLANE, (0.0, 0.0, 0.0)),
    (O.TOOL_SLICER, (0.05, 0.03, 0.0)),
    (O.TOOL_SEGMENT, (0.05, 0.02, 0.0)),
    (O.TOOL_ARC, (0.05, 1.0, 0.02)),
]


@pytest.mark.parametrize("tool_type,size", TOOLS)
def test_contact_adjoint_matches_finite_differences(tool_type, size):
    quat = np.array([0.9, 0.1, 0.3, -0.2])
    quat /= np.linalg.norm(quat)
    c0 = np.array([0.5, 0.5, 0.5])
    kw = dict(quat=quat, size=size, ang_vel=(0.5, -1.0, 0.7), mu=0.3, drag=0.9, margin=0.01)
    laws = set()
    worst = 0.0
    for _ in range(120):
        xI = c0 + 0.06 * RNG.standard_normal(3)
        vin = RNG.standard_normal(3)
        lv = RNG.standard_normal(3) * 0.3
        v, law = O.frame_contact(tool_type, c0, kw["quat"], size, lv, kw["ang_vel"], kw["mu"], kw["drag"],
                                 kw["margin"], xI, vin)
        ref, hit = O.node_contact(tool_type, c0, kw["quat"], size, lv, kw["ang_vel"], kw["mu"], kw["drag"],
                                  kw["margin"], xI, vin)
        assert hit == (law != 0)
        np.testing.assert_allclose(v, ref, rtol=0, atol=1e-13)
        laws.add(law)
        vb = RNG.standard_normal(3)
        gv, gc, gl = O.contact_adjoint(tool_type, c0, kw["quat"], size, lv, kw["ang_vel"], kw["mu"], kw["drag"],
                                       kw["margin"], xI, vin, vb)

        def out(vin=vin, c=c0, lv=lv):
            return vb @ O.frame_contact(tool_type, c, kw["quat"], size, lv, kw["ang_vel"], kw["mu"], kw["drag"],
                                        kw["margin"], xI, vin)[0]

        for grad, make in ((gv, lambda b: out(vin=b)), (gc, lambda b: out(c=b)), (gl, lambda b: out(lv=b))):
            base = {id(gv): vin, id(gc): c0, id(gl): lv}[id(grad)]
            num = np.array([fd(make, base, e, 1e-7) for e in np.eye(3)])
            worst = max(worst, np.abs(num - grad).max() / max(1.0, np.abs(num).max()))
    assert worst < 1e-6, worst
    assert len(laws - {0}) >= 1  # the samples reached the contact law


def test_sticky_spine_passes_only_the_rigid_velocity():
    """Beyond a slicer's spine the node takes the tool's rigid velocity: the
    cotangent goes to the tool's linear velocity (and, through av x r, to its
    centre), none to the node's velocity."""
    SL = (0.1, 0.05, 0.0)
    xI = (0.53, 0.5 + 0.05 + 0.002, 0.501)
    vb = np.array([0.3, -0.7, 0.2])
    gv, gc, gl = O.contact_adjoint(O.TOOL_SLICER, (0.5, 0.5, 0.5), (1, 0, 0, 0), SL, (0.0, 0.5, 0.0),
                                   (0.0, 0.0, 2.0), 0.0, 1.0, 0.004, np.array(xI), np.array([0.3, 0.2, -0.1]), vb)
    np.testing.assert_array_equal(gv, np.zeros(3))
    np.testing.assert_allclose(gl, vb, atol=0)
    w = np.array([0.0, 0.0, 2.0])
    np.testing.assert_allclose(gc, np.cross(w, vb), atol=1e-15)


# ---------------------------------------------------------------- velocity tables
def capsule_scene(seed=3):
    s = scenes.tiny_block(n_grid=16, per_axis=6, seed=seed, E_range=(2e3, 8e3), center=(0.5, 0.45, 0.5))
    dx = 1.0 / 16
    tool = dict(center=(0.5, 0.45 + 1.5 * dx + 0.6 * dx, 0.5), quat=(0.9, 0.1, 0.2, 0.0), size=(0.08, 1.2 * dx, 0),
                lin_vel=(0, 0, 0), ang_vel=(0.5, 0, 1.0), mu=0.3, drag=0.9, margin=0.0)
    return s, tool


def make_oracle(s, state, theta, tools, tables):
    o = O.Oracle(s.n_grid, s.dt, gravity=s.gravity, wall_band=s.wall_band, nu=s.nu)
    x, v, C, F = state
    o.set_state_f64(x, v, C, F, np.exp(theta), s.mass, s.vol0)
    for k, (tt, kw) in enumerate(tools):
        o.set_tool(k, tt, **kw)
    for k, tab in tables.items():
        o.set_velocity_table(k, tab)
    return o


def test_constant_table_equals_constant_velocity():
    s, tool = capsule_scene()
    state = [a.astype(float) for a in (s.x, s.v, s.C, s.F)]
    theta = np.log(s.E.astype(float))
    T = 12
    vel = (0.2, -1.0, 0.1)
    kw = dict(tool, lin_vel=vel)
    a = make_oracle(s, state, theta, [(O.TOOL_CAPSULE, kw)], {})
    b = make_oracle(s, state, theta, [(O.TOOL_CAPSULE, tool)], {0: np.tile(vel, (T, 1))})
    a.step(T)
    b.step(T)
    ra, rb = a.read(), b.read()
    for k in ("x", "v", "C", "F"):
        np.testing.assert_allclose(ra[k], rb[k], rtol=0, atol=1e-11 * max(1.0, np.abs(ra[k]).max()))


def test_table_end_resumes_constant_velocity_from_the_end_pose():
    """A 3-row table moving +y then the constant velocity (0,0,0): the tool
    stays where the table left it (pose = anchor + dt * sum of rows), which
    the same scene with the tool set there directly reproduces."""
    s, tool = capsule_scene()
    state = [a.astype(float) for a in (s.x, s.v, s.C, s.F)]
    theta = np.log(s.E.astype(float))
    rows = np.array([[0.0, 2.0, 0.0], [0.0, 3.0, 0.0], [0.0, 1.0, 0.0]])
    a = make_oracle(s, state, theta, [(O.TOOL_CAPSULE, tool)], {0: rows})
    a.step(5)
    # the same rows then rest, with the rest phase set explicitly as a table
    b = make_oracle(s, state, theta, [(O.TOOL_CAPSULE, tool)], {0: np.vstack([rows, np.zeros((2, 3))])})
    b.step(5)
    np.testing.assert_array_equal(a.read()["x"], b.read()["x"])


# ---------------------------------------------------------------- rollouts
def rollout_case(kind):
    s, tool = capsule_scene()
    dx = 1.0 / 16
    T = 8
    tables = {0: np.stack([0.3 * np.sin(np.arange(T)), -1.0 + 0.2 * np.cos(np.arange(T)), 0.1 * np.ones(T)], 1)}
    tools = [(O.TOOL_CAPSULE, tool)]
    if kind == "three_tools":
        tools = [
            (O.TOOL_BOX, dict(center=(0.5, 0.45 + 1.5 * dx + 0.4 * dx, 0.5), quat=(0.95, 0.0, 0.3, 0.1),
                              size=(0.06, 0.5 * dx, 0.06), lin_vel=(0, 0, 0), ang_vel=(0, 1.0, 0), mu=0.2, drag=1.0,
                              margin=0.0)),
            (O.TOOL_SEGMENT, dict(center=(0.47, 0.42, 0.46), quat=(0.9, 0.2, 0.0, 0.1), size=(0.1, 0.9 * dx, 0.0),
                                  lin_vel=(0.2, 0.3, 0.0), mu=0.2)),
            (O.TOOL_ARC, dict(center=(0.52, 0.43, 0.53), quat=(0.95, 0.0, 0.3, 0.0), size=(0.07, 1.2, 0.8 * dx),
                              lin_vel=(-0.1, 0.4, 0.2), ang_vel=(1.0, 0.0, 0.0), mu=0.1)),
        ]
        tables = {0: np.stack([0.2 * np.ones(T), -0.8 + 0.1 * np.arange(T), np.zeros(T)], 1)}
    state = [a.astype(float) for a in (s.x, s.v, s.C, s.F)]
    theta = np.log(s.E.astype(float))
    seeds = [RNG.standard_normal(a.shape) for a in state]
    return s, T, state, theta, tools, tables, seeds


@pytest.mark.parametrize("kind", ["capsule_table", "three_tools"])
def test_rollout_gradient_matches_finite_differences(kind):
    s, T, state, theta, tools, tables, seeds = rollout_case(kind)

    def loss(state=state, theta=theta, tables=tables):
        o = make_oracle(s, state, theta, tools, tables)
        assert o.step(T) == 0
        r = o.read()
        return sum(np.sum(a * b) for a, b in zip(seeds, (r["x"], r["v"], r["C"], r["F"])))

    o = make_oracle(s, state, theta, tools, tables)
    g = o.rollout_adjoint(T, *seeds)
    assert g["status"] == 0
    # every tool of the scene was in contact (their velocity gradient is non-zero)
    assert np.all(np.abs(g["vel"][: len(tools)]).sum(axis=(1, 2)) > 0)
    # (name, base, gradient, step, relative tolerance): the friction law is
    # strongly curved in the tool velocity, so its central differences carry
    # an O(h^2) error of ~1e-6 at h = 1e-5; a wrong term shows as O(1).
    checks = [
        ("theta", theta, g["theta"], 1e-4, 1e-6, lambda b: loss(theta=b)),
        ("table", tables[0], g["vel"][0], 1e-6, 1e-5, lambda b: loss(tables={**tables, 0: b})),
        ("x0", state[0], g["x0"], 1e-7, 1e-6, lambda b: loss(state=[b] + state[1:])),
        ("v0", state[1], g["v0"], 1e-5, 1e-6, lambda b: loss(state=[state[0], b] + state[2:])),
        ("C0", state[2], g["C0"], 1e-5, 1e-6, lambda b: loss(state=state[:2] + [b, state[3]])),
        ("F0", state[3], g["F0"], 1e-7, 1e-6, lambda b: loss(state=state[:3] + [b])),
    ]
    for name, base, grad, h, tol, fn in checks:
        for _ in range(3):
            d = RNG.standard_normal(base.shape)
            num = fd(fn, base, d, h)
            ana = np.sum(grad * d)
            assert abs(num - ana) <= tol * abs(num) + 1e-8, (name, num, ana)


def test_rollout_gradient_coordinates():
    """16 single coordinates of theta and of the velocity table."""
    s, T, state, theta, tools, tables, seeds = rollout_case("capsule_table")
    o = make_oracle(s, state, theta, tools, tables)
    g = o.rollout_adjoint(T, *seeds)

    def loss(theta=theta, tables=tables):
        o = make_oracle(s, state, theta, tools, tables)
        o.step(T)
        r = o.read()
        return sum(np.sum(a * b) for a, b in zip(seeds, (r["x"], r["v"], r["C"], r["F"])))

    for p in RNG.choice(s.N, 8, replace=False):
        e = np.zeros_like(theta)
        e[p] = 1.0
        num = fd(lambda b: loss(theta=b), theta, e, 1e-4)
        assert abs(num - g["theta"][p]) <= 1e-6 * max(abs(num), 1e-3), (p, num, g["theta"][p])
    for j, c in zip(RNG.choice(T, 8), RNG.choice(3, 8)):
        e = np.zeros_like(tables[0])
        e[j, c] = 1.0
        num = fd(lambda b: loss(tables={0: b}), tables[0], e, 1e-6)
        assert abs(num - g["vel"][0, j, c]) <= 1e-5 * max(abs(num), 1e-3), (j, c, num, g["vel"][0, j, c])


def test_momentum_closed_forms_without_tools_or_walls():
    """No tools, walls out of reach: the transfers conserve sum_p m v_p (APIC
    P2G and G2P, and internal forces sum to zero), so for L = sum_p a . x_T:
    dL/dv0_q = T dt a, dL/dx0_q = a and dL/dtheta = 0; for L = sum_p a . v_T:
    dL/dv0_q = a."""
    s = scenes.tiny_block(n_grid=16, per_axis=6, seed=5, E_range=(2e3, 8e3))
    s.v = (0.2 * s.v).astype(np.float32)
    state = [a.astype(float) for a in (s.x, s.v, s.C, s.F)]
    theta = np.log(s.E.astype(float))
    T = 10
    a = np.array([0.3, -1.1, 0.7])
    o = make_oracle(s, state, theta, [], {})
    g = o.rollout_adjoint(T, xb=np.tile(a, (s.N, 1)))
    assert g["status"] == 0
    np.testing.assert_allclose(g["v0"], np.tile(T * s.dt * a, (s.N, 1)), rtol=0, atol=1e-12)
    np.testing.assert_allclose(g["x0"], np.tile(a, (s.N, 1)), rtol=0, atol=1e-9)
    assert np.abs(g["theta"]).max() < 1e-9
    o = make_oracle(s, state, theta, [], {})
    g = o.rollout_adjoint(T, vb=np.tile(a, (s.N, 1)))
    np.testing.assert_allclose(g["v0"], np.tile(a, (s.N, 1)), rtol=0, atol=1e-12)


def test_zero_substep_rollout_returns_the_seeds():
    s, T, state, theta, tools, tables, seeds = rollout_case("capsule_table")
    o = make_oracle(s, state, theta, tools, tables)
    g = o.rollout_adjoint(0, *seeds)
    for k, sd in zip(("x0", "v0", "C0", "F0"), seeds):
        np.testing.assert_array_equal(g[k], sd)
    assert not g["theta"].any()

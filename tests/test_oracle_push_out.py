"""Pins of the oracle's particle push-out (Sec. IV-A: particles left inside a
rigid shape are pushed out, after the particle collision step of Stomakhin
et al. 2013; the reading: x <- x - phi n for phi < 0, with the tool at its
pose of the next substep). Closed forms for a plane, a box and a capsule,
the pose one substep ahead, tools that ignore it, and the independent NumPy
formulation."""
import numpy as np
import pytest

import oracle as O
from oracle.brute import Brute
from paper_2502_18437_amd import scenes

N_GRID, DT = 32, 1e-4


def one_substep(x, tool_type, center, size=(0, 0, 0), lin_vel=(0, 0, 0), push_out=True, quat=(1, 0, 0, 0)):
    """Particles at rest, no gravity: the substep itself moves nothing, so
    every change of x is the push-out."""
    o = O.Oracle(N_GRID, DT, gravity=(0.0, 0.0, 0.0))
    x = np.asarray(x, np.float32)
    o.set_particles(x, mass=1e-4, vol0=1e-7)
    o.set_tool(0, tool_type, center=center, quat=quat, size=size, lin_vel=lin_vel, push_out=push_out)
    assert o.step(1) == 0
    r = o.read()
    o.close()
    return x.astype(np.float64), r["x"]


def test_plane_pushes_particles_below_to_its_surface():
    x0, x = one_substep([[0.5, 0.45, 0.5], [0.4, 0.499, 0.6], [0.5, 0.55, 0.5]], O.TOOL_PLANE, (0.5, 0.5, 0.5))
    np.testing.assert_allclose(x[:2, 1], 0.5, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(x[:2, [0, 2]], x0[:2, [0, 2]])  # along the normal only
    np.testing.assert_array_equal(x[2], x0[2])                      # outside: unchanged


def test_box_pushes_to_the_nearest_face():
    c, h = (0.5, 0.5, 0.5), (0.1, 0.05, 0.08)
    # nearest faces: +x (0.02 from it), -y (0.01 from it), +z (0.005 from it)
    pts = [[0.58, 0.5, 0.5], [0.5, 0.46, 0.49], [0.51, 0.5, 0.575]]
    x0, x = one_substep(pts, O.TOOL_BOX, c, size=h)
    np.testing.assert_allclose(x[0], [0.6, 0.5, 0.5], rtol=0, atol=1e-7)
    np.testing.assert_allclose(x[1], [x0[1, 0], 0.45, x0[1, 2]], rtol=0, atol=1e-7)
    np.testing.assert_allclose(x[2], [x0[2, 0], x0[2, 1], 0.58], rtol=0, atol=1e-7)


def test_capsule_pushes_radially_from_its_axis():
    c, h, r = (0.5, 0.5, 0.5), 0.1, 0.04
    pts = [[0.53, 0.512, 0.5],   # 0.012 above the axis (inside, r = 0.04)
           [0.65, 0.5, 0.5],     # beyond the end cap: 0.05 from the end point, outside
           [0.61, 0.5, 0.51]]    # in the end cap, 0.01 * sqrt(2) from the end point
    x0, x = one_substep(pts, O.TOOL_CAPSULE, c, size=(h, r, 0.0))
    np.testing.assert_allclose(x[0], [x0[0, 0], 0.5 + r, 0.5], rtol=0, atol=1e-7)
    np.testing.assert_array_equal(x[1], x0[1])
    e = x0[2] - np.array([0.6, 0.5, 0.5])
    np.testing.assert_allclose(x[2], np.array([0.6, 0.5, 0.5]) + r * e / np.linalg.norm(e), rtol=0, atol=1e-7)


def test_push_uses_the_pose_of_the_next_substep():
    """A plane rising at 2 m/s: after one substep it is dt * 2 higher, and
    the particle ends on it there, not on the plane's starting height."""
    x0, x = one_substep([[0.5, 0.45, 0.5]], O.TOOL_PLANE, (0.5, 0.5, 0.5), lin_vel=(0.0, 2.0, 0.0))
    assert abs(x[0, 1] - (0.5 + 2.0 * DT)) < 1e-12


@pytest.mark.parametrize("tool_type,size", [(O.TOOL_SLICER, (0.05, 0.02, 0.0)), (O.TOOL_SEGMENT, (0.05, 0.02, 0.0))])
def test_thin_tools_and_switched_off_tools_do_not_push(tool_type, size):
    x0, x = one_substep([[0.5, 0.5, 0.5]], tool_type, (0.5, 0.5, 0.5), size=size)
    np.testing.assert_array_equal(x, x0)
    x0, x = one_substep([[0.5, 0.45, 0.5]], O.TOOL_PLANE, (0.5, 0.5, 0.5), push_out=False)
    np.testing.assert_array_equal(x, x0)


def push_scene(seed):
    """A block under a descending capsule, a box sweeping in from the side
    and a tilted plane under it; all three push out."""
    s = scenes.tiny_block(n_grid=16, per_axis=7, seed=seed, E_range=(2e3, 8e3), center=(0.5, 0.4, 0.5))
    dx = 1.0 / 16
    s.tools = [
        scenes.Tool(scenes.TOOL_CAPSULE, (0.5, 0.5, 0.47), (0.9, 0.1, -0.3, 0.2), (0.12, 2.2 * dx, 0.0),
                    (0.05, -3.0, 0.0), (0.0, 0.0, 1.5), mu=0.3, drag=0.9, push_out=True),
        scenes.Tool(scenes.TOOL_BOX, (0.33, 0.4, 0.5), (0.95, 0.0, 0.3, 0.0), (0.04, 0.1, 0.6 * dx),
                    (4.0, 0.0, 0.05), mu=0.5, push_out=True),
        scenes.Tool(scenes.TOOL_PLANE, (0.5, 0.3, 0.5), (0.98, 0.1, 0.0, 0.15), (0, 0, 0), (0.0, 1.0, 0.0),
                    mu=0.2, margin=0.5 * dx, push_out=True),
    ]
    return s


def run(cls, s, n, **kw):
    o = cls(s.n_grid, s.dt, gravity=s.gravity, wall_band=s.wall_band, nu=s.nu, E_default=s.E_default)
    o.set_particles(s.x, s.v, s.C, s.F, s.E, s.mass, s.vol0)
    for k, t in enumerate(s.tools):
        o.set_tool(k, t.type, **dict(t.kwargs(), **kw))
    for _ in range(n):
        st = o.step(1)
        assert st in (0, None)
    return o.read()


@pytest.mark.parametrize("seed", [0, 1])
def test_push_out_matches_numpy_twin_and_acts(seed):
    s = push_scene(seed)
    r, q = run(O.Oracle, s, 20), run(Brute, s, 20)
    for k, tol in (("x", 1e-12), ("v", 1e-12), ("C", 1e-9), ("F", 1e-12)):
        scale = max(1.0, np.max(np.abs(q[k])))
        np.testing.assert_allclose(r[k], q[k], rtol=0, atol=tol * scale, err_msg=k)
    off = run(O.Oracle, s, 20, push_out=False)
    assert np.max(np.abs(off["x"] - r["x"])) > 1e-4  # the tools do push particles here

"""Pins of the FP64 oracle's building blocks against facts fixed by the
mathematics, not by the oracle itself: B-spline moment identities, polar
decomposition by definition and against LAPACK's SVD, the fixed-corotated
stress as the derivative of its energy, closed-form SDFs, and hand-worked
contact cases (CRESSim-MPM Sec. III-A, III-B and IV-A)."""
import math

import numpy as np
import pytest

import oracle as O


# ---------------------------------------------------------------- T1: weights
@pytest.mark.parametrize("seed", range(5))
def test_bspline_moments(seed):
    """Quadratic B-spline (Sec. III-A): partition of unity, zero first moment,
    second moment 1/4 -- the identity behind D = dx^2/4 I (Sec. III-B)."""
    rng = np.random.default_rng(seed)
    for f in np.concatenate([[0.5, 1.0, 1.4999999], rng.uniform(0.5, 1.5, 200)]):
        w = O.weights(f)
        o = np.arange(3) - f
        assert abs(w.sum() - 1.0) < 1e-15
        assert abs((w * o).sum()) < 1e-15
        assert abs((w * o * o).sum() - 0.25) < 1e-15
        assert np.all(w >= 0)


def test_bspline_values_closed_form():
    # f = 1 (particle on a node): weights 1/8, 3/4, 1/8.
    np.testing.assert_allclose(O.weights(1.0), [0.125, 0.75, 0.125], rtol=0, atol=1e-16)
    # f = 1/2: the third node is at distance 3/2, weight 0.
    np.testing.assert_allclose(O.weights(0.5), [0.5, 0.5, 0.0], rtol=0, atol=1e-16)


# ---------------------------------------------------------------- T10: polar
def random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


@pytest.mark.parametrize("seed", range(10))
def test_polar_definition(seed):
    rng = np.random.default_rng(seed)
    for scale in (1e-3, 0.1, 0.5):
        F = np.eye(3) + scale * rng.normal(size=(3, 3))
        if np.linalg.det(F) <= 0:
            continue
        R, J = O.polar(F)
        assert abs(J - np.linalg.det(F)) < 1e-14
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1.0) < 1e-13
        S = R.T @ F
        np.testing.assert_allclose(S, S.T, atol=1e-13)
        assert np.all(np.linalg.eigvalsh(0.5 * (S + S.T)) > 0)
        # against LAPACK: the orthogonal polar factor U V^T
        U, _, Vt = np.linalg.svd(F)
        np.testing.assert_allclose(R, U @ Vt, atol=1e-12)


def test_polar_special_cases():
    rng = np.random.default_rng(42)
    Q = random_rotation(rng)
    R, _ = O.polar(Q)
    np.testing.assert_allclose(R, Q, atol=1e-14)
    # pure stretch: R = I
    R, _ = O.polar(np.diag([1.3, 0.7, 1.1]))
    np.testing.assert_allclose(R, np.eye(3), atol=1e-15)
    # repeated singular values (F = 2 Q)
    R, _ = O.polar(2.0 * Q)
    np.testing.assert_allclose(R, Q, atol=1e-14)


def test_polar_inverted_sign_fix():
    """det F < 0: R stays a rotation and R^T F is symmetric with one negative
    eigenvalue on the smallest singular direction (Irving et al. 2004)."""
    rng = np.random.default_rng(3)
    Q = random_rotation(rng)
    F = Q @ np.diag([1.2, 0.9, -0.3])
    R, J = O.polar(F)
    assert J < 0
    assert abs(np.linalg.det(R) - 1.0) < 1e-13
    S = R.T @ F
    np.testing.assert_allclose(S, S.T, atol=1e-13)
    ev = np.sort(np.linalg.eigvalsh(0.5 * (S + S.T)))
    np.testing.assert_allclose(ev, [-0.3, 0.9, 1.2], atol=1e-12)
    np.testing.assert_allclose(R, Q, atol=1e-12)


# ---------------------------------------------------------------- T6, T9: stress
def test_stress_zero_at_rest_and_rotation():
    tau, J = O.kirchhoff(np.eye(3), 5e3, 0.3)
    assert J == 1.0
    assert np.max(np.abs(tau)) == 0.0
    rng = np.random.default_rng(1)
    for _ in range(5):
        tau, _ = O.kirchhoff(random_rotation(rng), 5e3, 0.3)
        assert np.max(np.abs(tau)) < 1e-10


@pytest.mark.parametrize("seed", range(6))
def test_stress_is_energy_derivative(seed):
    """tau = (dPsi/dF) F^T with Psi = mu |F - R|^2 + lambda/2 (J - 1)^2,
    checked by central differences of Psi; tau symmetric."""
    rng = np.random.default_rng(seed)
    E, nu = 5e3 * (1 + seed), 0.3 + 0.02 * seed
    F = np.eye(3) + 0.2 * rng.normal(size=(3, 3))
    if np.linalg.det(F) < 0.2:
        F = np.eye(3) + 0.05 * rng.normal(size=(3, 3))
    h = 1e-6
    P = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            Fp, Fm = F.copy(), F.copy()
            Fp[i, j] += h
            Fm[i, j] -= h
            P[i, j] = (O.energy(Fp, E, nu) - O.energy(Fm, E, nu)) / (2 * h)
    tau, _ = O.kirchhoff(F, E, nu)
    np.testing.assert_allclose(tau, P @ F.T, rtol=1e-6, atol=1e-6 * E)
    np.testing.assert_allclose(tau, tau.T, atol=1e-9 * E)


def test_lame_parameters_uniaxial():
    """Small uniaxial stretch: tau_xx = (lambda + 2 mu) eps to first order."""
    E, nu, eps = 5e3, 0.3, 1e-7
    mu = E / (2 * (1 + nu))
    la = E * nu / ((1 + nu) * (1 - 2 * nu))
    tau, _ = O.kirchhoff(np.diag([1 + eps, 1.0, 1.0]), E, nu)
    assert abs(tau[0, 0] / eps - (la + 2 * mu)) < 1e-3 * (la + 2 * mu)
    assert abs(tau[1, 1] / eps - la) < 1e-3 * la


# ---------------------------------------------------------------- T12: SDFs
def fd_grad(tool_type, c, q, s, p, h=1e-7):
    g = np.zeros(3)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        g[a] = (O.sdf(tool_type, c, q, s, p + e)[0] - O.sdf(tool_type, c, q, s, p - e)[0]) / (2 * h)
    return g


def test_capsule_sdf_closed_form():
    c = np.array([0.5, 0.4, 0.5])
    q = np.array([1.0, 0, 0, 0])
    s = np.array([0.1, 0.03, 0.0])
    # above the middle of the segment
    phi, g = O.sdf(O.TOOL_CAPSULE, c, q, s, c + [0.02, 0.05, 0.0])
    assert abs(phi - 0.02) < 1e-15
    np.testing.assert_allclose(g, [0, 1, 0], atol=1e-15)
    # past the end cap along the axis
    phi, g = O.sdf(O.TOOL_CAPSULE, c, q, s, c + [0.15, 0.0, 0.0])
    assert abs(phi - 0.02) < 1e-15
    np.testing.assert_allclose(g, [1, 0, 0], atol=1e-15)
    # on the axis: normal +y of the body frame
    phi, g = O.sdf(O.TOOL_CAPSULE, c, q, s, c.copy())
    assert abs(phi + 0.03) < 1e-15
    np.testing.assert_allclose(g, [0, 1, 0], atol=1e-15)
    # rotated: axis along z (rotation of -90 deg about y maps body x to world z)
    qz = np.array([math.sqrt(0.5), 0, -math.sqrt(0.5), 0])
    phi, g = O.sdf(O.TOOL_CAPSULE, c, qz, s, c + [0.0, 0.0, 0.12])
    assert abs(phi - (0.02 - 0.03)) < 1e-12
    phi, g = O.sdf(O.TOOL_CAPSULE, c, qz, s, c + [0.05, 0.0, 0.09])
    assert abs(phi - 0.02) < 1e-12
    np.testing.assert_allclose(g, [1, 0, 0], atol=1e-12)


def test_box_sdf_closed_form():
    c = np.array([0.3, 0.3, 0.5])
    q = np.array([1.0, 0, 0, 0])
    e = np.array([0.15, 0.1, 0.01])
    phi, g = O.sdf(O.TOOL_BOX, c, q, e, c + [0.2, 0.0, 0.0])
    assert abs(phi - 0.05) < 1e-15
    np.testing.assert_allclose(g, [1, 0, 0], atol=1e-15)
    phi, g = O.sdf(O.TOOL_BOX, c, q, e, c + [0.18, 0.14, 0.0])  # outside a corner edge
    assert abs(phi - 0.05) < 1e-14
    np.testing.assert_allclose(g, [0.6, 0.8, 0], atol=1e-12)
    phi, g = O.sdf(O.TOOL_BOX, c, q, e, c + [0.0, 0.0, -0.004])  # inside, nearest face -z
    assert abs(phi + 0.006) < 1e-15
    np.testing.assert_allclose(g, [0, 0, -1], atol=1e-15)
    phi, g = O.sdf(O.TOOL_BOX, c, q, e, c.copy())  # on the mid-plane: sign(0) = +1
    assert abs(phi + 0.01) < 1e-15
    np.testing.assert_allclose(g, [0, 0, 1], atol=1e-15)


def test_plane_sdf_closed_form():
    c = np.array([0.0, 0.2, 0.0])
    phi, g = O.sdf(O.TOOL_PLANE, c, [1, 0, 0, 0], [0, 0, 0], np.array([0.3, 0.25, 0.7]))
    assert abs(phi - 0.05) < 1e-15
    np.testing.assert_allclose(g, [0, 1, 0], atol=1e-15)
    # tilted 90 deg about z: body +y maps to world -x
    qq = [math.sqrt(0.5), 0, 0, math.sqrt(0.5)]
    phi, g = O.sdf(O.TOOL_PLANE, c, qq, [0, 0, 0], np.array([0.1, 0.2, 0.0]))
    assert abs(phi + 0.1) < 1e-12
    np.testing.assert_allclose(g, [-1, 0, 0], atol=1e-12)


@pytest.mark.parametrize("tool_type", [O.TOOL_CAPSULE, O.TOOL_BOX, O.TOOL_PLANE])
def test_sdf_gradient_matches_fd(tool_type):
    rng = np.random.default_rng(tool_type)
    for _ in range(50):
        c = rng.uniform(0.3, 0.7, 3)
        q = rng.normal(size=4)
        s = rng.uniform(0.02, 0.1, 3)
        p = c + rng.uniform(-0.2, 0.2, 3)
        phi, g = O.sdf(tool_type, c, q, s, p)
        gf = fd_grad(tool_type, c, q, s, p)
        if np.linalg.norm(gf) < 0.999:  # FD straddles a kink (box medial surface)
            continue
        np.testing.assert_allclose(g / np.linalg.norm(g), gf, atol=1e-6)


# ---------------------------------------------------------------- T11: contact law
N_UP = np.array([0.0, 1.0, 0.0])


def test_contact_separating_unchanged():
    for u in ([0.1, 0.2, 0.0], [0.3, 0.0, -0.2]):  # u_n > 0 and u_n = 0
        np.testing.assert_array_equal(O.contact(N_UP, np.array(u), 0.3, 1.0), u)


def test_contact_normal_removed_frictionless():
    out = O.contact(N_UP, np.array([0.4, -1.0, 0.3]), 0.0, 1.0)
    np.testing.assert_allclose(out, [0.4, 0.0, 0.3], atol=1e-16)


def test_contact_friction_shrinks_tangent():
    # |t| = 0.5, u_n = -1, mu = 0.3: factor 1 - 0.3 / 0.5 = 0.4
    out = O.contact(N_UP, np.array([0.3, -1.0, 0.4]), 0.3, 1.0)
    np.testing.assert_allclose(out, [0.12, 0.0, 0.16], atol=1e-15)


def test_contact_friction_saturates_to_stick():
    out = O.contact(N_UP, np.array([0.1, -1.0, 0.0]), 0.3, 1.0)
    np.testing.assert_array_equal(out, [0.0, 0.0, 0.0])


def test_contact_zero_tangent_and_drag():
    np.testing.assert_array_equal(O.contact(N_UP, np.array([0.0, -2.0, 0.0]), 0.3, 1.0), [0, 0, 0])
    # c_d = 0: sticky
    np.testing.assert_array_equal(O.contact(N_UP, np.array([0.5, -0.1, 0.0]), 0.0, 0.0), [0, 0, 0])
    # c_d = 0.5 halves the corrected tangent
    out = O.contact(N_UP, np.array([0.5, -0.1, 0.0]), 0.0, 0.5)
    np.testing.assert_allclose(out, [0.25, 0, 0], atol=1e-16)


def test_contact_never_reverses_tangent():
    rng = np.random.default_rng(0)
    for _ in range(200):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        u = rng.normal(size=3)
        mu = rng.uniform(0, 2)
        out = O.contact(n, u, mu, 1.0)
        un = n @ u
        if un >= 0:
            np.testing.assert_array_equal(out, u)
        else:
            t = u - un * n
            assert abs(out @ n) < 1e-14
            assert out @ t >= -1e-15
            assert np.linalg.norm(out) <= np.linalg.norm(t) + 1e-15

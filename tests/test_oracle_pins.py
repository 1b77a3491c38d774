"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a closed form,
an invariant, a library routine, brute force, or a fixture read from the paper.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

from workload import QUAD, sample_nodes, xavier_params
from oracle.quadrotor import (nominal_f, nominal_jac, quat_mul, quat_conj, quat_rotate,
                              rotor_positions, ROTOR_SPIN, body_torque)
from oracle.mlp import MLP, pack_input, residual_in_state, silu_prime
from oracle.rk4 import (linearize_affine, linearize_exact, affine_phi, exact_phi, rk4_step)
from oracle.riccati import (riccati, riccati_batched, kkt_bruteforce, lq_rollout, lq_rollout_batched, box_lq,
                            box_lq_bruteforce, condense)

HERE = os.path.dirname(os.path.abspath(__file__))
DT = 0.05


def zero_output(Ws, bs):
    Ws = [W.copy() for W in Ws]
    bs = [b.copy() for b in bs]
    Ws[-1][:] = 0
    bs[-1][:] = 0
    return MLP(Ws, bs)


def yaw_quat(psi):
    return np.array([np.cos(psi / 2), 0.0, 0.0, np.sin(psi / 2)])


# ---------------------------------------------------------------- quaternions

def test_quat_rotate_matches_library_rotation():
    """q (.) v = q v q-bar equals scipy's rotation for unit q (Sec. VI, Notation)."""
    x, _ = sample_nodes(64, seed=11)
    q = x[:, 3:7].astype(np.float64)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    v = np.random.default_rng(0).normal(size=(64, 3))
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).apply(v)  # scipy uses scalar-last
    np.testing.assert_allclose(quat_rotate(q, v), ref, atol=1e-12)


def test_quat_mul_associative_and_norm_multiplicative():
    rng = np.random.default_rng(1)
    a, b, c = rng.normal(size=(3, 10, 4))
    np.testing.assert_allclose(quat_mul(quat_mul(a, b), c), quat_mul(a, quat_mul(b, c)), atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(quat_mul(a, b), axis=1),
                               np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1), rtol=1e-12)
    # i*j = k for Hamilton quaternions
    i, j, k = np.eye(4)[1], np.eye(4)[2], np.eye(4)[3]
    np.testing.assert_allclose(quat_mul(i, j), k)


# ---------------------------------------------------------------- rotor geometry

def test_rotor_geometry_matches_figure():
    """Body-frame rotor positions and spins re-derived from the figure's drawing coordinates."""
    fig = json.load(open(os.path.join(HERE, "golden", "quad_model_figure.json")))
    ex = np.array(fig["body_axis_x_dir"]); ex /= np.linalg.norm(ex)
    ey = np.array(fig["body_axis_y_dir"]); ey /= np.linalg.norm(ey)
    r = rotor_positions(QUAD)
    for i in range(4):
        hub = np.array(fig["rotor_hub_xy"][str(i)])
        body = np.array([hub @ ex, hub @ ey])
        body = body / np.linalg.norm(body)
        np.testing.assert_allclose(r[i, :2] / np.linalg.norm(r[i, :2]), body, atol=1e-3)
        np.testing.assert_allclose(np.linalg.norm(r[i]), QUAD.arm, rtol=1e-12)
        arc = fig["spin_arcs"][str(i)]
        sweep = np.sign(arc["end_deg"] - arc["start_deg"])  # +1: counter-clockwise path
        if arc["arrow"] == "<-":
            sweep = -sweep
        assert ROTOR_SPIN[i] == sweep


def test_mixer_is_cross_product_of_geometry():
    """tau = sum r_i x T_i e_z - spin_i c_tau T_i e_z, evaluated by hand for unit thrusts."""
    h = QUAD.arm / np.sqrt(2)
    tau = body_torque(np.eye(4), QUAD)
    np.testing.assert_allclose(tau[:, 0], h * np.array([-1, -1, 1, 1]), atol=1e-15)
    np.testing.assert_allclose(tau[:, 1], h * np.array([-1, 1, 1, -1]), atol=1e-15)
    np.testing.assert_allclose(tau[:, 2], QUAD.c_tau * np.array([-1, 1, -1, 1]), atol=1e-15)


# ---------------------------------------------------------------- nominal model

def test_hover_equilibrium():
    """Thrust sum m*g, level yawed attitude, at rest: f_F = 0 (eq. (6), g_W = -9.81 e_z)."""
    x = np.zeros((5, 13))
    for i, psi in enumerate(np.linspace(-2, 2, 5)):
        x[i, 3:7] = yaw_quat(psi)
    x[:, 0:3] = np.random.default_rng(2).uniform(-5, 5, size=(5, 3))
    u = np.full((5, 4), QUAD.mass * QUAD.g / 4)
    np.testing.assert_allclose(nominal_f(x, u), 0.0, atol=1e-14)


def test_nominal_jacobian_complex_step():
    """Hand-derived df/dx, df/du equal complex-step derivatives (exact to round-off)."""
    x, u = sample_nodes(32, seed=12)
    x = x.astype(np.float64); u = u.astype(np.float64)
    x[:, 3:7] *= 1.03  # off the unit sphere, as at RK4 stage points
    Fx, Fu = nominal_jac(x, u)
    hstep = 1e-30
    for j in range(13):
        xc = x.astype(complex); xc[:, j] += 1j * hstep
        np.testing.assert_allclose(nominal_f(xc, u.astype(complex)).imag / hstep, Fx[:, :, j], atol=1e-12)
    for j in range(4):
        uc = u.astype(complex); uc[:, j] += 1j * hstep
        np.testing.assert_allclose(nominal_f(x.astype(complex), uc).imag / hstep, Fu[:, :, j], atol=1e-12)


# ---------------------------------------------------------------- network

def fd_jacobian(fun, z, h=1e-6):
    cols = []
    for j in range(z.shape[1]):
        zp, zm = z.copy(), z.copy()
        zp[:, j] += h; zm[:, j] -= h
        cols.append((fun(zp) - fun(zm)) / (2 * h))
    return np.stack(cols, axis=-1)


def test_linear_network_jacobian_is_weight_product():
    Ws, bs = xavier_params(3, 16, seed=5)
    net = MLP(Ws, bs, act="identity")
    z = pack_input(*sample_nodes(7, seed=3))
    _, J = net.jacobian(z)
    prod = Ws[3].astype(np.float64) @ Ws[2] @ Ws[1] @ Ws[0]
    np.testing.assert_allclose(J, np.broadcast_to(prod, J.shape), atol=1e-12)


def test_silu_network_at_origin():
    """z0 = 0, zero biases: SiLU(0) = 0 and SiLU'(0) = 1/2, so y = 0, J = 2^-L W_{L+1}...W_1."""
    L = 3
    Ws, bs = xavier_params(L, 32, seed=6)
    net = MLP(Ws, bs)
    y, J = net.jacobian(np.zeros((1, 14)))
    np.testing.assert_allclose(y, 0.0, atol=1e-15)
    prod = Ws[3].astype(np.float64) @ Ws[2] @ Ws[1] @ Ws[0]
    np.testing.assert_allclose(J[0], prod / 2 ** L, atol=1e-14)
    assert silu_prime(np.array(0.0)) == 0.5


def test_network_jacobian_finite_differences():
    Ws, bs = xavier_params(4, 48, seed=7)
    bs = [np.random.default_rng(9).normal(size=b.shape) * 0.3 for b in bs]
    net = MLP(Ws, bs)
    z = pack_input(*sample_nodes(16, seed=4))
    _, J = net.jacobian(z)
    np.testing.assert_allclose(J, fd_jacobian(net.forward, z), atol=2e-8)


def test_residual_scatter_positions():
    """f_D = [0_3, 0_4, y_v, y_w] (eq. (7)); Jacobian columns follow z0 = [v, w, q, u]."""
    n = 3
    y = np.arange(n * 6, dtype=float).reshape(n, 6) + 1
    J = np.random.default_rng(1).normal(size=(n, 6, 14))
    f, Jx, Ju = residual_in_state(y, J)
    assert np.all(f[:, :7] == 0) and np.all(f[:, 7:] == y)
    assert np.all(Jx[:, :7] == 0) and np.all(Jx[:, :, 0:3] == 0)
    np.testing.assert_array_equal(Jx[:, 7:, 7:10], J[:, :, 0:3])
    np.testing.assert_array_equal(Jx[:, 7:, 10:13], J[:, :, 3:6])
    np.testing.assert_array_equal(Jx[:, 7:, 3:7], J[:, :, 6:10])
    np.testing.assert_array_equal(Ju[:, 7:], J[:, :, 10:14])


# ---------------------------------------------------------------- RK4 + sensitivities

def test_zero_output_hover_is_fixed_point():
    Ws, bs = xavier_params(2, 64)
    net = zero_output(Ws, bs)
    x = np.zeros((3, 13)); x[:, 3:7] = [yaw_quat(a) for a in (0.3, -1.0, 2.5)]
    x[:, 0:3] = [[1, 2, 3], [-4, 0, 1], [0, 0, 0]]
    u = np.full((3, 4), QUAD.mass * QUAD.g / 4)
    xn, A, B, y, _ = linearize_affine(x, u, net, DT)
    np.testing.assert_allclose(y, 0.0, atol=0)
    np.testing.assert_allclose(xn, x, atol=1e-14)


def test_free_fall_closed_form():
    """u = 0, w = 0, zero-output network: every entry of x_{k+1}, A_k, B_k in closed form."""
    Ws, bs = xavier_params(2, 64)
    net = zero_output(Ws, bs)
    x, _ = sample_nodes(9, seed=21)
    x = x.astype(np.float64); x[:, 10:13] = 0
    u = np.zeros((9, 4))
    xn, A, B, _, _ = linearize_affine(x, u, net, DT)
    g = np.array([0, 0, -QUAD.g])
    np.testing.assert_allclose(xn[:, 0:3], x[:, 0:3] + x[:, 7:10] * DT + 0.5 * g * DT ** 2, atol=1e-13)
    np.testing.assert_allclose(xn[:, 7:10], x[:, 7:10] + g * DT, atol=1e-13)
    np.testing.assert_allclose(xn[:, 3:7], x[:, 3:7], atol=1e-15)
    np.testing.assert_allclose(xn[:, 10:13], 0, atol=0)
    Jd = np.array([QUAD.Jx, QUAD.Jy, QUAD.Jz])
    h = QUAD.arm / np.sqrt(2)
    tau_unit = np.stack([h * np.array([-1, -1, 1, 1]), h * np.array([-1, 1, 1, -1]),
                         QUAD.c_tau * np.array([-1, 1, -1, 1])], axis=0)  # (3, 4)
    for i in range(9):
        q = x[i, 3:7]
        Aref = np.eye(13)
        Aref[0:3, 7:10] = DT * np.eye(3)
        for j in range(3):  # d q+ / d w_j = dt/2 * q (x) e_j
            e = np.zeros(4); e[1 + j] = 1
            Aref[3:7, 10 + j] = DT / 2 * quat_mul(q, e)
        np.testing.assert_allclose(A[i], Aref, atol=1e-13)
        d = quat_rotate(q, np.array([0, 0, 1.0]))
        Bref = np.zeros((13, 4))
        for r in range(4):
            wdot = tau_unit[:, r] / Jd
            Bref[0:3, r] = DT ** 2 / 2 * d / QUAD.mass
            Bref[7:10, r] = DT * d / QUAD.mass
            Bref[10:13, r] = DT * wdot
            Bref[3:7, r] = DT ** 2 / 4 * quat_mul(q, np.concatenate([[0], wdot]))
        np.testing.assert_allclose(B[i], Bref, atol=1e-12)


def test_quaternion_norm_closed_form():
    """Equal thrusts and w on a principal axis keep w constant; RK4 then scales |q| exactly
    by (1 - t^2/2 + t^4/24)^2 + (t - t^3/6)^2 with t = |w| dt / 2."""
    Ws, bs = xavier_params(2, 64)
    net = zero_output(Ws, bs)
    x, _ = sample_nodes(6, seed=31)
    x = x.astype(np.float64)
    x[:, 10:13] = 0
    rates = [3.0, -2.0, 5.0, 1.0, 7.0, -4.0]
    for i in range(6):
        x[i, 10 + i % 3] = rates[i]
    u = np.full((6, 4), 2.2)
    xn, _, _, _, _ = linearize_affine(x, u, net, DT)
    t = np.abs(rates) * DT / 2
    ref = (1 - t ** 2 / 2 + t ** 4 / 24) ** 2 + (t - t ** 3 / 6) ** 2
    ref *= np.sum(x[:, 3:7] ** 2, axis=1)  # the float32 inputs are unit only to ~1e-8
    np.testing.assert_allclose(np.sum(xn[:, 3:7] ** 2, axis=1), ref, rtol=1e-13)
    np.testing.assert_allclose(xn[:, 10:13], x[:, 10:13], atol=1e-13)


def test_position_columns_are_trivial():
    """Nothing depends on p: A[:, 0:3] = [I_3; 0] exactly, with a SiLU network."""
    Ws, bs = xavier_params(3, 32)
    x, u = sample_nodes(20)
    _, A, _, _, _ = linearize_affine(x, u, MLP(Ws, bs), DT)
    ref = np.zeros((13, 3)); ref[0:3] = np.eye(3)
    assert np.all(A[:, :, 0:3] == ref)


def _fd_map(phi, x, u, h=1e-6):
    A = np.stack([(phi(x + h * e, u) - phi(x - h * e, u)) / (2 * h) for e in np.eye(13)], axis=-1)
    B = np.stack([(phi(x, u + h * e) - phi(x, u - h * e)) / (2 * h) for e in np.eye(4)], axis=-1)
    return A, B


def test_affine_sensitivities_finite_differences():
    Ws, bs = xavier_params(3, 32, seed=8)
    net = MLP(Ws, bs)
    x, u = sample_nodes(12, seed=41)
    x = x.astype(np.float64); u = u.astype(np.float64)
    xn, A, B, y, J = linearize_affine(x, u, net, DT)
    phi = lambda xx, uu: affine_phi(xx, uu, x, u, y, J, DT)
    np.testing.assert_allclose(phi(x, u), xn, atol=1e-14)
    Afd, Bfd = _fd_map(phi, x, u)
    np.testing.assert_allclose(A, Afd, atol=1e-8)
    np.testing.assert_allclose(B, Bfd, atol=1e-8)


def test_exact_sensitivities_finite_differences():
    Ws, bs = xavier_params(2, 24, seed=9)
    net = MLP(Ws, bs)
    x, u = sample_nodes(8, seed=42)
    xn, A, B = linearize_exact(x, u, net, DT)
    phi = lambda xx, uu: exact_phi(xx, uu, net, DT)
    np.testing.assert_allclose(phi(x.astype(float), u.astype(float)), xn, atol=1e-14)
    Afd, Bfd = _fd_map(phi, x.astype(float), u.astype(float))
    np.testing.assert_allclose(A, Afd, atol=1e-8)
    np.testing.assert_allclose(B, Bfd, atol=1e-8)


def test_rk4_fourth_order():
    """The RK4 routine itself: global error slope 4 on x' = A x."""
    M = np.array([[0.0, 1.0], [-4.0, -0.3]])
    x0 = np.array([[1.0, 0.5]])
    exact = scipy.linalg.expm(M * 1.0) @ x0[0]
    errs = []
    for n in (10, 20, 40):
        x = x0.copy()
        for _ in range(n):
            x = rk4_step(lambda a, b: a @ M.T, x, None, 1.0 / n)
        errs.append(np.linalg.norm(x[0] - exact))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 4) < 0.2)


def test_linear_network_affine_equals_exact():
    Ws, bs = xavier_params(2, 16, seed=10)
    bs = [np.full_like(b, 0.1) for b in bs]
    net = MLP(Ws, bs, act="identity")
    x, u = sample_nodes(10, seed=43)
    xa, Aa, Ba, _, _ = linearize_affine(x, u, net, DT)
    xe, Ae, Be = linearize_exact(x, u, net, DT)
    np.testing.assert_allclose(xa, xe, atol=1e-12)
    np.testing.assert_allclose(Aa, Ae, atol=1e-12)
    np.testing.assert_allclose(Ba, Be, atol=1e-12)


def test_local_approximation_error_order():
    """First-order approximation: error O(dt^3) on x_{k+1}, O(dt^2) on A and B (Sec. IV-A)."""
    Ws, bs = xavier_params(2, 32, seed=11)
    Ws = [W * 3.0 for W in Ws]  # a strongly curved network
    net = MLP(Ws, bs)
    x, u = sample_nodes(8, seed=44)
    dts = np.array([0.04, 0.02, 0.01, 0.005])
    ex, eA = [], []
    for dt in dts:
        xa, Aa, Ba, _, _ = linearize_affine(x, u, net, dt)
        xe, Ae, Be = linearize_exact(x, u, net, dt)
        ex.append(np.max(np.abs(xa - xe)))
        eA.append(max(np.max(np.abs(Aa - Ae)), np.max(np.abs(Ba - Be))))
    sx = np.polyfit(np.log(dts), np.log(ex), 1)[0]
    sA = np.polyfit(np.log(dts), np.log(eA), 1)[0]
    assert abs(sx - 3) < 0.25, sx
    assert abs(sA - 2) < 0.25, sA


# ---------------------------------------------------------------- Riccati

def _random_lq(N, seed, nx=13, nu=4):
    rng = np.random.default_rng(seed)
    A = np.eye(nx) + 0.1 * rng.normal(size=(N, nx, nx))
    B = rng.normal(size=(N, nx, nu)) * 0.2
    c = rng.normal(size=(N, nx)) * 0.1
    q = rng.normal(size=(N, nx)); r = rng.normal(size=(N, nu)); qN = rng.normal(size=nx)
    Q = np.eye(nx); R = 0.1 * np.eye(nu); QN = 2 * np.eye(nx)
    return A, B, c, q, r, qN, Q, R, QN


@pytest.mark.parametrize("N", [1, 2, 3])
def test_riccati_matches_kkt(N):
    A, B, c, q, r, qN, Q, R, QN = _random_lq(N, seed=N)
    K, kff, P = riccati(A, B, Q, R, QN, c, q, r, qN)
    du0, _ = kkt_bruteforce(A, B, Q, R, QN, np.zeros(13), c, q, r, qN)
    np.testing.assert_allclose(kff[0], du0[0], atol=1e-11)
    for j in range(13):
        e = np.zeros(13); e[j] = 1
        du, dx = kkt_bruteforce(A, B, Q, R, QN, e, c, q, r, qN)
        np.testing.assert_allclose(K[0] @ e + kff[0], du[0], atol=1e-11)
        # the feedback law holds along the optimal trajectory at every node
        for k in range(N):
            np.testing.assert_allclose(K[k] @ dx[k] + kff[k], du[k], atol=1e-10)


def test_riccati_converges_to_dare():
    rng = np.random.default_rng(3)
    nx, nu, N = 13, 4, 500
    A0 = rng.normal(size=(nx, nx)); A0 *= 1.05 / np.max(np.abs(np.linalg.eigvals(A0)))
    B0 = rng.normal(size=(nx, nu))
    Q, R = np.eye(nx), 0.1 * np.eye(nu)
    K, kff, P = riccati(np.broadcast_to(A0, (N, nx, nx)), np.broadcast_to(B0, (N, nx, nu)), Q, R, Q)
    Pd = scipy.linalg.solve_discrete_are(A0, B0, Q, R)
    np.testing.assert_allclose(P[0], Pd, rtol=1e-9, atol=1e-9)
    Kd = -np.linalg.solve(R + B0.T @ Pd @ B0, B0.T @ Pd @ A0)
    np.testing.assert_allclose(K[0], Kd, rtol=1e-8, atol=1e-9)


def test_riccati_value_matrices_spd():
    A, B, c, q, r, qN, Q, R, QN = _random_lq(12, seed=7)
    _, _, P = riccati(A, B, Q, R, QN, c, q, r, qN)
    for Pk in P:
        np.testing.assert_allclose(Pk, Pk.T, atol=1e-12)
        assert np.min(np.linalg.eigvalsh(Pk)) > 0


def test_riccati_batched_ranges():
    A, B, c, q, r, qN, Q, R, QN = _random_lq(7, seed=8)
    off = np.array([0, 3, 7])
    K, kff, P = riccati_batched(off, A, B, Q, R, QN, c=c)
    K0, k0, _ = riccati(A[:3], B[:3], Q, R, QN, c[:3])
    K1, k1, _ = riccati(A[3:], B[3:], Q, R, QN, c[3:])
    np.testing.assert_array_equal(K, np.concatenate([K0, K1]))
    np.testing.assert_array_equal(kff, np.concatenate([k0, k1]))


@pytest.mark.parametrize("N", [1, 3, 6])
def test_lq_rollout_is_the_qp_minimiser(N):
    """The forward pass of the Riccati solution reproduces the dense KKT primal solution
    (every dx_k, du_k, and the terminal dx_N) for an arbitrary initial deviation."""
    A, B, c, q, r, qN, Q, R, QN = _random_lq(N, seed=20 + N)
    K, kff, _ = riccati(A, B, Q, R, QN, c, q, r, qN)
    dx0 = np.random.default_rng(N).normal(size=13)
    du_ref, dx_ref = kkt_bruteforce(A, B, Q, R, QN, dx0, c, q, r, qN)
    du, dx = lq_rollout(A, B, K, kff, dx0, c)
    np.testing.assert_allclose(du, du_ref, atol=1e-10)
    np.testing.assert_allclose(dx, dx_ref, atol=1e-10)


def test_lq_rollout_batched_ranges():
    A, B, c, q, r, qN, Q, R, QN = _random_lq(7, seed=9)
    off = np.array([0, 4, 7])
    K, kff, _ = riccati_batched(off, A, B, Q, R, QN, c=c)
    dx0 = np.random.default_rng(1).normal(size=(2, 13))
    du, dx, dxN = lq_rollout_batched(off, A, B, K, kff, dx0, c)
    for i, (a, b) in enumerate([(0, 4), (4, 7)]):
        du_ref, dx_ref = kkt_bruteforce(A[a:b], B[a:b], Q, R, QN, dx0[i], c[a:b])
        np.testing.assert_allclose(du[a:b], du_ref, atol=1e-10)
        np.testing.assert_allclose(dx[a:b], dx_ref[:-1], atol=1e-10)
        np.testing.assert_allclose(dxN[i], dx_ref[-1], atol=1e-10)


# ---------------------------------------------------------------- input box (QP with eq. (3) on u)

def test_box_lq_without_active_bounds_is_the_unconstrained_minimiser():
    A, B, c, q, r, qN, Q, R, QN = _random_lq(4, seed=31)
    dx0 = np.random.default_rng(2).normal(size=13)
    du_ref, dx_ref = kkt_bruteforce(A, B, Q, R, QN, dx0, c, q, r, qN)
    big = np.full((4, 4), 1e9)
    du, dx = box_lq(A, B, Q, R, QN, dx0, -big, big, c, q, r, qN)
    np.testing.assert_allclose(du, du_ref, atol=1e-10)
    np.testing.assert_allclose(dx, dx_ref, atol=1e-10)


@pytest.mark.parametrize("N,seed", [(1, 1), (2, 2), (2, 3)])
def test_box_lq_matches_active_set_enumeration(N, seed):
    A, B, c, q, r, qN, Q, R, QN = _random_lq(N, seed=40 + seed)
    rng = np.random.default_rng(seed)
    dx0 = rng.normal(size=13)
    lo, hi = -rng.uniform(0.05, 0.6, size=(N, 4)), rng.uniform(0.05, 0.6, size=(N, 4))
    du, dx = box_lq(A, B, Q, R, QN, dx0, lo, hi, c, q, r, qN)
    du_b, dx_b = box_lq_bruteforce(A, B, Q, R, QN, dx0, lo, hi, c, q, r, qN)
    np.testing.assert_allclose(du, du_b, atol=1e-10)
    np.testing.assert_allclose(dx, dx_b, atol=1e-10)
    assert np.sum(np.isclose(du, lo) | np.isclose(du, hi)) > 0  # the box is active somewhere


def test_box_lq_kkt_conditions():
    """Stationarity with sign-correct multipliers: the condensed gradient vanishes on free
    components, is >= 0 at lower bounds and <= 0 at upper bounds; dynamics hold."""
    N = 6
    A, B, c, q, r, qN, Q, R, QN = _random_lq(N, seed=51)
    rng = np.random.default_rng(5)
    dx0 = 3 * rng.normal(size=13)
    lo, hi = np.full((N, 4), -0.2), np.full((N, 4), 0.25)
    du, dx = box_lq(A, B, Q, R, QN, dx0, lo, hi, c, q, r, qN)
    H, h, S, s = condense(A, B, Q, R, QN, dx0, c, q, r, qN)
    g = H @ du.reshape(-1) + h
    x, l, u = du.reshape(-1), lo.reshape(-1), hi.reshape(-1)
    at_lo, at_hi = np.isclose(x, l, atol=1e-12), np.isclose(x, u, atol=1e-12)
    free = ~(at_lo | at_hi)
    assert at_lo.any() and at_hi.any() and free.any()
    assert np.all(np.abs(g[free]) < 1e-9)
    assert np.all(g[at_lo] > -1e-9) and np.all(g[at_hi] < 1e-9)
    for k in range(N):
        np.testing.assert_allclose(dx[k + 1], A[k] @ dx[k] + B[k] @ du[k] + c[k], atol=1e-10)


# ---------------------------------------------------------------- second-order approximation (eq. (4))

def _hess_net(act="silu"):
    Ws, bs = xavier_params(3, 32, seed=3)
    bs = [np.random.default_rng(1).normal(size=b.shape) * 0.1 for b in bs]
    return MLP(Ws, bs, act)


def test_hessian_matches_complex_step_of_the_jacobian():
    from oracle.mlp import pack_input as pk
    net = _hess_net()
    x, u = sample_nodes(6, seed=2)
    z = pk(x, u)
    _, J, H = net.hessian(z)
    _, J_ref = net.jacobian(z)
    np.testing.assert_array_equal(J, J_ref)
    h = 1e-20
    Hc = np.zeros_like(H)
    for c in range(14):
        zc = z.astype(complex)
        zc[:, c] += 1j * h
        Hc[:, :, :, c] = net.jacobian(zc)[1].imag / h
    assert np.abs(H - Hc).max() < 1e-12 * np.abs(H).max()
    np.testing.assert_allclose(H, H.transpose(0, 1, 3, 2), atol=1e-15)


def test_hessian_of_a_linear_network_vanishes():
    from oracle.mlp import pack_input as pk
    net = _hess_net("identity")
    x, u = sample_nodes(4, seed=3)
    _, _, H = net.hessian(pk(x, u))
    assert np.abs(H).max() == 0.0


def test_quadratic_linearisation_matches_finite_differences():
    from oracle.rk4 import linearize_quadratic, quadratic_phi
    net = _hess_net()
    x, u = sample_nodes(4, seed=4)
    dt = 0.05
    xq, A, B, yb, J, H = linearize_quadratic(x, u, net, dt)
    eps = 1e-6
    for j in range(13):
        xp, xm = x.astype(float).copy(), x.astype(float).copy()
        xp[:, j] += eps
        xm[:, j] -= eps
        fd = (quadratic_phi(xp, u, x, u, yb, J, H, dt) - quadratic_phi(xm, u, x, u, yb, J, H, dt)) / (2 * eps)
        np.testing.assert_allclose(A[:, :, j], fd, atol=1e-7)
    for j in range(4):
        up, um = u.astype(float).copy(), u.astype(float).copy()
        up[:, j] += eps
        um[:, j] -= eps
        fd = (quadratic_phi(x, up, x, u, yb, J, H, dt) - quadratic_phi(x, um, x, u, yb, J, H, dt)) / (2 * eps)
        np.testing.assert_allclose(B[:, :, j], fd, atol=1e-7)


def test_quadratic_with_zero_hessian_is_the_first_order_step():
    from oracle.rk4 import linearize_quadratic
    net = _hess_net("identity")
    x, u = sample_nodes(5, seed=5)
    q = linearize_quadratic(x, u, net, 0.05)
    a = linearize_affine(x, u, net, 0.05)
    for g, r in zip(q[:5], a):
        np.testing.assert_allclose(g, r, atol=1e-13)


def test_second_order_approximation_error_is_third_order():
    """Sec. IV-A: the error of the second-order approximation is of third order in the
    change between nodes: gap(x_{k+1}) ~ dt^4, gap(A, B) ~ dt^3 against the exact step."""
    from oracle.rk4 import linearize_quadratic
    net = _hess_net()
    x, u = sample_nodes(5, seed=2)
    dts = [0.04, 0.02, 0.01, 0.005]
    ex, eA = [], []
    for dt in dts:
        xq, Aq, Bq = linearize_quadratic(x, u, net, dt)[:3]
        xe, Ae, Be = linearize_exact(x, u, net, dt)[:3]
        ex.append(np.abs(xq - xe).max())
        eA.append(max(np.abs(Aq - Ae).max(), np.abs(Bq - Be).max()))
    sx = np.polyfit(np.log(dts), np.log(ex), 1)[0]
    sA = np.polyfit(np.log(dts), np.log(eA), 1)[0]
    assert abs(sx - 4) < 0.35, sx
    assert abs(sA - 3) < 0.5, sA


# ---------------------------------------------------------------- residual input variants (f_Da, f_Da,u)

def _variant_net(din, seed=0):
    rng = np.random.default_rng(seed)
    Ws = [rng.normal(size=(32, din)) * 0.3, rng.normal(size=(32, 32)) * 0.2, rng.normal(size=(3, 32)) * 0.3]
    bs = [rng.normal(size=32) * 0.1, rng.normal(size=32) * 0.1, rng.normal(size=3) * 0.1]
    return Ws, bs


def test_body_velocity_identity_and_norm():
    from oracle.mlp import body_velocity
    x, _ = sample_nodes(50, seed=11)
    x = x.astype(np.float64)
    vb = body_velocity(x)
    qn2 = np.sum(x[:, 3:7] ** 2, axis=1)
    np.testing.assert_allclose(np.linalg.norm(vb, axis=1), qn2 * np.linalg.norm(x[:, 7:10], axis=1), rtol=1e-12)
    xi = x.copy()
    xi[:, 3:7] = [1, 0, 0, 0]
    np.testing.assert_allclose(body_velocity(xi), xi[:, 7:10], atol=1e-15)
    # a yaw of +90 degrees maps world x to body -y
    xq = x[:1].copy()
    xq[0, 3:7] = [np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)]
    xq[0, 7:10] = [1, 0, 0]
    np.testing.assert_allclose(body_velocity(xq)[0], [0, -1, 0], atol=1e-15)


@pytest.mark.parametrize("mode", [1, 2])
def test_input_jacobian_matches_finite_differences(mode):
    from oracle.mlp import input_jacobian, pack_input_mode
    x, u = sample_nodes(6, seed=12)
    x, u = x.astype(np.float64), u.astype(np.float64)
    dzx, dzu = input_jacobian(x, u, mode)
    eps = 1e-6
    for i in range(13):
        xp, xm = x.copy(), x.copy()
        xp[:, i] += eps
        xm[:, i] -= eps
        np.testing.assert_allclose(dzx[:, :, i], (pack_input_mode(xp, u, mode) - pack_input_mode(xm, u, mode)) / (2 * eps),
                                   atol=1e-8)
    for i in range(4):
        up, um = u.copy(), u.copy()
        up[:, i] += eps
        um[:, i] -= eps
        np.testing.assert_allclose(dzu[:, :, i], (pack_input_mode(x, up, mode) - pack_input_mode(x, um, mode)) / (2 * eps),
                                   atol=1e-8)


@pytest.mark.parametrize("mode,din", [(1, 3), (2, 7)])
def test_variant_linearisation_matches_finite_differences(mode, din):
    Ws, bs = _variant_net(din)
    net = MLP(Ws, bs)
    x, u = sample_nodes(5, seed=13)
    xn, A, B, yb, J = linearize_affine(x, u, net, 0.05, mode=mode)
    assert yb.shape == (5, 3) and J.shape == (5, 3, din)
    eps = 1e-6
    for j in range(13):
        xp, xm = x.astype(float).copy(), x.astype(float).copy()
        xp[:, j] += eps
        xm[:, j] -= eps
        fd = (affine_phi(xp, u, x, u, yb, J, 0.05, mode=mode) - affine_phi(xm, u, x, u, yb, J, 0.05, mode=mode)) / (2 * eps)
        np.testing.assert_allclose(A[:, :, j], fd, atol=1e-7)
    for j in range(4):
        up, um = u.astype(float).copy(), u.astype(float).copy()
        up[:, j] += eps
        um[:, j] -= eps
        fd = (affine_phi(x, up, x, u, yb, J, 0.05, mode=mode) - affine_phi(x, um, x, u, yb, J, 0.05, mode=mode)) / (2 * eps)
        np.testing.assert_allclose(B[:, :, j], fd, atol=1e-7)


def test_variant_at_level_attitude_equals_full_model_embedding():
    """With q = identity, v_B = v: a v_B network gives the same step as the full-input
    network whose first layer reads v (other inputs weighted 0) and whose angular outputs
    are 0 -- as long as the attitude stays put during the step (zero body rates and equal
    thrusts, so no torque), since the v_B model also depends on q."""
    Ws, bs = _variant_net(3, seed=4)
    x, u = sample_nodes(8, seed=14)
    x = x.astype(np.float64)
    x[:, 3:7] = [1, 0, 0, 0]
    x[:, 10:13] = 0.0
    u = np.repeat(u[:, :1], 4, axis=1)
    W1 = np.zeros((32, 14)); W1[:, 0:3] = Ws[0]
    Wo = np.zeros((6, 32)); Wo[0:3] = Ws[2]
    bo = np.zeros(6); bo[0:3] = bs[2]
    full = MLP([W1, Ws[1], Wo], [bs[0], bs[1], bo])
    xv = linearize_affine(x, u, MLP(Ws, bs), 0.05, mode=1)[0]
    xf = linearize_affine(x, u, full, 0.05)[0]
    np.testing.assert_allclose(xv, xf, atol=1e-13)

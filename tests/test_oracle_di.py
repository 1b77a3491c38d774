"""Pins of the double-integrator oracle (the runtime workload of Sec. V) against
closed forms, finite differences and an independently written LQ solution.

* With no residual the continuous model is linear with constant input, so RK4
  is exact: x_{k+1} = [p + v dt + u dt^2/2, v + u dt], A = [[1, dt], [0, 1]],
  B = [dt^2/2, dt].
* With the affine residual the model is x-dot = M x + d (M = df_F/dx + J_D);
  RK4 of a linear system with constant forcing is the degree-4 Taylor
  polynomial of the flow: A = sum_{j<=4} (dt M)^j / j!, and the step and B are
  the matching series applied to F(x_k) and to df_F/du.
* The sensitivities equal central differences of the step map with the model
  held fixed.
* With no residual one real-time iteration is Newton's method on a linear-
  quadratic problem, so it lands on the exact optimum: the new iterate has no
  gaps and equals the minimiser of the condensed problem solved here directly.
"""
import math

import numpy as np
import pytest

from oracle.double_integrator import linearize, rti_step, nominal_f
from oracle.mlp import MLP
from workload import xavier_params

DT = 0.05
Q = np.eye(2)
R = np.array([[0.1]])


def di_net(L, H, seed, zero_out=False):
    Ws, bs = xavier_params(L, H, seed=seed, d_in=2, d_out=2)
    rng = np.random.default_rng(seed + 7)
    bs = [rng.uniform(-0.3, 0.3, size=b.shape) for b in bs]
    if zero_out:
        Ws[-1] = np.zeros_like(Ws[-1])
        bs[-1] = np.zeros_like(bs[-1])
    return Ws, bs


def di_nodes(n, seed):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.uniform(-2, 2, n), rng.normal(0, 1, n)], axis=1)
    u = rng.uniform(-1, 1, (n, 1))
    return x, u


def test_no_residual_is_exact_kinematics():
    x, u = di_nodes(7, 1)
    xn, A, B, y, J = linearize(x, u, None, DT)
    p, v, a = x[:, 0], x[:, 1], u[:, 0]
    np.testing.assert_allclose(xn[:, 0], p + v * DT + a * DT ** 2 / 2, rtol=0, atol=1e-15)
    np.testing.assert_allclose(xn[:, 1], v + a * DT, rtol=0, atol=1e-15)
    np.testing.assert_allclose(A, np.broadcast_to([[1, DT], [0, 1]], A.shape), atol=1e-16)
    np.testing.assert_allclose(B[:, :, 0], np.broadcast_to([DT ** 2 / 2, DT], (7, 2)), atol=1e-17)


def test_affine_residual_matches_taylor_polynomial():
    n = 6
    x, u = di_nodes(n, 2)
    rng = np.random.default_rng(3)
    y = rng.normal(0, 1, (n, 2))
    J = rng.normal(0, 2, (n, 2, 2))
    xn, A, B, _, _ = linearize(x, u, None, DT, params=(y, J))
    Fx = np.array([[0.0, 1.0], [0.0, 0.0]])
    Fu = np.array([[0.0], [1.0]])
    for i in range(n):
        M = Fx + J[i]
        F0 = nominal_f(x[i:i + 1], u[i:i + 1])[0] + y[i]
        Aw = sum(np.linalg.matrix_power(DT * M, j) / math.factorial(j) for j in range(5))
        # phi = dt * sum_{j=1..4} (dt M)^{j-1} / j!
        Phi = DT * sum(np.linalg.matrix_power(DT * M, j - 1) / math.factorial(j) for j in range(1, 5))
        np.testing.assert_allclose(A[i], Aw, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(xn[i], x[i] + Phi @ F0, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(B[i], Phi @ Fu, rtol=1e-13, atol=1e-15)


def test_network_sensitivities_match_finite_differences():
    Ws, bs = di_net(2, 16, seed=4)
    net = MLP(Ws, bs)
    x, u = di_nodes(5, 5)
    xn, A, B, y, J = linearize(x, u, net, DT)
    h = 1e-6
    for j in range(2):
        e = np.zeros(2)
        e[j] = h
        fp = linearize(x + e, u, None, DT, params=(y, J), xbar=x)[0]
        fm = linearize(x - e, u, None, DT, params=(y, J), xbar=x)[0]
        np.testing.assert_allclose(A[:, :, j], (fp - fm) / (2 * h), rtol=1e-7, atol=1e-9)
    fp = linearize(x, u + h, None, DT, params=(y, J), xbar=x)[0]
    fm = linearize(x, u - h, None, DT, params=(y, J), xbar=x)[0]
    np.testing.assert_allclose(B[:, :, 0], (fp - fm) / (2 * h), rtol=1e-7, atol=1e-9)
    # J_D itself: central differences of the network
    for j in range(2):
        e = np.zeros(2)
        e[j] = 1e-6
        np.testing.assert_allclose(J[:, :, j], (net.forward(x + e) - net.forward(x - e)) / 2e-6, rtol=1e-6, atol=1e-9)


def condensed_optimum(A, B, x0, N, xref, QN):
    """Minimiser of sum_k 1/2 |x_k - xref|_Q^2 + 1/2 |u_k|_R^2 + 1/2 |x_N - xref|_QN^2
    subject to x_{k+1} = A x_k + B u_k, by stacking x = Phi x0 + Gamma U."""
    Phi = np.zeros((N + 1, 2, 2))
    Gam = np.zeros((N + 1, 2, N))
    Phi[0] = np.eye(2)
    for k in range(N):
        Phi[k + 1] = A @ Phi[k]
        Gam[k + 1] = A @ Gam[k]
        Gam[k + 1][:, k] += B[:, 0]
    H = np.kron(np.eye(N), R)
    g = np.zeros(N)
    for k in range(N + 1):
        W = QN if k == N else Q
        H = H + Gam[k].T @ W @ Gam[k]
        g = g + Gam[k].T @ W @ (Phi[k] @ x0 - xref)
    U = np.linalg.solve(H, -g)
    X = np.stack([Phi[k] @ x0 + Gam[k] @ U for k in range(N + 1)])
    return U, X


@pytest.mark.parametrize("N", [1, 3, 10])
def test_rti_without_residual_reaches_the_optimum(N):
    rng = np.random.default_rng(N)
    offsets = np.array([0, N, 2 * N])
    x = rng.normal(0, 1, (2 * N, 2))
    u = rng.normal(0, 1, (2 * N, 1))
    xN = rng.normal(0, 1, (2, 2))
    x0 = rng.normal(0, 1, (2, 2))
    xref = rng.normal(0, 1, (2, 2))
    QN = 3.0 * np.eye(2)
    for model in (None, MLP(*di_net(2, 8, seed=9, zero_out=True))):
        du, dx, dxN, _ = rti_step(offsets, x, u, xN, x0, model, DT, Q, R, QN, xref=xref)
        Ad = np.array([[1, DT], [0, 1]])
        Bd = np.array([[DT ** 2 / 2], [DT]])
        for i in range(2):
            a, b = offsets[i], offsets[i + 1]
            Xn = np.concatenate([x[a:b] + dx[a:b], (xN[i] + dxN[i])[None]], axis=0)
            Un = (u[a:b] + du[a:b])[:, 0]
            np.testing.assert_allclose(Xn[0], x0[i], atol=1e-13)
            for k in range(N):  # gaps closed
                np.testing.assert_allclose(Xn[k + 1], Ad @ Xn[k] + Bd[:, 0] * Un[k], atol=1e-12)
            U, X = condensed_optimum(Ad, Bd, x0[i], N, xref[i], QN)
            np.testing.assert_allclose(Un, U, rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(Xn, X, rtol=1e-9, atol=1e-11)


def test_rti_with_residual_solves_its_linearised_problem():
    """With a residual the step is the minimiser of the LQ problem built from the
    oracle's own linearisation; the gaps and gradients are rebuilt here."""
    N = 6
    Ws, bs = di_net(2, 16, seed=11)
    net = MLP(Ws, bs)
    rng = np.random.default_rng(12)
    x = rng.normal(0, 1, (N, 2))
    u = rng.normal(0, 1, (N, 1))
    xN = rng.normal(0, 1, (1, 2))
    x0 = rng.normal(0, 1, (1, 2))
    du, dx, dxN, (xnext, A, B, _, _, c) = rti_step([0, N], x, u, xN, x0, net, DT, Q, R, Q)
    # the step is the minimiser over (dx, du) of the quadratic model with the rollout constraint
    def cost(dxs, dus):
        X = np.concatenate([x, xN], axis=0) + dxs
        return 0.5 * sum(X[k] @ Q @ X[k] for k in range(N + 1)) + 0.5 * float(np.sum((u + dus) ** 2) * R[0, 0])
    succ = np.concatenate([x[1:], xN], axis=0)
    np.testing.assert_allclose(c, xnext - succ, atol=0)
    def rollout(dus):
        dxs = np.zeros((N + 1, 2))
        dxs[0] = x0[0] - x[0]
        for k in range(N):
            dxs[k + 1] = A[k] @ dxs[k] + B[k] @ dus[k] + c[k]
        return dxs
    dxs = rollout(du)
    np.testing.assert_allclose(dxs[:-1], dx, atol=1e-12)
    np.testing.assert_allclose(dxs[-1], dxN[0], atol=1e-12)
    base = cost(dxs, du)
    for trial in range(20):  # every feasible perturbation costs more (strictly convex QP)
        pert = du + 1e-3 * rng.normal(0, 1, du.shape)
        assert cost(rollout(pert), pert) > base

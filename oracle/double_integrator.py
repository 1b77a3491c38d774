"""Runtime workload of the runtime analysis (Sec. V): a double
integrator with a network residual, solved by real-time iterations over N
shooting nodes -- TEST INFRASTRUCTURE (float64; only tests, the smoke check and
the CPU baseline of the benchmark use it).

Nominal model (the double-integrator equation of that section):
    x = [p, pdot],  f_F(x, u) = [pdot, u].
Residual f_D: a network from the state (2 values) to 2 values added to x-dot.
The paper does not print the network's input and output widths; the parameter
counts of its Table II (354 for two layers of 16, 17K for two of 128, 67K for
five of 128, 13M for fifty of 512) are those of a 2-input, 2-output network
with n_hidden hidden layers of the given width, which is the reading taken.
In the paper's runs the output layer is set so that f_D = 0; the arithmetic is
the same for any weights.

The local approximation is the first-order one of eq. (4) (Sec. IV-B), held
fixed inside one RK4 step (Sec. III):
    F(x) = f_F(x, u_k) + f_D-bar + J_D (x - x_k),
and the step's sensitivities A_k = d x_{k+1} / d x_k, B_k = d x_{k+1} / d u_k
(the continuity condition eq. (2) and the definitions after it).

One real-time iteration (Sec. IV-B: the preparation phase linearises at the
current iterate, the feedback phase solves the QP once the current state is
known) over instance i with iterate x_0..x_N, u_0..u_{N-1}:
    c_k = phi-bar_k - x_{k+1},            the multiple-shooting gaps
    q_k = Q (x_k - x_ref), r_k = R u_k,   q_N = Q_N (x_N - x_ref)
    dx_0 = x0_measured - x_0,
the LQ subproblem (oracle.riccati) gives du_k = K_k dx_k + kff_k and the
rollout dx_{k+1} = A_k dx_k + B_k du_k + c_k.  The tracking cost and its
weights are not printed for this experiment; Q = I, R = 0.1, Q_N = Q are the
values used by the tests and the benchmark.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .mlp import MLP
from .riccati import riccati, lq_rollout

NX, NU = 2, 1
RK4_C = (0.0, 0.5, 0.5, 1.0)
RK4_W = (1.0, 2.0, 2.0, 1.0)


def nominal_f(x: np.ndarray, u: np.ndarray) -> np.ndarray:
    """f_F(x, u) = [pdot, u] for x (n, 2), u (n, 1)."""
    return np.stack([x[:, 1], u[:, 0]], axis=1)


def nominal_jac(n: int):
    """(df_F/dx (n,2,2), df_F/du (n,2,1)); constant for the double integrator."""
    Fx = np.zeros((n, 2, 2))
    Fx[:, 0, 1] = 1.0
    Fu = np.zeros((n, 2, 1))
    Fu[:, 1, 0] = 1.0
    return Fx, Fu


def node_parameters(model: Optional[MLP], x: np.ndarray):
    """(f_D-bar (n,2), J_D (n,2,2)) at the nodes; zeros without a network."""
    n = x.shape[0]
    if model is None:
        return np.zeros((n, 2)), np.zeros((n, 2, 2))
    return model.jacobian(x)


def linearize(x: np.ndarray, u: np.ndarray, model: Optional[MLP], dt: float, params=None, xbar=None):
    """(x_next (n,2), A (n,2,2), B (n,2,1), f_D-bar (n,2), J_D (n,2,2)).

    The four RK4 stages of F with the tangent S_s = d x_s / d [x_k, u_k]
    carried beside each stage point: dK_s = (df_F/dx + J_D) S_s + [0 | df_F/du].
    The approximation's expansion point is x_k itself unless ``xbar`` gives it
    (with ``params``, to differentiate the step map with the model held fixed)."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n = x.shape[0]
    xbar = x if xbar is None else np.asarray(xbar, dtype=np.float64)
    y_bar, J = node_parameters(model, x) if params is None else (np.asarray(a, np.float64) for a in params)
    Fx, Fu = nominal_jac(n)
    S0 = np.zeros((n, 2, 3))
    S0[:, :, :2] = np.eye(2)
    k = np.zeros_like(x)
    dk = np.zeros((n, 2, 3))
    x_acc = np.zeros_like(x)
    S_acc = np.zeros_like(S0)
    for s in range(4):
        xs = x + RK4_C[s] * dt * k
        S = S0 + RK4_C[s] * dt * dk
        k = nominal_f(xs, u) + y_bar + np.einsum("nij,nj->ni", J, xs - xbar)
        dk = np.einsum("nij,njc->nic", Fx + J, S)
        dk[:, :, 2:] += Fu
        x_acc += RK4_W[s] * k
        S_acc += RK4_W[s] * dk
    x_next = x + dt / 6.0 * x_acc
    AB = S0 + dt / 6.0 * S_acc
    return x_next, AB[:, :, :2], AB[:, :, 2:], y_bar, J


def rti_step(offsets, x, u, xN, x0, model: Optional[MLP], dt: float, Q, R, QN, xref=None, params=None):
    """One real-time iteration for every CSR instance.

    x (n,2), u (n,1): iterate states x_0..x_{N_i-1} and inputs of each instance's
    nodes; xN (n_inst,2): terminal states; x0 (n_inst,2): measured states;
    xref (n_inst,2) or None (zero).  Returns du (n,1), dx (n,2), dxN (n_inst,2)
    and the linearisation (x_next, A, B, f_D-bar, J_D, c)."""
    offsets = np.asarray(offsets)
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    xN = np.asarray(xN, dtype=np.float64)
    x0 = np.asarray(x0, dtype=np.float64)
    Q, R, QN = (np.asarray(a, dtype=np.float64) for a in (Q, R, QN))
    n_inst = len(offsets) - 1
    xref = np.zeros((n_inst, 2)) if xref is None else np.asarray(xref, dtype=np.float64)
    x_next, A, B, y_bar, J = linearize(x, u, model, dt, params)
    n = x.shape[0]
    du = np.zeros((n, 1))
    dx = np.zeros((n, 2))
    dxN = np.zeros((n_inst, 2))
    c = np.zeros((n, 2))
    for i in range(n_inst):
        a, b = int(offsets[i]), int(offsets[i + 1])
        succ = np.concatenate([x[a + 1:b], xN[i:i + 1]], axis=0)  # x_{k+1} of every node
        c[a:b] = x_next[a:b] - succ
        q = (x[a:b] - xref[i]) @ Q.T
        r = u[a:b] @ R.T
        qN = QN @ (xN[i] - xref[i])
        K, kff, _ = riccati(A[a:b], B[a:b], Q, R, QN, c=c[a:b], q=q, r=r, qN=qN)
        ui, xi = lq_rollout(A[a:b], B[a:b], K, kff, x0[i] - x[a], c[a:b])
        du[a:b], dx[a:b], dxN[i] = ui, xi[:-1], xi[-1]
    return du, dx, dxN, (x_next, A, B, y_bar, J, c)

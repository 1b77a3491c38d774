"""Continuity parameters x_{k+1} = phi-bar_k, A_k, B_k in float64 -- TEST INFRASTRUCTURE.

Sec. IV-A: the QP's continuity condition (eq. (2)) needs, per shooting node,
phi-bar_k = phi(x_k, u_k, f, dt), A_k = d phi / d x_k and B_k = d phi / d u_k,
where phi is one explicit 4th-order Runge-Kutta step with the input held
constant over the step (Sec. III; Sec. VI uses RK4 for the quadrotor).

Real-time Neural MPC replaces the network inside phi by its first-order local
approximation about the node (eq. (4), first order per Sec. IV-B):

    f_D*(x, u) = f_D-bar + J_D [x - x_k; u - u_k]

whose parameters (x_k, u_k, f_D-bar, J_D) are held fixed while phi and its
derivatives are formed (they are passed to the QP builder as parameters,
Sec. IV-A).  ``linearize_affine`` computes exactly that: the RK4 step of
f_F + f_D* and the exact derivative of that discrete map, by carrying the
stage sensitivities through the four stages.

``linearize_exact`` is the "naive" linearisation of Sec. IV-A that evaluates
the network and its Jacobian at all four stage points (N*E function and
N*E*2 derivative evaluations); it serves only to measure the gap.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from workload import QUAD, QuadParams
from .quadrotor import nominal_f, nominal_jac
from .mlp import MLP, pack_input, residual_in_state, pack_input_mode, residual_in_state_mode, INPUT_FULL

RK4_C = (0.0, 0.5, 0.5, 1.0)
RK4_W = (1.0, 2.0, 2.0, 1.0)


def rk4_step(f, x: np.ndarray, u: np.ndarray, dt: float) -> np.ndarray:
    """One classical RK4 step of x-dot = f(x, u), u held constant."""
    k1 = f(x, u)
    k2 = f(x + 0.5 * dt * k1, u)
    k3 = f(x + 0.5 * dt * k2, u)
    k4 = f(x + dt * k3, u)
    return x + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def node_parameters(model: Optional[MLP], x: np.ndarray, u: np.ndarray, mode: int = INPUT_FULL):
    """f_D-bar (n,d_out), J_D (n,d_out,d_in) at the nodes (zeros without a network)."""
    n = x.shape[0]
    if model is None:
        return np.zeros((n, 6)), np.zeros((n, 6, 14))
    return model.jacobian(pack_input_mode(x, u, mode))


def affine_field(x_k, u_k, y_bar, J, quad: QuadParams = QUAD, mode: int = INPUT_FULL):
    """The frozen-parameter vector field F(x, u) = f_F(x, u) + f_D*(x, u)."""
    f_bar, J_x, J_u = residual_in_state_mode(np.asarray(y_bar, np.float64), np.asarray(J, np.float64),
                                             np.asarray(x_k, np.float64), np.asarray(u_k, np.float64), mode)
    x_k = np.asarray(x_k, dtype=np.float64)
    u_k = np.asarray(u_k, dtype=np.float64)

    def F(x, u):
        dx = x - x_k
        du = u - u_k
        return (nominal_f(x, u, quad) + f_bar
                + np.einsum("nij,nj->ni", J_x, dx) + np.einsum("nij,nj->ni", J_u, du))
    return F


def linearize_affine(x: np.ndarray, u: np.ndarray, model: Optional[MLP], dt: float,
                     quad: QuadParams = QUAD, params=None, mode: int = INPUT_FULL):
    """(x_next (n,13), A (n,13,13), B (n,13,4), f_D-bar (n,d_out), J_D (n,d_out,d_in)).

    ``params`` = (f_D-bar, J_D) supplies the local approximation's parameters
    directly (e.g. from a reduced-precision evaluation of the network); ``mode``
    selects the residual's input variant (the Jacobian w.r.t. the state then goes
    through v_B = conj(q) (.) v at the node)."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n = x.shape[0]
    if params is None:
        y_bar, J = node_parameters(model, x, u, mode)
    else:
        y_bar, J = (np.asarray(a, dtype=np.float64) for a in params)
    f_bar, J_x, J_u = residual_in_state_mode(y_bar, J, x, u, mode) if model is not None or params is not None \
        else residual_in_state(y_bar, J)

    # S = d x_s / d [x_k, u_k] (n, 13, 17); stage derivative K_s and dK_s.
    S0 = np.zeros((n, 13, 17))
    S0[:, :, :13] = np.eye(13)
    xs, S = x, S0
    x_acc = np.zeros_like(x)
    S_acc = np.zeros_like(S0)
    for s in range(4):
        if s > 0:
            xs = x + RK4_C[s] * dt * k
            S = S0 + RK4_C[s] * dt * dk
        Fx, Fu = nominal_jac(xs, u, quad)
        k = nominal_f(xs, u, quad) + f_bar + np.einsum("nij,nj->ni", J_x, xs - x)
        M = Fx + J_x
        dk = M @ S
        # the input enters directly through f_F and through J_u (zero-order hold on u_k)
        dk[:, :, 13:] += Fu + J_u
        # the linearisation point x_k is a parameter: the J_x (x_s - x_k) term contributes
        # J_x d x_s/d x_k only (already inside M @ S); nothing is differentiated w.r.t. it.
        x_acc = x_acc + RK4_W[s] * k
        S_acc = S_acc + RK4_W[s] * dk
    x_next = x + dt / 6.0 * x_acc
    AB = S0 + dt / 6.0 * S_acc
    return x_next, AB[:, :, :13], AB[:, :, 13:], y_bar, J


def affine_phi(x0: np.ndarray, u0: np.ndarray, x_k, u_k, y_bar, J, dt: float,
               quad: QuadParams = QUAD, mode: int = INPUT_FULL) -> np.ndarray:
    """phi(x0, u0) with the local approximation frozen at (x_k, u_k, y_bar, J)."""
    return rk4_step(affine_field(x_k, u_k, y_bar, J, quad, mode), np.asarray(x0, np.float64),
                    np.asarray(u0, np.float64), dt)


def exact_phi(x0: np.ndarray, u0: np.ndarray, model: Optional[MLP], dt: float,
              quad: QuadParams = QUAD) -> np.ndarray:
    """phi with the network itself evaluated at every stage (f = f_F + f_D)."""
    def F(x, u):
        out = nominal_f(x, u, quad)
        if model is not None:
            out = out.copy()
            out[:, 7:13] += model.forward(pack_input(x, u))
        return out
    return rk4_step(F, np.asarray(x0, np.float64), np.asarray(u0, np.float64), dt)


def linearize_exact(x: np.ndarray, u: np.ndarray, model: Optional[MLP], dt: float,
                    quad: QuadParams = QUAD):
    """Naive linearisation: network value and Jacobian at all four stage points."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n = x.shape[0]
    S0 = np.zeros((n, 13, 17))
    S0[:, :, :13] = np.eye(13)
    xs, S = x, S0
    x_acc = np.zeros_like(x)
    S_acc = np.zeros_like(S0)
    for s in range(4):
        if s > 0:
            xs = x + RK4_C[s] * dt * k
            S = S0 + RK4_C[s] * dt * dk
        y_s, J_s = node_parameters(model, xs, u)
        f_s, Jx_s, Ju_s = residual_in_state(y_s, J_s)
        Fx, Fu = nominal_jac(xs, u, quad)
        k = nominal_f(xs, u, quad) + f_s
        dk = (Fx + Jx_s) @ S
        dk[:, :, 13:] += Fu + Ju_s
        x_acc = x_acc + RK4_W[s] * k
        S_acc = S_acc + RK4_W[s] * dk
    x_next = x + dt / 6.0 * x_acc
    AB = S0 + dt / 6.0 * S_acc
    return x_next, AB[:, :, :13], AB[:, :, 13:]


# ---------------------------------------------------------------- second order
# eq. (4) with its second-order term: the local approximation about the node is
#     f_D**(x, u) = f_D-bar + J_D dz + 1/2 dz^T H_D dz,   dz = z_0(x, u) - z_0(x_k, u_k),
# (per output; z_0 = [v, w, q, u] is a linear selection of (x, u)), again with
# (x_k, u_k, f_D-bar, J_D, H_D) held fixed inside the RK4 step.  Its derivative
# w.r.t. the state or input is (J_D + H_D dz) applied to d z_0.

def quadratic_field(x_k, u_k, y_bar, J, H, quad: QuadParams = QUAD):
    z_k = pack_input(x_k, u_k)

    def F(x, u):
        dz = pack_input(x, u) - z_k
        y = y_bar + np.einsum("njc,nc->nj", J, dz) + 0.5 * np.einsum("nc,njcd,nd->nj", dz, H, dz)
        out = nominal_f(x, u, quad).copy()
        out[:, 7:13] += y
        return out
    return F


def quadratic_phi(x0, u0, x_k, u_k, y_bar, J, H, dt: float, quad: QuadParams = QUAD) -> np.ndarray:
    return rk4_step(quadratic_field(x_k, u_k, y_bar, J, H, quad), np.asarray(x0, np.float64),
                    np.asarray(u0, np.float64), dt)


def linearize_quadratic(x: np.ndarray, u: np.ndarray, model: Optional[MLP], dt: float,
                        quad: QuadParams = QUAD, params=None):
    """(x_next, A, B, f_D-bar, J_D, H_D): RK4 of f_F + f_D** and its exact derivative.
    ``params`` = (f_D-bar, J_D, H_D) supplies the approximation's parameters directly."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n = x.shape[0]
    if params is None:
        if model is None:
            y_bar, J, H = np.zeros((n, 6)), np.zeros((n, 6, 14)), np.zeros((n, 6, 14, 14))
        else:
            y_bar, J, H = model.hessian(pack_input(x, u))
    else:
        y_bar, J, H = (np.asarray(a, dtype=np.float64) for a in params)
    z_k = pack_input(x, u)
    S0 = np.zeros((n, 13, 17))
    S0[:, :, :13] = np.eye(13)
    xs, S = x, S0
    x_acc = np.zeros_like(x)
    S_acc = np.zeros_like(S0)
    for s in range(4):
        if s > 0:
            xs = x + RK4_C[s] * dt * k
            S = S0 + RK4_C[s] * dt * dk
        dz = pack_input(xs, u) - z_k
        y = y_bar + np.einsum("njc,nc->nj", J, dz) + 0.5 * np.einsum("nc,njcd,nd->nj", dz, H, dz)
        J_eff = J + np.einsum("njcd,nd->njc", H, dz)
        _, J_x, J_u = residual_in_state(y, J_eff)
        Fx, Fu = nominal_jac(xs, u, quad)
        k = nominal_f(xs, u, quad).copy()
        k[:, 7:13] += y
        dk = (Fx + J_x) @ S
        dk[:, :, 13:] += Fu + J_u
        x_acc = x_acc + RK4_W[s] * k
        S_acc = S_acc + RK4_W[s] * dk
    x_next = x + dt / 6.0 * x_acc
    AB = S0 + dt / 6.0 * S_acc
    return x_next, AB[:, :, :13], AB[:, :, 13:], y_bar, J, H

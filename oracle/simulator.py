"""Drag-augmented synthetic quadrotor plant and residual labels -- TEST INFRASTRUCTURE.

Sec. VII (system identification): each recorded transition is re-simulated
with the nominal model and the difference is the training label of the
residual network.  The paper's plants (a simplified simulator, a BEM
simulator, flight data) are not available; this synthetic plant stands in:

    f_sim(x, u) = f_F(x, u) + [0_7; q (.) F_B / m + eps_v; eps_w]
    v_B = conj(q) (.) v                                 (body-frame velocity)
    F_B = -diag(D) (|v_B| * v_B) - k_r (sum_i T_i) v_B  (quadratic body drag
                                                          and rotor drag)

with noise eps = [eps_v; eps_w] ~ N(0, sigma^2 I_6) drawn once per transition
and held constant over the step.  One step is one RK4 step of f_sim; the label
is ([v; w]^sim_{k+1} - [v; w]^nom_{k+1}) / dt, where "nom" is one RK4 step of
f_F from the same (x_k, u_k).
"""
from __future__ import annotations

import numpy as np

from workload import QUAD, QuadParams, TRAIN
from .quadrotor import nominal_f, quat_conj, quat_rotate
from .rk4 import rk4_step


def drag_accel(x: np.ndarray, u: np.ndarray, drag=TRAIN["drag"], rotor_drag=TRAIN["rotor_drag"],
               quad: QuadParams = QUAD) -> np.ndarray:
    """World-frame acceleration of the drag forces, (n, 3)."""
    q, v = x[:, 3:7], x[:, 7:10]
    v_B = quat_rotate(quat_conj(q), v)
    F_B = -np.asarray(drag) * np.abs(v_B) * v_B - rotor_drag * u.sum(axis=1, keepdims=True) * v_B
    return quat_rotate(q, F_B) / quad.mass


def sim_field(noise: np.ndarray, quad: QuadParams = QUAD, **kw):
    def f(x, u):
        out = nominal_f(x, u, quad).copy()
        out[:, 7:10] += drag_accel(x, u, quad=quad, **kw) + noise[:, 0:3]
        out[:, 10:13] += noise[:, 3:6]
        return out
    return f


def sim_step(x: np.ndarray, u: np.ndarray, dt: float, noise: np.ndarray,
             quad: QuadParams = QUAD) -> np.ndarray:
    return rk4_step(sim_field(noise, quad), np.asarray(x, np.float64), np.asarray(u, np.float64), dt)


def nominal_step(x: np.ndarray, u: np.ndarray, dt: float, quad: QuadParams = QUAD) -> np.ndarray:
    return rk4_step(lambda a, b: nominal_f(a, b, quad), np.asarray(x, np.float64),
                    np.asarray(u, np.float64), dt)


def make_transitions(x: np.ndarray, u: np.ndarray, dt: float, seed: int,
                     noise_std: float = TRAIN["noise_std"], quad: QuadParams = QUAD):
    """(x_next_sim (n,13), label (n,6)) for i.i.d. samples (x, u)."""
    rng = np.random.default_rng(seed)
    noise = rng.normal(0.0, noise_std, size=(x.shape[0], 6))
    xs = sim_step(x, u, dt, noise, quad)
    xn = nominal_step(x, u, dt, quad)
    label = np.concatenate([xs[:, 7:10] - xn[:, 7:10], xs[:, 10:13] - xn[:, 10:13]], axis=1) / dt
    return xs, label

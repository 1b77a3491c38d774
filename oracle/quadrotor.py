"""Nominal quadrotor model f_F (eq. (6), Sec. VI) in float64 -- TEST INFRASTRUCTURE.

State x = [p(3), q(4) = (q_w, q_x, q_y, q_z), v(3), w(3)], input u = rotor
thrusts T_0..T_3 (Sec. VI, nominal dynamics).  Quaternions are Hamilton
quaternions and the rotation of a vector is the product q v q-bar (Sec. VI,
Notation).  That product is used literally: for a quaternion that is not of
unit length (as happens at intermediate Runge-Kutta stages) it scales the
vector by |q|^2; nothing renormalises q.

Rotor geometry is read from Fig. quad_model: X configuration, rotor i at body
position r_i with arm length ``arm`` from the centre, x_B pointing between
rotors 0 and 3:
    r_0 = (+h, -h), r_1 = (-h, -h), r_2 = (-h, +h), r_3 = (+h, +h), h = arm/sqrt(2).
Spin directions from the figure's arrows: rotors 0 and 2 counter-clockwise,
rotors 1 and 3 clockwise (seen from above).  A rotor's drag torque on the body
opposes its spin with magnitude c_tau * T_i.
"""
from __future__ import annotations

import numpy as np

from workload import QUAD, QuadParams


def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product a (x) b, both (..., 4) in (w, x, y, z) order."""
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def quat_conj(q: np.ndarray) -> np.ndarray:
    return q * np.array([1.0, -1.0, -1.0, -1.0])


def pure(v: np.ndarray) -> np.ndarray:
    """Embed a 3-vector as the pure quaternion (0, v)."""
    return np.concatenate([np.zeros(v.shape[:-1] + (1,), dtype=v.dtype), v], axis=-1)


def quat_rotate(q: np.ndarray, v: np.ndarray) -> np.ndarray:
    """q (.) v = vector part of q (x) (0, v) (x) conj(q)  (Sec. VI, Notation)."""
    return quat_mul(quat_mul(q, pure(v)), quat_conj(q))[..., 1:]


def rotor_positions(quad: QuadParams = QUAD) -> np.ndarray:
    h = quad.arm / np.sqrt(2.0)
    return np.array([[h, -h, 0.0], [-h, -h, 0.0], [-h, h, 0.0], [h, h, 0.0]])


# +1 = counter-clockwise seen from above (positive about z_B), -1 = clockwise.
ROTOR_SPIN = np.array([1.0, -1.0, 1.0, -1.0])


def body_torque(u: np.ndarray, quad: QuadParams = QUAD) -> np.ndarray:
    """tau_B = sum_i r_i x (0, 0, T_i) - spin_i * c_tau * T_i * e_z."""
    r = rotor_positions(quad)
    T = np.asarray(u)
    T = T.astype(np.result_type(T, 1.0))
    thrust_vecs = np.zeros(T.shape + (3,), dtype=T.dtype)
    thrust_vecs[..., 2] = T
    arm_torque = np.cross(np.broadcast_to(r, thrust_vecs.shape), thrust_vecs).sum(axis=-2)
    drag = np.zeros_like(arm_torque)
    drag[..., 2] = -(ROTOR_SPIN * T).sum(axis=-1) * quad.c_tau
    return arm_torque + drag


def inertia(quad: QuadParams = QUAD) -> np.ndarray:
    return np.array([quad.Jx, quad.Jy, quad.Jz])


def nominal_f(x: np.ndarray, u: np.ndarray, quad: QuadParams = QUAD) -> np.ndarray:
    """x-dot = f_F(x, u), eq. (6).  x (n, 13), u (n, 4) -> (n, 13).

    Works for complex dtypes as well (used by the complex-step check)."""
    p, q, v, w = x[..., 0:3], x[..., 3:7], x[..., 7:10], x[..., 10:13]
    Jd = inertia(quad)
    T_B = np.zeros(u.shape[:-1] + (3,), dtype=np.result_type(u, 1.0))
    T_B[..., 2] = u.sum(axis=-1)
    p_dot = v
    q_dot = 0.5 * quat_mul(q, pure(w))
    g_W = np.array([0.0, 0.0, -quad.g])
    v_dot = quat_rotate(q, T_B) / quad.mass + g_W
    tau = body_torque(u, quad)
    w_dot = (tau - np.cross(w, Jd * w)) / Jd
    return np.concatenate([p_dot, q_dot, v_dot, w_dot], axis=-1)


def nominal_jac(x: np.ndarray, u: np.ndarray, quad: QuadParams = QUAD):
    """Hand-derived partials of eq. (6): (df/dx (n,13,13), df/du (n,13,4))."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n = x.shape[0]
    qw, qx, qy, qz = x[:, 3], x[:, 4], x[:, 5], x[:, 6]
    wx, wy, wz = x[:, 10], x[:, 11], x[:, 12]
    Jx, Jy, Jz = quad.Jx, quad.Jy, quad.Jz
    T = u.sum(axis=1)
    Fx = np.zeros((n, 13, 13))
    Fu = np.zeros((n, 13, 4))
    # p-dot = v
    for i in range(3):
        Fx[:, i, 7 + i] = 1.0
    # q-dot = 1/2 q (x) (0, w): derivative in q (columns w,x,y,z) ...
    Z = np.zeros(n)
    dq_dq = 0.5 * np.stack([
        np.stack([Z, -wx, -wy, -wz], axis=1),
        np.stack([wx, Z, wz, -wy], axis=1),
        np.stack([wy, -wz, Z, wx], axis=1),
        np.stack([wz, wy, -wx, Z], axis=1),
    ], axis=1)
    Fx[:, 3:7, 3:7] = dq_dq
    # ... and in w
    dq_dw = 0.5 * np.stack([
        np.stack([-qx, -qy, -qz], axis=1),
        np.stack([qw, -qz, qy], axis=1),
        np.stack([qz, qw, -qx], axis=1),
        np.stack([-qy, qx, qw], axis=1),
    ], axis=1)
    Fx[:, 3:7, 10:13] = dq_dw
    # v-dot = (T/m) d(q) + g with d = q (x) (0,0,1) (x) conj(q)
    d = np.stack([2 * (qx * qz + qw * qy), 2 * (qy * qz - qw * qx),
                  qw * qw - qx * qx - qy * qy + qz * qz], axis=1)
    dd_dq = np.stack([
        np.stack([2 * qy, 2 * qz, 2 * qw, 2 * qx], axis=1),
        np.stack([-2 * qx, -2 * qw, 2 * qz, 2 * qy], axis=1),
        np.stack([2 * qw, -2 * qx, -2 * qy, 2 * qz], axis=1),
    ], axis=1)
    Fx[:, 7:10, 3:7] = (T / quad.mass)[:, None, None] * dd_dq
    for i in range(4):
        Fu[:, 7:10, i] = d / quad.mass
    # w-dot = J^-1 (tau - w x J w)
    Fx[:, 10, 11] = -(Jz - Jy) * wz / Jx
    Fx[:, 10, 12] = -(Jz - Jy) * wy / Jx
    Fx[:, 11, 10] = -(Jx - Jz) * wz / Jy
    Fx[:, 11, 12] = -(Jx - Jz) * wx / Jy
    Fx[:, 12, 10] = -(Jy - Jx) * wy / Jz
    Fx[:, 12, 11] = -(Jy - Jx) * wx / Jz
    # torque is linear in the thrusts: column i is the torque of unit thrust on rotor i
    dtau = body_torque(np.eye(4), quad)  # (4 rotors, 3)
    Fu[:, 10:13, :] = (dtau / inertia(quad)).T[None]
    return Fx, Fu

"""Residual network f_D and its Jacobian J_D in float64 -- TEST INFRASTRUCTURE.

The learned part of the model partition f = f_F + f_D (Sec. III, eq. (1);
full residual model eq. (7)) is a multilayer perceptron

    z_0 = [v, w, q, u]  (14 values, raw, in this order)
    a_l = W_l h_{l-1} + b_l,  h_l = act(a_l),   l = 1..L      (h_0 = z_0)
    y   = W_{L+1} h_L + b_{L+1}                  (6 values)

with act = SiLU (a * logistic(a)) or identity.  Its output is placed in the
state derivative as f_D = [0_3 (p), 0_4 (q), y_0..2 (v-dot, world frame),
y_3..5 (w-dot, body frame)]; eq. (7) writes the two leading zero blocks as 0_2.

J_D = dy/dz_0 = W_{L+1} diag(act'(a_L)) W_L ... diag(act'(a_1)) W_1 (6 x 14) is the
chain rule written out; it is evaluated by reverse accumulation (6 outputs < 14
inputs).  f_D-bar and J_D at a node are the parameters of the local
approximation eq. (4) (Sec. IV-A).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

# z_0 index -> state index (columns of the state Jacobian the residual touches)
Z_V = slice(0, 3)    # v  -> x[7:10]
Z_W = slice(3, 6)    # w  -> x[10:13]
Z_Q = slice(6, 10)   # q  -> x[3:7]
Z_U = slice(10, 14)  # u
Z_TO_X = np.array([7, 8, 9, 10, 11, 12, 3, 4, 5, 6])


# residual input variants (Sec. VI, simplified residual models): the full model
# [v, w, q, u] -> 6 outputs, and the linear-acceleration models f_Da(v_B) and
# f_Da,u(v_B, u) -> 3 outputs, v_B = conj(q) (.) v the body-frame velocity
INPUT_FULL, INPUT_VB, INPUT_VB_U = 0, 1, 2
D_IN = {INPUT_FULL: 14, INPUT_VB: 3, INPUT_VB_U: 7}
D_OUT = {INPUT_FULL: 6, INPUT_VB: 3, INPUT_VB_U: 3}


def body_velocity(x: np.ndarray) -> np.ndarray:
    """v_B = conj(q) (.) v (the homogeneous form, like every q (.) v here)."""
    from .quadrotor import quat_conj, quat_rotate
    return quat_rotate(quat_conj(x[:, 3:7]), x[:, 7:10])


def pack_input_mode(x: np.ndarray, u: np.ndarray, mode: int) -> np.ndarray:
    if mode == INPUT_FULL:
        return pack_input(x, u)
    vb = body_velocity(np.asarray(x))
    return vb if mode == INPUT_VB else np.concatenate([vb, np.asarray(u, dtype=vb.dtype)], axis=1)


def input_jacobian(x: np.ndarray, u: np.ndarray, mode: int):
    """(dz/dx (n, d_in, 13), dz/du (n, d_in, 4)) of the network input at (x, u), by
    complex-step differentiation of pack_input_mode (exact to rounding)."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n, h = x.shape[0], 1e-30
    dzx = np.zeros((n, D_IN[mode], 13))
    dzu = np.zeros((n, D_IN[mode], 4))
    for i in range(13):
        xc = x.astype(complex)
        xc[:, i] += 1j * h
        dzx[:, :, i] = pack_input_mode(xc, u.astype(complex), mode).imag / h
    for i in range(4):
        uc = u.astype(complex)
        uc[:, i] += 1j * h
        dzu[:, :, i] = pack_input_mode(x.astype(complex), uc, mode).imag / h
    return dzx, dzu


def pack_input(x: np.ndarray, u: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    return np.concatenate([x[:, 7:10], x[:, 10:13], x[:, 3:7], u], axis=1)


def logistic(a):
    return 1.0 / (1.0 + np.exp(-a))


def silu(a):
    return a * logistic(a)


def silu_prime(a):
    s = logistic(a)
    return s * (1.0 + a * (1.0 - s))


def silu_second(a):
    """d^2/da^2 of a * logistic(a) = s (1 - s) (2 + a (1 - 2 s))."""
    s = logistic(a)
    return s * (1.0 - s) * (2.0 + a * (1.0 - 2.0 * s))


class MLP:
    """Float64 view of a residual network.  ``Ws[l]`` is (fan_out, fan_in)."""

    def __init__(self, Ws: Sequence[np.ndarray], bs: Sequence[np.ndarray], act: str = "silu"):
        self.Ws = [np.asarray(W, dtype=np.float64) for W in Ws]
        self.bs = [np.asarray(b, dtype=np.float64) for b in bs]
        if act not in ("silu", "identity"):
            raise ValueError(act)
        self.act = act

    @property
    def n_hidden(self) -> int:
        return len(self.Ws) - 1

    def _act(self, a):
        return silu(a) if self.act == "silu" else a

    def _act_prime(self, a):
        return silu_prime(a) if self.act == "silu" else np.ones_like(a)

    def _act_second(self, a):
        return silu_second(a) if self.act == "silu" else np.zeros_like(a)

    def forward(self, z: np.ndarray, keep: bool = False):
        """y (n, 6); with keep=True also the pre-activations a_1..a_L.  Complex inputs
        stay complex (complex-step differentiation in the tests)."""
        z = np.asarray(z)
        h = np.asarray(z, dtype=np.result_type(z, 1.0))
        pre = []
        for W, b in zip(self.Ws[:-1], self.bs[:-1]):
            a = h @ W.T + b
            pre.append(a)
            h = self._act(a)
        y = h @ self.Ws[-1].T + self.bs[-1]
        return (y, pre) if keep else y

    def jacobian(self, z: np.ndarray):
        """(y (n,6), J_D (n,6,14)) by reverse accumulation of the chain rule."""
        y, pre = self.forward(z, keep=True)
        n = y.shape[0]
        G = np.broadcast_to(self.Ws[-1], (n,) + self.Ws[-1].shape)
        for l in range(self.n_hidden - 1, -1, -1):
            G = (G * self._act_prime(pre[l])[:, None, :]) @ self.Ws[l]
        return y, np.ascontiguousarray(G)


    def hessian(self, z: np.ndarray):
        """(y (n,6), J_D (n,6,14), H_D (n,6,14,14)): the second derivatives of the outputs
        w.r.t. z_0 by the chain rule of second order,

            H_j = sum_l T_l^T diag((dy_j/dh_l) * act''(a_l)) T_l,   T_l = da_l/dz_0,

        with T_1 = W_1, T_l = W_l diag(act'(a_{l-1})) T_{l-1} (tangents, forward) and
        dy/dh_L = W_{L+1}, dy/dh_{l-1} = (dy/dh_l * act'(a_l)) W_l (adjoints, reverse);
        the last adjoint is J_D."""
        y, pre = self.forward(z, keep=True)
        n, L = y.shape[0], self.n_hidden
        T = [np.broadcast_to(self.Ws[0], (n,) + self.Ws[0].shape)]
        for l in range(1, L):
            T.append(np.einsum("fg,ngc->nfc", self.Ws[l], self._act_prime(pre[l - 1])[:, :, None] * T[l - 1]))
        Hs = np.zeros((n, 6, z.shape[1], z.shape[1]), dtype=np.result_type(z, 1.0))
        U = np.broadcast_to(self.Ws[-1], (n,) + self.Ws[-1].shape)  # dy/dh_L
        for l in range(L - 1, -1, -1):
            w = U * self._act_second(pre[l])[:, None, :]
            Hs = Hs + np.einsum("nfc,njf,nfd->njcd", T[l], w, T[l])
            U = (U * self._act_prime(pre[l])[:, None, :]) @ self.Ws[l]
        return y, np.ascontiguousarray(U), Hs


def residual_in_state(y: np.ndarray, J: np.ndarray):
    """Scatter the network value/Jacobian into state coordinates (eq. (7)).

    Returns f_bar (n,13), J_x (n,13,13), J_u (n,13,4)."""
    n = y.shape[0]
    f_bar = np.zeros((n, 13))
    f_bar[:, 7:13] = y
    J_x = np.zeros((n, 13, 13))
    J_x[:, 7:13, Z_TO_X] = J[:, :, 0:10]
    J_u = np.zeros((n, 13, 4))
    J_u[:, 7:13, :] = J[:, :, 10:14]
    return f_bar, J_x, J_u


def residual_in_state_mode(y: np.ndarray, J: np.ndarray, x: np.ndarray, u: np.ndarray, mode: int):
    """As residual_in_state for any input variant: the outputs fill v-dot (and w-dot for
    the full model); the state/input Jacobians are J dz/dx and J dz/du at the node."""
    if mode == INPUT_FULL:
        return residual_in_state(y, J)
    n, d = y.shape
    dzx, dzu = input_jacobian(x, u, mode)
    f_bar = np.zeros((n, 13))
    f_bar[:, 7:7 + d] = y
    J_x = np.zeros((n, 13, 13))
    J_x[:, 7:7 + d, :] = J @ dzx
    J_u = np.zeros((n, 13, 4))
    J_u[:, 7:7 + d, :] = J @ dzu
    return f_bar, J_x, J_u


def residual_value(model: Optional[MLP], x: np.ndarray, u: np.ndarray) -> np.ndarray:
    """f_D(x, u) as a 13-vector field (zeros without a network)."""
    n = x.shape[0]
    out = np.zeros((n, 13), dtype=np.result_type(x, 1.0))
    if model is not None:
        out[:, 7:13] = model.forward(pack_input(x, u))
    return out


def flatten_params(Ws: List[np.ndarray], bs: List[np.ndarray]) -> np.ndarray:
    """Parameters as one vector, layer by layer: W_l row-major then b_l."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in zip(Ws, bs)])

"""Feedback-phase LQ solve in float64 -- TEST INFRASTRUCTURE.

The QP of Sec. IV-A with a Gauss-Newton Hessian of the quadratic tracking cost
(Sec. VI, MPC cost formulation) and the continuity condition eq. (2), without
the inequality rows eq. (3):

    min  sum_{k<N} 1/2 [dx;du]^T blkdiag(Q,R) [dx;du] + q_k^T dx + r_k^T du
         + 1/2 dx_N^T Q_N dx_N + q_N^T dx_N
    s.t. dx_{k+1} = A_k dx_k + B_k du_k + c_k,   c_k = phi-bar_k - x_{k+1}

The optimal step is du_k = K_k dx_k + kff_k.  ``riccati`` is the backward
dynamic-programming recursion; ``kkt_bruteforce`` solves the same QP as one
dense equality-constrained linear system and is used only to check it.
"""
from __future__ import annotations

from typing import Optional

import numpy as np


def riccati(A, B, Q, R, QN, c=None, q=None, r=None, qN=None):
    """One instance.  A (N,13,13), B (N,13,4) -> K (N,4,13), kff (N,4), P (N+1,13,13).

    The value function after step k is 1/2 dx^T P_k dx + p_k^T dx."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    N, nx, nu = B.shape
    c = np.zeros((N, nx)) if c is None else np.asarray(c, dtype=np.float64)
    q = np.zeros((N, nx)) if q is None else np.asarray(q, dtype=np.float64)
    r = np.zeros((N, nu)) if r is None else np.asarray(r, dtype=np.float64)
    qN = np.zeros(nx) if qN is None else np.asarray(qN, dtype=np.float64)
    K = np.zeros((N, nu, nx))
    kff = np.zeros((N, nu))
    Ps = np.zeros((N + 1, nx, nx))
    P = np.array(QN, dtype=np.float64)
    p = qN.copy()
    Ps[N] = P
    for k in range(N - 1, -1, -1):
        Ak, Bk = A[k], B[k]
        Qxx = Q + Ak.T @ P @ Ak
        Quu = R + Bk.T @ P @ Bk
        Qux = Bk.T @ P @ Ak
        gvec = P @ c[k] + p
        qx = q[k] + Ak.T @ gvec
        qu = r[k] + Bk.T @ gvec
        K[k] = -np.linalg.solve(Quu, Qux)
        kff[k] = -np.linalg.solve(Quu, qu)
        P = Qxx + Qux.T @ K[k]
        P = 0.5 * (P + P.T)
        p = qx + Qux.T @ kff[k]
        Ps[k] = P
    return K, kff, Ps


def riccati_batched(offsets, A, B, Q, R, QN, c=None, q=None, r=None, qN=None):
    """Apply ``riccati`` to each CSR instance range.  Returns K, kff, P (node-major)."""
    offsets = np.asarray(offsets)
    n = int(offsets[-1])
    nx, nu = B.shape[1], B.shape[2]
    K = np.zeros((n, nu, nx))
    kff = np.zeros((n, nu))
    P = np.zeros((n, nx, nx))
    for i in range(len(offsets) - 1):
        a, b = int(offsets[i]), int(offsets[i + 1])
        Ki, ki, Pi = riccati(A[a:b], B[a:b], Q, R, QN,
                             None if c is None else c[a:b],
                             None if q is None else q[a:b],
                             None if r is None else r[a:b],
                             None if qN is None else qN[i])
        K[a:b], kff[a:b], P[a:b] = Ki, ki, Pi[:-1]
    return K, kff, P


def kkt_bruteforce(A, B, Q, R, QN, dx0, c=None, q=None, r=None, qN=None):
    """Solve the whole QP for a given initial deviation dx0 as one KKT system.

    Decision vector z = [dx_0, du_0, dx_1, du_1, ..., dx_N].  Returns (du (N,4), dx (N+1,13))."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    N, nx, nu = B.shape
    c = np.zeros((N, nx)) if c is None else c
    q = np.zeros((N, nx)) if q is None else q
    r = np.zeros((N, nu)) if r is None else r
    qN = np.zeros(nx) if qN is None else qN
    nz = N * (nx + nu) + nx
    H = np.zeros((nz, nz))
    h = np.zeros(nz)

    def xi(k):
        return k * (nx + nu)

    def ui(k):
        return k * (nx + nu) + nx

    for k in range(N):
        H[xi(k):xi(k) + nx, xi(k):xi(k) + nx] = Q
        H[ui(k):ui(k) + nu, ui(k):ui(k) + nu] = R
        h[xi(k):xi(k) + nx] = q[k]
        h[ui(k):ui(k) + nu] = r[k]
    H[xi(N):xi(N) + nx, xi(N):xi(N) + nx] = QN
    h[xi(N):xi(N) + nx] = qN
    # equality rows: dx_0 = dx0;  dx_{k+1} - A dx_k - B du_k = c_k
    neq = (N + 1) * nx
    E = np.zeros((neq, nz))
    e = np.zeros(neq)
    E[0:nx, 0:nx] = np.eye(nx)
    e[0:nx] = dx0
    for k in range(N):
        rows = slice((k + 1) * nx, (k + 2) * nx)
        E[rows, xi(k + 1):xi(k + 1) + nx] = np.eye(nx)
        E[rows, xi(k):xi(k) + nx] = -A[k]
        E[rows, ui(k):ui(k) + nu] = -B[k]
        e[rows] = c[k]
    KKT = np.block([[H, E.T], [E, np.zeros((neq, neq))]])
    rhs = np.concatenate([-h, e])
    sol = np.linalg.solve(KKT, rhs)
    z = sol[:nz]
    du = np.stack([z[ui(k):ui(k) + nu] for k in range(N)])
    dx = np.stack([z[xi(k):xi(k) + nx] for k in range(N + 1)])
    return du, dx


def lq_rollout(A, B, K, kff, dx0, c=None):
    """Forward pass of the LQ solution of one instance (the primal step of the QP):
    du_k = K_k dx_k + kff_k,  dx_{k+1} = A_k dx_k + B_k du_k + c_k  from dx_0 = dx0.

    Returns du (N,4) and dx (N+1,13), which equal the QP's minimiser
    (``kkt_bruteforce``) when K, kff come from ``riccati`` on the same data."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    N, nx, nu = B.shape
    c = np.zeros((N, nx)) if c is None else np.asarray(c, dtype=np.float64)
    dx = np.zeros((N + 1, nx))
    du = np.zeros((N, nu))
    dx[0] = dx0
    for k in range(N):
        du[k] = K[k] @ dx[k] + kff[k]
        dx[k + 1] = A[k] @ dx[k] + B[k] @ du[k] + c[k]
    return du, dx


def lq_rollout_batched(offsets, A, B, K, kff, dx0, c=None):
    """``lq_rollout`` per CSR instance.  dx0 (n_inst,13) -> du (n,4), dx (n,13) for
    k = 0..N_i-1 and the terminal dx_N (n_inst,13)."""
    offsets = np.asarray(offsets)
    n = int(offsets[-1])
    nx, nu = B.shape[1], B.shape[2]
    du = np.zeros((n, nu))
    dx = np.zeros((n, nx))
    dxN = np.zeros((len(offsets) - 1, nx))
    for i in range(len(offsets) - 1):
        a, b = int(offsets[i]), int(offsets[i + 1])
        ui, xi = lq_rollout(A[a:b], B[a:b], K[a:b], kff[a:b], dx0[i], None if c is None else c[a:b])
        du[a:b], dx[a:b], dxN[i] = ui, xi[:-1], xi[-1]
    return du, dx, dxN


# ---------------------------------------------------------------- input box
# The QP of Sec. IV-A with the inequality rows eq. (3) restricted to the input
# box: lo_k <= du_k <= hi_k (for 0 <= u <= u_max: lo = -u_k, hi = u_max - u_k).

def condense(A, B, Q, R, QN, dx0, c=None, q=None, r=None, qN=None):
    """Eliminate the states: dx = S du + s (stacked dx_1..dx_N), so the QP becomes
    min 1/2 du^T H du + h^T du over the stacked du (N*4).  Returns H, h, S, s."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    N, nx, nu = B.shape
    c = np.zeros((N, nx)) if c is None else np.asarray(c, dtype=np.float64)
    q = np.zeros((N, nx)) if q is None else np.asarray(q, dtype=np.float64)
    r = np.zeros((N, nu)) if r is None else np.asarray(r, dtype=np.float64)
    qN = np.zeros(nx) if qN is None else np.asarray(qN, dtype=np.float64)
    S = np.zeros((N * nx, N * nu))  # rows: dx_{k+1}
    s = np.zeros(N * nx)
    x_prev, S_prev = np.asarray(dx0, dtype=np.float64), np.zeros((nx, N * nu))
    for k in range(N):
        S_k = A[k] @ S_prev
        S_k[:, k * nu:(k + 1) * nu] += B[k]
        x_k = A[k] @ x_prev + c[k]
        S[k * nx:(k + 1) * nx], s[k * nx:(k + 1) * nx] = S_k, x_k
        S_prev, x_prev = S_k, x_k
    # state cost weights of dx_1..dx_N (dx_0 is fixed); linear terms q_k act on dx_k
    W = np.zeros((N * nx, N * nx))
    w = np.zeros(N * nx)
    for k in range(1, N):
        W[(k - 1) * nx:k * nx, (k - 1) * nx:k * nx] = Q
        w[(k - 1) * nx:k * nx] = q[k]
    W[(N - 1) * nx:, (N - 1) * nx:] = QN
    w[(N - 1) * nx:] = qN
    H = S.T @ W @ S + np.kron(np.eye(N), R)
    h = S.T @ (W @ s + w) + r.reshape(-1)
    return H, h, S, s


def box_lq(A, B, Q, R, QN, dx0, lo, hi, c=None, q=None, r=None, qN=None):
    """Exact minimiser of the box-constrained LQ of one instance: the condensed QP
    written as a bounded least-squares problem (H = L L^T) and solved by SciPy's
    bounded-variable least squares (an active-set method that ends at the exact
    solution).  Returns du (N,4) and dx (N+1,13)."""
    import scipy.linalg
    import scipy.optimize
    N, nx, nu = np.asarray(B).shape
    H, h, S, s = condense(A, B, Q, R, QN, dx0, c, q, r, qN)
    L = np.linalg.cholesky(H)
    # 1/2 x^T H x + h^T x = 1/2 |L^T x + L^{-1} h|^2 + const
    rhs = -scipy.linalg.solve_triangular(L, h, lower=True)
    res = scipy.optimize.lsq_linear(L.T, rhs, bounds=(np.asarray(lo).reshape(-1), np.asarray(hi).reshape(-1)),
                                    method="bvls", tol=1e-14, lsmr_tol=None)
    du = res.x
    dx = np.concatenate([np.asarray(dx0, dtype=np.float64), S @ du + s]).reshape(N + 1, nx)
    return du.reshape(N, nu), dx


def box_lq_bruteforce(A, B, Q, R, QN, dx0, lo, hi, c=None, q=None, r=None, qN=None):
    """Enumerate every assignment of each input component to {lower bound, upper
    bound, free}, solve the equality-reduced QP, keep the feasible candidate with the
    lowest cost.  Tiny instances only (3^(4N) systems)."""
    import itertools
    N, nx, nu = np.asarray(B).shape
    H, h, S, s = condense(A, B, Q, R, QN, dx0, c, q, r, qN)
    lo, hi = np.asarray(lo).reshape(-1), np.asarray(hi).reshape(-1)
    nv = N * nu
    best, best_x = np.inf, None
    for assign in itertools.product((0, 1, 2), repeat=nv):
        a = np.array(assign)
        x = np.where(a == 0, lo, np.where(a == 1, hi, 0.0))
        free = a == 2
        if free.any():
            Hff = H[np.ix_(free, free)]
            x[free] = np.linalg.solve(Hff, -(h[free] + H[np.ix_(free, ~free)] @ x[~free]))
            if np.any(x[free] < lo[free] - 1e-12) or np.any(x[free] > hi[free] + 1e-12):
                continue
        f = 0.5 * x @ H @ x + h @ x
        if f < best - 1e-13:
            best, best_x = f, x
    dx = np.concatenate([np.asarray(dx0, dtype=np.float64), S @ best_x + s]).reshape(N + 1, nx)
    return best_x.reshape(N, nu), dx

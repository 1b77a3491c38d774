"""Closed-loop real-time-iteration driver over the library's GPU calls -- TEST INFRASTRUCTURE.

One control tick per step, for a batch of MPC instances that each track a
horizontal circle (the feedback loop of Sec. IV-B around the QP of Sec. IV-A):

  1. rtn_linearize on the current iterate (x_k, u_k), k = 0..N-1  -> phi-bar_k, A_k, B_k
  2. defects c_k = phi-bar_k - x_{k+1} (x_N: the iterate's terminal state) and the
     gradient terms of the tracking cost q_k = Q (x_k - x_ref,k), r_k = R (u_k - u_hover)
  3. rtn_riccati -> K_k, kff_k;  rtn_lq_rollout from dx_0 = x_plant - x_0 -> dx_k, du_k
     (with ``box=True`` instead rtn_riccati_box with 0 <= u_k + du_k <= u_max)
  4. apply u = clip(u_0 + du_0, 0, u_max) to the plant: one RK4 step of the drag-augmented
     synthetic quadrotor with per-step acceleration noise (the training data's simulator)
  5. record the model's one-step prediction phi-bar_0 + A_0 dx_0 + B_0 (u - u_0) against
     the plant's next state, and the position tracking error
  6. take the full step on the iterate and shift it by one node.

With ``model=None`` the linearisation uses the nominal model alone (the fallback).
"""
from __future__ import annotations

import numpy as np

from workload import QUAD, hover_thrust
from oracle.simulator import sim_step

U_MAX = 4.0


def circle_reference(t: np.ndarray, radius, omega, phase) -> np.ndarray:
    """(n_inst, len(t), 13) states on horizontal circles: level attitude, zero body rates."""
    a = omega[:, None] * t[None, :] + phase[:, None]
    x = np.zeros((radius.size, t.size, 13))
    x[:, :, 0] = radius[:, None] * np.cos(a)
    x[:, :, 1] = radius[:, None] * np.sin(a)
    x[:, :, 3] = 1.0
    x[:, :, 7] = -radius[:, None] * omega[:, None] * np.sin(a)
    x[:, :, 8] = radius[:, None] * omega[:, None] * np.cos(a)
    return x


def run(torch, rtn, model, prec: str, n_inst: int = 4096, N: int = 20, dt: float = 0.05,
        steps: int = 40, seed: int = 5, noise_std: float = 0.05, device: str = "cuda", box: bool = False):
    rng = np.random.default_rng(seed)
    radius = rng.uniform(2.0, 4.0, n_inst)
    speed = rng.uniform(2.0, 4.0, n_inst)
    omega, phase = speed / radius, rng.uniform(0.0, 2 * np.pi, n_inst)
    noise = rng.normal(0.0, noise_std, size=(steps, n_inst, 6))
    uh = hover_thrust(QUAD)
    Q = np.diag([10.0] * 3 + [1.0] * 4 + [1.0] * 3 + [0.1] * 3)
    R = 0.1 * np.eye(4)
    dev = torch.device(device)
    Qt, Rt = torch.from_numpy(Q).to(dev), torch.from_numpy(R).to(dev)
    off = np.arange(0, n_inst * N + 1, N, dtype=np.int32)

    Xit = torch.from_numpy(circle_reference(np.arange(N) * dt, radius, omega, phase)).to(dev)
    Uit = torch.full((n_inst, N, 4), uh, dtype=torch.float64, device=dev)
    Xterm = torch.from_numpy(circle_reference(np.array([N * dt]), radius, omega, phase)[:, 0]).to(dev)
    xa = Xit[:, 0].cpu().numpy().copy()
    pred_err, track_err = [], []
    for t in range(steps):
        ref = torch.from_numpy(circle_reference(t * dt + np.arange(N + 1) * dt, radius, omega, phase)).to(dev)
        xin = Xit.reshape(-1, 13).float().contiguous()
        uin = Uit.reshape(-1, 4).float().contiguous()
        lin = rtn.linearize(xin, uin, model, prec, dt, offsets=off)
        phi = lin["x_next"].view(n_inst, N, 13).double()
        nxt = torch.cat([Xit[:, 1:], Xterm[:, None]], dim=1)
        c = (phi - nxt).reshape(-1, 13).contiguous()
        qv = ((Xit - ref[:, :N]) @ Qt).reshape(-1, 13).contiguous()
        rv = ((Uit - uh) @ Rt).reshape(-1, 4).contiguous()
        qN = ((Xterm - ref[:, N]) @ Qt).contiguous()
        dx0 = (torch.from_numpy(xa).to(dev) - Xit[:, 0]).contiguous()
        if box:
            lo = (-Uit).reshape(-1, 4).contiguous()
            hi = (U_MAX - Uit).reshape(-1, 4).contiguous()
            roll = rtn.riccati_box(lin["A"], lin["B"], Q, R, Q, dx0, lo, hi, offsets=off, c=c, q=qv, r=rv, qN=qN,
                                   rho=1.0, max_iter=200, tol=1e-6)
        else:
            ric = rtn.riccati(lin["A"], lin["B"], Q, R, Q, offsets=off, c=c, q=qv, r=rv, qN=qN)
            roll = rtn.lq_rollout(lin["A"], lin["B"], ric["K"], ric["kff"], dx0, offsets=off, c=c)
        du = roll["du"].view(n_inst, N, 4)
        dx = roll["dx"].view(n_inst, N, 13)
        u0 = torch.clamp(Uit[:, 0] + du[:, 0], 0.0, U_MAX)
        A0 = lin["A"].view(n_inst, N, 13, 13)[:, 0].double().contiguous()
        B0 = lin["B"].view(n_inst, N, 13, 4)[:, 0].double().contiguous()
        pred = phi[:, 0] + (A0 @ dx0[:, :, None])[:, :, 0] + (B0 @ (u0 - Uit[:, 0])[:, :, None])[:, :, 0]
        xa = sim_step(xa, u0.cpu().numpy(), dt, noise[t], QUAD)
        pred = pred.cpu().numpy()
        pred_err.append(np.linalg.norm(pred[:, 7:13] - xa[:, 7:13], axis=1))
        track_err.append(np.linalg.norm(xa[:, 0:3] - ref[:, 1, 0:3].cpu().numpy(), axis=1))
        Xnew, Unew = Xit + dx, torch.clamp(Uit + du, 0.0, U_MAX)
        Xterm = Xterm + roll["dxN"]
        Xit = torch.cat([Xnew[:, 1:], Xterm[:, None]], dim=1)
        Uit = torch.cat([Unew[:, 1:], Unew[:, -1:]], dim=1)
    pred_err, track_err = np.array(pred_err), np.array(track_err)
    return {"pred_err": float(pred_err.mean()), "track_err": float(track_err.mean()),
            "finite": bool(np.all(np.isfinite(xa))), "speed": float(np.linalg.norm(xa[:, 7:10], axis=1).mean())}

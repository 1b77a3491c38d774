"""Pins of the oracle's training reference, simulator and rounding emulation."""
import numpy as np
import pytest
import torch

from workload import QUAD, sample_nodes, xavier_params
from oracle.mlp import MLP, pack_input
from oracle.train import mse_and_grads, Adam, train_step
from oracle.simulator import make_transitions, drag_accel
from oracle.quant import round_bf16, round_e4m3


def test_mse_gradients_finite_differences():
    Ws, bs = xavier_params(2, 12, seed=3)
    bs = [np.random.default_rng(5).normal(size=b.shape) * 0.2 for b in bs]
    net = MLP(Ws, bs)
    x, u = sample_nodes(9, seed=6)
    z = pack_input(x, u)
    tgt = np.random.default_rng(7).normal(size=(9, 6))
    loss, dWs, dbs, dz = mse_and_grads(net, z, tgt)
    h = 1e-6
    for l in range(len(Ws)):
        for idx in [(0, 0), (1, 2), (Ws[l].shape[0] - 1, Ws[l].shape[1] - 1)]:
            P = [W.astype(np.float64).copy() for W in Ws]
            P[l][idx] += h
            lp = mse_and_grads(MLP(P, net.bs), z, tgt)[0]
            P[l][idx] -= 2 * h
            lm = mse_and_grads(MLP(P, net.bs), z, tgt)[0]
            assert abs((lp - lm) / (2 * h) - dWs[l][idx]) < 1e-8
        bP = [b.copy() for b in net.bs]
        bP[l][0] += h
        lp = mse_and_grads(MLP(net.Ws, bP), z, tgt)[0]
        bP[l][0] -= 2 * h
        lm = mse_and_grads(MLP(net.Ws, bP), z, tgt)[0]
        assert abs((lp - lm) / (2 * h) - dbs[l][0]) < 1e-8
    zp = z.copy(); zp[2, 5] += h
    zm = z.copy(); zm[2, 5] -= h
    fd = (mse_and_grads(net, zp, tgt)[0] - mse_and_grads(net, zm, tgt)[0]) / (2 * h)
    assert abs(fd - dz[2, 5]) < 1e-8


def test_zero_hidden_layer_gradient_closed_form():
    """y = W z + b: dL/dW = 2 (W z + b - y*) z^T / (6 B)."""
    rng = np.random.default_rng(1)
    W = rng.normal(size=(6, 14)); b = rng.normal(size=6)
    z = rng.normal(size=(5, 14)); tgt = rng.normal(size=(5, 6))
    loss, dWs, dbs, _ = mse_and_grads(MLP([W], [b]), z, tgt)
    err = z @ W.T + b - tgt
    np.testing.assert_allclose(dWs[0], 2 * err.T @ z / 30, atol=1e-14)
    np.testing.assert_allclose(dbs[0], 2 * err.sum(0) / 30, atol=1e-14)
    assert abs(loss - np.mean(err ** 2)) < 1e-14


def test_adam_first_two_steps_by_hand():
    """From zero moments the first bias-corrected step is lr * g / (|g| + eps)."""
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    p = np.array([0.5, -1.0, 2.0])
    g1 = np.array([0.1, -3.0, 0.0])
    g2 = np.array([-0.2, 1.0, 4.0])
    opt = Adam([p], lr, b1, b2, eps)
    p1 = opt.step([p], [g1])[0]
    np.testing.assert_allclose(p1, p - lr * g1 / (np.abs(g1) + eps), atol=1e-15)
    p2 = opt.step([p1], [g2])[0]
    m = 0.9 * 0.1 * g1 + 0.1 * g2
    v = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    ref = p1 - lr * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + eps)
    np.testing.assert_allclose(p2, ref, atol=1e-15)


def test_training_reduces_loss():
    Ws, bs = xavier_params(1, 16, seed=2)
    net = MLP(Ws, bs)
    rng = np.random.default_rng(3)
    z = rng.normal(size=(64, 14)); tgt = np.tanh(z[:, :6])
    opt = Adam(net.Ws + net.bs, lr=1e-2)
    first = None
    for _ in range(100):
        loss, net = train_step(net, opt, z, tgt)
        first = loss if first is None else first
    assert loss < 0.3 * first


def test_simulator_label_tends_to_drag_plus_noise():
    """Label = ([v;w]_sim - [v;w]_nom)/dt -> [drag accel + eps_v; eps_w] with error O(dt)."""
    x, u = sample_nodes(200, seed=8)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        _, label = make_transitions(x, u, dt, seed=9)
        noise = np.random.default_rng(9).normal(0.0, 0.05, size=(200, 6))
        ref = np.concatenate([drag_accel(x.astype(float), u.astype(float)), np.zeros((200, 3))], 1) + noise
        errs.append(np.max(np.abs(label - ref)))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 2.0) < 0.3), ratios


def test_drag_closed_form_level_attitude():
    """At identity attitude v_B = v: a = -(D |v| v + k_r T v) / m."""
    x = np.zeros((2, 13)); x[:, 3] = 1.0
    x[:, 7:10] = [[1.0, -2.0, 3.0], [0.5, 0.0, -1.5]]
    u = np.array([[1.0, 1.0, 1.0, 1.0], [0.5, 2.0, 0.0, 1.0]])
    D = np.array([0.3, 0.3, 0.5])
    ref = -(D * np.abs(x[:, 7:10]) * x[:, 7:10] + 0.02 * u.sum(1, keepdims=True) * x[:, 7:10]) / QUAD.mass
    np.testing.assert_allclose(drag_accel(x, u), ref, atol=1e-14)


def test_round_bf16_matches_torch():
    v = np.random.default_rng(0).normal(size=4096).astype(np.float32) * 10.0 ** np.random.default_rng(1).integers(-8, 8, 4096)
    v = np.concatenate([v, np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 0.0], np.float32)])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_bf16(v), ref)


def test_round_e4m3_matches_torch():
    rng = np.random.default_rng(2)
    v = rng.normal(size=8192) * 10.0 ** rng.uniform(-3, 2.6, size=8192)
    v = np.clip(v, -448, 448).astype(np.float32).astype(np.float64)
    v = np.concatenate([v, [2 ** -9, 3 * 2 ** -10, 2 ** -10, 1.0625, 1.1875, 448.0, 0.0]])
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_e4m3(v), ref)
    assert round_e4m3(np.array([1000.0, -500.0])).tolist() == [448.0, -448.0]


def test_emulation_exact_when_everything_is_representable():
    """With small-integer weights and inputs every rounding is exact, so the
    reduced-precision evaluation must reproduce the exact chain rule bit for bit."""
    from oracle.quant import emulated_jacobian
    rng = np.random.default_rng(4)
    Ws = [rng.integers(-1, 2, size=s).astype(np.float64) for s in [(8, 14), (8, 8), (6, 8)]]
    bs = [np.zeros(8), np.zeros(8), np.zeros(6)]
    net = MLP(Ws, bs, act="identity")
    z = rng.integers(-3, 4, size=(5, 14)).astype(np.float64)
    y, J = net.jacobian(z)
    ye, Je = emulated_jacobian(net, z, "bf16")
    np.testing.assert_array_equal(ye, y)
    np.testing.assert_array_equal(Je, J)

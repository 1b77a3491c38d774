"""Pins of the reduced-precision emulation (oracle/quant.py) and of the bounds the
GPU parity tests put on the network's part of a bf16 / fp8 linearisation.

The paper states no precision; the formats are OCP E4M3FN and bfloat16 with
static per-tensor scales amax/448 for E4M3.  Every expected value below is
worked by hand (in the comments) from those definitions, not from the oracle.
"""
import numpy as np
import pytest

from oracle.mlp import MLP, pack_input
from oracle.quant import calibrate_scales, emulated_jacobian, round_bf16, round_e4m3
from oracle.rk4 import linearize_affine
from workload import SEED_CALIB, config_workload, sample_nodes

from net_bounds import (EMULATION_BOUNDS, ORACLE_BOUNDS, network_errors, rel_rows, rms_rows,
                        within_oracle_bounds)

F32 = np.float32


def s448(m):
    """float32 amax / float32 448, the scale of a tensor whose largest magnitude is m."""
    return float(F32(m) / F32(448.0))


def test_calibrate_scales_by_hand_identity_network():
    """Linear 2-2-2-2 network, two calibration inputs; every amax worked by hand."""
    Ws = [np.array([[1.0, -2.0], [3.0, 0.5]]), np.array([[0.5, 1.0], [-1.0, 2.0]]),
          np.array([[4.0, -1.0], [0.25, 2.0]])]
    bs = [np.array([0.0, 1.0]), np.zeros(2), np.zeros(2)]
    z = np.array([[1.0, 1.0], [-2.0, 0.5]])
    sc = calibrate_scales(MLP(Ws, bs, act="identity"), z)
    # weights: amax 3, 2, 4
    assert sc["w"] == [s448(3.0), s448(2.0), s448(4.0)]
    # forward operands: z amax 2;
    # h1 = W1 z + b1 = [1 - 2, 3 + 0.5 + 1] = [-1, 4.5] and [-2 - 1, -6 + 0.25 + 1] = [-3, -4.75] -> 4.75;
    # h2 = W2 h1 = [-0.5 + 4.5, 1 + 9] = [4, 10] and [-1.5 - 4.75, 3 - 9.5] -> 10
    assert sc["a"] == [s448(2.0), s448(4.75), s448(10.0)]
    # reverse operands (identity: act' = 1): G_2 = W3 -> 4;
    # G_1 = W3 W2 = [[4 * 0.5 + 1, 4 - 2], [0.125 - 2, 0.25 + 4]] = [[3, 2], [-1.875, 4.25]] -> 4.25
    assert sc["g"] == [s448(4.25), s448(4.0)]


def test_calibrate_scales_silu_at_origin_and_zero_tensors():
    """SiLU network fed z = 0 with zero biases: every pre-activation is 0, so every
    hidden activation is SiLU(0) = 0 (scale 1 by the all-zero rule) and act'(0) = 1/2
    exactly: G_2 = W3 / 2, G_1 = (W3 / 2) W2 / 2."""
    Ws = [np.array([[1.0, -2.0], [3.0, 0.5]]), np.array([[0.5, 1.0], [-1.0, 2.0]]),
          np.array([[4.0, -1.0], [0.25, 2.0]])]
    bs = [np.zeros(2)] * 3
    sc = calibrate_scales(MLP(Ws, bs), np.zeros((3, 2)))
    assert sc["a"] == [1.0, 1.0, 1.0]
    assert sc["g"] == [s448(4.25 / 4), s448(2.0)]


def test_fp8_emulation_rounds_every_operand_by_hand():
    """One-input, one-output linear network; scales chosen so no rounding is exact.
    E4M3 has 3 mantissa bits: in the binade [2^e, 2^(e+1)) the spacing is 2^(e-3)."""
    Ws = [np.array([[0.3]]), np.array([[1.3]]), np.array([[0.7]])]
    bs = [np.zeros(1)] * 3
    sc = {"w": [0.5, 1.0, 0.25], "a": [1.0, 0.5, 0.25], "g": [0.125, 0.25]}
    y, J = emulated_jacobian(MLP(Ws, bs, act="identity"), np.array([[1.1]]), "fp8", sc)
    # W1: 0.3 / 0.5 = 0.6, spacing 1/16 -> 0.625 -> 0.3125;  W2: 1.3 / 1 -> spacing 1/8 -> 1.25;
    # W3: 0.7 / 0.25 = 2.8, spacing 1/4 -> 2.75 -> 0.6875;  z: 1.1 -> 1.125
    # a1 = 1.125 * 0.3125 = 0.3515625; h1: 0.703125 (spacing 1/16) -> 0.6875 -> 0.34375
    # a2 = 0.34375 * 1.25 = 0.4296875; h2: 1.71875 (spacing 1/8) -> 1.75 -> 0.4375
    # y = 0.4375 * 0.6875
    assert y[0, 0] == 0.30078125
    # G_2 = W3 (unrounded) * act' = 0.7; 0.7 / 0.25 = 2.8 -> 2.75 -> 0.6875
    # G_1 = (0.6875 * 1.25) = 0.859375; / 0.125 = 6.875 (spacing 1/2) -> 7 -> 0.875
    # J = 0.875 * 0.3125
    assert J[0, 0, 0] == 0.2734375


def test_fp8_emulation_exact_for_representable_values_with_small_scales():
    """Power-of-two scales and tensors whose values divided by their scale are small
    integers (E4M3 holds every integer up to 16 exactly): every rounding is exact and
    the emulation equals the exact chain rule.  Weights are +-2^-4 with scale 2^-8, so
    a weight multiplied by its scale instead of divided (2^-12) would fall below half
    the smallest E4M3 subnormal (2^-9) and round to zero."""
    rng = np.random.default_rng(3)
    c = 2.0 ** -4
    Ws = [rng.choice([-c, 0.0, c], size=s_) for s_ in [(4, 3), (4, 4), (2, 4)]]
    bs = [np.zeros(4), np.zeros(4), np.zeros(2)]
    net = MLP(Ws, bs, act="identity")
    z = rng.choice([-c, 0.0, c], size=(6, 3))
    # h1 = W1 z: integers in [-3, 3] times 2^-8;  h2 = W2 h1: integers in [-12, 12] times 2^-12
    # G_2 = W3 (act' = 1): +-16 times 2^-8;  G_1 = W3 W2: integers in [-4, 4] times 2^-8
    sc = {"w": [2.0 ** -8] * 3, "a": [2.0 ** -8, 2.0 ** -8, 2.0 ** -12], "g": [2.0 ** -8, 2.0 ** -8]}
    h1 = z @ Ws[0].T
    for t, s_ in ((h1, 2.0 ** -8), (h1 @ Ws[1].T, 2.0 ** -12), (Ws[2] @ Ws[1], 2.0 ** -8)):
        q = t / s_
        assert np.all(q == np.round(q)) and np.all(np.abs(q) <= 16)
    y, J = net.jacobian(z)
    ye, Je = emulated_jacobian(net, z, "fp8", sc)
    np.testing.assert_array_equal(ye, y)
    np.testing.assert_array_equal(Je, J)
    assert np.any(J != 0) and np.any(y != 0)
    assert np.all(round_e4m3(Ws[0] * 2.0 ** -8) == 0.0)


def test_bf16_rounding_points_by_hand():
    """bfloat16 keeps 7 stored mantissa bits (spacing 2^-7 in [1, 2))."""
    assert round_bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0           # tie -> even
    assert round_bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6  # tie -> even (up)
    assert round_bf16(np.array([1.0 + 2 ** -8 + 2 ** -12]))[0] == 1.0 + 2 ** -7


# --------------------------------------------------------------------------------------
# The bounds of the GPU parity tests on the network's part (tests/net_bounds.py): they
# must hold for the quantisation error alone and must fail for a wrong network.

def _emulated_case(key, fmt, n, n_calib):
    cfg, off, x, u, Ws, bs = config_workload(key)
    net = MLP(Ws, bs)
    xs, us = sample_nodes(n, seed=77)
    sc = None
    if fmt == "fp8":
        xc, uc = sample_nodes(n_calib, seed=SEED_CALIB)
        sc = calibrate_scales(net, pack_input(xc, uc))
    ref = linearize_affine(xs, us, net, cfg.dt)
    ref_nom = linearize_affine(xs, us, None, cfg.dt)
    y, J = emulated_jacobian(net, pack_input(xs, us), fmt, sc)
    em = linearize_affine(xs, us, net, cfg.dt, params=(y, J))
    return cfg, xs, us, ref, ref_nom, em


@pytest.fixture(scope="module", params=[("c3", "bf16", 300, 0), ("c4", "fp8", 120, 8192)],
                ids=["c3-bf16", "c4-fp8"])
def case(request):
    return request.param[1], _emulated_case(*request.param)


def test_bounds_hold_for_the_quantisation_error(case):
    fmt, (cfg, xs, us, ref, ref_nom, em) = case
    errs = network_errors(em[3], em[4], em[1], em[2], ref_nom[1], ref_nom[2], ref, ref_nom)
    w = {k: float(np.max(v)) for k, v in errs.items()}
    print(fmt, w)
    assert within_oracle_bounds(errs, fmt)
    # the bounds are not so loose that the quantisation error is negligible against them
    assert max(w[k] / ORACLE_BOUNDS[fmt][k] for k in w) > 0.2


@pytest.mark.parametrize("mistake", ["zero_J", "half_J", "zero_f", "zero_J_u", "sign_J", "no_gate"])
def test_bounds_fail_for_a_wrong_network(case, mistake):
    """Plant a mistake in the oracle's network part (on the CPU) and check that the
    bounds used on the GPU reject it."""
    fmt, (cfg, xs, us, ref, ref_nom, em) = case
    y, J = em[3].copy(), em[4].copy()
    if mistake == "zero_J":
        J[:] = 0.0
    elif mistake == "half_J":
        J *= 0.5
    elif mistake == "zero_f":
        y[:] = 0.0
    elif mistake == "zero_J_u":  # the input columns dropped
        J[:, :, 10:] = 0.0
    elif mistake == "sign_J":
        J = -J
    elif mistake == "no_gate":  # act' left out of the reverse sweep: J = W_{L+1} ... W_1
        net_W = config_workload("c3" if fmt == "bf16" else "c4")[4]
        P = np.asarray(net_W[-1], np.float64)
        for W in net_W[-2::-1]:
            P = P @ np.asarray(W, np.float64)
        J = np.broadcast_to(P, J.shape).copy()
    bad = linearize_affine(xs, us, None, cfg.dt, params=(y, J))
    errs = network_errors(y, J, bad[1], bad[2], ref_nom[1], ref_nom[2], ref, ref_nom)
    assert not within_oracle_bounds(errs, fmt)


def _emul_f32(model, z, fmt, scales=None):
    """The emulation with every matrix product accumulated in float32 (a different
    summation order and precision), same rounding points."""
    rnd = (lambda a, s: round_bf16(a)) if fmt == "bf16" else (lambda a, s: round_e4m3(np.asarray(a) / s) * s)
    L = model.n_hidden
    sw = scales["w"] if scales else [1.0] * (L + 1)
    sa = scales["a"] if scales else [1.0] * (L + 1)
    sg = scales["g"] if scales else [1.0] * L
    mm = lambda a, b: (np.asarray(a, F32) @ np.asarray(b, F32)).astype(np.float64)
    Wq = [rnd(W, sw[l]) for l, W in enumerate(model.Ws)]
    h = rnd(np.asarray(z, np.float64), sa[0])
    sps = []
    for l in range(L):
        a = mm(h, Wq[l].T) + model.bs[l]
        sps.append(round_bf16(model._act_prime(a)))
        h = rnd(model._act(a), sa[l + 1])
    y = mm(h, Wq[L].T) + model.bs[L]
    n = z.shape[0]
    G = rnd(np.broadcast_to(model.Ws[L], (n,) + model.Ws[L].shape) * sps[L - 1][:, None, :], sg[L - 1])
    for l in range(L - 1, 0, -1):
        G = rnd(mm(G, Wq[l]) * sps[l - 1][:, None, :], sg[l - 1])
    return y, mm(G, Wq[0])


@pytest.mark.parametrize("key,fmt,n,n_calib", [("c3", "bf16", 2000, 0), ("c4", "fp8", 300, 2048)])
def test_accumulation_order_spread(key, fmt, n, n_calib):
    """Only the accumulation changes (float64 -> float32), every rounding point stays:
    the typical node moves at float32 level, a few move by much more, because an
    operand crossing a rounding boundary carries its flip through every later layer.
    The GPU-vs-emulation bounds sit above this spread (maximum) and at float32 level
    (median)."""
    cfg, off, x, u, Ws, bs = config_workload(key)
    net = MLP(Ws, bs)
    sc = None
    if fmt == "fp8":
        xc, uc = sample_nodes(n_calib, seed=SEED_CALIB)
        sc = calibrate_scales(net, pack_input(xc, uc))
    z = pack_input(*sample_nodes(n, seed=1))
    y64, J64 = emulated_jacobian(net, z, fmt, sc)
    y32, J32 = _emul_f32(net, z, fmt, sc)
    ry, rJ = rms_rows(y32, y64), rel_rows(J32, J64)
    print(fmt, f"median {np.median(ry):.1e} {np.median(rJ):.1e}  max {ry.max():.1e} {rJ.max():.1e}")
    b = EMULATION_BOUNDS[fmt]
    assert np.median(ry) < b["median"] / 10 and np.median(rJ) < b["median"] / 10
    assert max(ry.max(), rJ.max()) > 1e3 * max(np.median(ry), np.median(rJ))  # flips exist
    assert max(ry.max(), rJ.max()) < b["max"] / 2


def test_fp8_accumulation_model_sizes_the_emulation_bounds():
    """The fp8 emulation bounds come from the emulation with every product output
    perturbed at the fp8 matrix cores' measured accumulation level (relative 3e-5):
    on the 14-4x1024-6 network that level flips enough later E4M3 roundings to move
    the typical node by ~1e-2, while a perturbation at fp32 level (1e-7) barely moves
    it; the bounds derived from it stay below what a zeroed or halved J_D gives."""
    from net_bounds import FP8_ACCUMULATION_EPS, fp8_emulation_bounds, perturbed_fp8_emulation
    cfg, off, x, u, Ws, bs = config_workload("c4")
    net = MLP(Ws, bs)
    xc, uc = sample_nodes(2048, seed=SEED_CALIB)
    sc = calibrate_scales(net, pack_input(xc, uc))
    z = pack_input(*sample_nodes(100, seed=1))
    ye, Je = emulated_jacobian(net, z, "fp8", sc)
    yp, Jp = perturbed_fp8_emulation(net, z, sc, eps=1e-7)
    assert np.median(rel_rows(Jp, Je)) < 1e-5 and np.median(rms_rows(yp, ye)) < 1e-5
    yp, Jp = perturbed_fp8_emulation(net, z, sc, eps=FP8_ACCUMULATION_EPS)
    med = np.median(rel_rows(Jp, Je))
    print(f"perturbed at {FP8_ACCUMULATION_EPS}: median J_D {med:.2e}")
    assert 1e-3 < med < 0.1
    b = fp8_emulation_bounds(net, z, sc, ye, Je)
    assert b["max"] <= 0.45 and b["median"] < 0.25
    assert np.median(rel_rows(0.5 * Je, Je)) > b["median"] and rel_rows(0.0 * Je, Je).max() > b["max"]

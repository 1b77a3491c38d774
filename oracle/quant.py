"""Rounding emulation for reduced-precision formats -- TEST INFRASTRUCTURE.

The paper states no numeric precision.  The reduced-precision GPU paths store
network operands in bfloat16 (8-bit exponent, 7 stored mantissa bits) or in
OCP FP8 E4M3FN (bias 7, 3 mantissa bits, largest finite 448, no infinities),
both rounded to nearest with ties to even; E4M3 values beyond +-448 saturate.
These functions produce the float64 value of the rounded number so that the
oracle can repeat a reduced-precision computation exactly where it rounds.
"""
from __future__ import annotations

import numpy as np


def round_bf16(a) -> np.ndarray:
    """float64 value of round-to-nearest-even bfloat16(float32(a))."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


E4M3_MAX = 448.0


def round_e4m3(a) -> np.ndarray:
    """float64 value of saturating round-to-nearest-even E4M3FN(a)."""
    a = np.asarray(a, dtype=np.float64)
    mag = np.abs(a)
    # exponent of the binade; values below 2^-6 use the subnormal quantum 2^-9
    e = np.floor(np.log2(np.maximum(mag, 2.0 ** -6)))
    quantum = 2.0 ** (e - 3)
    r = np.round(mag / quantum) * quantum  # numpy rounds halves to even
    r = np.minimum(r, E4M3_MAX)
    return np.sign(a) * r


# ---------------------------------------------------------------------------
# Reduced-precision evaluation of the residual network and its Jacobian.
#
# Same chain rule as oracle.mlp.MLP.jacobian, but every matrix-product operand is
# rounded where a reduced-precision implementation stores it: weights, the
# network input, every hidden activation h_l and every reverse-sweep operand
# G_l = (G_{l+1} W_{l+1}) * act'(a_l) are rounded to the format (FP8 values are
# divided by their per-tensor scale before rounding and multiplied back after);
# act'(a_l) is kept in bfloat16; biases, accumulations, the output weights used
# to seed the reverse sweep, y and J_D stay exact.

def _rounder(fmt):
    if fmt == "bf16":
        return lambda a, s: round_bf16(a)
    if fmt == "fp8":
        return lambda a, s: round_e4m3(np.asarray(a) / s) * s
    raise ValueError(fmt)


def calibrate_scales(model, z: np.ndarray) -> dict:
    """Static per-tensor E4M3 scales amax/448 (1 for an all-zero tensor), float32:
    weights W_1..W_{L+1}, forward operands z_0, h_1..h_L, reverse operands G_1..G_L,
    measured on the calibration inputs z (n, 14) in float64."""
    def sc(a):
        m = float(np.max(np.abs(a))) if np.size(a) else 0.0
        return float(np.float32(m) / np.float32(448.0)) if m > 0 else 1.0
    L = model.n_hidden
    w = [sc(W.astype(np.float32)) for W in model.Ws]
    y, pre = model.forward(z, keep=True)
    hs = [z] + [model._act(a) for a in pre]
    a = [sc(h) for h in hs]
    g = [0.0] * L
    n = z.shape[0]
    G = np.broadcast_to(model.Ws[-1], (n,) + model.Ws[-1].shape)
    for l in range(L - 1, -1, -1):
        G = G * model._act_prime(pre[l])[:, None, :]
        g[l] = sc(G)
        G = G @ model.Ws[l]
    return {"w": w, "a": a, "g": g}


def emulated_jacobian(model, z: np.ndarray, fmt: str, scales: dict = None):
    """(y (n,6), J_D (n,6,14)) with operands rounded as described above."""
    rnd = _rounder(fmt)
    L = model.n_hidden
    if fmt == "fp8" and scales is None:
        raise ValueError("fp8 emulation needs scales")
    sw = scales["w"] if scales else [1.0] * (L + 1)
    sa = scales["a"] if scales else [1.0] * (L + 1)
    sg = scales["g"] if scales else [1.0] * L
    Wq = [rnd(W, sw[l]) for l, W in enumerate(model.Ws)]
    h = rnd(np.asarray(z, dtype=np.float64), sa[0])
    sps = []
    for l in range(L):
        a = h @ Wq[l].T + model.bs[l]
        sps.append(round_bf16(model._act_prime(a)))
        h = rnd(model._act(a), sa[l + 1])
    y = h @ Wq[L].T + model.bs[L]
    n = z.shape[0]
    G = rnd(np.broadcast_to(model.Ws[L], (n,) + model.Ws[L].shape) * sps[L - 1][:, None, :], sg[L - 1])
    for l in range(L - 1, 0, -1):
        G = rnd((G @ Wq[l]) * sps[l - 1][:, None, :], sg[l - 1])
    J = G @ Wq[0]
    return y, J

"""Error measures and bounds for the network's part of a linearisation.

A_k = I + O(dt) terms, so a bound on the relative error of A_k, B_k or x_{k+1}
says almost nothing about the residual network: replacing the network by zero
moves them by ~5e-4 relative on the benchmarked networks.  The parity tests
therefore also bound, per node, the quantities the learned model hands to the
QP (Sec. IV-A: f_D-bar and J_D are the only interface between the network and
the solver) and the network's share of the continuity parameters:

* J_D, and (A_k - A_nominal), (B_k - B_nominal): relative Frobenius error
  |X - X_ref| / |X_ref| per node, where A_nominal, B_nominal come from the same
  step with the network removed (each side computes its own);
* f_D-bar: |f - f_ref| per node over the root-mean-square |f_ref| of the
  sample.  Rounding errors of the network's operands add up to an error of
  roughly constant size, so a per-node relative error is dominated by the few
  nodes whose output happens to be near zero.

Bounds against the FP64 oracle (the oracle uses the fp32 master weights, so
the bound covers the quantisation of weights and activations).  They are set
at about twice the error of the oracle's own rounding emulation on the
benchmarked networks (14-5x512-6 bf16: J_D 8.0e-3, dA 8.6e-3, dB 7.8e-3,
f_D 1.9e-2; 14-4x1024-6 fp8: J_D 9.7e-2, dA 9.7e-2, dB 9.9e-2, f_D 0.24), and
far below what a wrong network gives (a zero or halved J_D: error 1 or 0.5);
tests/test_oracle_quant.py checks both sides of that on the CPU.

Bounds against the rounding emulation (same rounding points as the GPU): the
typical node agrees to fp32-accumulation level (median); the maximum is set by
nodes where a different summation order moves an operand across a rounding
boundary and the flip propagates through the following layers.  Changing only
the emulation's accumulation from float64 to float32 moves it by up to 5.3e-3
(bf16, 14-5x512-6) and 5.4e-2 (fp8, 14-4x1024-6) at the maximum, ~1e-7 at the
median (tests/test_oracle_quant.py::test_accumulation_order_spread).
"""
from __future__ import annotations

import numpy as np

ORACLE_BOUNDS = {
    "bf16": {"f_D": 5e-2, "J_D": 2e-2, "dA": 2e-2, "dB": 2e-2},
    "fp8": {"f_D": 0.5, "J_D": 0.2, "dA": 0.2, "dB": 0.2},
}
EMULATION_BOUNDS = {
    "bf16": {"median": 1e-5, "max": 2e-2},
    "fp8": {"median": 1e-4, "max": 0.15},
}


def rel_rows(a, b) -> np.ndarray:
    """Per-node |a - b|_F / |b|_F over all trailing axes."""
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-30)


def rms_rows(f, f_ref) -> np.ndarray:
    """Per-node |f - f_ref| over the root-mean-square node norm of f_ref."""
    f = np.asarray(f, np.float64).reshape(f.shape[0], -1)
    f_ref = np.asarray(f_ref, np.float64).reshape(f_ref.shape[0], -1)
    scale = np.sqrt(np.mean(np.sum(f_ref ** 2, axis=1)))
    return np.linalg.norm(f - f_ref, axis=1) / max(scale, 1e-30)


def network_errors(f_D, J_D, A, B, A_nom, B_nom, ref, ref_nom) -> dict:
    """Per-node error arrays of the network's part.  ``ref`` and ``ref_nom`` are
    oracle linearisations (x_next, A, B, f_D, J_D) with and without the network."""
    return {
        "f_D": rms_rows(f_D, ref[3]),
        "J_D": rel_rows(J_D, ref[4]),
        "dA": rel_rows(np.asarray(A, np.float64) - np.asarray(A_nom, np.float64), ref[1] - ref_nom[1]),
        "dB": rel_rows(np.asarray(B, np.float64) - np.asarray(B_nom, np.float64), ref[2] - ref_nom[2]),
    }


def worst(errs: dict) -> dict:
    return {k: float(np.max(v)) for k, v in errs.items()}


def within_oracle_bounds(errs: dict, prec: str) -> bool:
    b = ORACLE_BOUNDS[prec]
    return all(float(np.max(errs[k])) <= b[k] for k in b)


def assert_within_oracle_bounds(errs: dict, prec: str) -> None:
    b = ORACLE_BOUNDS[prec]
    w = worst(errs)
    print(f"  network part vs FP64 ({prec}):", {k: f"{v:.2e}" for k, v in w.items()}, flush=True)
    for k in b:
        assert w[k] <= b[k], (prec, k, w[k], b[k])


def assert_within_emulation_bounds(f_D, J_D, f_em, J_em, prec: str) -> None:
    b = EMULATION_BOUNDS[prec]
    ry, rJ = rms_rows(f_D, f_em), rel_rows(J_D, J_em)
    print(f"  vs {prec} emulation: median f_D {np.median(ry):.2e} J_D {np.median(rJ):.2e}, "
          f"max f_D {ry.max():.2e} J_D {rJ.max():.2e}", flush=True)
    assert np.median(ry) <= b["median"] and np.median(rJ) <= b["median"], (prec, np.median(ry), np.median(rJ))
    assert ry.max() <= b["max"] and rJ.max() <= b["max"], (prec, ry.max(), rJ.max())

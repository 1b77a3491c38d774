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

Networks other than the two benchmarked ones (fewer inputs, other widths and
depths) carry other quantisation errors; there the bound of each quantity is the
larger of the fixed bound and twice the emulation's own error against the FP64
oracle on the same nodes, capped below 0.45 (0.9 for f_D-bar) so that a halved
or zeroed J_D, or a zeroed f_D-bar, still fails.

Bounds against the rounding emulation (same rounding points as the GPU): the
typical node agrees to the accumulation level of the matrix cores (median); the
maximum is set by nodes where a different summation moves an operand across a
rounding boundary and the flip propagates through the following layers.

* bf16 products accumulate in fp32 on the matrix cores.  Changing only the
  emulation's accumulation from float64 to float32 moves it by up to 5.3e-3
  (14-5x512-6) at the maximum, ~1e-7 at the median
  (tests/test_oracle_quant.py::test_accumulation_order_spread).
* fp8 products do not: the gfx950 fp8 matrix instruction adds the products of
  one 64-wide K block with a limited alignment window (a product 14 binades
  below the block's largest is lost: 256 + 2^-6 sums to 256, 256 + 2^-5 is
  exact), so on network data its results sit ~1e-5 (relative) from the exact
  sum -- against ~5e-8 for bf16 on the same one-hidden-layer networks, where
  nothing is rounded after the product.  Through a deep network these
  differences flip later E4M3 roundings.  The emulation with every product
  output perturbed by a seeded relative 3e-5 (FP8_ACCUMULATION_EPS)
  reproduces the spread measured on the GPU (14-4x1024-6: median 1.0e-2 f_D,
  2.9e-2 J_D; GPU 1.0e-2, 3.1e-2), so the fp8 emulation bounds are twice that
  model's spread on the nodes under test (at least 3e-5 median, 0.15 maximum;
  at most 0.45, which a zeroed or halved J_D still exceeds).
"""
from __future__ import annotations

import numpy as np

ORACLE_BOUNDS = {
    "bf16": {"f_D": 5e-2, "J_D": 2e-2, "dA": 2e-2, "dB": 2e-2},
    "fp8": {"f_D": 0.5, "J_D": 0.2, "dA": 0.2, "dB": 0.2},
}
EMULATION_BOUNDS = {
    "bf16": {"median": 1e-5, "max": 2e-2},
    "fp8": {"median": 3e-5, "max": 0.15},
}
FP8_ACCUMULATION_EPS = 3e-5


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


CAPS = {"f_D": 0.9, "J_D": 0.45, "dA": 0.45, "dB": 0.45}


def bounds_for(prec: str, emul_errs: dict = None, skip=()) -> dict:
    """The fixed bounds of `prec`, widened to twice the emulation's own worst error
    (emul_errs: network_errors of the rounding emulation against the oracle on the same
    nodes) where that is larger, never beyond CAPS; quantities in `skip` unbounded."""
    b = {k: v for k, v in ORACLE_BOUNDS[prec].items() if k not in skip}
    if emul_errs is not None:
        for k in b:
            b[k] = max(b[k], 2.0 * float(np.max(emul_errs[k])))
            assert b[k] <= CAPS[k], (prec, k, b[k], "the emulation's own error is too large to bound a network")
    return b


def assert_within_oracle_bounds(errs: dict, prec: str, bounds: dict = None) -> None:
    b = ORACLE_BOUNDS[prec] if bounds is None else bounds
    w = worst(errs)
    print(f"  network part vs FP64 ({prec}):", {k: f"{v:.2e}" for k, v in w.items()},
          "bounds", {k: f"{v:.2e}" for k, v in b.items()}, flush=True)
    for k in b:
        assert w[k] <= b[k], (prec, k, w[k], b[k])


def perturbed_fp8_emulation(model, z, scales, eps=FP8_ACCUMULATION_EPS, seed=0):
    """The fp8 rounding emulation (oracle.quant.emulated_jacobian) with every matrix
    product's output multiplied by (1 + eps n), n ~ N(0, 1) seeded: a model of an
    accumulation that is not exact, used only to size the emulation bounds."""
    from oracle.quant import round_bf16, round_e4m3
    rng = np.random.default_rng(seed)
    pert = lambda a: a * (1.0 + eps * rng.standard_normal(a.shape))
    rnd = lambda a, s: round_e4m3(np.asarray(a) / s) * s
    L = model.n_hidden
    sw, sa, sg = scales["w"], scales["a"], scales["g"]
    Wq = [rnd(W, sw[l]) for l, W in enumerate(model.Ws)]
    h = rnd(np.asarray(z, np.float64), sa[0])
    sps = []
    for l in range(L):
        a = pert(h @ Wq[l].T) + model.bs[l]
        sps.append(round_bf16(model._act_prime(a)))
        h = rnd(model._act(a), sa[l + 1])
    y = pert(h @ Wq[L].T) + model.bs[L]
    n = z.shape[0]
    G = rnd(np.broadcast_to(model.Ws[L], (n,) + model.Ws[L].shape) * sps[L - 1][:, None, :], sg[L - 1])
    for l in range(L - 1, 0, -1):
        G = rnd(pert(G @ Wq[l]) * sps[l - 1][:, None, :], sg[l - 1])
    return y, pert(G @ Wq[0])


def fp8_emulation_bounds(model, z, scales, f_em, J_em) -> dict:
    """Emulation bounds of an fp8 network on inputs z: twice the spread of the
    perturbed emulation around the emulation (f_em, J_em), within the floors and cap."""
    yp, Jp = perturbed_fp8_emulation(model, z, scales)
    ry, rJ = rms_rows(yp, f_em), rel_rows(Jp, J_em)
    b = EMULATION_BOUNDS["fp8"]
    return {"median": max(b["median"], 2.0 * max(np.median(ry), np.median(rJ))),
            "max": min(0.45, max(b["max"], 2.0 * max(ry.max(), rJ.max())))}


def assert_within_emulation_bounds(f_D, J_D, f_em, J_em, prec: str, bounds: dict = None) -> None:
    b = EMULATION_BOUNDS[prec] if bounds is None else bounds
    ry, rJ = rms_rows(f_D, f_em), rel_rows(J_D, J_em)
    print(f"  vs {prec} emulation: median f_D {np.median(ry):.2e} J_D {np.median(rJ):.2e}, "
          f"max f_D {ry.max():.2e} J_D {rJ.max():.2e}; bounds {b}", flush=True)
    assert np.median(ry) <= b["median"] and np.median(rJ) <= b["median"], (prec, np.median(ry), np.median(rJ))
    assert ry.max() <= b["max"] and rJ.max() <= b["max"], (prec, ry.max(), rJ.max())

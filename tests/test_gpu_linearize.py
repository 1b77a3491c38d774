"""GPU parity of rtn_linearize against the FP64 oracle (element by element).

Error measure per node and output: e = |X_gpu - X_oracle|_F / |X_oracle|_F; the
bound is on the maximum over nodes.  Bounds: FP32 1e-5, BF16 1e-2, FP8 5e-2 on
x_{k+1}, A_k, B_k.  Those bounds alone cannot see the network at bf16 / fp8 (a
zero network moves x, A, B by ~5e-4), so every reduced-precision case also
bounds the network's part per node -- f_D-bar, J_D, (A - A_nominal) and
(B - B_nominal) -- against the FP64 oracle and f_D-bar, J_D against the
oracle's evaluation with the same operand roundings (tests/net_bounds.py states
the bounds and tests/test_oracle_quant.py shows that a zeroed, halved or
ungated J_D fails them).
"""
import sys

import numpy as np
import pytest

from workload import (CONFIGS, QUAD, SEED_CALIB, config_workload, sample_nodes, xavier_params,
                      offsets_from_horizons, sample_horizons)
from oracle.mlp import MLP, pack_input
from oracle.rk4 import linearize_affine
from oracle.quant import emulated_jacobian, calibrate_scales

from net_bounds import (assert_within_emulation_bounds, assert_within_oracle_bounds, bounds_for, fp8_emulation_bounds,
                        network_errors)

pytestmark = pytest.mark.gpu
DT = 0.05


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def rel(a, b):
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-30)


def gpu_linearize(torch, x, u, Ws=None, bs=None, prec="fp32", act="silu", offsets=None, model=None, calib=None,
                  want_status=False):
    import paper_2203_07747_amd as rtn
    print(f"[gpu] linearize n={x.shape[0]} prec={prec} "
          f"L={len(Ws) - 1 if Ws else '-'} H={Ws[0].shape[0] if Ws else '-'}", flush=True)
    own = False
    if model is None and Ws is not None:
        model, own = rtn.Model(Ws, bs, act), True
    if calib is not None:
        model.calibrate(torch.from_numpy(calib[0]).cuda(), torch.from_numpy(calib[1]).cuda())
    out = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), model, prec, DT,
                        offsets=offsets, want_status=want_status)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    if own:
        model.close()
    return res


def check_against(res, ref, tol, idx=None, parts=("x_next", "A", "B")):
    names = ("x_next", "A", "B", "f_D", "J_D")
    errs = {}
    for name, r in zip(names, ref):
        g = res[name] if idx is None else res[name][idx]
        errs[name] = float(rel(g, r).max())
    print("  max rel err:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for p in parts:
        assert errs[p] <= tol, (p, errs[p], tol)
    return errs


def gpu_nominal(torch, x, u):
    """A_k, B_k of the same nodes with the network removed (the GPU's nominal step)."""
    import paper_2203_07747_amd as rtn
    out = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), None, "fp32", DT)
    torch.cuda.synchronize()
    return out["A"].cpu().numpy(), out["B"].cpu().numpy()


def check_network(torch, res, ref, x, u, net, prec, idx=None, scales=None):
    """Bounds on the network's part of a bf16 / fp8 linearisation of nodes x, u (the
    GPU result `res` may cover a superset of nodes, selected by idx) against the FP64
    oracle `ref` -- the fixed bounds of the precision, widened to twice the rounding
    emulation's own error on these nodes where that is larger -- and of f_D, J_D
    against the rounding emulation."""
    sel = (lambda a: a) if idx is None else (lambda a: a[idx])
    A_nom, B_nom = gpu_nominal(torch, x, u)
    ref_nom = linearize_affine(x, u, None, DT)
    errs = network_errors(sel(res["f_D"]), sel(res["J_D"]), sel(res["A"]), sel(res["B"]), A_nom, B_nom, ref,
                          ref_nom)
    ye, Je = emulated_jacobian(net, pack_input(x, u), prec, scales)
    em = linearize_affine(x, u, None, DT, params=(ye, Je))
    em_errs = network_errors(ye, Je, em[1], em[2], ref_nom[1], ref_nom[2], ref, ref_nom)
    assert_within_oracle_bounds(errs, prec, bounds_for(prec, em_errs))
    eb = fp8_emulation_bounds(net, pack_input(x, u), scales, ye, Je) if prec == "fp8" else None
    assert_within_emulation_bounds(sel(res["f_D"]), sel(res["J_D"]), ye, Je, prec, eb)
    return errs


@pytest.mark.parametrize("key", ["c1", "c2"])
def test_fp32_configs_match_oracle(torch, key):
    cfg, off, x, u, Ws, bs = config_workload(key)
    res = gpu_linearize(torch, x, u, Ws, bs, "fp32", offsets=off)
    ref = linearize_affine(x, u, MLP(Ws, bs), cfg.dt)
    errs = check_against(res, ref, 1e-5)
    assert errs["f_D"] < 1e-5 and errs["J_D"] < 1e-5


@pytest.mark.parametrize("H,L,n", [(64, 2, 1), (64, 3, 300), (128, 2, 257), (256, 3, 129), (512, 2, 97),
                                   (1024, 2, 67), (512, 1, 33)])
def test_fp32_widths_and_ragged_tails(torch, H, L, n):
    """Sizes span several row blocks of both kernels and end in a partial block."""
    Ws, bs = xavier_params(L, H, seed=H + L)
    bs = [np.random.default_rng(7).normal(size=b.shape).astype(np.float32) * 0.1 for b in bs]
    x, u = sample_nodes(n, seed=n)
    res = gpu_linearize(torch, x, u, Ws, bs, "fp32")
    ref = linearize_affine(x, u, MLP(Ws, bs), DT)
    errs = check_against(res, ref, 1e-5)
    assert errs["J_D"] < 2e-5


def test_identity_network_jacobian_is_constant(torch):
    Ws, bs = xavier_params(3, 128, seed=3)
    x, u = sample_nodes(50, seed=5)
    res = gpu_linearize(torch, x, u, Ws, bs, "fp32", act="identity")
    prod = Ws[3].astype(np.float64) @ Ws[2] @ Ws[1] @ Ws[0]
    np.testing.assert_allclose(res["J_D"], np.broadcast_to(prod, res["J_D"].shape), rtol=1e-4, atol=1e-6)
    ref = linearize_affine(x, u, MLP(Ws, bs, "identity"), DT)
    check_against(res, ref, 1e-5)


def test_nominal_only(torch):
    x, u = sample_nodes(1000, seed=9)
    res = gpu_linearize(torch, x, u)
    ref = linearize_affine(x, u, None, DT)
    check_against(res, ref, 1e-5, parts=("x_next", "A", "B"))
    assert np.all(res["f_D"] == 0) and np.all(res["J_D"] == 0)


def test_empty_batch(torch):
    import paper_2203_07747_amd as rtn
    Ws, bs = xavier_params(2, 64)
    m = rtn.Model(Ws, bs)
    z = torch.zeros((0, 13), device="cuda"), torch.zeros((0, 4), device="cuda")
    out = rtn.linearize(z[0], z[1], m, "bf16")
    torch.cuda.synchronize()
    assert out["A"].shape == (0, 13, 13)


def test_repeat_calls_bit_identical_and_offsets_irrelevant(torch):
    Ws, bs = xavier_params(3, 512)
    hz = sample_horizons(40, 10, 50)
    off = offsets_from_horizons(hz)
    x, u = sample_nodes(int(off[-1]), seed=3)
    a = gpu_linearize(torch, x, u, Ws, bs, "bf16", offsets=off)
    b = gpu_linearize(torch, x, u, Ws, bs, "bf16")
    for k in ("x_next", "A", "B", "f_D", "J_D"):
        np.testing.assert_array_equal(a[k], b[k])


def test_status_flags(torch):
    Ws, bs = xavier_params(2, 64)
    x, u = sample_nodes(40, seed=4)
    x[5, 7] = np.nan
    res = gpu_linearize(torch, x, u, Ws, bs, "fp32", want_status=True)
    st = res["status"]
    assert st[5] & 2 and st[5] & 1  # NaN input poisons the network output and the step
    assert np.all(st[np.arange(40) != 5] == 0)
    Ws[1][3, 4] = np.nan
    res = gpu_linearize(torch, sample_nodes(8)[0], sample_nodes(8)[1], Ws, bs, "fp32", want_status=True)
    assert np.all(res["status"] & 1)


def test_fp8_nan_reaches_status_and_new_params_need_calibration(torch):
    """A NaN operand stays NaN through the E4M3 conversion (rather than saturating to a
    finite value), so the node's network output is flagged; replacing the parameters
    clears the fp8 calibration (its scales belong to the old weights)."""
    import paper_2203_07747_amd as rtn
    from paper_2203_07747_amd._lib import RtnError, RTN_EINVAL
    Ws, bs = xavier_params(2, 256, seed=5)
    m = rtn.Model(Ws, bs)
    try:
        xc, uc = sample_nodes(2048, seed=SEED_CALIB)
        m.calibrate(torch.from_numpy(xc).cuda(), torch.from_numpy(uc).cuda())
        x, u = sample_nodes(40, seed=4)
        x[5, 7] = np.nan
        print("[gpu] fp8 NaN input", flush=True)
        out = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, "fp8", DT, want_status=True)
        torch.cuda.synchronize()
        st = out["status"].cpu().numpy()
        assert st[5] & 1 and st[5] & 2
        assert np.all(st[np.arange(40) != 5] == 0)
        m.set_params(Ws, bs)
        with pytest.raises(RtnError) as e:
            rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, "fp8", DT)
        assert e.value.code == RTN_EINVAL
    finally:
        m.close()


@pytest.mark.parametrize("H,path", [(64, 1), (256, 1), (64, 0), (256, 0)])
def test_status_flags_each_path(torch, H, path):
    """Status bits from the one-launch small network kernel (width 64), the tail kernel
    of the per-layer path (wider) and the layer-chain path, forced through the tuning table."""
    import paper_2203_07747_amd as rtn
    Ws, bs = xavier_params(2, H)
    x, u = sample_nodes(21, seed=6)
    x[17, 8] = np.nan
    m = rtn.Model(Ws, bs)
    try:
        rtn.tune_set("fp32", H, 2, 21, (path, 0, 0, 0, 0))
        print(f"[gpu] status flags H={H} path={path}", flush=True)
        out = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, "fp32", DT, want_status=True)
        torch.cuda.synchronize()
        st = out["status"].cpu().numpy()
    finally:
        rtn.tune_set("fp32", H, 2, 21, (0, 0, 0, 0, 0))
        m.close()
    assert st[17] & 1 and st[17] & 2
    assert np.all(st[np.arange(21) != 17] == 0)


def test_bf16_matches_emulation_and_oracle(torch):
    Ws, bs = xavier_params(5, 512, seed=0)
    x, u = sample_nodes(2000, seed=1)
    res = gpu_linearize(torch, x, u, Ws, bs, "bf16")
    net = MLP(Ws, bs)
    ref = linearize_affine(x, u, net, DT)
    check_against(res, ref, 1e-2)
    check_network(torch, res, ref, x, u, net, "bf16")


# (path, forward variant, forward workgroups, reverse variant, reverse workgroups) the
# autotuner keeps for 14-5x512-6 bf16 at 122,452 nodes on MI355X (one round of 256
# resident 128-row workgroups forward; one 128-row workgroup per block reverse, or
# 256 / 512 persistent ones, whose last partly filled round of the 5,740 blocks runs
# as 64-row blocks in a second launch), and the default shapes
C3_CHOICES = [(0, 4, 256, 4, 5740), (0, 4, 256, 4, 256), (0, 0, 0, 0, 0)]


@pytest.mark.parametrize("choice", C3_CHOICES, ids=["bench-shape", "bench-shape-persistent", "default-shape"])
def test_c3_full_size_sampled(torch, choice):
    """The benchmarked workload (4096 instances, ragged horizons, 14-5x512-6 bf16) at full size
    in the launch configuration the benchmark times; the oracle checks a seeded sample of
    nodes, the network's part included."""
    import paper_2203_07747_amd as rtn
    cfg, off, x, u, Ws, bs = config_workload("c3")
    n = x.shape[0]
    rtn.tune_set("bf16", 512, 5, n, choice)
    try:
        print(f"[gpu] c3 tile choice {choice}", flush=True)
        res = gpu_linearize(torch, x, u, Ws, bs, "bf16", offsets=off)
    finally:
        rtn.tune_set("bf16", 512, 5, n, (0, 0, 0, 0, 0))
    idx = np.sort(np.random.default_rng(11).choice(n, 1500, replace=False))
    idx = np.unique(np.concatenate([idx, [0, n - 1]]))
    net = MLP(Ws, bs)
    ref = linearize_affine(x[idx], u[idx], net, cfg.dt)
    check_against(res, ref, 1e-2, idx=idx)
    check_network(torch, res, ref, x[idx], u[idx], net, "bf16", idx=idx)
    for k in ("x_next", "A", "B"):
        assert np.all(np.isfinite(res[k]))


@pytest.mark.parametrize("L,H", [(1, 64), (1, 256), (4, 1024)])
def test_fp8_matches_emulation_and_oracle(torch, L, H):
    """The GPU repeats the oracle's E4M3 roundings (median agreement at accumulation
    level, a few nodes further off where a different summation order moves an operand
    across a rounding boundary); the network's part stays within the fp8 bounds of the
    FP64 oracle."""
    Ws, bs = xavier_params(L, H, seed=0)
    xc, uc = sample_nodes(8192, seed=SEED_CALIB)
    x, u = sample_nodes(600, seed=1)
    res = gpu_linearize(torch, x, u, Ws, bs, "fp8", calib=(xc, uc))
    net = MLP(Ws, bs)
    ref = linearize_affine(x, u, net, DT)
    check_against(res, ref, 5e-2)
    sc = calibrate_scales(net, pack_input(xc, uc))
    check_network(torch, res, ref, x, u, net, "fp8", scales=sc)


def test_fp8_calibration_scales_match_oracle(torch):
    import paper_2203_07747_amd as rtn
    Ws, bs = xavier_params(3, 256, seed=2)
    xc, uc = sample_nodes(4096, seed=SEED_CALIB)
    m = rtn.Model(Ws, bs)
    m.calibrate(torch.from_numpy(xc).cuda(), torch.from_numpy(uc).cuda())
    got = m.scales()
    sc = calibrate_scales(MLP(Ws, bs), pack_input(xc, uc))
    want = np.array(sc["w"] + sc["a"] + sc["g"])
    np.testing.assert_allclose(got, want, rtol=1e-5)
    m.close()


@pytest.mark.parametrize("variant", [0, 1])
def test_c4_fp8_full_size_sampled(torch, variant):
    """14-4x1024-6 fp8 over 65,536 instances x 20 nodes, default shape (the one the
    benchmark times) and the alternative shape, workgroup count as the benchmark launches
    it; calibrated on 8,192 seeded nodes on both sides, so the emulation uses the oracle's
    own scales."""
    import paper_2203_07747_amd as rtn
    cfg, off, x, u, Ws, bs = config_workload("c4")
    n = x.shape[0]
    xc, uc = sample_nodes(8192, seed=SEED_CALIB)
    rtn.tune_set("fp8", 1024, 4, n, (0, variant, 0, variant, 0))
    try:
        print(f"[gpu] c4 fp8 variant {variant}", flush=True)
        res = gpu_linearize(torch, x, u, Ws, bs, "fp8", offsets=off, calib=(xc, uc))
    finally:
        rtn.tune_set("fp8", 1024, 4, n, (0, 0, 0, 0, 0))
    idx = np.unique(np.concatenate([np.random.default_rng(12).choice(n, 400, replace=False), [0, n - 1]]))
    net = MLP(Ws, bs)
    ref = linearize_affine(x[idx], u[idx], net, cfg.dt)
    check_against(res, ref, 5e-2, idx=idx)
    sc = calibrate_scales(net, pack_input(xc, uc))
    check_network(torch, res, ref, x[idx], u[idx], net, "fp8", idx=idx, scales=sc)


def test_graph_replays_match_eager(torch):
    """rtn_linearize replays a captured graph for repeated argument sets; every replay (with new
    input values written into the same buffers, eager work and syncs in between) must equal
    the eager launches (profiling forces the eager path)."""
    import paper_2203_07747_amd as rtn
    Ws, bs = xavier_params(4, 512, seed=3)
    m = rtn.Model(Ws, bs)
    n = 777
    xt = torch.empty((n, 13), device="cuda"); ut = torch.empty((n, 4), device="cuda")
    out_g, out_e = {}, {}
    for rep in range(4):
        x, u = sample_nodes(n, seed=100 + rep)
        xt.copy_(torch.from_numpy(x)); ut.copy_(torch.from_numpy(u))
        rtn.profile_enable(True)
        rtn.linearize(xt, ut, m, "bf16", out=out_e)
        torch.cuda.synchronize()
        rtn.profile_collect()
        rtn.profile_enable(False)
        eager = {k: v.clone() for k, v in out_e.items()}
        rtn.linearize(xt, ut, m, "bf16", out=out_g)
        torch.cuda.synchronize()
        for k in ("x_next", "A", "B", "f_D", "J_D"):
            assert torch.equal(out_g[k], eager[k]), (rep, k)
    m.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 1e-2)])
def test_exact_linearisation_matches_oracle(torch, prec, tol):
    """rtn_linearize_exact (network at all four RK4 stage points) against the oracle's exact
    variant, the network's share of A and B included, and its gap to the local
    approximation of eq. (4)."""
    import paper_2203_07747_amd as rtn
    from oracle.rk4 import linearize_exact
    from net_bounds import ORACLE_BOUNDS, rel_rows
    Ws, bs = xavier_params(3, 256, seed=4)
    x, u = sample_nodes(300, seed=21)
    m = rtn.Model(Ws, bs)
    print(f"[gpu] linearize_exact n=300 prec={prec}", flush=True)
    out = rtn.linearize_exact(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, prec, DT)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    ref = linearize_exact(x, u, MLP(Ws, bs), DT)
    for name, r in zip(("x_next", "A", "B"), ref):
        e = rel(res[name], r).max()
        print(f"  {name} max rel err {e:.2e}")
        assert e <= tol
    A_nom, B_nom = gpu_nominal(torch, x, u)
    ref_nom = linearize_affine(x, u, None, DT)
    dA = rel_rows(res["A"].astype(np.float64) - A_nom, ref[1] - ref_nom[1]).max()
    dB = rel_rows(res["B"].astype(np.float64) - B_nom, ref[2] - ref_nom[2]).max()
    print(f"  network's share: dA {dA:.2e} dB {dB:.2e}")
    # fp32: A - A_nominal is ~1e-3 in norm while A and A_nominal hold the identity, so
    # their fp32 rounding (~1e-7 per element) alone is a few 1e-4 of the difference
    bound = 5e-3 if prec == "fp32" else ORACLE_BOUNDS["bf16"]["dA"]
    assert dA <= bound and dB <= bound
    aff = linearize_affine(x, u, MLP(Ws, bs), DT)
    gap = rel(aff[1], ref[1]).max()
    print(f"  affine-vs-exact gap on A: {gap:.2e}")
    m.close()


# --------------------------------------------------------------- tile autotuner
# Every tile shape and workgroup count the autotuner can choose is a code path
# of its own: each is forced here and checked against the oracle.

@pytest.mark.parametrize("prec,H,L,tol", [("fp32", 512, 2, 1e-5), ("bf16", 512, 3, 1e-2), ("bf16", 1024, 2, 1e-2),
                                          ("fp8", 512, 3, 5e-2), ("fp8", 1024, 2, 5e-2)])
def test_every_tile_variant_and_grid_matches_oracle(torch, prec, H, L, tol):
    # 733 nodes: ragged in every tile height (32, 64, 96) for both directions
    check_tile_choices(torch, prec, H, L, tol, 733,
                       [(0, 0, 0, 0, 0), (0, 1, 0, 1, 0), (0, 1, 1, 1, 1), (0, 0, 3, 1, 7), (0, 1, 5, 0, 2),
                        (0, 0, 10000, 0, 10000), (0, 2, 0, 2, 0), (0, 2, 3, 2, 5), (0, 2, 10000, 2, 1),
                        (0, 0, 0, 3, 0), (0, 2, 0, 3, 3), (0, 2, 0, 4, 0), (0, 0, 0, 4, 3), (0, 4, 0, 4, 0),
                        (0, 4, 5, 0, 0), (0, 0, 0, 4, 8), (0, 4, 0, 4, 16), (0, 4, 4, 4, 13)])


# Variant 4 hands a last round of 128-row blocks that leaves at most half of the
# workgroups busy to 64-row blocks, at most three quarters to 96-row blocks, in a
# second launch, whose first reverse row need not start a node.  850 nodes: the
# forward's 7 blocks on 4 workgroups leave 3 (96-row tail), on 7 none; the
# reverse's 40 blocks on 11 leave 7 (96-row tail from row 4224, a node start), on
# 17 leave 6 (64-row tail from row 4352 = 6 * 725 + 2), on 7 leave 5 (96-row tail
# from row 4480 = 6 * 746 + 4).
@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_tail_launch_shapes_match_oracle(torch, prec):
    check_tile_choices(torch, prec, 512, 3, 1e-2 if prec == "bf16" else 5e-2, 850,
                       [(0, 4, 4, 4, 11), (0, 4, 4, 4, 17), (0, 4, 7, 4, 7)])


def check_tile_choices(torch, prec, H, L, tol, n, choices):
    import paper_2203_07747_amd as rtn
    x, u = sample_nodes(n, seed=41)
    Ws, bs = xavier_params(L, H, seed=42)
    m = rtn.Model(Ws, bs)
    if prec == "fp8":
        xc, uc = sample_nodes(4096, seed=SEED_CALIB)
        m.calibrate(torch.from_numpy(xc).cuda(), torch.from_numpy(uc).cuda())
    net = MLP(Ws, bs)
    ref = linearize_affine(x, u, net, DT)
    sc = calibrate_scales(net, pack_input(xc, uc)) if prec == "fp8" else None
    xt, ut = torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda()
    try:
        for choice in choices:
            if (choice[3] in (3, 4) or choice[1] == 4) and (prec == "fp32" or H != 512):
                continue
            print(f"[gpu] tile choice {choice} prec={prec} H={H} L={L} n={n}", flush=True)
            rtn.tune_set(prec, H, L, n, choice)
            out = rtn.linearize(xt, ut, m, prec, DT)
            torch.cuda.synchronize()
            res = {k: v.cpu().numpy() for k, v in out.items()}
            errs = check_against(res, ref, tol)
            if prec == "fp32":
                assert errs["f_D"] < 1e-5 and errs["J_D"] < 2e-5
            else:
                check_network(torch, res, ref, x, u, net, prec, scales=sc)
    finally:
        rtn.tune_set(prec, H, L, n, (0, 0, 0, 0, 0))
        m.close()


def test_autotuner_keeps_a_valid_choice_and_results_match(torch):
    import paper_2203_07747_amd as rtn
    cfg, off, x, u, Ws, bs = config_workload("c2")
    x, u = np.tile(x, (300, 1)), np.tile(u, (300, 1))  # 6000 nodes: a size class no other test uses
    n = x.shape[0]
    m = rtn.Model(Ws, bs)
    rtn.tune_mode(True)
    assert rtn.tune_get("bf16", 512, 4, n) is None
    print(f"[gpu] autotune n={n}", flush=True)
    out = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, "bf16", DT)
    torch.cuda.synchronize()
    got = rtn.tune_get("bf16", 512, 4, n)
    assert got is not None
    choice, ms = got
    print(f"  kept {choice}, forward {ms[0]:.3f} ms, reverse {ms[1]:.3f} ms", flush=True)
    assert choice[0] == 0 and 0 <= choice[1] <= 4 and 0 <= choice[3] <= 4 and min(choice) >= 0
    assert ms[0] > 0 and ms[1] > 0
    ref = linearize_affine(x[:20], u[:20], MLP(Ws, bs), DT)
    res = {k: v.cpu().numpy() for k, v in out.items()}
    for k in range(0, n, 997):  # the tiled copies of the 20 nodes give the same outputs everywhere
        check_against({kk: vv[k - k % 20:k - k % 20 + 20] for kk, vv in res.items()}, ref, 1e-2)
    m.close()


# width 64 with <= 4 hidden layers takes the one-launch kernel (16 nodes per workgroup)
# and wider ones (L >= 2) end in the tail kernel: n = 1 and a last block of one node included
@pytest.mark.parametrize("H,L,n", [(64, 2, 10), (64, 1, 7), (64, 3, 45), (64, 4, 100), (64, 2, 16), (64, 5, 33),
                                   (512, 4, 20), (256, 3, 45), (1024, 2, 33), (128, 5, 300), (128, 2, 1),
                                   (512, 2, 17), (256, 1, 12)])
def test_small_batch_path_matches_oracle(torch, H, L, n):
    """The per-layer small-batch path (fp32), forced through the tuning table."""
    import paper_2203_07747_amd as rtn
    x, u = sample_nodes(n, seed=51)
    Ws, bs = xavier_params(L, H, seed=52)
    bs = [np.random.default_rng(53).normal(size=b.shape).astype(np.float32) * 0.1 for b in bs]
    m = rtn.Model(Ws, bs)
    try:
        rtn.tune_set("fp32", H, L, n, (1, 0, 0, 0, 0))
        print(f"[gpu] small-batch path H={H} L={L} n={n}", flush=True)
        out = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, "fp32", DT)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items()}
        errs = check_against(res, linearize_affine(x, u, MLP(Ws, bs), DT), 1e-5)
        assert errs["f_D"] < 1e-5 and errs["J_D"] < 1e-5
    finally:
        rtn.tune_set("fp32", H, L, n, (0, 0, 0, 0, 0))
        m.close()


def test_prepared_call_matches_and_sees_new_data(torch):
    """LinearizeCall marshals once; later calls use the current contents of x, u."""
    import paper_2203_07747_amd as rtn
    cfg, off, x, u, Ws, bs = config_workload("c1")
    m = rtn.Model(Ws, bs)
    xt, ut = torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda()
    call = rtn.LinearizeCall(xt, ut, m, "fp32", cfg.dt, offsets=off)
    for seed in (1, 2):
        x2, u2 = sample_nodes(x.shape[0], seed=seed)
        xt.copy_(torch.from_numpy(x2))
        ut.copy_(torch.from_numpy(u2))
        print(f"[gpu] prepared linearize call, seed {seed}", flush=True)
        out = call()
        ref = rtn.linearize(xt, ut, m, "fp32", cfg.dt, offsets=off)
        torch.cuda.synchronize()
        for k in ("x_next", "A", "B", "f_D", "J_D"):
            np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k].cpu().numpy())
        check_against({k: v.cpu().numpy() for k, v in out.items()}, linearize_affine(x2, u2, MLP(Ws, bs), cfg.dt),
                      1e-5)
    m.close()

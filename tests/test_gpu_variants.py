"""GPU parity of rtn_linearize for the simplified residual models of Sec. VI:
f_Da(v_B) and f_Da,u(v_B, u), whose input is the body-frame velocity
v_B = conj(q) (.) v (and u) and whose three outputs add to v-dot.

The oracle linearises them at the node with the state Jacobian taken through
v_B (oracle.rk4.linearize_affine with mode).  Bounds as for the full model:
FP32 1e-5, BF16 1e-2, FP8 5e-2 on x_{k+1}, A_k, B_k (maximum over nodes of the
per-node relative Frobenius error).  The library returns f_D and J_D in its
embedded layout (outputs 0..2, input slots 0..2 for v_B and 10..13 for u), which
the tests map back to the variant's own shapes.
"""
import numpy as np
import pytest

from workload import SEED_CALIB, sample_nodes, xavier_params
from oracle.mlp import MLP, INPUT_VB, INPUT_VB_U, D_IN, D_OUT, pack_input_mode
from oracle.rk4 import linearize_affine
from oracle.quant import emulated_jacobian, calibrate_scales

from net_bounds import (assert_within_emulation_bounds, assert_within_oracle_bounds, bounds_for, fp8_emulation_bounds,
                        network_errors)

pytestmark = pytest.mark.gpu
DT = 0.05
MODES = {"vb": INPUT_VB, "vb_u": INPUT_VB_U}


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


def variant_params(name, L, H, seed):
    mode = MODES[name]
    Ws, bs = xavier_params(L, H, seed=seed, d_in=D_IN[mode], d_out=D_OUT[mode])
    rng = np.random.default_rng(seed + 100)
    bs = [rng.uniform(-0.2, 0.2, size=b.shape).astype(np.float32) for b in bs]  # exercise every bias
    return Ws, bs


def embedded(name, y, J):
    """Variant (y (n,3), J (n,3,d_in)) in the library's 6-output / 14-slot layout."""
    n = y.shape[0]
    y6 = np.zeros((n, 6))
    y6[:, :3] = y
    J6 = np.zeros((n, 6, 14))
    J6[:, :3, 0:3] = J[:, :, 0:3]
    if name == "vb_u":
        J6[:, :3, 10:14] = J[:, :, 3:7]
    return y6, J6


def run(torch, name, x, u, Ws, bs, prec, calib=None, path=None):
    """rtn_linearize of a variant model; path 0/1 forces the layer-chain or the
    small-batch kernels for this (precision, width, depth, size class)."""
    import paper_2203_07747_amd as rtn
    H, L, n = Ws[0].shape[0], len(Ws) - 1, x.shape[0]
    print(f"[gpu] variant {name} linearize n={n} prec={prec} L={L} H={H} path={path}", flush=True)
    model = rtn.Model(Ws, bs, "silu", input=name)
    try:
        if calib is not None:
            model.calibrate(torch.from_numpy(calib[0]).cuda(), torch.from_numpy(calib[1]).cuda())
        if path is not None:
            rtn.tune_set(prec, H, L, n, (path, 0, 0, 0, 0))
        out = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), model, prec, DT,
                            want_status=True)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        if path is not None:
            rtn.tune_set(prec, H, L, n, (0, 0, 0, 0, 0))
        model.close()
    return res


def check_network(torch, name, res, ref, x, u, net, prec, idx=None, scales=None):
    """The network's part (f_D, J_D in the embedded layout, A - A_nominal, B - B_nominal)
    within the bounds of its precision against the FP64 oracle (widened to twice the
    rounding emulation's own error on these nodes where that is larger), and f_D, J_D
    against the rounding emulation.  f_Da(v_B) does not see u, so B's network share is
    only the state path's second-order cross term; it is bounded for f_Da,u only."""
    import paper_2203_07747_amd as rtn
    pick = (lambda a: a) if idx is None else (lambda a: a[idx])
    mode = MODES[name]
    xr, Ar, Br, yr, Jr = ref
    y6, J6 = embedded(name, yr, Jr)
    nom = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), None, "fp32", DT)
    torch.cuda.synchronize()
    ref_nom = linearize_affine(x, u, None, DT)
    errs = network_errors(pick(res["f_D"]), pick(res["J_D"]), pick(res["A"]), pick(res["B"]),
                          nom["A"].cpu().numpy(), nom["B"].cpu().numpy(), (xr, Ar, Br, y6, J6), ref_nom)
    ye, Je = emulated_jacobian(net, pack_input_mode(x, u, mode), prec, scales)
    em = linearize_affine(x, u, None, DT, params=(ye, Je), mode=mode)
    em_errs = network_errors(ye, Je, em[1], em[2], ref_nom[1], ref_nom[2], ref, ref_nom)
    skip = ("dB",) if name == "vb" else ()
    assert_within_oracle_bounds(errs, prec, bounds_for(prec, em_errs, skip))
    ye6, Je6 = embedded(name, ye, Je)
    eb = fp8_emulation_bounds(net, pack_input_mode(x, u, mode), scales, ye, Je) if prec == "fp8" else None
    assert_within_emulation_bounds(pick(res["f_D"]), pick(res["J_D"]), ye6, Je6, prec, eb)


def compare(name, res, ref, tol, idx=None):
    xr, Ar, Br, yr, Jr = ref
    y6, J6 = embedded(name, yr, Jr)
    pick = (lambda a: a) if idx is None else (lambda a: a[idx])
    errs = {k: float(rel(pick(res[k]), r).max()) for k, r in
            (("x_next", xr), ("A", Ar), ("B", Br), ("f_D", y6), ("J_D", J6))}
    print("  max rel err:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k in ("x_next", "A", "B"):
        assert errs[k] <= tol, (k, errs[k], tol)
    # the embedding's padding stays exactly zero
    assert np.all(pick(res["f_D"])[:, 3:] == 0)
    Jg = pick(res["J_D"])
    assert np.all(Jg[:, 3:, :] == 0) and np.all(Jg[:, :, 3:10] == 0)
    if name == "vb":
        assert np.all(Jg[:, :, 10:] == 0)
    assert np.all(pick(res["status"]) == 0)
    return errs


@pytest.mark.parametrize("name", ["vb", "vb_u"])
@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("H,L,n", [(64, 2, 1), (64, 3, 300), (256, 2, 129), (512, 4, 97)])
def test_variant_fp32_matches_oracle(torch, name, path, H, L, n):
    Ws, bs = variant_params(name, L, H, seed=H + L)
    x, u = sample_nodes(n, seed=3 + n)
    res = run(torch, name, x, u, Ws, bs, "fp32", path=path)
    ref = linearize_affine(x, u, MLP(Ws, bs), DT, mode=MODES[name])
    errs = compare(name, res, ref, 1e-5)
    assert errs["f_D"] < 1e-5 and errs["J_D"] < 1e-5


@pytest.mark.parametrize("name", ["vb", "vb_u"])
def test_variant_bf16_many_nodes(torch, name):
    """The layer-chain kernels at a batch of 20,000 nodes (several hundred row
    blocks and a ragged tail), bf16; the oracle checks a seeded sample."""
    Ws, bs = variant_params(name, 5, 512, seed=21)
    n = 20000
    x, u = sample_nodes(n, seed=17)
    res = run(torch, name, x, u, Ws, bs, "bf16")
    idx = np.unique(np.concatenate([np.random.default_rng(5).choice(n, 600, replace=False), [0, n - 1]]))
    net = MLP(Ws, bs)
    ref = linearize_affine(x[idx], u[idx], net, DT, mode=MODES[name])
    compare(name, res, ref, 1e-2, idx=idx)
    check_network(torch, name, res, ref, x[idx], u[idx], net, "bf16", idx=idx)


@pytest.mark.parametrize("name", ["vb", "vb_u"])
def test_variant_fp8_calibrated(torch, name):
    import paper_2203_07747_amd as rtn
    mode = MODES[name]
    Ws, bs = variant_params(name, 2, 256, seed=31)
    xc, uc = sample_nodes(4096, seed=SEED_CALIB)
    x, u = sample_nodes(600, seed=8)
    net = MLP(Ws, bs)
    # static scales: the embedding's zero rows and columns change no amax
    m = rtn.Model(Ws, bs, "silu", input=name)
    m.calibrate(torch.from_numpy(xc).cuda(), torch.from_numpy(uc).cuda())
    got = m.scales()
    m.close()
    sc = calibrate_scales(net, pack_input_mode(xc, uc, mode))
    np.testing.assert_allclose(got, np.array(sc["w"] + sc["a"] + sc["g"]), rtol=1e-5)
    res = run(torch, name, x, u, Ws, bs, "fp8", calib=(xc, uc))
    ref = linearize_affine(x, u, net, DT, mode=mode)
    compare(name, res, ref, 5e-2)
    check_network(torch, name, res, ref, x, u, net, "fp8", scales=sc)


@pytest.mark.parametrize("name", ["vb", "vb_u"])
def test_variant_params_round_trip_and_unsupported_calls(torch, name):
    import paper_2203_07747_amd as rtn
    from paper_2203_07747_amd._lib import RtnError, RTN_ENOTSUP
    Ws, bs = variant_params(name, 2, 64, seed=41)
    m = rtn.Model(Ws, bs, "silu", input=name)
    try:
        flat = np.concatenate([a.ravel() for W, b in zip(Ws, bs) for a in (W, b)])
        np.testing.assert_array_equal(m.get_params(), flat)
        # parameters replaced through the user layout take effect
        Ws2 = [1.5 * W for W in Ws]
        m.set_params(Ws2, bs)
        np.testing.assert_array_equal(m.get_params(),
                                      np.concatenate([a.ravel() for W, b in zip(Ws2, bs) for a in (W, b)]))
        x, u = sample_nodes(33, seed=2)
        out = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, "fp32", DT)
        torch.cuda.synchronize()
        ref = linearize_affine(x, u, MLP(Ws2, bs), DT, mode=MODES[name])
        assert rel(out["A"].cpu().numpy(), ref[1]).max() < 1e-5
        with pytest.raises(RtnError) as e:
            rtn.linearize_second(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, DT)
        assert e.value.code == RTN_ENOTSUP
        z = torch.zeros((8, 14), device="cuda")
        with pytest.raises(RtnError) as e:
            m.forward_batch(z, "fp32")
        assert e.value.code == RTN_ENOTSUP
    finally:
        m.close()

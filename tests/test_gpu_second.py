"""GPU parity of rtn_linearize_second (the second-order local approximation of
eq. (4), fp32) against the FP64 oracle: x_{k+1}, A_k, B_k within 1e-5 (per-node
relative Frobenius, max over nodes), f_D-bar and J_D within 1e-5, the network
Hessian H_D within 1e-4 (fp32 sums over the layer width)."""
import numpy as np
import pytest

from workload import config_workload, sample_nodes, xavier_params
from oracle.mlp import MLP
from oracle.rk4 import linearize_quadratic

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


def run(torch, x, u, Ws, bs, act="silu", offsets=None):
    import paper_2203_07747_amd as rtn
    print(f"[gpu] linearize_second n={x.shape[0]} L={len(Ws) - 1} H={Ws[0].shape[0]} act={act}", flush=True)
    m = rtn.Model(Ws, bs, act)
    out = rtn.linearize_second(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, DT, offsets=offsets)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    m.close()
    return res


def check(res, ref, tol_h=1e-4):
    names = ("x_next", "A", "B", "f_D", "J_D", "H_D")
    errs = {k: float(rel(res[k], r).max()) for k, r in zip(names, ref)}
    print("  max rel err:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k in names[:5]:
        assert errs[k] < 1e-5, (k, errs[k])
    assert errs["H_D"] < tol_h, errs["H_D"]


@pytest.mark.parametrize("key", ["c1", "c2"])
def test_configs_match_oracle(torch, key):
    cfg, off, x, u, Ws, bs = config_workload(key)
    check(run(torch, x, u, Ws, bs, offsets=off), linearize_quadratic(x, u, MLP(Ws, bs), cfg.dt))


@pytest.mark.parametrize("H,L,n", [(64, 1, 7), (128, 3, 33), (256, 2, 129), (1024, 2, 17), (64, 2, 4100)])
def test_widths_depths_and_chunks(torch, H, L, n):
    x, u = sample_nodes(n, seed=61)
    Ws, bs = xavier_params(L, H, seed=62)
    bs = [np.random.default_rng(63).normal(size=b.shape).astype(np.float32) * 0.1 for b in bs]
    check(run(torch, x, u, Ws, bs), linearize_quadratic(x, u, MLP(Ws, bs), DT))


def test_linear_network_has_zero_hessian_and_first_order_step(torch):
    import paper_2203_07747_amd as rtn
    x, u = sample_nodes(40, seed=64)
    Ws, bs = xavier_params(2, 64, seed=65)
    res = run(torch, x, u, Ws, bs, act="identity")
    assert np.abs(res["H_D"]).max() == 0.0
    m = rtn.Model(Ws, bs, "identity")
    first = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, "fp32", DT)
    torch.cuda.synchronize()
    for k in ("x_next", "A", "B"):
        np.testing.assert_allclose(res[k], first[k].cpu().numpy(), rtol=1e-5, atol=1e-6)
    m.close()

"""On-device training of the residual network (Sec. VII) against the FP64 oracle,
and the gain of the trained network over the nominal model."""
import numpy as np
import pytest

from workload import QUAD, SEED_TRAIN, TRAIN, sample_nodes, xavier_params
from oracle.mlp import MLP, pack_input, flatten_params
from oracle.train import mse_and_grads, Adam, train_step as oracle_train_step
from oracle.simulator import make_transitions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def batch(n, seed):
    x, u = sample_nodes(n, seed=seed)
    z = pack_input(x, u).astype(np.float32)
    t = np.random.default_rng(seed + 100).normal(size=(n, 6)).astype(np.float32)
    return z, t


def gpu_grads(torch, model, z, t, prec):
    import paper_2203_07747_amd as rtn
    zt, tt = torch.from_numpy(z).cuda(), torch.from_numpy(t).cuda()
    model.zero_grad()
    y = model.forward_batch(zt, prec)
    dy = 2.0 * (y - tt) / y.numel()
    din = model.backward_batch(dy)
    torch.cuda.synchronize()
    return y.cpu().numpy(), model.get_grad(), din.cpu().numpy()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-2)])
@pytest.mark.parametrize("L,H,B", [(2, 64, 100), (4, 512, 4096)])
def test_gradients_match_oracle(torch, prec, tol, L, H, B):
    import paper_2203_07747_amd as rtn
    print(f"[gpu] grads prec={prec} L={L} H={H} B={B}", flush=True)
    Ws, bs = xavier_params(L, H, seed=1)
    bs = [np.random.default_rng(2).normal(size=b.shape).astype(np.float32) * 0.1 for b in bs]
    m = rtn.Model(Ws, bs)
    z, t = batch(B, 3)
    y, g, din = gpu_grads(torch, m, z, t, prec)
    net = MLP(Ws, bs)
    loss, dWs, dbs, dz = mse_and_grads(net, z, t)
    ref = flatten_params(dWs, dbs)
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    erz = np.linalg.norm(din - dz) / np.linalg.norm(dz)
    print(f"  rel err grad {err:.2e} dz {erz:.2e}")
    assert err < tol and erz < tol
    # per layer as well (a wrong layer cannot hide behind the others)
    off = 0
    for W, b in zip(dWs, dbs):
        k = W.size + b.size
        e = np.linalg.norm(g[off:off + k] - ref[off:off + k]) / np.linalg.norm(ref[off:off + k])
        assert e < 3 * tol, e
        off += k
    m.close()


def test_gradient_finite_differences_on_gpu_loss(torch):
    """Central differences of the GPU's own fp32 loss agree with its backward pass."""
    import paper_2203_07747_amd as rtn
    Ws, bs = xavier_params(2, 64, seed=5)
    z, t = batch(64, 6)
    m = rtn.Model(Ws, bs)
    _, g, _ = gpu_grads(torch, m, z, t, "fp32")
    zt, tt = torch.from_numpy(z).cuda(), torch.from_numpy(t).cuda()

    def loss_at(Wp, bp):
        m.set_params(Wp, bp)
        y = m.forward_batch(zt, "fp32")
        return float(((y - tt) ** 2).mean().double())

    h = 1e-2
    off = 0
    rng = np.random.default_rng(7)
    for l in range(3):
        for _ in range(3):
            i, j = rng.integers(0, Ws[l].shape[0]), rng.integers(0, Ws[l].shape[1])
            Wp = [W.copy() for W in Ws]; Wp[l][i, j] += h
            Wm = [W.copy() for W in Ws]; Wm[l][i, j] -= h
            fd = (loss_at(Wp, bs) - loss_at(Wm, bs)) / (2 * h)
            an = g[off + i * Ws[l].shape[1] + j]
            assert abs(fd - an) < 2e-3 * max(1.0, abs(an)), (l, i, j, fd, an)
        off += Ws[l].size + bs[l].size
    m.close()


def test_train_step_matches_oracle_adam(torch):
    import paper_2203_07747_amd as rtn
    Ws, bs = xavier_params(2, 64, seed=8)
    z, t = batch(256, 9)
    m = rtn.Model(Ws, bs)
    zt, tt = torch.from_numpy(z).cuda(), torch.from_numpy(t).cuda()
    net = MLP(Ws, bs)
    opt = Adam(net.Ws + net.bs, lr=1e-3)
    for step in range(3):
        loss = m.train_step(zt, tt, lr=1e-3, prec="fp32")
        lo, net = oracle_train_step(net, opt, z, t)
        torch.cuda.synchronize()
        assert abs(float(loss.item()) - lo) < 1e-5 * max(1.0, lo)
    got = m.get_params()
    ref = flatten_params(net.Ws, net.bs)
    assert np.max(np.abs(got - ref)) < 1e-5
    mm, vv, st = m.get_adam()
    assert st == 3
    m.close()


def test_autograd_input_gradient_equals_linearizer_jacobian(torch):
    """d(sum of outputs)/dz through the training kernels = the Jacobian rows summed,
    as computed by the linearisation kernels (two independent GPU paths)."""
    import paper_2203_07747_amd as rtn
    Ws, bs = xavier_params(3, 256, seed=10)
    m = rtn.Model(Ws, bs)
    x, u = sample_nodes(500, seed=11)
    z = torch.from_numpy(pack_input(x, u).astype(np.float32)).cuda().requires_grad_(True)
    F = rtn.mlp_function()
    y = F.apply(z, m, "fp32")
    y.sum().backward()
    lin = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, "fp32")
    torch.cuda.synchronize()
    np.testing.assert_allclose(y.detach().cpu().numpy(), lin["f_D"].cpu().numpy(), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(z.grad.cpu().numpy(), lin["J_D"].cpu().numpy().sum(axis=1), rtol=1e-4, atol=1e-5)
    m.close()


@pytest.fixture(scope="module")
def trained(torch):
    """Fit 14-4x512-6 (bf16, Adam lr 1e-3, batch 4096) to 2M drag-simulator transitions
    (Sec. VII: recorded transitions, re-simulated with the nominal model, the difference
    as label), four epochs; prints the mean training loss of every epoch."""
    import paper_2203_07747_amd as rtn
    dt = TRAIN["dt"]
    n_train = TRAIN["n_transitions"]
    x, u = sample_nodes(n_train, seed=SEED_TRAIN)
    labels = []
    for c0 in range(0, n_train, 500_000):  # the simulator in chunks, with progress
        print(f"[gpu] simulating transitions {c0}..{min(n_train, c0 + 500_000)} of {n_train}", flush=True)
        labels.append(make_transitions(x[c0:c0 + 500_000], u[c0:c0 + 500_000], dt, seed=SEED_TRAIN + 1 + c0)[1])
    label = np.concatenate(labels)
    z = torch.from_numpy(pack_input(x, u).astype(np.float32)).cuda()
    y = torch.from_numpy(label.astype(np.float32)).cuda()
    del x, u, labels, label
    Ws, bs = xavier_params(TRAIN["n_hidden"], TRAIN["width"], seed=0)
    m = rtn.Model(Ws, bs)
    B = TRAIN["batch"]
    g = torch.Generator(device="cuda").manual_seed(0)
    epoch_loss = []
    first = None
    steps = n_train // B
    print(f"[gpu] training 14-4x512-6 bf16 on {n_train} transitions, {steps} steps per epoch", flush=True)
    for epoch in range(4):
        perm = torch.randperm(n_train, device="cuda", generator=g)
        total = torch.zeros((), device="cuda")
        for i in range(steps):
            idx = perm[i * B:(i + 1) * B]
            loss = m.train_step(z[idx].contiguous(), y[idx].contiguous(), lr=TRAIN["lr"], prec="bf16")
            if first is None:
                first = float(loss.item())
            total += loss[0]
        epoch_loss.append(float(total.item()) / steps)
        print(f"  epoch {epoch}: mean training loss {epoch_loss[-1]:.5f}", flush=True)
    print(f"  loss of the first batch {first:.4f}; mean loss per epoch:", [f"{v:.5f}" for v in epoch_loss])
    yield m, first, epoch_loss
    m.close()


def test_trained_residual_beats_nominal_model(torch, trained):
    """Next-state error of the linearisation with the trained network against the nominal
    model alone on held-out transitions."""
    import paper_2203_07747_amd as rtn
    m, first, losses = trained
    dt = TRAIN["dt"]
    xv, uv = sample_nodes(4096 * 20, seed=SEED_TRAIN + 7)
    xs, _ = make_transitions(xv, uv, dt, seed=SEED_TRAIN + 8)
    xt, ut = torch.from_numpy(xv).cuda(), torch.from_numpy(uv).cuda()
    off = np.arange(0, 4096 * 20 + 1, 20, dtype=np.int32)
    nom = rtn.linearize(xt, ut, None, "fp32", dt, offsets=off)["x_next"].cpu().numpy()
    lrn = rtn.linearize(xt, ut, m, "bf16", dt, offsets=off)["x_next"].cpu().numpy()
    e_nom = np.linalg.norm(nom[:, 7:13] - xs[:, 7:13], axis=1).mean()
    e_lrn = np.linalg.norm(lrn[:, 7:13] - xs[:, 7:13], axis=1).mean()
    print(f"  mean next-state [v, w] error: nominal {e_nom:.4e}  trained {e_lrn:.4e}  ratio {e_lrn / e_nom:.3f}")
    assert losses[-1] < 0.25 * first
    assert e_lrn < 0.5 * e_nom


def test_closed_loop_rollouts_trained_vs_nominal(torch, trained):
    """4096 MPC instances (N = 20) tracking circles at 2-4 m/s in closed loop with the
    drag plant, once with the trained residual and once with the nominal fallback: the
    trained model's one-step predictions are closer to the plant and it tracks better."""
    import paper_2203_07747_amd as rtn
    from closed_loop import run
    m, _, _ = trained
    print("[gpu] closed loop nominal", flush=True)
    nom = run(torch, rtn, None, "fp32")
    print(f"  nominal: {nom}", flush=True)
    print("[gpu] closed loop trained", flush=True)
    lrn = run(torch, rtn, m, "bf16")
    print(f"  trained: {lrn}", flush=True)
    assert nom["finite"] and lrn["finite"]
    assert lrn["pred_err"] < 0.5 * nom["pred_err"]
    assert lrn["track_err"] < nom["track_err"]


def test_closed_loop_with_input_box_trained_vs_nominal(torch, trained):
    """The same rollouts with the input box inside the QP (rtn_riccati_box)."""
    import paper_2203_07747_amd as rtn
    from closed_loop import run
    m, _, _ = trained
    print("[gpu] closed loop with input box, nominal", flush=True)
    nom = run(torch, rtn, None, "fp32", box=True)
    print(f"  nominal: {nom}", flush=True)
    print("[gpu] closed loop with input box, trained", flush=True)
    lrn = run(torch, rtn, m, "bf16", box=True)
    print(f"  trained: {lrn}", flush=True)
    assert nom["finite"] and lrn["finite"]
    assert lrn["pred_err"] < 0.5 * nom["pred_err"]
    assert lrn["track_err"] < nom["track_err"]

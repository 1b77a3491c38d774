"""GPU parity of rtn_riccati (fp64) against the oracle's recursion and brute-force KKT."""
import numpy as np
import pytest

from workload import config_workload, sample_horizons, offsets_from_horizons
from oracle.riccati import riccati_batched, kkt_bruteforce, lq_rollout_batched, box_lq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def random_lq(n, seed):
    rng = np.random.default_rng(seed)
    A = (np.eye(13) + 0.1 * rng.normal(size=(n, 13, 13))).astype(np.float32)
    B = (0.2 * rng.normal(size=(n, 13, 4))).astype(np.float32)
    return A, B, rng


def gpu_riccati(torch, A, B, Q, R, QN, off, c=None, q=None, r=None, qN=None):
    import paper_2203_07747_amd as rtn
    print(f"[gpu] riccati n={A.shape[0]} n_inst={len(off) - 1}", flush=True)
    dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = rtn.riccati(dev(A), dev(B), Q, R, QN, offsets=off, c=dev(c), q=dev(q), r=dev(r), qN=dev(qN), want_P=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def rel_max(a, b):
    a = a.reshape(a.shape[0], -1); b = b.reshape(b.shape[0], -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)))


def test_ragged_instances_with_affine_terms(torch):
    hz = sample_horizons(37, 1, 12, seed=4)
    off = offsets_from_horizons(hz)
    n = int(off[-1])
    A, B, rng = random_lq(n, 1)
    c = rng.normal(size=(n, 13)) * 0.1
    q = rng.normal(size=(n, 13)); r = rng.normal(size=(n, 4)); qN = rng.normal(size=(len(hz), 13))
    Q = np.eye(13); R = 0.1 * np.eye(4); QN = 2.0 * np.eye(13)
    res = gpu_riccati(torch, A, B, Q, R, QN, off, c, q, r, qN)
    K, kff, P = riccati_batched(off, A.astype(np.float64), B.astype(np.float64), Q, R, QN, c, q, r, qN)
    eK, ek, eP = rel_max(res["K"], K), rel_max(res["kff"], kff), rel_max(res["P"], P)
    print(f"  rel err K {eK:.2e} kff {ek:.2e} P {eP:.2e}")
    assert eK < 1e-9 and ek < 1e-9 and eP < 1e-9


def test_gains_match_bruteforce_kkt(torch):
    N = 3
    A, B, rng = random_lq(N, 2)
    c = rng.normal(size=(N, 13)) * 0.1
    Q = np.eye(13); R = 0.1 * np.eye(4); QN = np.eye(13)
    res = gpu_riccati(torch, A, B, Q, R, QN, np.array([0, N], np.int32), c=c)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    du0, _ = kkt_bruteforce(A64, B64, Q, R, QN, np.zeros(13), c)
    np.testing.assert_allclose(res["kff"][0], du0[0], atol=1e-10)
    for j in range(13):
        e = np.zeros(13); e[j] = 1
        du, _ = kkt_bruteforce(A64, B64, Q, R, QN, e, c)
        np.testing.assert_allclose(res["K"][0] @ e + res["kff"][0], du[0], atol=1e-10)


def test_linearized_c3_batch(torch):
    """Gains of the benchmarked workload's linearisation (4096 instances, ragged horizons)."""
    import paper_2203_07747_amd as rtn
    cfg, off, x, u, Ws, bs = config_workload("c3")
    m = rtn.Model(Ws, bs)
    lin = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), m, "bf16", cfg.dt, offsets=off)
    Q = np.eye(13); R = 0.1 * np.eye(4)
    out = rtn.riccati(lin["A"], lin["B"], Q, R, Q, offsets=off, want_P=False)
    torch.cuda.synchronize()
    A, B = lin["A"].cpu().numpy(), lin["B"].cpu().numpy()
    K = out["K"].cpu().numpy()
    assert np.all(np.isfinite(K))
    sel = np.random.default_rng(3).choice(len(off) - 1, 40, replace=False)
    for i in sel:
        a, b = off[i], off[i + 1]
        Ko, ko, _ = riccati_batched(np.array([0, b - a]), A[a:b].astype(np.float64), B[a:b].astype(np.float64), Q, R, Q)
        assert rel_max(K[a:b], Ko) < 1e-9
    m.close()


def test_indefinite_input_hessian_gives_nan(torch):
    A, B, _ = random_lq(4, 3)
    res = gpu_riccati(torch, A, B, np.eye(13), -np.eye(4), np.zeros((13, 13)), np.array([0, 4], np.int32))
    assert np.all(np.isnan(res["K"][3])) and np.all(np.isnan(res["kff"][3]))


def test_empty_and_single_node(torch):
    A, B, _ = random_lq(5, 5)
    off = np.array([0, 1, 2, 3, 4, 5], np.int32)
    Q = np.eye(13); R = np.eye(4)
    res = gpu_riccati(torch, A, B, Q, R, Q, off)
    K, kff, P = riccati_batched(off, A.astype(np.float64), B.astype(np.float64), Q, R, Q)
    assert rel_max(res["K"], K) < 1e-12


def test_lq_rollout_matches_oracle_and_kkt(torch):
    """rtn_lq_rollout on ragged instances vs the oracle's forward pass (same fp64 K, kff
    from the GPU Riccati), and the rolled-out trajectory vs the dense KKT minimiser."""
    import paper_2203_07747_amd as rtn
    hz = sample_horizons(29, 1, 9, seed=6)
    off = offsets_from_horizons(hz)
    n, ni = int(off[-1]), len(hz)
    A, B, rng = random_lq(n, 3)
    c = rng.normal(size=(n, 13)) * 0.1
    q = rng.normal(size=(n, 13)); r = rng.normal(size=(n, 4))
    dx0 = rng.normal(size=(ni, 13))
    Q = np.eye(13); R = 0.1 * np.eye(4); QN = np.eye(13)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    print(f"[gpu] lq_rollout n={n} n_inst={ni}", flush=True)
    At, Bt, ct = dev(A), dev(B), dev(c)
    ric = rtn.riccati(At, Bt, Q, R, QN, offsets=off, c=ct, q=dev(q), r=dev(r))
    out = rtn.lq_rollout(At, Bt, ric["K"], ric["kff"], dev(dx0), offsets=off, c=ct)
    torch.cuda.synchronize()
    K, kff = ric["K"].cpu().numpy(), ric["kff"].cpu().numpy()
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    du, dx, dxN = lq_rollout_batched(off, A64, B64, K, kff, dx0, c)
    assert rel_max(out["du"].cpu().numpy(), du) < 1e-12
    assert rel_max(out["dx"].cpu().numpy(), dx) < 1e-12
    assert rel_max(out["dxN"].cpu().numpy(), dxN) < 1e-12
    for i in (0, ni // 2, ni - 1):
        a, b = int(off[i]), int(off[i + 1])
        du_ref, dx_ref = kkt_bruteforce(A64[a:b], B64[a:b], Q, R, QN, dx0[i], c[a:b], q[a:b], r[a:b])
        np.testing.assert_allclose(out["du"].cpu().numpy()[a:b], du_ref, atol=1e-9)
        np.testing.assert_allclose(out["dxN"].cpu().numpy()[i], dx_ref[-1], atol=1e-9)


def test_box_constrained_lq_matches_exact_minimiser(torch):
    """rtn_riccati_box (ADMM, converged to 1e-11) on ragged instances against the oracle's
    exact box-QP minimiser; the inputs stay inside the box and the states are their rollout."""
    import paper_2203_07747_amd as rtn
    hz = sample_horizons(23, 1, 14, seed=8)
    off = offsets_from_horizons(hz)
    n, ni = int(off[-1]), len(hz)
    A, B, rng = random_lq(n, 5)
    c = rng.normal(size=(n, 13)) * 0.1
    q = rng.normal(size=(n, 13)); r = rng.normal(size=(n, 4)); qN = rng.normal(size=(ni, 13))
    dx0 = 2 * rng.normal(size=(ni, 13))
    lo = -rng.uniform(0.1, 0.4, size=(n, 4)); hi = rng.uniform(0.1, 0.4, size=(n, 4))
    Q = np.eye(13); R = 0.1 * np.eye(4); QN = np.eye(13)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    print(f"[gpu] riccati_box n={n} n_inst={ni}", flush=True)
    out = rtn.riccati_box(dev(A), dev(B), Q, R, QN, dev(dx0), dev(lo), dev(hi), offsets=off, c=dev(c), q=dev(q),
                          r=dev(r), qN=dev(qN), rho=1.0, max_iter=20000, tol=1e-11)
    torch.cuda.synchronize()
    du, dx, dxN = out["du"].cpu().numpy(), out["dx"].cpu().numpy(), out["dxN"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    print(f"  iterations: max {iters.max()} median {np.median(iters)}", flush=True)
    assert np.all(iters < 20000)
    assert np.all(du >= lo - 1e-12) and np.all(du <= hi + 1e-12)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    active = 0
    for i in range(ni):
        a, b = int(off[i]), int(off[i + 1])
        du_ref, dx_ref = box_lq(A64[a:b], B64[a:b], Q, R, QN, dx0[i], lo[a:b], hi[a:b], c[a:b], q[a:b], r[a:b],
                                qN[i])
        np.testing.assert_allclose(du[a:b], du_ref, atol=1e-8)
        np.testing.assert_allclose(dx[a:b], dx_ref[:-1], atol=1e-7)
        np.testing.assert_allclose(dxN[i], dx_ref[-1], atol=1e-7)
        active += int(np.sum(np.isclose(du_ref, lo[a:b]) | np.isclose(du_ref, hi[a:b])))
    assert active > 0


def test_box_lq_single_node_and_long_horizons(torch):
    """The box ADMM steps through an instance one node at a time in one wave, so horizons
    of 1, 2, 37 and 120 nodes in one batch (most inputs on a bound) must all reach the
    exact box-QP minimiser; the random A_k are kept near 0.97 I so the 120-node
    condensed QP stays well conditioned (cond < 1e4)."""
    import paper_2203_07747_amd as rtn
    hz = np.array([1, 2, 37, 120])
    off = offsets_from_horizons(hz)
    n, ni = int(off[-1]), len(hz)
    rng = np.random.default_rng(41)
    A = (0.97 * np.eye(13) + 0.03 * rng.normal(size=(n, 13, 13))).astype(np.float32)
    B = (0.2 * rng.normal(size=(n, 13, 4))).astype(np.float32)
    c = rng.normal(size=(n, 13)) * 0.1
    q = rng.normal(size=(n, 13)); r = rng.normal(size=(n, 4)); qN = rng.normal(size=(ni, 13))
    dx0 = 2 * rng.normal(size=(ni, 13))
    lo = -rng.uniform(0.1, 0.4, size=(n, 4)); hi = rng.uniform(0.1, 0.4, size=(n, 4))
    Q = np.eye(13); R = 0.1 * np.eye(4); QN = np.eye(13)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    print(f"[gpu] riccati_box horizons {hz.tolist()}", flush=True)
    out = rtn.riccati_box(dev(A), dev(B), Q, R, QN, dev(dx0), dev(lo), dev(hi), offsets=off, c=dev(c), q=dev(q),
                          r=dev(r), qN=dev(qN), rho=1.0, max_iter=20000, tol=1e-11)
    torch.cuda.synchronize()
    du, dx, dxN = out["du"].cpu().numpy(), out["dx"].cpu().numpy(), out["dxN"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    print(f"  iterations {iters.tolist()}", flush=True)
    assert np.all(iters < 20000)
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    for i in range(ni):
        a, b = int(off[i]), int(off[i + 1])
        du_ref, dx_ref = box_lq(A64[a:b], B64[a:b], Q, R, QN, dx0[i], lo[a:b], hi[a:b], c[a:b], q[a:b], r[a:b],
                                qN[i])
        np.testing.assert_allclose(du[a:b], du_ref, atol=1e-8)
        np.testing.assert_allclose(dx[a:b], dx_ref[:-1], atol=1e-7)
        np.testing.assert_allclose(dxN[i], dx_ref[-1], atol=1e-7)


def test_box_lq_with_inactive_box_equals_unconstrained_step(torch):
    import paper_2203_07747_amd as rtn
    hz = sample_horizons(9, 1, 10, seed=9)
    off = offsets_from_horizons(hz)
    n, ni = int(off[-1]), len(hz)
    A, B, rng = random_lq(n, 6)
    c = rng.normal(size=(n, 13)) * 0.1
    dx0 = rng.normal(size=(ni, 13))
    Q = np.eye(13); R = 0.1 * np.eye(4); QN = np.eye(13)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    big = np.full((n, 4), 1e6)
    At, Bt, ct = dev(A), dev(B), dev(c)
    box = rtn.riccati_box(At, Bt, Q, R, QN, dev(dx0), dev(-big), dev(big), offsets=off, c=ct, rho=1.0,
                          max_iter=5000, tol=1e-12)
    ric = rtn.riccati(At, Bt, Q, R, QN, offsets=off, c=ct)
    roll = rtn.lq_rollout(At, Bt, ric["K"], ric["kff"], dev(dx0), offsets=off, c=ct)
    torch.cuda.synchronize()
    np.testing.assert_allclose(box["du"].cpu().numpy(), roll["du"].cpu().numpy(), atol=1e-9)
    np.testing.assert_allclose(box["dxN"].cpu().numpy(), roll["dxN"].cpu().numpy(), atol=1e-8)


def test_prepared_call_matches_and_sees_new_data(torch):
    """RiccatiCall marshals once; later calls use the current contents of A, B."""
    import paper_2203_07747_amd as rtn
    off = offsets_from_horizons(sample_horizons(7, 3, 20, seed=11))
    n = int(off[-1])
    Q, R = np.eye(13), 0.1 * np.eye(4)
    A0, B0, _ = random_lq(n, 12)
    At, Bt = torch.from_numpy(A0).cuda(), torch.from_numpy(B0).cuda()
    call = rtn.RiccatiCall(At, Bt, Q, R, Q, offsets=off, want_P=True)
    for seed in (13, 14):
        A, B, _ = random_lq(n, seed)
        At.copy_(torch.from_numpy(A))
        Bt.copy_(torch.from_numpy(B))
        print(f"[gpu] prepared riccati call, seed {seed}", flush=True)
        got = {k: v.cpu().numpy() for k, v in call().items()}
        K, kff, P = riccati_batched(off, A.astype(np.float64), B.astype(np.float64), Q, R, Q)
        assert rel_max(got["K"], K) < 1e-9 and rel_max(got["P"], P) < 1e-9


@pytest.mark.parametrize("max_iter", [400, 4])
def test_box_lq_flags_every_unconverged_instance(torch, max_iter):
    """The box-constrained LQ of 4096 ragged instances (the benchmark's tolerance 1e-6,
    rho 1, hover inputs in the box 0 <= u <= 4): every instance either converged --
    fewer than max_iter iterations and both residuals of its last iteration below tol --
    or reports max_iter iterations with the residual it stopped at.  With 4 iterations
    most instances must be flagged, and the reported residual must be the one of the
    returned inputs (the primal residual bounds how far du is from the box-feasible z)."""
    import paper_2203_07747_amd as rtn
    hz = sample_horizons(4096, 10, 50, seed=31)
    off = offsets_from_horizons(hz)
    n = int(off[-1])
    from workload import sample_nodes
    x, u = sample_nodes(n, seed=32)
    print(f"[gpu] riccati_box flags n={n} max_iter={max_iter}", flush=True)
    lin = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), None, "fp32", 0.05, offsets=off)
    g = torch.Generator(device="cuda").manual_seed(1)
    dx0 = torch.randn((len(hz), 13), device="cuda", dtype=torch.float64, generator=g) * 0.5
    uk = torch.full((n, 4), 9.81 / 4, device="cuda", dtype=torch.float64)
    out = rtn.riccati_box(lin["A"], lin["B"], np.eye(13), 0.1 * np.eye(4), np.eye(13), dx0, (-uk).contiguous(),
                          (4.0 - uk).contiguous(), offsets=off, rho=1.0, max_iter=max_iter, tol=1e-6)
    torch.cuda.synchronize()
    it = out["iters"].cpu().numpy()
    rs = out["resid"].cpu().numpy()
    du = out["du"].cpu().numpy()
    assert np.all(np.isfinite(rs)) and np.all(rs >= 0) and np.all(np.isfinite(du))
    conv = it < max_iter
    assert np.all(rs[conv].max(axis=1) < 1e-6)
    flagged = ~conv
    print(f"  iterations max {it.max()} median {np.median(it)}; flagged {int(flagged.sum())} of {len(hz)}; "
          f"largest residual {rs.max():.2e}", flush=True)
    assert np.all(it[flagged] == max_iter)
    assert np.all((du >= -9.81 / 4 - 1e-12) & (du <= 4.0 - 9.81 / 4 + 1e-12))
    if max_iter == 4:
        assert flagged.sum() > len(hz) // 2 and rs[flagged].max() >= 1e-6

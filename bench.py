#!/usr/bin/env python3
"""Throughput of the Real-time Neural MPC linearisation path on one MI355X.

A step is one rtn_linearize call over the whole batch of one workload: pack ->
network forward -> reverse-mode Jacobian -> RK4 with sensitivities -> stores of
x_{k+1}, A_k, B_k (and f_D, J_D) for every node of every instance.  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

Default workload: 4096 MPC instances with horizons N_i ~ U{10..50}, residual
network 14-5x512-6 in bf16 (fp32 accumulation), dt = 0.05 s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from workload import CONFIGS, SEED_CALIB, config_workload, sample_nodes  # noqa: E402

METRIC = "node linearisations/sec (f, A_k, B_k) BF16/FP8 vs FP32 at stated err vs FP64"
# MI355X published dense peaks (TFLOP/s) and HBM bandwidth (GB/s)
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2516.6, "fp8": 5033.2}
PEAK_HBM_GBS = 8000.0


def flops_per_node(L: int, H: int, d_in: int = 14, d_out: int = 6):
    """Algorithmic flops: one forward pass and one reverse-mode Jacobian per node."""
    W = d_in * H + (L - 1) * H * H + H * d_out
    fwd = 2 * W
    rev = 2 * d_out * ((L - 1) * H * H + H * d_in)
    return fwd, rev


def measured_traffic(config_key: str, kernel_prefix: str, nodes: int):
    """HBM bytes of one call's launches of a kernel (every instance whose name starts with
    kernel_prefix: the reverse chain's tail runs as a second launch) over `nodes` nodes,
    scaled from the committed counter summary (profiles/linearize_<config>_*_hbm_traffic.json,
    bytes per node), only while every kernel source the counters were taken on is unchanged;
    else None."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", f"linearize_{config_key}_*_hbm_traffic.json")):
        rec = json.load(open(path))
        for src, digest in rec["sources"].items():
            f = os.path.join(ROOT, src)
            if not os.path.exists(f) or hashlib.sha256(open(f, "rb").read()).hexdigest() != digest:
                return None
        hits = [v for k, v in rec["per_launch"].items() if k.split("::")[-1].startswith(kernel_prefix)]
        if hits:
            return sum(v["read_bytes"] + v["write_bytes"] for v in hits) / rec["nodes_per_launch"] * nodes
    return None


def copy_probe():
    """A plain 64 MiB device-to-device copy, three times: the reference kernel whose
    FETCH_SIZE / WRITE_SIZE counter readings calibrate the HBM traffic figures."""
    import torch
    a = torch.empty(64 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 64 MiB x3", flush=True)


def tile_choice(rtn, prec, H, L, n):
    """The autotuner's kept path and shapes for this workload and the times it measured."""
    got = rtn.tune_get(prec, H, L, n)
    if got is None:
        return None
    ch, ms = got
    if ch[0] == 1:
        return {"path": "per-layer small-batch", "forward_tuning_ms": ms[0], "reverse_tuning_ms": ms[1]}
    return {"path": "layer chain",
            "forward": {"variant": ch[1], "workgroups": ch[2], "tuning_ms": ms[0]},
            "reverse": {"variant": ch[3], "workgroups": ch[4], "tuning_ms": ms[1]}}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--config", default="c3", choices=sorted(CONFIGS))
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-compare", action="store_true", help="skip the other-precision comparison runs")
    p.add_argument("--no-fp8-workload", action="store_true",
                   help="skip the fp8 configuration (65,536 instances x 20 nodes, 14-4x1024-6)")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--no-extras", action="store_true",
                   help="skip the latency, Riccati and training side measurements")
    p.add_argument("--copy-probe", action="store_true",
                   help="only run a 64 MiB device copy (counter calibration for the traffic figures)")
    p.add_argument("--di", metavar="LxH", default=None,
                   help="only time the double-integrator real-time iteration of one network (e.g. 2x8192)")
    return p.parse_args()


def time_steps(torch, fn, steps, warmup, stream, warm_s: float = 0.0):
    """Mean ms per call over `steps` back-to-back calls (HIP events on `stream`) and the
    host wall time per call, after `warmup` calls and at least `warm_s` seconds of them
    (short calls after a pause otherwise run before the clocks have come up)."""
    for _ in range(warmup):
        fn()
    t_end = time.perf_counter() + warm_s
    while time.perf_counter() < t_end:
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / steps, wall / steps * 1e3


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_rows(a, b):
    """Per-node |a - b|_F / |b|_F."""
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-30)


def stats(e):
    return {"max": float(e.max()), "p999": float(np.quantile(e, 0.999)), "median": float(np.median(e))}


def errors_vs_oracle(gpu, gpu_nom, ref, ref_nom):
    """Error of a GPU linearisation against the FP64 oracle on the same nodes: per-node
    relative Frobenius error of x_{k+1}, A_k, B_k, J_D; of the network's share of the
    continuity parameters (A - A_nominal, B - B_nominal, each side with its own nominal
    step), which A and B hide behind their identity and nominal parts; and of f_D-bar
    over the root-mean-square node norm of the oracle's f_D-bar."""
    errs = {}
    for name, r in zip(("x_next", "A", "B", "J_D"), (ref[0], ref[1], ref[2], ref[4])):
        errs[name] = stats(rel_rows(gpu[name], r))
    f = np.asarray(gpu["f_D"], np.float64)
    scale = np.sqrt(np.mean(np.sum(ref[3] ** 2, axis=1)))
    errs["f_D_over_rms"] = stats(np.linalg.norm(f - ref[3], axis=1) / scale)
    for name, i in (("A_minus_A_nominal", 1), ("B_minus_B_nominal", 2)):
        key = "A" if i == 1 else "B"
        errs[name] = stats(rel_rows(np.asarray(gpu[key], np.float64) - gpu_nom[key], ref[i] - ref_nom[i]))
    return errs


def nominal_gpu(torch, rtn, x, u, dt):
    out = rtn.linearize(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), None, "fp32", dt)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def sample_outputs(torch, rtn, cfg, x, u, gpu_out, n_sample, seed):
    """A seeded sample of the workload's nodes (first and last included): their inputs,
    the GPU outputs and the GPU's nominal step of the same nodes."""
    n = x.shape[0]
    idx = np.unique(np.concatenate([np.random.default_rng(seed).choice(n, min(n, n_sample), replace=False),
                                    [0, n - 1]]))
    return {"cfg": cfg, "x": x[idx], "u": u[idx], "gpu": {k: v[idx] for k, v in gpu_out.items()},
            "nom": nominal_gpu(torch, rtn, x[idx], u[idx], cfg.dt)}


def sampled_errors(sample, Ws, bs):
    """(CPU-baseline leg) errors_vs_oracle of a sample taken by sample_outputs."""
    from oracle.mlp import MLP
    from oracle.rk4 import linearize_affine
    x, u, dt = sample["x"], sample["u"], sample["cfg"].dt
    ref = linearize_affine(x, u, MLP(Ws, bs), dt)
    ref_nom = linearize_affine(x, u, None, dt)
    errs = errors_vs_oracle(sample["gpu"], sample["nom"], ref, ref_nom)
    errs["sample_nodes"] = int(x.shape[0])
    return errs


def cpu_baseline(torch, rtn, cfg, off, x, u, Ws, bs, gpu_out, gpu_K, seconds):
    """The FP64 oracle, as it stands, on a bounded prefix of the same nodes (all host
    threads, then one thread); also the error of the GPU outputs on that prefix against
    it, and of the GPU's fp64 Riccati gains (on the GPU's A_k, B_k, and end to end)."""
    import threadpoolctl
    from oracle.mlp import MLP
    from oracle.rk4 import linearize_affine
    from oracle.riccati import riccati_batched
    net = MLP(Ws, bs)
    n_sample = min(8192, x.shape[0])
    done, t0 = 0, time.perf_counter()
    ref = None
    while True:
        r = linearize_affine(x[:n_sample], u[:n_sample], net, cfg.dt)
        ref = r if ref is None else ref
        done += n_sample
        if time.perf_counter() - t0 >= seconds:
            break
    elapsed = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    n1 = min(1024, n_sample)
    with threadpoolctl.threadpool_limits(1):
        done1, t1 = 0, time.perf_counter()
        while time.perf_counter() - t1 < seconds / 4:
            linearize_affine(x[:n1], u[:n1], net, cfg.dt)
            done1 += n1
        rate1 = done1 / (time.perf_counter() - t1)
    ref_nom = linearize_affine(x[:n_sample], u[:n_sample], None, cfg.dt)
    errs = errors_vs_oracle({k: v[:n_sample] for k, v in gpu_out.items()},
                            nominal_gpu(torch, rtn, x[:n_sample], u[:n_sample], cfg.dt), ref, ref_nom)
    errs["sample_nodes"] = n_sample
    # Riccati gains (Q = I, R = 0.1 I, Q_N = Q) of the instances inside the prefix
    n_inst = int(np.searchsorted(off, n_sample, side="right")) - 1
    o = off[:n_inst + 1]
    Q, R = np.eye(13), 0.1 * np.eye(4)
    m = int(o[-1])
    K_same, _, _ = riccati_batched(o, gpu_out["A"][:m].astype(np.float64), gpu_out["B"][:m].astype(np.float64),
                                   Q, R, Q)
    K_ref, _, _ = riccati_batched(o, ref[1][:m], ref[2][:m], Q, R, Q)
    for name, Kr in (("K_same_AB", K_same), ("K_end_to_end", K_ref)):
        e = rel_rows(gpu_K[:m], Kr)
        errs[name] = {**stats(e), "instances": n_inst}
    cpu = {"value": done / elapsed, "unit": "nodes/s", "cores": int(threads), "kind": "oracle",
           "sample": f"first {n_sample} nodes of the workload, fp64 NumPy oracle, repeated for "
                     f"{elapsed:.1f} s ({done} node linearisations)",
           "single_thread_value": rate1, "single_thread_sample": f"first {n1} nodes",
           "cpu_model": cpu_model()}
    return cpu, errs


def extras(torch, rtn, lin_out, off, stream):
    """Side measurements: single-instance latency (the paper's real-time regime), the fp64
    Riccati solve of this workload's A_k, B_k, and one training step of the residual."""
    from workload import TRAIN, xavier_params as xp
    res = {}
    # floor: replay of a captured graph holding one trivial kernel
    cap = torch.cuda.Stream()
    t1 = torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    gph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gph, stream=cap):
        t1.add_(1.0)
    torch.cuda.synchronize()
    ms, _ = time_steps(torch, gph.replay, 200, 20, stream, warm_s=0.05)
    res["graph_launch_floor_us"] = ms * 1e3
    for key in ("c1", "c2"):
        cfg, o, x, u, Ws, bs = config_workload(key)
        m = rtn.Model(Ws, bs)
        xt, ut = torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda()
        out = {}
        f = lambda: rtn.linearize(xt, ut, m, "fp32", cfg.dt, offsets=o, out=out, stream=stream)
        ms_py, _ = time_steps(torch, f, 200, 20, stream, warm_s=0.05)
        call = rtn.LinearizeCall(xt, ut, m, "fp32", cfg.dt, offsets=o, stream=stream)
        ms, wall = time_steps(torch, call, 200, 20, stream, warm_s=0.05)
        # one call at a time, each waited for (a real-time loop): host wall time per call
        iso = []
        for _ in range(220):
            t0 = time.perf_counter()
            call()
            stream.synchronize()
            iso.append(time.perf_counter() - t0)
        iso_us = float(np.median(iso[20:])) * 1e6
        # one control iteration: the linearisation and the fp64 Riccati solve of its A_k, B_k
        lo = call()
        ric = rtn.RiccatiCall(lo["A"], lo["B"], np.eye(13), 0.1 * np.eye(4), np.eye(13), offsets=o, stream=stream)

        def iteration():
            call()
            ric()
        ms_it, _ = time_steps(torch, iteration, 200, 20, stream, warm_s=0.05)
        rtn.profile_enable(True)
        for _ in range(20):
            f()
        torch.cuda.synchronize()
        kern = rtn.profile_collect()
        rtn.profile_enable(False)
        res[f"latency_{key}"] = {"workload": cfg.name, "us_per_call": ms * 1e3, "host_us_per_call": wall * 1e3,
                                 "us_per_call_isolated_median": iso_us,
                                 "us_per_call_unprepared_python_call": ms_py * 1e3,
                                 "us_per_iteration_with_riccati_fp64": ms_it * 1e3,  # both calls prepared
                                 "tile_choice": tile_choice(rtn, "fp32", cfg.width, cfg.n_hidden, x.shape[0]),
                                 "kernel_us_unbatched": {k: v["avg_ms"] * 1e3 for k, v in kern.items()}}
        m.close()
    # second-order local approximation (fp32): one instance (c2) and a 4096-node batch of the c2 network
    cfg, o, x, u, Ws, bs = config_workload("c2")
    m = rtn.Model(Ws, bs)
    for label, reps in (("c2", 1), ("c2_x205", 205)):
        xt = torch.from_numpy(np.tile(x, (reps, 1))).cuda()
        ut = torch.from_numpy(np.tile(u, (reps, 1))).cuda()
        sout = {}
        f = lambda: rtn.linearize_second(xt, ut, m, cfg.dt, out=sout, stream=stream)
        ms, _ = time_steps(torch, f, 20, 3, stream)
        res[f"second_order_{label}"] = {"nodes": int(xt.shape[0]), "ms_per_call": ms,
                                        "nodes_per_s": xt.shape[0] / (ms * 1e-3)}
    m.close()
    Q = np.eye(13); R = 0.1 * np.eye(4)
    rout = {}
    f = lambda: rtn.riccati(lin_out["A"], lin_out["B"], Q, R, Q, offsets=off, out=rout, stream=stream)
    ms, _ = time_steps(torch, f, 10, 2, stream)
    res["riccati_fp64"] = {"ms_per_call": ms, "instances": int(len(off) - 1),
                           "nodes_per_s": float(off[-1]) / (ms * 1e-3)}
    # the same LQ with the input box 0 <= u_k + du_k <= 4 around hover inputs (ADMM, rho 1, tol 1e-6)
    n_all = int(off[-1])
    g = torch.Generator(device="cuda").manual_seed(1)
    dx0 = torch.randn((len(off) - 1, 13), device="cuda", dtype=torch.float64, generator=g) * 0.5
    uk = torch.full((n_all, 4), 9.81 / 4, device="cuda", dtype=torch.float64)
    lo, hi = (-uk).contiguous(), (4.0 - uk).contiguous()
    bout = {}
    max_iter, tol = 400, 1e-6
    f = lambda: rtn.riccati_box(lin_out["A"], lin_out["B"], Q, R, Q, dx0, lo, hi, offsets=off, rho=1.0,
                                max_iter=max_iter, tol=tol, out=bout, stream=stream)
    ms, _ = time_steps(torch, f, 5, 1, stream)
    it = bout["iters"].cpu().numpy()
    rs = bout["resid"].cpu().numpy()
    unconv = (it >= max_iter) & (rs.max(axis=1) >= tol)
    res["riccati_box_fp64"] = {"ms_per_call": ms, "instances": int(len(off) - 1), "tol": tol, "max_iter": max_iter,
                               "iterations_max": int(it.max()), "iterations_median": float(np.median(it)),
                               "unconverged_instances": int(unconv.sum()),
                               "residual_max_primal": float(rs[:, 0].max()), "residual_max_dual": float(rs[:, 1].max())}
    Ws, bs = xp(TRAIN["n_hidden"], TRAIN["width"], seed=0)
    m = rtn.Model(Ws, bs)
    B = TRAIN["batch"]
    g = torch.Generator(device="cuda").manual_seed(0)
    z = torch.randn((B, 14), device="cuda", generator=g)
    t = torch.randn((B, 6), device="cuda", generator=g)
    loss = torch.empty((1,), device="cuda")
    f = lambda: m.train_step(z, t, lr=TRAIN["lr"], prec="bf16", loss=loss, stream=stream)
    ms, _ = time_steps(torch, f, 20, 3, stream)
    W = sum(w.size for w in Ws)
    res["train_step_bf16"] = {"ms_per_step": ms, "batch": B, "tflops": 6 * W * B / (ms * 1e-3) / 1e12}
    m.close()
    return res


# The paper's control frequencies of its own implementation on an RTX 3000 laptop GPU
# (Sec. V): the two-layer width sweep (read from the plotted data) and Table II.
PAPER_RTX3000_HZ_TWO_LAYER = {2: 783.8, 4: 763.0, 8: 767.3, 16: 776.7, 32: 773.8, 64: 763.7, 128: 756.3,
                              256: 770.5, 512: 758.6, 1024: 737.8, 2048: 704.6, 4096: 500.9, 8192: 169.7}
PAPER_RTX3000_HZ_TABLE_II = {(2, 16): 781, (2, 128): 770, (5, 16): 586, (5, 128): 598, (12, 32): 363,
                             (12, 512): 363, (20, 512): 232, (50, 512): 117}


def di_runtime(torch, rtn, stream, only=None):
    """The runtime workload of Sec. V: one real-time iteration (network value and
    Jacobian, RK4 linearisation, Riccati recursion, rollout) of the double integrator
    with N = 10 nodes per call, for the two-layer width sweep and the networks of
    Table II.  The output layer is zero, as in the paper's runs; all work is done."""
    from workload import xavier_params as xp
    N, dt = 10, 0.05
    Q, R, QN = np.eye(2), np.array([0.1]), np.eye(2)
    g = np.random.default_rng(0)
    x = torch.from_numpy(g.normal(0, 1, (N, 2)).astype(np.float32)).cuda()
    u = torch.from_numpy(g.normal(0, 1, N).astype(np.float32)).cuda()
    xN = torch.from_numpy(g.normal(0, 1, (1, 2)).astype(np.float32)).cuda()
    x0 = torch.from_numpy(g.normal(0, 1, (1, 2)).astype(np.float32)).cuda()

    def tick_time(L, H):
        m = None
        if L:
            Ws, bs = xp(L, H, seed=H, d_in=2, d_out=2)
            Ws[-1][:] = 0.0
            m = rtn.DiModel(Ws, bs)
        call = rtn.DiRtiCall(x, u, xN, x0, m, Q, R, QN, dt, stream=stream)
        # warm up for 50 ms of back-to-back iterations (clocks settle after the model build)
        ms, wall = time_steps(torch, call, 400, 20, stream, warm_s=0.05)
        out = {}
        f = lambda: rtn.di_rti(x, u, xN, x0, m, Q, R, QN, dt, out=out, stream=stream)
        ms_py, _ = time_steps(torch, f, 200, 20, stream, warm_s=0.05)
        if m is not None:
            m.close()
        return {"us_per_iteration": ms * 1e3, "hz": 1e3 / ms, "host_us_per_call": wall * 1e3,
                "us_per_iteration_unprepared_python_call": ms_py * 1e3}

    if only is not None:
        L, H = only
        r = tick_time(L, H)
        r["weight_bytes"] = 4.0 * (3 * H + (L - 1) * (H * H + H) + 2 * H + 2)
        return {"nodes": N, "network": f"{L}x{H}", **r}
    res = {"nodes": N, "loop": "back-to-back rtn_di_rti calls (prepared arguments; one launch for widths "
                               "<= 64, else a captured graph), timed with events on the stream",
           "nominal_only": tick_time(0, 0), "two_layer": {}, "table_ii": {}}
    for H in sorted(PAPER_RTX3000_HZ_TWO_LAYER):
        r = tick_time(2, H)
        r["weight_GBps"] = 4.0 * (3 * H + H * H + H + 2 * H + 2) / (r["us_per_iteration"] * 1e-6) / 1e9
        r["paper_rtx3000_hz"] = PAPER_RTX3000_HZ_TWO_LAYER[H]
        res["two_layer"][H] = r
    for (L, H), hz in PAPER_RTX3000_HZ_TABLE_II.items():
        r = tick_time(L, H)
        r["paper_rtx3000_hz"] = hz
        res["table_ii"][f"{L}x{H}"] = r
    return res


def measure(torch, rtn, model, key, prec, xt, ut, off, cfg, steps, warmup, stream, out):
    """Time `steps` rtn_linearize calls of one workload at one precision (the first call
    tunes the tiles), then collect per-kernel event times over as many calls."""
    n = xt.shape[0]
    L, H = cfg.n_hidden, cfg.width

    def step():
        rtn.linearize(xt, ut, model, prec, cfg.dt, offsets=off, out=out, stream=stream)

    ms, wall_ms = time_steps(torch, step, steps, warmup, stream)
    rtn.profile_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    kern = rtn.profile_collect()
    rtn.profile_enable(False)
    f_fwd, f_rev = flops_per_node(L, H)
    nan = {"avg_ms": float("nan"), "total_ms": float("nan"), "calls": 0}
    krev = kern.get("mlp_reverse_chain", nan)
    launches = max(1, round(krev["calls"] / steps))
    # algorithmic flops of all reverse launches over their summed event durations
    achieved = n * f_rev * steps / (krev["total_ms"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    return {
        "value": n / (ms * 1e-3), "ms_per_step": ms, "steps": steps, "host_wall_ms_per_step": wall_ms,
        "roofline": {"bound": "mfma", "kernel": "mlp_reverse_chain", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(key, "mlp_reverse_chain", n // launches),
                     "algorithmic_flops_per_launch": n * f_rev / launches, "avg_launch_ms": krev["avg_ms"],
                     "launches_per_step": launches},
        "kernels_ms": {k: v["avg_ms"] for k, v in kern.items()},
        "tile_choice": tile_choice(rtn, prec, H, L, n // launches),
        "whole_step_mfma_frac": n * (f_fwd + f_rev) / (ms * 1e-3) / 1e12 / peak,
    }


def workload(torch, rtn, key, steps, warmup, stream, compare, fixed_fp32=False):
    """One configuration at its own precision and (compare) at the other two; returns the
    measurement record and what the side measurements need."""
    cfg, off, x, u, Ws, bs = config_workload(key)
    n = x.shape[0]
    model = rtn.Model(Ws, bs)
    xt, ut = torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda()
    calibrated = False

    def ensure_calibrated():
        nonlocal calibrated
        if not calibrated:
            xc, uc = sample_nodes(65536, seed=SEED_CALIB)
            model.calibrate(torch.from_numpy(xc).cuda(), torch.from_numpy(uc).cuda())
            calibrated = True

    prec = cfg.precision
    if prec == "fp8":
        ensure_calibrated()
    out = {}
    rec = measure(torch, rtn, model, key, prec, xt, ut, off, cfg, steps, warmup, stream, out)
    rec["config"] = {"workload": cfg.name, "n_inst": int(len(off) - 1), "n_nodes": int(n),
                     "hidden_layers": cfg.n_hidden, "width": cfg.width, "dt": cfg.dt}
    rec["dtype"] = prec
    gpu_out = {k: v.cpu().numpy() for k, v in out.items()}
    if compare:
        cmp = {}
        for p in ("fp32", "bf16", "fp8"):
            if p == prec:
                continue
            if p == "fp8":
                ensure_calibrated()
            if p == "fp32" and fixed_fp32:  # default shapes, no tuning sweep at this size
                rtn.tune_set("fp32", cfg.width, cfg.n_hidden, n, (0, 0, 0, 0, 0))
            cmp[p] = measure(torch, rtn, model, key, p, xt, ut, off, cfg, max(3, steps // 5), 2, stream, {})
            if fixed_fp32 and p == "fp32":
                cmp[p]["tile_choice"]["note"] = "default shapes, not tuned"
        rec["other_precisions_same_workload"] = cmp
    return rec, (cfg, off, x, u, Ws, bs, model, out, gpu_out)


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.di:
        import torch
        import paper_2203_07747_amd as rtn
        L, H = (int(v) for v in args.di.lower().split("x"))
        print(json.dumps(di_runtime(torch, rtn, torch.cuda.current_stream(), only=(L, H))), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(nodes are independent, so G GPUs would each take a contiguous range of instances)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2203_07747_amd as rtn

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    rec, (cfg, off, x, u, Ws, bs, model, out, gpu_out) = workload(torch, rtn, args.config, args.steps, args.warmup,
                                                                   stream, not args.no_compare)
    print(f"{args.config}: {rec['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    result = {
        "metric": METRIC, "value": rec["value"], "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": rec["dtype"], "data": "synthetic", "config": rec["config"],
        "roofline": rec["roofline"],
    }
    for k in ("kernels_ms", "tile_choice", "whole_step_mfma_frac", "host_wall_ms_per_step",
              "other_precisions_same_workload"):
        if k in rec:
            result[k] = rec[k]
    sample3 = sample_outputs(torch, rtn, cfg, x, u, gpu_out, 1500, 11) if not args.no_cpu else None
    sample8 = None
    if args.config != "c4" and not args.no_fp8_workload:
        # the fp8 configuration of the metric: 65,536 instances x 20 nodes, 14-4x1024-6 e4m3
        r8, (cfg8, _, x8, u8, Ws8, bs8, m8, out8, gpu8) = workload(
            torch, rtn, "c4", max(5, args.steps // 4), 3, stream, not args.no_compare, fixed_fp32=True)
        print(f"c4: {r8['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        if not args.no_cpu:
            sample8 = sample_outputs(torch, rtn, cfg8, x8, u8, gpu8, 256, 12)
        result["fp8_workload"] = r8
        m8.close()
        del out8, gpu8
        torch.cuda.empty_cache()
    if not args.no_extras:
        result["extras"] = extras(torch, rtn, out, off, stream)
        result["extras"]["double_integrator_rti"] = di_runtime(torch, rtn, stream)
    if not args.no_cpu:  # the CPU-baseline leg: the FP64 oracle timed, and the GPU's errors against it
        ric = rtn.riccati(out["A"], out["B"], np.eye(13), 0.1 * np.eye(4), np.eye(13), offsets=off, stream=stream)
        torch.cuda.synchronize()
        cpu, errs = cpu_baseline(torch, rtn, cfg, off, x, u, Ws, bs, gpu_out, ric["K"].cpu().numpy(),
                                 args.cpu_seconds)
        result["cpu_baseline"] = cpu
        result["err_vs_fp64"] = errs
        result["err_vs_fp64_sampled"] = sampled_errors(sample3, Ws, bs)
        if sample8 is not None:
            result["fp8_workload"]["err_vs_fp64_sampled"] = sampled_errors(sample8, Ws8, bs8)
    model.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

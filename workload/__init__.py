"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module only *draws numbers and states shapes*: quadrotor constants, the
five workload configurations, and seeded samplers for states, inputs, horizon
lengths and network weights.  It contains none of the method's arithmetic
(no dynamics, no network evaluation, no integration), so that the CPU oracle
and the GPU path can both take their inputs from here without sharing code.

Distributions (per node, i.i.d., drawn in this order from one
``numpy.random.default_rng(seed)``):

* position  p ~ U[-5, 5]^3
* attitude  q = n / |n| with n ~ N(0, I_4)  (Haar-uniform unit quaternion, w,x,y,z)
* velocity  v ~ N(0, 3^2 I_3)
* body rate w ~ N(0, I_3)
* input     u ~ U[0, 4]^4 rotor thrusts in newton

State layout is the paper's 13-vector x = [p(3), q(4) wxyz, v(3), w(3)]
(Sec. VI, nominal quadrotor model, eq. (6)); inputs are the four rotor
thrusts T_0..T_3.  Arrays are float32 (the precision the GPU path consumes);
the oracle promotes these exact values to float64.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

NX = 13  # state dimension, eq. (6)
NU = 4   # rotor thrusts, eq. (6)
D_IN = 14  # residual network input [v(3), w(3), q(4), u(4)]
D_OUT = 6  # residual network output: linear (3) and angular (3) accelerations, eq. (7)

# Seeds, one independent generator per purpose.
SEED_WEIGHTS = 0
SEED_NODES = 1
SEED_HORIZONS = 2
SEED_CALIB = 3
SEED_TRAIN = 4
SEED_ROLLOUT = 5


@dataclasses.dataclass(frozen=True)
class QuadParams:
    """Rigid-body constants of the quadrotor (eq. (6)); g is the magnitude of
    gravity, which acts along -z of the world frame."""
    mass: float = 1.0
    Jx: float = 0.003
    Jy: float = 0.003
    Jz: float = 0.005
    arm: float = 0.17      # centre-to-rotor distance of the X frame
    c_tau: float = 0.013   # rotor reaction-torque coefficient (N m per N)
    g: float = 9.81
    u_max: float = 4.0

    def as_tuple(self) -> Tuple[float, ...]:
        return (self.mass, self.Jx, self.Jy, self.Jz, self.arm, self.c_tau, self.g)


QUAD = QuadParams()


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n_inst: int
    horizon: Tuple[int, int]  # inclusive range of per-instance horizon lengths
    n_hidden: int
    width: int
    precision: str            # "fp32" | "bf16" | "fp8"
    dt: float = 0.05


CONFIGS = {
    "c1": Config("c1: 1 instance, N=10, MLP 14-2x64-6, fp32", 1, (10, 10), 2, 64, "fp32"),
    "c2": Config("c2: 1 instance, N=20, MLP 14-4x512-6, fp32", 1, (20, 20), 4, 512, "fp32"),
    "c3": Config("c3: 4096 instances, N~U{10..50}, MLP 14-5x512-6, bf16", 4096, (10, 50), 5, 512, "bf16"),
    "c4": Config("c4: 65536 instances, N=20, MLP 14-4x1024-6, fp8 e4m3", 65536, (20, 20), 4, 1024, "fp8"),
}

# Training workload: residual 14-4x512-6, Adam lr 1e-3, batch 4096, 2M transitions
# from the drag-augmented simulator.
TRAIN = dict(n_hidden=4, width=512, batch=4096, lr=1e-3, n_transitions=2_000_000,
             drag=(0.3, 0.3, 0.5), rotor_drag=0.02, noise_std=0.05, dt=0.05)


def layer_dims(n_hidden: int, width: int, d_in: int = D_IN, d_out: int = D_OUT) -> List[Tuple[int, int]]:
    """(fan_out, fan_in) of every affine layer, input layer first."""
    dims = [(width, d_in)] + [(width, width)] * (n_hidden - 1) + [(d_out, width)]
    return dims


def xavier_params(n_hidden: int, width: int, seed: int = SEED_WEIGHTS,
                  d_in: int = D_IN, d_out: int = D_OUT) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """Glorot/Xavier-uniform weights W_l[out][in] (bound sqrt(6/(fan_in+fan_out))),
    drawn in layer order from one generator; zero biases.  float32."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for fo, fi in layer_dims(n_hidden, width, d_in, d_out):
        a = np.sqrt(6.0 / (fi + fo))
        Ws.append(rng.uniform(-a, a, size=(fo, fi)).astype(np.float32))
        bs.append(np.zeros(fo, dtype=np.float32))
    return Ws, bs


def sample_nodes(n: int, seed: int = SEED_NODES) -> Tuple[np.ndarray, np.ndarray]:
    """n i.i.d. (state, input) pairs, float32, shapes (n,13) and (n,4)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(-5.0, 5.0, size=(n, 3))
    qn = rng.standard_normal(size=(n, 4))
    q = qn / np.linalg.norm(qn, axis=1, keepdims=True)
    v = rng.normal(0.0, 3.0, size=(n, 3))
    w = rng.normal(0.0, 1.0, size=(n, 3))
    u = rng.uniform(0.0, QUAD.u_max, size=(n, 4))
    x = np.concatenate([p, q, v, w], axis=1).astype(np.float32)
    return x, u.astype(np.float32)


def sample_horizons(n_inst: int, lo: int, hi: int, seed: int = SEED_HORIZONS) -> np.ndarray:
    """Per-instance horizon lengths N_i ~ U{lo..hi} (inclusive), int32."""
    if lo == hi:
        return np.full(n_inst, lo, dtype=np.int32)
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=n_inst).astype(np.int32)


def offsets_from_horizons(horizons: Sequence[int]) -> np.ndarray:
    """CSR offsets (n_inst+1,) int32 of node-major instance ranges."""
    off = np.zeros(len(horizons) + 1, dtype=np.int32)
    off[1:] = np.cumsum(np.asarray(horizons, dtype=np.int64))
    return off


def config_workload(key: str):
    """(config, offsets, x, u, weights, biases) for a named configuration."""
    cfg = CONFIGS[key]
    hz = sample_horizons(cfg.n_inst, *cfg.horizon)
    off = offsets_from_horizons(hz)
    x, u = sample_nodes(int(off[-1]))
    Ws, bs = xavier_params(cfg.n_hidden, cfg.width)
    return cfg, off, x, u, Ws, bs


def hover_thrust(quad: QuadParams = QUAD) -> float:
    return quad.mass * quad.g / 4.0

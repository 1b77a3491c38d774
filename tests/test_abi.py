"""The C ABI library loads, exports every declared symbol, and validates arguments
on the host before touching the GPU (these tests run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2203_07747_amd import _lib
from paper_2203_07747_amd._lib import MlpDesc, Quad, load, RTN_OK, RTN_EINVAL, RTN_ENOTSUP
from workload import QUAD

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rtn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rtn_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("librtn.so not built")
    return load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_version(lib):
    assert b"gfx950" in lib.rtn_version()


def desc(L=2, W=64, act=0, d_in=14, d_out=6, inp=0):
    return MlpDesc(d_in, d_out, L, W, act, inp)


def test_param_count(lib):
    n = ctypes.c_int64()
    assert lib.rtn_param_count(ctypes.byref(desc(2, 64)), ctypes.byref(n)) == RTN_OK
    assert n.value == 64 * 14 + 64 + 64 * 64 + 64 + 6 * 64 + 6  # 5510
    assert lib.rtn_param_count(ctypes.byref(desc(4, 512)), ctypes.byref(n)) == RTN_OK
    assert n.value == 798726
    assert lib.rtn_param_count(ctypes.byref(desc(5, 512)), ctypes.byref(n)) == RTN_OK
    assert n.value == 1061382
    # the residual variants of Sec. VI count their own (smaller) first and last layers
    assert lib.rtn_param_count(ctypes.byref(desc(2, 64, d_in=3, d_out=3, inp=1)), ctypes.byref(n)) == RTN_OK
    assert n.value == 64 * 3 + 64 + 64 * 64 + 64 + 3 * 64 + 3
    assert lib.rtn_param_count(ctypes.byref(desc(2, 64, d_in=7, d_out=3, inp=2)), ctypes.byref(n)) == RTN_OK
    assert n.value == 64 * 7 + 64 + 64 * 64 + 64 + 3 * 64 + 3


@pytest.mark.parametrize("d,code", [
    (desc(d_in=13), RTN_EINVAL), (desc(d_out=5), RTN_EINVAL), (desc(L=0), RTN_EINVAL),
    (desc(L=17), RTN_EINVAL), (desc(act=7), RTN_EINVAL), (desc(W=96), RTN_ENOTSUP), (desc(W=0), RTN_EINVAL),
    (desc(inp=3), RTN_EINVAL), (desc(inp=1), RTN_EINVAL), (desc(d_in=3, d_out=6, inp=1), RTN_EINVAL),
    (desc(d_in=7, d_out=3, inp=1), RTN_EINVAL), (desc(d_in=3, d_out=3, inp=2), RTN_EINVAL),
    (desc(d_in=3, d_out=3, inp=0), RTN_EINVAL)])
def test_bad_descriptor(lib, d, code):
    n = ctypes.c_int64()
    assert lib.rtn_param_count(ctypes.byref(d), ctypes.byref(n)) == code
    assert len(lib.rtn_last_error()) > 0


def call_linearize(lib, quad=True, dt=0.05, n_inst=1, offsets=None, n=0, prec=0, ptrs=False):
    q = Quad(QUAD.mass, QUAD.Jx, QUAD.Jy, QUAD.Jz, QUAD.arm, QUAD.c_tau, QUAD.g)
    off = None
    if offsets is not None:
        arr = np.asarray(offsets, dtype=np.int32)
        off = arr.ctypes.data_as(ctypes.c_void_p)
        call_linearize._keep = arr
    p = ctypes.c_void_p(16) if ptrs else None  # never dereferenced: validation fails first
    return lib.rtn_linearize(None, prec, ctypes.byref(q) if quad else None, ctypes.c_float(dt), n_inst, off, n,
                             p, p, p, p, p, None, None, None, None)


def test_linearize_validation(lib):
    assert call_linearize(lib, quad=False) == RTN_EINVAL
    assert call_linearize(lib, dt=0.0) == RTN_EINVAL
    assert call_linearize(lib, dt=float("nan")) == RTN_EINVAL
    assert call_linearize(lib, n=-1) == RTN_EINVAL
    assert call_linearize(lib, n_inst=0) == RTN_EINVAL
    assert call_linearize(lib, n_inst=2, offsets=None, n=4) == RTN_EINVAL        # NULL offsets need n_inst == 1
    assert call_linearize(lib, n_inst=2, offsets=[1, 2, 4], n=4, ptrs=True) == RTN_EINVAL  # offsets[0] != 0
    assert call_linearize(lib, n_inst=2, offsets=[0, 2, 2], n=2, ptrs=True) == RTN_EINVAL  # empty instance
    assert call_linearize(lib, n_inst=2, offsets=[0, 2, 5], n=4, ptrs=True) == RTN_EINVAL  # end != n_nodes
    assert call_linearize(lib, n=5) == RTN_EINVAL                                 # NULL arrays
    assert b"device pointers" in lib.rtn_last_error()
    # an empty batch is valid and does no work
    assert call_linearize(lib, n=0) == RTN_OK
    assert call_linearize(lib, n_inst=1, offsets=[0, 0], n=0) == RTN_EINVAL       # an instance must have a node


def test_model_calls_reject_null(lib):
    assert lib.rtn_model_create(ctypes.byref(desc()), None, ctypes.byref(ctypes.c_void_p())) == RTN_EINVAL
    assert lib.rtn_model_destroy(None) == RTN_OK
    assert lib.rtn_model_set_params(None, None) == RTN_EINVAL
    assert lib.rtn_model_calibrate(None, 4, None, None, None) == RTN_EINVAL


def test_riccati_validation(lib):
    Q = np.eye(13); R = 0.1 * np.eye(4)
    qp = Q.ctypes.data_as(ctypes.c_void_p); rp = R.ctypes.data_as(ctypes.c_void_p)
    z = ctypes.c_void_p(16)
    assert lib.rtn_riccati(1, None, 0, None, None, None, qp, rp, qp, None, None, None, None, None, None, None) == RTN_OK
    assert lib.rtn_riccati(1, None, 3, None, None, None, None, rp, qp, None, None, None, z, z, None, None) == RTN_EINVAL
    assert lib.rtn_riccati(1, None, 3, None, None, None, qp, rp, qp, None, None, None, z, z, None, None) == RTN_EINVAL
    off = np.array([0, 2, 2], dtype=np.int32)
    assert lib.rtn_riccati(2, off.ctypes.data_as(ctypes.c_void_p), 2, z, z, None, qp, rp, qp, None, None, None, z, z,
                           None, None) == RTN_EINVAL
    Rbad = R.copy(); Rbad[0, 0] = np.inf
    assert lib.rtn_riccati(1, None, 3, z, z, None, qp, Rbad.ctypes.data_as(ctypes.c_void_p), qp, None, None, None,
                           z, z, None, None) == RTN_EINVAL


def test_linearize_second_validation(lib):
    q = Quad(QUAD.mass, QUAD.Jx, QUAD.Jy, QUAD.Jz, QUAD.arm, QUAD.c_tau, QUAD.g)
    z = ctypes.c_void_p(16)
    f = lambda model, prec, n: lib.rtn_linearize_second(model, prec, ctypes.byref(q), ctypes.c_float(0.05), 1, None,
                                                        n, z, z, z, z, z, None, None, None, None)
    assert f(None, 0, 4) == RTN_EINVAL                      # model required
    assert f(z, 1, 4) == RTN_ENOTSUP                        # fp32 only
    assert lib.rtn_linearize_second(z, 0, None, ctypes.c_float(0.05), 1, None, 4, z, z, z, z, z, None, None, None,
                                    None) == RTN_EINVAL     # quad


def test_riccati_box_validation(lib):
    Q = np.eye(13); R = 0.1 * np.eye(4)
    qp = Q.ctypes.data_as(ctypes.c_void_p); rp = R.ctypes.data_as(ctypes.c_void_p)
    z = ctypes.c_void_p(16)
    args = lambda n, rho, it, tol, du=z: (1, None, n, z, z, None, qp, rp, qp, None, None, None, z, z, z,
                                         rho, it, tol, du, None, None, None, None, None)
    assert lib.rtn_riccati_box(*args(0, 1.0, 10, 1e-8)) == RTN_OK
    assert lib.rtn_riccati_box(*args(3, 0.0, 10, 1e-8)) == RTN_EINVAL       # rho
    assert lib.rtn_riccati_box(*args(3, float("nan"), 10, 1e-8)) == RTN_EINVAL
    assert lib.rtn_riccati_box(*args(3, 1.0, 0, 1e-8)) == RTN_EINVAL        # max_iter
    assert lib.rtn_riccati_box(*args(3, 1.0, 10, -1.0)) == RTN_EINVAL       # tol
    assert lib.rtn_riccati_box(*args(3, 1.0, 10, 1e-8, None)) == RTN_EINVAL  # du


def test_lq_rollout_validation(lib):
    z = ctypes.c_void_p(16)
    assert lib.rtn_lq_rollout(1, None, 0, None, None, None, None, None, None, None, None, None, None) == RTN_OK
    assert lib.rtn_lq_rollout(1, None, 3, z, z, None, None, z, z, None, z, None, None) == RTN_EINVAL
    assert lib.rtn_lq_rollout(1, None, 3, z, z, None, z, z, z, None, None, None, None) == RTN_EINVAL
    off = np.array([0, 3, 2], dtype=np.int32)
    assert lib.rtn_lq_rollout(2, off.ctypes.data_as(ctypes.c_void_p), 2, z, z, None, z, z, z, None, z, None,
                              None) == RTN_EINVAL


def test_tune_table_host_logic(lib, tmp_path):
    """The autotuner's table: validation of keys and choices, set/get, save/load (no GPU)."""
    ch = (ctypes.c_int32 * 5)
    ms = (ctypes.c_float * 2)()
    out = ch()
    assert lib.rtn_tune_mode(2) == RTN_EINVAL
    assert lib.rtn_tune_get(7, 512, 4, 100, out, None) == RTN_EINVAL          # precision
    assert lib.rtn_tune_get(1, 500, 4, 100, out, None) == RTN_EINVAL          # width without kernels
    assert lib.rtn_tune_get(1, 512, 0, 100, out, None) == RTN_EINVAL          # depth
    assert lib.rtn_tune_get(1, 512, 4, 0, out, None) == RTN_EINVAL           # size
    assert lib.rtn_tune_set(1, 64, 2, 100, ch(0, 1, 0, 0, 0)) == RTN_EINVAL   # no alternative shape at width 64
    assert lib.rtn_tune_set(0, 1024, 2, 100, ch(0, 0, 0, 1, 0)) == RTN_EINVAL  # fp32 width 1024 has none either
    assert lib.rtn_tune_set(1, 512, 4, 100, ch(0, 0, -1, 0, 0)) == RTN_EINVAL  # negative workgroups
    assert lib.rtn_tune_set(1, 512, 4, 100, ch(1, 0, 0, 0, 0)) == RTN_EINVAL   # small-batch path is fp32 only
    assert lib.rtn_tune_set(0, 512, 4, 100, ch(2, 0, 0, 0, 0)) == RTN_EINVAL   # no such path
    assert lib.rtn_tune_set(0, 512, 4, 100, ch(1, 0, 0, 0, 0)) == RTN_OK
    assert lib.rtn_tune_set(1, 512, 4, 100, ch(0, 1, 300, 0, 512)) == RTN_OK
    assert lib.rtn_tune_get(1, 512, 4, 127, out, ms) == RTN_OK                # same size class (64..127)
    assert tuple(out) == (0, 1, 300, 0, 512)
    assert lib.rtn_tune_get(1, 512, 4, 128, out, None) == RTN_EINVAL         # next size class
    path = str(tmp_path / "tune.txt")
    assert lib.rtn_tune_save(path.encode()) == RTN_OK
    text = open(path).read()
    assert "1 512 4 6 0 1 300 0 512" in text and "0 512 4 6 1 0 0 0 0" in text
    assert lib.rtn_tune_set(1, 512, 4, 100, ch(0, 0, 0, 1, 0)) == RTN_OK
    assert lib.rtn_tune_load(path.encode()) == RTN_OK
    assert lib.rtn_tune_get(1, 512, 4, 100, out, None) == RTN_OK and tuple(out) == (0, 1, 300, 0, 512)
    assert lib.rtn_tune_load(str(tmp_path / "missing.txt").encode()) == RTN_EINVAL


def test_training_and_exact_validation(lib):
    z = ctypes.c_void_p(16)
    assert lib.rtn_train_step(None, 1, 8, z, z, 1e-3, 0.9, 0.999, 1e-8, None, None) == RTN_EINVAL
    assert lib.rtn_mlp_forward(None, 1, 8, z, z, None) == RTN_EINVAL
    assert lib.rtn_mlp_backward(None, 8, z, None, None) == RTN_EINVAL
    assert lib.rtn_adam_step(None, 1e-3, 0.9, 0.999, 1e-8, None) == RTN_EINVAL
    q = Quad(QUAD.mass, QUAD.Jx, QUAD.Jy, QUAD.Jz, QUAD.arm, QUAD.c_tau, QUAD.g)
    assert lib.rtn_linearize_exact(None, 0, ctypes.byref(q), ctypes.c_float(0.05), 1, None, 4,
                                   z, z, z, z, z, None) == RTN_EINVAL
    assert b"needs a network" in lib.rtn_last_error()


def test_profile_read_without_records(lib):
    n = ctypes.c_int32(-1)
    assert lib.rtn_profile_enable(0) == RTN_OK
    assert lib.rtn_profile_read(None, 0, ctypes.byref(n)) == RTN_OK
    assert n.value == 0


def test_di_param_count_matches_table_ii(lib):
    """Parameter counts of the double-integrator networks of Table II (2 inputs, 2 outputs)."""
    n = ctypes.c_int64()
    printed = {(2, 16): 354, (2, 128): 17e3, (5, 16): 1.2e3, (5, 128): 67e3, (12, 32): 12e3, (50, 512): 13e6}
    for (L, H), want in printed.items():
        assert lib.rtn_di_param_count(L, H, ctypes.byref(n)) == RTN_OK
        if L == 2 and H == 16:
            assert n.value == want
        else:
            assert abs(n.value - want) / want < 0.05, (L, H, n.value, want)
    for L, H in ((0, 16), (65, 16), (2, 0), (2, 8193)):
        assert lib.rtn_di_param_count(L, H, ctypes.byref(n)) == RTN_EINVAL


def test_di_validation(lib):
    z = ctypes.c_void_p(16)
    assert lib.rtn_di_model_create(2, 16, 0, None, ctypes.byref(ctypes.c_void_p())) == RTN_EINVAL
    assert lib.rtn_di_model_create(2, 16, 5, z, ctypes.byref(ctypes.c_void_p())) == RTN_EINVAL
    assert lib.rtn_di_model_destroy(None) == RTN_OK
    lin = lambda dt, n, p=z: lib.rtn_di_linearize(None, ctypes.c_float(dt), n, p, p, p, p, p, None, None, None)
    assert lin(0.0, 4) == RTN_EINVAL
    assert lin(0.05, -1) == RTN_EINVAL
    assert lin(0.05, 4, None) == RTN_EINVAL
    assert lin(0.05, 0, None) == RTN_OK
    Q = np.eye(2)
    R = np.array([0.1])
    Rbad = np.array([0.0])
    qp, rp, rb = (a.ctypes.data_as(ctypes.c_void_p) for a in (Q, R, Rbad))

    def rti(n_inst, off, n, r=rp, q=qp, p=z):
        o = None
        if off is not None:
            arr = np.asarray(off, dtype=np.int32)
            rti._keep = arr
            o = arr.ctypes.data_as(ctypes.c_void_p)
        return lib.rtn_di_rti(None, ctypes.c_float(0.05), n_inst, o, n, q, r, q, p, p, p, p, None, p, p, p,
                              None, None, None, None)
    assert rti(1, None, 0) == RTN_OK
    assert rti(1, None, 4, r=rb) == RTN_EINVAL
    assert rti(1, None, 4, q=None) == RTN_EINVAL
    assert rti(2, [0, 2, 2], 2) == RTN_EINVAL
    assert rti(1, None, 4, p=None) == RTN_EINVAL
    assert rti(2, [0, 3, 516], 516) == RTN_ENOTSUP                     # 513 nodes in one instance
    assert b"at most 512" in lib.rtn_last_error()

"""Real-time Neural MPC linearisation path on MI355X (gfx950).

Thin Python binding of librtn.so (C ABI in include/rtn.h).  Arrays are torch
tensors on the GPU; this module only checks and marshals arguments -- every
step of the computation runs in the library's HIP kernels.  There is no CPU
fallback: if librtn.so is missing or the tensors are not on a GPU, calls fail.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import PREC, ACT, INPUT, MlpDesc, Quad, check, load

__all__ = ["Model", "DiModel", "DiRtiCall", "LinearizeCall", "RiccatiCall", "di_linearize", "di_rti", "linearize", "linearize_exact", "linearize_second", "riccati", "riccati_noalloc", "riccati_box", "lq_rollout", "version", "quad_struct", "PREC",
           "profile_enable", "profile_collect", "tune_mode", "tune_get", "tune_set", "tune_save", "tune_load"]


def version() -> str:
    return load().rtn_version().decode()


def profile_enable(on: bool = True) -> None:
    """Bracket every library kernel with HIP events on its stream (see rtn_profile_enable)."""
    check(load().rtn_profile_enable(1 if on else 0), "rtn_profile_enable")


def tune_mode(on: bool) -> None:
    """Turn the first-use tile autotuner on or off (rtn_tune_mode)."""
    check(load().rtn_tune_mode(1 if on else 0), "rtn_tune_mode")


def tune_get(prec: str, width: int, n_hidden: int, n_nodes: int):
    """The kept (path, forward variant, forward workgroups, reverse variant, reverse
    workgroups) and the (forward, reverse) milliseconds measured when tuned, or None
    without an entry."""
    ch = (ctypes.c_int32 * 5)()
    ms = (ctypes.c_float * 2)()
    if load().rtn_tune_get(PREC[prec], width, n_hidden, n_nodes, ch, ms) != 0:
        return None
    return tuple(ch), tuple(ms)


def tune_set(prec: str, width: int, n_hidden: int, n_nodes: int, choice) -> None:
    ch = (ctypes.c_int32 * 5)(*[int(c) for c in choice])
    check(load().rtn_tune_set(PREC[prec], width, n_hidden, n_nodes, ch), "rtn_tune_set")


def tune_save(path: str) -> None:
    check(load().rtn_tune_save(path.encode()), "rtn_tune_save")


def tune_load(path: str) -> None:
    check(load().rtn_tune_load(path.encode()), "rtn_tune_load")


def profile_collect() -> Dict[str, Dict[str, float]]:
    buf = (_lib.KernelTime * 64)()
    n = ctypes.c_int32()
    check(load().rtn_profile_read(buf, 64, ctypes.byref(n)), "rtn_profile_read")
    out = {}
    for i in range(min(n.value, 64)):
        r = buf[i]
        out[r.name.decode()] = {"calls": r.calls, "total_ms": r.total_ms,
                                "avg_ms": r.total_ms / max(r.calls, 1)}
    return out


def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, shape, name):
    """Check a device tensor's dtype/shape/contiguity and return its address."""
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def quad_struct(q) -> Quad:
    return Quad(q.mass, q.Jx, q.Jy, q.Jz, q.arm, q.c_tau, q.g)


class Model:
    """A residual network owned by the library (fp32 master weights on the GPU)."""

    def __init__(self, Ws: Sequence[np.ndarray], bs: Sequence[np.ndarray], activation: str = "silu",
                 input: str = "full"):
        """input: "full" ([v, omega, q, u] -> 6 outputs), "vb" (v_B -> 3) or "vb_u"
        ([v_B, u] -> 3), the residual variants of Sec. VI."""
        L = len(Ws) - 1
        width = Ws[0].shape[0]
        self.input = input
        self.desc = MlpDesc(Ws[0].shape[1], Ws[-1].shape[0], L, width, ACT[activation], INPUT[input])
        self.n_hidden, self.width = L, width
        flat = self._flatten(Ws, bs)
        n = ctypes.c_int64()
        check(load().rtn_param_count(ctypes.byref(self.desc), ctypes.byref(n)), "rtn_param_count")
        if n.value != flat.size:
            raise ValueError(f"parameter count {flat.size} does not match the descriptor ({n.value})")
        h = ctypes.c_void_p()
        check(load().rtn_model_create(ctypes.byref(self.desc), flat.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(h)), "rtn_model_create")
        self._h = h
        self.n_params = n.value

    @staticmethod
    def _flatten(Ws, bs) -> np.ndarray:
        parts = []
        for W, b in zip(Ws, bs):
            parts += [np.ascontiguousarray(W, dtype=np.float32).ravel(), np.ascontiguousarray(b, dtype=np.float32).ravel()]
        return np.ascontiguousarray(np.concatenate(parts), dtype=np.float32)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("model has been closed")
        return self._h

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        check(load().rtn_model_get_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)), "rtn_model_get_params")
        return out

    def set_params(self, Ws, bs) -> None:
        flat = self._flatten(Ws, bs)
        check(load().rtn_model_set_params(self.handle, flat.ctypes.data_as(ctypes.c_void_p)), "rtn_model_set_params")

    def calibrate(self, x, u, stream=None) -> None:
        torch = _torch()
        n = x.shape[0]
        check(load().rtn_model_calibrate(self.handle, n, _dev(x, torch.float32, (n, 13), "x"),
                                         _dev(u, torch.float32, (n, 4), "u"), _stream(stream)),
              "rtn_model_calibrate")

    def scales(self) -> np.ndarray:
        k = ctypes.c_int32()
        check(load().rtn_model_get_scales(self.handle, None, ctypes.byref(k)), "rtn_model_get_scales")
        out = np.zeros(k.value, dtype=np.float32)
        check(load().rtn_model_get_scales(self.handle, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(k)),
              "rtn_model_get_scales")
        return out

    # ---- training (Sec. VII): the library's own forward/backward kernels -------------
    def forward_batch(self, z, prec: str = "bf16", stream=None):
        """Network output y [B,6] for inputs z [B,14]; stashes what backward_batch needs."""
        torch = _torch()
        B = z.shape[0]
        y = torch.empty((B, 6), dtype=torch.float32, device=z.device)
        check(load().rtn_mlp_forward(self.handle, PREC[prec], B, _dev(z, torch.float32, (B, 14), "z"),
                                     _dev(y, torch.float32, (B, 6), "y"), _stream(stream)), "rtn_mlp_forward")
        return y

    def backward_batch(self, dy, want_din: bool = True, stream=None):
        """Add dL/dparams for upstream dy [B,6] to the gradient buffer; return dL/dz [B,14]."""
        torch = _torch()
        B = dy.shape[0]
        din = torch.empty((B, 14), dtype=torch.float32, device=dy.device) if want_din else None
        check(load().rtn_mlp_backward(self.handle, B, _dev(dy.contiguous(), torch.float32, (B, 6), "dy"),
                                      _dev(din, torch.float32, (B, 14), "din") if din is not None else None,
                                      _stream(stream)), "rtn_mlp_backward")
        return din

    def zero_grad(self, stream=None) -> None:
        check(load().rtn_model_zero_grad(self.handle, _stream(stream)), "rtn_model_zero_grad")

    def get_grad(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        check(load().rtn_model_get_grad(self.handle, out.ctypes.data_as(ctypes.c_void_p)), "rtn_model_get_grad")
        return out

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None) -> None:
        check(load().rtn_adam_step(self.handle, lr, beta1, beta2, eps, _stream(stream)), "rtn_adam_step")

    def train_step(self, z, target, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, prec: str = "bf16",
                   loss=None, stream=None):
        """Fused forward + MSE + backward + Adam; returns the (device) loss before the update."""
        torch = _torch()
        B = z.shape[0]
        if loss is None:
            loss = torch.empty((1,), dtype=torch.float32, device=z.device)
        check(load().rtn_train_step(self.handle, PREC[prec], B, _dev(z, torch.float32, (B, 14), "z"),
                                    _dev(target, torch.float32, (B, 6), "target"), lr, beta1, beta2, eps,
                                    _dev(loss, torch.float32, (1,), "loss"), _stream(stream)), "rtn_train_step")
        return loss

    def get_adam(self):
        m = np.empty(self.n_params, dtype=np.float32)
        v = np.empty(self.n_params, dtype=np.float32)
        t = ctypes.c_int64()
        check(load().rtn_model_get_adam(self.handle, m.ctypes.data_as(ctypes.c_void_p),
                                        v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t)), "rtn_model_get_adam")
        return m, v, t.value

    def set_adam(self, m, v, step: int) -> None:
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        check(load().rtn_model_set_adam(self.handle, m.ctypes.data_as(ctypes.c_void_p),
                                        v.ctypes.data_as(ctypes.c_void_p), step), "rtn_model_set_adam")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            load().rtn_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def linearize(x, u, model: Optional[Model] = None, prec: str = "fp32", dt: float = 0.05, quad=None,
              offsets: Optional[np.ndarray] = None, want_fd: bool = True, want_status: bool = False,
              out: Optional[Dict[str, object]] = None, stream=None) -> Dict[str, object]:
    """rtn_linearize over device tensors x [n,13], u [n,4] (fp32).

    Returns a dict with x_next [n,13], A [n,13,13], B [n,13,4] and, on request,
    f_D [n,6], J_D [n,6,14], status [n] (uint8).  ``out`` may supply the output
    tensors to avoid allocation."""
    torch = _torch()
    from workload import QUAD
    q = quad_struct(quad if quad is not None else QUAD)
    n = x.shape[0]
    dev = x.device
    if out is None:
        out = {}
    def get(name, shape, dtype=torch.float32):
        t = out.get(name)
        if t is None:
            t = torch.empty(shape, dtype=dtype, device=dev)
            out[name] = t
        return t
    xn = get("x_next", (n, 13))
    A = get("A", (n, 13, 13))
    B = get("B", (n, 13, 4))
    fD = get("f_D", (n, 6)) if want_fd else None
    JD = get("J_D", (n, 6, 14)) if want_fd else None
    st = get("status", (n,), torch.uint8) if want_status else None
    if offsets is None:
        n_inst, off_ptr, off_arr = 1, None, None
    else:
        off_arr = np.ascontiguousarray(offsets, dtype=np.int32)
        n_inst, off_ptr = off_arr.size - 1, off_arr.ctypes.data_as(ctypes.c_void_p)
    check(load().rtn_linearize(model.handle if model is not None else None, PREC[prec], ctypes.byref(q),
                               ctypes.c_float(dt), n_inst, off_ptr, n,
                               _dev(x, torch.float32, (n, 13), "x"), _dev(u, torch.float32, (n, 4), "u"),
                               _dev(xn, torch.float32, (n, 13), "x_next"), _dev(A, torch.float32, (n, 13, 13), "A"),
                               _dev(B, torch.float32, (n, 13, 4), "B"),
                               _dev(fD, torch.float32, (n, 6), "f_D") if fD is not None else None,
                               _dev(JD, torch.float32, (n, 6, 14), "J_D") if JD is not None else None,
                               _dev(st, torch.uint8, (n,), "status") if st is not None else None,
                               _stream(stream)), "rtn_linearize")
    return out


class LinearizeCall:
    """rtn_linearize with its arguments checked and marshalled once: each call only
    enqueues the linearisation (one launch, or the replay of a captured graph), for
    real-time loops that refill the same x, u tensors every tick."""

    def __init__(self, x, u, model: Optional[Model] = None, prec: str = "fp32", dt: float = 0.05, quad=None,
                 offsets: Optional[np.ndarray] = None, want_fd: bool = True, want_status: bool = False,
                 stream=None):
        self.out = linearize(x, u, model, prec, dt, quad, offsets, want_fd, want_status, stream=stream)
        torch = _torch()
        from workload import QUAD
        self._q = quad_struct(quad if quad is not None else QUAD)
        n = x.shape[0]
        self._off = None if offsets is None else np.ascontiguousarray(offsets, dtype=np.int32)
        n_inst = 1 if self._off is None else self._off.size - 1
        o = self.out
        f32 = torch.float32
        self._fn = load().rtn_linearize
        self._args = (model.handle if model is not None else None, PREC[prec], ctypes.byref(self._q),
                      ctypes.c_float(dt), n_inst,
                      None if self._off is None else self._off.ctypes.data_as(ctypes.c_void_p), n,
                      _dev(x, f32, (n, 13), "x"), _dev(u, f32, (n, 4), "u"), _dev(o["x_next"], f32, (n, 13), "x_next"),
                      _dev(o["A"], f32, (n, 13, 13), "A"), _dev(o["B"], f32, (n, 13, 4), "B"),
                      _dev(o.get("f_D"), f32, (n, 6), "f_D"), _dev(o.get("J_D"), f32, (n, 6, 14), "J_D"),
                      _dev(o.get("status"), torch.uint8, (n,), "status"), _stream(stream))
        self._tensors = (x, u, model)  # keep the buffers alive

    def __call__(self) -> Dict[str, object]:
        code = self._fn(*self._args)
        if code != 0:
            check(code, "rtn_linearize")
        return self.out


def linearize_exact(x, u, model: Model, prec: str = "fp32", dt: float = 0.05, quad=None,
                    offsets: Optional[np.ndarray] = None, out: Optional[Dict[str, object]] = None,
                    stream=None) -> Dict[str, object]:
    """rtn_linearize_exact: network and Jacobian at all four RK4 stage points (the naive
    linearisation the paper's local approximation avoids).  Returns x_next, A, B."""
    torch = _torch()
    from workload import QUAD
    q = quad_struct(quad if quad is not None else QUAD)
    n = x.shape[0]
    out = {} if out is None else out
    for name, shape in (("x_next", (n, 13)), ("A", (n, 13, 13)), ("B", (n, 13, 4))):
        if out.get(name) is None:
            out[name] = torch.empty(shape, dtype=torch.float32, device=x.device)
    if offsets is None:
        n_inst, off_ptr = 1, None
    else:
        off_arr = np.ascontiguousarray(offsets, dtype=np.int32)
        n_inst, off_ptr = off_arr.size - 1, off_arr.ctypes.data_as(ctypes.c_void_p)
    check(load().rtn_linearize_exact(model.handle, PREC[prec], ctypes.byref(q), ctypes.c_float(dt), n_inst, off_ptr,
                                     n, _dev(x, torch.float32, (n, 13), "x"), _dev(u, torch.float32, (n, 4), "u"),
                                     _dev(out["x_next"], torch.float32, (n, 13), "x_next"),
                                     _dev(out["A"], torch.float32, (n, 13, 13), "A"),
                                     _dev(out["B"], torch.float32, (n, 13, 4), "B"), _stream(stream)),
          "rtn_linearize_exact")
    return out


def linearize_second(x, u, model: Model, dt: float = 0.05, quad=None, offsets: Optional[np.ndarray] = None,
                     want_hessian: bool = True, out: Optional[Dict[str, object]] = None,
                     stream=None) -> Dict[str, object]:
    """rtn_linearize_second (fp32): RK4 of f_F plus the second-order local approximation.
    Returns x_next, A, B, f_D, J_D and optionally H_D [n,6,14,14]."""
    torch = _torch()
    from workload import QUAD
    q = quad_struct(quad if quad is not None else QUAD)
    n = x.shape[0]
    out = {} if out is None else out
    shapes = [("x_next", (n, 13)), ("A", (n, 13, 13)), ("B", (n, 13, 4)), ("f_D", (n, 6)), ("J_D", (n, 6, 14))]
    if want_hessian:
        shapes.append(("H_D", (n, 6, 14, 14)))
    for name, shape in shapes:
        if out.get(name) is None:
            out[name] = torch.empty(shape, dtype=torch.float32, device=x.device)
    if offsets is None:
        n_inst, off_ptr = 1, None
    else:
        off_arr = np.ascontiguousarray(offsets, dtype=np.int32)
        n_inst, off_ptr = off_arr.size - 1, off_arr.ctypes.data_as(ctypes.c_void_p)
    f32 = torch.float32
    check(load().rtn_linearize_second(model.handle, PREC["fp32"], ctypes.byref(q), ctypes.c_float(dt), n_inst,
                                      off_ptr, n, _dev(x, f32, (n, 13), "x"), _dev(u, f32, (n, 4), "u"),
                                      _dev(out["x_next"], f32, (n, 13), "x_next"), _dev(out["A"], f32, (n, 13, 13), "A"),
                                      _dev(out["B"], f32, (n, 13, 4), "B"), _dev(out["f_D"], f32, (n, 6), "f_D"),
                                      _dev(out["J_D"], f32, (n, 6, 14), "J_D"),
                                      _dev(out["H_D"], f32, (n, 6, 14, 14), "H_D") if want_hessian else None,
                                      _stream(stream)), "rtn_linearize_second")
    return out


def riccati(A, B, Q, R, QN, offsets=None, c=None, q=None, r=None, qN=None, want_P: bool = False,
            out: Optional[Dict[str, object]] = None, stream=None, _entry: str = "rtn_riccati") -> Dict[str, object]:
    """rtn_riccati over device tensors A [n,13,13], B [n,13,4] (fp32); Q, R, QN host arrays (fp64).

    Returns K [n,4,13], kff [n,4] and optionally P [n,13,13] (fp64 device tensors)."""
    torch = _torch()
    n = A.shape[0]
    dev = A.device
    if out is None:
        out = {}
    def get(name, shape):
        t = out.get(name)
        if t is None:
            t = out[name] = torch.empty(shape, dtype=torch.float64, device=dev)
        return t
    K = get("K", (n, 4, 13))
    kff = get("kff", (n, 4))
    P = get("P", (n, 13, 13)) if want_P else None
    if offsets is None:
        n_inst, off_ptr = 1, None
    else:
        off_arr = np.ascontiguousarray(offsets, dtype=np.int32)
        n_inst, off_ptr = off_arr.size - 1, off_arr.ctypes.data_as(ctypes.c_void_p)
    Qh = np.ascontiguousarray(Q, dtype=np.float64)
    Rh = np.ascontiguousarray(R, dtype=np.float64)
    QNh = np.ascontiguousarray(QN, dtype=np.float64)
    f64 = torch.float64
    check(getattr(load(), _entry)(n_inst, off_ptr, n, _dev(A, torch.float32, (n, 13, 13), "A"),
                             _dev(B, torch.float32, (n, 13, 4), "B"),
                             _dev(c, f64, (n, 13), "c") if c is not None else None,
                             Qh.ctypes.data_as(ctypes.c_void_p), Rh.ctypes.data_as(ctypes.c_void_p),
                             QNh.ctypes.data_as(ctypes.c_void_p),
                             _dev(q, f64, (n, 13), "q") if q is not None else None,
                             _dev(r, f64, (n, 4), "r") if r is not None else None,
                             _dev(qN, f64, (n_inst, 13), "qN") if qN is not None else None,
                             _dev(K, f64, (n, 4, 13), "K"), _dev(kff, f64, (n, 4), "kff"),
                             _dev(P, f64, (n, 13, 13), "P") if P is not None else None,
                             _stream(stream)), _entry)
    return out


def riccati_noalloc(A, B, Q, R, QN, offsets=None, c=None, q=None, r=None, qN=None, want_P: bool = False,
                    out: Optional[Dict[str, object]] = None, stream=None) -> Dict[str, object]:
    """rtn_riccati_noalloc: rtn_riccati without any device allocation in the library
    (at most 65536 instances).  Pass `out` with K, kff (and P) to allocate nothing here either."""
    return riccati(A, B, Q, R, QN, offsets, c, q, r, qN, want_P, out, stream, _entry="rtn_riccati_noalloc")


class RiccatiCall:
    """rtn_riccati with its arguments checked and marshalled once (no affine terms):
    each call only enqueues the recursion over the current contents of A, B."""

    def __init__(self, A, B, Q, R, QN, offsets=None, want_P: bool = False, stream=None):
        self.out = riccati(A, B, Q, R, QN, offsets=offsets, want_P=want_P, stream=stream)
        torch = _torch()
        n = A.shape[0]
        self._off = None if offsets is None else np.ascontiguousarray(offsets, dtype=np.int32)
        n_inst = 1 if self._off is None else self._off.size - 1
        self._h = [np.ascontiguousarray(M, dtype=np.float64) for M in (Q, R, QN)]
        f64, o = torch.float64, self.out
        self._fn = load().rtn_riccati
        self._args = (n_inst, None if self._off is None else self._off.ctypes.data_as(ctypes.c_void_p), n,
                      _dev(A, torch.float32, (n, 13, 13), "A"), _dev(B, torch.float32, (n, 13, 4), "B"), None,
                      *(M.ctypes.data_as(ctypes.c_void_p) for M in self._h), None, None, None,
                      _dev(o["K"], f64, (n, 4, 13), "K"), _dev(o["kff"], f64, (n, 4), "kff"),
                      _dev(o.get("P"), f64, (n, 13, 13), "P"), _stream(stream))
        self._tensors = (A, B)  # keep the buffers alive

    def __call__(self) -> Dict[str, object]:
        code = self._fn(*self._args)
        if code != 0:
            check(code, "rtn_riccati")
        return self.out


def riccati_box(A, B, Q, R, QN, dx0, du_lo, du_hi, offsets=None, c=None, q=None, r=None, qN=None,
                rho: float = 1.0, max_iter: int = 500, tol: float = 1e-8, want_dx: bool = True,
                out: Optional[Dict[str, object]] = None, stream=None) -> Dict[str, object]:
    """rtn_riccati_box: the LQ step with the input box du_lo <= du <= du_hi (ADMM).
    Returns du [n,4], iters [n_inst] (int32), resid [n_inst,2] (primal, dual residual of
    the last iteration) and optionally dx [n,13], dxN [n_inst,13]."""
    torch = _torch()
    n = A.shape[0]
    dev = A.device
    if offsets is None:
        n_inst, off_ptr = 1, None
    else:
        off_arr = np.ascontiguousarray(offsets, dtype=np.int32)
        n_inst, off_ptr = off_arr.size - 1, off_arr.ctypes.data_as(ctypes.c_void_p)
    if out is None:
        out = {}
    def get(name, shape, dtype=torch.float64):
        t = out.get(name)
        if t is None:
            t = out[name] = torch.empty(shape, dtype=dtype, device=dev)
        return t
    f64 = torch.float64
    du = get("du", (n, 4))
    iters = get("iters", (n_inst,), torch.int32)
    resid = get("resid", (n_inst, 2))
    dx = get("dx", (n, 13)) if want_dx else None
    dxN = get("dxN", (n_inst, 13)) if want_dx else None
    Qh = np.ascontiguousarray(Q, dtype=np.float64)
    Rh = np.ascontiguousarray(R, dtype=np.float64)
    QNh = np.ascontiguousarray(QN, dtype=np.float64)
    check(load().rtn_riccati_box(n_inst, off_ptr, n, _dev(A, torch.float32, (n, 13, 13), "A"),
                                 _dev(B, torch.float32, (n, 13, 4), "B"),
                                 _dev(c, f64, (n, 13), "c") if c is not None else None,
                                 Qh.ctypes.data_as(ctypes.c_void_p), Rh.ctypes.data_as(ctypes.c_void_p),
                                 QNh.ctypes.data_as(ctypes.c_void_p),
                                 _dev(q, f64, (n, 13), "q") if q is not None else None,
                                 _dev(r, f64, (n, 4), "r") if r is not None else None,
                                 _dev(qN, f64, (n_inst, 13), "qN") if qN is not None else None,
                                 _dev(dx0, f64, (n_inst, 13), "dx0"), _dev(du_lo, f64, (n, 4), "du_lo"),
                                 _dev(du_hi, f64, (n, 4), "du_hi"), float(rho), int(max_iter), float(tol),
                                 _dev(du, f64, (n, 4), "du"),
                                 _dev(dx, f64, (n, 13), "dx") if dx is not None else None,
                                 _dev(dxN, f64, (n_inst, 13), "dxN") if dxN is not None else None,
                                 _dev(iters, torch.int32, (n_inst,), "iters"), _dev(resid, f64, (n_inst, 2), "resid"),
                                 _stream(stream)), "rtn_riccati_box")
    return out


def lq_rollout(A, B, K, kff, dx0, offsets=None, c=None, want_dx: bool = True,
               out: Optional[Dict[str, object]] = None, stream=None) -> Dict[str, object]:
    """rtn_lq_rollout: the primal step of the LQ solution from per-instance initial
    deviations dx0 [n_inst,13] (fp64).  Returns du [n,4], and optionally dx [n,13] and
    the terminal dxN [n_inst,13] (fp64 device tensors)."""
    torch = _torch()
    n = A.shape[0]
    dev = A.device
    if offsets is None:
        n_inst, off_ptr = 1, None
    else:
        off_arr = np.ascontiguousarray(offsets, dtype=np.int32)
        n_inst, off_ptr = off_arr.size - 1, off_arr.ctypes.data_as(ctypes.c_void_p)
    if out is None:
        out = {}
    def get(name, shape):
        t = out.get(name)
        if t is None:
            t = out[name] = torch.empty(shape, dtype=torch.float64, device=dev)
        return t
    f64 = torch.float64
    du = get("du", (n, 4))
    dx = get("dx", (n, 13)) if want_dx else None
    dxN = get("dxN", (n_inst, 13)) if want_dx else None
    check(load().rtn_lq_rollout(n_inst, off_ptr, n, _dev(A, torch.float32, (n, 13, 13), "A"),
                                _dev(B, torch.float32, (n, 13, 4), "B"),
                                _dev(c, f64, (n, 13), "c") if c is not None else None,
                                _dev(K, f64, (n, 4, 13), "K"), _dev(kff, f64, (n, 4), "kff"),
                                _dev(dx0, f64, (n_inst, 13), "dx0"),
                                _dev(dx, f64, (n, 13), "dx") if dx is not None else None,
                                _dev(du, f64, (n, 4), "du"),
                                _dev(dxN, f64, (n_inst, 13), "dxN") if dxN is not None else None,
                                _stream(stream)), "rtn_lq_rollout")
    return out


def mlp_function():
    """torch.autograd.Function over the library's forward/backward kernels.

    ``MLP.apply(z, model, prec)`` returns y [B,6]; its backward returns dL/dz and
    adds dL/dparams to the model's gradient buffer (step with model.adam_step)."""
    torch = _torch()

    class MLP(torch.autograd.Function):
        @staticmethod
        def forward(ctx, z, model, prec="bf16"):
            ctx.model = model
            return model.forward_batch(z.contiguous(), prec)

        @staticmethod
        def backward(ctx, dy):
            return ctx.model.backward_batch(dy.contiguous(), want_din=True), None, None

    return MLP


# ---- runtime workload of Sec. V: double integrator with a network residual ------------
class DiModel:
    """A 2-in / 2-out residual network of the double-integrator workload (fp32 on the GPU)."""

    def __init__(self, Ws: Sequence[np.ndarray], bs: Sequence[np.ndarray], activation: str = "silu"):
        L = len(Ws) - 1
        width = Ws[0].shape[0]
        flat = Model._flatten(Ws, bs)
        n = ctypes.c_int64()
        check(load().rtn_di_param_count(L, width, ctypes.byref(n)), "rtn_di_param_count")
        if n.value != flat.size:
            raise ValueError(f"parameter count {flat.size} does not match n_hidden={L}, width={width} ({n.value})")
        h = ctypes.c_void_p()
        check(load().rtn_di_model_create(L, width, ACT[activation], flat.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(h)), "rtn_di_model_create")
        self._h = h
        self.n_hidden, self.width, self.n_params = L, width, n.value

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("model has been closed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            load().rtn_di_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def di_linearize(x, u, model: Optional[DiModel] = None, dt: float = 0.05, want_fd: bool = True,
                 stream=None) -> Dict[str, object]:
    """rtn_di_linearize over device tensors x [n,2], u [n] (fp32): x_next [n,2], A [n,2,2],
    B [n,2] and, on request, f_D [n,2], J_D [n,2,2]."""
    torch = _torch()
    n = x.shape[0]
    f32 = torch.float32
    out = {k: torch.empty(s, dtype=f32, device=x.device)
           for k, s in (("x_next", (n, 2)), ("A", (n, 2, 2)), ("B", (n, 2)))}
    if want_fd:
        out["f_D"] = torch.empty((n, 2), dtype=f32, device=x.device)
        out["J_D"] = torch.empty((n, 2, 2), dtype=f32, device=x.device)
    check(load().rtn_di_linearize(model.handle if model is not None else None, ctypes.c_float(dt), n,
                                  _dev(x, f32, (n, 2), "x"), _dev(u, f32, (n,), "u"),
                                  _dev(out["x_next"], f32, (n, 2), "x_next"), _dev(out["A"], f32, (n, 2, 2), "A"),
                                  _dev(out["B"], f32, (n, 2), "B"),
                                  _dev(out.get("f_D"), f32, (n, 2), "f_D"), _dev(out.get("J_D"), f32, (n, 2, 2), "J_D"),
                                  _stream(stream)), "rtn_di_linearize")
    return out


def di_rti(x, u, xN, x0, model: Optional[DiModel], Q, R, QN, dt: float = 0.05, offsets=None, x_ref=None,
           want_linearisation: bool = False, out: Optional[Dict[str, object]] = None,
           stream=None) -> Dict[str, object]:
    """rtn_di_rti: one real-time iteration of every instance.  x [n,2], u [n], xN, x0 (and
    x_ref) [n_inst,2] device fp32; Q, R, QN host fp64.  Returns du [n], dx [n,2],
    dxN [n_inst,2] (fp64) and, on request, the linearisation A, B, x_next (fp32)."""
    torch = _torch()
    n = x.shape[0]
    if offsets is None:
        n_inst, off_ptr = 1, None
    else:
        off_arr = np.ascontiguousarray(offsets, dtype=np.int32)
        n_inst, off_ptr = off_arr.size - 1, off_arr.ctypes.data_as(ctypes.c_void_p)
    if out is None:
        out = {}
    dev = x.device
    f32, f64 = torch.float32, torch.float64

    def get(name, shape, dtype):
        t = out.get(name)
        if t is None:
            t = out[name] = torch.empty(shape, dtype=dtype, device=dev)
        return t
    du, dx, dxN = get("du", (n,), f64), get("dx", (n, 2), f64), get("dxN", (n_inst, 2), f64)
    A = get("A", (n, 2, 2), f32) if want_linearisation else None
    B = get("B", (n, 2), f32) if want_linearisation else None
    xn = get("x_next", (n, 2), f32) if want_linearisation else None
    Qh = np.ascontiguousarray(Q, dtype=np.float64).reshape(2, 2)
    Rh = np.ascontiguousarray(R, dtype=np.float64).reshape(1)
    QNh = np.ascontiguousarray(QN, dtype=np.float64).reshape(2, 2)
    check(load().rtn_di_rti(model.handle if model is not None else None, ctypes.c_float(dt), n_inst, off_ptr, n,
                            Qh.ctypes.data_as(ctypes.c_void_p), Rh.ctypes.data_as(ctypes.c_void_p),
                            QNh.ctypes.data_as(ctypes.c_void_p),
                            _dev(x, f32, (n, 2), "x"), _dev(u, f32, (n,), "u"), _dev(xN, f32, (n_inst, 2), "xN"),
                            _dev(x0, f32, (n_inst, 2), "x0"), _dev(x_ref, f32, (n_inst, 2), "x_ref"),
                            _dev(du, f64, (n,), "du"), _dev(dx, f64, (n, 2), "dx"), _dev(dxN, f64, (n_inst, 2), "dxN"),
                            _dev(A, f32, (n, 2, 2), "A"), _dev(B, f32, (n, 2), "B"), _dev(xn, f32, (n, 2), "x_next"),
                            _stream(stream)), "rtn_di_rti")
    return out


class DiRtiCall:
    """rtn_di_rti with its arguments checked and marshalled once: each call only
    enqueues the iteration (one launch, or the replay of a captured graph), for control
    loops that refill the same input tensors every tick."""

    def __init__(self, x, u, xN, x0, model: Optional[DiModel], Q, R, QN, dt: float = 0.05, offsets=None,
                 x_ref=None, want_linearisation: bool = False, stream=None):
        self.out = di_rti(x, u, xN, x0, model, Q, R, QN, dt, offsets, x_ref, want_linearisation, stream=stream)
        torch = _torch()
        n = x.shape[0]
        self._keep = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (Q, R, QN)]
        if offsets is None:
            n_inst, off = 1, None
        else:
            off_arr = np.ascontiguousarray(offsets, dtype=np.int32)
            self._keep.append(off_arr)
            n_inst, off = off_arr.size - 1, off_arr.ctypes.data_as(ctypes.c_void_p)
        o = self.out
        f32, f64 = torch.float32, torch.float64
        self._fn = load().rtn_di_rti
        self._args = (model.handle if model is not None else None, ctypes.c_float(dt), n_inst, off, n,
                      *(a.ctypes.data_as(ctypes.c_void_p) for a in self._keep[:3]),
                      _dev(x, f32, (n, 2), "x"), _dev(u, f32, (n,), "u"), _dev(xN, f32, (n_inst, 2), "xN"),
                      _dev(x0, f32, (n_inst, 2), "x0"), _dev(x_ref, f32, (n_inst, 2), "x_ref"),
                      _dev(o["du"], f64, (n,), "du"), _dev(o["dx"], f64, (n, 2), "dx"),
                      _dev(o["dxN"], f64, (n_inst, 2), "dxN"),
                      _dev(o.get("A"), f32, (n, 2, 2), "A"), _dev(o.get("B"), f32, (n, 2), "B"),
                      _dev(o.get("x_next"), f32, (n, 2), "x_next"), _stream(stream))
        self._tensors = (x, u, xN, x0, x_ref, model)  # keep the buffers alive

    def __call__(self) -> Dict[str, object]:
        code = self._fn(*self._args)
        if code != 0:
            check(code, "rtn_di_rti")
        return self.out

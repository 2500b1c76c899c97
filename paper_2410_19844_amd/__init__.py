"""Python binding of libsos: the over-parameterised SOS method on MI355X.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libsos.so`` (built by ``paper_2410_19844_amd.build``).  PyTorch
provides device memory and the stream; tensors are passed to the C ABI as
raw data pointers.  Importing this package fails loudly if the library is
missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsos.so")

FP64, FP32, BF16X3, FP16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp16x3": FP16X3}
FLAG_EXACT_FORWARD = 1
FLAG_COPIES_VALID = 2
FLAG_SINGLE_BACKWARD = 4
FLAG_FP32_FORWARD = 8
FLAG_OZAKI_FORWARD = 16
FLAG_DETERMINISTIC = 32
FLAG_UNFUSED_SCATTER = 64
FLAG_UNMERGED_SCATTER = 128
FLAG_OZAKI_FIVE_SLICES = 256
FLAG_SINGLE_FORWARD = 512
FLAG_OZAKI_FOUR_SLICES = 1024
OK, NOT_CONVERGED = 0, 1
EINVAL, ERANGE, ENOMEM, EHIP, ENUMERIC = -1, -2, -3, -4, -5


class SosError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsos error {code}: {msg}")
        self.code = code


class _Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("check_every", ctypes.c_int64), ("ladder", ctypes.c_int32),
                ("stall_checks", ctypes.c_int32), ("stall_ratio", ctypes.c_double),
                ("switch_rel", ctypes.c_double), ("lr_exact", ctypes.c_double),
                ("rollback_ratio", ctypes.c_double), ("single_backward", ctypes.c_int32),
                ("finisher", ctypes.c_int32), ("mid_rel", ctypes.c_double),
                ("step_flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("single_rel", ctypes.c_double), ("four_rel", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("exact_steps", ctypes.c_int64),
                ("loss", ctypes.c_double), ("rel", ctypes.c_double),
                ("best_rel", ctypes.c_double), ("status", ctypes.c_int32),
                ("phase", ctypes.c_int32)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: run `python paper_2410_19844_amd/build.py`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, V, I, I64 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    sig = {
        "sos_plan": (I, [I, I, I, I, ctypes.POINTER(P)]),
        "sos_plan_query": (I, [P, ctypes.POINTER(I64), ctypes.POINTER(I64),
                               ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "sos_plan_bind": (I, [P, V, ctypes.c_size_t, V]),
        "sos_plan_destroy": (None, [P]),
        "sos_exponents": (I, [P, I, V]),
        "sos_pair_ranks": (I, [P, V, V]),
        "sos_loss_grad": (I, [P, V, V, V, V, V, I, V]),
        "sos_loss_grad_noalloc": (I, [P, V, V, V, V, V, I, V]),
        "sos_step": (I, [P, V, V, I64, V, ctypes.POINTER(_Adam), V, I, V]),
        "sos_solve": (I, [P, V, V, V, ctypes.POINTER(_Adam), ctypes.POINTER(_SolveOpts),
                          ctypes.POINTER(_Result), V]),
        "sos_verify": (I, [P, V, V, ctypes.POINTER(ctypes.c_double), V, V]),
        "sos_step_batch": (I, [ctypes.POINTER(P), ctypes.POINTER(V), ctypes.POINTER(V),
                               ctypes.POINTER(I64), ctypes.POINTER(V), ctypes.POINTER(_Adam), V, I, V]),
        "sos_loss_batch": (I, [ctypes.POINTER(P), ctypes.POINTER(V), ctypes.POINTER(V), V, I, V]),
        "sos_net_query": (I, [P, I, I, ctypes.POINTER(ctypes.c_size_t)]),
        "sos_net_weights": (I, [P, I, I, V, V, V, V, V]),
        "sos_net_grad": (I, [P, I, I, V, V, V, V, V, V, V, I, V]),
        "sos_net_step": (I, [P, I, I, V, V, V, I64, V, ctypes.POINTER(_Adam), V, I, I, V]),
        "sos_net_solve": (I, [P, I, I, V, V, V, V, ctypes.POINTER(_Adam), ctypes.POINTER(_SolveOpts), I,
                              ctypes.POINTER(_Result), V]),
        "sos_timing": (I, [P, I]),
        "sos_timing_read": (I, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]),
        "sos_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTS = ("sos_plan", "sos_plan_query", "sos_plan_bind", "sos_plan_destroy", "sos_exponents",
           "sos_pair_ranks", "sos_loss_grad", "sos_loss_grad_noalloc", "sos_step", "sos_solve", "sos_verify",
           "sos_step_batch", "sos_loss_batch", "sos_net_query", "sos_net_weights", "sos_net_grad", "sos_net_step",
           "sos_net_solve", "sos_timing", "sos_timing_read", "sos_last_error")
KERNEL_CLASSES = ("prep", "init_r", "gram", "loss", "gather", "rw", "adam", "scatter")


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        raise SosError(rc, _lib.sos_last_error().decode())
    return rc


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _oz_flags(ozaki):
    """Flags of the Ozaki forward: False (off), True or 6 (six digit slices), 5 or 4."""
    if ozaki is False or ozaki is None or ozaki == 0:
        return 0
    if ozaki is True or ozaki == 6:
        return FLAG_OZAKI_FORWARD
    if ozaki == 5:
        return FLAG_OZAKI_FORWARD | FLAG_OZAKI_FIVE_SLICES
    if ozaki == 4:
        return FLAG_OZAKI_FORWARD | FLAG_OZAKI_FOUR_SLICES
    raise ValueError("ozaki must be False, True, 4, 5 or 6")


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def c(self):
        return _Adam(self.lr, self.beta1, self.beta2, self.eps)


def sos_plan(n: int, d: int, rank: int, precision="fp32"):
    """Host-only plan (no device memory).  See ``Plan`` for a bound plan."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    h = ctypes.c_void_p()
    _check(_lib.sos_plan(n, d, rank, prec, ctypes.byref(h)))
    return h


class Plan:
    """A bound plan: host tables plus a device workspace owned by this object.

    With bind=False no workspace is allocated and the plan stays unbound: only
    ``loss_grad_noalloc`` (the library's static workspace) can run it."""

    def __init__(self, n: int, d: int, rank: int, precision="fp32", device="cuda", stream=None, bind=True):
        self.n, self.d, self.rank = n, d, rank
        self.prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self._h = sos_plan(n, d, rank, self.prec)
        N, M = ctypes.c_int64(), ctypes.c_int64()
        ws, st = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.sos_plan_query(self._h, ctypes.byref(N), ctypes.byref(M), ctypes.byref(ws), ctypes.byref(st)))
        self.N, self.M = N.value, M.value
        self.ws_bytes, self.state_bytes = ws.value, st.value
        self.wdtype = torch.float64 if self.prec == FP64 else torch.float32
        self.device = torch.device(device)
        self.ws = None
        if self.device.type == "cuda" and bind:
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            self._ws_view = self.ws[off:off + self.ws_bytes]
            _check(_lib.sos_plan_bind(self._h, ctypes.c_void_p(self._ws_view.data_ptr()),
                                      self.ws_bytes, _stream(stream)))

    _destroy = _lib.sos_plan_destroy

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    # -- host queries ------------------------------------------------------
    def exponents(self, which: int = 0):
        import numpy as np
        rows = self.N if which == 0 else self.M
        out = np.empty((rows, self.n), dtype=np.uint8)
        _check(_lib.sos_exponents(self._h, which, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    # -- device calls ------------------------------------------------------
    def new_state(self):
        return torch.zeros(self.state_bytes, dtype=torch.uint8, device=self.device)

    def _w(self, W):
        if W.dtype != self.wdtype or not W.is_contiguous() or tuple(W.shape) != (self.N, self.rank):
            raise ValueError(f"W must be a contiguous {self.wdtype} tensor of shape ({self.N}, {self.rank})")
        return W

    def _p(self, p):
        if p.dtype != torch.float64 or not p.is_contiguous() or p.numel() != self.M:
            raise ValueError(f"p must be a contiguous float64 tensor of {self.M} elements")
        return p

    def pair_ranks(self, stream=None):
        out = torch.empty((self.N, self.N), dtype=torch.int32, device=self.device)
        _check(_lib.sos_pair_ranks(self._h, _ptr(out), _stream(stream)))
        return out

    def loss_grad(self, W, p, grad=True, want_r=False, exact=False, single_backward=False,
                  fp32_forward=False, ozaki=False, deterministic=False, unfused_scatter=False,
                  unmerged_scatter=False, single_forward=False, stream=None):
        self._w(W), self._p(p)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        g = torch.empty_like(W) if grad else None
        r = torch.empty(self.M, dtype=torch.float64, device=self.device) if want_r else None
        _check(_lib.sos_loss_grad(self._h, _ptr(W), _ptr(p), _ptr(loss), _ptr(g), _ptr(r),
                                  (FLAG_EXACT_FORWARD if exact else 0) |
                                  (FLAG_SINGLE_BACKWARD if single_backward else 0) |
                                  (FLAG_FP32_FORWARD if fp32_forward else 0) |
                                  _oz_flags(ozaki) |
                                  (FLAG_DETERMINISTIC if deterministic else 0) |
                                  (FLAG_UNFUSED_SCATTER if unfused_scatter else 0) |
                                  (FLAG_UNMERGED_SCATTER if unmerged_scatter else 0) |
                                  (FLAG_SINGLE_FORWARD if single_forward else 0), _stream(stream)))
        return loss, g, r

    def loss_grad_noalloc(self, W, p, loss, g=None, r=None, exact=False, single_backward=False,
                          fp32_forward=False, ozaki=False, stream=None):
        """sos_loss_grad_noalloc on an unbound plan (bind=False): the outputs
        (loss, and g and r when given) are caller tensors, so the call makes
        no device allocation at all."""
        self._w(W), self._p(p)
        _check(_lib.sos_loss_grad_noalloc(self._h, _ptr(W), _ptr(p), _ptr(loss), _ptr(g), _ptr(r),
                                          (FLAG_EXACT_FORWARD if exact else 0) |
                                          (FLAG_SINGLE_BACKWARD if single_backward else 0) |
                                          (FLAG_FP32_FORWARD if fp32_forward else 0) |
                                          _oz_flags(ozaki), _stream(stream)))
        return loss, g, r

    def step(self, W, state, t, p, adam: Adam, loss=None, flags=0, stream=None):
        self._w(W), self._p(p)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=self.device)
        _check(_lib.sos_step(self._h, _ptr(W), _ptr(state), int(t), _ptr(p), ctypes.byref(adam.c()),
                             _ptr(loss), int(flags), _stream(stream)))
        return loss

    def verify(self, W, p, want_r=False, stream=None):
        self._w(W), self._p(p)
        rel = ctypes.c_double()
        r = torch.empty(self.M, dtype=torch.float64, device=self.device) if want_r else None
        _check(_lib.sos_verify(self._h, _ptr(W), _ptr(p), ctypes.byref(rel), _ptr(r), _stream(stream)))
        return (rel.value, r) if want_r else rel.value

    def timing(self, enable: bool):
        _check(_lib.sos_timing(self._h, 1 if enable else 0))

    def timing_read(self):
        """{kernel class: (total ms, launches)} since timing(True)."""
        n = len(KERNEL_CLASSES)
        ms = (ctypes.c_double * n)()
        calls = (ctypes.c_int64 * n)()
        _check(_lib.sos_timing_read(self._h, ms, calls))
        return {name: (ms[i], calls[i]) for i, name in enumerate(KERNEL_CLASSES)}

    def solve(self, W, p, adam: Adam, tol=1e-8, max_steps=10000, check_every=50, ladder=True,
              stall_checks=4, stall_ratio=0.7, switch_rel=0.0, lr_exact=0.0, rollback_ratio=0.0,
              single_backward=False, mid_rel=0.0, finisher="fp64", deterministic=False, state=None,
              single_rel=0.0, four_rel=0.0, stream=None):
        """sos_solve: Adam to an FP64-verified ||r||/||p|| <= tol; W ends as the best iterate.
        finisher: forward of the exact phase, "fp64" (FP64 MFMA), "ozaki" (six int8 slices) or
        "ozaki5" (five int8 slices).  single_rel: split plans start with the single-product
        forward until rel <= single_rel (0: off).  four_rel: with finisher "ozaki5", four slices
        until rel <= four_rel (0: off)."""
        self._w(W), self._p(p)
        state = self.new_state() if state is None else state
        fin = {"fp64": 0, "ozaki": 1, "ozaki5": 2}[finisher]
        opts = _SolveOpts(tol, max_steps, check_every, 1 if ladder else 0, stall_checks, stall_ratio,
                          switch_rel, lr_exact, rollback_ratio, 1 if single_backward else 0, fin, mid_rel,
                          FLAG_DETERMINISTIC if deterministic else 0, 0, single_rel, four_rel)
        res = _Result()
        _check(_lib.sos_solve(self._h, _ptr(W), _ptr(state), _ptr(p), ctypes.byref(adam.c()),
                              ctypes.byref(opts), ctypes.byref(res), _stream(stream)),
               allow=(OK, NOT_CONVERGED))
        return {f: getattr(res, f) for f, _ in _Result._fields_}


BATCH_MAX_N = 1024   # largest basis size N of a plan the grouped calls take


def step_batch(plans, Ws, states, ts, ps, adam: Adam, losses, stream=None):
    """sos_step_batch: one Adam step for several independent problems (serving).

    FP32 plans with N <= BATCH_MAX_N; losses[q] gets problem q's loss at the
    W before the update.  A problem's results do not depend on the others.
    """
    n = len(plans)
    for pl, W, p in zip(plans, Ws, ps):
        pl._w(W), pl._p(p)
    P = (ctypes.c_void_p * n)(*[pl._h for pl in plans])
    Wv = (ctypes.c_void_p * n)(*[W.data_ptr() for W in Ws])
    Sv = (ctypes.c_void_p * n)(*[s.data_ptr() for s in states])
    Tv = (ctypes.c_int64 * n)(*[int(t) for t in ts])
    Pv = (ctypes.c_void_p * n)(*[p.data_ptr() for p in ps])
    _check(_lib.sos_step_batch(P, Wv, Sv, Tv, Pv, ctypes.byref(adam.c()), _ptr(losses), n, _stream(stream)))
    return losses


def loss_batch(plans, Ws, ps, losses, stream=None):
    """sos_loss_batch: FP64 loss of each W_q (the serving certificate)."""
    n = len(plans)
    for pl, W, p in zip(plans, Ws, ps):
        pl._w(W), pl._p(p)
    P = (ctypes.c_void_p * n)(*[pl._h for pl in plans])
    Wv = (ctypes.c_void_p * n)(*[W.data_ptr() for W in Ws])
    Pv = (ctypes.c_void_p * n)(*[p.data_ptr() for p in ps])
    _check(_lib.sos_loss_batch(P, Wv, Pv, _ptr(losses), n, _stream(stream)))
    return losses


class Net:
    """The paper's two-layer network ||B Z A x||^2 for quartic forms in n
    variables (Section 2): weights At = A^T (n x m) and Bt = B^T (n m x k),
    FP32 on the device, trained through a plan (n - 1, 2) of rank k."""

    def __init__(self, n: int, m: int, k: int, precision="bf16x3", At=None, Bt=None, device="cuda"):
        self.n, self.m, self.k = n, m, k
        self.plan = Plan(n - 1, 2, k, precision, device=device)
        sz = ctypes.c_size_t()
        _check(_lib.sos_net_query(self.plan._h, n, m, ctypes.byref(sz)))
        self.state = torch.zeros(sz.value, dtype=torch.uint8, device=device)
        f32 = dict(dtype=torch.float32, device=device)
        self.At = torch.zeros((n, m), **f32) if At is None else At.to(**f32).contiguous()
        self.Bt = torch.zeros((n * m, k), **f32) if Bt is None else Bt.to(**f32).contiguous()
        if tuple(self.At.shape) != (n, m) or tuple(self.Bt.shape) != (n * m, k):
            raise ValueError(f"At must be ({n}, {m}) and Bt ({n * m}, {k})")

    def weights(self, stream=None):
        W = torch.empty((self.plan.N, self.k), dtype=self.plan.wdtype, device=self.At.device)
        _check(_lib.sos_net_weights(self.plan._h, self.n, self.m, _ptr(self.At), _ptr(self.Bt), _ptr(W),
                                    _ptr(self.state), _stream(stream)))
        return W

    def grad(self, p, flags=0, want_dA=True, stream=None):
        """(loss, dL/dAt or None, dL/dBt) at the current weights."""
        self.plan._p(p)
        loss = torch.empty(1, dtype=torch.float64, device=self.At.device)
        dA = torch.empty_like(self.At) if want_dA else None
        dB = torch.empty_like(self.Bt)
        _check(_lib.sos_net_grad(self.plan._h, self.n, self.m, _ptr(self.At), _ptr(self.Bt), _ptr(self.state),
                                 _ptr(p), _ptr(loss), _ptr(dA), _ptr(dB), int(flags), _stream(stream)))
        return loss, dA, dB

    def step(self, t, p, adam: Adam, loss=None, flags=0, train_first=True, stream=None):
        self.plan._p(p)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=self.At.device)
        _check(_lib.sos_net_step(self.plan._h, self.n, self.m, _ptr(self.At), _ptr(self.Bt), _ptr(self.state),
                                 int(t), _ptr(p), ctypes.byref(adam.c()), _ptr(loss), int(flags),
                                 1 if train_first else 0, _stream(stream)))
        return loss

    def solve(self, p, adam: Adam, tol=1e-8, max_steps=10000, check_every=10, ladder=True, switch_rel=3e-6,
              lr_exact=0.0, single_backward=True, train_first=True, rollback_ratio=0.0, stream=None):
        self.plan._p(p)
        opts = _SolveOpts(tol, max_steps, check_every, 1 if ladder else 0, 0, 0.0, switch_rel, lr_exact,
                          rollback_ratio, 1 if single_backward else 0, 0, 0.0)
        res = _Result()
        _check(_lib.sos_net_solve(self.plan._h, self.n, self.m, _ptr(self.At), _ptr(self.Bt), _ptr(self.state),
                                  _ptr(p), ctypes.byref(adam.c()), ctypes.byref(opts), 1 if train_first else 0,
                                  ctypes.byref(res), _stream(stream)),
               allow=(OK, NOT_CONVERGED))
        return {f: getattr(res, f) for f, _ in _Result._fields_}


class SosLoss(torch.autograd.Function):
    """L(W) = ||coeff(m_d^T W W^T m_d) - p||^2 with the hand-derived gradient 4 R W.

    The forward already produces r, so it computes the gradient in the same
    call and keeps it for backward (which scales it by the incoming grad).
    """

    @staticmethod
    def forward(ctx, W, p, plan: Plan, exact: bool = False):
        loss, g, _ = plan.loss_grad(W.detach().contiguous(), p, grad=True, exact=exact)
        ctx.save_for_backward(g)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return (grad_out.to(g.dtype) * g, None, None, None)


def rel_residual(loss: float, p_norm: float) -> float:
    return math.sqrt(max(loss, 0.0)) / (p_norm if p_norm > 0 else 1.0)

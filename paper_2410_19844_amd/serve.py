"""Serving: SOS checks of mixed (n, d) with continuous batching.

Each request runs the first-order loop of Section 3 (Adam on
L(W) = ||coeff(m_d^T W W^T m_d) - p||^2 from its own starting W) until its
FP64-verified relative residual ||r|| / ||p|| reaches ``tol`` (verdict
"sos": the returned W is the certificate, eq. basicsos), its best residual
stops improving (``stall_checks`` checks in a row without a factor
``stall_ratio``), its step budget runs out, or its loss turns non-finite
(verdict "not certified").

The server keeps every active request's W, Adam state and plan workspace
resident on the GPU.  Each iteration advances all active requests by
``check_every`` steps with grouped launches (``sos_step_batch``: one launch
per kernel type for up to 64 requests), then reads all their losses with one
device-to-host copy.  Requests that arrive meanwhile are admitted as soon as
a slot is free and their device footprint fits the HBM budget, so they join
the work already on the device instead of waiting for a batch to drain.
A request's arithmetic never depends on the other requests in its launches,
so its result is bitwise the same alone and in any mix.
"""
from __future__ import annotations

import ctypes
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import FP32, Adam, Plan, _check, _lib, _stream, sos_plan

__all__ = ["Request", "Result", "Server", "footprint", "sos_request", "motzkin_request"]


@dataclass
class Request:
    """One SOS check: is p (FP64 coefficients, library order) a sum of squares?"""
    id: int
    n: int
    d: int
    rank: int
    p: torch.Tensor              # (M,) float64 on the device
    W_init: torch.Tensor         # (N, rank) float32 on the device; not modified
    arrival: float = 0.0         # seconds after Server.run starts
    label: str | None = None     # what the generator knows ("sos", "non-sos"); not used by the server


@dataclass
class Result:
    id: int
    verdict: str                 # "sos" or "not certified"
    reason: str                  # "certified", "stalled", "budget", "nonfinite"
    rel: float                   # FP64-verified ||r|| / ||p|| of W (certificate) or best seen
    steps: int
    arrival: float
    admitted: float
    finished: float
    W: torch.Tensor | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


_SIZES: dict = {}


def footprint(n: int, d: int, rank: int) -> int:
    """Device bytes one request holds while active: plan workspace, Adam m and v,
    W, p (the plan is created on the host only, to read its sizes)."""
    key = (n, d, rank)
    if key not in _SIZES:
        h = sos_plan(n, d, rank, FP32)
        N, M = ctypes.c_int64(), ctypes.c_int64()
        ws, st = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.sos_plan_query(h, ctypes.byref(N), ctypes.byref(M), ctypes.byref(ws), ctypes.byref(st)))
        _lib.sos_plan_destroy(h)
        _SIZES[key] = (ws.value + 256) + st.value // 2 + N.value * rank * 4 + M.value * 8
    return _SIZES[key]


class _Active:
    """A request admitted to the device."""

    def __init__(self, req: Request, now: float):
        self.req = req
        self.plan = Plan(req.n, req.d, req.rank, "fp32")
        self.W = req.W_init.clone()
        self.state = torch.zeros(self.plan.state_bytes // 2, dtype=torch.uint8, device=self.W.device)
        self.t = 0
        self.pnorm = math.nan     # ||p||, set by the server's first grouped call after admission
        self.best = math.inf      # best relative residual read so far
        self.anchor = math.inf    # residual at the last drop by the stall ratio
        self.since = 0            # checks since that drop
        self.admitted = now
        self.bytes = footprint(req.n, req.d, req.rank)


class Server:
    """Continuous-batching SOS checker on one GPU.

    hbm_budget    bytes of device memory the active requests may hold
    max_active    slots (requests on the device at once)
    check_every   steps between loss reads (one device-to-host copy each)
    tol           FP64-verified relative residual that certifies "sos"
    max_steps     step budget per request
    stall_checks, stall_ratio
                  retire as "not certified" when the best relative residual
                  has not dropped below stall_ratio x its value of
                  stall_checks checks ago
    """

    def __init__(self, hbm_budget: int = 8 << 30, max_active: int = 48, check_every: int = 50,
                 tol: float = 1e-6, max_steps: int = 20000, adam: Adam | None = None,
                 stall_checks: int = 10, stall_ratio: float = 0.5, keep_W: bool = False, stream=None):
        self.hbm_budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.check_every = int(check_every)
        self.tol = float(tol)
        self.max_steps = int(max_steps)
        self.adam = adam if adam is not None else Adam(lr=3e-2)
        self.stall_checks = int(stall_checks)
        self.stall_ratio = float(stall_ratio)
        self.keep_W = keep_W
        self.stream = stream
        self.peak_bytes = 0          # largest total footprint held at once
        self.peak_active = 0
        self.iterations = 0

    # -- the grouped calls, with argument arrays rebuilt only when the active set changes
    def _bind(self, active):
        n = len(active)
        self._P = (ctypes.c_void_p * n)(*[a.plan._h for a in active])
        self._W = (ctypes.c_void_p * n)(*[a.W.data_ptr() for a in active])
        self._S = (ctypes.c_void_p * n)(*[a.state.data_ptr() for a in active])
        self._T = (ctypes.c_int64 * n)(*[a.t for a in active])
        self._p = (ctypes.c_void_p * n)(*[a.req.p.data_ptr() for a in active])
        self._n = n

    def _steps(self, active, losses, count):
        adam = ctypes.byref(self.adam.c())
        s = _stream(self.stream)
        lp = ctypes.c_void_p(losses.data_ptr())
        for _ in range(count):
            for q, a in enumerate(active):
                a.t += 1
                self._T[q] = a.t
            _check(_lib.sos_step_batch(self._P, self._W, self._S, self._T, self._p, adam, lp, self._n, s))

    def _pnorms(self, items, losses):
        """||p|| of newly admitted requests from the library's own FP64 sum of
        squares: the grouped certificate at W = 0 is ||coeff(0) - p||^2."""
        for q0 in range(0, len(items), len(losses)):
            part = items[q0:q0 + len(losses)]
            zero = [torch.zeros_like(a.W) for a in part]
            n = len(part)
            P = (ctypes.c_void_p * n)(*[a.plan._h for a in part])
            W = (ctypes.c_void_p * n)(*[z.data_ptr() for z in zero])
            p = (ctypes.c_void_p * n)(*[a.req.p.data_ptr() for a in part])
            _check(_lib.sos_loss_batch(P, W, p, ctypes.c_void_p(losses.data_ptr()), n, _stream(self.stream)))
            for a, x in zip(part, losses[:n].cpu().numpy()):
                a.pnorm = math.sqrt(max(float(x), 0.0))

    def _certify(self, items, losses):
        n = len(items)
        P = (ctypes.c_void_p * n)(*[a.plan._h for a in items])
        W = (ctypes.c_void_p * n)(*[a.W.data_ptr() for a in items])
        p = (ctypes.c_void_p * n)(*[a.req.p.data_ptr() for a in items])
        _check(_lib.sos_loss_batch(P, W, p, ctypes.c_void_p(losses.data_ptr()), n, _stream(self.stream)))
        L = losses[:n].cpu().numpy()
        return [math.sqrt(max(float(x), 0.0)) / a.pnorm if a.pnorm > 0 else math.sqrt(max(float(x), 0.0))
                for x, a in zip(L, items)]

    def run(self, requests) -> list[Result]:
        """Serve `requests` (any order; each starts at its arrival time) to completion."""
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.id)))
        dev = pending[0].p.device if pending else torch.device("cuda")
        losses = torch.empty(max(self.max_active, 1), dtype=torch.float64, device=dev)
        active: list[_Active] = []
        results: list[Result] = []
        used = 0
        t0 = time.perf_counter()
        changed = True
        while pending or active:
            now = time.perf_counter() - t0
            admitted = []
            while pending and pending[0].arrival <= now and len(active) < self.max_active:
                need = footprint(pending[0].n, pending[0].d, pending[0].rank)
                if need > self.hbm_budget:
                    raise ValueError(f"request {pending[0].id} needs {need} B, above the whole HBM budget")
                if used + need > self.hbm_budget:
                    break
                active.append(_Active(pending.popleft(), now))
                admitted.append(active[-1])
                used += active[-1].bytes
                changed = True
            if admitted:
                self._pnorms(admitted, losses)
            self.peak_bytes = max(self.peak_bytes, used)
            self.peak_active = max(self.peak_active, len(active))
            if not active:
                time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                continue
            if changed:
                self._bind(active)
                changed = False
            self._steps(active, losses, self.check_every)
            self.iterations += 1
            L = losses[:len(active)].cpu().numpy()        # one device-to-host copy per check
            done, cand = [], []
            for a, x in zip(active, L):
                x = float(x)
                if not math.isfinite(x):
                    # the loss went NaN or infinite: nothing can be certified from here
                    done.append((a, "nonfinite"))
                    continue
                rel = math.sqrt(max(x, 0.0)) / a.pnorm if a.pnorm > 0 else math.sqrt(max(x, 0.0))
                if rel <= self.tol:
                    cand.append(a)
                    continue
                a.best = min(a.best, rel)
                if rel <= self.stall_ratio * a.anchor:
                    a.anchor, a.since = rel, 0
                else:
                    a.since += 1
                if a.t >= self.max_steps:
                    done.append((a, "budget"))
                elif a.since >= self.stall_checks:
                    done.append((a, "stalled"))
            certified = []
            if cand:
                # the loss read is of the W before the last update: certify the current W
                for a, rel in zip(cand, self._certify(cand, losses)):
                    if rel <= self.tol:
                        certified.append((a, rel))
                    elif a.t >= self.max_steps:
                        done.append((a, "budget"))
            end = time.perf_counter() - t0
            for a, rel in certified:
                results.append(self._result(a, "sos", "certified", rel, end))
            for a, reason in done:
                results.append(self._result(a, "not certified", reason, a.best, end))
            gone = {id(a) for a, _ in certified} | {id(a) for a, _ in done}
            if gone:
                for a in active:
                    if id(a) in gone:
                        used -= a.bytes
                active = [a for a in active if id(a) not in gone]
                changed = True
        return sorted(results, key=lambda r: r.id)

    def _result(self, a: _Active, verdict, reason, rel, end):
        return Result(id=a.req.id, verdict=verdict, reason=reason, rel=rel, steps=a.t,
                      arrival=a.req.arrival, admitted=a.admitted, finished=end,
                      W=a.W if self.keep_W else None)


# ---------------------------------------------------------------------------
# Request construction (inputs of the serving workload)
# ---------------------------------------------------------------------------

def _coeff_of(n, d, W, device):
    """coeff(W W^T) in FP64 on the GPU (exact products of the FP32 entries)."""
    pl = Plan(n, d, W.shape[1], "fp32", device=device)
    zeros = torch.zeros(pl.M, dtype=torch.float64, device=device)
    _, _, c = pl.loss_grad(W, zeros, grad=False, want_r=True, exact=True)
    return c


def sos_request(id, n, d, rank, W0, W_init, arrival=0.0, device="cuda") -> Request:
    """p = coeff(W0 W0^T): SOS by construction (W0 rounded to FP32 first)."""
    W0 = torch.as_tensor(np.ascontiguousarray(W0), dtype=torch.float32, device=device)
    p = _coeff_of(n, d, W0, device)
    Wi = torch.as_tensor(np.ascontiguousarray(W_init), dtype=torch.float32, device=device)
    return Request(id=id, n=n, d=d, rank=rank, p=p, W_init=Wi, arrival=arrival, label="sos")


def motzkin_request(id, n, d, rank, terms, V, W_init, scale=1e-3, arrival=0.0, device="cuda") -> Request:
    """p = Motzkin form + scale * s / ||s||, s = coeff(V V^T) (a random SOS).

    `terms` lists (exponent tuple, coefficient) of the form in the first three
    variables; the Motzkin form is nonnegative but not SOS, and a perturbation
    this small keeps p outside the SOS cone."""
    pl = Plan(n, d, 1, "fp32", device="cpu")
    cexp = pl.exponents(1)
    where = {tuple(int(v) for v in row): i for i, row in enumerate(cexp)}
    m = np.zeros(len(cexp))
    for e, c in terms:
        m[where[tuple(e)]] += c
    Vt = torch.as_tensor(np.ascontiguousarray(V), dtype=torch.float32, device=device)
    s = _coeff_of(n, d, Vt, device)
    p = torch.as_tensor(m, dtype=torch.float64, device=device) + (scale / torch.linalg.vector_norm(s)) * s
    Wi = torch.as_tensor(np.ascontiguousarray(W_init), dtype=torch.float32, device=device)
    return Request(id=id, n=n, d=d, rank=rank, p=p.contiguous(), W_init=Wi, arrival=arrival, label="non-sos")

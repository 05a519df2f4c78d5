"""Continuous-batching server for VQE and noisy-TFIM requests.

The paper motivates simulators as shared infrastructure for variational
algorithms whose circuits are generated on the fly (Abstract; Sec. III VQE
and noisy TFIM).  This module serves a stream of such requests on one GPU:

* SV VQE requests (register n, ansatz depth L, energy or energy+gradient,
  several optimiser steps each with a new parameter vector and the
  request's own field h);
* DM noisy-TFIM requests (register n, the Sec. III noise model), returning
  Tr(rho Z_i), purity and trace.

Policy (host side, device-independent, tested on the CPU with a fake
executor and a virtual clock):

* admission by HBM footprint, strictly in arrival order: a request is
  admitted when its footprint fits the free budget; one larger than the whole
  budget is rejected with an error; an admitted request keeps its slot
  (its state stays resident) until its last step completes;
* continuous batching: admitted SV requests with a pending step are grouped
  by shape class (n, L, gradient or not) into one batched launch per class;
  a class launches again as soon as its previous batch completes, taking
  every request of that class that became ready meanwhile, so requests that
  arrive while others are on the GPU join the next batch of their class;
  classes run concurrently on their own streams, DM requests on worker
  threads with a stream each;
* a failing request (bad parameters) completes with an error and does not
  affect the others of its batch.

Results are deterministic per request: the batched kernels give each
parameter vector a fixed reduction order, so a request's outputs are the
same bit for bit alone or in any mix.
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import threading
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional, Tuple

import numpy as np


@dataclass
class ServeResult:
    rid: int
    kind: str
    arrival: float
    admitted: Optional[float] = None
    finished: Optional[float] = None
    outputs: List[Any] = field(default_factory=list)   # SV: [(E, grad or None)] per step; DM: [dict]
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


def sv_footprint(n: int, want_grad: bool) -> int:
    return (16 << n) * (2 if want_grad else 1)


def dm_footprint(n: int) -> int:
    return 16 << (2 * n)


class _Active:
    __slots__ = ("req", "res", "step", "thetas", "fp", "busy")

    def __init__(self, req, res, thetas, fp):
        self.req, self.res, self.thetas, self.fp = req, res, thetas, fp
        self.step = 0
        self.busy = False


class Server:
    """Event loop over an executor.  `clock()` returns seconds; `sleep(dt)`
    waits (a virtual clock advances instead in CPU tests)."""

    def __init__(self, executor, budget_bytes: int, max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 poll_s: float = 50e-6):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.clock = clock
        self.sleep = sleep
        self.poll_s = poll_s
        self.in_use = 0
        self.max_in_use = 0
        self.batches: List[Tuple[Tuple, int]] = []      # (class key, batch size) in launch order

    def footprint(self, req) -> int:
        return self.ex.footprint(req)

    def run(self, trace, time_scale: float = 1.0) -> List[ServeResult]:
        """Serve `trace` (objects with rid, arrival, kind, n, L, want_grad,
        steps, ...); arrivals are replayed against the clock (scaled)."""
        reqs = sorted(trace, key=lambda r: (r.arrival, r.rid))
        results: Dict[int, ServeResult] = {r.rid: ServeResult(r.rid, r.kind, r.arrival * time_scale) for r in reqs}
        pending = deque(reqs)
        waiting: deque = deque()
        active_sv: "OrderedDict[int, _Active]" = OrderedDict()
        inflight: Dict[Tuple, Tuple[Any, List[_Active]]] = {}
        dm_jobs: Dict[int, Tuple[Any, _Active]] = {}
        t0 = self.clock()
        done = 0
        total = len(reqs)

        def now():
            return self.clock() - t0

        def finish(a: _Active, err: Optional[str] = None):
            nonlocal done
            a.res.finished = now()
            if err is not None:
                a.res.error = err
            self.in_use -= a.fp
            done += 1

        while done < total:
            progressed = False
            t = now()
            while pending and pending[0].arrival * time_scale <= t:
                waiting.append(pending.popleft())
                progressed = True
            # admission: strict arrival order by footprint
            while waiting:
                r = waiting[0]
                res = results[r.rid]
                try:
                    fp = self.footprint(r)
                    err = self.ex.validate(r)
                except Exception as e:          # malformed request
                    fp, err = 0, str(e)
                if err is not None:
                    waiting.popleft()
                    res.admitted = t
                    res.finished = t
                    res.error = err
                    done += 1
                    progressed = True
                    continue
                if fp > self.budget:
                    waiting.popleft()
                    res.finished = t
                    res.error = f"footprint {fp} B exceeds the budget {self.budget} B"
                    done += 1
                    progressed = True
                    continue
                if self.in_use + fp > self.budget:
                    break
                waiting.popleft()
                self.in_use += fp
                self.max_in_use = max(self.max_in_use, self.in_use)
                res.admitted = t
                a = _Active(r, res, self.ex.thetas(r) if r.kind == "sv_vqe" else None, fp)
                if r.kind == "sv_vqe":
                    active_sv[r.rid] = a
                else:
                    dm_jobs[r.rid] = (self.ex.start_dm(r), a)
                progressed = True
            # launch one batch per idle class, FIFO within the class
            ready: "OrderedDict[Tuple, List[_Active]]" = OrderedDict()
            for a in active_sv.values():
                if not a.busy:
                    key = self.ex.class_key(a.req)
                    if key not in inflight:
                        lst = ready.setdefault(key, [])
                        if len(lst) < self.max_batch:
                            lst.append(a)
            for key, items in ready.items():
                for a in items:
                    a.busy = True
                token = self.ex.start_sv(key, [(a.req, a.thetas[a.step]) for a in items])
                inflight[key] = (token, items)
                self.batches.append((key, len(items)))
                progressed = True
            # completions
            for key in list(inflight):
                token, items = inflight[key]
                if self.ex.ready(token):
                    outs = self.ex.collect(token)
                    del inflight[key]
                    for a, o in zip(items, outs):
                        a.busy = False
                        if isinstance(o, Exception):
                            a.res.outputs.append(None)
                            active_sv.pop(a.req.rid, None)
                            finish(a, str(o))
                            continue
                        a.res.outputs.append(o)
                        a.step += 1
                        if a.step >= a.req.steps:
                            active_sv.pop(a.req.rid, None)
                            finish(a)
                    progressed = True
            for rid in list(dm_jobs):
                token, a = dm_jobs[rid]
                if self.ex.ready(token):
                    o = self.ex.collect(token)
                    del dm_jobs[rid]
                    if isinstance(o, Exception):
                        finish(a, str(o))
                    else:
                        a.res.outputs.append(o)
                        finish(a)
                    progressed = True
            if not progressed:
                if pending and not inflight and not dm_jobs and not active_sv and not waiting:
                    self.sleep(max(pending[0].arrival * time_scale - now(), 0.0))
                else:
                    self.sleep(self.poll_s)
        self.ex.drain()
        return [results[r.rid] for r in reqs]


def summarize(results: List[ServeResult]) -> dict:
    ok = [r for r in results if r.error is None and r.finished is not None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(0)
    span = (max(r.finished for r in ok) - min(r.arrival for r in results)) if ok else 0.0
    return {"requests": len(results), "completed": len(ok), "errors": len(results) - len(ok),
            "throughput_req_per_s": (len(ok) / span) if span > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
            "mean_ms": float(lat.mean() * 1e3) if len(lat) else None}


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------
class GpuExecutor:
    """Runs SV batches through nwq_vqe_eval_coeffs (one VQE context and one
    stream per shape class) and DM jobs through the DM engine on worker
    threads, each with its own stream."""

    def __init__(self, dm_workers: int = 4, sv_mode: int = 0):
        import torch
        import workloads as W
        from . import nwq, vqe
        self.torch, self.W, self.nwq, self.vqe = torch, W, nwq, vqe
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.ctx: Dict[Tuple[int, int], Any] = {}
        self.streams: Dict[Tuple, Any] = {}
        self.sv_mode = sv_mode
        self.pool = cf.ThreadPoolExecutor(max_workers=dm_workers)
        self._tls = threading.local()          # one stream per DM worker thread

    # --- policy hooks
    def footprint(self, r) -> int:
        return sv_footprint(r.n, r.want_grad) if r.kind == "sv_vqe" else dm_footprint(r.n)

    def validate(self, r) -> Optional[str]:
        if r.kind == "sv_vqe":
            if not (1 <= r.n <= 26) or r.L < 1 or r.steps < 1:
                return f"bad SV request n={r.n} L={r.L} steps={r.steps}"
        elif r.kind == "dm_tfim":
            if not (2 <= r.n <= 13):
                return f"bad DM request n={r.n}"
        else:
            return f"unknown request kind {r.kind}"
        return None

    def class_key(self, r) -> Tuple:
        return (r.n, r.L, bool(r.want_grad))

    def thetas(self, r) -> np.ndarray:
        return self.W.request_thetas(r, 2 * r.n * r.L)

    # --- SV batches
    def _context(self, n: int, L: int):
        c = self.ctx.get((n, L))
        if c is None:
            prog = self.W.hea_ansatz(n, L)
            terms = self.W.tfim_hamiltonian(n, 1.0, 1.0)
            with self.torch.cuda.stream(self._stream(("ctx", n, L))):
                c = self.vqe.VQE(n, prog, terms, n_params=2 * n * L, stream=self._stream(("ctx", n, L)))
            if self.sv_mode:
                c.set_config(self.sv_mode, 256 if n > 8 else 128, 0)
            self.ctx[(n, L)] = c
        return c

    def _stream(self, key):
        s = self.streams.get(key)
        if s is None:
            s = self.torch.cuda.Stream()
            self.streams[key] = s
        return s

    def start_sv(self, key, items):
        torch = self.torch
        n, L, want_grad = key
        ctx = self._context(n, L)
        s = self._stream(("ctx", n, L))
        theta = np.stack([th for _, th in items])
        coeffs = np.stack([np.array([t[2] for t in self.W.tfim_hamiltonian(n, 1.0, r.h)]) for r, _ in items])
        with torch.cuda.stream(s):
            t = torch.from_numpy(theta).to(self.dev, non_blocking=False)
            c = torch.from_numpy(coeffs).to(self.dev, non_blocking=False)
            E, G = ctx.eval_coeffs(t, c, grad=want_grad)
            ev = torch.cuda.Event()
            ev.record(s)
        return ("sv", ev, E, G, t, c)

    # --- DM jobs
    def _dm_stream(self):
        s = getattr(self._tls, "stream", None)
        if s is None:
            self.torch.cuda.set_device(self.dev)
            s = self._tls.stream = self.torch.cuda.Stream(device=self.dev)
        return s

    def _dm_job(self, r):
        torch = self.torch
        try:
            stream = self._dm_stream()
            with torch.cuda.stream(stream):
                st = self.nwq.DMState(r.n, stream=stream)
                if r.n >= 8:   # 1q superoperators as fused blocks over the 2n bits
                    st.set_fusion(12)
                st.run(self.W.noisy_tfim_circuit(r.n, r.steps))
                Z = st.expvals(self.W.single_site_terms(r.n, "Z"))
                pur = st.purity()
                tr, tri = st.trace()
                st.close()
                del st
            return {"Z": Z, "purity": pur, "trace": tr, "trace_imag": tri}
        except Exception as e:   # returned, not raised: the server records it per request
            return e

    def start_dm(self, r):
        return ("dm", self.pool.submit(self._dm_job, r))

    # --- completion
    def ready(self, token) -> bool:
        if token[0] == "sv":
            return token[1].query()
        return token[1].done()

    def collect(self, token):
        if token[0] == "sv":
            _, ev, E, G, _, _ = token
            ev.synchronize()
            e = E.cpu().numpy()
            g = G.cpu().numpy() if G is not None else None
            return [(float(e[i]), None if g is None else g[i].copy()) for i in range(len(e))]
        return token[1].result()

    def drain(self):
        self.torch.cuda.synchronize()

    def close(self):
        self.pool.shutdown(wait=True)
        for c in self.ctx.values():
            c.close()
        self.ctx.clear()

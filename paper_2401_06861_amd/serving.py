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

* admission by device memory, strictly in arrival order.  Each SV shape
  class (n, L) runs on one VQE context whose per-vector buffers grow to the
  largest batch it has served; the server charges every class the bytes its
  context will hold with all of the class's admitted requests in one batch
  (the executor asks the library, nwq_vqe_memory), and every DM request the
  bytes of its density matrix and scratch.  A request is admitted when the
  charge it adds fits the budget; if it does not, contexts of classes with
  no admitted request are freed, least recently used first; one larger than
  the whole budget is rejected with an error; an admitted request keeps its
  slot (its state stays resident) until its last step completes;
* continuous batching: admitted SV requests with a pending step are grouped
  by shape class (n, L) into one batched launch per class, energy-only and
  gradient requests together (the batch computes gradients if any member
  asked; the energies are the same bits either way, and members that did not
  ask get only the energy); a class launches again as soon as its previous
  batch completes, taking every request of that class that became ready
  meanwhile, so requests that arrive while others are on the GPU join the
  next batch of their class; classes run concurrently on their own streams,
  DM requests on worker threads with a stream each;
* a failing request (bad parameters) completes with an error and does not
  affect the others of its batch.

Results are deterministic per request: the batched kernels give each
parameter vector a fixed reduction order, so a request's outputs are the
same bit for bit alone or in any mix.
"""
from __future__ import annotations

import concurrent.futures as cf
import threading
import time
from collections import OrderedDict, defaultdict, deque
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


def sv_footprint(n: int, want_grad: bool = True) -> int:
    """Device bytes per parameter vector of the batched VQE path: the state
    phi and lambda = H phi (both are kept whether or not a gradient is asked)."""
    return 2 * (16 << n)


# scratch of a DM handle beside its 16 4^n-byte matrix: the 4 MiB upload
# ring, reduction partials and the fused-block program
DM_SCRATCH_BYTES = 8 << 20


def dm_footprint(n: int) -> int:
    return (16 << (2 * n)) + DM_SCRATCH_BYTES


class _Active:
    __slots__ = ("req", "res", "step", "thetas", "fp", "busy", "key")

    def __init__(self, req, res, thetas, fp, key=None):
        self.req, self.res, self.thetas, self.fp, self.key = req, res, thetas, fp, key
        self.step = 0
        self.busy = False


class Server:
    """Event loop over an executor.  `clock()` returns seconds; `sleep(dt)`
    waits (a virtual clock advances instead in CPU tests).  `on_tick`, if
    given, is called once per loop iteration (the GPU test samples device
    memory there)."""

    def __init__(self, executor, budget_bytes: int, max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 poll_s: float = 50e-6, on_tick: Optional[Callable[["Server"], None]] = None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.clock = clock
        self.sleep = sleep
        self.poll_s = poll_s
        self.on_tick = on_tick
        self.in_use = 0
        self.max_in_use = 0
        self.released = 0                                 # contexts freed to make room
        self.batches: List[Tuple[Tuple, int]] = []      # (class key, batch size) in launch order

    def footprint(self, req) -> int:
        return self.ex.footprint(req)

    def run(self, trace, time_scale: float = 1.0) -> List[ServeResult]:
        """Serve `trace` (objects with rid, arrival, kind, n, L, want_grad,
        steps, ...); arrivals are replayed against the clock (scaled)."""
        ex = self.ex
        reqs = sorted(trace, key=lambda r: (r.arrival, r.rid))
        results: Dict[int, ServeResult] = {r.rid: ServeResult(r.rid, r.kind, r.arrival * time_scale) for r in reqs}
        pending = deque(reqs)
        waiting: deque = deque()
        active_sv: "OrderedDict[int, _Active]" = OrderedDict()
        inflight: Dict[Tuple, Tuple[Any, List[_Active]]] = {}
        dm_jobs: Dict[int, Tuple[Any, _Active]] = {}
        # memory charged per SV class (its context) and the admitted requests per class
        class_active: Dict[Tuple, int] = defaultdict(int)
        charge: Dict[Tuple, int] = {k: ex.class_bytes(k, 0) for k in ex.classes()}
        last_used: Dict[Tuple, int] = {}
        self.in_use = sum(charge.values())
        self.max_in_use = self.in_use
        tick = 0
        t0 = self.clock()
        done = 0
        total = len(reqs)

        def now():
            return self.clock() - t0

        def set_charge(key, new):
            self.in_use += new - charge.get(key, 0)
            charge[key] = new
            self.max_in_use = max(self.max_in_use, self.in_use)

        def free_idle(need: int, keep=None):
            """Free contexts of classes with no admitted request, least
            recently used first, until `need` more bytes fit."""
            idle = [k for k in charge if class_active[k] == 0 and k not in inflight and k != keep]
            idle.sort(key=lambda k: last_used.get(k, -1))
            for k in idle:
                if self.in_use + need <= self.budget:
                    break
                ex.release(k)
                self.in_use -= charge.pop(k)
                self.released += 1

        def finish(a: _Active, err: Optional[str] = None):
            nonlocal done
            a.res.finished = now()
            if err is not None:
                a.res.error = err
            if a.key is not None:
                class_active[a.key] -= 1
                set_charge(a.key, ex.class_bytes(a.key, class_active[a.key]))
            else:
                self.in_use -= a.fp
            done += 1

        while done < total:
            progressed = False
            t = now()
            while pending and pending[0].arrival * time_scale <= t:
                waiting.append(pending.popleft())
                progressed = True
            # admission: strict arrival order by device memory
            while waiting:
                r = waiting[0]
                res = results[r.rid]
                try:
                    fp = self.footprint(r)
                    err = ex.validate(r)
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
                key = ex.class_key(r) if r.kind == "sv_vqe" else None
                if key is not None:
                    if key not in charge:       # the class's context (created now): its tables are charged
                        set_charge(key, ex.class_bytes(key, 0))
                    need = ex.class_bytes(key, class_active[key] + 1) - charge[key]
                else:
                    need = fp
                if self.in_use + need > self.budget:
                    free_idle(need, keep=key)
                    if self.in_use + need > self.budget:
                        break
                waiting.popleft()
                res.admitted = t
                if key is not None:
                    class_active[key] += 1
                    set_charge(key, charge[key] + need)
                    a = _Active(r, res, ex.thetas(r), need, key)
                    active_sv[r.rid] = a
                else:
                    self.in_use += fp
                    self.max_in_use = max(self.max_in_use, self.in_use)
                    a = _Active(r, res, None, fp)
                    dm_jobs[r.rid] = (ex.start_dm(r), a)
                progressed = True
            # launch one batch per idle class, FIFO within the class
            ready: "OrderedDict[Tuple, List[_Active]]" = OrderedDict()
            for a in active_sv.values():
                if not a.busy and a.key not in inflight:
                    lst = ready.setdefault(a.key, [])
                    if len(lst) < self.max_batch:
                        lst.append(a)
            for key, items in ready.items():
                for a in items:
                    a.busy = True
                want_grad = any(a.req.want_grad for a in items)
                token = ex.start_sv(key, [(a.req, a.thetas[a.step]) for a in items], want_grad)
                inflight[key] = (token, items)
                last_used[key] = tick
                self.batches.append((key, len(items)))
                progressed = True
            # completions
            for key in list(inflight):
                token, items = inflight[key]
                if ex.ready(token):
                    outs = ex.collect(token)
                    del inflight[key]
                    for a, o in zip(items, outs):
                        a.busy = False
                        if isinstance(o, Exception):
                            a.res.outputs.append(None)
                            active_sv.pop(a.req.rid, None)
                            finish(a, str(o))
                            continue
                        if not a.req.want_grad:
                            o = (o[0], None)
                        a.res.outputs.append(o)
                        a.step += 1
                        if a.step >= a.req.steps:
                            active_sv.pop(a.req.rid, None)
                            finish(a)
                    progressed = True
            for rid in list(dm_jobs):
                token, a = dm_jobs[rid]
                if ex.ready(token):
                    o = ex.collect(token)
                    del dm_jobs[rid]
                    if isinstance(o, Exception):
                        finish(a, str(o))
                    else:
                        a.res.outputs.append(o)
                        finish(a)
                    progressed = True
            tick += 1
            if self.on_tick is not None:
                self.on_tick(self)
            if not progressed:
                if pending and not inflight and not dm_jobs and not active_sv and not waiting:
                    self.sleep(max(pending[0].arrival * time_scale - now(), 0.0))
                else:
                    self.sleep(self.poll_s)
        ex.drain()
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


def batch_stats(batches: List[Tuple[Tuple, int]], top: int = 6) -> dict:
    """Occupancy of the batched launches: mean batch size per launch, the
    mean size seen by a served vector (sum b^2 / sum b), the largest batch,
    and per class (the `top` classes with the most vector-steps) the launch
    count and mean batch."""
    if not batches:
        return {"launches": 0}
    b = np.array([s for _, s in batches], dtype=float)
    per: Dict[Tuple, List[int]] = defaultdict(list)
    for k, s in batches:
        per[k].append(s)
    rows = sorted(per.items(), key=lambda kv: -sum(kv[1]))[:top]
    return {"launches": len(batches), "classes": len(per), "mean_batch": round(float(b.mean()), 3),
            "mean_batch_per_vector": round(float((b * b).sum() / b.sum()), 3), "max_batch": int(b.max()),
            "launches_with_2_or_more": int((b >= 2).sum()),
            "top_classes": [{"n": k[0], "L": k[1], "launches": len(v), "vector_steps": int(sum(v)),
                             "mean_batch": round(float(np.mean(v)), 2)} for k, v in rows]}


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------
class GpuExecutor:
    """Runs SV batches through nwq_vqe_eval_coeffs (one VQE context and one
    stream per shape class) and DM jobs through the DM engine on worker
    threads, each with its own stream and a density matrix the library
    allocates and frees."""

    # device bytes per class beyond what the context reports: the fused-block
    # program before it is built and the batch's theta / coefficient /
    # energy / gradient tensors
    CLASS_EXTRA_BYTES = 2 << 20

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
        """Smallest charge the request can be served with (a fresh context
        holding its vector alone); larger than the budget means rejected."""
        return sv_footprint(r.n) + self.CLASS_EXTRA_BYTES if r.kind == "sv_vqe" else dm_footprint(r.n)

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
        return (r.n, r.L)

    def thetas(self, r) -> np.ndarray:
        return self.W.request_thetas(r, 2 * r.n * r.L)

    def classes(self) -> List[Tuple]:
        return list(self.ctx)

    def class_bytes(self, key, count: int) -> int:
        """Device bytes the class's context holds while serving `count`
        vectors in one batch (at least what it holds now)."""
        _, at = self._context(*key).memory(count)
        return at + self.CLASS_EXTRA_BYTES

    def release(self, key) -> None:
        c = self.ctx.pop(key, None)
        if c is not None:
            c.close()

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

    def start_sv(self, key, items, want_grad: bool):
        torch = self.torch
        n, L = key
        ctx = self._context(n, L)
        s = self._stream(("ctx", n, L))
        # parameters and fields staged in pinned host memory, copied without blocking the loop
        theta = torch.from_numpy(np.stack([th for _, th in items])).pin_memory()
        coeffs = torch.from_numpy(np.stack([np.array([t[2] for t in self.W.tfim_hamiltonian(n, 1.0, r.h)])
                                            for r, _ in items])).pin_memory()
        with torch.cuda.stream(s):
            t = theta.to(self.dev, non_blocking=True)
            c = coeffs.to(self.dev, non_blocking=True)
            E, G = ctx.eval_coeffs(t, c, grad=want_grad)
            ev = torch.cuda.Event()
            ev.record(s)
        return ("sv", ev, E, G, t, c, theta, coeffs)

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
                st = self.nwq.DMState(r.n, stream=stream, owned=True)
                try:
                    if r.n >= 8:   # the superoperators as fused blocks over the 2n bits
                        st.set_fusion(12)
                    st.run(self.W.noisy_tfim_circuit(r.n, r.steps))
                    Z = st.expvals(self.W.single_site_terms(r.n, "Z"))
                    pur = st.purity()
                    tr, tri = st.trace()
                    held = self.nwq.nwq_memory(st.h)
                finally:
                    st.close()
            return {"Z": Z, "purity": pur, "trace": tr, "trace_imag": tri, "device_bytes": held}
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
            _, ev, E, G = token[:4]
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

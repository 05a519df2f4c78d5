#!/usr/bin/env python3
"""Benchmark of the MI355X state-vector / density-matrix hot path.

One step = one pass of the SV hot path over the deep-circuit workload:
reset to |0...0>, the depth-40 brickwork random circuit (U3 on every qubit
then CX on alternating neighbour pairs, seed 0) on n=30 qubits in
complex128 with one kernel per gate, then <Z_i> for all i in one reduction
pass.  `value` is the step's algorithmic HBM bytes (each touched amplitude
read once and written once: 32N per U3, 16N per CX since only the moved half
is touched, 16N for the reset write and the reduction read) divided by the
step time, in GB/s, with the state resident in HBM.

Extra legs, reported beside `value` (not part of it): the same circuit
through fused k-qubit LDS blocks, a per-target-qubit U3/CX sweep, the noisy
density-matrix gate at n=14, and the oracle on the host CPU.

    python bench.py [--steps K] [--warmup W] [--n 30] [--depth 40]
    python bench.py --profile-mode {trace,pmc,fused,vqe,dm}   (short runs for rocprofv3)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "30q SV gate HBM GB/s (%peak); batched VQE energy+grad evals/s; p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--depth", type=int, default=40)
    ap.add_argument("--fuse-k", type=int, default=None,
                    help="fusion width for the fused leg (default: picked by the fusion autotuner)")
    ap.add_argument("--fuse-kernel", type=int, default=1, choices=[0, 1, 2],
                    help="fused kernel with --fuse-k: 0 per-gate LDS, 1 / 2 register-blocked with 4 / 3 bits")
    ap.add_argument("--tune-depth", type=int, default=6, help="brickwork depth the fusion autotuner times")
    ap.add_argument("--no-n32", action="store_true", help="skip the n=32 sweep")
    ap.add_argument("--no-extras", action="store_true", help="only the timed step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-vqe", action="store_true", help="skip the batched VQE leg")
    ap.add_argument("--vqe-sizes", default="8:4,8:8,12:4,12:8,16:4,16:8,20:4,20:8", help="n:L pairs for the VQE leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--profile-mode", choices=["trace", "pmc", "fused", "vqe", "dm"], default=None)
    return ap.parse_args()


_T0 = time.perf_counter()


def log(*a):
    print(f"[{time.perf_counter() - _T0:7.1f}s]", *a, file=sys.stderr, flush=True)


def step_bytes(n, gates):
    N = 1 << n
    b = 16 * N + 16 * N                       # reset write + reduction read
    for name, q, _ in gates:
        b += 16 * N if name in ("cx", "swap") else 32 * N
    return b


def kernel_sha():
    h = hashlib.sha256()
    for f in ("kernels_sv.hip",):
        h.update(open(os.path.join(ROOT, "paper_2401_06861_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(name):
    """Measured HBM bytes per launch from a committed rocprofv3 --pmc summary,
    or None when missing or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_sha():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---------------------------------------------------------------- CPU leg
def host_info():
    """Core count, CPU model and RAM of the host the benchmark runs on."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["ram_GB"] = round(int(line.split()[1]) * 1024 / 1e9, 1)
                break
    except OSError:
        pass
    return info


def cpu_baseline(seconds: float, n: int = 30):
    """The oracle's C-loop tier (plain OpenMP loops, as written) applying the
    same depth-40 brickwork gates (seed 0) in order on the same n-qubit
    register from |0...0>: first with every thread OpenMP is given, then the
    following gates on one thread; each run stops after its share of
    `seconds` (at least one gate).  GB/s uses the GPU line's per-gate
    algorithmic bytes (32N per U3, 16N per CX)."""
    import workloads as W
    from oracle import loops
    gates = W.brickwork_circuit(n, 40, seed=0)
    threads = loops.get_threads()
    t0 = time.perf_counter()
    psi = loops.sv_zero(n)
    t_alloc = time.perf_counter() - t0

    def run(first, budget):
        done, byt = 0, 0
        t = time.perf_counter()
        for g in gates[first:]:
            loops.sv_apply(psi, g, n)
            done += 1
            byt += (16 if g[0] in ("cx", "swap") else 32) << n
            if time.perf_counter() - t > budget:
                break
        return done, byt, time.perf_counter() - t

    d_all, b_all, t_all = run(0, 0.6 * seconds)
    loops.set_threads(1)
    try:
        d_one, b_one, t_one = run(d_all, 0.4 * seconds)
    finally:
        loops.set_threads(threads)
    del psi
    return {"value": round(b_all / t_all / 1e9, 3), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle C-loop tier (OpenMP, {threads} threads), the first {d_all} gates of the same depth-40 "
                      f"brickwork (seed 0) on the same n={n} register (2^{n} complex128 amplitudes) from |0...0>, "
                      f"{t_all:.1f} s; then gates {d_all}-{d_all + d_one - 1} on 1 thread",
            "one_thread_GBs": round(b_one / t_one / 1e9, 3), "one_thread_gates": d_one,
            "gates_per_s": round(d_all / t_all, 3), "reset_s": round(t_alloc, 2), "host": host_info()}


# ---------------------------------------------------------------- GPU legs
def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; sharding over several GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2401_06861_amd import nwq

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    N = 1 << n
    gates = W.brickwork_circuit(n, args.depth, seed=0)
    arrays = nwq.circuit_arrays(gates)
    zterms = W.single_site_terms(n, "Z")
    stream = torch.cuda.current_stream()
    if args.profile_mode == "dm":
        # the noisy TFIM at n=14 (10 Trotter steps, one superoperator pass per
        # noisy gate, then <Z_i> and purity), twice, after the launch-shape
        # autotuner; a one-element torch kernel marks where the autotuner ends
        from paper_2401_06861_amd import autotune
        nd = 14
        dm = nwq.DMState(nd)
        autotune.tune(dm.h, reps=1, cache_path=None)
        torch.cuda.synchronize()
        torch.ones(1, dtype=torch.float64, device=dev).add_(1.0)
        torch.cuda.synchronize()
        circ = W.noisy_tfim_circuit(nd, 10)
        zt = W.single_site_terms(nd, "Z")
        for _ in range(2):
            dm.reset()
            dm.run(circ)
            dm.expvals(zt)
            dm.purity()
        torch.cuda.synchronize()
        # then the same with the superoperators queued and run as fused blocks (k=12,
        # 4 register bits), twice, after a second marker
        torch.ones(2, dtype=torch.float64, device=dev).add_(1.0)
        torch.cuda.synchronize()
        dm.set_fusion(12)
        nwq.nwq_set_fusion_kernel(dm.h, 1)
        for _ in range(2):
            dm.reset()
            dm.run(circ)
            dm.expvals(zt)
            dm.purity()
        torch.cuda.synchronize()
        dm.close()
        log("[bench] profile mode dm done")
        print(json.dumps({"profile_mode": args.profile_mode, "n": nd}))
        return
    log(f"[bench] allocating n={n} state ({16 * N / 1e9:.2f} GB)")
    psi = torch.empty(N, dtype=torch.complex128, device=dev)
    st = nwq.SVState(n, tensor=psi, stream=stream)

    if args.profile_mode == "fused":
        # the whole brickwork through fused blocks at k = --fuse-k (default 13), 4 register
        # bits, twice (nwq_run_circuit: reset, then the circuit, as the fused leg runs it)
        nwq.nwq_set_fusion(st.h, args.fuse_k or 13)
        nwq.nwq_set_fusion_kernel(st.h, 1)
        full = nwq.circuit_arrays(W.brickwork_circuit(n, args.depth, seed=0))
        for _ in range(2):
            nwq.nwq_run_circuit(st.h, *full)
        torch.cuda.synchronize()
        log(f"[bench] profile mode done: {nwq.nwq_fusion_stats(st.h)} blocks/gates per run")
        print(json.dumps({"profile_mode": args.profile_mode, "n": n}))
        return
    if args.profile_mode == "vqe":
        # fused-graph VQE energy + gradient: n=20, B=256 (64 workgroups per state, the
        # configuration the VQE autotuner picks there) and n=24, B=1 (L=8), three evaluations each
        from paper_2401_06861_amd import vqe as V
        del st, psi
        torch.cuda.empty_cache()
        for nv, B in ((20, 256), (24, 1)):
            theta, h = W.vqe_batch(nv, 8, B=B)
            ctx = V.VQE(nv, W.hea_ansatz(nv, 8), W.tfim_hamiltonian(nv, 1.0, h))
            if B == 256:
                ctx.set_config(3, 256, 64)
            t = torch.from_numpy(theta).cuda()
            for _ in range(3):
                ctx.eval(t)
            torch.cuda.synchronize()
            log(f"[bench] profile mode vqe n={nv} B={B} config {ctx.get_config()}")
            ctx.close()
        print(json.dumps({"profile_mode": args.profile_mode}))
        return
    if args.profile_mode is not None:
        # short, fixed work for rocprofv3: a plain copy of known size (counter
        # calibration), the launch-shape autotuner, then U3 and CX launches at
        # n in the tuned shapes (the last 3 x 3 U3 and 3 x 4 CX dispatches:
        # CX(3,4), then the low pairs (0,1), (1,2), (2,3))
        src = torch.empty(1 << 27, dtype=torch.complex128, device=dev)   # 2 GiB
        src.fill_(0.5)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        from paper_2401_06861_amd import autotune
        tuned = autotune.tune(st.h, reps=1, cache_path=None)      # the timed run's shapes
        log(f"[bench] profile mode launch shapes: {tuned}")
        torch.cuda.synchronize()
        reps = 3 if args.profile_mode == "pmc" else 10
        for r in range(reps):
            for q in (0, 7, n - 1):
                st.apply("u3", (q,), (0.3, 0.2, 0.1))
            st.apply("cx", (3, 4), ())
            for qs in ((0, 1), (1, 2), (2, 3)):
                st.apply("cx", qs, ())
        torch.cuda.synchronize()
        log("[bench] profile mode done")
        print(json.dumps({"profile_mode": args.profile_mode, "n": n}))
        return

    total_bytes = step_bytes(n, gates)
    from paper_2401_06861_amd import autotune
    tuned = autotune.tune(st.h, reps=2, cache_path=None)     # launch shapes for this state size
    log(f"[bench] autotuned launch shapes: {tuned}")

    def step():
        st.reset()
        nwq.nwq_apply_circuit(st.h, *arrays)
        return st.expvals(zterms)          # synchronises the stream

    for i in range(args.warmup):
        t = time.perf_counter()
        step()
        log(f"[bench] warmup {i} {time.perf_counter() - t:.2f}s")
    nwq.nwq_timing_read(st.h, reset=True)
    nwq.nwq_timing_enable(st.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log(f"[bench] step {i} done at {time.perf_counter() - t0:.2f}s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nwq.nwq_timing_enable(st.h, False)
    tim = nwq.nwq_timing_read(st.h, reset=True)
    ms_per_step = dt * 1e3 / args.steps
    value = total_bytes / (dt / args.steps) / 1e9

    cnt, ms = tim["sv_1q_dense"]
    u3_avg_ms = ms / max(cnt, 1)
    achieved = 32 * N / (u3_avg_ms * 1e-3) / 1e9
    traffic = load_traffic("sv_1q_dense_n30_pmc.md") if n == 30 else None
    roofline = {"kernel": "k_sv_1q (U3, one pass of 2^30 pairs)", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "avg_launch_ms": round(u3_avg_ms, 4), "launches": cnt}
    per_class = {k: {"launches": c, "avg_ms": round(m / c, 4)} for k, (c, m) in tim.items() if c}

    ceiling = copy_ceiling(torch, 16 * N) if not args.no_extras else None
    if ceiling:
        roofline["measured_ceiling_GBs"] = ceiling["best_GBs"]
        roofline["frac_of_measured_ceiling"] = round(achieved / ceiling["best_GBs"], 4)

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"brickwork random circuit depth {args.depth}, n={n} state vector complex128, "
                                  "one kernel per gate, then <Z_i> for all i", "n": n, "depth": args.depth,
                      "gates": len(gates), "seed": 0, "parallelism": "single GPU"},
           "pct_peak": round(value / HBM_PEAK_GBS, 4), "roofline": roofline, "kernels": per_class,
           "launch_shapes": {k: {b: {"ppt": v[0], "flags": v[1]} for b, v in per.items()}
                             for k, per in tuned.items()}}

    if ceiling:
        out["copy_ceiling"] = ceiling
    if not args.no_extras:
        out["fused"] = fused_leg(nwq, st, arrays, n, args, ms_per_step)
        out["seeds"] = seeds_leg(nwq, st, n, args, out["fused"])
        out["sweep"] = sweep_leg(nwq, st, n)
        out["measure"] = measure_leg(nwq, st, n)
        del st, psi
        torch.cuda.empty_cache()
        if n == 30 and not args.no_n32:
            out["sweep_n32"] = sweep_n32_leg(nwq, torch, tuned)
        out["dm_noisy_gate_n14"] = dm_leg(nwq, torch)
        out["dm_noisy_gate_n15"] = dm15_leg(nwq, torch)
    if not args.no_extras and not args.no_vqe:
        out["vqe"] = vqe_leg(torch)
    if not args.no_extras and not args.no_serving:
        out["serving"] = serving_leg(torch, args.serving_requests)
    if not args.no_cpu:
        log("[bench] cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out))


def copy_ceiling(torch, nbytes, reps=5):
    """Measured streaming ceilings at the state's footprint (GB/s counts the
    read and the write): the library's in-place scale and copy kernels (one
    entry per thread, non-temporal, XCD-contiguous order: the gate kernels'
    layout with no arithmetic), a device-to-device hipMemcpy, and torch's
    elementwise in-place scale."""
    from paper_2401_06861_amd import nwq
    log(f"[bench] copy ceiling at {nbytes / 1e9:.2f} GB")
    src = torch.empty(nbytes // 16, dtype=torch.complex128, device="cuda")
    src.fill_(0.5)
    dst = torch.empty_like(src)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms = {"stream_scale": timed(lambda: nwq.nwq_stream_scale(src, 1.0)),
          "stream_copy": timed(lambda: nwq.nwq_stream_copy(dst, src)),
          "hipmemcpy_d2d": timed(lambda: dst.copy_(src)),
          "torch_inplace_scale": timed(lambda: src.mul_(1.0))}
    del src, dst
    torch.cuda.empty_cache()
    gbs = {k: 2 * nbytes / (v * 1e-3) / 1e9 for k, v in ms.items()}
    best = max(gbs["stream_scale"], gbs["stream_copy"])
    return {"footprint_GB": round(nbytes / 1e9, 2), "ms": {k: round(v, 3) for k, v in ms.items()},
            "GBs": {k: round(v, 1) for k, v in gbs.items()}, "best_GBs": round(best, 1),
            "best_frac_of_spec": round(best / HBM_PEAK_GBS, 4)}


def seeds_leg(nwq, st, n, args, fused):
    """The brickwork with seeds 1 and 2 (seed 0 is the timed step): one kernel
    per gate and through fused blocks at the width and kernel the fusion
    autotuner picked, one timed run each after a warm-up."""
    import torch
    import workloads as W
    res = {}
    zterms = W.single_site_terms(n, "Z")
    for seed in (1, 2):
        log(f"[bench] brickwork seed {seed}")
        arr = nwq.circuit_arrays(W.brickwork_circuit(n, args.depth, seed=seed))
        row = {}
        for label, k in (("unfused", 0), ("fused", fused["k"])):
            nwq.nwq_set_fusion(st.h, k)
            if k:
                nwq.nwq_set_fusion_kernel(st.h, fused["kernel_id"])
            nwq.nwq_run_circuit(st.h, *arr)
            st.flush()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nwq.nwq_run_circuit(st.h, *arr)
            z = st.expvals(zterms)
            dt = time.perf_counter() - t0
            row[label + "_ms"] = round(dt * 1e3, 2)
            row[label + "_z"] = z
        nwq.nwq_set_fusion(st.h, 0)
        row["max_abs_dz_fused_vs_unfused"] = float(np.max(np.abs(row.pop("fused_z") - row.pop("unfused_z"))))
        row["unfused_GBs"] = round(step_bytes(n, W.brickwork_circuit(n, args.depth, seed=seed)) /
                                   (row["unfused_ms"] * 1e-3) / 1e9, 1)
        res[f"seed{seed}"] = row
    return res


def fused_leg(nwq, st, arrays, n, args, unfused_ms):
    """The same circuit through fused k-qubit blocks (nwq_run_circuit: reset,
    then the circuit; the first block runs only the tile holding index 0).
    The fusion width and kernel are picked by the library's fusion autotuner
    timing the first --tune-depth layers under every candidate (or fixed by
    --fuse-k)."""
    import torch
    import workloads as W
    table = None
    if args.fuse_k is None:
        log(f"[bench] fusion autotuner on depth {args.tune_depth}")
        t0 = time.perf_counter()
        k, rb, table = nwq.nwq_autotune_fusion(st.h, *nwq.circuit_arrays(W.brickwork_circuit(n, args.tune_depth, seed=0)))
        log(f"[bench] fusion autotuner picked k={k} rb={rb} in {time.perf_counter() - t0:.1f}s")
        # the three fastest candidates on the short prefix, timed once on the whole circuit
        full = {}
        for _, kk, r in sorted((v, kk, r) for (kk, r), v in table.items() if kk > 0)[:3]:
            nwq.nwq_set_fusion(st.h, kk)
            nwq.nwq_set_fusion_kernel(st.h, r)
            nwq.nwq_run_circuit(st.h, *arrays)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            nwq.nwq_run_circuit(st.h, *arrays)
            torch.cuda.synchronize()
            full[(kk, r)] = (time.perf_counter() - t1) * 1e3
        k, rb = min(full, key=full.get)
        log(f"[bench] whole-circuit check of the top three: {full} -> k={k} rb={rb}")
    else:
        k, rb = args.fuse_k, args.fuse_kernel
        nwq.nwq_set_fusion(st.h, k)
        nwq.nwq_set_fusion_kernel(st.h, rb)
    log(f"[bench] fused leg k={k} rb={rb}")
    nwq.nwq_set_fusion(st.h, k)
    nwq.nwq_set_fusion_kernel(st.h, rb)
    nwq.nwq_run_circuit(st.h, *arrays)            # warm-up (and plan): reset, then the circuit
    st.flush()
    torch.cuda.synchronize()
    reps = 2
    nwq.nwq_timing_read(st.h, reset=True)
    nwq.nwq_timing_enable(st.h, True)
    t0 = time.perf_counter()
    for _ in range(reps):
        nwq.nwq_run_circuit(st.h, *arrays)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    nwq.nwq_timing_enable(st.h, False)
    tim = nwq.nwq_timing_read(st.h, reset=True)
    blocks, fg = nwq.nwq_fusion_stats(st.h)
    phases = nwq.nwq_fusion_phases(st.h)
    nwq.nwq_set_fusion(st.h, 0)
    c, ms = tim["sv_fused"]
    N = 1 << n
    avg = ms / max(c, 1)
    kname = ["one LDS pass per gate", "register-blocked (4 register bits per phase)",
             "register-blocked (3 register bits per phase)"][rb]
    res = {"k": k, "kernel": kname, "kernel_id": rb,
           "blocks": blocks, "phases": phases, "gates": fg, "mean_gates_per_block": round(fg / max(blocks, 1), 2),
           "circuit_ms": round(dt * 1e3, 2), "speedup_vs_one_kernel_per_gate": round(unfused_ms / (dt * 1e3), 2),
           "avg_block_ms": round(avg, 3), "block_hbm_GBs": round(32 * N / (avg * 1e-3) / 1e9, 1)}
    if table is not None:
        res["autotuner"] = {"depth": args.tune_depth,
                            "ms_per_circuit": {("unfused" if kk == 0 else f"k{kk}_{nwq.FUSION_KERNELS[r]}"): round(v, 1)
                                               for (kk, r), v in sorted(table.items())},
                            "whole_circuit_ms_of_top3": {f"k{kk}_{nwq.FUSION_KERNELS[r]}": round(v, 1)
                                                         for (kk, r), v in sorted(full.items())}}
    return res


def sweep_leg(nwq, st, n):
    log("[bench] per-qubit sweep")
    import torch
    N = 1 << n
    res = {}
    for name, qs_list, bytes_per in (("u3", [(q,) for q in (0, 1, 2, 3, 5, 6, 7, 8, 9, 10, 20, n - 1)], 32 * N),
                                     ("cx", [(0, 1), (1, 2), (2, 3), (3, 4), (5, 6), (14, 15), (n - 2, n - 1)],
                                      16 * N),
                                     ("rz", [(0,), (n - 1,)], 32 * N), ("rzz", [(0, 1), (n - 2, n - 1)], 32 * N)):
        for qs in qs_list:
            p = {"u3": (0.3, 0.2, 0.1), "cx": (), "rz": (0.4,), "rzz": (0.4,)}[name]
            st.apply(name, qs, p)
            torch.cuda.synchronize()
            nwq.nwq_timing_read(st.h, reset=True)
            nwq.nwq_timing_enable(st.h, True)
            for _ in range(5):
                st.apply(name, qs, p)
            nwq.nwq_timing_enable(st.h, False)
            tim = nwq.nwq_timing_read(st.h, reset=True)
            c, ms = max(tim.values(), key=lambda v: v[0])
            avg = ms / c
            res[f"{name}{list(qs)}"] = {"ms": round(avg, 3), "GBs": round(bytes_per / (avg * 1e-3) / 1e9, 1)}
    return res


def measure_leg(nwq, st, n, shots=1 << 20):
    """Outcome probabilities of the final brickwork state, readout noise with
    per-qubit confusion (P(1|0) = 1%, P(0|1) = 2%), and shot sampling."""
    import torch
    import workloads as W
    log("[bench] measurement leg")
    N = 1 << n
    st.reset()
    nwq.nwq_apply_circuit(st.h, *nwq.circuit_arrays(W.brickwork_circuit(n, 4, seed=0)))
    p = torch.empty(N, dtype=torch.float64, device="cuda")
    work = torch.empty(nwq.nwq_sample_workspace_bytes(n) // 8, dtype=torch.int64, device="cuda")
    u = torch.rand(shots, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    outs = torch.empty(shots, dtype=torch.int64, device="cuda")
    conf = [[[0.99, 0.02], [0.01, 0.98]]] * n

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    tp = timed(lambda: nwq.nwq_probabilities(st.h, p))
    tr = timed(lambda: nwq.nwq_readout_noise(n, p, conf), reps=1)
    ts = timed(lambda: nwq.nwq_sample(n, p, u, outs, work))
    passes = (n + 4) // 5   # up to five qubits per pass
    return {"n": n, "shots": shots,
            "probabilities_ms": round(tp * 1e3, 3), "probabilities_GBs": round(24 * N / tp / 1e9, 1),
            "readout_ms": round(tr * 1e3, 3), "readout_passes": passes,
            "readout_GBs": round(16 * N * passes / tr / 1e9, 1),
            "sample_ms": round(ts * 1e3, 3), "sample_scan_GBs": round(24 * N / ts / 1e9, 1),
            "shots_per_s": round(shots / ts, 1)}


def sweep_n32_leg(nwq, torch, tuned):
    """Per-target U3 and CX launches on a 32-qubit state (68.7 GB), with the
    launch shapes tuned at 30 qubits."""
    log("[bench] n=32 sweep")
    from paper_2401_06861_amd import autotune
    n = 32
    N = 1 << n
    st = nwq.SVState(n)
    for name, per in tuned.items():
        for bname, v in per.items():
            nwq.nwq_set_launch(st.h, autotune.CLASS_IDS[name], nwq.LAUNCH_BUCKETS.index(bname), v[0], v[1])
    res = {}
    for name, qs_list, bytes_per in (("u3", [(q,) for q in (0, 5, 6, 16, n - 1)], 32 * N),
                                     ("cx", [(0, 1), (n - 2, n - 1)], 16 * N)):
        for qs in qs_list:
            p = (0.3, 0.2, 0.1) if name == "u3" else ()
            st.apply(name, qs, p)
            torch.cuda.synchronize()
            nwq.nwq_timing_read(st.h, reset=True)
            nwq.nwq_timing_enable(st.h, True)
            for _ in range(3):
                st.apply(name, qs, p)
            nwq.nwq_timing_enable(st.h, False)
            c, ms = max(nwq.nwq_timing_read(st.h, reset=True).values(), key=lambda v: v[0])
            avg = ms / c
            res[f"{name}{list(qs)}"] = {"ms": round(avg, 3), "GBs": round(bytes_per / (avg * 1e-3) / 1e9, 1)}
    st.close()
    torch.cuda.empty_cache()
    return res


def noisy_gate_ops(label, qs):
    """One noisy gate of the DM sweeps: 1q: U3 + depolarising + amplitude and
    phase damping (one 4x4 superoperator); 2q: RZZ + two-qubit depolarising (a
    Pauli-pattern 16x16: coherences scaled, populations mixed); 2q_cx: CX +
    two-qubit depolarising (a dense 16x16)."""
    if label == "1q":
        return [("u3", qs, (0.3, 0.2, 0.1)), ("depolarize", qs, (1e-3,)), ("amp_damp", qs, (1e-3,)),
                ("phase_damp", qs, (2e-3,))]
    gate = ("rzz", qs, (0.2,)) if label == "2q" else ("cx", qs, ())
    return [gate, ("depolarize2", qs, (1e-2,))]


def dm_leg(nwq, torch):
    log("[bench] DM n=14 noisy gate leg")
    from paper_2401_06861_amd import autotune
    n = 14
    st = nwq.DMState(n)
    tuned = autotune.tune(st.h, reps=2, cache_path=None)
    nbytes = 32 * (1 << (2 * n))
    out = {}
    for label, ops, cls in (("1q_u3_dep_ad_pd", [("u3", (3,), (0.3, 0.2, 0.1)), ("depolarize", (3,), (1e-3,)),
                                                 ("amp_damp", (3,), (1e-3,)), ("phase_damp", (3,), (2e-3,))],
                             "dm_superop_1q"),
                            ("2q_rzz_dep2", [("rzz", (3, 4), (0.2,)), ("depolarize2", (3, 4), (1e-2,))], "dm_superop_2q")):
        st.run(ops)
        st.flush()
        torch.cuda.synchronize()
        nwq.nwq_timing_read(st.h, reset=True)
        nwq.nwq_timing_enable(st.h, True)
        for _ in range(5):
            st.run(ops)
            st.flush()
        nwq.nwq_timing_enable(st.h, False)
        c, ms = nwq.nwq_timing_read(st.h, reset=True)[cls]
        avg = ms / max(c, 1)
        out[label] = {"ms": round(avg, 3), "GBs": round(nbytes / (avg * 1e-3) / 1e9, 1)}
    # per-qubit sweep: each noisy gate on low, middle and high qubits (row and column bits q, q+n)
    sweep = {}
    for label, qs_list, cls in (("1q", [(0,), (1,), (2,), (7,), (n - 1,)], "dm_superop_1q"),
                                ("2q", [(0, 1), (2, 3), (6, 7), (n - 2, n - 1)], "dm_superop_2q"),
                                ("2q_cx", [(0, 1), (2, 3), (6, 7)], "dm_superop_2q")):
        for qs in qs_list:
            ops = noisy_gate_ops(label, qs)
            st.run(ops)
            st.flush()
            torch.cuda.synchronize()
            nwq.nwq_timing_read(st.h, reset=True)
            nwq.nwq_timing_enable(st.h, True)
            for _ in range(3):
                st.run(ops)
                st.flush()
            nwq.nwq_timing_enable(st.h, False)
            c, ms = nwq.nwq_timing_read(st.h, reset=True)[cls]
            avg = ms / max(c, 1)
            sweep[f"{label}{list(qs)}"] = {"ms": round(avg, 3), "GBs": round(nbytes / (avg * 1e-3) / 1e9, 1)}
    out["sweep"] = sweep
    # the whole noisy TFIM workload at n=14: 10 Trotter steps, each gate followed by its
    # channels (one superoperator pass per noisy gate), then Tr(rho Z_i), purity and trace
    import workloads as W
    circ = W.noisy_tfim_circuit(n, 10)
    zterms = W.single_site_terms(n, "Z")

    def run_all():
        st.reset()
        st.run(circ)
        z = st.expvals(zterms)
        return z, st.purity(), st.trace()

    run_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z, pur, tr = run_all()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gates = sum(1 for g in circ if g[0] in W.GATE_ARITY)
    out["tfim_n14_10_steps"] = {"ms": round(dt * 1e3, 2), "noisy_gate_passes": gates,
                                "GBs": round(gates * nbytes / dt / 1e9, 1), "purity": pur,
                                "trace_re": tr[0], "z0": float(z[0])}
    # the same with the superoperators (1q 4x4 and 2q 16x16) queued and run as fused blocks over the 28 bits
    fused = {}
    for k in (10, 12):
        st.set_fusion(k)
        nwq.nwq_set_fusion_kernel(st.h, 1)
        run_all()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        zf, purf, _ = run_all()
        torch.cuda.synchronize()
        dtf = time.perf_counter() - t0
        fused[f"k{k}"] = {"ms": round(dtf * 1e3, 2), "max_abs_dz_vs_unfused": float(np.max(np.abs(zf - z))),
                          "dpurity": abs(purf - pur)}
    st.set_fusion(0)
    out["tfim_n14_10_steps_fused"] = fused
    out["launch_shapes"] = {k: {b: {"ppt": v[0], "flags": v[1]} for b, v in per.items()}
                            for k, per in tuned.items()}
    st.close()
    return out


def dm15_leg(nwq, torch):
    """Noisy-gate sweep on a 15-qubit density matrix (17.18 GB, the footprint
    of the 30-qubit state vector) after the launch-shape autotuner."""
    log("[bench] DM n=15 noisy gate sweep")
    from paper_2401_06861_amd import autotune
    n = 15
    st = nwq.DMState(n)
    autotune.tune(st.h, reps=2, cache_path=None)
    nbytes = 32 * (1 << (2 * n))
    sweep = {}
    for label, qs_list, cls in (("1q", [(0,), (3,), (7,), (n - 1,)], "dm_superop_1q"),
                                ("2q", [(0, 1), (2, 3), (6, 7), (n - 2, n - 1)], "dm_superop_2q"),
                                ("2q_cx", [(0, 1), (2, 3), (6, 7)], "dm_superop_2q")):
        for qs in qs_list:
            ops = noisy_gate_ops(label, qs)
            st.run(ops)
            st.flush()
            torch.cuda.synchronize()
            nwq.nwq_timing_read(st.h, reset=True)
            nwq.nwq_timing_enable(st.h, True)
            for _ in range(3):
                st.run(ops)
                st.flush()
            nwq.nwq_timing_enable(st.h, False)
            c, ms = nwq.nwq_timing_read(st.h, reset=True)[cls]
            avg = ms / max(c, 1)
            sweep[f"{label}{list(qs)}"] = {"ms": round(avg, 3), "GBs": round(nbytes / (avg * 1e-3) / 1e9, 1)}
    st.close()
    torch.cuda.empty_cache()
    return {"n": n, "state_GB": round(16 * (1 << (2 * n)) / 1e9, 2), "sweep": sweep}


def vqe_leg(torch, sizes=None, B=256):
    """Energy + full adjoint gradient for B parameter vectors on the batched
    path (autotuned) against the plain per-circuit path (one vector at a time,
    one kernel per gate, no graph)."""
    import workloads as W
    from paper_2401_06861_amd import vqe as V
    sizes = sizes or [tuple(int(x) for x in p.split(":")) for p in parse().vqe_sizes.split(",")]
    res = {}
    for n, L in sizes:
        log(f"[bench] vqe n={n} L={L}")
        prog = W.hea_ansatz(n, L)
        theta, h = W.vqe_batch(n, L, B=B)
        ctx = V.VQE(n, prog, W.tfim_hamiltonian(n, 1.0, h))
        t = torch.from_numpy(theta).cuda()
        tune_B = B if n <= 16 else 32
        ctx.autotune(tune_B)
        cfg = ctx.get_config()
        E, G = ctx.eval(t)
        torch.cuda.synchronize()
        reps = 3 if n <= 16 else 1
        t0 = time.perf_counter()
        for _ in range(reps):
            E, G = ctx.eval(t)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        k = 16 if n <= 12 else 4
        Es = []
        ctx.eval_single(t[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(k):
            e1, g1 = ctx.eval_single(t[b])
            Es.append(e1)
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t0) / k
        dE = max(abs(Es[b].item() - E[b].item()) for b in range(k))
        dG = float(torch.max(torch.abs(g1[0] - G[k - 1])).item())
        per_gate = None
        if n > 12:     # the unfused batched schedule, for comparison with the chosen one
            ctx.set_config(2, cfg[1], 0)
            ctx.eval(t)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.eval(t)
            torch.cuda.synchronize()
            per_gate = round(B / (time.perf_counter() - t0), 1)
            ctx.set_config(*cfg)
        res[f"n{n}_L{L}"] = {"B": B, "batched_evals_per_s": round(B / tb, 1), "batched_ms": round(tb * 1e3, 3),
                             "single_evals_per_s": round(1.0 / ts, 1), "speedup": round(ts * B / tb, 2),
                             "config": {"mode": ["auto", "lds", "per_gate_graph", "fused_graph"][cfg[0]],
                                        "threads": cfg[1], "blocks_per_state": cfg[2]},
                             "per_gate_graph_evals_per_s": per_gate,
                             "max_abs_dE_batched_vs_single": dE, "max_abs_dgrad": dG}
        ctx.close()
        del t, E, G
        torch.cuda.empty_cache()
    return res


def serving_leg(torch, num, num_side=600):
    """Continuous-batching server on a Poisson stream: 70% SV VQE (n 10..24,
    L 4..8, half with gradient, 1..20 optimiser steps with the state resident
    between them), 30% noisy DM TFIM (n 6..12, 10 Trotter steps).  First all
    `num` requests arrive at once (saturation throughput), then Poisson
    arrivals at 0.8 x that rate (`num` requests, the reported latency) and at
    0.5 and 0.95 x (`num_side` requests each).  Admission is by the device
    memory the library reports for each class's context; the budget is 64 GiB."""
    import workloads as W
    from paper_2401_06861_amd.serving import GpuExecutor, Server, batch_stats, summarize
    log(f"[bench] serving leg, {num} requests (saturation and 0.8 load), {num_side} at 0.5 and 0.95")
    kw = dict(seed=7, sv_n=(10, 24), dm_n=(6, 12), L_range=(4, 8), opt_steps=(1, 20), dm_steps=10)
    ex = GpuExecutor()
    budget = 64 << 30
    warm = W.serving_trace(rate=1e9, **{**kw, "num": 60, "seed": 8})
    Server(ex, budget).run(warm)                       # contexts, graphs, allocator warm
    t0 = time.perf_counter()
    srv = Server(ex, budget)
    sat = summarize(srv.run(W.serving_trace(rate=1e9, num=num, **kw)))
    sat_batches = batch_stats(srv.batches)
    log(f"[bench] saturation {sat['throughput_req_per_s']:.1f} req/s in {time.perf_counter() - t0:.1f}s")
    loads = {}
    main = None
    for frac in (0.8, 0.5, 0.95):
        rate = frac * sat["throughput_req_per_s"]
        cnt = num if frac == 0.8 else num_side
        srv = Server(ex, budget)
        lat = summarize(srv.run(W.serving_trace(rate=rate, num=cnt, **kw)))
        log(f"[bench] load {frac} ({cnt} requests): p50 {lat['p50_ms']:.1f} ms p99 {lat['p99_ms']:.1f} ms")
        loads[str(frac)] = {"requests": cnt, "offered_req_per_s": round(rate, 2),
                            "throughput_req_per_s": round(lat["throughput_req_per_s"], 2),
                            "p50_ms": round(lat["p50_ms"], 2), "p99_ms": round(lat["p99_ms"], 2),
                            "batches": batch_stats(srv.batches), "max_charged_GB": round(srv.max_in_use / 1e9, 2),
                            "contexts_released": srv.released, "errors": lat["errors"]}
        if frac == 0.8:
            main = loads[str(frac)]
    # one shape class: the same loop on a stream of n=20, L=8 VQE requests (half with gradient,
    # 1-20 optimiser steps), where arrivals do overlap in flight
    kw1 = dict(seed=9, sv_frac=1.0, sv_n=(20, 20), L_range=(8, 8), opt_steps=(1, 20))
    srv = Server(ex, budget)
    sat1 = summarize(srv.run(W.serving_trace(rate=1e9, num=400, **kw1)))
    rate1 = 0.8 * sat1["throughput_req_per_s"]
    srv = Server(ex, budget)
    lat1 = summarize(srv.run(W.serving_trace(rate=rate1, num=400, **kw1)))
    log(f"[bench] single class n=20 L=8: saturation {sat1['throughput_req_per_s']:.1f} req/s, "
        f"0.8 load p50 {lat1['p50_ms']:.1f} ms p99 {lat1['p99_ms']:.1f} ms")
    single = {"requests": 400, "mix": "SV VQE n=20 L=8 only (half +grad, 1-20 steps)",
              "saturation_req_per_s": round(sat1["throughput_req_per_s"], 2), "offered_req_per_s": round(rate1, 2),
              "throughput_req_per_s": round(lat1["throughput_req_per_s"], 2), "p50_ms": round(lat1["p50_ms"], 2),
              "p99_ms": round(lat1["p99_ms"], 2), "batches": batch_stats(srv.batches, top=1),
              "errors": lat1["errors"]}
    ex.close()
    torch.cuda.empty_cache()
    return {"requests": num, "mix": "70% SV VQE n10-24 L4-8 (half +grad, 1-20 steps), 30% DM TFIM n6-12",
            "single_class_0.8": single,
            "budget_GB": budget / 1e9, "saturation_req_per_s": round(sat["throughput_req_per_s"], 2),
            "saturation_batches": sat_batches,
            "offered_req_per_s": main["offered_req_per_s"], "throughput_req_per_s": main["throughput_req_per_s"],
            "p50_ms": main["p50_ms"], "p99_ms": main["p99_ms"], "errors": main["errors"], "by_load": loads}


if __name__ == "__main__":
    main()

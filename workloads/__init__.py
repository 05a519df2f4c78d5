"""Seeded synthetic inputs shared by the CPU oracle and the HIP engine.

This module only produces *inputs*: gate lists (name, qubits, params), noise
specifications, parameter batches, Pauli-sum Hamiltonians as (x, z, coeff)
triples, random normalised states and request traces.  It contains none of
the simulation arithmetic (no gate matrices, no state updates, no
expectation values), so that the oracle and the engine, which both read
these inputs, share no code beyond the inputs themselves.

Workloads follow the experiments of the paper:

* Transverse-field Ising (TFIM) time evolution of a spin chain from the
  all-up state, as used for the magnetisation curve (Sec. III, Fig. 3), as a
  first-order Trotter circuit.
* The same circuit with a device-style noise model made of depolarising and
  thermal-relaxation (amplitude + phase damping) channels (Sec. III).
* A brickwork random circuit for deep-circuit throughput (Sec. III, the
  QASMBench-style throughput experiment of Fig. 5; the suite itself is not
  used, a seeded random circuit of the same gate mix stands in).
* A hardware-efficient VQE ansatz for the Ising model (Sec. III, Fig. 4).
* A Poisson request stream mixing VQE and noisy TFIM evaluations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

Gate = Tuple[str, Tuple[int, ...], Tuple[float, ...]]

# Gate names understood by both sides, with (number of qubits, number of params).
GATE_ARITY = {
    "id": (1, 0), "x": (1, 0), "y": (1, 0), "z": (1, 0), "h": (1, 0),
    "s": (1, 0), "sdg": (1, 0), "t": (1, 0), "tdg": (1, 0),
    "rx": (1, 1), "ry": (1, 1), "rz": (1, 1), "u3": (1, 3),
    "cx": (2, 0), "cz": (2, 0), "swap": (2, 0), "rzz": (2, 1),
}
# Channel names: (number of qubits, number of params).
CHANNEL_ARITY = {
    "depolarize": (1, 1), "amp_damp": (1, 1), "phase_damp": (1, 1),
    "depolarize2": (2, 1), "depolarize_nc": (1, 1), "depolarize2_nc": (2, 1),
    "thermal_relax": (1, 3),   # (T1, T2, duration), T2 <= 2 T1
}


# --------------------------------------------------------------------------
# TFIM Trotter circuit (Sec. III, Fig. 3 setting)
# --------------------------------------------------------------------------
def tfim_trotter_circuit(n: int, J: float = 1.0, h: float = 1.0,
                         dt: float = 0.1, steps: int = 20) -> List[Gate]:
    """First-order Trotter circuit of the open-chain TFIM.

    Each step applies RZZ(2*J*dt) on neighbour pairs (0,1), (1,2), ...,
    (n-2,n-1) in that order, then RX(2*h*dt) on qubits 0..n-1 in order.
    """
    gates: List[Gate] = []
    for _ in range(steps):
        for i in range(n - 1):
            gates.append(("rzz", (i, i + 1), (2.0 * J * dt,)))
        for i in range(n):
            gates.append(("rx", (i,), (2.0 * h * dt,)))
    return gates


@dataclass(frozen=True)
class NoiseSpec:
    """Device-style noise applied after every gate (Sec. III noise model).

    After a 1-qubit gate: depolarising p1, then amplitude damping gamma,
    then phase damping lam.  After a 2-qubit gate: 2-qubit depolarising p2.
    """
    p1: float = 1e-3
    gamma: float = 1e-3
    lam: float = 2e-3
    p2: float = 1e-2


def with_noise(gates: Sequence[Gate], noise: NoiseSpec) -> List[Gate]:
    """Interleave the channels of `noise` after each gate of `gates`."""
    out: List[Gate] = []
    for g in gates:
        out.append(g)
        q = g[1]
        if len(q) == 1:
            out.append(("depolarize", q, (noise.p1,)))
            out.append(("amp_damp", q, (noise.gamma,)))
            out.append(("phase_damp", q, (noise.lam,)))
        else:
            out.append(("depolarize2", q, (noise.p2,)))
    return out


def noisy_tfim_circuit(n: int, steps: int = 10, J: float = 1.0, h: float = 1.0,
                       dt: float = 0.1, noise: NoiseSpec = NoiseSpec()) -> List[Gate]:
    return with_noise(tfim_trotter_circuit(n, J, h, dt, steps), noise)


# --------------------------------------------------------------------------
# Brickwork random circuit (deep-circuit throughput)
# --------------------------------------------------------------------------
def brickwork_circuit(n: int, depth: int = 40, seed: int = 0) -> List[Gate]:
    """Layer l applies U3 with angles ~U[0, 2pi) on qubits 0..n-1, then CX on
    (2i, 2i+1) for even l or (2i+1, 2i+2) for odd l (control = lower index).
    Angles are drawn once as uniform(0, 2pi, size=(depth, n, 3)) in order
    (theta, phi, lambda)."""
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, 2.0 * math.pi, size=(depth, n, 3))
    gates: List[Gate] = []
    for l in range(depth):
        for q in range(n):
            gates.append(("u3", (q,), tuple(float(a) for a in ang[l, q])))
        start = 0 if l % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            gates.append(("cx", (a, a + 1), ()))
    return gates


def random_u3_angles(count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * math.pi, size=(count, 3))


def random_state(n: int, seed: int = 0) -> np.ndarray:
    """Normalised complex128 state with i.i.d. Gaussian amplitudes."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v /= np.sqrt(np.vdot(v, v).real)
    return v.astype(np.complex128)


def random_density_matrix(n: int, seed: int = 0, rank: int = 3) -> np.ndarray:
    """Random mixed state sum_k w_k |v_k><v_k| with Gaussian vectors (for
    tests of single noisy gates on a generic input)."""
    rng = np.random.default_rng(seed)
    d = 1 << n
    rho = np.zeros((d, d), dtype=np.complex128)
    w = rng.uniform(0.2, 1.0, size=rank)
    w /= w.sum()
    for k in range(rank):
        v = rng.standard_normal(d) + 1j * rng.standard_normal(d)
        v /= np.linalg.norm(v)
        rho += w[k] * np.outer(v, v.conj())
    return rho


def random_gate_list(n: int, count: int, seed: int) -> List[Gate]:
    """Random mix of every gate kind on random qubits (parity sweeps)."""
    rng = np.random.default_rng(seed)
    names = sorted(GATE_ARITY)
    gates: List[Gate] = []
    for _ in range(count):
        name = names[rng.integers(len(names))]
        nq, npar = GATE_ARITY[name]
        if nq > n:
            continue
        qs = tuple(int(x) for x in rng.choice(n, size=nq, replace=False))
        ps = tuple(float(x) for x in rng.uniform(-math.pi, math.pi, size=npar))
        gates.append((name, qs, ps))
    return gates


def qasm_text(gates: List[Gate], n: int, split: int = 0, seed: int = 0) -> str:
    """An OpenQASM 2.0 program for a gate list on n qubits.  With split > 0
    the qubits are declared as two registers a[split], b[n - split] (qubit q
    is a[q] below split, b[q - split] above).  Angles are written as exact
    decimal literals, some as multiples of pi, some with a unary minus or
    parentheses, and comments, barriers and measurements are sprinkled in,
    so a reader sees the syntax it has to accept."""
    rng = np.random.default_rng(seed)
    if split:
        def ref(q):
            return f"a[{q}]" if q < split else f"b[{q - split}]"
        decl = [f"qreg a[{split}];", f"qreg b[{n - split}];", f"creg c[{n}];"]
    else:
        def ref(q):
            return f"q[{q}]"
        decl = [f"qreg q[{n}];", f"creg c[{n}];"]
    lines = ["// generated", "OPENQASM 2.0;", 'include "qelib1.inc";'] + decl
    for i, (name, qs, ps) in enumerate(gates):
        args = []
        for x in ps:
            style = rng.integers(4)
            if style == 0:
                args.append(repr(float(x)))
            elif style == 1:
                args.append(f"({float(x)!r})")
            elif style == 2:
                args.append(f"{float(x) / math.pi!r}*pi")
            else:
                args.append(f"-({-float(x)!r})")
        head = name + (f"({', '.join(args)})" if args else "")
        lines.append(f"{head} {', '.join(ref(q) for q in qs)};")
        if i % 7 == 3:
            lines.append(f"barrier {ref(qs[0])};  // a barrier")
    lines.append("measure " + ref(0) + " -> c[0];")
    return "\n".join(lines) + "\n"


# --------------------------------------------------------------------------
# Pauli sums: (xmask, zmask, coeff); qubit q is bit q.
# --------------------------------------------------------------------------
PauliTerm = Tuple[int, int, float]


def pauli_term(ops: dict, coeff: float = 1.0) -> PauliTerm:
    """ops maps qubit -> 'X' | 'Y' | 'Z'."""
    x = z = 0
    for q, p in ops.items():
        if p in ("X", "Y"):
            x |= 1 << q
        if p in ("Z", "Y"):
            z |= 1 << q
    return (x, z, float(coeff))


def tfim_hamiltonian(n: int, J: float = 1.0, h=1.0) -> List[PauliTerm]:
    """H = -J sum_{i<n-1} Z_i Z_{i+1} - sum_i h_i X_i (open chain)."""
    hs = np.broadcast_to(np.asarray(h, dtype=float), (n,))
    terms = [pauli_term({i: "Z", i + 1: "Z"}, -J) for i in range(n - 1)]
    terms += [pauli_term({i: "X"}, -float(hs[i])) for i in range(n)]
    return terms


def single_site_terms(n: int, op: str) -> List[PauliTerm]:
    return [pauli_term({i: op}, 1.0) for i in range(n)]


def random_pauli_sum(n: int, count: int, seed: int) -> List[PauliTerm]:
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(count):
        x = int(rng.integers(0, 1 << n))
        z = int(rng.integers(0, 1 << n))
        terms.append((x, z, float(rng.uniform(-1, 1))))
    return terms


# --------------------------------------------------------------------------
# VQE: hardware-efficient ansatz program with parameter slots (Sec. III, Fig. 4)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class AnsatzGate:
    name: str              # 'ry' | 'rz' | 'rx' | 'cx' | ...
    qubits: Tuple[int, ...]
    param: int             # index into theta, or -1 for a fixed gate


def hea_ansatz(n: int, L: int) -> List[AnsatzGate]:
    """L layers of RY on 0..n-1, RZ on 0..n-1, then CX(0,1), ..., CX(n-2,n-1).
    Parameters are layer-major: RY block then RZ block (P = 2 n L)."""
    prog: List[AnsatzGate] = []
    for l in range(L):
        for q in range(n):
            prog.append(AnsatzGate("ry", (q,), l * 2 * n + q))
        for q in range(n):
            prog.append(AnsatzGate("rz", (q,), l * 2 * n + n + q))
        for q in range(n - 1):
            prog.append(AnsatzGate("cx", (q, q + 1), -1))
    return prog


def ansatz_num_params(prog: Sequence[AnsatzGate]) -> int:
    return 1 + max((g.param for g in prog), default=-1)


def bind_ansatz(prog: Sequence[AnsatzGate], theta: np.ndarray) -> List[Gate]:
    """Gate list of the ansatz with parameters substituted."""
    out: List[Gate] = []
    for g in prog:
        ps = (float(theta[g.param]),) if g.param >= 0 else ()
        out.append((g.name, g.qubits, ps))
    return out


def vqe_batch(n: int, L: int, B: int = 256, seed: int | None = None):
    """theta ~ U(-pi, pi) of shape (B, 2nL) and one field h ~ U[0.5, 1.5]
    shared by the batch, seeded by 1000 + 10 n + L unless given."""
    if seed is None:
        seed = 1000 + n * 10 + L
    rng = np.random.default_rng(seed)
    h = float(rng.uniform(0.5, 1.5))
    theta = rng.uniform(-math.pi, math.pi, size=(B, 2 * n * L))
    return theta, h


# --------------------------------------------------------------------------
# Serving request stream
# --------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival: float            # seconds from stream start
    kind: str                 # 'sv_vqe' | 'dm_tfim'
    n: int
    L: int = 0
    want_grad: bool = False
    steps: int = 1            # sv_vqe: optimiser steps (new theta each); dm_tfim: Trotter steps
    seed: int = 0
    h: float = 1.0
    extra: dict = field(default_factory=dict)


def serving_trace(num: int = 2000, rate: float = 100.0, seed: int = 7,
                  sv_frac: float = 0.7, sv_n=(10, 24), dm_n=(6, 12),
                  L_range=(4, 8), opt_steps=(1, 20), dm_steps: int = 10) -> List[Request]:
    """Poisson arrivals at `rate` per second of a request mix.  `steps` is the
    number of optimiser steps of an SV request and the number of Trotter
    steps of a DM request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out: List[Request] = []
    for i in range(num):
        t += float(rng.exponential(1.0 / rate))
        if rng.uniform() < sv_frac:
            r = Request(i, t, "sv_vqe", int(rng.integers(sv_n[0], sv_n[1] + 1)),
                        L=int(rng.integers(L_range[0], L_range[1] + 1)),
                        want_grad=bool(rng.uniform() < 0.5),
                        steps=int(rng.integers(opt_steps[0], opt_steps[1] + 1)),
                        seed=int(rng.integers(1 << 31)),
                        h=float(rng.uniform(0.5, 1.5)))
        else:
            r = Request(i, t, "dm_tfim", int(rng.integers(dm_n[0], dm_n[1] + 1)), steps=dm_steps,
                        seed=int(rng.integers(1 << 31)))
        out.append(r)
    return out


def request_thetas(req: Request, P: int) -> np.ndarray:
    """Parameter vectors of the successive optimiser steps of one request."""
    rng = np.random.default_rng(req.seed)
    return rng.uniform(-math.pi, math.pi, size=(req.steps, P))

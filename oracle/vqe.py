"""VQE energy and gradients.  (Test infrastructure only.)

The VQE experiment of Sec. III (Fig. 4) evaluates E(theta) = <psi(theta)| H
|psi(theta)> for a parametrised circuit.  Gradients are given here in two
independent ways:

* parameter shift (exact for gates exp(-i theta P / 2)):
  dE/dtheta_k = [E(theta + pi/2 e_k) - E(theta - pi/2 e_k)] / 2,
  applied per gate occurrence so shared parameters are summed;
* central finite differences with step h.

The circuit is simulated with tier 0 (dense) for n <= 6, tier 1 as tensor
contractions (pinned to tier 0) up to n = 12, and tier 1 as C loops (pinned to
tiers 0 and 1) above.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from . import dense, loops, tensor


DENSE_MAX_N = 6    # tier 0 up to here
TENSOR_MAX_N = 12  # then tier 1 as tensor contractions, then as C loops


def _run(gates, n):
    if n <= DENSE_MAX_N:
        return dense.sv_run(gates, n)
    if n <= TENSOR_MAX_N:
        return tensor.sv_run(gates, n)
    return loops.sv_run(gates, n)


def _pauli_sum(psi, terms, n):
    if n <= DENSE_MAX_N:
        return dense.sv_pauli_sum(psi, terms, n)
    if n <= TENSOR_MAX_N:
        return tensor.sv_pauli_sum(psi, terms, n)
    return loops.sv_pauli_sum(psi, terms, n)


def bind(prog, theta, shift_gate: int = -1, shift: float = 0.0):
    """Gate list with parameters substituted; optionally the angle of gate
    number `shift_gate` is offset by `shift`."""
    out = []
    for idx, g in enumerate(prog):
        if g.param >= 0:
            a = float(theta[g.param]) + (shift if idx == shift_gate else 0.0)
            out.append((g.name, g.qubits, (a,)))
        else:
            out.append((g.name, g.qubits, ()))
    return out


def energy(prog, theta, terms, n: int) -> float:
    return _pauli_sum(_run(bind(prog, theta), n), terms, n)


def state(prog, theta, n: int) -> np.ndarray:
    return _run(bind(prog, theta), n)


def grad_parameter_shift(prog, theta, terms, n: int, params: Sequence[int] | None = None) -> np.ndarray:
    P = len(theta)
    g = np.zeros(P)
    want = set(range(P)) if params is None else set(params)
    for idx, gate in enumerate(prog):
        if gate.param < 0 or gate.param not in want:
            continue
        ep = _pauli_sum(_run(bind(prog, theta, idx, math.pi / 2), n), terms, n)
        em = _pauli_sum(_run(bind(prog, theta, idx, -math.pi / 2), n), terms, n)
        g[gate.param] += 0.5 * (ep - em)
    return g


def grad_finite_difference(prog, theta, terms, n: int, h: float = 1e-5,
                           params: Sequence[int] | None = None) -> np.ndarray:
    P = len(theta)
    g = np.zeros(P)
    for k in (range(P) if params is None else params):
        tp = np.array(theta, dtype=float)
        tm = np.array(theta, dtype=float)
        tp[k] += h
        tm[k] -= h
        g[k] = (energy(prog, tp, terms, n) - energy(prog, tm, terms, n)) / (2 * h)
    return g

"""Batched VQE energies and adjoint gradients (ctypes marshalling over the C
ABI's nwq_vqe_* calls) and a torch.autograd.Function around them.

The VQE experiment of the paper (Sec. III, Fig. 4) evaluates the Ising
energy of a parametrised circuit; here every evaluation also returns the
full gradient from the adjoint kernels, for B parameter vectors at once.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence, Tuple

import numpy as np
import torch

from . import nwq
from .nwq import _check, _dp, _ip, _up, lib

_vh = C.c_void_p
for _name, _args in {
    "nwq_vqe_create": [C.c_int, C.c_int, _ip, _ip, _ip, C.c_int, C.c_int, _up, _up, _dp, C.c_void_p, C.POINTER(_vh)],
    "nwq_vqe_destroy": [_vh],
    "nwq_vqe_info": [_vh, _ip, _ip, _ip],
    "nwq_vqe_eval": [_vh, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p],
    "nwq_vqe_eval_coeffs": [_vh, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "nwq_vqe_eval_single": [_vh, C.c_void_p, C.c_void_p, C.c_void_p],
    "nwq_vqe_set_config": [_vh, C.c_int, C.c_int, C.c_int],
    "nwq_vqe_get_config": [_vh, _ip, _ip, _ip],
    "nwq_vqe_autotune": [_vh, C.c_int, C.c_int, _dp],
    "nwq_vqe_batch": [C.c_int, C.c_int, _dp, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "nwq_vqe_batch_release": [],
    "nwq_vqe_memory": [_vh, C.c_int, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
    "nwq_vqe_set_flags": [_vh, C.c_int],
    "nwq_vqe_set_lowbits": [_vh, C.c_int],
}.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int

EXPORTED = ("nwq_vqe_create", "nwq_vqe_destroy", "nwq_vqe_info", "nwq_vqe_eval", "nwq_vqe_eval_coeffs",
            "nwq_vqe_eval_single",
            "nwq_vqe_set_config", "nwq_vqe_get_config", "nwq_vqe_autotune", "nwq_vqe_batch",
            "nwq_vqe_batch_release", "nwq_vqe_memory", "nwq_vqe_set_flags", "nwq_vqe_set_lowbits")


def program_arrays(prog) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(types, qubits[2i], params[i]) of a list of workloads.AnsatzGate-like
    entries with .name, .qubits and .param (-1 for fixed gates)."""
    types = np.array([nwq.GATES[g.name] for g in prog], dtype=np.int32)
    qs = np.full(2 * len(prog), -1, dtype=np.int32)
    ps = np.array([g.param for g in prog], dtype=np.int32)
    for i, g in enumerate(prog):
        qs[2 * i:2 * i + len(g.qubits)] = g.qubits
    return types, qs, ps


class VQE:
    """Context for one (register size, ansatz program, Hamiltonian)."""

    def __init__(self, n: int, prog, terms: Sequence[Tuple[int, int, float]], n_params: int | None = None,
                 stream=None):
        types, qs, ps = program_arrays(prog)
        if n_params is None:
            n_params = int(ps.max()) + 1 if len(ps) and ps.max() >= 0 else 0
        terms = list(terms)
        xm = np.array([t[0] for t in terms], dtype=np.uint64)
        zm = np.array([t[1] for t in terms], dtype=np.uint64)
        co = np.array([t[2] for t in terms], dtype=np.float64)
        self.n, self.P = n, n_params
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = _vh()
        _check(lib.nwq_vqe_create(n, len(types), types.ctypes.data_as(_ip), qs.ctypes.data_as(_ip),
                                  ps.ctypes.data_as(_ip), n_params, len(terms), xm.ctypes.data_as(_up),
                                  zm.ctypes.data_as(_up), co.ctypes.data_as(_dp), self.stream.cuda_stream,
                                  C.byref(h)))
        self.h = h.value

    def close(self):
        if getattr(self, "h", None):
            lib.nwq_vqe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _theta2d(self, theta: torch.Tensor) -> torch.Tensor:
        t = theta.detach()
        if t.dim() == 1:
            t = t.unsqueeze(0)
        assert t.shape[-1] == self.P and t.is_cuda
        return t.to(torch.float64).contiguous()

    def eval(self, theta: torch.Tensor, grad: bool = True):
        """theta [B, P] (or [P]) on the GPU -> (E [B], dE/dtheta [B, P] or None)."""
        t = self._theta2d(theta)
        B = t.shape[0]
        E = torch.empty(B, dtype=torch.float64, device=t.device)
        G = torch.empty(B, self.P, dtype=torch.float64, device=t.device) if grad else None
        _check(lib.nwq_vqe_eval(self.h, B, t.data_ptr(), E.data_ptr(), G.data_ptr() if grad else None))
        return E, G

    def eval_coeffs(self, theta: torch.Tensor, coeffs: torch.Tensor, grad: bool = True):
        """As eval, with per-vector Hamiltonian coefficients coeffs [B, n_terms] (device)."""
        t = self._theta2d(theta)
        B = t.shape[0]
        c = coeffs.detach().to(torch.float64).contiguous()
        assert c.is_cuda and c.shape[0] == B
        E = torch.empty(B, dtype=torch.float64, device=t.device)
        G = torch.empty(B, self.P, dtype=torch.float64, device=t.device) if grad else None
        _check(lib.nwq_vqe_eval_coeffs(self.h, B, t.data_ptr(), c.data_ptr(), E.data_ptr(),
                                       G.data_ptr() if grad else None))
        return E, G

    def eval_single(self, theta: torch.Tensor, grad: bool = True):
        """Plain per-circuit path for one vector theta [P]."""
        t = self._theta2d(theta)
        assert t.shape[0] == 1
        E = torch.empty(1, dtype=torch.float64, device=t.device)
        G = torch.empty(1, self.P, dtype=torch.float64, device=t.device) if grad else None
        _check(lib.nwq_vqe_eval_single(self.h, t.data_ptr(), E.data_ptr(), G.data_ptr() if grad else None))
        return E, G

    def set_config(self, mode: int = 0, threads: int = 256, blocks_per_state: int = 0):
        _check(lib.nwq_vqe_set_config(self.h, mode, threads, blocks_per_state))

    def set_flags(self, flags: int) -> None:
        _check(lib.nwq_vqe_set_flags(self.h, flags))

    def set_lowbits(self, c: int) -> None:
        """Low tile bits of the fused schedule's blocks: 0 = default (3), else 3..8."""
        _check(lib.nwq_vqe_set_lowbits(self.h, c))

    def get_config(self) -> Tuple[int, int, int]:
        m, t, b = C.c_int(), C.c_int(), C.c_int()
        _check(lib.nwq_vqe_get_config(self.h, C.byref(m), C.byref(t), C.byref(b)))
        return m.value, t.value, b.value

    def memory(self, B: int = 0) -> Tuple[int, int]:
        """(bytes held now, bytes held after evaluating B vectors)."""
        held, at = C.c_size_t(), C.c_size_t()
        _check(lib.nwq_vqe_memory(self.h, B, C.byref(held), C.byref(at)))
        return held.value, at.value

    def autotune(self, B: int, with_grad: bool = True) -> float:
        ms = C.c_double()
        _check(lib.nwq_vqe_autotune(self.h, B, int(with_grad), C.byref(ms)))
        return ms.value


def vqe_batch(n: int, L: int, J: float, h: float, theta: torch.Tensor, grad: bool = True, stream=None):
    """nwq_vqe_batch: energies (and gradients) of the hardware-efficient
    ansatz with L layers under the open-chain Ising Hamiltonian
    -J sum Z_i Z_{i+1} - h sum X_i, for theta [B, 2 n L] on the GPU."""
    t = theta.detach()
    if t.dim() == 1:
        t = t.unsqueeze(0)
    assert t.is_cuda and t.shape[-1] == 2 * n * L
    t = t.to(torch.float64).contiguous()
    B = t.shape[0]
    s = stream if stream is not None else torch.cuda.current_stream()
    E = torch.empty(B, dtype=torch.float64, device=t.device)
    G = torch.empty(B, 2 * n * L, dtype=torch.float64, device=t.device) if grad else None
    jh = (C.c_double * 2)(float(J), float(h))
    _check(lib.nwq_vqe_batch(n, L, jh, B, t.data_ptr(), E.data_ptr(), G.data_ptr() if grad else None, s.cuda_stream))
    return E, G


def vqe_batch_release() -> None:
    _check(lib.nwq_vqe_batch_release())


class AdjointEnergy(torch.autograd.Function):
    """E = AdjointEnergy.apply(theta, vqe): energies of theta [B, P] (or [P]);
    backward returns dE/dtheta from the adjoint kernels (computed in the same
    forward launch), scaled by the incoming gradient."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, vqe: VQE):
        E, G = vqe.eval(theta, grad=True)
        ctx.save_for_backward(G)
        ctx.squeeze = theta.dim() == 1
        return E[0] if ctx.squeeze else E

    @staticmethod
    def backward(ctx, gE):
        (G,) = ctx.saved_tensors
        if ctx.squeeze:
            return gE * G[0], None
        return gE.unsqueeze(-1) * G, None

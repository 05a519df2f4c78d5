"""ctypes binding of the C ABI in include/nwq.h (argument marshalling only).

Functions keep the C names (nwq_sv_create, nwq_apply_gate, ...) and raise
NwqError on a non-zero status.  Every numerical step runs in the HIP
library; if libnwq.so is missing this module fails at import with an
ImportError -- there is no fallback path.

`SVState` / `DMState` are small conveniences over the same calls that take
their device memory from PyTorch (a complex128 CUDA tensor) and their stream
from torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Sequence, Tuple

import numpy as np

# torch ships its own HIP runtime with the same soname as the system one; it
# must be loaded first so that libnwq.so binds to that single runtime instead
# of pulling a second copy into the process.
import torch  # noqa: F401

# NWQ_LIB may name another build of the same ABI (the host-only sanitizer
# build used by the CPU tests); by default the in-tree libnwq.so.
_LIB_PATH = os.environ.get("NWQ_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnwq.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"HIP engine not built ({_LIB_PATH} missing); run `python -m paper_2401_06861_amd.build`")
lib = C.CDLL(_LIB_PATH)

NWQ_OK, NWQ_EINVAL, NWQ_ERANGE, NWQ_EDUP, NWQ_EKIND, NWQ_ENOTCPTP, NWQ_ENOMEM, NWQ_EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "NWQ_OK", -1: "NWQ_EINVAL", -2: "NWQ_ERANGE", -3: "NWQ_EDUP", -4: "NWQ_EKIND",
                -5: "NWQ_ENOTCPTP", -6: "NWQ_ENOMEM", -7: "NWQ_EDEVICE"}
KIND_SV, KIND_DM = 0, 1
TIMING_CLASSES = ("reset", "sv_1q_dense", "sv_diag", "sv_perm", "sv_2q_dense", "sv_fused",
                  "dm_superop_1q", "dm_superop_2q", "reduce")

GATES = {"id": 0, "x": 1, "y": 2, "z": 3, "h": 4, "s": 5, "sdg": 6, "t": 7, "tdg": 8,
         "rx": 9, "ry": 10, "rz": 11, "u3": 12, "cx": 13, "cz": 14, "swap": 15, "rzz": 16}


class NwqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_h = C.c_void_p
_ip = C.POINTER(C.c_int)
_dp = C.POINTER(C.c_double)
_up = C.POINTER(C.c_uint64)
_SIG = {
    "nwq_sv_create": [C.c_int, C.c_void_p, C.POINTER(_h)],
    "nwq_dm_create": [C.c_int, C.c_void_p, C.POINTER(_h)],
    "nwq_sv_create_from": [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(_h)],
    "nwq_dm_create_from": [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(_h)],
    "nwq_destroy": [_h],
    "nwq_info": [_h, _ip, _ip, C.POINTER(C.c_void_p)],
    "nwq_reset": [_h],
    "nwq_get_state": [_h, _dp, C.c_size_t],
    "nwq_set_state": [_h, _dp, C.c_size_t],
    "nwq_flush": [_h],
    "nwq_apply_gate": [_h, C.c_int, _ip, C.c_int, _dp, C.c_int],
    "nwq_apply_matrix": [_h, _ip, C.c_int, _dp],
    "nwq_apply_circuit": [_h, C.c_int, _ip, _ip, _dp],
    "nwq_run_circuit": [_h, C.c_int, _ip, _ip, _dp],
    "nwq_set_fusion": [_h, C.c_int, _ip],
    "nwq_fusion_stats": [_h, _ip, _ip],
    "nwq_set_fusion_kernel": [_h, C.c_int],
    "nwq_set_fusion_flags": [_h, C.c_int],
    "nwq_set_fusion_lowbits": [_h, C.c_int],
    "nwq_fusion_phases": [_h, _ip],
    "nwq_fusion_plan": [C.c_int, C.c_int, C.c_int, _ip, _ip, _ip, _ip, _ip],
    "nwq_apply_channel": [_h, _ip, C.c_int, _dp, C.c_int],
    "nwq_depolarize": [_h, _ip, C.c_int, C.c_double],
    "nwq_depolarize_ex": [_h, _ip, C.c_int, C.c_double, C.c_int],
    "nwq_thermal_relax": [_h, C.c_int, C.c_double, C.c_double, C.c_double],
    "nwq_amp_damp": [_h, C.c_int, C.c_double],
    "nwq_phase_damp": [_h, C.c_int, C.c_double],
    "nwq_expval_pauli_sum": [_h, C.c_int, _up, _up, _dp, _dp],
    "nwq_expval_pauli_terms": [_h, C.c_int, _up, _up, _dp],
    "nwq_expval_pauli_terms_complex": [_h, C.c_int, _up, _up, _dp, _dp],
    "nwq_trace": [_h, _dp, _dp],
    "nwq_memory": [_h, C.POINTER(C.c_size_t)],
    "nwq_purity": [_h, _dp],
    "nwq_timing_enable": [_h, C.c_int],
    "nwq_set_launch": [_h, C.c_int, C.c_int, C.c_int, C.c_int],
    "nwq_get_launch": [_h, C.c_int, C.c_int, _ip, _ip],
    "nwq_set_launch_target": [_h, C.c_int, C.c_int, C.c_int, C.c_int],
    "nwq_get_launch_target": [_h, C.c_int, C.c_int, _ip, _ip],
    "nwq_autotune": [_h, C.c_int, _dp],
    "nwq_autotune_fusion": [_h, C.c_int, _ip, _ip, _dp, C.c_int, _ip, _ip, _dp],
    "nwq_qasm_parse": [C.c_char_p, _ip, _ip, C.c_int, _ip, _ip, _dp],
    "nwq_apply_qasm": [_h, C.c_char_p],
    "nwq_probabilities": [_h, C.c_void_p],
    "nwq_readout_noise": [C.c_int, C.c_void_p, _dp, C.c_void_p],
    "nwq_sample_workspace_bytes": [C.c_int],
    "nwq_sample": [C.c_int, C.c_void_p, C.c_void_p, C.c_longlong, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p],
    "nwq_sample_noalloc": [C.c_int, C.c_void_p, C.c_void_p, C.c_longlong, C.c_void_p, C.c_void_p],
    "nwq_timing_read": [_h, C.POINTER(C.c_longlong), _dp, C.c_int],
    "nwq_stream_scale": [C.c_void_p, C.c_size_t, C.c_double, C.c_void_p],
    "nwq_stream_copy": [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p],
}
for _name, _args in _SIG.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
lib.nwq_last_error.argtypes = []
lib.nwq_last_error.restype = C.c_char_p
lib.nwq_sample_workspace_bytes.restype = C.c_size_t

EXPORTED = tuple(_SIG) + ("nwq_last_error",)


def nwq_last_error() -> str:
    return lib.nwq_last_error().decode()


def _check(rc: int) -> None:
    if rc != NWQ_OK:
        raise NwqError(rc, nwq_last_error())


def _ints(xs: Sequence[int]):
    arr = (C.c_int * max(len(xs), 1))(*[int(x) for x in xs])
    return arr


def _doubles(xs: Sequence[float]):
    return (C.c_double * max(len(xs), 1))(*[float(x) for x in xs])


def _u64(xs: Sequence[int]):
    return (C.c_uint64 * max(len(xs), 1))(*[int(x) for x in xs])


# ------------------------------------------------------------ C-named calls
def nwq_sv_create(n: int, stream: int | None = None) -> int:
    h = _h()
    _check(lib.nwq_sv_create(n, stream, C.byref(h)))
    return h.value


def nwq_dm_create(n: int, stream: int | None = None) -> int:
    h = _h()
    _check(lib.nwq_dm_create(n, stream, C.byref(h)))
    return h.value


def nwq_sv_create_from(dev_ptr: int, n: int, stream: int | None = None) -> int:
    h = _h()
    _check(lib.nwq_sv_create_from(dev_ptr, n, stream, C.byref(h)))
    return h.value


def nwq_dm_create_from(dev_ptr: int, n: int, stream: int | None = None) -> int:
    h = _h()
    _check(lib.nwq_dm_create_from(dev_ptr, n, stream, C.byref(h)))
    return h.value


def nwq_destroy(h: int) -> None:
    _check(lib.nwq_destroy(h))


def nwq_info(h: int) -> Tuple[int, int, int]:
    k, n, p = C.c_int(), C.c_int(), C.c_void_p()
    _check(lib.nwq_info(h, C.byref(k), C.byref(n), C.byref(p)))
    return k.value, n.value, p.value or 0


def nwq_reset(h: int) -> None:
    _check(lib.nwq_reset(h))


def nwq_get_state(h: int, out: np.ndarray) -> None:
    assert out.dtype == np.complex128 and out.flags.c_contiguous
    _check(lib.nwq_get_state(h, out.ctypes.data_as(_dp), out.size * 2))


def nwq_set_state(h: int, src: np.ndarray) -> None:
    src = np.ascontiguousarray(src, dtype=np.complex128)
    _check(lib.nwq_set_state(h, src.ctypes.data_as(_dp), src.size * 2))


def nwq_flush(h: int) -> None:
    _check(lib.nwq_flush(h))


def nwq_apply_gate(h: int, gate, qubits: Sequence[int], params: Sequence[float] = ()) -> None:
    t = GATES[gate] if isinstance(gate, str) else int(gate)
    _check(lib.nwq_apply_gate(h, t, _ints(qubits), len(qubits), _doubles(params), len(params)))


def nwq_apply_matrix(h: int, qubits: Sequence[int], m: np.ndarray) -> None:
    m = np.ascontiguousarray(m, dtype=np.complex128)
    _check(lib.nwq_apply_matrix(h, _ints(qubits), len(qubits), m.ctypes.data_as(_dp)))


def circuit_arrays(gates: Iterable) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(types, qubits[2*i], params[3*i]) arrays of a gate list."""
    gates = list(gates)
    types = np.zeros(len(gates), dtype=np.int32)
    qs = np.zeros(2 * len(gates), dtype=np.int32)
    ps = np.zeros(3 * len(gates), dtype=np.float64)
    for i, (name, q, p) in enumerate(gates):
        types[i] = GATES[name]
        qs[2 * i:2 * i + len(q)] = q
        ps[3 * i:3 * i + len(p)] = p
    return types, qs, ps


def nwq_apply_circuit(h: int, types: np.ndarray, qubits: np.ndarray, params: np.ndarray) -> None:
    types = np.ascontiguousarray(types, dtype=np.int32)
    qubits = np.ascontiguousarray(qubits, dtype=np.int32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    _check(lib.nwq_apply_circuit(h, len(types), types.ctypes.data_as(_ip), qubits.ctypes.data_as(_ip),
                                 params.ctypes.data_as(_dp)))


def nwq_run_circuit(h: int, types: np.ndarray, qubits: np.ndarray, params: np.ndarray) -> None:
    """Reset to |0...0> and apply the circuit (arrays of circuit_arrays)."""
    types = np.ascontiguousarray(types, dtype=np.int32)
    qubits = np.ascontiguousarray(qubits, dtype=np.int32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    _check(lib.nwq_run_circuit(h, len(types), types.ctypes.data_as(_ip), qubits.ctypes.data_as(_ip),
                               params.ctypes.data_as(_dp)))


def nwq_set_fusion(h: int, k: int) -> int:
    out = C.c_int()
    _check(lib.nwq_set_fusion(h, k, C.byref(out)))
    return out.value


def nwq_fusion_stats(h: int) -> Tuple[int, int]:
    b, g = C.c_int(), C.c_int()
    _check(lib.nwq_fusion_stats(h, C.byref(b), C.byref(g)))
    return b.value, g.value


def nwq_set_fusion_kernel(h: int, kernel: int) -> None:
    """0: one LDS pass per gate; 1: register-blocked, 4 register bits; 2: register-blocked, 3 bits."""
    _check(lib.nwq_set_fusion_kernel(h, int(kernel)))


def nwq_set_fusion_flags(h: int, flags: int) -> None:
    _check(lib.nwq_set_fusion_flags(h, flags))


def nwq_set_fusion_lowbits(h: int, c: int) -> None:
    """Low tile bits of fused blocks: 0 = default (6 for SV, 4 for DM), else 3..8."""
    _check(lib.nwq_set_fusion_lowbits(h, int(c)))


def nwq_fusion_phases(h: int) -> int:
    p = C.c_int()
    _check(lib.nwq_fusion_phases(h, C.byref(p)))
    return p.value


def nwq_fusion_plan(n: int, k: int, types: np.ndarray, qubits: np.ndarray):
    """(n_blocks, block_of_gate[], tile qubit mask per block) without a device."""
    types = np.ascontiguousarray(types, dtype=np.int32)
    qubits = np.ascontiguousarray(qubits, dtype=np.int32)
    g = len(types)
    nb = C.c_int()
    bog = np.zeros(max(g, 1), dtype=np.int32)
    bq = np.zeros(2 * max(g, 1), dtype=np.int32)
    _check(lib.nwq_fusion_plan(n, k, g, types.ctypes.data_as(_ip), qubits.ctypes.data_as(_ip), C.byref(nb),
                               bog.ctypes.data_as(_ip), bq.ctypes.data_as(_ip)))
    masks = [(int(bq[2 * b]) & 0xffffffff) | ((int(bq[2 * b + 1]) & 0xffffffff) << 32) for b in range(nb.value)]
    return nb.value, bog[:g], masks


def nwq_apply_channel(h: int, qubits: Sequence[int], kraus: Sequence[np.ndarray]) -> None:
    ks = np.ascontiguousarray(np.stack([np.asarray(K, dtype=np.complex128) for K in kraus]))
    _check(lib.nwq_apply_channel(h, _ints(qubits), len(qubits), ks.ctypes.data_as(_dp), len(kraus)))


def nwq_depolarize(h: int, qubits: Sequence[int], p: float) -> None:
    _check(lib.nwq_depolarize(h, _ints(qubits), len(qubits), p))


DEPOL_REPLACE, DEPOL_PAULI = 0, 1


def nwq_depolarize_ex(h: int, qubits: Sequence[int], p: float, convention: int) -> None:
    _check(lib.nwq_depolarize_ex(h, _ints(qubits), len(qubits), p, convention))


def nwq_thermal_relax(h: int, q: int, t1: float, t2: float, t: float) -> None:
    _check(lib.nwq_thermal_relax(h, q, t1, t2, t))


def nwq_amp_damp(h: int, q: int, gamma: float) -> None:
    _check(lib.nwq_amp_damp(h, q, gamma))


def nwq_phase_damp(h: int, q: int, lam: float) -> None:
    _check(lib.nwq_phase_damp(h, q, lam))


def nwq_expval_pauli_sum(h: int, terms) -> float:
    terms = list(terms)
    out = C.c_double()
    _check(lib.nwq_expval_pauli_sum(h, len(terms), _u64([t[0] for t in terms]), _u64([t[1] for t in terms]),
                                    _doubles([t[2] for t in terms]), C.byref(out)))
    return out.value


def nwq_expval_pauli_terms(h: int, terms) -> np.ndarray:
    terms = list(terms)
    out = np.zeros(max(len(terms), 1))
    _check(lib.nwq_expval_pauli_terms(h, len(terms), _u64([t[0] for t in terms]), _u64([t[1] for t in terms]),
                                      out.ctypes.data_as(_dp)))
    return out[:len(terms)]


def nwq_expval_pauli_terms_complex(h: int, terms) -> np.ndarray:
    """Complex <P_t> per term (DM: the kernel's imaginary parts of Tr(rho P_t);
    SV: imaginary parts are 0 by construction)."""
    terms = list(terms)
    re = np.zeros(max(len(terms), 1))
    im = np.zeros(max(len(terms), 1))
    _check(lib.nwq_expval_pauli_terms_complex(h, len(terms), _u64([t[0] for t in terms]),
                                              _u64([t[1] for t in terms]), re.ctypes.data_as(_dp),
                                              im.ctypes.data_as(_dp)))
    return (re + 1j * im)[:len(terms)]


def nwq_memory(h: int) -> int:
    """Device bytes the handle holds."""
    b = C.c_size_t()
    _check(lib.nwq_memory(h, C.byref(b)))
    return b.value


def nwq_trace(h: int) -> Tuple[float, float]:
    re, im = C.c_double(), C.c_double()
    _check(lib.nwq_trace(h, C.byref(re), C.byref(im)))
    return re.value, im.value


def nwq_purity(h: int) -> float:
    out = C.c_double()
    _check(lib.nwq_purity(h, C.byref(out)))
    return out.value


LAUNCH_BUCKETS = ("low", "mid", "high")   # lowest target bit 0-2, 3-10, 11 and up


def nwq_set_launch(h: int, cls: int, bucket: int, ppt: int, nontemporal: int) -> None:
    _check(lib.nwq_set_launch(h, cls, bucket, ppt, nontemporal))


def nwq_get_launch(h: int, cls: int, bucket: int) -> Tuple[int, int]:
    p, t = C.c_int(), C.c_int()
    _check(lib.nwq_get_launch(h, cls, bucket, C.byref(p), C.byref(t)))
    return p.value, t.value


LAUNCH_TARGET_BITS = 64


def nwq_set_launch_target(h: int, cls: int, bit: int, ppt: int, nontemporal: int) -> None:
    """Shape of launches whose lowest target bit is `bit` (ppt 0 clears it)."""
    _check(lib.nwq_set_launch_target(h, cls, bit, ppt, nontemporal))


def nwq_get_launch_target(h: int, cls: int, bit: int) -> Tuple[int, int]:
    p, t = C.c_int(), C.c_int()
    _check(lib.nwq_get_launch_target(h, cls, bit, C.byref(p), C.byref(t)))
    return p.value, t.value


def nwq_autotune(h: int, reps: int = 3) -> dict:
    """{class name: {bucket name: ms per launch}} for the classes and buckets tuned."""
    nb = len(LAUNCH_BUCKETS)
    ms = (C.c_double * (len(TIMING_CLASSES) * nb))()
    _check(lib.nwq_autotune(h, reps, ms))
    out = {}
    for i, name in enumerate(TIMING_CLASSES):
        for b, bname in enumerate(LAUNCH_BUCKETS):
            if ms[i * nb + b] >= 0:
                out.setdefault(name, {})[bname] = float(ms[i * nb + b])
    return out


FUSION_CANDIDATES = 25
FUSION_KERNELS = ("lds", "rb4", "rb3")   # nwq_set_fusion_kernel values 0, 1, 2


def nwq_autotune_fusion(h: int, types: np.ndarray, qubits: np.ndarray, params: np.ndarray, reps: int = 1):
    """(best width (0 = unfused), fused kernel (0 per-gate LDS, 1 / 2 register-blocked with 4 / 3
    register bits), {(k, kernel): ms per circuit});
    the best setting is left on the handle and the state at |0...0>."""
    types = np.ascontiguousarray(types, dtype=np.int32)
    qubits = np.ascontiguousarray(qubits, dtype=np.int32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    k, rb = C.c_int(), C.c_int()
    ms = (C.c_double * FUSION_CANDIDATES)()
    _check(lib.nwq_autotune_fusion(h, len(types), types.ctypes.data_as(_ip), qubits.ctypes.data_as(_ip),
                                   params.ctypes.data_as(_dp), reps, C.byref(k), C.byref(rb), ms))
    table = {}
    for i in range(FUSION_CANDIDATES):
        if ms[i] >= 0:
            table[(0, 0) if i == 0 else (6 + (i - 1) // 3, (i - 1) % 3)] = float(ms[i])
    return k.value, rb.value, table


# ------------------------------------------------------------ OpenQASM 2.0
def nwq_qasm_parse(text: str):
    """(n_qubits, types, qubits[2*i], params[3*i]) of an OpenQASM 2.0 program."""
    src = text.encode()
    nq, ng = C.c_int(), C.c_int()
    _check(lib.nwq_qasm_parse(src, C.byref(nq), C.byref(ng), 0, None, None, None))
    types = np.zeros(ng.value, dtype=np.int32)
    qs = np.zeros(2 * ng.value, dtype=np.int32)
    ps = np.zeros(3 * ng.value, dtype=np.float64)
    _check(lib.nwq_qasm_parse(src, C.byref(nq), C.byref(ng), ng.value, types.ctypes.data_as(_ip),
                              qs.ctypes.data_as(_ip), ps.ctypes.data_as(_dp)))
    return nq.value, types, qs, ps


def nwq_apply_qasm(h: int, text: str) -> None:
    _check(lib.nwq_apply_qasm(h, text.encode()))


# ------------------------------------------------------------ measurement
def nwq_probabilities(h: int, probs) -> None:
    """probs: float64 cuda tensor of 2^n entries (written on the handle's stream)."""
    _check(lib.nwq_probabilities(h, probs.data_ptr()))


def nwq_readout_noise(n: int, probs, confusion, stream=None) -> None:
    """confusion: n x 2 x 2 array, C[q][r][t] = P(read r | true t)."""
    import torch
    cm = np.ascontiguousarray(np.asarray(confusion, dtype=np.float64).reshape(n, 4))
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.nwq_readout_noise(n, probs.data_ptr(), cm.ctypes.data_as(_dp), s.cuda_stream))


def nwq_sample_workspace_bytes(n: int) -> int:
    return int(lib.nwq_sample_workspace_bytes(n))


def nwq_sample(n: int, probs, u, out, work, stream=None) -> None:
    """probs: float64 cuda [2^n]; u: float64 cuda [shots]; out: int64 cuda
    [shots]; work: cuda tensor of at least nwq_sample_workspace_bytes(n)
    bytes (its first 2^n int64 entries hold the integer CDF afterwards)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.nwq_sample(n, probs.data_ptr(), u.data_ptr(), u.numel(), out.data_ptr(), work.data_ptr(),
                          work.numel() * work.element_size(), s.cuda_stream))


def nwq_sample_noalloc(n: int, probs, u, out, stream=None) -> None:
    """As nwq_sample, with the library's own device scratch instead of a
    workspace (n <= 20; calls on one GPU must not overlap)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.nwq_sample_noalloc(n, probs.data_ptr(), u.data_ptr(), u.numel(), out.data_ptr(), s.cuda_stream))


def nwq_stream_scale(buf, s: float, stream=None) -> None:
    """In-place a <- s a over a complex128 cuda tensor (streaming yardstick)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.nwq_stream_scale(buf.data_ptr(), buf.numel(), float(s), st.cuda_stream))


def nwq_stream_copy(dst, src, stream=None) -> None:
    """dst <- src for complex128 cuda tensors of equal size (streaming yardstick)."""
    import torch
    assert dst.numel() == src.numel()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib.nwq_stream_copy(dst.data_ptr(), src.data_ptr(), src.numel(), st.cuda_stream))


def nwq_timing_enable(h: int, enable: bool = True) -> None:
    _check(lib.nwq_timing_enable(h, int(bool(enable))))


def nwq_timing_read(h: int, reset: bool = True) -> dict:
    cnt = (C.c_longlong * len(TIMING_CLASSES))()
    ms = (C.c_double * len(TIMING_CLASSES))()
    _check(lib.nwq_timing_read(h, cnt, ms, int(bool(reset))))
    return {name: (int(cnt[i]), float(ms[i])) for i, name in enumerate(TIMING_CLASSES)}


# ------------------------------------------------------------ conveniences
class _State:
    kind = KIND_SV

    def __init__(self, n: int, tensor=None, stream=None, reset: bool = True, owned: bool = False):
        """The state lives in `tensor` (a torch complex128 buffer, allocated
        here if None) or, with owned=True, in memory the library allocates
        and frees itself (nwq_sv_create / nwq_dm_create)."""
        import torch
        self.n = n
        size = (1 << n) if self.kind == KIND_SV else (1 << (2 * n))
        self.size = size
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if owned:
            assert tensor is None
            self.tensor = None
            create = nwq_sv_create if self.kind == KIND_SV else nwq_dm_create
            self.h = create(n, self.stream.cuda_stream)
        else:
            if tensor is None:
                tensor = torch.empty(size, dtype=torch.complex128, device="cuda")
            assert tensor.dtype == torch.complex128 and tensor.is_cuda and tensor.is_contiguous()
            assert tensor.numel() == size
            self.tensor = tensor
            create = nwq_sv_create_from if self.kind == KIND_SV else nwq_dm_create_from
            self.h = create(tensor.data_ptr(), n, self.stream.cuda_stream)
        if reset:
            nwq_reset(self.h)

    def close(self):
        if getattr(self, "h", None):
            nwq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def reset(self):
        nwq_reset(self.h)

    def apply(self, name, qubits, params=()):
        nwq_apply_gate(self.h, name, qubits, params)

    def apply_matrix(self, qubits, m):
        nwq_apply_matrix(self.h, qubits, m)

    def run(self, gates):
        """Apply a gate list (and, on DM, channel entries) in order."""
        for name, q, p in gates:
            if name == "depolarize" or name == "depolarize2":
                nwq_depolarize(self.h, q, p[0])
            elif name == "depolarize_nc" or name == "depolarize2_nc":
                nwq_depolarize_ex(self.h, q, p[0], DEPOL_PAULI)
            elif name == "thermal_relax":
                nwq_thermal_relax(self.h, q[0], p[0], p[1], p[2])
            elif name == "amp_damp":
                nwq_amp_damp(self.h, q[0], p[0])
            elif name == "phase_damp":
                nwq_phase_damp(self.h, q[0], p[0])
            else:
                nwq_apply_gate(self.h, name, q, p)

    def run_circuit(self, gates):
        nwq_apply_circuit(self.h, *circuit_arrays(gates))

    def set_fusion(self, k: int) -> int:
        return nwq_set_fusion(self.h, k)

    def expvals(self, terms) -> np.ndarray:
        return nwq_expval_pauli_terms(self.h, terms)

    def expvals_complex(self, terms) -> np.ndarray:
        return nwq_expval_pauli_terms_complex(self.h, terms)

    def pauli_sum(self, terms) -> float:
        return nwq_expval_pauli_sum(self.h, terms)

    def purity(self) -> float:
        return nwq_purity(self.h)

    def probabilities(self):
        """Outcome probabilities as a float64 cuda tensor of 2^n entries."""
        import torch
        p = torch.empty(1 << self.n, dtype=torch.float64, device="cuda")
        nwq_probabilities(self.h, p)
        return p

    def numpy(self) -> np.ndarray:
        out = np.empty(self.size, dtype=np.complex128)
        nwq_get_state(self.h, out)
        return out

    def load(self, arr: np.ndarray):
        nwq_set_state(self.h, np.asarray(arr, dtype=np.complex128).reshape(-1))

    def flush(self):
        nwq_flush(self.h)


def sample_shots(n: int, probs, u, work=None):
    """Outcome indices (int64 cuda tensor) for the uniforms u drawn from probs."""
    import torch
    if work is None:
        work = torch.empty(nwq_sample_workspace_bytes(n) // 8, dtype=torch.int64, device=probs.device)
    out = torch.empty(u.numel(), dtype=torch.int64, device=probs.device)
    nwq_sample(n, probs, u, out, work)
    return out


class SVState(_State):
    kind = KIND_SV


class DMState(_State):
    kind = KIND_DM

    def channel(self, qubits, kraus):
        nwq_apply_channel(self.h, qubits, kraus)

    def trace(self) -> Tuple[float, float]:
        return nwq_trace(self.h)

    def numpy(self) -> np.ndarray:
        return super().numpy().reshape(1 << self.n, 1 << self.n)

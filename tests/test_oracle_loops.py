"""Pins of the C-loop tier of the oracle (oracle/loops.c): against tier 0
(dense Kronecker operators) and tier 1 (tensor contractions) on random
circuits, channels and Pauli strings; closed forms (Bell, GHZ, bit flips,
channel Bloch maps); the noise-free density matrix equal to psi psi^dagger;
and updated states independent of the thread count."""
import math

import numpy as np
import pytest

from oracle import dense, gates as G, loops, tensor
import workloads as W


def _all_channels_circuit(n, seed):
    """Random gates, each followed by every channel kind of the noise model in
    both depolarising conventions."""
    rng = np.random.default_rng(seed)
    ops = []
    for g in W.random_gate_list(n, 12, seed=seed):
        ops.append(g)
        q = g[1]
        if len(q) == 1:
            kind = ["depolarize", "amp_damp", "phase_damp", "depolarize_nc"][int(rng.integers(4))]
            ops.append((kind, q, (float(rng.uniform(0.01, 0.3)),)))
        else:
            kind = ["depolarize2", "depolarize2_nc"][int(rng.integers(2))]
            ops.append((kind, q, (float(rng.uniform(0.01, 0.3)),)))
    return ops


@pytest.mark.parametrize("n", [1, 2, 5, 6])
def test_sv_matches_dense(n):
    gates = W.random_gate_list(n, 80, seed=10 + n)
    a = loops.sv_run(gates, n)
    b = dense.sv_run(gates, n)
    assert np.abs(a - b).max() < 1e-14


def test_sv_matches_tensor_n11():
    n = 11
    gates = W.random_gate_list(n, 150, seed=3)
    assert np.abs(loops.sv_run(gates, n) - tensor.sv_run(gates, n)).max() < 1e-13


@pytest.mark.parametrize("n", [2, 3, 4])
def test_dm_matches_dense_every_channel(n):
    ops = _all_channels_circuit(n, seed=20 + n)
    a = loops.dm_run(ops, n)
    b = dense.dm_run(ops, n)
    assert np.abs(a - b).max() < 1e-14


def test_dm_matches_tensor_noisy_tfim_n6():
    n = 6
    ops = W.noisy_tfim_circuit(n, 3)
    assert np.abs(loops.dm_run(ops, n) - tensor.dm_run(ops, n)).max() < 1e-14


def test_expvals_match_dense():
    n = 5
    psi = W.random_state(n, seed=4)
    rho = W.random_density_matrix(4, seed=5)
    for x, z, _ in W.random_pauli_sum(n, 30, seed=6):
        assert abs(loops.sv_expval(psi, x, z, n) - dense.sv_expval(psi, x, z, n)) < 1e-14
    for x, z, _ in W.random_pauli_sum(4, 30, seed=7):
        assert abs(loops.dm_expval(rho, x, z, 4) - dense.dm_expval(rho, x, z, 4)) < 1e-14
    assert abs(loops.dm_purity(rho, 4) - dense.dm_purity(rho)) < 1e-14
    assert abs(loops.dm_trace(rho, 4) - np.trace(rho)) < 1e-14


def test_bell_ghz_and_bit_flips():
    psi = loops.sv_run([("h", (0,), ()), ("cx", (0, 1), ())], 2)
    assert np.abs(psi - np.array([1, 0, 0, 1]) / math.sqrt(2)).max() < 1e-15
    n = 7
    ghz = loops.sv_run([("h", (0,), ())] + [("cx", (i, i + 1), ()) for i in range(n - 1)], n)
    want = np.zeros(1 << n, dtype=complex)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.abs(ghz - want).max() < 1e-15
    for q in range(n):
        e = loops.sv_run([("x", (q,), ())], n)
        assert e[1 << q] == 1 and np.count_nonzero(e) == 1
    # <Z_q> of a basis state is the sign of its bit; <X_q> of |+> is 1
    e = loops.sv_run([("x", (2,), ()), ("h", (4,), ())], n)
    assert abs(loops.sv_expval(e, 0, 1 << 2, n) + 1) < 1e-15
    assert abs(loops.sv_expval(e, 0, 1 << 3, n) - 1) < 1e-15
    assert abs(loops.sv_expval(e, 1 << 4, 0, n) - 1) < 1e-15


def _bloch(rho):
    return np.array([2 * rho[0, 1].real, -2 * rho[0, 1].imag, (rho[0, 0] - rho[1, 1]).real])


def test_channel_bloch_maps():
    rng = np.random.default_rng(8)
    v = rng.normal(size=3)
    r = 0.9 * v / np.linalg.norm(v)
    rho0 = 0.5 * (np.eye(2) + r[0] * G.X + r[1] * G.Y + r[2] * G.Z)
    p, g, lam = 0.2, 0.3, 0.4
    cases = {("depolarize", p): (1 - p) * r,
             ("depolarize_nc", p): (1 - 4 * p / 3) * r,
             ("amp_damp", g): np.array([math.sqrt(1 - g) * r[0], math.sqrt(1 - g) * r[1], (1 - g) * r[2] + g]),
             ("phase_damp", lam): np.array([math.sqrt(1 - lam) * r[0], math.sqrt(1 - lam) * r[1], r[2]])}
    for (name, prm), want in cases.items():
        rho = np.array(rho0, dtype=np.complex128)
        loops.dm_apply(rho, (name, (0,), (prm,)), 1)
        assert np.abs(_bloch(rho) - want).max() < 1e-15, name
    # full depolarisation sends any two-qubit state to I/4; AD(1) to |0><0|
    rho = W.random_density_matrix(2, seed=9)
    loops.dm_apply(rho, ("depolarize2", (0, 1), (1.0,)), 2)
    assert np.abs(rho - np.eye(4) / 4).max() < 1e-15
    rho = np.array(rho0, dtype=np.complex128)
    loops.dm_apply(rho, ("amp_damp", (0,), (1.0,)), 1)
    assert np.abs(rho - np.diag([1, 0])).max() < 1e-15


def test_noise_free_dm_is_outer_product_of_sv():
    n = 5
    gates = W.random_gate_list(n, 60, seed=11)
    psi = loops.sv_run(gates, n)
    rho = loops.dm_run(gates, n)
    assert np.abs(rho - np.outer(psi, psi.conj())).max() < 1e-14
    assert abs(loops.dm_purity(rho, n) - 1) < 1e-13


def test_noisy_dm_invariants():
    n = 5
    rho = loops.dm_run(W.noisy_tfim_circuit(n, 4), n)
    assert abs(loops.dm_trace(rho, n) - 1) < 1e-13
    assert np.abs(rho - rho.conj().T).max() < 1e-15
    assert np.linalg.eigvalsh(rho).min() > -1e-13
    assert loops.dm_purity(rho, n) < 1


def test_states_do_not_depend_on_thread_count():
    n = 16
    gates = W.random_gate_list(n, 40, seed=12)
    before = loops.get_threads()
    try:
        loops.set_threads(1)
        a = loops.sv_run(gates, n)
        loops.set_threads(max(before, 2))
        b = loops.sv_run(gates, n)
    finally:
        loops.set_threads(before)
    assert np.array_equal(a, b)


def test_rejects_bad_qubits():
    psi = loops.sv_zero(3)
    with pytest.raises(ValueError):
        loops.sv_apply(psi, ("cx", (1, 1), ()), 3)
    with pytest.raises(ValueError):
        loops.sv_apply(psi, ("x", (3,), ()), 3)
    with pytest.raises(ValueError):
        loops.sv_apply(np.zeros(4, dtype=np.complex128), ("x", (0,), ()), 3)

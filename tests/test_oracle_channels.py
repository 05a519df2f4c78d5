"""Pins of the oracle's noise channels (Sec. III noise model) and of its
density-matrix pipeline: Bloch-vector closed forms, the defining formula of
the depolarising channel via an explicit partial trace, CPTP, special
cases, and reduction of the noise-free DM path to the SV path."""
import math

import numpy as np
import pytest

from oracle import dense, gates as G, tensor
import workloads as W


def close(a, b, tol=1e-14):
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) <= tol


def bloch(rho):
    return np.array([np.trace(rho @ P).real for P in (G.X, G.Y, G.Z)])


def from_bloch(r):
    return 0.5 * (G.I2 + r[0] * G.X + r[1] * G.Y + r[2] * G.Z)


def apply1(kraus, rho):
    return sum(K @ rho @ K.conj().T for K in kraus)


@pytest.mark.parametrize("name", ["depolarize", "amp_damp", "phase_damp", "depolarize2", "depolarize_nc",
                                  "depolarize2_nc"])
def test_cptp(name):
    for p in (0.0, 1e-3, 0.3, 1.0):
        ks = G.channel_kraus(name, (p,))
        d = ks[0].shape[0]
        assert close(sum(K.conj().T @ K for K in ks), np.eye(d))


def test_bloch_closed_forms():
    rng = np.random.default_rng(1)
    for _ in range(20):
        r = rng.standard_normal(3)
        r *= rng.uniform(0, 1) / np.linalg.norm(r)
        rho = from_bloch(r)
        p, g, l = rng.uniform(0, 1, 3)
        assert close(bloch(apply1(G.kraus_depolarize(p), rho)), (1 - p) * r)
        want = np.array([math.sqrt(1 - g) * r[0], math.sqrt(1 - g) * r[1], (1 - g) * r[2] + g])
        assert close(bloch(apply1(G.kraus_amp_damp(g), rho)), want)
        want = np.array([math.sqrt(1 - l) * r[0], math.sqrt(1 - l) * r[1], r[2]])
        assert close(bloch(apply1(G.kraus_phase_damp(l), rho)), want)


def _ptrace_reinsert(rho, qubits, n):
    """I/2^k (x) Tr_qubits(rho), by explicit index loops."""
    d = 1 << n
    mask = sum(1 << q for q in qubits)
    out = np.zeros_like(rho)
    k = len(qubits)
    for r in range(d):
        for c in range(d):
            if (r & mask) != (c & mask):
                continue
            # (I (x) Tr rho)[r, c] = sum over the traced bits u of rho[rest_r|u, rest_c|u] / 2^k
            s = 0
            for u in range(1 << k):
                bits = sum(((u >> j) & 1) << q for j, q in enumerate(qubits))
                s += rho[(r & ~mask) | bits, (c & ~mask) | bits]
            out[r, c] = s / (1 << k)
    return out


def test_depolarize_matches_definition():
    n = 3
    rho = W.random_density_matrix(n, seed=2)
    p = 0.37
    for qs, name in (([1], "depolarize"), ([2, 0], "depolarize2")):
        want = (1 - p) * rho + p * _ptrace_reinsert(rho, qs, n)
        got = dense.dm_apply(rho, (name, tuple(qs), (p,)), n)
        assert close(got, want, 1e-14)


def test_channel_special_cases():
    n = 2
    rho = W.random_density_matrix(n, seed=3)
    out = dense.dm_apply(dense.dm_apply(rho, ("amp_damp", (0,), (1.0,)), n), ("amp_damp", (1,), (1.0,)), n)
    assert close(out, dense.dm_initial(n))
    out = dense.dm_apply(rho, ("depolarize2", (0, 1), (1.0,)), n)
    assert close(out, np.eye(4) / 4)
    one = dense.dm_apply(W.random_density_matrix(1, seed=4), ("depolarize", (0,), (1.0,)), 1)
    assert close(one, np.eye(2) / 2)
    # the two depolarising conventions differ (the convention is a real choice)
    r1 = apply1(G.kraus_depolarize(0.3), from_bloch([0, 0, 1]))
    r2 = apply1(G.kraus_depolarize_nc(0.3), from_bloch([0, 0, 1]))
    assert not close(r1, r2, 1e-3)


def test_dm_pipeline_invariants():
    n = 5
    ops = W.noisy_tfim_circuit(n, steps=4)
    rho = dense.dm_initial(n)
    prev_purity = 1.0
    for op in ops:
        rho = dense.dm_apply(rho, op, n)
        pur = dense.dm_purity(rho)
        if op[0] in ("depolarize", "depolarize2", "phase_damp"):   # unital: purity cannot grow
            assert pur <= prev_purity + 1e-14
        elif op[0] not in ("amp_damp",):                         # unitary: purity kept
            assert abs(pur - prev_purity) < 1e-13
        prev_purity = pur
    assert abs(dense.dm_trace(rho) - 1) < 1e-13
    assert close(rho, rho.conj().T)
    assert np.linalg.eigvalsh(rho).min() >= -1e-12
    assert prev_purity <= 1 + 1e-13


def test_noise_free_dm_equals_sv():
    n = 5
    g = W.tfim_trotter_circuit(n, steps=3) + W.random_gate_list(n, 20, seed=9)
    psi = dense.sv_run(g, n)
    rho = dense.dm_run(g, n)
    assert close(rho, np.outer(psi, psi.conj()), 1e-13)
    assert close(np.diag(rho).real, np.abs(psi) ** 2, 1e-13)
    rho1 = tensor.dm_run(g, n)
    assert close(rho1, rho, 1e-13)


def test_tier1_dm_matches_tier0():
    n = 4
    rng = np.random.default_rng(6)
    ops = W.with_noise(W.random_gate_list(n, 25, seed=6), W.NoiseSpec(0.05, 0.07, 0.03, 0.1))
    rho0 = W.random_density_matrix(n, seed=6)
    a = dense.dm_run(ops, n, rho0)
    b = tensor.dm_run(ops, n, rho0)
    assert close(a, b, 1e-13)
    for x, z, _ in W.random_pauli_sum(n, 10, seed=7):
        assert abs(dense.dm_expval(a, x, z, n) - tensor.dm_expval(a, x, z, n)) < 1e-13
    assert abs(dense.dm_purity(a) - tensor.dm_purity(a)) < 1e-13


def test_superop_groups_match_kraus():
    """vec(sum K rho K^dag) restricted to one group equals (sum K (x) K*) applied
    to the group's entries (row-major vec, row bits above column bits)."""
    n = 3
    rho = W.random_density_matrix(n, seed=8)
    vec = rho.reshape(-1)
    for qs, name, p in (([1], "amp_damp", 0.3), ([2, 0], "depolarize2", 0.2), ([0], "phase_damp", 0.4)):
        ks = G.channel_kraus(name, (p,))
        want = dense.dm_apply(rho, (name, tuple(qs), (p,)), n).reshape(-1)
        vq = list(qs) + [q + n for q in qs]       # column bits first, then row bits
        mask = sum(1 << q for q in vq)
        base = np.array([i for i in range(1 << (2 * n)) if i & mask == 0])
        idx = tensor.group_indices(base, vq)
        got = tensor.groups_apply(vec[idx], tensor.dm_superop(ks))
        assert close(got, want[idx], 1e-14)


def test_pauli_error_convention():
    """The uniform-Pauli-error form (1-p) rho + p/(4^k-1) sum_{P != I} P rho P
    is the replacement form at p' = p 4^k / (4^k - 1), because the Pauli
    twirl sum_P P rho P over all 4^k Paulis is 2^k Tr(rho) I; on one qubit
    the Bloch vector shrinks by 1 - 4p/3."""
    rng = np.random.default_rng(9)
    for p in (0.0, 0.01, 0.3, 0.75):
        r = rng.standard_normal(3)
        r *= 0.9 / np.linalg.norm(r)
        assert close(bloch(apply1(G.kraus_depolarize_nc(p), from_bloch(r))), (1 - 4 * p / 3) * r)
        n = 3
        rho = W.random_density_matrix(n, seed=int(100 * p) + 1)
        for name, qs, scale in (("depolarize", (1,), 4 / 3), ("depolarize2", (2, 0), 16 / 15)):
            a = dense.dm_apply(rho, (name + "_nc", qs, (p,)), n)
            b = dense.dm_apply(rho, (name, qs, (p * scale,)), n)
            assert close(a, b, 1e-13)


def choi(channel, n=1):
    """Choi matrix sum_{ij} |i><j| (x) E(|i><j|) of a one-qubit map."""
    out = np.zeros((4, 4), dtype=np.complex128)
    for i in range(2):
        for j in range(2):
            E = np.zeros((2, 2), dtype=np.complex128)
            E[i, j] = 1
            out += np.kron(E, channel(E))
    return out


def test_thermal_relaxation_definition():
    """Closed forms of the relaxation map: identity at t = 0, relaxation to
    |0><0| for t >> T1, Bloch components z -> 1 - (1 - z) e^{-t/T1} and
    x, y -> x e^{-t/T2}; trace preserving; completely positive exactly when
    T2 <= 2 T1 (the Choi matrix turns indefinite beyond), which is the
    physical range; on a qubit of a larger register it acts on that qubit
    only."""
    rho = from_bloch([0.3, -0.4, 0.5])
    assert close(dense.thermal_relax(rho, 0, 50.0, 70.0, 0.0, 1), rho)
    assert close(dense.thermal_relax(rho, 0, 1.0, 1.5, 200.0, 1), from_bloch([0, 0, 1]), 1e-12)
    t1, t2, t = 40.0, 55.0, 7.0
    out = bloch(dense.thermal_relax(rho, 0, t1, t2, t, 1))
    e1, e2 = math.exp(-t / t1), math.exp(-t / t2)
    assert close(out, [0.3 * e2, -0.4 * e2, 1 - (1 - 0.5) * e1])
    ch = lambda E: dense.thermal_relax(E, 0, t1, t2, t, 1)
    assert np.min(np.linalg.eigvalsh(choi(ch))) >= -1e-14
    bad = lambda E: dense.thermal_relax(E, 0, 10.0, 30.0, 5.0, 1)      # T2 > 2 T1
    assert np.min(np.linalg.eigvalsh(choi(bad))) < -1e-6
    n = 3
    rho3 = W.random_density_matrix(n, seed=8)
    out3 = dense.thermal_relax(rho3, 1, t1, t2, t, n)
    assert abs(np.trace(out3) - 1) <= 1e-14
    # the partial trace over qubit 1 is unchanged (the map is local and trace preserving)
    red_in = rho3.reshape(2, 2, 2, 2, 2, 2)
    red_out = out3.reshape(2, 2, 2, 2, 2, 2)
    assert close(np.einsum("ajbcjd->abcd", red_in), np.einsum("ajbcjd->abcd", red_out), 1e-14)

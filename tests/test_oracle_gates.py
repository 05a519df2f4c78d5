"""Pins of the oracle's gate matrices and of its Kronecker embedding against
closed forms, scipy's matrix exponential and brute-force index
construction (none of which the oracle itself uses)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense, gates as G, tensor
import workloads as W

TOL = 1e-15 * 16


def close(a, b, tol=1e-14):
    return np.max(np.abs(np.asarray(a) - np.asarray(b))) <= tol


@pytest.mark.parametrize("name", sorted(W.GATE_ARITY))
def test_unitary(name):
    nq, npar = W.GATE_ARITY[name]
    rng = np.random.default_rng(3)
    for _ in range(5):
        p = rng.uniform(-7, 7, size=npar)
        U = G.gate_matrix(name, list(range(nq)), p)
        assert close(U.conj().T @ U, np.eye(1 << nq))


@pytest.mark.parametrize("pname", ["X", "Y", "Z"])
def test_rotations_match_expm(pname):
    P = G.PAULI[pname]
    for th in (-2.3, 0.0, 0.4, 1.7, 5.9):
        want = sla.expm(-0.5j * th * P)
        got = G.one_qubit_matrix("r" + pname.lower(), (th,))
        assert close(got, want)


def test_fixed_gate_identities():
    H = G.one_qubit_matrix("h")
    assert close(H, np.array([[1, 1], [1, -1]]) / math.sqrt(2))
    assert close(H @ H, np.eye(2))
    S, T = G.one_qubit_matrix("s"), G.one_qubit_matrix("t")
    assert close(S @ S, G.Z)
    assert close(T @ T, S)
    assert close(G.one_qubit_matrix("sdg"), S.conj().T)
    assert close(G.one_qubit_matrix("tdg"), T.conj().T)
    assert close(G.one_qubit_matrix("rx", (2 * math.pi,)), -np.eye(2))


def test_u3_special_cases():
    for th in (0.3, 1.1, 2.9):
        assert close(G.u3(th, -math.pi / 2, math.pi / 2), G.one_qubit_matrix("rx", (th,)))
        assert close(G.u3(th, 0, 0), G.one_qubit_matrix("ry", (th,)))
        assert close(G.u3(0, 0, th), np.diag([1, np.exp(1j * th)]))
    assert close(G.u3(math.pi / 2, 0, math.pi), G.one_qubit_matrix("h"))


def _perm_matrix(fn, k):
    m = np.zeros((1 << k, 1 << k), dtype=complex)
    for u in range(1 << k):
        m[fn(u), u] = 1
    return m


def test_two_qubit_gates_brute_force():
    # index u = bit(q0) + 2 bit(q1); CX control q0, target q1
    cx = _perm_matrix(lambda u: u ^ ((u & 1) << 1), 2)
    assert close(G.gate_matrix("cx", [0, 1]), cx)
    swap = _perm_matrix(lambda u: ((u & 1) << 1) | (u >> 1), 2)
    assert close(G.gate_matrix("swap", [0, 1]), swap)
    assert close(G.gate_matrix("cz", [0, 1]), np.diag([1, 1, 1, -1]))
    cx2 = G.gate_matrix("cx", [0, 1])
    assert close(cx2 @ cx2, np.eye(4))
    for th in (0.2, 1.3, -2.2):
        rzz = G.gate_matrix("rzz", [0, 1], (th,))
        assert close(rzz, sla.expm(-0.5j * th * np.kron(G.Z, G.Z)))
        # CX (I (x) RZ on target) CX = RZZ
        rz_t = np.kron(G.one_qubit_matrix("rz", (th,)), np.eye(2))
        assert close(cx @ rz_t @ cx, rzz)


def test_matrix_terms_roundtrip():
    rng = np.random.default_rng(11)
    for _ in range(10):
        m = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        assert close(G.small_matrix(G.matrix_terms(m, [3, 1]), [3, 1]), m, 1e-13)


def _brute_embed(m, qubits, n):
    """U[i', i] = m[u(i'), u(i)] when i, i' agree outside `qubits`."""
    k = len(qubits)
    mask = sum(1 << q for q in qubits)
    U = np.zeros((1 << n, 1 << n), dtype=complex)

    def u_of(i):
        return sum(((i >> q) & 1) << j for j, q in enumerate(qubits))
    for i in range(1 << n):
        for ip in range(1 << n):
            if (i & ~mask) == (ip & ~mask):
                U[ip, i] = m[u_of(ip), u_of(i)]
    return U


def test_embedding_matches_brute_force():
    n = 4
    rng = np.random.default_rng(5)
    for g in W.random_gate_list(n, 40, seed=5):
        name, qs, ps = g
        want = _brute_embed(G.gate_matrix(name, qs, ps), qs, n)
        assert close(dense.embed_gate(name, qs, ps, n), want), g
    for _ in range(6):
        qs = list(rng.choice(n, 2, replace=False))
        m = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        assert close(dense.embed_matrix(m, qs, n), _brute_embed(m, qs, n), 1e-13)


def test_bell_ghz_and_bit_flips():
    psi = dense.sv_run([("h", (0,), ()), ("cx", (0, 1), ())], 2)
    assert close(psi, np.array([1, 0, 0, 1]) / math.sqrt(2))
    for n in (3, 5):
        g = [("h", (0,), ())] + [("cx", (i, i + 1), ()) for i in range(n - 1)]
        psi = dense.sv_run(g, n)
        want = np.zeros(1 << n, complex)
        want[0] = want[-1] = 1 / math.sqrt(2)
        assert close(psi, want)
    n = 5
    for q in range(n):
        psi = dense.sv_run([("x", (q,), ())], n)
        assert close(psi, dense.basis_state(n, 1 << q))
    # CX permutes basis states by j -> j ^ (bit_c(j) << t)
    for j in range(1 << n):
        for c, t in ((0, 3), (4, 1), (2, 3)):
            out = dense.sv_run([("cx", (c, t), ())], n, dense.basis_state(n, j))
            assert close(out, dense.basis_state(n, j ^ (((j >> c) & 1) << t)))


def test_pauli_expvals_closed_forms():
    n = 3
    for j in range(1 << n):
        e = dense.basis_state(n, j)
        for q in range(n):
            assert close(dense.sv_expval(e, 0, 1 << q, n), (-1) ** ((j >> q) & 1))
            assert close(dense.sv_expval(e, 1 << q, 0, n), 0)
    plus = dense.sv_run([("h", (1,), ())], n)
    assert close(dense.sv_expval(plus, 2, 0, n), 1)
    plus_i = dense.sv_run([("h", (1,), ()), ("s", (1,), ())], n)
    assert close(dense.sv_expval(plus_i, 2, 2, n), 1)   # <Y_1> = 1
    for x in range(1 << n):
        for z in range(1 << n):
            P = dense.pauli_operator(x, z, n)
            assert close(P, P.conj().T)
            assert close(P @ P, np.eye(1 << n))


def test_tier1_matches_tier0_sv():
    n = 5
    psi0 = W.random_state(n, seed=1)
    g = W.random_gate_list(n, 60, seed=2)
    a = dense.sv_run(g, n, psi0)
    b = tensor.sv_run(g, n, psi0)
    assert close(a, b, 1e-13)
    for x, z, _ in W.random_pauli_sum(n, 20, seed=3):
        assert abs(dense.sv_expval(a, x, z, n) - tensor.sv_expval(a, x, z, n)) < 1e-13


def test_groups_apply_matches_embedding():
    n = 5
    rng = np.random.default_rng(8)
    psi = W.random_state(n, seed=4)
    for qs in ([0], [3], [4, 1], [0, 2], [2, 4, 0, 3]):
        k = len(qs)
        m = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        full = _brute_embed(m, qs, n) @ psi
        mask = sum(1 << q for q in qs)
        base = np.array([i for i in range(1 << n) if i & mask == 0])
        idx = tensor.group_indices(base, qs)
        got = tensor.groups_apply(psi[idx], m)
        assert close(got, full[idx], 1e-13)

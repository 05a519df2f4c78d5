"""Pins of the oracle's TFIM references and VQE energy/gradients: exact
diagonalisation vs the free-fermion closed form, hand-derived small cases,
Trotter terms vs scipy's matrix exponential, first-order Trotter error
scaling against exact dynamics (the "exact result" of Fig. 3), reflection
symmetry, the variational bound, and parameter shift vs finite differences."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense, tensor, tfim, vqe
import workloads as W


def test_free_fermion_matches_ed():
    rng = np.random.default_rng(0)
    for n in range(1, 9):
        J = rng.uniform(0.2, 2.0, size=max(n - 1, 1))
        h = rng.uniform(0.2, 2.0, size=n)
        assert abs(tfim.ground_energy_ed(n, J, h) - tfim.ground_energy_free_fermion(n, J, h)) < 1e-12


def test_small_chain_closed_forms():
    for J, h in ((1.0, 1.0), (0.7, 1.3), (2.0, 0.1)):
        assert abs(tfim.ground_energy_ed(1, J, h) + h) < 1e-14
        assert abs(tfim.ground_energy_ed(2, J, h) + math.sqrt(J * J + 4 * h * h)) < 1e-13


def test_trotter_terms_are_exact_exponentials():
    n, J, h, dt = 4, 1.0, 0.8, 0.1
    for i in range(n - 1):
        ZZ = dense.pauli_operator(0, (1 << i) | (1 << (i + 1)), n)
        got = dense.embed_gate("rzz", (i, i + 1), (2 * J * dt,), n)
        assert np.abs(got - sla.expm(-1j * J * dt * ZZ)).max() < 1e-13
    for i in range(n):
        Xi = dense.pauli_operator(1 << i, 0, n)
        got = dense.embed_gate("rx", (i,), (2 * h * dt,), n)
        assert np.abs(got - sla.expm(-1j * h * dt * Xi)).max() < 1e-13


def test_trotter_error_is_first_order():
    n, t = 6, 2.0
    psi0 = dense.basis_state(n)
    # the circuit evolves under +J ZZ + h X, i.e. H(J=-1, h=-1) of tfim.hamiltonian
    exact = tfim.exact_evolution(n, t, psi0, J=-1.0, h=-1.0)
    errs = []
    for steps in (20, 40, 80):
        psi = tensor.sv_run(W.tfim_trotter_circuit(n, 1.0, 1.0, t / steps, steps), n)
        errs.append(np.linalg.norm(psi - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.9 < r1 < 2.1 and 1.9 < r2 < 2.1, errs
    # the sign of H does not change <Z_i> from a real start state
    ex2 = tfim.exact_evolution(n, t, psi0, J=1.0, h=1.0)
    for i in range(n):
        assert abs(dense.sv_expval(exact, 0, 1 << i, n) - dense.sv_expval(ex2, 0, 1 << i, n)) < 1e-12


def test_reflection_symmetry_config1():
    n = 10
    psi = tensor.sv_run(W.tfim_trotter_circuit(n, 1.0, 1.0, 0.1, 20), n)
    for i in range(n):
        j = n - 1 - i
        for x, z in ((0, 1), (1, 0)):
            a = tensor.sv_expval(psi, x << i, z << i, n).real
            b = tensor.sv_expval(psi, x << j, z << j, n).real
            assert abs(a - b) < 1e-12
    assert abs(np.vdot(psi, psi) - 1) < 1e-13


def test_vqe_energy_special_cases_and_bound():
    n, L = 4, 2
    prog = W.hea_ansatz(n, L)
    terms = W.tfim_hamiltonian(n, 1.0, 0.9)
    P = W.ansatz_num_params(prog)
    assert P == 2 * n * L
    assert abs(vqe.energy(prog, np.zeros(P), terms, n) + (n - 1)) < 1e-13
    E0 = tfim.ground_energy_free_fermion(n, 1.0, 0.9)
    rng = np.random.default_rng(1)
    H = tfim.hamiltonian(n, 1.0, 0.9)
    for _ in range(5):
        th = rng.uniform(-math.pi, math.pi, P)
        e = vqe.energy(prog, th, terms, n)
        assert e >= E0 - 1e-12
        psi = vqe.state(prog, th, n)
        assert abs(e - np.vdot(psi, H @ psi).real) < 1e-12


def test_parameter_shift_vs_finite_difference():
    n, L = 4, 2
    prog = W.hea_ansatz(n, L)
    terms = W.tfim_hamiltonian(n, 1.0, 1.2)
    th = np.random.default_rng(2).uniform(-math.pi, math.pi, W.ansatz_num_params(prog))
    gs = vqe.grad_parameter_shift(prog, th, terms, n)
    gf = vqe.grad_finite_difference(prog, th, terms, n)
    assert np.abs(gs - gf).max() < 1e-6
    assert np.abs(gs).max() > 1e-2     # non-trivial


def test_last_layer_rz_gradient_vanishes_at_zero():
    n, L = 4, 3
    prog = W.hea_ansatz(n, L)
    terms = W.tfim_hamiltonian(n, 1.0, 0.7)
    P = W.ansatz_num_params(prog)
    g = vqe.grad_parameter_shift(prog, np.zeros(P), terms, n)
    last_rz = [(L - 1) * 2 * n + n + q for q in range(n)]
    assert np.abs(g[last_rz]).max() < 1e-12

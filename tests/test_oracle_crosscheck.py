"""Convention regression and gradient pins of the oracle.

1. Cross-check values computed before the oracle existed, by a separate
   throwaway numpy implementation that used the same conventions (qubit q is
   bit q; rotations exp(-i theta P / 2); first-order Trotter order RZZ on
   (0,1)..(n-2,n-1) then RX on 0..n-1; noise after each gate in the order
   depolarising, amplitude damping, phase damping; Qiskit's depolarising
   convention unless stated).  They are not printed in the paper; they fix the
   conventions of the TFIM workloads of Sec. III (Fig. 3 setting) and of its
   noise model, to the digits given:
   * pure TFIM, n=10, J=h=1, dt=0.1, 20 steps: <Z_i>, <X_i> for i = 0..4
     (the chain is reflection symmetric, so i = 5..9 mirror them);
   * noisy TFIM, n=8, 10 steps, depolarising 1e-3, amplitude damping 1e-3,
     phase damping 2e-3, two-qubit depolarising 1e-2: purity and every
     Tr(rho Z_i); and with the (1-p) rho + p/(4^k-1) sum P rho P convention,
     purity and Tr(rho Z_0).
2. Parameter-shift gradients of programs with shared parameters, RX and RZZ
   generators (the VQE of Sec. III, Fig. 4, on programs other than the
   hardware-efficient ansatz): closed forms on one and two qubits, and central
   finite differences on a four-qubit program.
"""
import math

import numpy as np
import pytest

from oracle import dense, loops, tensor, vqe
import workloads as W

CFG1_Z = [0.05939344, -0.07882894, 0.01371098, 0.08443755, 0.09390115]
CFG1_X = [0.49368819, 0.47332008, 0.43126711, 0.42434675, 0.47822951]
CFG2_PURITY = 0.3072127634
CFG2_Z = [-0.03062288, 0.2404609, 0.25875507, 0.25861381, 0.2586127, 0.2586556, 0.23908888, -0.03063369]
CFG2_NC_PURITY = 0.2802557527
CFG2_NC_Z0 = -0.03082144


def _tol(printed: float) -> float:
    """Half a unit in the last printed digit (8 or 10 decimals)."""
    s = repr(printed).split(".")[1]
    return 0.5 * 10.0 ** (-len(s)) + 1e-15


def test_config1_pure_tfim_values():
    n = 10
    gates = W.tfim_trotter_circuit(n, 1.0, 1.0, 0.1, 20)
    for psi, ev in ((tensor.sv_run(gates, n), tensor.sv_expval), (loops.sv_run(gates, n), loops.sv_expval)):
        for i in range(n):
            m = min(i, n - 1 - i)
            z = ev(psi, 0, 1 << i, n).real
            x = ev(psi, 1 << i, 0, n).real
            assert abs(z - CFG1_Z[m]) <= _tol(CFG1_Z[m]), (i, z)
            assert abs(x - CFG1_X[m]) <= _tol(CFG1_X[m]), (i, x)


def test_config2_noisy_tfim_values_qiskit_convention():
    n = 8
    ops = W.noisy_tfim_circuit(n, 10)
    rho = dense.dm_run(ops, n)
    assert abs(dense.dm_trace(rho) - 1) < 1e-13
    assert abs(dense.dm_purity(rho) - CFG2_PURITY) <= _tol(CFG2_PURITY)
    for i in range(n):
        z = dense.dm_expval(rho, 0, 1 << i, n).real
        assert abs(z - CFG2_Z[i]) <= _tol(CFG2_Z[i]), (i, z)
    rho2 = loops.dm_run(ops, n)
    assert abs(loops.dm_purity(rho2, n) - CFG2_PURITY) <= _tol(CFG2_PURITY)


def test_config2_noisy_tfim_values_pauli_convention():
    n = 8
    conv = {"depolarize": "depolarize_nc", "depolarize2": "depolarize2_nc"}
    ops = [(conv.get(name, name), q, p) for name, q, p in W.noisy_tfim_circuit(n, 10)]
    rho = dense.dm_run(ops, n)
    assert abs(dense.dm_purity(rho) - CFG2_NC_PURITY) <= _tol(CFG2_NC_PURITY)
    z0 = dense.dm_expval(rho, 0, 1, n).real
    assert abs(z0 - CFG2_NC_Z0) <= _tol(CFG2_NC_Z0)
    # the two conventions differ at the 1e-2 level in these outputs
    assert abs(CFG2_NC_PURITY - CFG2_PURITY) > 1e-2


# ---------------------------------------------------------------- gradients
A = W.AnsatzGate


@pytest.mark.parametrize("theta", [0.3, -1.1, 2.5])
def test_shared_rx_closed_form(theta):
    """RX(t) twice on |0>: E = <Z> = cos 2t, dE/dt = -2 sin 2t (both
    occurrences of the shared parameter contribute)."""
    prog = [A("rx", (0,), 0), A("rx", (0,), 0)]
    terms = [(0, 1, 1.0)]
    assert abs(vqe.energy(prog, [theta], terms, 1) - math.cos(2 * theta)) < 1e-14
    g = vqe.grad_parameter_shift(prog, [theta], terms, 1)
    assert abs(g[0] + 2 * math.sin(2 * theta)) < 1e-14


@pytest.mark.parametrize("theta", [0.4, -2.0])
def test_rzz_closed_form(theta):
    """RZZ(t) on |++>: <X_0> = cos t, so dE/dt = -sin t; a second RZZ(t) on
    the same pair makes it cos 2t and -2 sin 2t."""
    prep = [A("h", (0,), -1), A("h", (1,), -1)]
    terms = [(1, 0, 1.0)]
    prog = prep + [A("rzz", (0, 1), 0)]
    assert abs(vqe.energy(prog, [theta], terms, 2) - math.cos(theta)) < 1e-14
    assert abs(vqe.grad_parameter_shift(prog, [theta], terms, 2)[0] + math.sin(theta)) < 1e-14
    prog2 = prog + [A("rzz", (0, 1), 0)]
    assert abs(vqe.grad_parameter_shift(prog2, [theta], terms, 2)[0] + 2 * math.sin(2 * theta)) < 1e-14


def _generic_program():
    """Four qubits, parameters shared between RX, RY, RZ and RZZ gates, with
    fixed H and CX between them."""
    return [A("h", (0,), -1), A("rx", (0,), 0), A("rzz", (0, 1), 1), A("ry", (1,), 0),
            A("rzz", (1, 2), 1), A("rx", (2,), 2), A("cx", (2, 3), -1), A("rz", (3,), 3),
            A("rx", (3,), 2), A("rzz", (2, 3), 3), A("h", (1,), -1), A("rx", (1,), 4),
            A("rzz", (0, 3), 4), A("ry", (2,), 1)]


def test_shared_parameters_shift_vs_finite_difference():
    n = 4
    prog = _generic_program()
    terms = W.tfim_hamiltonian(n, 1.0, 0.8) + [(0b0101, 0b0011, 0.3)]
    rng = np.random.default_rng(21)
    for _ in range(3):
        th = rng.uniform(-math.pi, math.pi, 5)
        gs = vqe.grad_parameter_shift(prog, th, terms, n)
        gf = vqe.grad_finite_difference(prog, th, terms, n)
        assert np.abs(gs - gf).max() < 1e-6
        assert np.abs(gs).min() > 1e-4      # every shared parameter contributes


def test_loops_tier_energy_matches_tensor_tier():
    """The VQE oracle switches to the C-loop tier above 12 qubits; both tiers
    give the same energy and gradient components on the same program."""
    n, L = 9, 2
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=2)
    terms = W.tfim_hamiltonian(n, 1.0, h)
    psi_t = tensor.sv_run(vqe.bind(prog, theta[0]), n)
    psi_l = loops.sv_run(vqe.bind(prog, theta[0]), n)
    assert np.abs(psi_t - psi_l).max() < 1e-14
    assert abs(tensor.sv_pauli_sum(psi_t, terms, n) - loops.sv_pauli_sum(psi_l, terms, n)) < 1e-13

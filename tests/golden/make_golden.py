"""Writes the stored expected values under tests/golden/ by calling only the
oracle (no value here comes from the HIP engine).

    python tests/golden/make_golden.py

tfim_sv_n10.json  -- TFIM Trotter circuit (Sec. III, Fig. 3 setting), n=10,
                     J=h=1, dt=0.1, 20 steps from |0...0>: <Z_i>, <X_i>.
tfim_dm_n8.json   -- the same circuit with the Sec. III noise model
                     (depolarising 1e-3, amplitude damping 1e-3, phase
                     damping 2e-3 after 1-qubit gates; 2-qubit depolarising
                     1e-2 after 2-qubit gates), n=8, 10 steps: Tr(rho Z_i),
                     purity, trace.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dense, tensor  # noqa: E402
import workloads as W  # noqa: E402


def main():
    n = 10
    psi = dense.sv_run(W.tfim_trotter_circuit(n, 1.0, 1.0, 0.1, 20), n)
    out = {"n": n, "J": 1.0, "h": 1.0, "dt": 0.1, "steps": 20,
           "Z": [dense.sv_expval(psi, 0, 1 << i, n).real for i in range(n)],
           "X": [dense.sv_expval(psi, 1 << i, 0, n).real for i in range(n)]}
    with open(os.path.join(HERE, "tfim_sv_n10.json"), "w") as f:
        json.dump(out, f, indent=1)
    n = 8
    rho = dense.dm_run(W.noisy_tfim_circuit(n, 10), n)
    out = {"n": n, "steps": 10, "noise": {"p1": 1e-3, "gamma": 1e-3, "lam": 2e-3, "p2": 1e-2},
           "Z": [dense.dm_expval(rho, 0, 1 << i, n).real for i in range(n)],
           "purity": dense.dm_purity(rho), "trace": dense.dm_trace(rho).real}
    with open(os.path.join(HERE, "tfim_dm_n8.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()

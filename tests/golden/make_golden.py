"""Writes the stored expected values under tests/golden/ by calling only the
oracle (no value here comes from the HIP engine).

    python tests/golden/make_golden.py [small] [dm14] [vqe20] [sv30]

With no argument only the small files are written.  The large ones run the
C-loop tier of the oracle on the full-size workloads and take minutes
(vqe20), about an hour (dm14) or more (sv30, which needs 17 GB of memory);
each prints its progress.

tfim_sv_n10.json  -- TFIM Trotter circuit (Sec. III, Fig. 3 setting), n=10,
                     J=h=1, dt=0.1, 20 steps from |0...0>: <Z_i>, <X_i>.
tfim_dm_n8.json   -- the same circuit with the Sec. III noise model
                     (depolarising 1e-3, amplitude damping 1e-3, phase
                     damping 2e-3 after 1-qubit gates; 2-qubit depolarising
                     1e-2 after 2-qubit gates), n=8, 10 steps: Tr(rho Z_i),
                     purity, trace.
tfim_dm_n14.json  -- the same noisy circuit at n=14, 10 steps: Tr(rho Z_i),
                     purity, trace, and 256 sampled entries of rho.
vqe_n20_L8.json   -- the VQE of Sec. III (Fig. 4): Ising energy of the
                     hardware-efficient ansatz at n=20, L=8 for selected
                     vectors of the seeded B=256 batch, and parameter-shift
                     gradient components of two of them.
brickwork_n30_seed0.json -- the depth-40 brickwork random circuit (stand-in
                     for the deep-circuit benchmark of Fig. 5) at n=30, seed
                     0: <Z_i> for every qubit, the norm, and 1024 sampled
                     amplitudes of the final state.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dense, loops, vqe  # noqa: E402
import workloads as W  # noqa: E402


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def small():
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


def dm14():
    n, steps = 14, 10
    ops = W.noisy_tfim_circuit(n, steps)
    rho = loops.dm_zero(n)
    t0 = time.time()
    for i, op in enumerate(ops):
        loops.dm_apply(rho, op, n)
        if i % 50 == 0:
            log(f"[dm14] op {i}/{len(ops)} {op[0]} {op[1]} at {time.time() - t0:.0f}s")
    D = 1 << n
    rng = np.random.default_rng(14)
    rows = rng.integers(0, D, size=256)
    cols = rng.integers(0, D, size=256)
    cols[:32] = rows[:32]                     # some diagonal entries
    tr = loops.dm_trace(rho, n)
    out = {"n": n, "steps": steps, "noise": {"p1": 1e-3, "gamma": 1e-3, "lam": 2e-3, "p2": 1e-2},
           "Z": [loops.dm_expval(rho, 0, 1 << i, n).real for i in range(n)],
           "Z_imag": [loops.dm_expval(rho, 0, 1 << i, n).imag for i in range(n)],
           "purity": loops.dm_purity(rho, n), "trace": [tr.real, tr.imag],
           "samples": [[int(r), int(c), float(rho[r, c].real), float(rho[r, c].imag)]
                       for r, c in zip(rows, cols)]}
    with open(os.path.join(HERE, "tfim_dm_n14.json"), "w") as f:
        json.dump(out, f, indent=1)
    log(f"[dm14] done in {time.time() - t0:.0f}s")


VQE_ENERGY_VECTORS = [0, 1, 2, 3, 64, 127, 128, 200, 254, 255]
VQE_GRAD_VECTORS = [0, 255]
# first-layer RY/RZ on the end and middle qubits, middle-layer RY/RZ, last-layer RY/RZ
VQE_GRAD_PARAMS = [0, 10, 19, 20, 30, 39, 120, 150, 160, 179, 280, 299, 300, 310, 319]


def vqe20():
    n, L, B = 20, 8, 256
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=B)
    terms = W.tfim_hamiltonian(n, 1.0, h)
    t0 = time.time()
    energies = {}
    for b in VQE_ENERGY_VECTORS:
        energies[str(b)] = vqe.energy(prog, theta[b], terms, n)
        log(f"[vqe20] E[{b}] = {energies[str(b)]:.15f} at {time.time() - t0:.0f}s")
    grads = {}
    for b in VQE_GRAD_VECTORS:
        g = vqe.grad_parameter_shift(prog, theta[b], terms, n, params=VQE_GRAD_PARAMS)
        grads[str(b)] = {str(p): float(g[p]) for p in VQE_GRAD_PARAMS}
        log(f"[vqe20] gradient of vector {b} at {time.time() - t0:.0f}s")
    out = {"n": n, "L": L, "B": B, "J": 1.0, "h": h, "seed": 1000 + 10 * n + L,
           "energy": energies, "grad_parameter_shift": grads}
    with open(os.path.join(HERE, "vqe_n20_L8.json"), "w") as f:
        json.dump(out, f, indent=1)


def sv30():
    n, depth, seed = 30, 40, 0
    gates = W.brickwork_circuit(n, depth, seed=seed)
    psi = loops.sv_zero(n)
    t0 = time.time()
    for i, g in enumerate(gates):
        loops.sv_apply(psi, g, n)
        if i % 20 == 0:
            log(f"[sv30] gate {i}/{len(gates)} at {time.time() - t0:.0f}s")
    rng = np.random.default_rng(30)
    idx = np.sort(rng.choice(1 << n, size=1024, replace=False))
    out = {"n": n, "depth": depth, "seed": seed,
           "Z": [loops.sv_expval(psi, 0, 1 << i, n).real for i in range(n)],
           "norm2": float(loops.sv_expval(psi, 0, 0, n).real),
           "samples": [[int(j), float(psi[j].real), float(psi[j].imag)] for j in idx]}
    with open(os.path.join(HERE, "brickwork_n30_seed0.json"), "w") as f:
        json.dump(out, f, indent=1)
    log(f"[sv30] done in {time.time() - t0:.0f}s")


def main():
    which = sys.argv[1:] or ["small"]
    for w in which:
        {"small": small, "dm14": dm14, "vqe20": vqe20, "sv30": sv30}[w]()


if __name__ == "__main__":
    main()

"""CPU FP64 oracle for the SV / DM simulation hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the package
``paper_2401_06861_amd``) imports, links or calls anything here; only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
use it.  It shares no code with the HIP engine: the only common inputs come
from the seeded generators in ``workloads``.

What it computes is fixed by the two simulators the paper describes
(Sec. II: a state-vector simulator and a density-matrix simulator for
noise-aware runs), the noise model of Sec. III (depolarisation and thermal
relaxation, represented here by amplitude + phase damping), the TFIM
magnetisation and VQE energy observables of Sec. III, and the textbook
definitions behind them:

* ``gates``   -- gate matrices and Kraus sets written from their definitions.
* ``dense``   -- tier 0: every operator embedded as a full 2^n x 2^n
                 Kronecker product; psi <- U psi, rho <- sum_k K rho K^dagger,
                 <P> = psi^dagger P psi, Tr(rho P).  Small n only.
* ``tensor``  -- tier 1: the same maths as a contraction over the qubit's
                 tensor axis (no dense 2^n operator), for larger n, plus the
                 per-group form used for sampled checks at full size.
* ``loops``   -- tier 1 again, as plain C index loops (``loops.c``, gcc +
                 OpenMP) for the full-size workloads: a 14-qubit density
                 matrix, a 20-qubit VQE, a 30-qubit state vector.
* ``tfim``    -- exact diagonalisation of the Ising chain and the
                 free-fermion ground energy (the exact reference of Fig. 3).
* ``vqe``     -- VQE energy, parameter-shift and finite-difference
                 gradients.

Parity status: every function is pinned by a ``-m "not gpu"`` test against
something other than itself (closed forms, brute force, ED, invariants);
see tests/test_oracle_*.py.
"""

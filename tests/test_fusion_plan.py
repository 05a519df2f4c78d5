"""Host-side checks of the fusion planner (no device): every gate lands in
exactly one block, a block's tile holds all its gates' qubits and at most k
qubits, gates that share a qubit keep their order across blocks, and the
planner terminates for every width (including k = 6 on wider registers)."""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def nwq():
    from paper_2401_06861_amd import nwq as mod
    return mod


def check_plan(nwq, gates, n, k):
    types, qs, _ = nwq.circuit_arrays(gates)
    nb, bog, masks = nwq.nwq_fusion_plan(n, k, types, qs)
    assert nb >= 1 and len(masks) == nb
    assert np.all((bog >= 0) & (bog < nb))
    for b in range(nb):
        assert bin(masks[b]).count("1") <= max(k, 0) or n <= k
    last = {}
    for i, (name, q, _) in enumerate(gates):
        b = int(bog[i])
        for x in q:
            assert (masks[b] >> x) & 1, (i, name, q, b)
            if x in last:
                assert last[x] <= b, (i, name, q)
            last[x] = b
    return nb


@pytest.mark.parametrize("n", [2, 5, 8, 11, 16, 24, 30])
@pytest.mark.parametrize("k", [6, 7, 8, 10, 12, 13])
def test_random_circuits_plan(nwq, n, k):
    gates = [g for g in W.random_gate_list(n, 300, seed=n * 100 + k)]
    check_plan(nwq, gates, n, k)


@pytest.mark.parametrize("k", [6, 9, 12, 13])
def test_brickwork_plan(nwq, k):
    n = 30
    gates = W.brickwork_circuit(n, 40, seed=0)
    nb = check_plan(nwq, gates, n, k)
    assert nb < len(gates) / (3 if k < 9 else 7)   # fusion actually groups gates


def test_whole_register_in_one_tile(nwq):
    n = 10
    gates = W.tfim_trotter_circuit(n, 1.0, 1.0, 0.1, 20)
    assert check_plan(nwq, gates, n, 12) == 1


def test_plan_rejects_bad_input(nwq):
    types, qs, _ = nwq.circuit_arrays([("cx", (0, 4), ())])
    with pytest.raises(nwq.NwqError):
        nwq.nwq_fusion_plan(4, 8, types, qs)      # qubit 4 out of range
    with pytest.raises(nwq.NwqError):
        nwq.nwq_fusion_plan(8, 5, types, qs)      # width below 6

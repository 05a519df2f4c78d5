"""GPU parity of the density-matrix path (Sec. II DM simulator, Sec. III
noise model) against the oracle: gates on every qubit, every channel,
arbitrary CPTP Kraus sets, the noisy TFIM circuit (n=8, 10 steps) with
Tr(rho Z_i), purity and trace, and error handling.  Max abs entry error of
rho <= 1e-12."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import gates as G, tensor

pytestmark = pytest.mark.gpu
TOL = 1e-12
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def nwq():
    from paper_2401_06861_amd import nwq as mod
    return mod


def maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


@pytest.mark.parametrize("n", [1, 2, 4, 6])
def test_gates_on_every_qubit(nwq, n):
    rng = np.random.default_rng(n)
    rho0 = W.random_density_matrix(n, seed=n)
    st = nwq.DMState(n, reset=False)
    for name, (nq, npar) in sorted(W.GATE_ARITY.items()):
        if nq > n:
            continue
        qsets = [(q,) for q in range(n)] if nq == 1 else list(itertools.permutations(range(n), 2))
        for qs in qsets:
            ps = tuple(float(x) for x in rng.uniform(-math.pi, math.pi, npar))
            st.load(rho0)
            st.apply(name, qs, ps)
            want = tensor.dm_apply(rho0, (name, qs, ps), n)
            assert maxerr(st.numpy(), want) <= TOL, (name, qs)
    st.close()


@pytest.mark.parametrize("n", [1, 3, 5])
def test_channels_on_every_qubit(nwq, n):
    rho0 = W.random_density_matrix(n, seed=10 + n)
    st = nwq.DMState(n, reset=False)
    ops = []
    for q in range(n):
        ops += [("depolarize", (q,), (0.13,)), ("amp_damp", (q,), (0.21,)), ("phase_damp", (q,), (0.37,))]
    for a, b in itertools.permutations(range(n), 2):
        ops.append(("depolarize2", (a, b), (0.29,)))
    for op in ops:
        st.load(rho0)
        st.run([op])
        want = tensor.dm_apply(rho0, op, n)
        assert maxerr(st.numpy(), want) <= TOL, op
    st.close()


def random_kraus(k, count, rng):
    """CPTP set from a random isometry V (count*d x d): K_i = rows block i."""
    d = 1 << k
    A = rng.standard_normal((count * d, d)) + 1j * rng.standard_normal((count * d, d))
    Q, _ = np.linalg.qr(A)
    return [Q[i * d:(i + 1) * d, :] for i in range(count)]


def test_generic_kraus_and_fused_gate_channel_runs(nwq):
    n = 4
    rng = np.random.default_rng(3)
    rho0 = W.random_density_matrix(n, seed=3)
    st = nwq.DMState(n, reset=False)
    for qs, count in (([2], 3), ([0, 3], 5), ([3, 1], 2), ([1], 1)):
        ks = random_kraus(len(qs), count, rng)
        st.load(rho0)
        st.channel(qs, ks)
        want = tensor.dm_kraus(rho0, ks, qs, n)
        assert maxerr(st.numpy(), want) <= TOL, qs
    # gate followed by several channels on the same qubits (one fused pass),
    # then a gate on other qubits (flush), compared op by op
    ops = [("u3", (1,), (0.3, 1.2, -0.4)), ("depolarize", (1,), (0.1,)), ("amp_damp", (1,), (0.2,)),
           ("phase_damp", (1,), (0.3,)), ("rzz", (0, 2), (0.7,)), ("depolarize2", (0, 2), (0.05,)),
           ("cx", (3, 0), ()), ("amp_damp", (2,), (0.5,))]
    st.load(rho0)
    st.run(ops)
    assert maxerr(st.numpy(), tensor.dm_run(ops, n, rho0)) <= TOL
    st.close()


def test_noisy_tfim_n8(nwq):
    n = 8
    ops = W.noisy_tfim_circuit(n, 10)
    want = tensor.dm_run(ops, n)
    gold = json.load(open(os.path.join(HERE, "golden", "tfim_dm_n8.json")))
    st = nwq.DMState(n)
    st.run(ops)
    rho = st.numpy()
    assert maxerr(rho, want) <= TOL
    assert maxerr(rho, rho.conj().T) <= TOL
    Z = st.expvals(W.single_site_terms(n, "Z"))
    assert maxerr(Z, gold["Z"]) <= TOL
    tr, tri = st.trace()
    assert abs(tr - 1) <= TOL and abs(tri) <= 1e-13
    assert abs(st.purity() - gold["purity"]) <= TOL
    # one-body terms with their imaginary parts: Hermitian rho gives |Im| <= 1e-13
    terms = W.single_site_terms(n, "Z") + W.single_site_terms(n, "X") + W.single_site_terms(n, "Y")
    zc = st.expvals_complex(terms)
    wantc = np.array([tensor.dm_expval(want, x, z, n) for x, z, _ in terms])
    assert maxerr(zc.real, wantc.real) <= TOL
    assert float(np.max(np.abs(zc.imag))) <= 1e-13
    st.close()


def test_dm_pauli_terms(nwq):
    n = 5
    rho = W.random_density_matrix(n, seed=21)
    terms = W.random_pauli_sum(n, 30, seed=22)
    st = nwq.DMState(n, reset=False)
    st.load(rho)
    got = st.expvals(terms)
    want = np.array([tensor.dm_expval(rho, x, z, n).real for x, z, _ in terms])
    assert maxerr(got, want) <= TOL
    assert abs(st.pauli_sum(terms) - sum(c * w for (_, _, c), w in zip(terms, want))) <= TOL
    # complex values on a matrix that is not Hermitian: the imaginary parts are summed, not assumed
    g = np.random.default_rng(23)
    m = (g.standard_normal((1 << n, 1 << n)) + 1j * g.standard_normal((1 << n, 1 << n))) / (1 << n)
    st.load(m)
    gotc = st.expvals_complex(terms)
    wantc = np.array([tensor.dm_expval(m, x, z, n) for x, z, _ in terms])
    assert maxerr(gotc, wantc) <= TOL
    assert float(np.max(np.abs(wantc.imag))) > 1e-3
    st.close()


def test_noise_free_dm_equals_sv_outer_product(nwq):
    n = 6
    gates = W.random_gate_list(n, 60, seed=5)
    sv = nwq.SVState(n)
    sv.run(gates)
    psi = sv.numpy()
    dm = nwq.DMState(n)
    dm.run(gates)
    assert maxerr(dm.numpy(), np.outer(psi, psi.conj())) <= TOL
    sv.close()
    dm.close()


@pytest.mark.parametrize("nt", [0, 1])
def test_superop_launch_shapes(nwq, nt):
    """Noisy 1- and 2-qubit gates with each hint on both superoperator
    kernels, on low and high qubits."""
    n = 7
    rho0 = W.random_density_matrix(n, seed=40 + nt)
    st = nwq.DMState(n, reset=False)
    for cls in (6, 7):
        nwq.nwq_set_launch(st.h, cls, -1, 1, nt)
        assert nwq.nwq_get_launch(st.h, cls, 2) == (1, nt)
    ops = [("u3", (0,), (0.3, 1.2, -0.4)), ("depolarize", (0,), (0.05,)), ("amp_damp", (6,), (0.1,)),
           ("rzz", (1, 5), (0.7,)), ("depolarize2", (1, 5), (0.02,)), ("cx", (6, 2), ()), ("depolarize2", (2, 6), (0.03,))]
    st.load(rho0)
    st.run(ops)
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    assert maxerr(st.numpy(), want) <= TOL
    with pytest.raises(nwq.NwqError):
        nwq.nwq_set_launch(st.h, 7, -1, 4, nt)
    st.close()


@pytest.mark.parametrize("n", [6, 7])
def test_low_qubit_superoperators_every_shape(nwq, n):
    """Noisy 1q gates on qubits 0..2 (4x4 superoperator on bits q and q + n:
    the lane-exchange kernel) and a noisy 2q gate, under every groups-per-
    thread and hint choice of the 1q superoperator class."""
    rho0 = W.random_density_matrix(n, seed=60 + n)
    st = nwq.DMState(n, reset=False)
    ops = []
    for q in range(3):
        ops += [("u3", (q,), (0.3 + q, 1.2, -0.4)), ("depolarize", (q,), (0.05,)), ("amp_damp", (q,), (0.1,)),
                ("phase_damp", (q,), (0.07,))]
    ops += [("rzz", (0, 1), (0.7,)), ("depolarize2", (0, 1), (0.02,))]
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    for ppt in (1, 2, 4, 8):
        for nt in (0, 1):
            nwq.nwq_set_launch(st.h, 6, -1, ppt, nt)
            st.load(rho0)
            st.run(ops)
            assert maxerr(st.numpy(), want) <= TOL, (ppt, nt)
    st.close()


@pytest.mark.parametrize("n", [5, 6, 7])
def test_split_workgroup_superoperators(nwq, n):
    """Noisy 1q gates on every qubit (the 4x4 superoperator on bits q and
    q + n) under the split-workgroup shapes 32, 64 and 128 of the 1q
    superoperator class, and noisy 2q gates under shapes 64 and 128 of the 2q
    class (16 x 16; 512 threads with two members each, or 1024 with one), with every flag (hint, XCD-contiguous order; n=7
    has grids of a multiple of 8 workgroups for every shape, n=6 for shapes
    32 and 64, n=5 for none, which keeps dispatch order), plus a noisy 2q
    gate.  Qubits whose bit q is below 3 with q + n at or above 6 keep the
    lane-exchange kernel."""
    rho0 = W.random_density_matrix(n, seed=80 + n)
    st = nwq.DMState(n, reset=False)
    ops = []
    for q in range(n):
        ops += [("u3", (q,), (0.3 + q, 1.2, -0.4)), ("depolarize", (q,), (0.05,)), ("amp_damp", (q,), (0.1,))]
    for a, b in [(0, n - 1), (2, 1), (n - 1, 3), (n - 2, n - 3)]:
        ops += [("rzz", (a, b), (0.7,)), ("depolarize2", (a, b), (0.02,))]
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    for cls, ppt in [(6, 32), (6, 64), (6, 128), (7, 64), (7, 128)]:
        for nt in (0, 1, 2, 3):
            nwq.nwq_set_launch(st.h, cls, -1, ppt, nt)
            assert nwq.nwq_get_launch(st.h, cls, 1) == (ppt, nt)
            st.load(rho0)
            st.run(ops)
            assert maxerr(st.numpy(), want) <= TOL, (cls, ppt, nt)
        nwq.nwq_set_launch(st.h, cls, -1, 1, 1)
    st.close()


@pytest.mark.parametrize("n", [8, 9])
def test_staged_two_qubit_superoperators(nwq, n):
    """Noisy 2q gates whose superoperator has its two lower bits inside a
    256-entry run and the lowest below 3 (qubit pairs with both qubits below
    8, lowest below 3: the LDS-staged 16 x 16 kernel), in both operator
    orders and with each hint, plus one pair outside that case."""
    rho0 = W.random_density_matrix(n, seed=70 + n)
    st = nwq.DMState(n, reset=False)
    ops = []
    for a, b in [(0, 1), (1, 0), (1, 2), (2, 5), (0, 7), (6, 2), (3, 4), (0, n - 1)]:
        ops += [("rzz", (a, b), (0.7,)), ("cx", (a, b), ()), ("depolarize2", (a, b), (0.02,))]
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    # the staged kernel (shape 1) and, on the same pairs, the split-workgroup
    # kernels the tuner compares with it (shapes 64, 128, both workgroup orders)
    for ppt, flags in ((1, 0), (1, 1), (64, 1), (128, 1), (64, 3), (128, 3)):
        nwq.nwq_set_launch(st.h, 7, -1, ppt, flags)
        st.load(rho0)
        st.run(ops)
        assert maxerr(st.numpy(), want) <= TOL, (ppt, flags)
    st.close()


@pytest.mark.parametrize("n", [6, 7])
def test_pauli_pattern_two_qubit_superoperators(nwq, n):
    """Noisy 2q gates whose superoperator only scales the coherences and mixes
    the four populations (RZZ or CZ, then depolarising noise in either
    convention: the compact Pauli-pattern pass), interleaved with ones that do
    not (CX or SWAP before the noise: the dense 16 x 16), on pairs that take
    the LDS-staged kernel, the one-group-per-thread kernel and, under shapes
    64 and 128, the split-workgroup kernels, in both operator orders."""
    rho0 = W.random_density_matrix(n, seed=90 + n)
    st = nwq.DMState(n, reset=False)
    pairs = [(0, 1), (1, 0), (2, 5), (5, 2), (4, 5), (0, 3), (3, n - 1), (n - 1, 1)]
    ops = []
    for i, (a, b) in enumerate(pairs):
        noise = ("depolarize2", (a, b), (0.02 + 0.01 * i,)) if i % 3 else ("depolarize2_nc", (a, b), (0.05,))
        ops += [("rzz", (a, b), (0.7 + 0.1 * i,)) if i % 2 else ("cz", (a, b), ()), noise]   # Pauli pattern
        ops += [("cx", (a, b), ()) if i % 2 else ("swap", (a, b), ()), noise]                   # dense
    ops += [("depolarize2", (2, 3), (0.04,))]   # the channel alone
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    for ppt, flags in ((1, 0), (1, 1), (64, 1), (128, 1), (64, 3), (128, 3)):
        nwq.nwq_set_launch(st.h, 7, -1, ppt, flags)
        st.load(rho0)
        st.run(ops)
        assert maxerr(st.numpy(), want) <= TOL, (ppt, flags)
    st.close()


@pytest.mark.parametrize("n,k,kernel", [(4, 8, 1), (5, 8, 2), (6, 10, 1), (7, 12, 1), (7, 8, 0), (8, 12, 2)])
def test_fused_superoperator_queue(nwq, n, k, kernel):
    """With fusion on, the 1q superoperators (gate + channels, 4x4 on bits
    q and q + n) queue up and run as fused blocks over the 2n bits of vec(rho)
    when a 2q superoperator or a read needs the state; every fused kernel
    matches the oracle.  Reads in the middle, switching fusion off with work
    queued, and a reset that drops queued work are covered too."""
    rng = np.random.default_rng(500 + n)
    rho0 = W.random_density_matrix(n, seed=90 + n)
    ops = W.noisy_tfim_circuit(n, 2)
    for _ in range(3 * n):   # 1q noisy gates on random qubits
        q = (int(rng.integers(n)),)
        ops += [("u3", q, tuple(float(x) for x in rng.uniform(-3, 3, 3))), ("depolarize", q, (0.03,)),
                ("amp_damp", q, (0.05,))]
    ops += [("cx", (0, n - 1), ()), ("depolarize2", (0, n - 1), (0.01,)), ("ry", (n - 1,), (0.4,))]
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    st = nwq.DMState(n, reset=False)
    st.set_fusion(k)
    nwq.nwq_set_fusion_kernel(st.h, kernel)
    st.load(rho0)
    half = len(ops) // 2
    st.run(ops[:half])
    mid = rho0
    for op in ops[:half]:
        mid = tensor.dm_apply(mid, op, n)
    assert maxerr(st.numpy(), mid) <= TOL            # a read runs the queue
    st.run(ops[half:])
    assert maxerr(st.numpy(), want) <= TOL
    assert nwq.nwq_fusion_stats(st.h)[0] >= 1
    st.load(rho0)
    st.run(ops[:half])
    st.set_fusion(0)                                 # queued work runs before fusion goes off
    st.run(ops[half:])
    assert maxerr(st.numpy(), want) <= TOL
    st.set_fusion(k)
    st.load(rho0)
    st.run([("u3", (0,), (0.3, 0.2, 0.1)), ("depolarize", (0,), (0.2,)), ("rx", (1,), (0.5,))])
    st.reset()                                       # drops the queued work
    zero = np.zeros_like(rho0)
    zero[0, 0] = 1.0
    assert maxerr(st.numpy(), zero) == 0.0
    st.close()


@pytest.mark.parametrize("n,k", [(4, 8), (6, 10), (7, 12), (9, 12)])
def test_fused_queue_two_qubit_superoperators(nwq, n, k):
    """With the 4-register-bit kernel, 2q superoperators (16x16 on bits q0,
    q1, q0 + n, q1 + n) queue with the 1q ones and run inside the fused
    blocks: random pairs in both operator orders, dense and diagonal gates
    with one- and two-qubit channels, against the oracle; switching the
    fused kernel with 2q work queued runs it first."""
    rng = np.random.default_rng(700 + 10 * n + k)
    rho0 = W.random_density_matrix(n, seed=30 + n)
    ops = []
    for _ in range(4 * n):
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        kind = int(rng.integers(4))
        if kind == 0:
            ops += [("rzz", (a, b), (float(rng.uniform(-3, 3)),)), ("depolarize2", (a, b), (0.02,))]
        elif kind == 1:
            ops += [("cx", (a, b), ()), ("depolarize2", (b, a), (0.01,))]
        elif kind == 2:
            ops += [("u3", (a,), tuple(float(x) for x in rng.uniform(-3, 3, 3))), ("amp_damp", (a,), (0.04,))]
        else:
            ops += [("swap", (a, b), ()), ("phase_damp", (b,), (0.05,))]
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    st = nwq.DMState(n, reset=False)
    st.set_fusion(k)
    nwq.nwq_set_fusion_kernel(st.h, 1)
    st.load(rho0)
    st.run(ops)
    assert maxerr(st.numpy(), want) <= TOL
    assert nwq.nwq_fusion_stats(st.h)[0] >= 1
    st.load(rho0)
    half = len(ops) // 2
    st.run(ops[:half])
    nwq.nwq_set_fusion_kernel(st.h, 2)               # queued 16x16 work runs first, on the 4-bit kernel
    st.run(ops[half:])
    assert maxerr(st.numpy(), want) <= TOL
    st.close()


@pytest.mark.parametrize("n,k,c", [(7, 8, 0), (7, 8, 6), (8, 9, 6), (9, 12, 0), (9, 12, 3), (9, 12, 5),
                                   (9, 12, 8), (9, 13, 4), (10, 10, 0)])
def test_fused_queue_low_tile_bits(nwq, n, k, c):
    """Fused DM blocks under each low-tile-bit setting (0: the default 4 for
    density matrices; the width clamps it to [k - 8, k - 2]): noisy 1q and 2q
    gates on every qubit against the oracle.  Where the width leaves fewer
    than four bits above the low ones (k=8 or 9 with 6 low bits), a 2q
    superoperator whose four bits all lie above them cannot share a block,
    so it runs as its own pass after the queue."""
    rng = np.random.default_rng(900 + 10 * n + k + c)
    rho0 = W.random_density_matrix(n, seed=60 + n)
    ops = []
    for q in range(n):
        ops += [("u3", (q,), tuple(float(x) for x in rng.uniform(-3, 3, 3))), ("amp_damp", (q,), (0.03,))]
    for a in range(n - 1):
        ops += [("rzz", (a, a + 1), (float(rng.uniform(-3, 3)),)), ("depolarize2", (a, a + 1), (0.02,))]
        ops += [("cx", (a + 1, a), ()), ("phase_damp", (a,), (0.04,))]
    ops += [("swap", (n - 1, n - 2), ()), ("depolarize2", (n - 2, n - 1), (0.01,))]
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    st = nwq.DMState(n, reset=False)
    st.set_fusion(k)
    nwq.nwq_set_fusion_kernel(st.h, 1)
    nwq.nwq_set_fusion_lowbits(st.h, c)
    st.load(rho0)
    st.run(ops)
    assert maxerr(st.numpy(), want) <= TOL
    assert nwq.nwq_fusion_stats(st.h)[0] >= 1
    st.load(rho0)                                    # changing the setting runs the queued work first
    half = len(ops) // 2
    st.run(ops[:half])
    nwq.nwq_set_fusion_lowbits(st.h, 6 if c != 6 else 0)
    st.run(ops[half:])
    assert maxerr(st.numpy(), want) <= TOL
    for bad in (-1, 1, 2, 9):
        with pytest.raises(nwq.NwqError):
            nwq.nwq_set_fusion_lowbits(st.h, bad)
    st.close()


def test_fused_queue_long_circuit_runs_in_pieces(nwq):
    """A noisy circuit with more queued superoperators than one queue run
    holds (1 MiB of matrices: 256 two-qubit ones) and no read in between runs
    in pieces and still matches the oracle."""
    n = 5
    rng = np.random.default_rng(811)
    rho0 = W.random_density_matrix(n, seed=812)
    ops = []
    for _ in range(330):
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        ops += [("rzz", (a, b), (float(rng.uniform(-3, 3)),)), ("depolarize2", (a, b), (0.002,)),
                ("ry", (a,), (float(rng.uniform(-3, 3)),))]
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    st = nwq.DMState(n, reset=False)
    st.set_fusion(8)
    nwq.nwq_set_fusion_kernel(st.h, 1)
    st.load(rho0)
    st.run(ops)
    assert maxerr(st.numpy(), want) <= TOL
    st.close()


def test_depolarizing_conventions(nwq):
    """Both depolarising conventions on one and two qubits against the
    oracle's Kraus sets, alone and fused after a gate."""
    n = 4
    rho0 = W.random_density_matrix(n, seed=77)
    st = nwq.DMState(n, reset=False)
    ops = [("depolarize_nc", (2,), (0.2,)), ("h", (1,), ()), ("depolarize_nc", (1,), (0.05,)),
           ("depolarize2_nc", (3, 0), (0.3,)), ("cz", (0, 2), ()), ("depolarize2_nc", (0, 2), (0.01,)),
           ("depolarize", (1,), (0.1,))]
    st.load(rho0)
    st.run(ops)
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    assert maxerr(st.numpy(), want) <= TOL
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_depolarize_ex(st.h, (0,), 0.1, 2)
    assert e.value.code == nwq.NWQ_EINVAL
    st.close()


def test_thermal_relaxation_against_definition(nwq):
    """The engine's amplitude + phase damping mapping of (T1, T2, t) against
    the oracle's relaxation map written from its definition, fused after
    gates, on several qubits and durations, including T2 = 2 T1."""
    n = 4
    rho0 = W.random_density_matrix(n, seed=91)
    st = nwq.DMState(n, reset=False)
    ops = [("thermal_relax", (0,), (50.0, 70.0, 3.0)), ("h", (2,), ()), ("thermal_relax", (2,), (30.0, 60.0, 9.0)),
           ("cx", (2, 3), ()), ("thermal_relax", (3,), (80.0, 20.0, 25.0)), ("thermal_relax", (1,), (5.0, 4.0, 0.0))]
    st.load(rho0)
    st.run(ops)
    want = rho0
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    assert maxerr(st.numpy(), want) <= TOL
    for bad in ((10.0, 25.0, 1.0), (0.0, 1.0, 1.0), (10.0, 5.0, -1.0)):
        with pytest.raises(nwq.NwqError) as e:
            nwq.nwq_thermal_relax(st.h, 0, *bad)
        assert e.value.code == nwq.NWQ_EINVAL
    st.close()
    sv = nwq.SVState(2)
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_thermal_relax(sv.h, 0, 10.0, 10.0, 1.0)
    assert e.value.code == nwq.NWQ_EKIND
    sv.close()


def test_dm_errors(nwq):
    n = 3
    rho0 = W.random_density_matrix(n, seed=2)
    st = nwq.DMState(n, reset=False)
    st.load(rho0)
    bad = [np.eye(2) * 0.9]                    # not trace preserving
    with pytest.raises(nwq.NwqError) as e:
        st.channel([0], bad)
    assert e.value.code == nwq.NWQ_ENOTCPTP
    with pytest.raises(nwq.NwqError) as e:
        st.channel([0, 0], [np.eye(4)])
    assert e.value.code == nwq.NWQ_EDUP
    with pytest.raises(nwq.NwqError) as e:
        st.channel([3], [np.eye(2)])
    assert e.value.code == nwq.NWQ_ERANGE
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_depolarize(st.h, [0], 1.5)
    assert e.value.code == nwq.NWQ_EINVAL
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_set_fusion(st.h, 5)
    assert e.value.code == nwq.NWQ_EINVAL
    assert maxerr(st.numpy(), rho0) == 0.0
    st.close()

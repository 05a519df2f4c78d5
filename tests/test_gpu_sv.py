"""GPU parity of the state-vector path against the oracle: every gate kind
on every qubit (and many qubit pairs) from random states, arbitrary
matrices, whole circuits unfused and fused, the TFIM circuit of Sec. III
(config n=10), Pauli-term reductions, and error handling.  Max abs
amplitude error <= 1e-12, expectation values <= 1e-12."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import dense, tensor

pytestmark = pytest.mark.gpu
TOL = 1e-12
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def nwq():
    from paper_2401_06861_amd import nwq as mod
    return mod


def maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def qubit_choices(n, nq, rng):
    if nq == 1:
        return [(q,) for q in range(n)]
    pairs = list(itertools.permutations(range(n), 2))
    if len(pairs) <= 24:
        return pairs
    pick = [(0, 1), (1, 0), (0, n - 1), (n - 1, 0), (n - 2, n - 1), (n - 1, n - 2)]
    pick += [pairs[i] for i in rng.choice(len(pairs), 12, replace=False)]
    return pick


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11, 14, 17])
def test_every_gate_every_qubit(nwq, n):
    rng = np.random.default_rng(100 + n)
    psi0 = W.random_state(n, seed=n)
    st = nwq.SVState(n)
    for name, (nq, npar) in sorted(W.GATE_ARITY.items()):
        if nq > n:
            continue
        for qs in qubit_choices(n, nq, rng):
            ps = tuple(float(x) for x in rng.uniform(-math.pi, math.pi, npar))
            st.load(psi0)
            st.apply(name, qs, ps)
            want = tensor.sv_apply(psi0, (name, qs, ps), n)
            err = maxerr(st.numpy(), want)
            assert err <= TOL, (name, qs, ps, err)
    st.close()


def test_apply_matrix_general(nwq):
    n = 7
    rng = np.random.default_rng(7)
    psi0 = W.random_state(n, seed=3)
    st = nwq.SVState(n)
    for qs in ([0], [6], [3], [0, 1], [1, 0], [6, 2], [2, 6], [5, 4]):
        k = len(qs)
        m = (rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))) / 2
        st.load(psi0)
        st.apply_matrix(qs, m)
        want = tensor.apply_op(psi0, m, qs, n)
        assert maxerr(st.numpy(), want) <= TOL, qs
    st.close()


def test_tfim_config1_state_and_magnetisation(nwq):
    n = 10
    gates = W.tfim_trotter_circuit(n, 1.0, 1.0, 0.1, 20)
    want = dense.sv_run(gates, n)
    gold = json.load(open(os.path.join(HERE, "golden", "tfim_sv_n10.json")))
    st = nwq.SVState(n)
    for mode in ("per_gate", "circuit", "fused"):
        st.reset()
        st.set_fusion(12 if mode == "fused" else 0)
        if mode == "per_gate":
            st.run(gates)
        else:
            st.run_circuit(gates)
        psi = st.numpy()
        assert maxerr(psi, want) <= TOL, mode
        Z = st.expvals(W.single_site_terms(n, "Z"))
        X = st.expvals(W.single_site_terms(n, "X"))
        assert maxerr(Z, gold["Z"]) <= TOL and maxerr(X, gold["X"]) <= TOL, mode
    st.close()


@pytest.mark.parametrize("n,k", [(11, 0), (11, 6), (11, 8), (11, 11), (11, 13), (16, 8), (16, 10), (16, 12),
                                 (18, 12), (18, 13)])
def test_random_circuits_fused_and_unfused(nwq, n, k):
    gates = W.random_gate_list(n, 250, seed=n * 31 + k)
    psi0 = W.random_state(n, seed=k + 1)
    want = tensor.sv_run(gates, n, psi0)
    st = nwq.SVState(n, reset=False)
    st.load(psi0)
    st.set_fusion(k)
    st.run_circuit(gates)
    err = maxerr(st.numpy(), want)
    blocks, fused = nwq.nwq_fusion_stats(st.h)
    assert err <= TOL, (n, k, err, blocks)
    if k:
        assert blocks >= 1 and fused == len([g for g in gates if g[0] != "id"])
    st.close()


def test_brickwork_fused_equals_unfused(nwq):
    n = 16
    gates = W.brickwork_circuit(n, 12, seed=1)
    psi0 = W.random_state(n, seed=9)
    want = tensor.sv_run(gates, n, psi0)
    outs = []
    for k in (0, 9, 12):
        st = nwq.SVState(n, reset=False)
        st.load(psi0)
        st.set_fusion(k)
        st.run_circuit(gates)
        outs.append(st.numpy())
        st.close()
    for o in outs:
        assert maxerr(o, want) <= TOL
    assert maxerr(outs[1], outs[0]) <= TOL and maxerr(outs[2], outs[0]) <= TOL


@pytest.mark.parametrize("n", [1, 2, 4, 9, 12, 13, 16, 19])
def test_pauli_terms_and_sums(nwq, n):
    psi = W.random_state(n, seed=50 + n)
    terms = W.random_pauli_sum(n, 40, seed=n)
    # add terms whose flipped bits are all high, all low, and single-site ones
    terms += [(1 << (n - 1), 0, 0.3), (0, (1 << n) - 1, -0.2), ((1 << n) - 1, (1 << n) - 1, 0.7)]
    terms += [(1 << i, 0, 1.0) for i in range(n)] + [(0, 1 << i, 1.0) for i in range(n)]
    st = nwq.SVState(n, reset=False)
    st.load(psi)
    got = st.expvals(terms)
    want = np.array([tensor.sv_expval(psi, x, z, n).real for x, z, _ in terms])
    assert maxerr(got, want) <= TOL
    total = st.pauli_sum(terms)
    assert abs(total - sum(c * w for (_, _, c), w in zip(terms, want))) <= TOL
    assert abs(st.purity() - 1.0) <= TOL
    # deterministic: same value bit for bit on a repeat
    assert np.array_equal(st.expvals(terms), got)
    # complex form: the same real parts, imaginary parts 0 (Hermitian P; the oracle's within 1e-13)
    gotc = st.expvals_complex(terms)
    assert np.array_equal(gotc.real, got) and not gotc.imag.any()
    wanti = np.array([tensor.sv_expval(psi, x, z, n).imag for x, z, _ in terms])
    assert float(np.max(np.abs(wanti))) <= 1e-13
    st.close()


@pytest.mark.parametrize("n", [3, 11, 14])
def test_diagonal_terms_streaming_pass(nwq, n):
    """Z strings (no flipped bits) run in streaming passes of up to 16
    consecutive terms: runs longer than 16, runs cut by terms with flips, and
    z masks over the thread, entry and chunk bit fields of that pass (bits
    0-7, 8-10 and 11 up) all match the oracle."""
    rng = np.random.default_rng(7 + n)
    psi = W.random_state(n, seed=60 + n)
    full = (1 << n) - 1
    terms = [(0, int(rng.integers(1, full + 1)), 1.0) for _ in range(21)]
    terms += [(1 << (n // 2), 1, 1.0)]
    terms += [(0, 1 << q, 1.0) for q in range(n)] + [(0, full, 1.0), (0, full & 0x700, 1.0), (0, full & ~0xFF, 1.0)]
    terms += [(3 & full, 0, 1.0)] + [(0, int(rng.integers(1, full + 1)), 1.0) for _ in range(5)]
    st = nwq.SVState(n, reset=False)
    st.load(psi)
    got = st.expvals(terms)
    want = np.array([tensor.sv_expval(psi, x, z, n).real for x, z, _ in terms])
    assert maxerr(got, want) <= TOL
    assert np.array_equal(st.expvals(terms), got)
    st.close()


def test_tfim_energy_matches_dense(nwq):
    n = 9
    terms = W.tfim_hamiltonian(n, 1.0, 0.8)
    psi = W.random_state(n, seed=4)
    st = nwq.SVState(n, reset=False)
    st.load(psi)
    want = dense.sv_pauli_sum(psi, terms, n)
    assert abs(st.pauli_sum(terms) - want) <= 1e-10
    st.close()


def test_errors_leave_state_unchanged(nwq):
    n = 4
    psi = W.random_state(n, seed=1)
    st = nwq.SVState(n, reset=False)
    st.load(psi)
    cases = [(("h", [4], ()), nwq.NWQ_ERANGE), (("cx", [1, 1], ()), nwq.NWQ_EDUP),
             (("rx", [0], ()), nwq.NWQ_EINVAL), (("h", [0, 1], ()), nwq.NWQ_EINVAL),
             ((99, [0], ()), nwq.NWQ_EINVAL), (("rz", [0], (float("nan"),)), nwq.NWQ_EINVAL)]
    for (g, q, p), code in cases:
        with pytest.raises(nwq.NwqError) as e:
            nwq.nwq_apply_gate(st.h, g, q, p)
        assert e.value.code == code, (g, q)
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_amp_damp(st.h, 0, 0.1)
    assert e.value.code == nwq.NWQ_EKIND
    with pytest.raises(nwq.NwqError) as e:   # one bad gate in a circuit: nothing runs
        st.run_circuit([("h", (0,), ()), ("x", (7,), ())])
    assert e.value.code == nwq.NWQ_ERANGE
    assert np.array_equal(st.numpy(), psi)
    st.close()


def test_owned_allocation_and_reset(nwq):
    h = nwq.nwq_sv_create(5)
    out = np.empty(32, dtype=np.complex128)
    nwq.nwq_get_state(h, out)
    assert out[0] == 1 and np.count_nonzero(out) == 1
    nwq.nwq_apply_gate(h, "x", [3])
    nwq.nwq_get_state(h, out)
    assert out[8] == 1 and np.count_nonzero(out) == 1
    kind, n, ptr = nwq.nwq_info(h)
    assert kind == nwq.KIND_SV and n == 5 and ptr != 0
    nwq.nwq_reset(h)
    nwq.nwq_get_state(h, out)
    assert out[0] == 1 and np.count_nonzero(out) == 1
    nwq.nwq_destroy(h)


@pytest.mark.parametrize("n", [3, 10, 13])
def test_every_launch_shape_matches_oracle(nwq, n):
    """Each kernel class under every (groups per thread, non-temporal) shape,
    on low and high target bits, including blocks that are only partly filled
    (small n)."""
    psi0 = W.random_state(n, seed=70 + n)
    st = nwq.SVState(n, reset=False)
    ops = {1: [("u3", (n - 1,), (0.3, 1.1, -0.7)), ("ry", (0,), (0.4,)), ("h", (2,), ())],
           2: [("rz", (n // 2,), (0.9,)), ("rzz", (0, 1), (0.3,)), ("t", (n - 1,), ())],
           3: [("cx", (0, n - 1), ()), ("x", (1,), ()), ("swap", (n - 1, n - 2), ()), ("x", (n - 2,), ())]}
    m2 = np.array([[0.6, 0.8j, 0, 0.1], [0.2, -0.3, 0.5j, 0], [0, 0.4, 0.1 - 0.2j, 0.7], [0.3j, 0, 0.2, -0.5]])
    for cls in (1, 2, 3, 4):
        for ppt in {1: (1, 2, 4, 8, 16, 32, 64, 128), 3: (1, 2, 4, 8, 16, 32, 64, 128),
                    4: (1, 2, 4, 8, 32, 64, 128)}.get(cls, (1, 2, 4, 8, 16)):
            for nt in ((0, 1, 2, 3) if ppt >= 32 or (cls == 2 and ppt == 1) else (0, 1)):
                nwq.nwq_set_launch(st.h, cls, -1, ppt, nt)
                st.load(psi0)
                if cls == 4:
                    st.apply_matrix([1, n - 1], m2)
                    st.apply_matrix([0, 2], m2)
                    want = tensor.apply_op(tensor.apply_op(psi0, m2, [1, n - 1], n), m2, [0, 2], n)
                else:
                    st.run(ops[cls])
                    want = tensor.sv_run(ops[cls], n, psi0)
                assert maxerr(st.numpy(), want) <= TOL, (cls, ppt, nt)
    st.close()


@pytest.mark.parametrize("n", [8, 10, 12])
def test_lane_exchange_kernels(nwq, n):
    """Dense 1q gates on every target (LDS partner exchange on targets 0..8),
    and gates whose bits are all lane bits (below 6, the lower below 3) with
    lane exchanges: X on targets 0..2, CX and SWAP on every
    ordered pair of bits 0..5 with a bit below 3 (DPP partners at distance
    1, 2, 4, 8 and ds_bpermute otherwise; whole-line and masked stores), under
    every entries-per-thread and hint choice, and with one entry per thread in
    XCD-contiguous workgroup order (flags 2 and 3; n=12 has grids of a
    multiple of 8 workgroups, smaller n fall back to dispatch order)."""
    psi0 = W.random_state(n, seed=90 + n)
    st = nwq.SVState(n, reset=False)
    ops = [("u3", (q,), (0.3 + q, 1.1, -0.7)) for q in range(n)] + [("x", (q,), ()) for q in range(3)]
    for a, b in itertools.permutations(range(6), 2):
        if min(a, b) < 3:
            ops.append(("cx", (a, b), ()))
            ops.append(("swap", (a, b), ()))
    for ppt in (1, 2, 4, 16, 32):
        for nt in ((0, 1, 2, 3) if ppt >= 32 else (0, 1)):
            nwq.nwq_set_launch(st.h, 1, -1, ppt, nt)
            nwq.nwq_set_launch(st.h, 3, -1, ppt, nt)
            st.load(psi0)
            state = psi0
            for op in ops:
                st.apply(*op)
                state = tensor.sv_apply(state, op, n)
                err = maxerr(st.numpy(), state)
                assert err <= TOL, (op, ppt, nt, err)
    st.close()


@pytest.mark.parametrize("n", [8, 11])
def test_lane_exchange_dense_4x4(nwq, n):
    """Dense 4x4 operators with one bit below 3 and the other at or above 6
    (the lane-exchange 4x4 kernel, either bit first in operator order), under
    every entries-per-thread and hint choice."""
    rng = np.random.default_rng(300 + n)
    psi0 = W.random_state(n, seed=80 + n)
    st = nwq.SVState(n, reset=False)
    pairs = [(lo, hi) for lo in range(3) for hi in (6, n - 1)] + [(hi, lo) for lo in range(3) for hi in (6, n - 1)]
    mats = [rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)) for _ in pairs]
    for ppt in (1, 2, 4, 8):
        for nt in (0, 1):
            nwq.nwq_set_launch(st.h, 4, -1, ppt, nt)
            st.load(psi0)
            state = psi0
            for qs, m in zip(pairs, mats):
                st.apply_matrix(list(qs), m)
                state = tensor.apply_op(state, m, list(qs), n)
                err = maxerr(st.numpy(), state) / max(1.0, float(np.max(np.abs(state))))
                assert err <= TOL, (qs, ppt, nt, err)
    st.close()


def test_launch_shape_buckets(nwq):
    """Different shapes in the three target buckets are kept apart and give
    the oracle's result on a circuit touching all of them."""
    n = 14
    st = nwq.SVState(n, reset=False)
    for cls in (1, 2, 3, 4):
        shapes = [(1, 0), (8, 1), (16 if cls != 4 else 2, 1)]
        for b, (ppt, nt) in enumerate(shapes):
            nwq.nwq_set_launch(st.h, cls, b, ppt, nt)
        for b, shape in enumerate(shapes):
            assert nwq.nwq_get_launch(st.h, cls, b) == shape
    gates = W.random_gate_list(n, 300, seed=11)
    psi0 = W.random_state(n, seed=12)
    st.load(psi0)
    st.run_circuit(gates)
    assert maxerr(st.numpy(), tensor.sv_run(gates, n, psi0)) <= TOL
    for bad in ((1, 3, 4, 0), (1, -2, 4, 0), (1, 0, 3, 0), (4, 0, 16, 0), (6, -1, 16, 1)):
        with pytest.raises(nwq.NwqError) as e:
            nwq.nwq_set_launch(st.h, *bad)
        assert e.value.code == nwq.NWQ_EINVAL
    with pytest.raises(nwq.NwqError):
        nwq.nwq_get_launch(st.h, 1, -1)
    st.close()


def test_per_target_launch_shapes(nwq):
    """A shape set for one lowest target bit overrides its bucket's for that
    bit only; nwq_set_launch on the bucket clears it; a circuit run with a
    different shape on every bit matches the oracle."""
    n = 14
    st = nwq.SVState(n, reset=False)
    cycle = [(1, 1), (2, 1), (4, 0), (8, 1), (16, 1), (1, 0), (32, 1), (64, 0), (128, 1), (32, 3), (64, 2), (128, 3)]
    for cls in (1, 2, 3, 4):
        nwq.nwq_set_launch(st.h, cls, -1, 4, 1)
        for q in range(n):
            ppt, nt = cycle[(q + cls) % len(cycle)]
            if cls == 2 and ppt >= 32:
                ppt, nt = 2, nt & 1
            if cls == 4 and ppt == 16:
                ppt = 8
            nwq.nwq_set_launch_target(st.h, cls, q, ppt, nt)
            assert nwq.nwq_get_launch_target(st.h, cls, q) == (ppt, nt)
        assert nwq.nwq_get_launch(st.h, cls, 2) == (4, 1)
    gates = W.random_gate_list(n, 300, seed=21)
    psi0 = W.random_state(n, seed=22)
    st.load(psi0)
    st.run_circuit(gates)
    assert maxerr(st.numpy(), tensor.sv_run(gates, n, psi0)) <= TOL
    nwq.nwq_set_launch(st.h, 1, 1, 2, 0)               # bucket 1 (bits 3..10) back to one shape
    assert nwq.nwq_get_launch_target(st.h, 1, 5) == (2, 0)
    assert nwq.nwq_get_launch_target(st.h, 1, 12) == cycle[(12 + 1) % len(cycle)]
    nwq.nwq_set_launch_target(st.h, 1, 12, 0, 0)       # cleared: the bucket's shape again
    assert nwq.nwq_get_launch_target(st.h, 1, 12) == (4, 1)
    for bad in ((1, 64, 4, 0), (1, -1, 4, 0), (1, 3, 3, 0), (4, 3, 16, 0), (7, 3, 2, 1), (2, 3, 32, 1),
                (1, 3, 4, 2), (3, 3, 16, 3), (1, 3, 64, 4), (3, 3, 32, -1), (7, 3, 32, 1), (4, 3, 8, 3),
                (2, 3, 2, 3), (4, 3, 1, 3), (1, 3, 1, 2)):
        with pytest.raises(nwq.NwqError) as e:
            nwq.nwq_set_launch_target(st.h, *bad)
        assert e.value.code == nwq.NWQ_EINVAL
    st.close()


def test_autotune_keeps_state_and_parity(nwq):
    from paper_2401_06861_amd import autotune
    import tempfile, os
    n = 16
    psi0 = W.random_state(n, seed=5)
    st = nwq.SVState(n, reset=False)
    st.load(psi0)
    cache = os.path.join(tempfile.mkdtemp(), "tune.json")
    chosen = autotune.tune(st.h, reps=2, cache_path=cache)
    assert set(chosen) == {"sv_1q_dense", "sv_diag", "sv_perm", "sv_2q_dense"}
    assert all(set(v) == {"low", "mid", "high"} for v in chosen.values())
    assert np.array_equal(st.numpy(), psi0)           # the tuner's operator pairs are exact
    again = autotune.tune(st.h, reps=2, cache_path=cache)   # from the cache
    shapes = lambda e: {(k, b): tuple(v[:2]) for k, per in e.items() for b, v in per.items()}
    assert shapes(again) == shapes(chosen)
    for (name, b), shape in shapes(chosen).items():
        assert nwq.nwq_get_launch(st.h, autotune.CLASS_IDS[name], nwq.LAUNCH_BUCKETS.index(b)) == shape
    import json
    cached = json.load(open(cache))
    (entry,) = cached.values()
    for name, per_bit in entry["targets"].items():   # per-target shapes restored from the cache
        assert len(per_bit) == n
        for bit, shape in enumerate(per_bit):
            assert nwq.nwq_get_launch_target(st.h, autotune.CLASS_IDS[name], bit) == tuple(shape)
    gates = W.random_gate_list(n, 120, seed=3)
    st.load(psi0)
    st.run_circuit(gates)
    assert maxerr(st.numpy(), tensor.sv_run(gates, n, psi0)) <= TOL
    st.close()
    dm = nwq.DMState(4, reset=False)
    rho0 = W.random_density_matrix(4, seed=1)
    dm.load(rho0)
    ms = nwq.nwq_autotune(dm.h, 2)
    assert set(ms) == {"dm_superop_1q", "dm_superop_2q"}
    assert set(ms["dm_superop_1q"]) == {"low", "mid"} and set(ms["dm_superop_2q"]) == {"low"}   # n = 4
    assert maxerr(dm.numpy(), rho0) == 0.0
    dm.close()


@pytest.mark.parametrize("n,k", [(8, 8), (12, 8), (14, 12), (17, 13), (20, 12)])
def test_register_blocked_fused_kernel(nwq, n, k):
    """Both fused-block kernels (register-blocked phases and one LDS pass per
    gate) against the oracle on a random circuit with every gate kind."""
    gates = W.random_gate_list(n, 300, seed=7 * n + k) + W.brickwork_circuit(n, 6, seed=n)
    psi0 = W.random_state(n, seed=n)
    want = tensor.sv_run(gates, n, psi0)
    outs = {}
    for rb, flags in ((2, 0), (1, 0), (0, 0), (2, 1), (1, 1), (2, 3), (1, 3), (1, 2), (1, 7), (2, 7), (1, 4)):
        st = nwq.SVState(n, reset=False)
        st.load(psi0)
        st.set_fusion(k)
        nwq.nwq_set_fusion_kernel(st.h, rb)
        nwq.nwq_set_fusion_flags(st.h, flags)
        st.run_circuit(gates)
        outs[(rb, flags)] = st.numpy()
        assert maxerr(outs[(rb, flags)], want) <= TOL, (n, k, rb, flags)
        if rb:
            assert nwq.nwq_fusion_phases(st.h) > 0
        st.close()
    # the non-temporal tile accesses change nothing but the cache hints, and
    # the direct first / last phase nothing but where the registers come from
    # (gate products, bit 2, change the rounding: checked against the oracle)
    groups = {}
    for (rb, flags), out in outs.items():
        if rb:
            groups.setdefault((rb, flags & 4), []).append(out)
    for key, same in groups.items():
        for out in same[1:]:
            assert np.array_equal(same[0], out), key


@pytest.mark.parametrize("n,k", [(16, 10), (18, 12), (20, 13)])
def test_fused_low_tile_bits(nwq, n, k):
    """Fused SV blocks under every low-tile-bit setting (clamped to [k - 8,
    k - 2] at width k) and every fused kernel, applied to a random state and
    run from |0...0> (the sparse start), against the oracle; the setting
    changes the grouping into blocks (and so the block count), not the
    result beyond rounding."""
    gates = W.random_gate_list(n, 200, seed=11 * n + k) + W.brickwork_circuit(n, 8, seed=n + 1)
    psi0 = W.random_state(n, seed=n + 2)
    want = tensor.sv_run(gates, n, psi0)
    zero = np.zeros(1 << n, dtype=np.complex128)
    zero[0] = 1.0
    want0 = tensor.sv_run(gates, n, zero)
    blocks = {}
    st = nwq.SVState(n, reset=False)
    st.set_fusion(k)
    for c in (0, 3, 4, 5, 7, 8):
        nwq.nwq_set_fusion_lowbits(st.h, c)
        for rb in (1, 2, 0):
            nwq.nwq_set_fusion_kernel(st.h, rb)
            st.load(psi0)
            st.run_circuit(gates)
            assert maxerr(st.numpy(), want) <= TOL, (c, rb)
            blocks[(c, rb)] = nwq.nwq_fusion_stats(st.h)[0]
            nwq.nwq_run_circuit(st.h, *nwq.circuit_arrays(gates))
            assert maxerr(st.numpy(), want0) <= TOL, (c, rb, "from zero")
    assert len({blocks[(c, 1)] for c in (0, 4, 8)}) > 1   # the setting reaches the planner
    st.close()


def _product_circuits(n, seed):
    """Gate runs that the block products rewrite: U3 pairs around CX on both
    operator orders, diagonal-only runs (RZ, T, S, CZ, RZZ: a diagonal
    product), runs of one-qubit gates on one qubit, and SWAP between dense
    gates."""
    rng = np.random.default_rng(seed)
    ang = lambda k: tuple(float(x) for x in rng.uniform(-3, 3, size=k))
    out = []
    for _ in range(12):
        a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
        out += [("u3", (a,), ang(3)), ("u3", (b,), ang(3)), ("cx", (a, b), ()), ("u3", (a,), ang(3)),
                ("u3", (b,), ang(3)), ("cx", (b, a), ()), ("ry", (a,), ang(1))]
        c, d = (int(x) for x in rng.choice(n, size=2, replace=False))
        out += [("rz", (c,), ang(1)), ("t", (d,), ()), ("cz", (c, d), ()), ("s", (c,), ()),
                ("rzz", (d, c), ang(1)), ("rz", (d,), ang(1))]
        e = int(rng.integers(n))
        out += [("h", (e,), ()), ("rx", (e,), ang(1)), ("u3", (e,), ang(3)), ("x", (e,), ())]
        f, g = (int(x) for x in rng.choice(n, size=2, replace=False))
        out += [("u3", (f,), ang(3)), ("swap", (f, g), ()), ("u3", (g,), ang(3)), ("ry", (f,), ang(1))]
    return out


@pytest.mark.parametrize("n,k", [(10, 8), (14, 12), (20, 13)])
def test_gate_products_in_blocks(nwq, n, k):
    """Fused blocks with gate products (fusion flags bit 2) against the
    oracle, for both register-blocked kernels, on circuits built to exercise
    every product form (dense 4x4, diagonal 4x4, dense and diagonal 2x2)."""
    gates = _product_circuits(n, seed=n + k) + W.brickwork_circuit(n, 4, seed=n + 2)
    psi0 = W.random_state(n, seed=n + 5)
    want = tensor.sv_run(gates, n, psi0)
    for rb in (1, 2):
        for flags in (3, 7):
            st = nwq.SVState(n, reset=False)
            st.load(psi0)
            st.set_fusion(k)
            nwq.nwq_set_fusion_kernel(st.h, rb)
            nwq.nwq_set_fusion_flags(st.h, flags)
            st.run_circuit(gates)
            assert maxerr(st.numpy(), want) <= TOL, (n, k, rb, flags)
            st.close()


def test_fused_identity_only_circuit(nwq):
    """A circuit of identities through the fused path (gate products drop
    them): no error, the state unchanged, no block launched."""
    n = 10
    psi0 = W.random_state(n, seed=3)
    st = nwq.SVState(n, reset=False)
    st.load(psi0)
    st.set_fusion(8)
    st.run_circuit([("id", (q,), ()) for q in range(n)])
    assert np.array_equal(st.numpy(), psi0)
    assert nwq.nwq_fusion_stats(st.h)[0] == 0
    nwq.nwq_run_circuit(st.h, *nwq.circuit_arrays([("id", (0,), ())]))
    out = st.numpy()
    assert out[0] == 1 and np.count_nonzero(out) == 1
    st.close()


@pytest.mark.parametrize("n,k", [(14, 12), (20, 12), (20, 13)])
def test_fused_direct_phase_blocks(nwq, n, k):
    """Blocks whose first and last register phases hold only high tile bits
    (gates on qubits above the low contiguous bits, a single phase moving
    straight between HBM and registers with no LDS at all, and two-phase
    blocks) against the oracle, with direct I/O on and off."""
    rng = np.random.default_rng(n + k)
    hi = list(range(6, n))
    gates = []
    for _ in range(40):
        a, b = rng.choice(hi, size=2, replace=False)
        gates.append(("cx", (int(a), int(b)), ()))
        gates.append(("u3", (int(rng.choice(hi)),), tuple(rng.uniform(-3, 3, size=3))))
    gates += W.brickwork_circuit(n, 3, seed=n + 1)
    psi0 = W.random_state(n, seed=n + 3)
    want = tensor.sv_run(gates, n, psi0)
    outs = {}
    for flags in (1, 3):
        st = nwq.SVState(n, reset=False)
        st.load(psi0)
        st.set_fusion(k)
        nwq.nwq_set_fusion_flags(st.h, flags)
        st.run_circuit(gates)
        outs[flags] = st.numpy()
        assert maxerr(outs[flags], want) <= TOL, (n, k, flags)
        st.close()
    assert np.array_equal(outs[1], outs[3])


def test_fusion_autotuner(nwq):
    """The fusion autotuner times every candidate, keeps the fastest, leaves
    the state at |0...0>, and the circuit then matches the oracle."""
    n = 14
    gates = W.brickwork_circuit(n, 8, seed=2)
    arrays = nwq.circuit_arrays(gates)
    st = nwq.SVState(n)
    k, rb, table = nwq.nwq_autotune_fusion(st.h, *arrays, reps=1)
    assert set(table) == {(0, 0)} | {(w, r) for w in range(6, 14) for r in (0, 1, 2)}
    assert table[(k, rb)] == min(table.values())
    out = st.numpy()
    assert out[0] == 1 and np.count_nonzero(out) == 1
    st.run_circuit(gates)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1
    assert maxerr(st.numpy(), tensor.sv_run(gates, n, psi0)) <= TOL
    blocks, _ = nwq.nwq_fusion_stats(st.h)
    assert (blocks > 0) == (k > 0)
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_autotune_fusion(st.h, *arrays, reps=0)
    assert e.value.code == nwq.NWQ_EINVAL
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_set_fusion_kernel(st.h, 3)
    assert e.value.code == nwq.NWQ_EINVAL
    st.close()
    small = nwq.SVState(7)
    k, rb, table = nwq.nwq_autotune_fusion(small.h, *nwq.circuit_arrays(W.brickwork_circuit(7, 3, seed=1)))
    assert set(table) == {(0, 0), (6, 0), (7, 0)}                   # widths up to n; no register-blocked tiles below 8
    small.close()
    dm = nwq.DMState(3)
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_autotune_fusion(dm.h, *nwq.circuit_arrays([("h", (0,), ())]))
    assert e.value.code == nwq.NWQ_EKIND
    dm.close()


@pytest.mark.parametrize("fuse", [0, 8])
def test_apply_qasm_program(nwq, fuse):
    """An OpenQASM 2.0 program through the library's front-end against the
    oracle's reader and tensor simulator; with fusion the whole program goes
    through the block planner."""
    from oracle import qasm
    n = 11
    text = W.qasm_text(W.random_gate_list(n, 200, seed=31) + W.brickwork_circuit(n, 3, seed=2), n, split=4, seed=1)
    st = nwq.SVState(n)
    st.set_fusion(fuse)
    nwq.nwq_apply_qasm(st.h, text)
    nq, gates = qasm.parse(text)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1
    assert maxerr(st.numpy(), tensor.sv_run(gates, n, psi0)) <= TOL
    if fuse:
        assert nwq.nwq_fusion_stats(st.h)[0] > 0
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_apply_qasm(st.h, "OPENQASM 2.0;\nqreg q[3];\nh q[0];\n")
    assert e.value.code == nwq.NWQ_ERANGE
    st.close()


@pytest.mark.parametrize("size", [1, 1000, 4096 + 3, 1 << 16])
def test_streaming_ceiling_kernels(nwq, size):
    """The yardstick kernels: in-place scale and copy, exact, on sizes that
    do and do not fill whole workgroups (grids with and without XCD order)."""
    import torch
    g = torch.Generator().manual_seed(size)
    x = torch.complex(torch.randn(size, generator=g, dtype=torch.float64),
                      torch.randn(size, generator=g, dtype=torch.float64)).cuda()
    y = torch.empty_like(x)
    nwq.nwq_stream_copy(y, x)
    nwq.nwq_stream_scale(x, 2.0)
    torch.cuda.synchronize()
    assert torch.equal(y * 2.0, x)


@pytest.mark.parametrize("n,k,lead", [(9, 8, 0), (14, 10, 0), (20, 12, 0), (20, 12, 1), (22, 13, 1)])
def test_run_circuit_from_zero(nwq, n, k, lead):
    """nwq_run_circuit (reset, then the circuit; each fused block runs only
    the tiles that can hold nonzero amplitudes: zero on the qubits no earlier
    block touched) equals reset + nwq_apply_circuit bit for bit and the
    oracle, for every fused kernel and unfused, on a state that held other
    values before.  lead = 1 starts with gates on a few high qubits, so the
    next blocks' supports are partial."""
    gates = []
    if lead:
        hi = list(range(n - 5, n))
        gates += [("h", (q,), ()) for q in hi] + [("cx", (hi[0], hi[3]), ()), ("rx", (hi[1],), (0.7,))]
    gates += W.brickwork_circuit(n, 6, seed=n) + W.random_gate_list(n, 40, seed=n)
    want = tensor.sv_run(gates, n)
    arrays = nwq.circuit_arrays(gates)
    for rb in (1, 2, 0, None):
        st = nwq.SVState(n, reset=False)
        st.load(W.random_state(n, seed=3))
        if rb is None:
            st.set_fusion(0)
        else:
            st.set_fusion(k)
            nwq.nwq_set_fusion_kernel(st.h, rb)
        nwq.nwq_run_circuit(st.h, *arrays)
        got = st.numpy()
        assert maxerr(got, want) <= TOL, (n, k, rb)
        st.reset()
        nwq.nwq_apply_circuit(st.h, *arrays)
        assert np.array_equal(st.numpy(), got), (n, k, rb)
        st.close()

"""GPU parity of the measurement path against the oracle: Born-rule
probabilities (SV and DM), readout noise through per-qubit confusion
matrices, and shot sampling (bit-exact: the sampler works on an exact
integer CDF), plus edge cases and a 28-qubit run checked by properties."""
import numpy as np
import pytest

import workloads as W
from oracle import measure as M, tensor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nwq():
    from paper_2401_06861_amd import nwq as mod
    return mod


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def confusions(n, seed, identity_every=3):
    rng = np.random.default_rng(seed)
    cs = []
    for q in range(n):
        if q % identity_every == 0:
            cs.append(np.eye(2))
            continue
        e01, e10 = rng.uniform(0, 0.1, 2)
        cs.append(np.array([[1 - e01, e10], [e01, 1 - e10]]))
    return cs


def test_probabilities_sv_and_dm(nwq, torch):
    for n in (3, 12, 15):   # one partial workgroup; grids of 16 and 128 (XCD order)
        psi = W.random_state(n, seed=21 + n)
        st = nwq.SVState(n, reset=False)
        st.load(psi)
        p = st.probabilities().cpu().numpy()
        assert np.max(np.abs(p - M.probabilities_sv(psi))) <= 1e-15, n
        st.close()
    n = 5
    rho = W.random_density_matrix(n, seed=22)
    dm = nwq.DMState(n, reset=False)
    dm.load(rho)
    ops = [("h", (1,), ()), ("depolarize", (1,), (0.1,)), ("cx", (1, 3), ())]
    dm.run(ops)                                   # deferred superoperators are flushed first
    want = rho
    for op in ops:
        want = tensor.dm_apply(want, op, n)
    assert np.max(np.abs(dm.probabilities().cpu().numpy() - M.probabilities_dm(want))) <= 1e-14
    dm.close()


@pytest.mark.parametrize("n", [1, 3, 10, 14, 16])
def test_readout_noise(nwq, torch, n):
    """Passes of one to five qubits (every third matrix is the identity and is
    skipped: n=14 leaves 9 matrices, in passes of five and four; n=16 leaves
    10, in two passes of five)."""
    rng = np.random.default_rng(n)
    p = rng.dirichlet(np.ones(1 << n))
    cs = confusions(n, seed=n + 1, identity_every=3 if n > 1 else 5)
    t = torch.from_numpy(p).cuda()
    nwq.nwq_readout_noise(n, t, cs)
    assert np.max(np.abs(t.cpu().numpy() - M.readout_noise(p, cs, n))) <= 1e-15


def test_readout_noise_rejects_bad_matrices(nwq, torch):
    t = torch.zeros(8, dtype=torch.float64, device="cuda")
    bad = [np.eye(2), np.array([[0.9, 0.0], [0.2, 1.0]]), np.eye(2)]    # column 0 sums to 1.1
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_readout_noise(3, t, bad)
    assert e.value.code == nwq.NWQ_EINVAL


@pytest.mark.parametrize("n,zeros", [(1, []), (5, [0, 7]), (13, [1, 2, 3, 4095, 8191])])
def test_sampling_bit_exact(nwq, torch, n, zeros):
    rng = np.random.default_rng(100 + n)
    p = rng.dirichlet(np.ones(1 << n) * 0.5)
    p[zeros] = 0.0
    p /= p.sum()
    u = rng.uniform(0, 1, 20000)
    u[:3] = [0.0, 0.5, 1.0 - 2.0 ** -53]
    pt, ut = torch.from_numpy(p).cuda(), torch.from_numpy(u).cuda()
    work = torch.empty(nwq.nwq_sample_workspace_bytes(n) // 8, dtype=torch.int64, device="cuda")
    out = nwq.sample_shots(n, pt, ut, work)
    want = M.sample(p, u)
    assert np.array_equal(out.cpu().numpy(), want)
    cdf = work[: 1 << n].cpu().numpy().view(np.uint64)
    assert np.array_equal(cdf, np.cumsum(M.quantize(p), dtype=np.uint64))
    assert not np.isin(out.cpu().numpy(), zeros).any()


def test_sampling_edges(nwq, torch):
    n = 6
    work = torch.empty(nwq.nwq_sample_workspace_bytes(n) // 8, dtype=torch.int64, device="cuda")
    zero = torch.zeros(1 << n, dtype=torch.float64, device="cuda")
    out = nwq.sample_shots(n, zero, torch.rand(10, dtype=torch.float64, device="cuda"), work)
    assert out.tolist() == [-1] * 10
    empty = nwq.sample_shots(n, zero, torch.empty(0, dtype=torch.float64, device="cuda"), work)
    assert empty.numel() == 0
    small = torch.empty(8, dtype=torch.int64, device="cuda")
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_sample(n, zero, torch.rand(4, dtype=torch.float64, device="cuda"),
                       torch.empty(4, dtype=torch.int64, device="cuda"), small)
    assert e.value.code == nwq.NWQ_EINVAL
    assert nwq.nwq_sample_workspace_bytes(0) == 0


def test_sampling_28_qubits_properties(nwq, torch):
    """A 28-qubit circuit state: probabilities sampled against the oracle's
    Born rule on gathered amplitudes; every shot lands on an outcome with
    q_j > 0 inside its CDF interval; Q equals the exact quantised total."""
    n = 28
    st = nwq.SVState(n)
    st.run_circuit(W.brickwork_circuit(n, 3, seed=5))
    p = st.probabilities()
    idx = torch.from_numpy(np.random.default_rng(1).integers(0, 1 << n, 1 << 16)).cuda()
    amps = st.tensor.index_select(0, idx).cpu().numpy()
    assert np.max(np.abs(p.index_select(0, idx).cpu().numpy() - M.probabilities_sv(amps))) <= 1e-15
    u = torch.from_numpy(np.random.default_rng(2).uniform(0, 1, 1 << 18)).cuda()
    work = torch.empty(nwq.nwq_sample_workspace_bytes(n) // 8, dtype=torch.int64, device="cuda")
    out = nwq.sample_shots(n, p, u, work).cpu().numpy()
    cdf = work[: 1 << n]
    ph = p.cpu().numpy()
    q = M.quantize(ph)
    Q = int(np.sum(q, dtype=np.uint64))
    assert int(cdf[-1].item()) == Q
    j = torch.from_numpy(out).cuda()
    cj = cdf.index_select(0, j).cpu().numpy().view(np.uint64)
    cprev = cdf.index_select(0, (j - 1).clamp(min=0)).cpu().numpy().view(np.uint64)
    cprev[out == 0] = 0
    assert np.all(q[out] > 0)
    uu = u.cpu().numpy()
    for s in range(0, len(out), 997):
        target = (int(min(max(uu[s] * 2.0 ** 53, 0.0), 2.0 ** 53 - 1)) * Q) >> 53
        assert int(cprev[s]) <= target < int(cj[s])
    st.close()

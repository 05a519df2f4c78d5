"""GPU serving loop: a mixed request stream (SV VQE on the LDS-resident and
the per-gate graph paths, noisy DM TFIM) is served with continuous batching;
every request's outputs equal, bit for bit, those of the same request served
alone, and sampled outputs match the oracle (energies <= 1e-10, gradients
<= 1e-10 vs parameter shift, DM magnetisations <= 1e-12)."""
import numpy as np
import pytest

import workloads as W
from oracle import tensor, vqe as OV

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    from paper_2401_06861_amd.serving import GpuExecutor, Server, summarize
    reqs = W.serving_trace(num=24, rate=3000.0, seed=11, sv_n=(5, 14), dm_n=(3, 6), L_range=(1, 3),
                           opt_steps=(1, 3), dm_steps=4)
    ex = GpuExecutor()
    srv = Server(ex, budget_bytes=8 << 30)
    res = srv.run(reqs)
    yield reqs, res, ex, srv, summarize(res)
    ex.close()


def test_all_served(served):
    reqs, res, ex, srv, summ = served
    assert all(r.error is None for r in res), [r.error for r in res if r.error]
    assert summ["completed"] == len(reqs)
    assert any(b > 1 for _, b in srv.batches)          # batching happened
    assert srv.max_in_use <= 8 << 30


def test_mix_equals_alone_bitwise(served):
    from paper_2401_06861_amd.serving import Server
    reqs, res, ex, _, _ = served
    by = {r.rid: r for r in res}
    for q in reqs[:12]:
        q1 = W.Request(q.rid, 0.0, q.kind, q.n, L=q.L, want_grad=q.want_grad, steps=q.steps, seed=q.seed, h=q.h)
        alone = Server(ex, budget_bytes=8 << 30).run([q1])[0]
        mix = by[q.rid]
        assert len(alone.outputs) == len(mix.outputs)
        for a, m in zip(alone.outputs, mix.outputs):
            if q.kind == "sv_vqe":
                assert a[0] == m[0]
                if q.want_grad:
                    assert np.array_equal(a[1], m[1])
            else:
                assert np.array_equal(a["Z"], m["Z"]) and a["purity"] == m["purity"] and a["trace"] == m["trace"]


def test_outputs_match_oracle(served):
    reqs, res, _, _, _ = served
    by = {r.rid: r for r in res}
    sv = [q for q in reqs if q.kind == "sv_vqe" and q.n <= 9][:3]
    for q in sv:
        prog = W.hea_ansatz(q.n, q.L)
        terms = W.tfim_hamiltonian(q.n, 1.0, q.h)
        th = W.request_thetas(q, 2 * q.n * q.L)
        for s, out in enumerate(by[q.rid].outputs):
            assert abs(out[0] - OV.energy(prog, th[s], terms, q.n)) <= 1e-10
            if q.want_grad:
                assert np.max(np.abs(out[1] - OV.grad_parameter_shift(prog, th[s], terms, q.n))) <= 1e-10
    dm = [q for q in reqs if q.kind == "dm_tfim"][:2]
    for q in dm:
        rho = tensor.dm_run(W.noisy_tfim_circuit(q.n, q.steps), q.n)
        want = [tensor.dm_expval(rho, 0, 1 << i, q.n).real for i in range(q.n)]
        out = by[q.rid].outputs[0]
        assert np.max(np.abs(out["Z"] - np.array(want))) <= 1e-12
        assert abs(out["purity"] - tensor.dm_purity(rho)) <= 1e-12

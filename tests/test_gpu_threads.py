"""Several host threads driving their own handles at once (as the server's
worker threads do): fused SV circuits with gate products and fused DM
circuits with queued one- and two-qubit superoperators, each thread on its own
stream.  Every result must equal the same work done on one thread, bit for
bit (the kernels are deterministic), and nothing may fail."""
import threading

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nwq():
    from paper_2401_06861_amd import nwq as mod
    return mod


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _sv_job(nwq, torch, seed):
    n = 16
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        st = nwq.SVState(n, stream=stream, owned=True)
        try:
            st.set_fusion(12 + seed % 2)
            nwq.nwq_run_circuit(st.h, *nwq.circuit_arrays(W.brickwork_circuit(n, 12, seed=seed)))
            return np.array(st.expvals(W.single_site_terms(n, "Z")))
        finally:
            st.close()


def _dm_job(nwq, torch, seed):
    n = 8
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        st = nwq.DMState(n, stream=stream, owned=True)
        try:
            st.set_fusion(12)
            st.run(W.noisy_tfim_circuit(n, 3 + seed % 3))
            return np.array(st.expvals(W.single_site_terms(n, "Z"))), st.purity()
        finally:
            st.close()


def test_concurrent_handles_match_one_thread(nwq, torch):
    jobs = [(_sv_job, s) for s in range(4)] + [(_dm_job, s) for s in range(4)]
    want = [fn(nwq, torch, s) for fn, s in jobs]
    got = [None] * len(jobs)
    errors = []

    def work(i):
        try:
            torch.cuda.set_device(0)
            for _ in range(3):
                got[i] = jobs[i][0](nwq, torch, jobs[i][1])
        except Exception as e:   # reported below, not lost in the thread
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for i, (w, g) in enumerate(zip(want, got)):
        if isinstance(w, tuple):
            assert np.array_equal(w[0], g[0]) and w[1] == g[1], i
        else:
            assert np.array_equal(w, g), i

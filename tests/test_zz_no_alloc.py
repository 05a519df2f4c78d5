"""The allocation-free shot sampler (nwq_sample_noalloc) against the
workspace sampler (nwq_sample), both called through the C ABI: bit-identical
outcomes on two calls in a row, the second on a smaller distribution, and
the size limit rejected before any launch."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2401_06861_amd import nwq
    return torch, nwq


def distribution(torch, n, seed):
    g = np.random.default_rng(seed)
    w = g.exponential(size=1 << n)
    w[g.random(1 << n) < 0.25] = 0.0            # zero-probability outcomes must never be drawn
    return torch.from_numpy(w / w.sum()).cuda()


def abi_sample(torch, nwq, n, p, u):
    """Both entry points through the raw C ABI on the current stream."""
    s = torch.cuda.current_stream().cuda_stream
    shots = u.numel()
    ws = nwq.lib.nwq_sample_workspace_bytes(n)
    work = torch.empty(ws // 8, dtype=torch.int64, device="cuda")
    ref = torch.full((shots,), -7, dtype=torch.int64, device="cuda")
    rc = nwq.lib.nwq_sample(C.c_int(n), C.c_void_p(p.data_ptr()), C.c_void_p(u.data_ptr()), C.c_longlong(shots),
                            C.c_void_p(ref.data_ptr()), C.c_void_p(work.data_ptr()), C.c_size_t(ws), C.c_void_p(s))
    assert rc == 0, nwq.nwq_last_error()
    out = torch.full((shots,), -9, dtype=torch.int64, device="cuda")
    rc = nwq.lib.nwq_sample_noalloc(C.c_int(n), C.c_void_p(p.data_ptr()), C.c_void_p(u.data_ptr()),
                                    C.c_longlong(shots), C.c_void_p(out.data_ptr()), C.c_void_p(s))
    assert rc == 0, nwq.nwq_last_error()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_matches_workspace_sampler_twice(env):
    torch, nwq = env
    print("noalloc: n=20 then n=13, 2^16 / 5000 shots", flush=True)
    for n, shots, seed in ((20, 1 << 16, 1), (13, 5000, 2)):
        p = distribution(torch, n, seed)
        u = torch.rand(shots, dtype=torch.float64, device="cuda",
                       generator=torch.Generator("cuda").manual_seed(seed))
        ref, out = abi_sample(torch, nwq, n, p, u)
        assert (ref >= 0).all() and (ref < (1 << n)).all()
        assert np.array_equal(out, ref), n
        pz = p.cpu().numpy()
        assert (pz[out] > 0).all()


def test_noalloc_size_limit_and_empty(env):
    torch, nwq = env
    p = distribution(torch, 4, 3)
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    out = torch.empty(0, dtype=torch.int64, device="cuda")
    nwq.nwq_sample_noalloc(4, p, empty, out)           # zero shots: scan only
    big = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_sample_noalloc(21, big, empty, out)
    assert e.value.code == nwq.NWQ_ERANGE
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_sample_noalloc(0, big, empty, out)
    assert e.value.code == nwq.NWQ_ERANGE
    torch.cuda.synchronize()

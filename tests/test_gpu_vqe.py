"""GPU parity of the VQE path (Sec. III, Fig. 4): energies against the
oracle (<= 1e-10), adjoint gradients against the oracle's parameter-shift
rule (<= 1e-10) and finite differences (<= 1e-6), on the LDS-resident
batched path, the per-gate graph path and the plain per-circuit path;
bit-identical results alone and inside a batch; the autograd wrapper."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import vqe as OV

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def V():
    from paper_2401_06861_amd import vqe as mod
    return mod


def run_all_paths(V, torch, n, prog, terms, theta):
    ctx = V.VQE(n, prog, terms, n_params=theta.shape[1])
    t = torch.from_numpy(theta).cuda()
    out = {}
    modes = [("lds", 1), ("graph", 2)] if n <= 12 else [("graph", 2)]
    if n >= 8:
        modes.append(("fused", 3))
    for name, mode in modes:
        ctx.set_config(mode, 256, 0)
        E, G = ctx.eval(t, grad=True)
        out[name] = (E.cpu().numpy(), G.cpu().numpy())
    Es, Gs = [], []
    for b in range(theta.shape[0]):
        E, G = ctx.eval_single(t[b])
        Es.append(E.cpu().numpy()[0])
        Gs.append(G.cpu().numpy()[0])
    out["single"] = (np.array(Es), np.array(Gs))
    ctx.close()
    return out


@pytest.mark.parametrize("n,L", [(2, 1), (4, 2), (6, 3), (9, 2)])
def test_hea_energy_and_gradient(V, torch, n, L):
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=3)
    terms = W.tfim_hamiltonian(n, 1.0, h)
    outs = run_all_paths(V, torch, n, prog, terms, theta)
    for b in range(theta.shape[0]):
        e_ref = OV.energy(prog, theta[b], terms, n)
        g_ps = OV.grad_parameter_shift(prog, theta[b], terms, n)
        for name, (E, G) in outs.items():
            assert abs(E[b] - e_ref) <= 1e-10, (name, b)
            assert np.max(np.abs(G[b] - g_ps)) <= 1e-10, (name, b)
    g_fd = OV.grad_finite_difference(prog, theta[0], terms, n)
    assert np.max(np.abs(outs["single"][1][0] - g_fd)) <= 1e-6


def test_generic_program_with_fixed_gates_and_rzz(V, torch):
    n = 5
    A = W.AnsatzGate
    prog = [A("h", (0,), -1), A("rx", (1,), 0), A("cz", (0, 2), -1), A("rzz", (1, 3), 1), A("s", (4,), -1),
            A("ry", (4,), 2), A("swap", (2, 4), -1), A("t", (3,), -1), A("rz", (0,), 0), A("cx", (4, 1), -1),
            A("y", (2,), -1), A("rzz", (4, 0), 3), A("sdg", (1,), -1), A("rx", (3,), 1)]
    terms = W.random_pauli_sum(n, 12, seed=4)
    theta = np.random.default_rng(2).uniform(-math.pi, math.pi, (4, 4))
    outs = run_all_paths(V, torch, n, prog, terms, theta)
    for b in range(4):
        e_ref = OV.energy(prog, theta[b], terms, n)
        g_ps = OV.grad_parameter_shift(prog, theta[b], terms, n)   # shared parameters: summed per occurrence
        for name, (E, G) in outs.items():
            assert abs(E[b] - e_ref) <= 1e-10, name
            assert np.max(np.abs(G[b] - g_ps)) <= 1e-10, name


def test_theta_zero_special_cases(V, torch):
    n, L = 6, 3
    prog = W.hea_ansatz(n, L)
    terms = W.tfim_hamiltonian(n, 1.0, 0.8)
    ctx = V.VQE(n, prog, terms)
    E, G = ctx.eval(torch.zeros(2, 2 * n * L, dtype=torch.float64, device="cuda"))
    assert np.max(np.abs(E.cpu().numpy() + (n - 1))) <= 1e-12
    last_rz = [(L - 1) * 2 * n + n + q for q in range(n)]
    assert np.max(np.abs(G.cpu().numpy()[:, last_rz])) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("n,mode", [(7, 1), (7, 2), (13, 2), (13, 3), (9, 3)])
def test_alone_equals_in_the_mix_bitwise(V, torch, n, mode):
    L = 2
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=16)
    ctx = V.VQE(n, prog, W.tfim_hamiltonian(n, 1.0, h))
    ctx.set_config(mode, 256, 0)
    t = torch.from_numpy(theta).cuda()
    E, G = ctx.eval(t)
    for b in (0, 5, 15):
        E1, G1 = ctx.eval(t[b:b + 1])
        assert E1.item() == E[b].item()
        assert torch.equal(G1[0], G[b])
    ctx.close()


def test_energy_only_matches(V, torch):
    n, L = 8, 2
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=5)
    ctx = V.VQE(n, prog, W.tfim_hamiltonian(n, 1.0, h))
    t = torch.from_numpy(theta).cuda()
    for mode in (1, 2, 3):
        ctx.set_config(mode, 128, 0)
        E1, _ = ctx.eval(t, grad=False)
        E2, _ = ctx.eval(t, grad=True)
        assert torch.max(torch.abs(E1 - E2)).item() <= 1e-13
    ctx.close()


def test_larger_register_global_path(V, torch):
    n, L = 14, 2
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=2)
    terms = W.tfim_hamiltonian(n, 1.0, h)
    ctx = V.VQE(n, prog, terms)
    t = torch.from_numpy(theta).cuda()
    E, G = ctx.eval(t)
    E = E.cpu().numpy()
    G = G.cpu().numpy()
    pick = [0, 7, 13, 20, 41, 55]
    for b in range(2):
        assert abs(E[b] - OV.energy(prog, theta[b], terms, n)) <= 1e-10
        g_ps = OV.grad_parameter_shift(prog, theta[b], terms, n, params=pick)
        assert np.max(np.abs(G[b][pick] - g_ps[pick])) <= 1e-10
    ctx.close()


def test_autograd_wrapper(V, torch):
    n, L = 5, 2
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=4)
    ctx = V.VQE(n, prog, W.tfim_hamiltonian(n, 1.0, h))
    t = torch.from_numpy(theta).cuda().requires_grad_(True)
    w = torch.arange(1, 5, dtype=torch.float64, device="cuda")
    loss = (V.AdjointEnergy.apply(t, ctx) * w).sum()
    loss.backward()
    _, G = ctx.eval(t.detach())
    assert torch.max(torch.abs(t.grad - w[:, None] * G)).item() <= 1e-14
    t1 = torch.from_numpy(theta[0]).cuda().requires_grad_(True)
    e = V.AdjointEnergy.apply(t1, ctx)
    e.backward()
    assert torch.max(torch.abs(t1.grad - G[0])).item() <= 1e-14
    ctx.close()


def test_autotune_picks_a_valid_config(V, torch):
    n, L = 10, 2
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=32)
    terms = W.tfim_hamiltonian(n, 1.0, h)
    ctx = V.VQE(n, prog, terms)
    ms = ctx.autotune(32)
    assert ms > 0
    mode, threads, bps = ctx.get_config()
    assert mode in (1, 2)
    E, G = ctx.eval(torch.from_numpy(theta).cuda())
    assert abs(E[0].item() - OV.energy(prog, theta[0], terms, n)) <= 1e-10
    ctx.close()


def test_vqe_create_errors(V, torch):
    from paper_2401_06861_amd import nwq
    A = W.AnsatzGate
    with pytest.raises(nwq.NwqError) as e:
        V.VQE(3, [A("rx", (3,), 0)], [(1, 0, 1.0)], n_params=1)
    assert e.value.code == nwq.NWQ_ERANGE
    with pytest.raises(nwq.NwqError) as e:
        V.VQE(3, [A("rx", (1,), 2)], [(1, 0, 1.0)], n_params=1)
    assert e.value.code == nwq.NWQ_EINVAL
    with pytest.raises(nwq.NwqError) as e:
        V.VQE(3, [A("u3", (1,), -1)], [(1, 0, 1.0)], n_params=1)
    assert e.value.code == nwq.NWQ_EINVAL
    with pytest.raises(nwq.NwqError) as e:
        V.VQE(3, [A("cx", (1, 1), -1)], [(1, 0, 1.0)], n_params=1)
    assert e.value.code == nwq.NWQ_EDUP


@pytest.mark.parametrize("n,L,bps", [(13, 2, 0), (15, 2, 4), (16, 3, 0)])
def test_fused_path_matches_oracle(V, torch, n, L, bps):
    """Fused-block schedule (register-blocked forward over the batch, LDS
    backward tiles) at sizes with several tiles per state; gradients checked
    against parameter shift on a sample of parameters, energies exactly."""
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=3)
    terms = W.tfim_hamiltonian(n, 1.0, h)
    ctx = V.VQE(n, prog, terms)
    ctx.set_config(3, 256, bps)
    t = torch.from_numpy(theta).cuda()
    E, G = ctx.eval(t)
    ctx.set_flags(1)                           # no direct first / last phase: the same bits
    E1, G1 = ctx.eval(t)
    assert torch.equal(E, E1) and torch.equal(G, G1)
    ctx.set_flags(0)
    E2, G2 = ctx.eval_single(t[1])
    E = E.cpu().numpy()
    G = G.cpu().numpy()
    pick = [0, 1, n - 1, n, 2 * n - 1, 2 * n * L - 1, n * L]
    for b in range(3):
        assert abs(E[b] - OV.energy(prog, theta[b], terms, n)) <= 1e-10
        g_ps = OV.grad_parameter_shift(prog, theta[b], terms, n, params=pick)
        assert np.max(np.abs(G[b][pick] - g_ps[pick])) <= 1e-10
    assert abs(E2.item() - E[1]) <= 1e-12
    assert np.max(np.abs(G2.cpu().numpy()[0] - G[1])) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("n,L", [(14, 3), (16, 2)])
def test_fused_low_tile_bits(V, torch, n, L):
    """The fused schedule planned with each low-tile-bit setting (0: the
    default 3; clamped to [k - 8, k - 2] at tile width k): energies and
    parameter-shift gradient components against the oracle, and the same
    values across settings to rounding."""
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=2)
    terms = W.tfim_hamiltonian(n, 1.0, h)
    ctx = V.VQE(n, prog, terms)
    ctx.set_config(3, 256, 0)
    t = torch.from_numpy(theta).cuda()
    pick = [0, n - 1, n, 2 * n * L - 1]
    ref = None
    for c in (0, 3, 4, 5, 6, 8):
        ctx.set_lowbits(c)
        E, G = ctx.eval(t)
        E = E.cpu().numpy()
        G = G.cpu().numpy()
        if ref is None:
            ref = (E, G)
            for b in range(2):
                assert abs(E[b] - OV.energy(prog, theta[b], terms, n)) <= 1e-10
                g_ps = OV.grad_parameter_shift(prog, theta[b], terms, n, params=pick)
                assert np.max(np.abs(G[b][pick] - g_ps[pick])) <= 1e-10
        assert np.max(np.abs(E - ref[0])) <= 1e-12, c
        assert np.max(np.abs(G - ref[1])) <= 1e-12, c
    from paper_2401_06861_amd import nwq
    for bad in (-1, 2, 9):
        with pytest.raises(nwq.NwqError):
            ctx.set_lowbits(bad)
    ctx.close()


def test_fused_generic_program(V, torch):
    """Fused path with fixed gates, CZ, SWAP and RZZ on a 10-qubit register
    (one tile) and with several tiles at 13 and 17 qubits; at 17 qubits the
    random Pauli sum needs every kind of lambda = H phi pass (the low-bit
    tile with the diagonal terms, tiles over high bits, and gathered terms
    whose flipped bits fit no tile)."""
    A = W.AnsatzGate
    for n in (10, 13, 17):
        prog = []
        for l in range(2):
            prog += [A("h", (q,), -1) for q in range(0, n, 3)]
            prog += [A("rx", (q,), l * 4 + (q % 4)) for q in range(n)]
            prog += [A("rzz", (q, (q + 5) % n), 8 + l) for q in range(0, n, 2)]
            prog += [A("cz", (n - 1, 0), -1), A("swap", (1, n - 2), -1), A("s", (3,), -1), A("cx", (n - 1, 2), -1)]
            prog += [A("ry", (q,), 10 + l) for q in range(1, n, 2)]
        terms = W.random_pauli_sum(n, 10, seed=n)
        if n == 17:   # flips only on high bits, flips over many high bits, Z strings, one-body X
            terms += [(0b11 << 14, 1 << 15, 0.3), (0b1111111101 << 7, 0, -0.4), (0, 0b101 << 12, 0.2),
                      (1 << 16, 0, 0.5), (1 << 13, 1 << 2, -0.7)]
        theta = np.random.default_rng(n).uniform(-math.pi, math.pi, (2, 12))
        ctx = V.VQE(n, prog, terms, n_params=12)
        ctx.set_config(3, 256, 0)
        E, G = ctx.eval(torch.from_numpy(theta).cuda())
        for b in range(2):
            assert abs(E[b].item() - OV.energy(prog, theta[b], terms, n)) <= 1e-10
            g_ps = OV.grad_parameter_shift(prog, theta[b], terms, n)
            assert np.max(np.abs(G[b].cpu().numpy() - g_ps)) <= 1e-10
        ctx.close()


@pytest.mark.parametrize("n,mode", [(10, 1), (13, 2), (13, 3)])
def test_graph_replays_with_eager_work_between(V, torch, n, mode):
    """The captured schedule replayed several times with new parameters,
    with eager per-circuit evaluations between the replays: every replay
    matches the eager result, and replaying the same parameters again gives
    the same bits."""
    L = 2
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=4 * 3)
    ctx = V.VQE(n, prog, W.tfim_hamiltonian(n, 1.0, h))
    ctx.set_config(mode, 256, 0)
    t = torch.from_numpy(theta).cuda()
    first = []
    for r in range(3):
        chunk = t[4 * r: 4 * r + 4]
        E, G = ctx.eval(chunk)
        first.append((E.clone(), G.clone()))
        for b in range(4):
            e1, g1 = ctx.eval_single(chunk[b])                      # eager work between replays
            assert abs(e1.item() - E[b].item()) <= 1e-12
            assert torch.max(torch.abs(g1[0] - G[b])).item() <= 1e-12
    for r in range(3):
        E, G = ctx.eval(t[4 * r: 4 * r + 4])
        assert torch.equal(E, first[r][0]) and torch.equal(G, first[r][1])
    ctx.close()


def test_vqe_batch_one_call(V, torch):
    """nwq_vqe_batch builds the ansatz and the Ising Hamiltonian in the
    library: energies and gradients against the oracle, bit-identical to a
    context built from the same program, and a new (J, h) on the same shape
    (term table rewritten in place) matches the oracle again."""
    n, L, B = 9, 2, 4
    prog = W.hea_ansatz(n, L)
    theta, h = W.vqe_batch(n, L, B=B)
    t = torch.from_numpy(theta).cuda()
    for J, hx in ((1.0, h), (0.7, 1.3), (1.0, h)):
        E, G = V.vqe_batch(n, L, J, hx, t)
        terms = W.tfim_hamiltonian(n, J, hx)
        for b in range(B):
            assert abs(E[b].item() - OV.energy(prog, theta[b], terms, n)) <= 1e-10
        g_ps = OV.grad_parameter_shift(prog, theta[0], terms, n)
        assert np.max(np.abs(G[0].cpu().numpy() - g_ps)) <= 1e-10
        ctx = V.VQE(n, prog, terms)
        E2, G2 = ctx.eval(t)
        assert torch.equal(E, E2) and torch.equal(G, G2)
        ctx.close()
    E3, G3 = V.vqe_batch(n, L, 1.0, h, t, grad=False)
    assert G3 is None and torch.equal(E3, E)
    for nn, LL in ((14, 1), (5, 3)):               # more shapes in the cache, one above the LDS size
        th, hh = W.vqe_batch(nn, LL, B=2)
        E, G = V.vqe_batch(nn, LL, 1.0, hh, torch.from_numpy(th).cuda())
        pr = W.hea_ansatz(nn, LL)
        te = W.tfim_hamiltonian(nn, 1.0, hh)
        assert abs(E[1].item() - OV.energy(pr, th[1], te, nn)) <= 1e-10
    V.vqe_batch_release()
    from paper_2401_06861_amd import nwq
    with pytest.raises(nwq.NwqError) as e:
        V.vqe_batch(31, 1, 1.0, 1.0, torch.zeros(1, 62, dtype=torch.float64, device="cuda"))
    assert e.value.code == nwq.NWQ_ERANGE

"""Pins of the measurement oracle: Born-rule probabilities, readout noise
against an explicit Kronecker product and bit-flip permutations, and the
integer inverse-transform sampler against hand-worked cases and empirical
frequencies."""
import math

import numpy as np
import pytest

from oracle import dense, measure as M
import workloads as W


def test_born_probabilities():
    bell = dense.sv_run([("h", (0,), ()), ("cx", (0, 1), ())], 2)
    assert np.allclose(M.probabilities_sv(bell), [0.5, 0, 0, 0.5], atol=1e-15)
    psi = W.random_state(5, seed=3)
    rho = np.outer(psi, psi.conj())
    assert np.max(np.abs(M.probabilities_dm(rho) - M.probabilities_sv(psi))) <= 1e-15
    assert abs(M.probabilities_sv(psi).sum() - 1) <= 1e-14


def test_readout_matches_kronecker_product():
    rng = np.random.default_rng(4)
    n = 3
    p = rng.dirichlet(np.ones(1 << n))
    cs = []
    for q in range(n):
        e01, e10 = rng.uniform(0, 0.2, 2)   # P(read 1 | 0), P(read 0 | 1)
        cs.append(np.array([[1 - e01, e10], [e01, 1 - e10]]))
    big = np.kron(np.kron(cs[2], cs[1]), cs[0])   # qubit 0 is the lowest bit
    assert np.max(np.abs(M.readout_noise(p, cs, n) - big @ p)) <= 1e-15
    assert abs(M.readout_noise(p, cs, n).sum() - 1) <= 1e-14


def test_readout_bit_flip_and_identity():
    rng = np.random.default_rng(5)
    n = 4
    p = rng.dirichlet(np.ones(1 << n))
    eye = [np.eye(2)] * n
    assert np.array_equal(M.readout_noise(p, eye, n), p)
    for q in range(n):
        cs = [np.eye(2)] * n
        cs = cs[:q] + [np.array([[0.0, 1.0], [1.0, 0.0]])] + cs[q + 1:]
        out = M.readout_noise(p, cs, n)
        assert np.array_equal(out, p[np.arange(1 << n) ^ (1 << q)])


def test_sampler_worked_cases():
    p = np.array([0.5, 0.0, 0.25, 0.25])
    u = np.array([0.0, 0.499, 0.5, 0.74, 0.75, 1.0 - 2.0 ** -53])
    assert M.sample(p, u).tolist() == [0, 0, 2, 2, 3, 3]
    assert M.sample(np.zeros(4), np.array([0.3])).tolist() == [-1]
    # quantisation is exact power-of-two scaling
    assert int(M.quantize(np.array([0.5]))[0]) == 2 ** 60
    assert int(M.quantize(np.array([1.0]))[0]) == 2 ** 61
    assert int(M.quantize(np.array([-1e-17]))[0]) == 0


def test_sampler_frequencies_and_zeros():
    rng = np.random.default_rng(6)
    p = rng.dirichlet(np.ones(32))
    p[[3, 7, 20]] = 0.0
    p /= p.sum()
    u = rng.uniform(0, 1, 200000)
    s = M.sample(p, u)
    assert not np.isin(s, [3, 7, 20]).any()
    freq = np.bincount(s, minlength=32) / len(u)
    sigma = np.sqrt(p * (1 - p) / len(u))
    assert np.all(np.abs(freq - p) <= 6 * sigma + 1e-12)

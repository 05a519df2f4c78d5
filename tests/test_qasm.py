"""OpenQASM 2.0 front-end: the oracle's reader is pinned by hand-written
programs; the library's parser (host code of the C ABI, no device calls) must
give the same gate arrays; errors name the line."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import qasm


@pytest.fixture(scope="module")
def nwq():
    from paper_2401_06861_amd import nwq as mod
    return mod


HAND = """OPENQASM 2.0;
include "qelib1.inc";
qreg q[2];   // first register: qubits 0, 1
qreg r[3];   // second register: qubits 2, 3, 4
creg c[5];
h q;                       // broadcast: h q[0]; h q[1];
cx q[1], r[2];
u1(pi/2) r[0];
p(-pi) r[1];
u2(0, pi) q[0];
U(2*pi/3, sqrt(2), cos(0)) r[2];
rz(2^3 - 7.5) q[1];
rx(-(-1)) r;               // broadcast over r
cx q[0], r[0];
barrier q, r;
swap r[1], q[0];
id q[1];
measure q[0] -> c[0];
"""

HAND_GATES = [
    ("h", (0,), ()), ("h", (1,), ()), ("cx", (1, 4), ()), ("u3", (2,), (0.0, 0.0, math.pi / 2)),
    ("u3", (3,), (0.0, 0.0, -math.pi)), ("u3", (0,), (math.pi / 2, 0.0, math.pi)),
    ("u3", (4,), (2 * math.pi / 3, math.sqrt(2), 1.0)), ("rz", (1,), (0.5,)),
    ("rx", (2,), (1.0,)), ("rx", (3,), (1.0,)), ("rx", (4,), (1.0,)), ("cx", (0, 2), ()),
    ("swap", (3, 0), ()), ("id", (1,), ()),
]


def test_oracle_reader_hand_program():
    n, gates = qasm.parse(HAND)
    assert n == 5
    assert [(g, q) for g, q, _ in gates] == [(g, q) for g, q, _ in HAND_GATES]
    for (_, _, a), (_, _, b) in zip(gates, HAND_GATES):
        assert np.allclose(a, b, atol=1e-15, rtol=0)


@pytest.mark.parametrize("split", [0, 3])
def test_oracle_reader_round_trip(split):
    g = W.random_gate_list(7, 80, seed=11 + split)
    n, back = qasm.parse(W.qasm_text(g, 7, split=split, seed=split))
    assert n == 7 and [(a[0], a[1]) for a in back] == [(a[0], a[1]) for a in g]
    assert max(abs(x - y) for a, b in zip(g, back) for x, y in zip(a[2], b[2])) <= 1e-15


@pytest.mark.parametrize("split", [0, 4])
def test_library_parser_matches_oracle_reader(nwq, split):
    for text in (HAND, W.qasm_text(W.random_gate_list(9, 120, seed=5), 9, split=split, seed=9)):
        n, gates = qasm.parse(text)
        nq, types, qs, ps = nwq.nwq_qasm_parse(text)
        t2, q2, p2 = nwq.circuit_arrays(gates)
        assert nq == n
        assert np.array_equal(types, t2) and np.array_equal(qs, q2)
        assert np.max(np.abs(ps - p2), initial=0.0) <= 1e-15


@pytest.mark.parametrize("text,line", [
    ("OPENQASM 3.0;\nqreg q[1];", 1),
    ("qreg q[1];", 1),
    ("OPENQASM 2.0;\nqreg q[2];\nfoo q[0];\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\ngate g a { x a; }\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\n\nrx q[0];\n", 4),
    ("OPENQASM 2.0;\nqreg q[2];\nx q[2];\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\ncx q[1], q[1];\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\nx r[0];\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\nrz(pi/) q[0];\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\nqreg r[3];\ncx q, r;\n", 4),
    ("OPENQASM 2.0;\nqreg q[2];\nif (c==1) x q[0];\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\nrz(" + "(" * 500 + "1" + ")" * 500 + ") q[0];\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\nrz(" + "-" * 500 + "1) q[0];\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\nrz(" + "sin(" * 100000 + "1" + ")" * 100000 + ") q[0];\n", 3),
    ("OPENQASM 2.0;\nqreg q[2];\nrz(" + "2^" * 500 + "1) q[0];\n", 3),
])
def test_library_parser_errors(nwq, text, line):
    with pytest.raises(nwq.NwqError) as e:
        nwq.nwq_qasm_parse(text)
    assert e.value.code == nwq.NWQ_EINVAL
    assert f"line {line}:" in str(e.value)


def test_library_parser_survives_random_token_soup(nwq):
    """Random sequences of OpenQASM tokens and stray bytes: the reader either
    parses them or returns NWQ_EINVAL, never anything else (run under the
    host sanitizers too)."""
    rng = np.random.default_rng(5)
    toks = ["OPENQASM 2.0;", "include \"qelib1.inc\";", "qreg", "creg", "q", "c", "[", "]", "(", ")", ",", ";",
            "->", "u3", "cx", "rz", "sin", "cos", "pi", "^", "-", "+", "*", "/", "1", "0.5", "2e3", "1e400",
            "measure", "barrier", "gate", "if", "==", "{", "}", "\n", " ", "//", "\x00", "\xff", "ＱＡ"]
    for i in range(300):
        parts = ["OPENQASM 2.0;\nqreg q[3];\n"] if i % 2 else []
        parts += [toks[j] for j in rng.integers(0, len(toks), size=int(rng.integers(1, 60)))]
        text = " ".join(parts)
        try:
            nwq.nwq_qasm_parse(text)
        except nwq.NwqError as e:
            assert e.code == nwq.NWQ_EINVAL, (text, e)

"""Reader of OpenQASM 2.0 programs for the oracle (TEST INFRASTRUCTURE ONLY:
used by tests and the smoke check, never by the product).

Turns a program into the oracle's gate list: quantum registers are laid out
in declaration order; u1(l) and p(l) are U3(0, 0, l), u2(f, l) is
U3(pi/2, f, l), u and U are u3; gates on whole registers apply qubit by
qubit; barrier, measure, creg and include lines carry no gate.  Parameter
expressions are evaluated from a parsed syntax tree restricted to numbers,
pi, the four operations, powers, unary signs and sin cos tan exp ln sqrt.
"""
from __future__ import annotations

import ast
import math
import re
from typing import List, Tuple

_FUNCS = {"sin": math.sin, "cos": math.cos, "tan": math.tan, "exp": math.exp, "ln": math.log, "sqrt": math.sqrt}
_NAMES = {"id": "id", "x": "x", "y": "y", "z": "z", "h": "h", "s": "s", "sdg": "sdg", "t": "t", "tdg": "tdg",
          "rx": "rx", "ry": "ry", "rz": "rz", "u3": "u3", "u": "u3", "U": "u3", "u1": "u1", "p": "u1",
          "u2": "u2", "cx": "cx", "CX": "cx", "cz": "cz", "swap": "swap", "rzz": "rzz"}


def _eval(node):
    if isinstance(node, ast.Expression):
        return _eval(node.body)
    if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
        return float(node.value)
    if isinstance(node, ast.Name) and node.id == "pi":
        return math.pi
    if isinstance(node, ast.UnaryOp) and isinstance(node.op, (ast.USub, ast.UAdd)):
        v = _eval(node.operand)
        return -v if isinstance(node.op, ast.USub) else v
    if isinstance(node, ast.BinOp):
        a, b = _eval(node.left), _eval(node.right)
        ops = {ast.Add: lambda: a + b, ast.Sub: lambda: a - b, ast.Mult: lambda: a * b,
               ast.Div: lambda: a / b, ast.Pow: lambda: a ** b}
        for k, f in ops.items():
            if isinstance(node.op, k):
                return f()
    if isinstance(node, ast.Call) and isinstance(node.func, ast.Name) and node.func.id in _FUNCS \
            and len(node.args) == 1:
        return _FUNCS[node.func.id](_eval(node.args[0]))
    raise ValueError("unsupported expression")


def _param(text: str) -> float:
    return _eval(ast.parse(text.replace("^", "**"), mode="eval"))


def _split_args(text: str) -> List[str]:
    out, depth, cur = [], 0, ""
    for ch in text:
        if ch == "," and depth == 0:
            out.append(cur)
            cur = ""
            continue
        depth += ch == "("
        depth -= ch == ")"
        cur += ch
    if cur.strip():
        out.append(cur)
    return [a.strip() for a in out]


def parse(text: str) -> Tuple[int, list]:
    """(number of qubits, [(name, qubits, params), ...])."""
    body = re.sub(r"//[^\n]*", "", text)
    stmts = [s.strip() for s in body.split(";") if s.strip()]
    if not stmts or not re.fullmatch(r"OPENQASM\s+2\.0", stmts[0]):
        raise ValueError("not an OpenQASM 2.0 program")
    regs, nq, gates = {}, 0, []
    for st in stmts[1:]:
        m = re.fullmatch(r"(qreg|creg)\s+(\w+)\s*\[\s*(\d+)\s*\]", st)
        if m:
            if m.group(1) == "qreg":
                regs[m.group(2)] = (nq, int(m.group(3)))
                nq += int(m.group(3))
            continue
        if st.startswith(("include", "barrier", "measure")):
            continue
        m = re.fullmatch(r"(\w+)\s*(?:\((.*)\))?\s+(.+)", st, re.S)
        if not m or m.group(1) not in _NAMES:
            raise ValueError(f"unsupported statement: {st}")
        name = _NAMES[m.group(1)]
        ps = [_param(a) for a in _split_args(m.group(2) or "")]
        args = []
        for a in _split_args(m.group(3)):
            r = re.fullmatch(r"(\w+)\s*(?:\[\s*(\d+)\s*\])?", a)
            base, size = regs[r.group(1)]
            args.append([base + int(r.group(2))] if r.group(2) is not None else list(range(base, base + size)))
        reps = max(len(a) for a in args)
        for k in range(reps):
            qs = tuple(a[k] if len(a) > 1 else a[0] for a in args)
            if name == "u1":
                gates.append(("u3", qs, (0.0, 0.0, ps[0])))
            elif name == "u2":
                gates.append(("u3", qs, (math.pi / 2, ps[0], ps[1])))
            else:
                gates.append((name, qs, tuple(ps)))
    return nq, gates

// OpenQASM 2.0 front-end (the paper's simulators accept circuits from
// several front-ends, OpenQASM among them, Sec. II; its benchmark suite is
// written in it, Sec. III).  Host code only: the text is parsed into the gate
// arrays of nwq_apply_circuit, so the fusion planner sees the whole circuit.
//
// Accepted: the OPENQASM 2.0 header, include lines, qreg / creg
// declarations (quantum registers are laid out in declaration order, the
// first register's qubit 0 being qubit 0), the qelib1 gates id x y z h s sdg
// t tdg rx ry rz u1 u2 u3 u p cx CX cz swap rzz, the built-in U, register
// broadcast (a gate on whole registers of equal size applies qubit by
// qubit), parameter expressions of numbers, pi, + - * / ^, unary minus,
// parentheses and the functions sin cos tan exp ln sqrt, and barrier /
// measure / reset-free programs (barrier and measure are skipped).
// Anything else (gate definitions, if, reset, opaque) is rejected with
// NWQ_EINVAL and the line number.  Rotations keep the engine's convention
// exp(-i theta P / 2), which can differ from a library's textual definition
// (rz as u1, say) by a global phase only.
#include <cctype>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "engine.h"

namespace nwq {
namespace {

struct QGate {
  int type;
  int q[2];
  double p[3];
};

class Parser {
 public:
  explicit Parser(const char* s) : src_(s) {}

  int run(std::vector<QGate>& out, int& nqubits) {
    skip();
    if (!word("OPENQASM")) return fail("expected the OPENQASM 2.0 header");
    double ver = 0;
    if (!number(ver) || ver != 2.0) return fail("only OpenQASM 2.0 is accepted");
    if (!expect(';')) return err_;
    while (true) {
      skip();
      if (!*pos()) break;
      std::string id;
      if (!ident(id)) return fail("expected a statement");
      int rc = NWQ_OK;
      if (id == "include") rc = include();
      else if (id == "qreg" || id == "creg") rc = reg(id == "qreg");
      else if (id == "barrier") rc = skip_statement();
      else if (id == "measure") rc = skip_statement();
      else if (id == "gate" || id == "opaque" || id == "if" || id == "reset")
        rc = fail("'" + id + "' is not supported");
      else rc = gate(id, out);
      if (rc) return rc;
    }
    nqubits = nq_;
    return NWQ_OK;
  }

 private:
  const char* src_;
  size_t i_ = 0;
  int line_ = 1;
  int nq_ = 0;
  int err_ = NWQ_EINVAL;
  int depth_ = 0;         // nesting of parentheses, signs and powers in an expression
  struct Reg { int base, size; };
  std::map<std::string, Reg> qregs_;
  std::map<std::string, int> cregs_;

  const char* pos() const { return src_ + i_; }
  int fail(const std::string& m) { return set_error(NWQ_EINVAL, "qasm line " + std::to_string(line_) + ": " + m); }

  void skip() {
    while (true) {
      const char c = src_[i_];
      if (c == '\n') { ++line_; ++i_; }
      else if (c == ' ' || c == '\t' || c == '\r') ++i_;
      else if (c == '/' && src_[i_ + 1] == '/') { while (src_[i_] && src_[i_] != '\n') ++i_; }
      else break;
    }
  }
  bool peek(char c) { skip(); return src_[i_] == c; }
  bool accept(char c) {
    if (peek(c)) { ++i_; return true; }
    return false;
  }
  bool expect(char c) {
    if (accept(c)) return true;
    err_ = fail(std::string("expected '") + c + "'");
    return false;
  }
  bool ident(std::string& s) {
    skip();
    if (!(std::isalpha((unsigned char)src_[i_]) || src_[i_] == '_')) return false;
    size_t j = i_;
    while (std::isalnum((unsigned char)src_[j]) || src_[j] == '_') ++j;
    s.assign(src_ + i_, j - i_);
    i_ = j;
    return true;
  }
  bool word(const char* w) {
    skip();
    const size_t n = std::strlen(w);
    if (std::strncmp(src_ + i_, w, n) != 0) return false;
    i_ += n;
    return true;
  }
  bool number(double& v) {
    skip();
    const char* b = src_ + i_;
    char* e = nullptr;
    if (!(std::isdigit((unsigned char)*b) || *b == '.')) return false;
    v = std::strtod(b, &e);
    if (e == b) return false;
    i_ += (size_t)(e - b);
    return true;
  }
  bool integer(int& v) {
    skip();
    if (!std::isdigit((unsigned char)src_[i_])) return false;
    long x = 0;
    while (std::isdigit((unsigned char)src_[i_])) {
      x = x * 10 + (src_[i_++] - '0');
      if (x > (1L << 30)) return false;
    }
    v = (int)x;
    return true;
  }
  int skip_statement() {
    while (src_[i_] && src_[i_] != ';') {
      if (src_[i_] == '\n') ++line_;
      ++i_;
    }
    if (!src_[i_]) return fail("missing ';'");
    ++i_;
    return NWQ_OK;
  }
  int include() {
    skip();
    if (src_[i_] != '"') return fail("expected a file name");
    ++i_;
    while (src_[i_] && src_[i_] != '"' && src_[i_] != '\n') ++i_;
    if (src_[i_] != '"') return fail("unterminated file name");
    ++i_;
    return expect(';') ? NWQ_OK : err_;
  }
  int reg(bool quantum) {
    std::string name;
    int size = 0;
    if (!ident(name)) return fail("expected a register name");
    if (!expect('[')) return err_;
    if (!integer(size) || size < 1) return fail("bad register size");
    if (!expect(']') || !expect(';')) return err_;
    if (qregs_.count(name) || cregs_.count(name)) return fail("register '" + name + "' declared twice");
    if (quantum) {
      if (nq_ + size > 34) return fail("more than 34 qubits");
      qregs_[name] = Reg{nq_, size};
      nq_ += size;
    } else {
      cregs_[name] = size;
    }
    return NWQ_OK;
  }

  // expression grammar: sum := prod {(+|-) prod}; prod := power {(*|/) power};
  // power := unary [^ power]; unary := -unary | primary
  bool expr(double& v) { return sum(v); }
  bool sum(double& v) {
    if (!prod(v)) return false;
    while (true) {
      if (accept('+')) { double r; if (!prod(r)) return false; v += r; }
      else if (accept('-')) { double r; if (!prod(r)) return false; v -= r; }
      else return true;
    }
  }
  bool prod(double& v) {
    if (!power(v)) return false;
    while (true) {
      if (accept('*')) { double r; if (!power(r)) return false; v *= r; }
      else if (accept('/')) { double r; if (!power(r)) return false; v /= r; }
      else return true;
    }
  }
  bool power(double& v) {
    if (!unary(v)) return false;
    if (accept('^')) {
      double r;
      if (++depth_ > 64) return false;
      const bool ok = power(r);
      --depth_;
      if (!ok) return false;
      v = std::pow(v, r);
    }
    return true;
  }
  bool unary(double& v) {
    if (accept('-') || accept('+')) {
      const bool neg = src_[i_ - 1] == '-';
      if (++depth_ > 64) return false;
      const bool ok = unary(v);
      --depth_;
      if (ok && neg) v = -v;
      return ok;
    }
    return primary(v);
  }
  bool primary(double& v) {
    if (accept('(')) {
      if (++depth_ > 64) return false;   // bounded nesting
      const bool ok = expr(v) && expect(')');
      --depth_;
      return ok;
    }
    if (number(v)) return true;
    std::string id;
    if (!ident(id)) return false;
    if (id == "pi") { v = M_PI; return true; }
    double (*f)(double) = nullptr;
    if (id == "sin") f = std::sin;
    else if (id == "cos") f = std::cos;
    else if (id == "tan") f = std::tan;
    else if (id == "exp") f = std::exp;
    else if (id == "ln") f = std::log;
    else if (id == "sqrt") f = std::sqrt;
    if (!f || !expect('(')) return false;
    if (++depth_ > 64) return false;     // nested calls count like parentheses
    double a;
    if (!expr(a) || !expect(')')) return false;
    --depth_;
    v = f(a);
    return true;
  }

  // an argument: reg[i] (one qubit) or reg (the whole register)
  bool argument(std::vector<int>& qs) {
    std::string name;
    if (!ident(name)) { fail("expected a qubit argument"); return false; }
    auto it = qregs_.find(name);
    if (it == qregs_.end()) { fail("unknown quantum register '" + name + "'"); return false; }
    if (accept('[')) {
      int k;
      if (!integer(k)) { fail("expected a qubit index"); return false; }
      if (!expect(']')) return false;
      if (k >= it->second.size) { fail("index out of range for '" + name + "'"); return false; }
      qs.assign(1, it->second.base + k);
    } else {
      qs.clear();
      for (int k = 0; k < it->second.size; ++k) qs.push_back(it->second.base + k);
    }
    return true;
  }

  int gate(const std::string& id, std::vector<QGate>& out) {
    struct Def { int type, nq, np; };
    static const std::map<std::string, Def> defs = {
        {"id", {NWQ_GATE_I, 1, 0}},   {"x", {NWQ_GATE_X, 1, 0}},     {"y", {NWQ_GATE_Y, 1, 0}},
        {"z", {NWQ_GATE_Z, 1, 0}},    {"h", {NWQ_GATE_H, 1, 0}},     {"s", {NWQ_GATE_S, 1, 0}},
        {"sdg", {NWQ_GATE_SDG, 1, 0}}, {"t", {NWQ_GATE_T, 1, 0}},    {"tdg", {NWQ_GATE_TDG, 1, 0}},
        {"rx", {NWQ_GATE_RX, 1, 1}},  {"ry", {NWQ_GATE_RY, 1, 1}},   {"rz", {NWQ_GATE_RZ, 1, 1}},
        {"u1", {NWQ_GATE_U3, 1, 1}},  {"p", {NWQ_GATE_U3, 1, 1}},    {"u2", {NWQ_GATE_U3, 1, 2}},
        {"u3", {NWQ_GATE_U3, 1, 3}},  {"u", {NWQ_GATE_U3, 1, 3}},    {"U", {NWQ_GATE_U3, 1, 3}},
        {"cx", {NWQ_GATE_CX, 2, 0}},  {"CX", {NWQ_GATE_CX, 2, 0}},   {"cz", {NWQ_GATE_CZ, 2, 0}},
        {"swap", {NWQ_GATE_SWAP, 2, 0}}, {"rzz", {NWQ_GATE_RZZ, 2, 1}}};
    auto it = defs.find(id);
    if (it == defs.end()) return fail("unknown gate '" + id + "'");
    const Def& d = it->second;
    double a[3] = {0, 0, 0};
    int np = 0;
    if (accept('(')) {
      if (!accept(')')) {
        do {
          if (np == 3) return fail("too many parameters");
          if (!expr(a[np])) return fail("bad parameter expression");
          ++np;
        } while (accept(','));
        if (!expect(')')) return err_;
      }
    }
    if (np != d.np) return fail("'" + id + "' takes " + std::to_string(d.np) + " parameters");
    for (int k = 0; k < np; ++k)
      if (!std::isfinite(a[k])) return fail("non-finite parameter");
    std::vector<int> args[2];
    for (int k = 0; k < d.nq; ++k) {
      if (k > 0 && !expect(',')) return err_;
      if (!argument(args[k])) return NWQ_EINVAL;   // message set by argument()
    }
    if (!expect(';')) return err_;
    // parameters of the engine's U3(theta, phi, lambda)
    double p[3] = {a[0], a[1], a[2]};
    if (id == "u1" || id == "p") { p[0] = 0; p[1] = 0; p[2] = a[0]; }
    else if (id == "u2") { p[0] = M_PI / 2; p[1] = a[0]; p[2] = a[1]; }
    size_t reps = 1;
    for (int k = 0; k < d.nq; ++k)
      if (args[k].size() > 1) {
        if (reps > 1 && args[k].size() != reps) return fail("registers of different sizes");
        reps = args[k].size();
      }
    for (size_t r = 0; r < reps; ++r) {
      QGate g{};
      g.type = d.type;
      for (int k = 0; k < d.nq; ++k) g.q[k] = args[k].size() > 1 ? args[k][r] : args[k][0];
      if (d.nq == 1) g.q[1] = 0;
      if (d.nq == 2 && g.q[0] == g.q[1]) return fail("repeated qubit");
      for (int k = 0; k < 3; ++k) g.p[k] = p[k];
      out.push_back(g);
    }
    return NWQ_OK;
  }
};

}  // namespace
}  // namespace nwq

using namespace nwq;

extern "C" {

int nwq_qasm_parse(const char* text, int* n_qubits, int* n_gates, int capacity, int* types, int* qubits,
                   double* params) {
  if (!text || !n_qubits || !n_gates) return set_error(NWQ_EINVAL, "NULL argument");
  if (capacity < 0 || (capacity > 0 && (!types || !qubits || !params))) return set_error(NWQ_EINVAL, "bad output arrays");
  std::vector<QGate> gates;
  int nq = 0;
  Parser parser(text);
  const int rc = parser.run(gates, nq);
  if (rc) return rc;
  *n_qubits = nq;
  *n_gates = (int)gates.size();
  const int m = std::min<int>(capacity, (int)gates.size());
  for (int i = 0; i < m; ++i) {
    types[i] = gates[i].type;
    qubits[2 * i] = gates[i].q[0];
    qubits[2 * i + 1] = gates[i].q[1];
    for (int k = 0; k < 3; ++k) params[3 * i + k] = gates[i].p[k];
  }
  return NWQ_OK;
}

int nwq_apply_qasm(nwq_handle h, const char* text) {
  if (!h) return set_error(NWQ_EINVAL, "NULL handle");
  int nq = 0, ng = 0;
  int rc = nwq_qasm_parse(text, &nq, &ng, 0, nullptr, nullptr, nullptr);
  if (rc) return rc;
  if (nq != h->n) return set_error(NWQ_ERANGE, "program declares " + std::to_string(nq) + " qubits, handle has " +
                                                   std::to_string(h->n));
  std::vector<int> types(ng), qubits(2 * (size_t)ng);
  std::vector<double> params(3 * (size_t)ng);
  rc = nwq_qasm_parse(text, &nq, &ng, ng, types.data(), qubits.data(), params.data());
  if (rc) return rc;
  return nwq_apply_circuit(h, ng, types.data(), qubits.data(), params.data());
}

}  // extern "C"

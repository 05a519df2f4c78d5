// Whole-circuit application and the fusion planner.
//
// The planner walks the gate list and builds blocks greedily: a block owns a
// tile set T = {0..c-1} u H with |H| <= k - c high qubits.  A gate joins the
// current block when none of its qubits is held by an earlier gate that was
// left out (so moving it forward never crosses a gate it does not commute
// with by disjointness) and its qubits fit in T after adding the new high
// qubits it needs.  Left-out gates start the next block.  Each block is one
// read and one write of the state through LDS.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "engine.h"

namespace nwq {
namespace {

struct PGate {
  int type;
  int q[2];
  int nq;
  double p[3];
};

struct Block {
  int c = 0, m = 0;
  int hi[8] = {0};
  std::vector<int> gates;    // indices into the circuit
};

// Every block has at least two high slots (c <= k - 2), so the first
// remaining gate always fits and each round absorbs at least one gate.
std::vector<Block> plan_blocks(const std::vector<PGate>& g, int n, int k) {
  const int c = n <= k ? n : std::min(6, k - 2);
  const int mmax = n <= k ? 0 : k - c;
  std::vector<int> rem(g.size());
  for (size_t i = 0; i < g.size(); ++i) rem[i] = (int)i;
  std::vector<Block> out;
  std::vector<char> blocked(n);
  while (!rem.empty()) {
    Block b;
    b.c = c;
    std::vector<int> keep;
    std::fill(blocked.begin(), blocked.end(), 0);
    int nblocked = 0;
    std::vector<int> H;
    for (int idx : rem) {
      const PGate& gg = g[idx];
      bool hit = false;
      for (int j = 0; j < gg.nq; ++j) hit |= blocked[gg.q[j]] != 0;
      bool take = false;
      if (!hit && nblocked < n) {
        std::vector<int> need;
        for (int j = 0; j < gg.nq; ++j)
          if (gg.q[j] >= c && std::find(H.begin(), H.end(), gg.q[j]) == H.end()) need.push_back(gg.q[j]);
        if ((int)(H.size() + need.size()) <= mmax) {
          H.insert(H.end(), need.begin(), need.end());
          take = true;
        }
      }
      if (take) {
        b.gates.push_back(idx);
      } else {
        keep.push_back(idx);
        for (int j = 0; j < gg.nq; ++j)
          if (!blocked[gg.q[j]]) {
            blocked[gg.q[j]] = 1;
            ++nblocked;
          }
      }
    }
    if (b.gates.empty()) return {};   // cannot happen with two high slots; caller reports it
    std::sort(H.begin(), H.end());
    b.m = (int)H.size();
    for (int i = 0; i < b.m; ++i) b.hi[i] = H[i];
    out.push_back(std::move(b));
    rem.swap(keep);
  }
  return out;
}

int local_bit(const Block& b, int q) {
  if (q < b.c) return q;
  for (int i = 0; i < b.m; ++i)
    if (b.hi[i] == q) return b.c + i;
  return -1;
}

}  // namespace

static int apply_fused(nwq_state* h, const std::vector<PGate>& gates) {
  const std::vector<Block> blocks = plan_blocks(gates, h->n, h->fuse_k);
  if (blocks.empty()) return set_error(NWQ_EINVAL, "fusion planner made no progress");
  // Program: FusedOp table then double2 matrix table, in one upload.
  std::vector<FusedOp> ops;
  std::vector<double2> mats;
  std::vector<FusedBlockDev> bdev;
  for (const Block& b : blocks) {
    FusedBlockDev d{};
    d.c = b.c;
    d.m = b.m;
    for (int i = 0; i < b.m; ++i) d.hi[i] = b.hi[i];
    d.op_begin = (int)ops.size();
    for (int gi : b.gates) {
      const PGate& g = gates[gi];
      cd m[16];
      gate_matrix(g.type, g.p, m);
      FusedOp op{};
      op.mat = (int)mats.size();
      const int l0 = local_bit(b, g.q[0]);
      const int l1 = g.nq == 2 ? local_bit(b, g.q[1]) : -1;
      op.lo = g.nq == 2 ? std::min(l0, l1) : l0;
      op.hi = g.nq == 2 ? std::max(l0, l1) : 0;
      switch (g.type) {
        case NWQ_GATE_I:
          continue;
        case NWQ_GATE_Z: case NWQ_GATE_S: case NWQ_GATE_SDG: case NWQ_GATE_T: case NWQ_GATE_TDG: case NWQ_GATE_RZ:
          op.kind = 1;
          mats.push_back(make_double2(m[0].real(), m[0].imag()));
          mats.push_back(make_double2(m[3].real(), m[3].imag()));
          break;
        case NWQ_GATE_CX:
          op.kind = 3;
          op.o0 = 1 << l0;
          op.o1 = (1 << l0) + (1 << l1);
          break;
        case NWQ_GATE_SWAP:
          op.kind = 3;
          op.o0 = 1 << l0;
          op.o1 = 1 << l1;
          break;
        case NWQ_GATE_CZ: case NWQ_GATE_RZZ:
          op.kind = 4;
          op.o0 = l0;
          op.o1 = l1;
          for (int u = 0; u < 4; ++u) mats.push_back(make_double2(m[5 * u].real(), m[5 * u].imag()));
          break;
        default:
          op.kind = 0;
          for (int i = 0; i < 4; ++i) mats.push_back(make_double2(m[i].real(), m[i].imag()));
          break;
      }
      ops.push_back(op);
    }
    d.op_count = (int)ops.size() - d.op_begin;
    if (d.op_count > 0) bdev.push_back(d);
  }
  const size_t ops_bytes = ops.size() * sizeof(FusedOp);
  const size_t mats_off = (ops_bytes + 255) & ~size_t(255);
  const size_t total = mats_off + mats.size() * sizeof(double2) + 16;
  std::vector<char> prog(total, 0);
  if (!ops.empty()) std::memcpy(prog.data(), ops.data(), ops_bytes);
  if (!mats.empty()) std::memcpy(prog.data() + mats_off, mats.data(), mats.size() * sizeof(double2));
  void* dev = nullptr;
  if (total <= (2u << 20)) {
    const int rc = arena_put(h, prog.data(), total, &dev);
    if (rc) return rc;
  } else {
    if (total > h->fuse_cap) {
      if (h->fuse_dev) {
        int rc = check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        if (rc) return rc;
        (void)hipFree(h->fuse_dev);
        h->fuse_dev = nullptr;
      }
      int rc = check_hip(hipMalloc(&h->fuse_dev, total), "hipMalloc(fusion program)");
      if (rc) return rc;
      h->fuse_cap = total;
    }
    int rc = check_hip(hipMemcpyAsync(h->fuse_dev, prog.data(), total, hipMemcpyHostToDevice, h->stream),
                       "hipMemcpyAsync(fusion program)");
    if (rc) return rc;
    rc = check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize(fusion program)");
    if (rc) return rc;
    dev = h->fuse_dev;
  }
  const FusedOp* dops = static_cast<const FusedOp*>(dev);
  const double2* dmats = reinterpret_cast<const double2*>(static_cast<char*>(dev) + mats_off);
  for (const FusedBlockDev& d : bdev) {
    timing_begin(h, KC_FUSED);
    launch_fused_block(h->stream, h->data, h->nbits, d, dops, dmats, h->fuse_k);
    timing_end(h);
    const int rc = check_hip(hipGetLastError(), "fused_block");
    if (rc) return rc;
  }
  h->last_blocks = (int)bdev.size();
  h->last_fused_gates = (int)ops.size();
  return NWQ_OK;
}

}  // namespace nwq

using namespace nwq;

extern "C" {

static int parse_circuit(int n, int n_gates, const int* types, const int* qubits, const double* params,
                         bool need_params, std::vector<PGate>& gates) {
  if (n_gates < 0 || (n_gates > 0 && (!types || !qubits))) return set_error(NWQ_EINVAL, "bad circuit arrays");
  gates.assign(n_gates, PGate{});
  for (int i = 0; i < n_gates; ++i) {
    PGate& g = gates[i];
    g.type = types[i];
    int nq = 0, np = 0;
    switch (g.type) {
      case NWQ_GATE_RX: case NWQ_GATE_RY: case NWQ_GATE_RZ: nq = 1; np = 1; break;
      case NWQ_GATE_U3: nq = 1; np = 3; break;
      case NWQ_GATE_CX: case NWQ_GATE_CZ: case NWQ_GATE_SWAP: nq = 2; break;
      case NWQ_GATE_RZZ: nq = 2; np = 1; break;
      default:
        if (g.type < 0 || g.type >= NWQ_GATE_COUNT) return set_error(NWQ_EINVAL, "gate " + std::to_string(i) + ": unknown type");
        nq = 1;
    }
    g.nq = nq;
    g.q[0] = qubits[2 * i];
    g.q[1] = nq == 2 ? qubits[2 * i + 1] : -1;
    for (int j = 0; j < 3; ++j) g.p[j] = params ? params[3 * i + j] : 0.0;
    if (np > 0 && need_params && params == nullptr) return set_error(NWQ_EINVAL, "params pointer is NULL");
    for (int j = 0; j < np; ++j)
      if (!std::isfinite(g.p[j])) return set_error(NWQ_EINVAL, "gate " + std::to_string(i) + ": non-finite parameter");
    for (int j = 0; j < nq; ++j)
      if (g.q[j] < 0 || g.q[j] >= n) return set_error(NWQ_ERANGE, "gate " + std::to_string(i) + ": qubit out of range");
    if (nq == 2 && g.q[0] == g.q[1]) return set_error(NWQ_EDUP, "gate " + std::to_string(i) + ": repeated qubit");
  }
  return NWQ_OK;
}

int nwq_apply_circuit(nwq_handle h, int n_gates, const int* types, const int* qubits, const double* params) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  std::vector<PGate> gates;
  // validate everything before launching anything
  int rc0 = parse_circuit(h->n, n_gates, types, qubits, params, true, gates);
  if (rc0) return rc0;
  h->last_blocks = 0;
  h->last_fused_gates = 0;
  if (h->kind == NWQ_KIND_SV && h->fuse_k > 0 && n_gates > 0) return apply_fused(h, gates);
  for (const PGate& g : gates) {
    int rc;
    if (h->kind == NWQ_KIND_SV) {
      rc = sv_apply_gate_validated(h, g.type, g.q, g.p);
    } else {
      cd m[16];
      gate_matrix(g.type, g.p, m);
      rc = dm_apply_unitary(h, g.q, g.nq, m);
    }
    if (rc) return rc;
  }
  return NWQ_OK;
}

int nwq_set_fusion(nwq_handle h, int k, int* k_out) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  if (k != 0 && (k < 6 || k > 13)) return set_error(NWQ_EINVAL, "fusion width must be 0 or in [6, 13]");
  if (h->kind != NWQ_KIND_SV && k != 0) return set_error(NWQ_EKIND, "fusion applies to state-vector handles");
  h->fuse_k = k;
  if (k_out) *k_out = k;
  return NWQ_OK;
}

int nwq_fusion_plan(int n, int k, int n_gates, const int* types, const int* qubits, int* n_blocks,
                    int* block_of_gate, int* block_qubits) {
  if (n < 1 || n > 34) return set_error(NWQ_ERANGE, "n outside [1, 34]");
  if (k < 6 || k > 13) return set_error(NWQ_EINVAL, "fusion width must be in [6, 13]");
  if (!n_blocks || (n_gates > 0 && !block_of_gate)) return set_error(NWQ_EINVAL, "NULL output pointer");
  std::vector<PGate> gates;
  int rc = parse_circuit(n, n_gates, types, qubits, nullptr, false, gates);
  if (rc) return rc;
  const std::vector<Block> blocks = plan_blocks(gates, n, k);
  if (n_gates > 0 && blocks.empty()) return set_error(NWQ_EINVAL, "fusion planner made no progress");
  *n_blocks = (int)blocks.size();
  for (size_t b = 0; b < blocks.size(); ++b) {
    for (int gi : blocks[b].gates) block_of_gate[gi] = (int)b;
    if (block_qubits) {
      unsigned long long mask = (1ull << blocks[b].c) - 1ull;
      for (int i = 0; i < blocks[b].m; ++i) mask |= 1ull << blocks[b].hi[i];
      block_qubits[2 * b] = (int)(mask & 0xffffffffull);
      block_qubits[2 * b + 1] = (int)(mask >> 32);
    }
  }
  return NWQ_OK;
}

int nwq_fusion_stats(nwq_handle h, int* blocks, int* gates) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  if (blocks) *blocks = h->last_blocks;
  if (gates) *gates = h->last_fused_gates;
  return NWQ_OK;
}

}  // extern "C"

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
#include <array>
#include <cmath>
#include <cstring>

#include "engine.h"

namespace nwq {

// A state vector's blocks keep 6 low bits (each wave's loads cover 1 KiB
// runs).  On vec(rho) a qubit above the low bits takes two high slots (its
// column bit q and row bit q + n), so density matrices keep 4: at n=14,
// k=12 the noisy TFIM needs 35 blocks instead of 46.
int fusion_low_bits(const nwq_state* h, int nbits, int k) {
  if (nbits <= k) return nbits;
  const int c = h->fuse_c > 0 ? h->fuse_c : (h->kind == NWQ_KIND_DM ? 4 : 6);
  return std::min(std::max(c, k - 8), k - 2);
}

// Every block has at least two high slots (c <= k - 2), so the first
// remaining one- or two-qubit gate always fits and each round absorbs at
// least one gate (a four-bit DM superoperator is queued only when the width
// leaves four).
std::vector<Block> plan_blocks(const std::vector<PGate>& g, int n, int k, int c_req) {
  int c = c_req < 0 ? std::min(6, k - 2) : std::min(std::max(c_req, k - 8), k - 2);
  if (n <= k) c = n;
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
    for (size_t r = 0; r < rem.size(); ++r) {
      if (nblocked == n) {   // every qubit is held by a left-out gate: the rest waits
        keep.insert(keep.end(), rem.begin() + r, rem.end());
        break;
      }
      const int idx = rem[r];
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

// Widen a block's tile with unused high qubits (ascending) up to width
// k_target (or n): more amplitudes per tile, same gates, same result.
void pad_block(Block& b, int n, int k_target) {
  const int want = std::min(k_target, n);
  for (int q = b.c; q < n && b.c + b.m < want && b.m < 8; ++q) {
    bool used = false;
    for (int i = 0; i < b.m; ++i) used |= b.hi[i] == q;
    if (!used) b.hi[b.m++] = q;
  }
  std::sort(b.hi, b.hi + b.m);
}

int local_bit(const Block& b, int q) {
  if (q < b.c) return q;
  for (int i = 0; i < b.m; ++i)
    if (b.hi[i] == q) return b.c + i;
  return -1;
}

// Encode one gate as a FusedOp (bits are tile-local for the per-gate LDS
// kernel, register-bit indices for the register-blocked kernel) and append
// its matrix entries.  Returns false for the identity (nothing to do).
static bool encode_op(const PGate& g, int b0, int b1, std::vector<double2>& mats, FusedOp& op, bool reg,
                      const std::vector<cd>* side) {
  op = FusedOp{};
  if (g.type == kGateDiag4) {   // diagonal 4x4 from the side table, operator order (q[0], q[1])
    op.mat = (int)mats.size();
    op.lo = std::min(b0, b1);
    op.hi = std::max(b0, b1);
    op.kind = 4;
    op.o0 = b0;
    op.o1 = b1;
    const cd* M = side->data() + (size_t)g.p[0];
    for (int u = 0; u < 4; ++u) mats.push_back(make_double2(M[5 * u].real(), M[5 * u].imag()));
    return true;
  }
  if (g.type == kGateMat2) {   // 2x2 from the side table
    const cd* M = side->data() + (size_t)g.p[0];
    op.mat = (int)mats.size();
    op.lo = b0;
    if (M[1] == 0.0 && M[2] == 0.0) {
      op.kind = 1;
      mats.push_back(make_double2(M[0].real(), M[0].imag()));
      mats.push_back(make_double2(M[3].real(), M[3].imag()));
      return true;
    }
    op.kind = 0;
    bool real = true;
    for (int i = 0; i < 4; ++i) real = real && M[i].imag() == 0.0;
    op.real00 = real ? 2 : (M[0].imag() == 0.0 ? 1 : 0);
    for (int i = 0; i < 4; ++i) mats.push_back(make_double2(M[i].real(), M[i].imag()));
    return true;
  }
  if (g.type == kGateMat4) {   // dense 4x4 from the side table, operator order (q[0], q[1])
    op.mat = (int)mats.size();
    op.lo = std::min(b0, b1);
    op.hi = std::max(b0, b1);
    op.kind = 2;
    op.o0 = reg ? b0 : (1 << b0);
    op.o1 = reg ? b1 : (1 << b1);
    const cd* M = side->data() + (size_t)g.p[0];
    for (int i = 0; i < 16; ++i) mats.push_back(make_double2(M[i].real(), M[i].imag()));
    return true;
  }
  cd m[16];
  gate_matrix(g.type, g.p, m);
  op.mat = (int)mats.size();
  op.lo = g.nq == 2 ? std::min(b0, b1) : b0;
  op.hi = g.nq == 2 ? std::max(b0, b1) : 0;
  switch (g.type) {
    case NWQ_GATE_I:
      return false;
    case NWQ_GATE_Z: case NWQ_GATE_S: case NWQ_GATE_SDG: case NWQ_GATE_T: case NWQ_GATE_TDG: case NWQ_GATE_RZ:
      op.kind = 1;
      mats.push_back(make_double2(m[0].real(), m[0].imag()));
      mats.push_back(make_double2(m[3].real(), m[3].imag()));
      return true;
    case NWQ_GATE_CX:
      op.kind = 3;
      op.o0 = reg ? b0 : (1 << b0);
      op.o1 = reg ? b1 : (1 << b0) + (1 << b1);
      return true;
    case NWQ_GATE_SWAP:
      op.kind = reg ? 5 : 3;
      op.o0 = reg ? b0 : (1 << b0);
      op.o1 = reg ? b1 : (1 << b1);
      return true;
    case NWQ_GATE_CZ: case NWQ_GATE_RZZ:
      op.kind = 4;
      op.o0 = b0;
      op.o1 = b1;
      for (int u = 0; u < 4; ++u) mats.push_back(make_double2(m[5 * u].real(), m[5 * u].imag()));
      return true;
    default:
      op.kind = 0;
      op.real00 = (m[0].imag() == 0.0 && m[1].imag() == 0.0 && m[2].imag() == 0.0 && m[3].imag() == 0.0)
                      ? 2
                      : (m[0].imag() == 0.0 ? 1 : 0);
      for (int i = 0; i < 4; ++i) mats.push_back(make_double2(m[i].real(), m[i].imag()));
      return true;
  }
}

// ---------------------------------------------------------------------------
// Gate products.  A two-qubit gate takes the one-qubit gates next to it on
// its two qubits (back to the previous and on to the next two-qubit gate on
// each: each of them commutes with everything it is moved past) and the
// product becomes one gate, when that costs less FP64 work than the gates one
// by one.  Runs of one-qubit gates on one qubit that are left become one 2x2
// the same way.  Costs are FP64 instructions per amplitude in the
// register-blocked kernel plus one per op for its dispatch.  Products act on
// at most two qubits, so blocks and register phases are planned over them as
// over gates.
// ---------------------------------------------------------------------------
namespace {

struct FuseItem {
  int gate = -1;              // an original gate (index into the gate list), or -1: a product
  int nb = 0, r[2] = {0, 0};  // product: its qubits; r[0] is bit 0 of the operator index
  cd m[16];                   // product: 2x2 (nb = 1) or 4x4 (nb = 2), row-major
};

bool is_diag(const cd* m, int dim) {
  for (int u = 0; u < dim; ++u)
    for (int v = 0; v < dim; ++v)
      if (u != v && m[u * dim + v] != 0.0) return false;
  return true;
}

int matrix_cost(const cd* m, int nb) {
  if (nb == 2) return is_diag(m, 4) ? 4 : 16;
  if (is_diag(m, 2)) return 4;
  bool real = true;
  for (int i = 0; i < 4; ++i) real = real && m[i].imag() == 0.0;
  return real ? 4 : (m[0].imag() == 0.0 ? 7 : 8);
}

int gate_cost(const PGate& g) {
  switch (g.type) {
    case NWQ_GATE_I: return 0;
    case NWQ_GATE_CX: case NWQ_GATE_SWAP: return 0;   // register permutations
    case NWQ_GATE_CZ: case NWQ_GATE_RZZ: return 4;
    case kGateMat4: return 16;
    case kGateDiag4: return 4;
    default: {
      cd m[16];
      gate_matrix(g.type, g.p, m);
      return matrix_cost(m, 1);
    }
  }
}

// M <- G M, G acting on bit `pos` (0 or 1) of the 4x4 operator index
void lmul_1q(cd* M, const cd* G, int pos) {
  cd R[16];
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) {
      cd acc = 0.0;
      for (int w = 0; w < 4; ++w)
        if ((u & ~(1 << pos)) == (w & ~(1 << pos))) acc += G[((u >> pos) & 1) * 2 + ((w >> pos) & 1)] * M[w * 4 + v];
      R[u * 4 + v] = acc;
    }
  std::memcpy(M, R, sizeof R);
}

// M <- G M, G a 4x4 in its own (q0, q1) index order; swapped: q0 is bit 1 here
void lmul_2q(cd* M, const cd* G, bool swapped) {
  auto sw = [&](int u) { return swapped ? ((u & 1) << 1) | (u >> 1) : u; };
  cd R[16];
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) {
      cd acc = 0.0;
      for (int w = 0; w < 4; ++w) acc += G[sw(u) * 4 + sw(w)] * M[w * 4 + v];
      R[u * 4 + v] = acc;
    }
  std::memcpy(M, R, sizeof R);
}

// seq: the gates in order (indices into gates); r0 / r1: their qubits (r1 <
// 0 for one-qubit gates).  Returns the ops in application order.
std::vector<FuseItem> gate_products(const std::vector<int>& seq, const std::vector<PGate>& gates,
                                  const std::vector<int>& r0, const std::vector<int>& r1) {
  const int n = (int)seq.size();
  auto two = [&](int i) { return r1[i] >= 0; };
  // positions touching each bit, and each position's place in its bits' lists
  int nbit = 0;
  for (int i = 0; i < n; ++i) nbit = std::max(nbit, std::max(r0[i], r1[i]) + 1);
  std::vector<std::vector<int>> on(nbit);
  std::vector<int> at0(n), at1(n, -1);
  for (int i = 0; i < n; ++i) {
    at0[i] = (int)on[r0[i]].size();
    on[r0[i]].push_back(i);
    if (two(i)) {
      at1[i] = (int)on[r1[i]].size();
      on[r1[i]].push_back(i);
    }
  }
  std::vector<int> owner(n, -1), unit_at(n, -1);
  std::vector<FuseItem> units;
  for (int p = 0; p < n; ++p) {
    if (!two(p)) continue;
    std::vector<int> take;
    for (int side = 0; side < 2; ++side) {
      const std::vector<int>& lst = on[side == 0 ? r0[p] : r1[p]];
      const int here = side == 0 ? at0[p] : at1[p];
      for (int j = here - 1; j >= 0; --j) {
        const int t = lst[j];
        if (two(t) || owner[t] != -1) break;
        take.push_back(t);
      }
      for (int j = here + 1; j < (int)lst.size(); ++j) {
        const int t = lst[j];
        if (two(t)) break;
        take.push_back(t);
      }
    }
    if (take.empty()) continue;
    take.push_back(p);
    std::sort(take.begin(), take.end());
    FuseItem u;
    u.nb = 2;
    u.r[0] = r0[p];
    u.r[1] = r1[p];
    for (int i = 0; i < 16; ++i) u.m[i] = (i % 5 == 0) ? 1.0 : 0.0;
    int unfused = 0;
    for (int i : take) {
      const PGate& g = gates[seq[i]];
      unfused += gate_cost(g) + 1;
      cd G[16];
      gate_matrix(g.type, g.p, G);
      if (two(i)) lmul_2q(u.m, G, r0[i] != u.r[0]);
      else lmul_1q(u.m, G, r0[i] == u.r[0] ? 0 : 1);
    }
    if (matrix_cost(u.m, 2) + 1 >= unfused) continue;
    for (int i : take) owner[i] = (int)units.size();
    unit_at[p] = (int)units.size();
    units.push_back(u);
  }
  std::vector<FuseItem> out;
  for (int i = 0; i < n; ++i) {
    if (unit_at[i] >= 0) {
      out.push_back(units[unit_at[i]]);
      continue;
    }
    if (owner[i] != -1) continue;
    if (two(i)) {
      out.push_back(FuseItem{});
      out.back().gate = seq[i];
      continue;
    }
    std::vector<int> run{i};
    const std::vector<int>& lst = on[r0[i]];
    for (int j = at0[i] + 1; j < (int)lst.size(); ++j) {
      const int t = lst[j];
      if (two(t) || owner[t] != -1) break;
      run.push_back(t);
    }
    FuseItem u;
    u.nb = 1;
    u.r[0] = r0[i];
    u.m[0] = u.m[3] = 1.0;
    int unfused = 0;
    for (int t : run) {
      const PGate& g = gates[seq[t]];
      unfused += gate_cost(g) + 1;
      cd G[16];
      gate_matrix(g.type, g.p, G);
      const cd a = G[0] * u.m[0] + G[1] * u.m[2], b = G[0] * u.m[1] + G[1] * u.m[3];
      const cd c = G[2] * u.m[0] + G[3] * u.m[2], d = G[2] * u.m[1] + G[3] * u.m[3];
      u.m[0] = a; u.m[1] = b; u.m[2] = c; u.m[3] = d;
    }
    if (run.size() > 1 && matrix_cost(u.m, 1) + 1 < unfused) {
      for (int t : run) owner[t] = -2;
      out.push_back(u);
    } else {
      out.push_back(FuseItem{});
      out.back().gate = seq[i];
    }
  }
  return out;
}

}  // namespace

// Split a block's gates (tile-local bits) into register phases: greedily
// take, in order, every gate whose bits fit the phase's rbits register bits
// and that no earlier left-out gate shares a bit with; pad the set to rbits,
// from tile bit c up first (a set above the low c bits keeps each wave's
// lanes on contiguous amplitudes, so the phase can move between registers and
// HBM directly when it is the block's first or last).
std::vector<Phase> plan_phases(const std::vector<int>& order, const std::vector<std::array<int, 4>>& lb,
                               const std::vector<int>& nq, int k, int c, int rbits) {
  std::vector<Phase> out;
  std::vector<int> rem = order;
  while (!rem.empty()) {
    unsigned S = 0, blocked = 0;
    Phase ph;
    std::vector<int> keep;
    for (int gi : rem) {
      unsigned B = 0;
      for (int t = 0; t < nq[gi]; ++t) B |= 1u << lb[gi][t];
      if (B & blocked) {
        blocked |= B;
        keep.push_back(gi);
        continue;
      }
      if (__builtin_popcount(S | B) <= rbits) {
        S |= B;
        ph.gates.push_back(gi);
      } else {
        blocked |= B;
        keep.push_back(gi);
      }
    }
    for (int b = c; b < k && __builtin_popcount(S) < rbits; ++b) S |= 1u << b;
    for (int b = 0; b < k && __builtin_popcount(S) < rbits; ++b) S |= 1u << b;
    int r = 0;
    for (int b = 0; b < k; ++b)
      if ((S >> b) & 1u) ph.reg[r++] = b;
    for (; r < 4; ++r) ph.reg[r] = -1;
    out.push_back(std::move(ph));
    rem.swap(keep);
  }
  return out;
}

// Global offsets of the tile entries j * 2^(k - rbits), j < 2^rbits: the low
// c bits stay in place, tile bit c + i lands on qubit hi[i].
static unsigned long long tile_entry_offset(const FusedBlockDev& d, unsigned l) {
  unsigned long long g = l & ((1u << d.c) - 1u);
  for (int i = 0; i < d.m; ++i)
    if ((l >> (d.c + i)) & 1u) g |= 1ull << d.hi[i];
  return g;
}

void fill_entry_offsets(FusedBlockDev& d, int rbits) {
  const int k = d.c + d.m;
  d.direct = 0;
  for (int j = 0; j < 16; ++j) {
    d.joff[j] = d.jdir[j] = d.sdir[j] = 0;
    if (j < (1 << rbits)) d.joff[j] = tile_entry_offset(d, (unsigned)j << (k - rbits));
  }
}

// A phase's LDS offsets are padded by one entry per 16 (o + o / 16); the
// entry offset is recovered from them.
void set_direct_io(FusedBlockDev& d, const FusedPhase& first, const FusedPhase& last, int rbits) {
  auto above_c = [&](const FusedPhase& ph) {
    for (int r = 0; r < rbits; ++r)
      if (ph.reg[r] < d.c) return false;
    return true;
  };
  auto unpad = [](unsigned p) { return 16u * (p / 17u) + p % 17u; };
  d.direct = 0;
  if (above_c(first)) {
    d.direct |= 1;
    for (int j = 0; j < (1 << rbits); ++j) d.jdir[j] = tile_entry_offset(d, unpad(first.ld_off[j]));
  }
  if (above_c(last)) {
    d.direct |= 2;
    for (int j = 0; j < (1 << rbits); ++j) d.sdir[j] = tile_entry_offset(d, unpad(last.st_off[j]));
  }
}

// Runs a gate list through fused blocks over `nbits` bits of the vector (the
// qubit count for a state vector; 2n for the vectorised density matrix, whose
// queued 1q superoperators arrive as kGateMat4 gates with matrices in `side`).
int apply_fused(nwq_state* h, const std::vector<PGate>& gates_in, int nbits, const std::vector<cd>* side_in,
                bool from_zero) {
  // Gate products over the whole circuit (state vectors, register-blocked
  // kernels): they act on at most two qubits, so the blocks and their register
  // phases are planned over them as over gates, and no boundary cuts one.
  std::vector<PGate> prod_gates;
  std::vector<cd> prod_side;
  const bool products = (h->fuse_flags & kFusedGateFusion) && side_in == nullptr && h->fuse_rb != 0;
  if (products) {
    std::vector<int> seq, r0, r1;
    for (size_t i = 0; i < gates_in.size(); ++i) {
      if (gates_in[i].type == NWQ_GATE_I) continue;
      seq.push_back((int)i);
      r0.push_back(gates_in[i].q[0]);
      r1.push_back(gates_in[i].nq == 2 ? gates_in[i].q[1] : -1);
    }
    for (const FuseItem& it : gate_products(seq, gates_in, r0, r1)) {
      if (it.gate >= 0) {
        prod_gates.push_back(gates_in[it.gate]);
        continue;
      }
      PGate g{};
      g.nq = it.nb;
      g.q[0] = it.r[0];
      g.q[1] = it.nb == 2 ? it.r[1] : 0;
      g.type = it.nb == 1 ? kGateMat2 : (is_diag(it.m, 4) ? kGateDiag4 : kGateMat4);
      g.p[0] = (double)prod_side.size();
      for (int i = 0; i < 16; ++i) prod_side.push_back(it.m[i]);
      prod_gates.push_back(g);
    }
  }
  const std::vector<PGate>& gates = products ? prod_gates : gates_in;
  const std::vector<cd>* side = products ? &prod_side : side_in;
  if (gates.empty()) {   // identities only
    h->last_blocks = h->last_fused_gates = h->last_phases = 0;
    return NWQ_OK;
  }
  const std::vector<Block> blocks = plan_blocks(gates, nbits, h->fuse_k, fusion_low_bits(h, nbits, h->fuse_k));
  if (blocks.empty()) return set_error(NWQ_EINVAL, "fusion planner made no progress");
  // Program: [phase table][op table][matrix table] in one upload.
  std::vector<FusedPhase> phases;
  std::vector<FusedOp> ops;
  std::vector<double2> mats;
  struct Launch { FusedBlockDev d; bool rb; int rbits; };
  std::vector<Launch> launches;
  for (Block b : blocks) {
    if (h->fuse_rb != 0 && b.c + b.m < 8 && nbits >= 8) pad_block(b, nbits, 8);
    FusedBlockDev d{};
    d.c = b.c;
    d.m = b.m;
    for (int i = 0; i < b.m; ++i) d.hi[i] = b.hi[i];
    const int k = b.c + b.m;
    const bool rb = h->fuse_rb != 0 && k >= 8;
    const int rbits = h->fuse_rb == 2 ? 3 : 4;
    if (!rb) {
      d.op_begin = (int)ops.size();
      for (int gi : b.gates) {
        const PGate& g = gates[gi];
        if (g.nq > 2) return set_error(NWQ_EINVAL, "a four-bit operator needs the register-blocked kernel");
        FusedOp op;
        if (encode_op(g, local_bit(b, g.q[0]), g.nq == 2 ? local_bit(b, g.q[1]) : 0, mats, op, false, side))
          ops.push_back(op);
      }
      d.op_count = (int)ops.size() - d.op_begin;
      if (d.op_count > 0) launches.push_back({d, false, 0});
      continue;
    }
    // the block's gates by block-local index (gid: the gate each one is), so
    // that planning costs time in the block's size, not the circuit's
    std::vector<int> gid, nq, order;
    std::vector<std::array<int, 4>> lb;
    for (int gi : b.gates) {
      if (gates[gi].type == NWQ_GATE_I) continue;
      if (gates[gi].nq > rbits) return set_error(NWQ_EINVAL, "an operator wider than the phase's register bits");
      std::array<int, 4> bits{};
      for (int t = 0; t < gates[gi].nq; ++t) bits[t] = local_bit(b, gates[gi].q[t]);
      order.push_back((int)gid.size());
      gid.push_back(gi);
      lb.push_back(bits);
      nq.push_back(gates[gi].nq);
    }
    if (order.empty()) continue;
    d.op_begin = (int)phases.size();
    for (const Phase& ph : plan_phases(order, lb, nq, k, b.c, rbits)) {
      FusedPhase fp{};
      for (int i = 0; i < 4; ++i) fp.reg[i] = ph.reg[i] < 0 ? 0 : ph.reg[i];
      fp.op_begin = (int)ops.size();
      auto ridx = [&](int bit) {
        for (int i = 0; i < rbits; ++i)
          if (ph.reg[i] == bit) return i;
        return -1;
      };
      std::vector<FusedOp> pops;
      for (int li : ph.gates) {
        const PGate& gate = gates[gid[li]];
        if (gate.type == kGateMat16) {   // all four register bits: the matrix in register order
          FusedOp op{};
          op.kind = 7;
          op.mat = (int)mats.size();
          int rt[4];
          for (int t = 0; t < 4; ++t) rt[t] = ridx(lb[li][t]);
          auto reg_index = [&](int u) {   // operator index -> register index
            int j = 0;
            for (int t = 0; t < 4; ++t) j |= ((u >> t) & 1) << rt[t];
            return j;
          };
          int inv[16];
          for (int u = 0; u < 16; ++u) inv[reg_index(u)] = u;
          const cd* M = side->data() + (size_t)gate.p[0];
          cd P[256];
          for (int r = 0; r < 16; ++r)
            for (int c2 = 0; c2 < 16; ++c2) P[r * 16 + c2] = M[inv[r] * 16 + inv[c2]];
          // a Pauli channel after a diagonal gate (RZZ, CZ, ...) leaves the
          // entries of rho off the 4x4 diagonal scaled and mixes only the
          // diagonal ones (registers 0, 5, 10, 15 in either qubit order)
          auto blk = [](int u) { return u % 5 == 0; };
          bool pauli = true;
          for (int r = 0; r < 16 && pauli; ++r)
            for (int c2 = 0; c2 < 16 && pauli; ++c2)
              if (r != c2 && !(blk(r) && blk(c2)) && P[r * 16 + c2] != 0.0) pauli = false;
          if (pauli) {
            op.kind = 8;
            for (int u = 0; u < 16; ++u) mats.push_back(make_double2(P[u * 17].real(), P[u * 17].imag()));
            for (int i = 0; i < 4; ++i)
              for (int j = 0; j < 4; ++j) mats.push_back(make_double2(P[5 * i * 16 + 5 * j].real(), P[5 * i * 16 + 5 * j].imag()));
          } else {
            for (int i = 0; i < 256; ++i) mats.push_back(make_double2(P[i].real(), P[i].imag()));
          }
          op.code = rb_op_code(op);
          pops.push_back(op);
          continue;
        }
        FusedOp op;
        if (encode_op(gate, ridx(lb[li][0]), nq[li] == 2 ? ridx(lb[li][1]) : 0, mats, op, true, side)) {
          op.code = rb_op_code(op);
          pops.push_back(op);
        }
      }
      int ld_perm[16], st_perm[16];
      fold_permutations(
          pops, rbits, [](const FusedOp& o) { return o.kind == 3 || o.kind == 5; },
          [](const FusedOp& o) {
            if (o.kind == 7 || o.kind == 8) return 15u;
            return (o.kind == 0 || o.kind == 1 || o.kind == 6) ? (1u << o.lo) : ((1u << o.o0) | (1u << o.o1));
          },
          [](const FusedOp& o, int j) { return o.kind == 3 ? reg_cx(o.o0, o.o1, j) : reg_swap(o.o0, o.o1, j); },
          ld_perm, st_perm);
      ops.insert(ops.end(), pops.begin(), pops.end());
      fp.op_count = (int)ops.size() - fp.op_begin;
      fill_phase_offsets(fp, rbits, ld_perm, st_perm);
      phases.push_back(fp);
    }
    d.op_count = (int)phases.size() - d.op_begin;
    fill_entry_offsets(d, rbits);
    set_direct_io(d, phases[d.op_begin], phases.back(), rbits);
    launches.push_back({d, true, rbits});
  }
  const size_t ph_bytes = phases.size() * sizeof(FusedPhase);
  const size_t ops_off = (ph_bytes + 255) & ~size_t(255);
  const size_t ops_bytes = ops.size() * sizeof(FusedOp);
  const size_t mats_off = (ops_off + ops_bytes + 255) & ~size_t(255);
  const size_t total = mats_off + mats.size() * sizeof(double2) + 16;
  std::vector<char> prog(total, 0);
  if (!phases.empty()) std::memcpy(prog.data(), phases.data(), ph_bytes);
  if (!ops.empty()) std::memcpy(prog.data() + ops_off, ops.data(), ops_bytes);
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
  const FusedPhase* dph = static_cast<const FusedPhase*>(dev);
  const FusedOp* dops = reinterpret_cast<const FusedOp*>(static_cast<char*>(dev) + ops_off);
  const double2* dmats = reinterpret_cast<const double2*>(static_cast<char*>(dev) + mats_off);
  // From |0...0>, amplitudes can be nonzero only where every bit outside the
  // qubits touched so far (`support`) is zero; a block maps each tile to
  // itself and zero tiles to zero, so it runs only the tiles whose index is
  // zero on its non-tile qubits outside the support (the first block: tile 0).
  unsigned long long support = 0;
  for (size_t li = 0; li < launches.size(); ++li) {
    const Launch& L = launches[li];
    unsigned long long tile_mask = ~0ull, tiles_of = 0;
    for (int q = 0; q < L.d.c; ++q) tiles_of |= 1ull << q;
    for (int i = 0; i < L.d.m; ++i) tiles_of |= 1ull << L.d.hi[i];
    if (from_zero) {
      tile_mask = 0;
      int j = 0;   // tile index bit j = the j-th qubit (ascending) outside the tile
      for (int q = 0; q < h->nbits; ++q) {
        if ((tiles_of >> q) & 1ull) continue;
        if ((support >> q) & 1ull) tile_mask |= 1ull << j;
        ++j;
      }
      support |= tiles_of;
    }
    timing_begin(h, KC_FUSED);
    if (L.rb) launch_fused_rb(h->stream, h->data, h->nbits, L.d, dph, dops, dmats, L.rbits, 1, 0, 0, h->fuse_flags,
                              0, tile_mask);
    else launch_fused_block(h->stream, h->data, h->nbits, L.d, dops, dmats, h->fuse_k);
    timing_end(h);
    const int rc = check_hip(hipGetLastError(), "fused_block");
    if (rc) return rc;
  }
  h->last_blocks = (int)launches.size();
  h->last_fused_gates = 0;
  for (const PGate& g : gates_in) h->last_fused_gates += g.type != NWQ_GATE_I;
  h->last_phases = (int)phases.size();
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

static int apply_circuit_common(nwq_handle h, int n_gates, const int* types, const int* qubits, const double* params,
                                bool from_zero) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  std::vector<PGate> gates;
  // validate everything before launching anything
  int rc0 = parse_circuit(h->n, n_gates, types, qubits, params, true, gates);
  if (rc0) return rc0;
  if (from_zero) {
    rc0 = nwq_reset(h);
    if (rc0) return rc0;
  }
  h->last_blocks = 0;
  h->last_fused_gates = 0;
  h->last_phases = 0;
  if (h->kind == NWQ_KIND_SV && h->fuse_k > 0 && n_gates > 0) return apply_fused(h, gates, h->n, nullptr, from_zero);
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

int nwq_apply_circuit(nwq_handle h, int n_gates, const int* types, const int* qubits, const double* params) {
  return apply_circuit_common(h, n_gates, types, qubits, params, false);
}

int nwq_run_circuit(nwq_handle h, int n_gates, const int* types, const int* qubits, const double* params) {
  return apply_circuit_common(h, n_gates, types, qubits, params, true);
}

int nwq_set_fusion_kernel(nwq_handle h, int kernel) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  if (kernel < 0 || kernel > 2) return set_error(NWQ_EINVAL, "fusion kernel must be 0, 1 or 2");
  if (h->kind == NWQ_KIND_DM && kernel != h->fuse_rb) {   // queued work runs on the kernel it was queued for
    const int rc = flush_all(h);
    if (rc) return rc;
  }
  h->fuse_rb = kernel;
  return NWQ_OK;
}

int nwq_set_fusion_flags(nwq_handle h, int flags) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  if (flags < 0 || flags > 7) return set_error(NWQ_EINVAL, "fusion flags must be in [0, 7]");
  h->fuse_flags = flags;
  return NWQ_OK;
}

int nwq_set_fusion_lowbits(nwq_handle h, int c) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  if (c != 0 && (c < 3 || c > 8)) return set_error(NWQ_EINVAL, "low tile bits must be 0 or in [3, 8]");
  if (h->kind == NWQ_KIND_DM && c != h->fuse_c) {   // queued superoperators run under the old tiles first
    const int rc = flush_all(h);
    if (rc) return rc;
  }
  h->fuse_c = c;
  return NWQ_OK;
}

int nwq_set_fusion(nwq_handle h, int k, int* k_out) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  if (k != 0 && (k < 6 || k > 13)) return set_error(NWQ_EINVAL, "fusion width must be 0 or in [6, 13]");
  if (h->kind == NWQ_KIND_DM) {   // queued superoperators are flushed under the old width first
    const int rc = flush_all(h);
    if (rc) return rc;
  }
  h->fuse_k = k;
  if (k_out) *k_out = k;
  return NWQ_OK;
}

int nwq_autotune_fusion(nwq_handle h, int n_gates, const int* types, const int* qubits, const double* params,
                        int reps, int* best_k, int* best_rb, double* ms_out) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  if (h->kind != NWQ_KIND_SV) return set_error(NWQ_EKIND, "fusion applies to state-vector handles");
  if (reps < 1 || reps > 100) return set_error(NWQ_EINVAL, "reps must be in [1, 100]");
  if (!best_k || !best_rb) return set_error(NWQ_EINVAL, "NULL output pointer");
  std::vector<PGate> gates;
  int rc = parse_circuit(h->n, n_gates, types, qubits, params, true, gates);
  if (rc) return rc;
  if (ms_out)
    for (int i = 0; i < NWQ_FUSION_CANDIDATES; ++i) ms_out[i] = -1.0;
  struct Cand { int k, rb; };
  std::vector<Cand> cands = {{0, 0}};
  for (int k = 6; k <= std::min(13, h->n); ++k) {
    cands.push_back({k, 0});
    if (h->n >= 8) {
      cands.push_back({k, 1});
      cands.push_back({k, 2});
    }
  }
  const int saved_k = h->fuse_k;
  const int saved_rb = h->fuse_rb;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rc = check_hip(hipEventCreate(&e0), "hipEventCreate");
  if (!rc) rc = check_hip(hipEventCreate(&e1), "hipEventCreate");
  double best = 1e300;
  Cand pick{saved_k, saved_rb};
  for (const Cand& c : cands) {
    if (rc) break;
    h->fuse_k = c.k;
    h->fuse_rb = c.rb;
    double total = 0.0;
    for (int r = 0; r <= reps && !rc; ++r) {   // r == 0 is the untimed run
      rc = check_hip(hipEventRecord(e0, h->stream), "hipEventRecord");
      if (!rc) rc = apply_circuit_common(h, n_gates, types, qubits, params, true);   // from |0...0>
      if (!rc) rc = flush_all(h);
      if (!rc) rc = check_hip(hipEventRecord(e1, h->stream), "hipEventRecord");
      if (!rc) rc = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      if (r > 0) total += ms;
    }
    if (rc) break;
    const double per = total / reps;
    if (ms_out) ms_out[c.k == 0 ? 0 : 1 + 3 * (c.k - 6) + c.rb] = per;
    if (per < best) {
      best = per;
      pick = c;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc) {
    h->fuse_k = saved_k;
    h->fuse_rb = saved_rb;
    return rc;
  }
  h->fuse_k = pick.k;
  h->fuse_rb = pick.rb;
  *best_k = pick.k;
  *best_rb = pick.rb;
  return nwq_reset(h);
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

int nwq_fusion_phases(nwq_handle h, int* phases) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  if (phases) *phases = h->last_phases;
  return NWQ_OK;
}

}  // extern "C"

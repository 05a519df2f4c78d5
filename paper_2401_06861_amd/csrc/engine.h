// The handle behind nwq_handle and the engine-internal entry points shared
// between engine.hip (state, gates, channels, reductions) and circuit.hip
// (whole-circuit application and the fusion planner).
#pragma once

#include <array>
#include <utility>
#include <vector>

#include "nwq_internal.h"

struct TimedLaunch {
  int cls;
  hipEvent_t a, b;
};

struct nwq_state {
  int kind = NWQ_KIND_SV;
  int n = 0;                       // qubits
  int nbits = 0;                   // bits of the vector index: n (SV) or 2n (DM)
  unsigned long long len = 0;      // 2^nbits entries
  double2* data = nullptr;
  bool owns = false;
  hipStream_t stream = nullptr;

  // launch shapes per kernel class and target bucket (autotuned)
  nwq::LaunchCfg cfg[nwq::KC_COUNT][nwq::kBuckets];
  // per-target shapes chosen by the autotuner; a target without one uses its bucket's
  nwq::LaunchCfg tcfg[nwq::KC_COUNT][nwq::kMaxTargetBits];
  bool tset[nwq::KC_COUNT][nwq::kMaxTargetBits] = {};
  const nwq::LaunchCfg& shape(int cls, int lowest_bit) const {
    if (lowest_bit >= 0 && lowest_bit < nwq::kMaxTargetBits && tset[cls][lowest_bit]) return tcfg[cls][lowest_bit];
    return cfg[cls][nwq::bucket_of(lowest_bit)];
  }

  // reduction scratch
  double* partials = nullptr;
  size_t partials_cap = 0;
  double* results_dev = nullptr;
  double* results_host = nullptr;  // pinned
  size_t results_cap = 0;

  // upload arena (pinned host ring + device ring)
  void* arena_dev = nullptr;
  void* arena_host = nullptr;
  size_t arena_off = 0;

  // DM: pending superoperator (gate + following channels on the same qubits)
  bool pend_active = false;
  int pend_k = 0;
  int pend_q[2] = {-1, -1};
  std::vector<nwq::cd> pend_S;

  // SV fusion
  int fuse_k = 0;                  // 0 = off
  int last_blocks = 0, last_fused_gates = 0, last_phases = 0;
  int fuse_rb = 1;                 // fused kernel: 0 one LDS pass per gate, 1 / 2 register-blocked with 4 / 3 register bits
  int fuse_c = 0;                  // low tile bits of a fused block: 0 = the kind's default (fusion_low_bits)
  int fuse_flags = 7;              // register-blocked kernels: bit 0 non-temporal tile loads and stores, bit 1
                                   // first / last phase straight between HBM and registers, bit 2 gate
                                   // products inside a phase (SV circuits)
  void* fuse_dev = nullptr;        // device copy of the compiled block program
  // DM with fusion on: superoperators (1q: 4x4 on bits q, q + n; 2q with the
  // 4-register-bit kernel: 16x16 on bits q0, q1, q0 + n, q1 + n) wait here and
  // run as fused blocks when a read needs the state (a 2q superoperator too
  // when it cannot be queued)
  std::vector<std::array<int, 3>> dmq_ops;   // queued superoperators: (k, q0, q1)
  std::vector<nwq::cd> dmq_S;                // their matrices back to back (16 or 256 entries)
  size_t fuse_cap = 0;

  // timing
  bool timing = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> event_pool;
  long long t_count[nwq::KC_COUNT] = {0};
  double t_ms[nwq::KC_COUNT] = {0};
};

namespace nwq {
// A gate of a circuit (type nwq_gate, qubits, up to 3 parameters).
struct PGate {
  int type;
  int q[4];   // nq qubits (4 only for the queued DM two-qubit superoperators)
  int nq;
  double p[3];
};
// A fused block: tile qubits {0..c-1} u hi[0..m), and its gates in order.
struct Block {
  int c = 0, m = 0;
  int hi[8] = {0};
  std::vector<int> gates;
};
// A register phase of a block: 4 tile-local register bits and its gates.
struct Phase {
  int reg[4];
  std::vector<int> gates;
};
// c: the low bits every block's tile holds (c <= k - 2, k - c <= 8); -1 =
// min(6, k - 2).  Ignored when the n bits fit one tile.
std::vector<Block> plan_blocks(const std::vector<PGate>& g, int n, int k, int c = -1);
// Low tile bits for a handle's fused blocks of width k over nbits bits.
int fusion_low_bits(const nwq_state* h, int nbits, int k);
// internal gate type: dense 4x4 whose matrix is entry p[0] of a side table
// Internal gate types whose matrix sits in a side table from entry p[0] on:
// a dense 4x4 (16 entries), a diagonal 4x4 (16 entries, the diagonal at 5u),
// a 2x2 (4 entries), and a dense 16x16 on the four bits q[0..3] (256 entries,
// operator index bit t on q[t]; DM two-qubit superoperators).
constexpr int kGateMat4 = 1000;
constexpr int kGateDiag4 = 1001;
constexpr int kGateMat2 = 1002;
constexpr int kGateMat16 = 1003;
// from_zero: the state is |0...0> (the first block then runs tile 0 only)
int apply_fused(nwq_state* h, const std::vector<PGate>& gates, int nbits, const std::vector<cd>* side,
                bool from_zero = false);
// Fold the permutation gates that can open or close a register phase into its
// LDS offsets instead of moving registers.  A permutation moves past a
// following (preceding) non-permutation gate on other register bits, since the
// two commute (for adjoint sweeps too: the gradient term of a gate is
// unchanged when both vectors are transformed by a unitary that commutes with
// its generator).  The trailing run T_1..T_m then means that register j holds
// the entry of index T_m(...T_1(j)), so it is stored there; the leading run
// L_1..L_l means that register j must hold the entry the data had at
// (L_l...L_1)^-1 (j) = L_1(...L_l(j)) (the gates are involutions), so it is
// loaded from there.  The remaining ops keep their order.  is_perm(op),
// bits(op) (register-bit mask) and apply(op, j) (index map of a permutation)
// describe the op type.
template <class Op, class IsPerm, class Bits, class Apply>
void fold_permutations(std::vector<Op>& ops, int rbits, IsPerm is_perm, Bits bits, Apply apply, int* ld_perm,
                       int* st_perm) {
  const int nv = 1 << rbits;
  for (int j = 0; j < 16; ++j) ld_perm[j] = st_perm[j] = j;
  bool moved = true;
  while (moved) {   // permutations towards the end
    moved = false;
    for (size_t i = 0; i + 1 < ops.size(); ++i)
      if (is_perm(ops[i]) && !is_perm(ops[i + 1]) && !(bits(ops[i]) & bits(ops[i + 1]))) {
        std::swap(ops[i], ops[i + 1]);
        moved = true;
      }
  }
  size_t end = ops.size();
  while (end > 0 && is_perm(ops[end - 1])) --end;
  for (int j = 0; j < nv; ++j)
    for (size_t i = end; i < ops.size(); ++i) st_perm[j] = apply(ops[i], st_perm[j]);
  ops.resize(end);
  moved = true;
  while (moved) {   // the rest towards the start
    moved = false;
    for (size_t i = ops.size(); i-- > 1;)
      if (is_perm(ops[i]) && !is_perm(ops[i - 1]) && !(bits(ops[i]) & bits(ops[i - 1]))) {
        std::swap(ops[i], ops[i - 1]);
        moved = true;
      }
  }
  size_t lead = 0;
  while (lead < ops.size() && is_perm(ops[lead])) ++lead;
  for (int j = 0; j < nv; ++j)
    for (size_t i = lead; i-- > 0;) ld_perm[j] = apply(ops[i], ld_perm[j]);
  ops.erase(ops.begin(), ops.begin() + (long)lead);
}
// Index map of CX (control c, target t: flips t where c is set) and SWAP on register indices.
inline int reg_cx(int c, int t, int j) { return j ^ (((j >> c) & 1) << t); }
inline int reg_swap(int a, int b, int j) {
  return ((j >> a) & 1) == ((j >> b) & 1) ? j : j ^ ((1 << a) | (1 << b));
}
int local_bit(const Block& b, int q);
void pad_block(Block& b, int n, int k_target);
void fill_entry_offsets(FusedBlockDev& d, int rbits);
// Marks the block's first / last phase for direct HBM loads / stores when its
// register bits all lie above the low c tile bits (FusedBlockDev::direct).
void set_direct_io(FusedBlockDev& d, const FusedPhase& first, const FusedPhase& last, int rbits);
// c: the block's low tile bits; a phase with fewer gate bits than rbits is
// padded with tile bits from c up first.
std::vector<Phase> plan_phases(const std::vector<int>& order, const std::vector<std::array<int, 4>>& lb,
                               const std::vector<int>& nq, int k, int c, int rbits);

void gate_matrix(int type, const double* p, cd* m);
int arena_put(nwq_state* h, const void* src, size_t bytes, void** dev_out);
void timing_begin(nwq_state* h, int cls);
void timing_end(nwq_state* h);
int sv_apply_gate_validated(nwq_state* h, int type, const int* q, const double* p);
int dm_apply_unitary(nwq_state* h, const int* q, int k, const cd* U);
int flush_all(nwq_state* h);
}  // namespace nwq

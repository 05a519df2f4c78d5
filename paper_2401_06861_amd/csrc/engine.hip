// Host side of the engine: handles, validation, host-built gate matrices and
// superoperators, dispatch to the gfx950 kernels, deferred fusion of a DM
// gate with the channels that follow it, reductions and per-kernel timing.
//
// The state-vector simulator (Sec. II) applies psi <- U psi gate by gate or
// in fused blocks; the density-matrix simulator (Sec. II) applies
// rho <- sum_k K_k rho K_k^dag, here as one superoperator S = sum_k K_k (x)
// conj(K_k) acting on the row-major vec of rho, with a gate and the noise
// channels of Sec. III that follow it composed into one S before launch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <set>

#include "nwq_internal.h"
#include "engine.h"

namespace nwq {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return NWQ_OK;
  if (e == hipErrorOutOfMemory) return set_error(NWQ_ENOMEM, std::string(what) + ": out of device memory");
  return set_error(NWQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int enable_dynamic_lds(const void* kernel) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({kernel, dev})) return NWQ_OK;
  hipFuncAttributes attr{};
  rc = check_hip(hipFuncGetAttributes(&attr, kernel), "hipFuncGetAttributes");
  if (rc) return rc;
  // the static LDS a kernel declares comes out of the same 160 KiB
  rc = check_hip(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     kMaxDynamicLds - (int)attr.sharedSizeBytes),
                 "hipFuncSetAttribute");
  if (rc) return rc;
  done.insert({kernel, dev});
  return NWQ_OK;
}

#define NWQ_TRY_HIP(expr, what)                   \
  do {                                            \
    const int rc__ = check_hip((expr), (what));   \
    if (rc__ != NWQ_OK) return rc__;              \
  } while (0)

// ---------------------------------------------------------------------------
// Host gate matrices (FP64, std math): row-major, index u = sum_j bit(q_j) 2^j
// ---------------------------------------------------------------------------
static int gate_arity(int type, int* nq, int* np) {
  switch (type) {
    case NWQ_GATE_I: case NWQ_GATE_X: case NWQ_GATE_Y: case NWQ_GATE_Z: case NWQ_GATE_H:
    case NWQ_GATE_S: case NWQ_GATE_SDG: case NWQ_GATE_T: case NWQ_GATE_TDG:
      *nq = 1; *np = 0; return 0;
    case NWQ_GATE_RX: case NWQ_GATE_RY: case NWQ_GATE_RZ:
      *nq = 1; *np = 1; return 0;
    case NWQ_GATE_U3:
      *nq = 1; *np = 3; return 0;
    case NWQ_GATE_CX: case NWQ_GATE_CZ: case NWQ_GATE_SWAP:
      *nq = 2; *np = 0; return 0;
    case NWQ_GATE_RZZ:
      *nq = 2; *np = 1; return 0;
    default:
      return -1;
  }
}

void gate_matrix(int type, const double* p, cd* m) {
  const cd I(0.0, 1.0);
  auto set2 = [&](cd a, cd b, cd c, cd d) { m[0] = a; m[1] = b; m[2] = c; m[3] = d; };
  switch (type) {
    case NWQ_GATE_I: set2(1.0, 0.0, 0.0, 1.0); break;
    case NWQ_GATE_X: set2(0.0, 1.0, 1.0, 0.0); break;
    case NWQ_GATE_Y: set2(0.0, -I, I, 0.0); break;
    case NWQ_GATE_Z: set2(1.0, 0.0, 0.0, -1.0); break;
    case NWQ_GATE_H: { const double r = 1.0 / std::sqrt(2.0); set2(r, r, r, -r); break; }
    case NWQ_GATE_S: set2(1.0, 0.0, 0.0, I); break;
    case NWQ_GATE_SDG: set2(1.0, 0.0, 0.0, -I); break;
    case NWQ_GATE_T: set2(1.0, 0.0, 0.0, std::polar(1.0, M_PI / 4)); break;
    case NWQ_GATE_TDG: set2(1.0, 0.0, 0.0, std::polar(1.0, -M_PI / 4)); break;
    case NWQ_GATE_RX: { const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2); set2(c, -I * s, -I * s, c); break; }
    case NWQ_GATE_RY: { const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2); set2(c, -s, s, c); break; }
    case NWQ_GATE_RZ: set2(std::polar(1.0, -p[0] / 2), 0.0, 0.0, std::polar(1.0, p[0] / 2)); break;
    case NWQ_GATE_U3: {
      const double c = std::cos(p[0] / 2), s = std::sin(p[0] / 2);
      set2(c, -std::polar(s, p[2]), std::polar(s, p[1]), std::polar(c, p[1] + p[2]));
      break;
    }
    default: {
      for (int i = 0; i < 16; ++i) m[i] = 0.0;
      if (type == NWQ_GATE_CX) {            // control q0 (bit 0 of u), target q1
        m[0 * 4 + 0] = 1.0; m[2 * 4 + 2] = 1.0; m[1 * 4 + 3] = 1.0; m[3 * 4 + 1] = 1.0;
      } else if (type == NWQ_GATE_CZ) {
        m[0] = 1.0; m[5] = 1.0; m[10] = 1.0; m[15] = -1.0;
      } else if (type == NWQ_GATE_SWAP) {
        m[0] = 1.0; m[1 * 4 + 2] = 1.0; m[2 * 4 + 1] = 1.0; m[15] = 1.0;
      } else if (type == NWQ_GATE_RZZ) {
        const cd e = std::polar(1.0, -p[0] / 2), f = std::polar(1.0, p[0] / 2);
        m[0] = e; m[5] = f; m[10] = f; m[15] = e;
      }
    }
  }
}

static double2 d2(cd z) { return make_double2(z.real(), z.imag()); }

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
static int check_qubits(const nwq_state* h, const int* qubits, int k) {
  if (k > 0 && qubits == nullptr) return set_error(NWQ_EINVAL, "qubits pointer is NULL");
  for (int i = 0; i < k; ++i) {
    if (qubits[i] < 0 || qubits[i] >= h->n)
      return set_error(NWQ_ERANGE, "qubit " + std::to_string(qubits[i]) + " out of range for n=" + std::to_string(h->n));
    for (int j = 0; j < i; ++j)
      if (qubits[j] == qubits[i]) return set_error(NWQ_EDUP, "qubit " + std::to_string(qubits[i]) + " repeated");
  }
  return NWQ_OK;
}

static int check_handle(const nwq_state* h) {
  if (h == nullptr) return set_error(NWQ_EINVAL, "NULL handle");
  return NWQ_OK;
}

// ---------------------------------------------------------------------------
// Arena: small stream-ordered uploads (matrices, term tables) through a
// pinned host ring and a device ring of the same size.  On wrap the stream
// is synchronised so no pending copy still reads a slot being reused.
// ---------------------------------------------------------------------------
static constexpr size_t kArenaBytes = 4u << 20;

int arena_put(nwq_state* h, const void* src, size_t bytes, void** dev_out) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes > kArenaBytes) return set_error(NWQ_EINVAL, "upload larger than the arena");
  if (h->arena_dev == nullptr) {
    NWQ_TRY_HIP(hipMalloc(&h->arena_dev, kArenaBytes), "hipMalloc(arena)");
    NWQ_TRY_HIP(hipHostMalloc(&h->arena_host, kArenaBytes, hipHostMallocDefault), "hipHostMalloc(arena)");
    h->arena_off = 0;
  }
  if (h->arena_off + bytes > kArenaBytes) {
    NWQ_TRY_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize(arena wrap)");
    h->arena_off = 0;
  }
  char* hp = static_cast<char*>(h->arena_host) + h->arena_off;
  char* dp = static_cast<char*>(h->arena_dev) + h->arena_off;
  std::memcpy(hp, src, bytes);
  NWQ_TRY_HIP(hipMemcpyAsync(dp, hp, bytes, hipMemcpyHostToDevice, h->stream), "hipMemcpyAsync(arena)");
  h->arena_off += bytes;
  *dev_out = dp;
  return NWQ_OK;
}

int ensure_partials(nwq_state* h, size_t doubles) {
  if (doubles <= h->partials_cap) return NWQ_OK;
  if (h->partials) {
    NWQ_TRY_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    NWQ_TRY_HIP(hipFree(h->partials), "hipFree(partials)");
    h->partials = nullptr;
  }
  size_t cap = std::max<size_t>(doubles, 1u << 16);
  NWQ_TRY_HIP(hipMalloc(&h->partials, cap * sizeof(double)), "hipMalloc(partials)");
  h->partials_cap = cap;
  return NWQ_OK;
}

int ensure_results(nwq_state* h, size_t doubles) {
  if (doubles <= h->results_cap) return NWQ_OK;
  if (h->results_dev) {
    NWQ_TRY_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    NWQ_TRY_HIP(hipFree(h->results_dev), "hipFree(results)");
    NWQ_TRY_HIP(hipHostFree(h->results_host), "hipHostFree(results)");
    h->results_dev = nullptr;
    h->results_host = nullptr;
  }
  size_t cap = std::max<size_t>(doubles, 1024);
  NWQ_TRY_HIP(hipMalloc(&h->results_dev, cap * sizeof(double)), "hipMalloc(results)");
  NWQ_TRY_HIP(hipHostMalloc(&h->results_host, cap * sizeof(double), hipHostMallocDefault), "hipHostMalloc(results)");
  h->results_cap = cap;
  return NWQ_OK;
}

// ---------------------------------------------------------------------------
// Timing
// ---------------------------------------------------------------------------
void timing_begin(nwq_state* h, int cls) {
  if (!h->timing) return;
  TimedLaunch t;
  t.cls = cls;
  if (!h->event_pool.empty()) {
    t.a = h->event_pool.back(); h->event_pool.pop_back();
  } else {
    (void)hipEventCreate(&t.a);
  }
  if (!h->event_pool.empty()) {
    t.b = h->event_pool.back(); h->event_pool.pop_back();
  } else {
    (void)hipEventCreate(&t.b);
  }
  (void)hipEventRecord(t.a, h->stream);
  h->timed.push_back(t);
}

void timing_end(nwq_state* h) {
  if (!h->timing || h->timed.empty()) return;
  (void)hipEventRecord(h->timed.back().b, h->stream);
}

static int drain_timing(nwq_state* h) {
  if (h->timed.empty()) return NWQ_OK;
  NWQ_TRY_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize(timing)");
  for (auto& t : h->timed) {
    float ms = 0.f;
    NWQ_TRY_HIP(hipEventElapsedTime(&ms, t.a, t.b), "hipEventElapsedTime");
    h->t_count[t.cls] += 1;
    h->t_ms[t.cls] += ms;
    h->event_pool.push_back(t.a);
    h->event_pool.push_back(t.b);
  }
  h->timed.clear();
  return NWQ_OK;
}

// ---------------------------------------------------------------------------
// SV dispatch of one validated gate
// ---------------------------------------------------------------------------
static int last_launch(const char* what) { return check_hip(hipGetLastError(), what); }

int sv_apply_gate_validated(nwq_state* h, int type, const int* q, const double* p) {
  cd m[16];
  gate_matrix(type, p, m);
  const int nb = h->nbits;
  switch (type) {
    case NWQ_GATE_I:
      return NWQ_OK;
    case NWQ_GATE_X:
      timing_begin(h, KC_PERM);
      launch_sv_swap1(h->stream, h->data, nb, q[0], h->shape(KC_PERM, q[0]));
      timing_end(h);
      return last_launch("sv_swap1");
    case NWQ_GATE_Z: case NWQ_GATE_S: case NWQ_GATE_SDG: case NWQ_GATE_T: case NWQ_GATE_TDG:
    case NWQ_GATE_RZ: {
      Diag4 d{};
      d.d[0] = d2(m[0]); d.d[1] = d2(m[3]); d.d[2] = d.d[0]; d.d[3] = d.d[1];
      timing_begin(h, KC_DIAG);
      launch_sv_diag(h->stream, h->data, nb, q[0], -1, d, h->shape(KC_DIAG, q[0]));
      timing_end(h);
      return last_launch("sv_diag");
    }
    case NWQ_GATE_Y: case NWQ_GATE_H: case NWQ_GATE_RX: case NWQ_GATE_RY: case NWQ_GATE_U3: {
      Mat2 M;
      for (int i = 0; i < 4; ++i) M.m[i] = d2(m[i]);
      timing_begin(h, KC_SV1Q);
      launch_sv_1q(h->stream, h->data, nb, q[0], M, h->shape(KC_SV1Q, q[0]));
      timing_end(h);
      return last_launch("sv_1q");
    }
    case NWQ_GATE_CX:
      timing_begin(h, KC_PERM);
      launch_sv_swap2(h->stream, h->data, nb, q[0], q[1], 1ull << q[0], (1ull << q[0]) + (1ull << q[1]),
                      h->shape(KC_PERM, std::min(q[0], q[1])));
      timing_end(h);
      return last_launch("sv_swap2(cx)");
    case NWQ_GATE_SWAP:
      timing_begin(h, KC_PERM);
      launch_sv_swap2(h->stream, h->data, nb, q[0], q[1], 1ull << q[0], 1ull << q[1],
                      h->shape(KC_PERM, std::min(q[0], q[1])));
      timing_end(h);
      return last_launch("sv_swap2(swap)");
    case NWQ_GATE_CZ: case NWQ_GATE_RZZ: {
      Diag4 d{};
      for (int u = 0; u < 4; ++u) d.d[u] = d2(m[5 * u]);
      timing_begin(h, KC_DIAG);
      launch_sv_diag(h->stream, h->data, nb, q[0], q[1], d, h->shape(KC_DIAG, std::min(q[0], q[1])));
      timing_end(h);
      return last_launch("sv_diag2");
    }
    default:
      return set_error(NWQ_EINVAL, "unknown gate type");
  }
}

int sv_apply_matrix_validated(nwq_state* h, const int* q, int k, const cd* m) {
  if (k == 1) {
    Mat2 M;
    for (int i = 0; i < 4; ++i) M.m[i] = d2(m[i]);
    timing_begin(h, KC_SV1Q);
    launch_sv_1q(h->stream, h->data, h->nbits, q[0], M, h->shape(KC_SV1Q, q[0]));
    timing_end(h);
    return last_launch("sv_1q");
  }
  Mat4 M;
  for (int i = 0; i < 16; ++i) M.m[i] = d2(m[i]);
  timing_begin(h, KC_SV2Q);
  launch_sv_2q(h->stream, h->data, h->nbits, q[0], q[1], M, h->shape(KC_SV2Q, std::min(q[0], q[1])));
  timing_end(h);
  return last_launch("sv_2q");
}

// ---------------------------------------------------------------------------
// DM: superoperators on the row-major vec, composed lazily
// ---------------------------------------------------------------------------
// S = sum_k K_k (x) conj(K_k), index (r, c) -> r * 2^k + c
static void superop(const cd* kraus, int nk, int k, std::vector<cd>& S) {
  const int d = 1 << k, D = d * d;
  S.assign((size_t)D * D, cd(0.0));
  for (int t = 0; t < nk; ++t) {
    const cd* K = kraus + (size_t)t * d * d;
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c)
        for (int rp = 0; rp < d; ++rp)
          for (int cp = 0; cp < d; ++cp)
            S[(size_t)(r * d + c) * D + (rp * d + cp)] += K[r * d + rp] * std::conj(K[c * d + cp]);
  }
}

static constexpr size_t kDmQueueEntries = (1u << 20) / sizeof(cd);

// One pass of a 2q superoperator S (16x16, u = c0 + 2 c1 + 4 r0 + 8 r1) on
// qubits (q0, q1).
// A two-qubit superoperator (u = c0 + 2 c1 + 4 r0 + 8 r1) has the Pauli
// pattern when it only scales the coherences (the entries whose row and
// column bits differ on either qubit) and mixes the four populations u = 0,
// 5, 10, 15 among themselves: a Pauli channel after a diagonal gate (RZZ, CZ
// and depolarising noise, Sec. III noise model).  Then the pass needs 7 FP64
// operations per entry instead of 64.  The compact form: the 16 diagonal
// entries, then the 4 x 4 among the populations.
static bool superop2_pauli(const cd* S, std::vector<double2>& compact) {
  for (int r = 0; r < 16; ++r)
    for (int c = 0; c < 16; ++c)
      if (r != c && !(r % 5 == 0 && c % 5 == 0) && S[r * 16 + c] != 0.0) return false;
  compact.resize(32);
  for (int u = 0; u < 16; ++u) compact[u] = d2(S[u * 16 + u]);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) compact[16 + 4 * i + j] = d2(S[(5 * i) * 16 + 5 * j]);
  return true;
}

static int dm_superop2_pass(nwq_state* h, int q0, int q1, const cd* S) {
  std::vector<double2> buf;
  const bool pauli = superop2_pauli(S, buf);
  if (!pauli) {
    buf.resize(256);
    for (int i = 0; i < 256; ++i) buf[i] = d2(S[i]);
  }
  void* dev = nullptr;
  const int rc = arena_put(h, buf.data(), buf.size() * sizeof(double2), &dev);
  if (rc != NWQ_OK) return rc;
  const int vq[4] = {q0, q1, q0 + h->n, q1 + h->n};
  timing_begin(h, KC_DM2);
  launch_sv_kq(h->stream, h->data, h->nbits, 4, vq, static_cast<const double2*>(dev), h->shape(KC_DM2, std::min(q0, q1)),
               pauli);
  timing_end(h);
  return last_launch("dm_superop_2q");
}

// Runs the queued superoperators: through fused blocks over the 2n bits of
// vec(rho) when there are two or more, else as one pass.
static int dm_run_queue(nwq_state* h) {
  const size_t cnt = h->dmq_ops.size();
  if (cnt == 0) return NWQ_OK;
  int rc = NWQ_OK;
  if (cnt == 1 && h->dmq_ops[0][0] == 1) {
    Mat4 M;
    for (int i = 0; i < 16; ++i) M.m[i] = d2(h->dmq_S[i]);
    const int q = h->dmq_ops[0][1];
    timing_begin(h, KC_DM1);
    launch_sv_2q(h->stream, h->data, h->nbits, q, q + h->n, M, h->shape(KC_DM1, q));
    timing_end(h);
    rc = last_launch("dm_superop_1q");
  } else if (cnt == 1) {
    rc = dm_superop2_pass(h, h->dmq_ops[0][1], h->dmq_ops[0][2], h->dmq_S.data());
  } else {
    std::vector<PGate> gates(cnt);
    size_t off = 0;
    for (size_t i = 0; i < cnt; ++i) {
      PGate& g = gates[i];
      const int k = h->dmq_ops[i][0], q0 = h->dmq_ops[i][1], q1 = h->dmq_ops[i][2];
      g.p[0] = (double)off;
      g.p[1] = g.p[2] = 0.0;
      if (k == 1) {
        g.type = kGateMat4;
        g.nq = 2;
        g.q[0] = q0;              // column bit: u bit 0
        g.q[1] = q0 + h->n;       // row bit: u bit 1
        off += 16;
      } else {
        g.type = kGateMat16;      // u = c0 + 2 c1 + 4 r0 + 8 r1
        g.nq = 4;
        g.q[0] = q0;
        g.q[1] = q1;
        g.q[2] = q0 + h->n;
        g.q[3] = q1 + h->n;
        off += 256;
      }
    }
    rc = apply_fused(h, gates, h->nbits, &h->dmq_S);
  }
  h->dmq_ops.clear();
  h->dmq_S.clear();
  return rc;
}

int dm_flush(nwq_state* h) {
  if (!h->pend_active) return NWQ_OK;
  const int k = h->pend_k, n = h->n;
  // queue it for the next fused run: 1q always, 2q when the blocks run on the
  // 4-register-bit kernel (a 16x16 takes all four register bits of a phase)
  // and a block can hold its four bits (the whole state fits one tile, or the
  // width leaves four bits above the low tile bits)
  const bool fits4 = h->nbits <= h->fuse_k || h->fuse_k - fusion_low_bits(h, h->nbits, h->fuse_k) >= 4;
  if (h->fuse_k > 0 && (k == 1 || (h->fuse_rb == 1 && h->nbits >= 8 && fits4))) {
    h->dmq_ops.push_back({k, h->pend_q[0], k == 2 ? h->pend_q[1] : -1});
    h->dmq_S.insert(h->dmq_S.end(), h->pend_S.begin(), h->pend_S.end());
    h->pend_active = false;
    // a long circuit with no read in between runs in pieces of at most 1 MiB
    // of matrices (host memory stays bounded, the block program small)
    if (h->dmq_S.size() >= kDmQueueEntries) return dm_run_queue(h);
    return NWQ_OK;
  }
  int rc = dm_run_queue(h);   // queued work comes first
  if (rc) return rc;
  if (k == 1) {
    Mat4 M;
    for (int i = 0; i < 16; ++i) M.m[i] = d2(h->pend_S[i]);
    timing_begin(h, KC_DM1);
    // vec bits (column q, row q + n): u = c + 2 r
    launch_sv_2q(h->stream, h->data, h->nbits, h->pend_q[0], h->pend_q[0] + n, M, h->shape(KC_DM1, h->pend_q[0]));
    timing_end(h);
    h->pend_active = false;
    return last_launch("dm_superop_1q");
  }
  h->pend_active = false;
  return dm_superop2_pass(h, h->pend_q[0], h->pend_q[1], h->pend_S.data());
}

// Compose S_new after the pending superoperator (or start a new one).
int dm_push(nwq_state* h, const int* q, int k, const std::vector<cd>& S) {
  const bool same = h->pend_active && h->pend_k == k && h->pend_q[0] == q[0] && (k == 1 || h->pend_q[1] == q[1]);
  if (!same) {
    const int rc = dm_flush(h);
    if (rc != NWQ_OK) return rc;
    h->pend_active = true;
    h->pend_k = k;
    h->pend_q[0] = q[0];
    h->pend_q[1] = k == 2 ? q[1] : -1;
    h->pend_S = S;
    return NWQ_OK;
  }
  const int D = 1 << (2 * k);
  std::vector<cd> out((size_t)D * D, cd(0.0));
  for (int i = 0; i < D; ++i)
    for (int l = 0; l < D; ++l) {
      const cd a = S[(size_t)i * D + l];
      if (a == cd(0.0)) continue;
      for (int j = 0; j < D; ++j) out[(size_t)i * D + j] += a * h->pend_S[(size_t)l * D + j];
    }
  h->pend_S.swap(out);
  return NWQ_OK;
}

int dm_apply_unitary(nwq_state* h, const int* q, int k, const cd* U) {
  std::vector<cd> S;
  superop(U, 1, k, S);
  return dm_push(h, q, k, S);
}

int flush_all(nwq_state* h) {
  if (h->kind != NWQ_KIND_DM) return NWQ_OK;
  const int rc = dm_flush(h);
  return rc ? rc : dm_run_queue(h);
}

}  // namespace nwq

// ===========================================================================
// C ABI
// ===========================================================================
using namespace nwq;

extern "C" {

const char* nwq_last_error(void) { return g_last_error.c_str(); }

static int create_common(int kind, int n, void* dev_ptr, void* stream, nwq_handle* out) {
  if (out == nullptr) return set_error(NWQ_EINVAL, "out handle pointer is NULL");
  *out = nullptr;
  const int nmax = kind == NWQ_KIND_SV ? 34 : 17;
  if (n < 1 || n > nmax)
    return set_error(NWQ_ERANGE, "n=" + std::to_string(n) + " outside [1, " + std::to_string(nmax) + "]");
  std::unique_ptr<nwq_state> h(new nwq_state());
  for (int b = 0; b < kBuckets; ++b) h->cfg[KC_DM2][b].ppt = 1;   // one 16-entry group per thread
  h->kind = kind;
  h->n = n;
  h->nbits = kind == NWQ_KIND_SV ? n : 2 * n;
  h->len = 1ull << h->nbits;
  h->stream = static_cast<hipStream_t>(stream);
  if (dev_ptr != nullptr) {
    if ((reinterpret_cast<uintptr_t>(dev_ptr) & 15u) != 0) return set_error(NWQ_EINVAL, "device pointer not 16-byte aligned");
    h->data = static_cast<double2*>(dev_ptr);
    h->owns = false;
  } else {
    void* p = nullptr;
    NWQ_TRY_HIP(hipMalloc(&p, h->len * sizeof(double2)), "hipMalloc(state)");
    h->data = static_cast<double2*>(p);
    h->owns = true;
    timing_begin(h.get(), KC_RESET);
    launch_fill_basis0(h->stream, h->data, h->len);
    timing_end(h.get());
    const int rc = last_launch("fill_basis0");
    if (rc != NWQ_OK) {
      (void)hipFree(p);
      return rc;
    }
  }
  *out = h.release();
  return NWQ_OK;
}

int nwq_sv_create(int n, void* s, nwq_handle* out) { return create_common(NWQ_KIND_SV, n, nullptr, s, out); }
int nwq_dm_create(int n, void* s, nwq_handle* out) { return create_common(NWQ_KIND_DM, n, nullptr, s, out); }
int nwq_sv_create_from(void* p, int n, void* s, nwq_handle* out) {
  if (p == nullptr) return set_error(NWQ_EINVAL, "device pointer is NULL");
  return create_common(NWQ_KIND_SV, n, p, s, out);
}
int nwq_dm_create_from(void* p, int n, void* s, nwq_handle* out) {
  if (p == nullptr) return set_error(NWQ_EINVAL, "device pointer is NULL");
  return create_common(NWQ_KIND_DM, n, p, s, out);
}

int nwq_destroy(nwq_handle h) {
  if (h == nullptr) return NWQ_OK;
  int rc = check_hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize(destroy)");
  if (h->owns && h->data) (void)hipFree(h->data);
  if (h->partials) (void)hipFree(h->partials);
  if (h->results_dev) (void)hipFree(h->results_dev);
  if (h->results_host) (void)hipHostFree(h->results_host);
  if (h->arena_dev) (void)hipFree(h->arena_dev);
  if (h->arena_host) (void)hipHostFree(h->arena_host);
  if (h->fuse_dev) (void)hipFree(h->fuse_dev);
  for (auto& t : h->timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
  for (auto e : h->event_pool) (void)hipEventDestroy(e);
  delete h;
  return rc;
}

int nwq_info(nwq_handle h, int* kind, int* n, void** dev_ptr) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (kind) *kind = h->kind;
  if (n) *n = h->n;
  if (dev_ptr) *dev_ptr = h->data;
  return NWQ_OK;
}

int nwq_reset(nwq_handle h) {
  int rc = check_handle(h);
  if (rc) return rc;
  h->pend_active = false;   // pending work on the old state is discarded
  h->dmq_ops.clear();
  h->dmq_S.clear();
  timing_begin(h, KC_RESET);
  launch_fill_basis0(h->stream, h->data, h->len);
  timing_end(h);
  return last_launch("fill_basis0");
}

int nwq_get_state(nwq_handle h, double* host, size_t n_doubles) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (host == nullptr || n_doubles != 2 * h->len)
    return set_error(NWQ_EINVAL, "host buffer must hold " + std::to_string(2 * h->len) + " doubles");
  rc = flush_all(h);
  if (rc) return rc;
  NWQ_TRY_HIP(hipMemcpyAsync(host, h->data, h->len * sizeof(double2), hipMemcpyDeviceToHost, h->stream),
              "hipMemcpyAsync(get_state)");
  NWQ_TRY_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize(get_state)");
  return NWQ_OK;
}

int nwq_set_state(nwq_handle h, const double* host, size_t n_doubles) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (host == nullptr || n_doubles != 2 * h->len)
    return set_error(NWQ_EINVAL, "host buffer must hold " + std::to_string(2 * h->len) + " doubles");
  h->pend_active = false;
  h->dmq_ops.clear();
  h->dmq_S.clear();
  NWQ_TRY_HIP(hipMemcpyAsync(h->data, host, h->len * sizeof(double2), hipMemcpyHostToDevice, h->stream),
              "hipMemcpyAsync(set_state)");
  NWQ_TRY_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize(set_state)");
  return NWQ_OK;
}

int nwq_flush(nwq_handle h) {
  int rc = check_handle(h);
  if (rc) return rc;
  return flush_all(h);
}

static int validate_gate(nwq_state* h, int type, const int* qubits, int n_q, const double* params, int n_p) {
  int nq, np;
  if (gate_arity(type, &nq, &np) != 0) return set_error(NWQ_EINVAL, "unknown gate type " + std::to_string(type));
  if (n_q != nq)
    return set_error(NWQ_EINVAL, "gate type " + std::to_string(type) + " takes " + std::to_string(nq) + " qubits");
  if (n_p != np)
    return set_error(NWQ_EINVAL, "gate type " + std::to_string(type) + " takes " + std::to_string(np) + " parameters");
  if (np > 0 && params == nullptr) return set_error(NWQ_EINVAL, "params pointer is NULL");
  for (int i = 0; i < np; ++i)
    if (!std::isfinite(params[i])) return set_error(NWQ_EINVAL, "non-finite gate parameter");
  return check_qubits(h, qubits, n_q);
}

int nwq_apply_gate(nwq_handle h, int type, const int* qubits, int n_q, const double* params, int n_p) {
  int rc = check_handle(h);
  if (rc) return rc;
  rc = validate_gate(h, type, qubits, n_q, params, n_p);
  if (rc) return rc;
  if (h->kind == NWQ_KIND_SV) return sv_apply_gate_validated(h, type, qubits, params);
  cd m[16];
  gate_matrix(type, params, m);
  return dm_apply_unitary(h, qubits, n_q, m);
}

int nwq_apply_matrix(nwq_handle h, const int* qubits, int k, const double* m) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (k < 1 || k > 2) return set_error(NWQ_EINVAL, "apply_matrix supports k = 1 or 2");
  if (m == nullptr) return set_error(NWQ_EINVAL, "matrix pointer is NULL");
  rc = check_qubits(h, qubits, k);
  if (rc) return rc;
  const int d = 1 << k;
  std::vector<cd> M((size_t)d * d);
  for (int i = 0; i < d * d; ++i) {
    M[i] = cd(m[2 * i], m[2 * i + 1]);
    if (!std::isfinite(m[2 * i]) || !std::isfinite(m[2 * i + 1])) return set_error(NWQ_EINVAL, "non-finite matrix entry");
  }
  if (h->kind == NWQ_KIND_SV) return sv_apply_matrix_validated(h, qubits, k, M.data());
  return dm_apply_unitary(h, qubits, k, M.data());
}

int nwq_apply_channel(nwq_handle h, const int* qubits, int k, const double* kraus, int n_kraus) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->kind != NWQ_KIND_DM) return set_error(NWQ_EKIND, "channels need a density-matrix handle");
  if (k < 1 || k > 2) return set_error(NWQ_EINVAL, "channels act on k = 1 or 2 qubits");
  if (kraus == nullptr || n_kraus < 1 || n_kraus > 256) return set_error(NWQ_EINVAL, "bad Kraus list");
  rc = check_qubits(h, qubits, k);
  if (rc) return rc;
  const int d = 1 << k;
  std::vector<cd> K((size_t)n_kraus * d * d);
  for (size_t i = 0; i < K.size(); ++i) {
    if (!std::isfinite(kraus[2 * i]) || !std::isfinite(kraus[2 * i + 1])) return set_error(NWQ_EINVAL, "non-finite Kraus entry");
    K[i] = cd(kraus[2 * i], kraus[2 * i + 1]);
  }
  // CPTP: sum_k K^dag K = I
  double err = 0.0;
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      cd s = 0.0;
      for (int t = 0; t < n_kraus; ++t)
        for (int l = 0; l < d; ++l) s += std::conj(K[(size_t)t * d * d + l * d + r]) * K[(size_t)t * d * d + l * d + c];
      err = std::max(err, std::abs(s - (r == c ? cd(1.0) : cd(0.0))));
    }
  if (err > 1e-12) return set_error(NWQ_ENOTCPTP, "Kraus set is not trace preserving (max |sum K^dag K - I| = " + std::to_string(err) + ")");
  std::vector<cd> S;
  superop(K.data(), n_kraus, k, S);
  return dm_push(h, qubits, k, S);
}

int nwq_depolarize(nwq_handle h, const int* qubits, int k, double p) {
  return nwq_depolarize_ex(h, qubits, k, p, NWQ_DEPOL_REPLACE);
}

int nwq_depolarize_ex(nwq_handle h, const int* qubits, int k, double p, int convention) {
  if (!(p >= 0.0 && p <= 1.0)) return set_error(NWQ_EINVAL, "depolarising p outside [0, 1]");
  if (k < 1 || k > 2) return set_error(NWQ_EINVAL, "depolarising channel on k = 1 or 2 qubits");
  if (convention != NWQ_DEPOL_REPLACE && convention != NWQ_DEPOL_PAULI)
    return set_error(NWQ_EINVAL, "depolarising convention must be NWQ_DEPOL_REPLACE or NWQ_DEPOL_PAULI");
  // Kraus form over the 4^k Paulis: identity weight w0, every other Pauli w.
  // Replacement: w0 = sqrt(1 - (4^k - 1) p / 4^k), w = sqrt(p / 4^k) (Pauli twirl);
  // uniform Pauli errors: w0 = sqrt(1 - p), w = sqrt(p / (4^k - 1)).
  const cd I1(0, 1);
  const cd paulis[4][4] = {{1.0, 0.0, 0.0, 1.0}, {0.0, 1.0, 1.0, 0.0}, {0.0, -I1, I1, 0.0}, {1.0, 0.0, 0.0, -1.0}};
  const int d = 1 << k, npl = d * d;
  std::vector<double> kr((size_t)npl * d * d * 2, 0.0);
  const bool repl = convention == NWQ_DEPOL_REPLACE;
  const double w0 = std::sqrt(std::max(0.0, repl ? 1.0 - (npl - 1) * p / npl : 1.0 - p));
  const double w = std::sqrt(repl ? p / npl : p / (npl - 1));
  for (int t = 0; t < npl; ++t) {
    const double wt = t == 0 ? w0 : w;
    const int a = t % 4, b = t / 4;   // factor a on qubits[0], b on qubits[1]
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) {
        cd v;
        if (k == 1) v = paulis[a][r * 2 + c];
        else v = paulis[a][(r & 1) * 2 + (c & 1)] * paulis[b][(r >> 1) * 2 + (c >> 1)];
        v *= wt;
        kr[((size_t)t * d * d + r * d + c) * 2] = v.real();
        kr[((size_t)t * d * d + r * d + c) * 2 + 1] = v.imag();
      }
  }
  return nwq_apply_channel(h, qubits, k, kr.data(), npl);
}

int nwq_thermal_relax(nwq_handle h, int q, double t1, double t2, double t) {
  if (!h) return set_error(NWQ_EINVAL, "NULL handle");
  if (h->kind != NWQ_KIND_DM) return set_error(NWQ_EKIND, "thermal relaxation applies to density-matrix handles");
  if (!(t1 > 0.0) || !(t2 > 0.0) || !(t >= 0.0) || !std::isfinite(t))
    return set_error(NWQ_EINVAL, "thermal relaxation needs T1 > 0, T2 > 0, t >= 0");
  if (t2 > 2.0 * t1 * (1.0 + 1e-12)) return set_error(NWQ_EINVAL, "thermal relaxation needs T2 <= 2 T1");
  // Populations: amplitude damping with 1 - gamma = e^{-t/T1}.  Coherences:
  // sqrt(1 - gamma) sqrt(1 - lambda) = e^{-t/T2}, so the remaining pure
  // dephasing is 1 - lambda = e^{-t (2/T2 - 1/T1)}.
  const double gamma = -std::expm1(-t / t1);
  const double lambda = std::max(0.0, -std::expm1(-t * (2.0 / t2 - 1.0 / t1)));
  int rc = nwq_amp_damp(h, q, gamma);
  if (!rc) rc = nwq_phase_damp(h, q, lambda);
  return rc;
}

int nwq_amp_damp(nwq_handle h, int q, double g) {
  if (!(g >= 0.0 && g <= 1.0)) return set_error(NWQ_EINVAL, "amplitude damping gamma outside [0, 1]");
  const double kr[16] = {1, 0, 0, 0, 0, 0, std::sqrt(1 - g), 0,
                         0, 0, std::sqrt(g), 0, 0, 0, 0, 0};
  return nwq_apply_channel(h, &q, 1, kr, 2);
}

int nwq_phase_damp(nwq_handle h, int q, double l) {
  if (!(l >= 0.0 && l <= 1.0)) return set_error(NWQ_EINVAL, "phase damping lambda outside [0, 1]");
  const double kr[16] = {1, 0, 0, 0, 0, 0, std::sqrt(1 - l), 0,
                         0, 0, 0, 0, 0, 0, std::sqrt(l), 0};
  return nwq_apply_channel(h, &q, 1, kr, 2);
}

// ----------------------------------------------------------- reductions ----
// Plan the tile passes of an SV Pauli-term reduction.
struct PassPlan {
  TileShape shape;
  std::vector<int> terms;
};

static std::vector<PassPlan> plan_pauli_passes(int n, const std::vector<int>& ids, const uint64_t* xm) {
  std::vector<PassPlan> passes;
  const int c = n <= 11 ? n : 6;
  const int mmax = n <= 11 ? 0 : std::min(5, n - c);   // tile <= 2^11 amplitudes (32 KiB LDS)
  const uint64_t lowmask = c >= 64 ? ~0ull : ((1ull << c) - 1ull);
  for (int t : ids) {
    const uint64_t hx = xm[t] & ~lowmask;
    std::vector<int> bits;
    for (int b = 0; b < n; ++b)
      if ((hx >> b) & 1ull) bits.push_back(b);
    int chosen = -1;
    for (size_t p = 0; p < passes.size() && chosen < 0; ++p) {
      if ((int)passes[p].terms.size() >= 16 || passes[p].shape.m < 0) continue;
      std::vector<int> u(passes[p].shape.hi, passes[p].shape.hi + passes[p].shape.m);
      for (int b : bits)
        if (std::find(u.begin(), u.end(), b) == u.end()) u.push_back(b);
      if ((int)u.size() <= mmax) {
        std::sort(u.begin(), u.end());
        passes[p].shape.m = (int)u.size();
        for (size_t i = 0; i < u.size(); ++i) passes[p].shape.hi[i] = u[i];
        passes[p].terms.push_back(t);
        chosen = (int)p;
      }
    }
    if (chosen < 0) {
      if ((int)bits.size() > mmax) {   // wider than a tile: a pair pass of its own (m = -1)
        PassPlan pp{};
        pp.shape.c = c;
        pp.shape.m = -1;
        pp.terms.push_back(t);
        passes.push_back(pp);
        continue;
      }
      PassPlan pp{};
      pp.shape.c = c;
      pp.shape.m = (int)bits.size();
      for (size_t i = 0; i < bits.size(); ++i) pp.shape.hi[i] = bits[i];
      pp.terms.push_back(t);
      passes.push_back(pp);
    }
  }
  // widen every tile to the full 2^(c + mmax) amplitudes with unused high bits
  for (auto& pp : passes) {
    if (pp.shape.m < 0) continue;
    for (int b = c; b < n && pp.shape.m < mmax; ++b) {
      if (std::find(pp.shape.hi, pp.shape.hi + pp.shape.m, b) == pp.shape.hi + pp.shape.m)
        pp.shape.hi[pp.shape.m++] = b;
    }
    std::sort(pp.shape.hi, pp.shape.hi + pp.shape.m);
  }
  return passes;
}

static uint64_t to_local(uint64_t mask, const TileShape& s) {
  const uint64_t low = mask & ((s.c >= 64) ? ~0ull : ((1ull << s.c) - 1ull));
  uint64_t l = low;
  for (int i = 0; i < s.m; ++i)
    if ((mask >> s.hi[i]) & 1ull) l |= 1ull << (s.c + i);
  return l;
}

static uint64_t inside_mask(const TileShape& s) {
  uint64_t m = (s.c >= 64) ? ~0ull : ((1ull << s.c) - 1ull);
  for (int i = 0; i < s.m; ++i) m |= 1ull << s.hi[i];
  return m;
}

// Reduce T Pauli terms; results_dev[0..T) = Re <P_t>, and if coeffs:
// results_dev[T] = sum_t coeffs[t] Re <P_t>.  Leaves the copy to the caller.
static int run_pauli(nwq_state* h, int T, const uint64_t* xm, const uint64_t* zm, const double* coeffs,
                     int* rows_out) {
  const int n = h->n;
  for (int t = 0; t < T; ++t) {
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    if ((xm[t] & ~all) || (zm[t] & ~all)) return set_error(NWQ_ERANGE, "Pauli mask has bits beyond n");
  }
  if (h->kind == NWQ_KIND_DM) {
    // rows 2t, 2t+1: Re and Im of Tr(rho P_t)
    std::vector<TermDev> td(T);
    for (int t = 0; t < T; ++t) {
      td[t] = TermDev{xm[t], zm[t], 0ull, __builtin_popcountll(xm[t] & zm[t]) & 3, 0};
    }
    const int G = dm_pauli_grid(n);
    int rc = ensure_partials(h, (size_t)2 * T * G);
    if (rc) return rc;
    rc = ensure_results(h, (size_t)2 * T + 1);
    if (rc) return rc;
    for (int t0 = 0; t0 < T; t0 += 64) {
      const int cnt = std::min(64, T - t0);
      void* dterms = nullptr;
      rc = arena_put(h, td.data() + t0, cnt * sizeof(TermDev), &dterms);
      if (rc) return rc;
      timing_begin(h, KC_REDUCE);
      launch_dm_pauli(h->stream, h->data, n, static_cast<const TermDev*>(dterms), cnt,
                      h->partials + (size_t)2 * t0 * G, G);
      timing_end(h);
      rc = last_launch("dm_pauli");
      if (rc) return rc;
    }
    const double* dco = nullptr;
    if (coeffs) {
      std::vector<double> c2(2 * T, 0.0);
      for (int t = 0; t < T; ++t) c2[2 * t] = coeffs[t];
      void* p = nullptr;
      rc = arena_put(h, c2.data(), c2.size() * sizeof(double), &p);
      if (rc) return rc;
      dco = static_cast<const double*>(p);
    }
    timing_begin(h, KC_REDUCE);
    launch_reduce_rows(h->stream, h->partials, 2 * T, G, dco, h->results_dev);
    timing_end(h);
    *rows_out = 2 * T;
    return last_launch("reduce_rows");
  }
  // terms with no flipped bits (Z strings) run in streaming passes of their
  // own, up to 16 consecutive rows each; the others are planned into tiles
  std::vector<int> flip_ids;
  for (int t = 0; t < T; ++t)
    if (xm[t] != 0) flip_ids.push_back(t);
  std::vector<PassPlan> passes = plan_pauli_passes(n, flip_ids, xm);
  const int G = pauli_tile_grid(n, TileShape{n <= 11 ? n : 6, n <= 11 ? 0 : 5, {}});
  int rc = ensure_partials(h, (size_t)T * G);
  if (rc) return rc;
  rc = ensure_results(h, (size_t)T + 1);
  if (rc) return rc;
  for (int t = 0; t < T;) {
    if (xm[t] != 0) {
      ++t;
      continue;
    }
    ZMasks zs{};
    int cnt = 0;
    while (t + cnt < T && cnt < 16 && xm[t + cnt] == 0) {
      zs.z[cnt] = zm[t + cnt];
      ++cnt;
    }
    timing_begin(h, KC_REDUCE);
    launch_pauli_diag(h->stream, h->data, n, zs, cnt, h->partials, t, G);
    timing_end(h);
    rc = last_launch("pauli_diag");
    if (rc) return rc;
    t += cnt;
  }
  // rows follow the caller's term order
  for (auto& pp : passes) {
    if (pp.shape.m < 0) {
      const int t = pp.terms[0];
      timing_begin(h, KC_REDUCE);
      launch_pauli_pairs(h->stream, h->data, n, xm[t], zm[t], __builtin_popcountll(xm[t] & zm[t]) & 3,
                         h->partials + (size_t)t * G, G);
      timing_end(h);
      rc = last_launch("pauli_pairs");
      if (rc) return rc;
      continue;
    }
    std::vector<TermDev> td;
    for (int t : pp.terms) {
      const uint64_t in = inside_mask(pp.shape);
      td.push_back(TermDev{to_local(xm[t], pp.shape), to_local(zm[t] & in, pp.shape), zm[t] & ~in,
                           __builtin_popcountll(xm[t] & zm[t]) & 3, 0});
    }
    // terms of one pass are contiguous rows only if in order; launch per run of consecutive rows
    size_t i = 0;
    while (i < pp.terms.size()) {
      size_t j = i + 1;
      while (j < pp.terms.size() && pp.terms[j] == pp.terms[j - 1] + 1) ++j;
      void* dterms = nullptr;
      rc = arena_put(h, td.data() + i, (j - i) * sizeof(TermDev), &dterms);
      if (rc) return rc;
      timing_begin(h, KC_REDUCE);
      launch_pauli_tile(h->stream, h->data, n, pp.shape, static_cast<const TermDev*>(dterms), (int)(j - i),
                        h->partials, pp.terms[i], G);
      timing_end(h);
      rc = last_launch("pauli_tile");
      if (rc) return rc;
      i = j;
    }
  }
  const double* dco = nullptr;
  if (coeffs) {
    void* p = nullptr;
    rc = arena_put(h, coeffs, T * sizeof(double), &p);
    if (rc) return rc;
    dco = static_cast<const double*>(p);
  }
  timing_begin(h, KC_REDUCE);
  launch_reduce_rows(h->stream, h->partials, T, G, dco, h->results_dev);
  timing_end(h);
  *rows_out = T;
  return last_launch("reduce_rows");
}

static int fetch_results(nwq_state* h, int count) {
  NWQ_TRY_HIP(hipMemcpyAsync(h->results_host, h->results_dev, count * sizeof(double), hipMemcpyDeviceToHost, h->stream),
              "hipMemcpyAsync(results)");
  NWQ_TRY_HIP(hipStreamSynchronize(h->stream), "hipStreamSynchronize(results)");
  return NWQ_OK;
}

int nwq_expval_pauli_terms(nwq_handle h, int T, const uint64_t* xm, const uint64_t* zm, double* out) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (T < 0 || (T > 0 && (!xm || !zm || !out))) return set_error(NWQ_EINVAL, "bad term arrays");
  if (T == 0) return NWQ_OK;
  rc = flush_all(h);
  if (rc) return rc;
  int rows = 0;
  rc = run_pauli(h, T, xm, zm, nullptr, &rows);
  if (rc) return rc;
  rc = fetch_results(h, rows);
  if (rc) return rc;
  for (int t = 0; t < T; ++t) out[t] = h->kind == NWQ_KIND_DM ? h->results_host[2 * t] : h->results_host[t];
  return NWQ_OK;
}

int nwq_memory(nwq_handle h, size_t* bytes) {
  if (!h) return set_error(NWQ_EINVAL, "NULL handle");
  if (!bytes) return set_error(NWQ_EINVAL, "NULL output pointer");
  size_t b = h->owns ? (size_t)h->len * sizeof(double2) : 0;
  if (h->arena_dev) b += kArenaBytes;
  b += h->partials_cap * sizeof(double) + h->results_cap * sizeof(double) + h->fuse_cap;
  *bytes = b;
  return NWQ_OK;
}

int nwq_expval_pauli_terms_complex(nwq_handle h, int T, const uint64_t* xm, const uint64_t* zm, double* out_re,
                                   double* out_im) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (T < 0 || (T > 0 && (!xm || !zm || !out_re))) return set_error(NWQ_EINVAL, "bad term arrays");
  if (T == 0) return NWQ_OK;
  rc = flush_all(h);
  if (rc) return rc;
  int rows = 0;
  rc = run_pauli(h, T, xm, zm, nullptr, &rows);
  if (rc) return rc;
  rc = fetch_results(h, rows);
  if (rc) return rc;
  const bool dm = h->kind == NWQ_KIND_DM;
  for (int t = 0; t < T; ++t) {
    out_re[t] = dm ? h->results_host[2 * t] : h->results_host[t];
    if (out_im) out_im[t] = dm ? h->results_host[2 * t + 1] : 0.0;
  }
  return NWQ_OK;
}

int nwq_expval_pauli_sum(nwq_handle h, int T, const uint64_t* xm, const uint64_t* zm, const double* coeffs,
                         double* out) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (out == nullptr || T < 0 || (T > 0 && (!xm || !zm || !coeffs))) return set_error(NWQ_EINVAL, "bad term arrays");
  if (T == 0) {
    *out = 0.0;
    return NWQ_OK;
  }
  rc = flush_all(h);
  if (rc) return rc;
  int rows = 0;
  rc = run_pauli(h, T, xm, zm, coeffs, &rows);
  if (rc) return rc;
  rc = fetch_results(h, rows + 1);
  if (rc) return rc;
  *out = h->results_host[rows];
  return NWQ_OK;
}

int nwq_trace(nwq_handle h, double* out, double* imag_out) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->kind != NWQ_KIND_DM) return set_error(NWQ_EKIND, "trace needs a density-matrix handle");
  if (out == nullptr) return set_error(NWQ_EINVAL, "out pointer is NULL");
  rc = flush_all(h);
  if (rc) return rc;
  const uint64_t zero = 0;
  int rows = 0;
  rc = run_pauli(h, 1, &zero, &zero, nullptr, &rows);
  if (rc) return rc;
  rc = fetch_results(h, 2);
  if (rc) return rc;
  *out = h->results_host[0];
  if (imag_out) *imag_out = h->results_host[1];
  return NWQ_OK;
}

int nwq_purity(nwq_handle h, double* out) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (out == nullptr) return set_error(NWQ_EINVAL, "out pointer is NULL");
  rc = flush_all(h);
  if (rc) return rc;
  const int G = sumsq_grid(h->len);
  rc = ensure_partials(h, G);
  if (rc) return rc;
  rc = ensure_results(h, 2);
  if (rc) return rc;
  timing_begin(h, KC_REDUCE);
  launch_sumsq(h->stream, h->data, h->len, h->partials, G);
  launch_reduce_rows(h->stream, h->partials, 1, G, nullptr, h->results_dev);
  timing_end(h);
  rc = last_launch("sumsq");
  if (rc) return rc;
  rc = fetch_results(h, 1);
  if (rc) return rc;
  *out = h->results_host[0];
  return NWQ_OK;
}

int nwq_timing_enable(nwq_handle h, int enable) {
  int rc = check_handle(h);
  if (rc) return rc;
  h->timing = enable != 0;
  return NWQ_OK;
}

int nwq_timing_read(nwq_handle h, long long* count, double* ms, int reset) {
  int rc = check_handle(h);
  if (rc) return rc;
  rc = drain_timing(h);
  if (rc) return rc;
  for (int i = 0; i < NWQ_TIMING_CLASSES; ++i) {
    if (count) count[i] = h->t_count[i];
    if (ms) ms[i] = h->t_ms[i];
    if (reset) {
      h->t_count[i] = 0;
      h->t_ms[i] = 0.0;
    }
  }
  return NWQ_OK;
}

}  // extern "C"

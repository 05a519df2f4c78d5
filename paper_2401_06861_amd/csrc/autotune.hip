// Launch-shape autotuner for the streaming gate kernels of a handle.
//
// For each kernel class and target bucket (lowest target bit 0-2, 3-10 or
// 11 and up) it times every candidate (groups per thread in {1, 2, 4, 8},
// and 16 for the 1q, diagonal and permutation kernels, x non-temporal hint
// off/on) with HIP events on the handle's own stream and
// state, and keeps the fastest.  Candidates apply self-inverse operations in
// pairs on up to three target bits of the bucket (X as a dense 2x2 twice for
// the dense 1-qubit kernel, Z Z for the diagonal kernel, CX CX for the
// permutation kernel, CZ as a dense 4x4 twice for the 2-qubit kernel, and on
// a density matrix Z (x) conj(Z) twice for the 1-qubit superoperator kernel
// and the diagonal superoperator of Z (x) Z twice for the 16 x 16 kernel).
// Every operator entry is 0 or +-1, so each product and sum is exact in
// FP64 and the pairs leave the state's values unchanged (a zero may change
// the sign of its zero).  The kernels' timing does not depend on the values.
//
// The fusion autotuner times a caller's circuit under every fusion width and
// fused-kernel choice and keeps the fastest.
#include <algorithm>
#include <cmath>

#include "engine.h"

namespace nwq {
namespace {

struct Cand { int ppt, nt; };
// Without the hint only 1 and 4 groups per thread are offered: on the MI355X
// the other hint-free shapes never won a target bit at 30 qubits.
// Shapes 32, 64 and 128 (and one entry per thread of the diagonal class) are
// timed in dispatch order and in XCD-contiguous order (flags 3).
const Cand kCands[] = {{1, 1}, {2, 1}, {4, 1}, {8, 1}, {16, 1}, {1, 0}, {4, 0}, {32, 1},
                       {64, 1}, {128, 1}, {32, 3}, {64, 3}, {128, 3}, {1, 3}};

// 16 groups per thread is offered to the kernels with at most two streams
// per group (the 4x4 kernel would run out of registers).
bool allows16(int cls) { return cls == KC_SV1Q || cls == KC_DIAG || cls == KC_PERM; }
// Shapes 32, 64 and 128 select the split-workgroup kernels (256, 512 or 1024
// threads) of the dense 1q class (targets from 9 up), the permutation class
// and the 4x4 classes (SV 2q dense, DM 1q superoperator), where no lane
// exchange applies.
bool allows_x2(int cls) { return cls == KC_SV1Q || cls == KC_PERM || cls == KC_SV2Q || cls == KC_DM1; }
bool valid_ppt(int cls, int ppt) {
  // class 7: one group per thread, or the split-workgroup kernels of 1024 or
  // 512 threads (one or two members per thread)
  if (cls == KC_DM2) return ppt == 1 || ppt == 64 || ppt == 128;
  if (ppt == 1 || ppt == 2 || ppt == 4 || ppt == 8) return true;
  if (ppt == 16) return allows16(cls);
  return (ppt == 32 || ppt == 64 || ppt == 128) && allows_x2(cls);
}
// Flags: bit 0 the non-temporal hint; bit 1 the XCD-contiguous workgroup
// order, which the split-workgroup shapes and one entry per thread of the
// diagonal class take.
bool valid_flags(int cls, int ppt, int flags) {
  if (flags == 0 || flags == 1) return true;
  return (flags == 2 || flags == 3) && (ppt >= 32 || (cls == KC_DIAG && ppt == 1));
}
constexpr const char* kShapeMsg =
    "groups per thread must be 1, 2, 4 or 8 (or 16 for classes 1, 2 and 3; 32, 64 or 128 for classes 1, 3, 4 "
    "and 6); class 7 takes 1, 64 or 128";
constexpr const char* kFlagsMsg = "flags must be 0 or 1 (0 to 3 with shapes 32, 64 and 128, and with shape 1 of class 2)";

using Runner = void (*)(nwq_state*, const LaunchCfg&, int);

void run_1q(nwq_state* h, const LaunchCfg& c, int q) {
  Mat2 m;   // X through the dense kernel
  m.m[0] = make_double2(0, 0); m.m[1] = make_double2(1, 0); m.m[2] = make_double2(1, 0); m.m[3] = make_double2(0, 0);
  launch_sv_1q(h->stream, h->data, h->nbits, q, m, c);
  launch_sv_1q(h->stream, h->data, h->nbits, q, m, c);
}
void run_diag(nwq_state* h, const LaunchCfg& c, int q) {
  Diag4 d{};
  d.d[0] = make_double2(1, 0); d.d[1] = make_double2(-1, 0); d.d[2] = d.d[0]; d.d[3] = d.d[1];
  launch_sv_diag(h->stream, h->data, h->nbits, q, -1, d, c);
  launch_sv_diag(h->stream, h->data, h->nbits, q, -1, d, c);
}
void run_perm(nwq_state* h, const LaunchCfg& c, int q) {
  const int t = q + 1 < h->nbits ? q + 1 : q - 1;
  launch_sv_swap2(h->stream, h->data, h->nbits, q, t, 1ull << q, (1ull << q) + (1ull << t), c);
  launch_sv_swap2(h->stream, h->data, h->nbits, q, t, 1ull << q, (1ull << q) + (1ull << t), c);
}
void run_2q(nwq_state* h, const LaunchCfg& c, int q) {
  const int t = q + 1 < h->nbits ? q + 1 : q - 1;
  Mat4 m{};
  for (int i = 0; i < 4; ++i) m.m[5 * i] = make_double2(i == 3 ? -1.0 : 1.0, 0);
  launch_sv_2q(h->stream, h->data, h->nbits, q, t, m, c);
  launch_sv_2q(h->stream, h->data, h->nbits, q, t, m, c);
}
void run_dm2(nwq_state* h, const LaunchCfg& c, int q) {
  // (Z (x) Z) (x) conj(Z (x) Z) on (a, b, a + n, b + n): diagonal +-1, self-inverse,
  // twice as a dense 16 x 16 and twice in the compact form of a Pauli-pattern
  // superoperator (a noisy two-qubit gate takes one or the other, and their
  // fastest shapes differ): the shape is picked for both
  const int t = q + 1;
  const int vq[4] = {q, t, q + h->n, t + h->n};
  std::vector<double2> S(256 + 32, make_double2(0.0, 0.0));
  for (int u = 0; u < 16; ++u) {
    const double d = __builtin_popcount(u) % 2 ? -1.0 : 1.0;
    S[17 * u] = make_double2(d, 0.0);
    S[256 + u] = make_double2(d, 0.0);                                 // diagonal entries
    if (u % 5 == 0) S[256 + 16 + 5 * (u / 5)] = make_double2(d, 0.0);  // 4 x 4 among 0, 5, 10, 15
  }
  void* dev = nullptr;
  if (arena_put(h, S.data(), S.size() * sizeof(double2), &dev) != NWQ_OK) return;
  const double2* dense = static_cast<const double2*>(dev);
  launch_sv_kq(h->stream, h->data, h->nbits, 4, vq, dense, c);
  launch_sv_kq(h->stream, h->data, h->nbits, 4, vq, dense, c);
  launch_sv_kq(h->stream, h->data, h->nbits, 4, vq, dense + 256, c, true);
  launch_sv_kq(h->stream, h->data, h->nbits, 4, vq, dense + 256, c, true);
}
void run_dm1(nwq_state* h, const LaunchCfg& c, int q) {
  Mat4 m{};   // Z (x) conj(Z) on (column q, row q + n): diag(1, -1, -1, 1)
  const double dz[4] = {1, -1, -1, 1};
  for (int i = 0; i < 4; ++i) m.m[5 * i] = make_double2(dz[i], 0);
  launch_sv_2q(h->stream, h->data, h->nbits, q, q + h->n, m, c);
  launch_sv_2q(h->stream, h->data, h->nbits, q, q + h->n, m, c);
}

}  // namespace
}  // namespace nwq

using namespace nwq;

extern "C" {

int nwq_set_launch(nwq_handle h, int cls, int bucket, int ppt, int nontemporal) {
  if (!h) return set_error(NWQ_EINVAL, "NULL handle");
  if (cls < 0 || cls >= KC_COUNT) return set_error(NWQ_EINVAL, "kernel class out of range");
  if (bucket < -1 || bucket >= kBuckets) return set_error(NWQ_EINVAL, "bucket must be -1, 0, 1 or 2");
  if (!valid_ppt(cls, ppt)) return set_error(NWQ_EINVAL, kShapeMsg);
  if (!valid_flags(cls, ppt, nontemporal)) return set_error(NWQ_EINVAL, kFlagsMsg);
  for (int b = 0; b < kBuckets; ++b) {
    if (bucket >= 0 && b != bucket) continue;
    h->cfg[cls][b].ppt = ppt;
    h->cfg[cls][b].nt = nontemporal;
  }
  for (int q = 0; q < kMaxTargetBits; ++q)   // the bucket's shape now holds for each of its targets
    if (bucket < 0 || bucket_of(q) == bucket) h->tset[cls][q] = false;
  return NWQ_OK;
}

int nwq_set_launch_target(nwq_handle h, int cls, int bit, int ppt, int nontemporal) {
  if (!h) return set_error(NWQ_EINVAL, "NULL handle");
  if (cls < 0 || cls >= KC_COUNT) return set_error(NWQ_EINVAL, "kernel class out of range");
  if (bit < 0 || bit >= kMaxTargetBits) return set_error(NWQ_EINVAL, "target bit out of range");
  if (ppt == 0) {
    h->tset[cls][bit] = false;
    return NWQ_OK;
  }
  if (!valid_ppt(cls, ppt)) return set_error(NWQ_EINVAL, kShapeMsg);
  if (!valid_flags(cls, ppt, nontemporal)) return set_error(NWQ_EINVAL, kFlagsMsg);
  h->tcfg[cls][bit].ppt = ppt;
  h->tcfg[cls][bit].nt = nontemporal;
  h->tset[cls][bit] = true;
  return NWQ_OK;
}

int nwq_get_launch_target(nwq_handle h, int cls, int bit, int* ppt, int* nontemporal) {
  if (!h) return set_error(NWQ_EINVAL, "NULL handle");
  if (cls < 0 || cls >= KC_COUNT) return set_error(NWQ_EINVAL, "kernel class out of range");
  if (bit < 0 || bit >= kMaxTargetBits) return set_error(NWQ_EINVAL, "target bit out of range");
  const LaunchCfg& c = h->shape(cls, bit);
  if (ppt) *ppt = c.ppt;
  if (nontemporal) *nontemporal = c.nt;
  return NWQ_OK;
}

int nwq_get_launch(nwq_handle h, int cls, int bucket, int* ppt, int* nontemporal) {
  if (!h) return set_error(NWQ_EINVAL, "NULL handle");
  if (cls < 0 || cls >= KC_COUNT) return set_error(NWQ_EINVAL, "kernel class out of range");
  if (bucket < 0 || bucket >= kBuckets) return set_error(NWQ_EINVAL, "bucket must be 0, 1 or 2");
  if (ppt) *ppt = h->cfg[cls][bucket].ppt;
  if (nontemporal) *nontemporal = h->cfg[cls][bucket].nt;
  return NWQ_OK;
}

int nwq_autotune(nwq_handle h, int reps, double* best_ms) {
  if (!h) return set_error(NWQ_EINVAL, "NULL handle");
  if (reps < 1 || reps > 100) return set_error(NWQ_EINVAL, "reps must be in [1, 100]");
  int rc = flush_all(h);
  if (rc) return rc;
  if (best_ms)
    for (int i = 0; i < KC_COUNT * kBuckets; ++i) best_ms[i] = -1.0;
  // lo_max: largest lowest-target bit the runner allows; launches: per run
  struct Job { int cls; Runner run; int lo_max; int launches; };
  std::vector<Job> jobs;
  if (h->kind == NWQ_KIND_SV) {
    jobs.push_back({KC_SV1Q, run_1q, h->n - 1, 2});
    jobs.push_back({KC_DIAG, run_diag, h->n - 1, 2});
    if (h->n >= 2) {
      jobs.push_back({KC_PERM, run_perm, h->n - 2, 2});
      jobs.push_back({KC_SV2Q, run_2q, h->n - 2, 2});
    }
  } else {
    jobs.push_back({KC_DM1, run_dm1, h->n - 1, 2});
    if (h->n >= 2) jobs.push_back({KC_DM2, run_dm2, h->n - 2, 4});
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rc = check_hip(hipEventCreate(&e0), "hipEventCreate");
  if (!rc) rc = check_hip(hipEventCreate(&e1), "hipEventCreate");
  // Every lowest target bit is timed under every candidate shape (reps timed
  // pairs; one warm-up pair per candidate).  Each target keeps its fastest
  // shape; each bucket keeps the shape with the least total time over its
  // targets.
  for (const Job& j : jobs) {
    const int nq = std::min(j.lo_max + 1, kMaxTargetBits);
    std::vector<LaunchCfg> cands;
    for (const Cand& c : kCands) {
      if (!valid_ppt(j.cls, c.ppt) || !valid_flags(j.cls, c.ppt, c.nt)) continue;
      LaunchCfg cfg;
      cfg.ppt = c.ppt;
      cfg.nt = c.nt;
      cands.push_back(cfg);
    }
    std::vector<double> t(cands.size() * (size_t)nq, 0.0);   // ms per launch [cand][q]
    for (size_t ci = 0; ci < cands.size() && !rc; ++ci)
      for (int q = 0; q < nq && !rc; ++q) {
        if (q == 0) j.run(h, cands[ci], q);   // warm-up
        rc = check_hip(hipEventRecord(e0, h->stream), "hipEventRecord");
        for (int r = 0; r < reps && !rc; ++r) j.run(h, cands[ci], q);
        if (!rc) rc = check_hip(hipGetLastError(), "autotune launch");
        if (!rc) rc = check_hip(hipEventRecord(e1, h->stream), "hipEventRecord");
        if (!rc) rc = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        t[ci * nq + q] = ms / ((double)j.launches * reps);
      }
    if (rc) break;
    double bsum[kBuckets] = {0.0, 0.0, 0.0};
    int bcnt[kBuckets] = {0, 0, 0};
    for (int q = 0; q < nq; ++q) {
      size_t best = 0;
      for (size_t ci = 1; ci < cands.size(); ++ci)
        if (t[ci * nq + q] < t[best * nq + q]) best = ci;
      h->tcfg[j.cls][q] = cands[best];
      h->tset[j.cls][q] = true;
      bsum[bucket_of(q)] += t[best * nq + q];
      ++bcnt[bucket_of(q)];
    }
    for (int b = 0; b < kBuckets; ++b) {
      if (bcnt[b] == 0) continue;
      size_t best = 0;
      double best_total = 1e300;
      for (size_t ci = 0; ci < cands.size(); ++ci) {
        double tot = 0.0;
        for (int q = 0; q < nq; ++q)
          if (bucket_of(q) == b) tot += t[ci * nq + q];
        if (tot < best_total) {
          best_total = tot;
          best = ci;
        }
      }
      h->cfg[j.cls][b] = cands[best];
      if (best_ms) best_ms[j.cls * kBuckets + b] = bsum[b] / bcnt[b];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"

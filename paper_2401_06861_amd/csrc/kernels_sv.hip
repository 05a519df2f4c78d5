// Streaming gate kernels for gfx950: one pass over the amplitude vector per
// gate.  The vector holds 2^nbits interleaved complex128 entries (nbits = n
// for a state vector, 2n for the row-major vec of a density matrix, whose
// superoperators are applied by the same kernels on (column, row) bit sets).
//
// Every kernel is HBM-bound (<= 4 flop/byte against a ~9.8 flop/byte FP64
// ridge), so the design goals are: 16-byte (dwordx4) loads of whole
// amplitudes, several independent groups per thread with all loads issued
// before any arithmetic (bytes in flight), wave-contiguous addressing for
// targets q >= 6 and cache-line-local addressing below, 64-bit byte offsets
// only in address arithmetic, and an optional non-temporal hint (the data is
// touched once per pass).  The launch shape (groups per thread PPT and the
// hint) is a template choice picked per kernel class and target bucket by
// the autotuner; the 4x4 kernel stops at 8 groups per thread (register
// budget).
#include "nwq_internal.h"

namespace nwq {
namespace {

// Clang vector of two doubles: a first-class 16-byte value that stays in
// registers (HIP's double2 struct can take a round trip through scratch
// when only copied).
typedef double vd2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned long long insert0(unsigned long long p, int q) {
  const unsigned long long lo = p & ((1ull << q) - 1ull);
  return ((p >> q) << (q + 1)) | lo;
}

__device__ __forceinline__ vd2 mk(double a, double b) { vd2 r; r.x = a; r.y = b; return r; }
__device__ __forceinline__ vd2 tov(const double2& d) { return mk(d.x, d.y); }
__device__ __forceinline__ vd2 cmul(vd2 a, vd2 b) { return mk(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)); }
// a * b + c
__device__ __forceinline__ vd2 cfma(vd2 a, vd2 b, vd2 c) {
  return mk(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}

template <bool NTM>
__device__ __forceinline__ vd2 gld(const double2* p) {
  if constexpr (NTM) return __builtin_nontemporal_load(reinterpret_cast<const vd2*>(p));
  else return *reinterpret_cast<const vd2*>(p);
}
template <bool NTM>
__device__ __forceinline__ void gst(double2* p, vd2 v) {
  if constexpr (NTM) __builtin_nontemporal_store(v, reinterpret_cast<vd2*>(p));
  else *reinterpret_cast<vd2*>(p) = v;
}

// |0...0> (entry 0 = 1, rest 0) written with plain stores (no memset node,
// so the kernel is safe inside captured graphs).
template <int EPT>
__global__ __launch_bounds__(kBlock) void k_fill_basis0(double2* __restrict__ a, unsigned long long u0, unsigned long long len) {
  const unsigned long long start = u0 + (unsigned long long)blockIdx.x * (kBlock * EPT) + threadIdx.x;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const unsigned long long i = start + (unsigned long long)j * kBlock;
    if (i < len) gst<false>(a + i, mk(i == 0 ? 1.0 : 0.0, 0.0));
  }
}

// 1-qubit dense gate: for each pair p, i0 = insert0(p, q), i1 = i0 | 2^q,
// (a_i0, a_i1) <- M (a_i0, a_i1).
template <int PPT, bool NTM>
__global__ __launch_bounds__(kBlock) void k_sv_1q(double2* __restrict__ a, unsigned long long u0, unsigned long long npairs,
                                                  int q, Mat2 m) {
  const unsigned long long start = u0 + (unsigned long long)blockIdx.x * (kBlock * PPT) + threadIdx.x;
  const unsigned long long off = 1ull << q;
  const vd2 m0 = tov(m.m[0]), m1 = tov(m.m[1]), m2 = tov(m.m[2]), m3 = tov(m.m[3]);
  if (start + (unsigned long long)(PPT - 1) * kBlock < npairs) {
    vd2 x0[PPT], x1[PPT];
    unsigned long long i0[PPT];
    // up to 8 groups: the two loads of a group back to back; 16 groups: all
    // lower members, then all upper members (longer runs per stream)
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      i0[j] = insert0(start + (unsigned long long)j * kBlock, q);
      x0[j] = gld<NTM>(a + i0[j]);
      if constexpr (PPT < 16) x1[j] = gld<NTM>(a + i0[j] + off);
    }
    if constexpr (PPT >= 16) {
#pragma unroll
      for (int j = 0; j < PPT; ++j) x1[j] = gld<NTM>(a + i0[j] + off);
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      gst<NTM>(a + i0[j], cfma(m0, x0[j], cmul(m1, x1[j])));
      gst<NTM>(a + i0[j] + off, cfma(m2, x0[j], cmul(m3, x1[j])));
    }
  } else {
    for (int j = 0; j < PPT; ++j) {
      const unsigned long long p = start + (unsigned long long)j * kBlock;
      if (p >= npairs) break;
      const unsigned long long i = insert0(p, q);
      const vd2 v0 = gld<NTM>(a + i), v1 = gld<NTM>(a + i + off);
      gst<NTM>(a + i, cfma(m0, v0, cmul(m1, v1)));
      gst<NTM>(a + i + off, cfma(m2, v0, cmul(m3, v1)));
    }
  }
}

// Diagonal gate on one or two qubits: a_i <- d[u(i)] a_i, u = bit q0 + 2 bit q1
// (q1 < 0: one qubit).  Entries are chosen with selects, not an indexed load.
template <int EPT, bool NTM>
__global__ __launch_bounds__(kBlock) void k_sv_diag(double2* __restrict__ a, unsigned long long u0, unsigned long long len,
                                                    int q0, int q1, Diag4 d) {
  const unsigned long long start = u0 + (unsigned long long)blockIdx.x * (kBlock * EPT) + threadIdx.x;
  const vd2 d0 = tov(d.d[0]), d1 = tov(d.d[1]), d2 = tov(d.d[2]), d3 = tov(d.d[3]);
  const bool two = q1 >= 0;
  const int qq = two ? q1 : q0;
  if (start + (unsigned long long)(EPT - 1) * kBlock < len) {
    vd2 v[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) v[j] = gld<NTM>(a + start + (unsigned long long)j * kBlock);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const unsigned long long i = start + (unsigned long long)j * kBlock;
      const bool b0 = (i >> q0) & 1ull, b1 = two && ((i >> qq) & 1ull);
      const vd2 f = b1 ? (b0 ? d3 : d2) : (b0 ? d1 : d0);
      gst<NTM>(a + i, cmul(f, v[j]));
    }
  } else {
    for (int j = 0; j < EPT; ++j) {
      const unsigned long long i = start + (unsigned long long)j * kBlock;
      if (i >= len) break;
      const bool b0 = (i >> q0) & 1ull, b1 = two && ((i >> qq) & 1ull);
      const vd2 f = b1 ? (b0 ? d3 : d2) : (b0 ? d1 : d0);
      gst<NTM>(a + i, cmul(f, gld<NTM>(a + i)));
    }
  }
}

// X gate: swap the two members of each pair (no arithmetic).
template <int PPT, bool NTM>
__global__ __launch_bounds__(kBlock) void k_sv_swap1(double2* __restrict__ a, unsigned long long u0, unsigned long long npairs,
                                                     int q) {
  const unsigned long long start = u0 + (unsigned long long)blockIdx.x * (kBlock * PPT) + threadIdx.x;
  const unsigned long long off = 1ull << q;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const unsigned long long p = start + (unsigned long long)j * kBlock;
    if (p < npairs) {
      const unsigned long long i = insert0(p, q);
      const vd2 v0 = gld<NTM>(a + i), v1 = gld<NTM>(a + i + off);
      gst<NTM>(a + i, v1);
      gst<NTM>(a + i + off, v0);
    }
  }
}

// Two-qubit permutation that exchanges two members of each quad (CX: the
// control=1 pair; SWAP: |01> <-> |10>).  Only the moved half of the vector
// is read and written.
template <int PPT, bool NTM>
__global__ __launch_bounds__(kBlock) void k_sv_swap2(double2* __restrict__ a, unsigned long long u0, unsigned long long nquads,
                                                     int qlo, int qhi, unsigned long long offA,
                                                     unsigned long long offB) {
  const unsigned long long start = u0 + (unsigned long long)blockIdx.x * (kBlock * PPT) + threadIdx.x;
  if (start + (unsigned long long)(PPT - 1) * kBlock < nquads) {
    vd2 va[PPT], vb[PPT];
    unsigned long long b[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      b[j] = insert0(insert0(start + (unsigned long long)j * kBlock, qlo), qhi);
      va[j] = gld<NTM>(a + b[j] + offA);
      vb[j] = gld<NTM>(a + b[j] + offB);
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      gst<NTM>(a + b[j] + offA, vb[j]);
      gst<NTM>(a + b[j] + offB, va[j]);
    }
  } else {
    for (int j = 0; j < PPT; ++j) {
      const unsigned long long p = start + (unsigned long long)j * kBlock;
      if (p >= nquads) break;
      const unsigned long long base = insert0(insert0(p, qlo), qhi);
      const vd2 x = gld<NTM>(a + base + offA), y = gld<NTM>(a + base + offB);
      gst<NTM>(a + base + offA, y);
      gst<NTM>(a + base + offB, x);
    }
  }
}

// Two-qubit dense gate: quads over the sorted bit pair; member u sits at
// base + bit0(u) 2^{q0} + bit1(u) 2^{q1} (operator order); out = M v.
template <int PPT, bool NTM>
__global__ __launch_bounds__(kBlock) void k_sv_2q(double2* __restrict__ a, unsigned long long u0, unsigned long long nquads,
                                                  int qlo, int qhi, unsigned long long o0,
                                                  unsigned long long o1, Mat4 m) {
  const unsigned long long start = u0 + (unsigned long long)blockIdx.x * (kBlock * PPT) + threadIdx.x;
  vd2 M[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) M[i] = tov(m.m[i]);
  if (start + (unsigned long long)(PPT - 1) * kBlock < nquads) {
    vd2 v[PPT][4];
    unsigned long long b[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      b[j] = insert0(insert0(start + (unsigned long long)j * kBlock, qlo), qhi);
      v[j][0] = gld<NTM>(a + b[j]);
      v[j][1] = gld<NTM>(a + b[j] + o0);
      v[j][2] = gld<NTM>(a + b[j] + o1);
      v[j][3] = gld<NTM>(a + b[j] + o0 + o1);
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const unsigned long long idx[4] = {b[j], b[j] + o0, b[j] + o1, b[j] + o0 + o1};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        vd2 acc = cmul(M[4 * r], v[j][0]);
#pragma unroll
        for (int c = 1; c < 4; ++c) acc = cfma(M[4 * r + c], v[j][c], acc);
        gst<NTM>(a + idx[r], acc);
      }
    }
  } else {
    for (int j = 0; j < PPT; ++j) {
      const unsigned long long p = start + (unsigned long long)j * kBlock;
      if (p >= nquads) break;
      const unsigned long long base = insert0(insert0(p, qlo), qhi);
      const unsigned long long idx[4] = {base, base + o0, base + o1, base + o0 + o1};
      vd2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = gld<NTM>(a + idx[u]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        vd2 acc = cmul(M[4 * r], v[0]);
#pragma unroll
        for (int c = 1; c < 4; ++c) acc = cfma(M[4 * r + c], v[c], acc);
        gst<NTM>(a + idx[r], acc);
      }
    }
  }
}

// k-qubit dense operator (k = 3 or 4; the 16 x 16 case is the fused
// two-qubit gate + channel superoperator of the density matrix).  The
// matrix lives in device memory and is read with wave-uniform addresses.
template <int K, bool NTM>
__global__ __launch_bounds__(kBlock) void k_sv_kq(double2* __restrict__ a, unsigned long long ngroups,
                                                  QSet qs, const double2* __restrict__ M) {
  constexpr int D = 1 << K;
  const unsigned long long g = (unsigned long long)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ngroups) return;
  unsigned long long base = g;
#pragma unroll
  for (int j = 0; j < K; ++j) base = insert0(base, qs.sorted[j]);
  unsigned long long idx[D];
  vd2 v[D];
#pragma unroll
  for (int u = 0; u < D; ++u) {
    unsigned long long o = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
      if ((u >> j) & 1) o += qs.off[j];
    idx[u] = base + o;
    v[u] = gld<NTM>(a + idx[u]);
  }
#pragma unroll
  for (int r = 0; r < D; ++r) {
    vd2 acc = cmul(tov(M[r * D]), v[0]);
#pragma unroll
    for (int c = 1; c < D; ++c) acc = cfma(tov(M[r * D + c]), v[c], acc);
    gst<NTM>(a + idx[r], acc);
  }
}

inline unsigned grid_for(unsigned long long units, int per_block) {
  return (unsigned)((units + per_block - 1) / per_block);
}

}  // namespace

// A dispatch packet holds the grid size in work-items as a 32-bit value, so
// a launch covers at most kMaxItems work-items; larger passes (states above
// 30 qubits at one group per thread) are split into launches that each take
// their first unit u0.  Every launch but the last covers whole blocks.
constexpr unsigned long long kMaxItems = 1ull << 30;

void launch_fill_basis0(hipStream_t s, double2* a, unsigned long long len) {
  const unsigned long long per = kMaxItems * 4;
  for (unsigned long long u0 = 0; u0 < len; u0 += per) {
    const unsigned long long cnt = len - u0 < per ? len - u0 : per;
    hipLaunchKernelGGL(k_fill_basis0<4>, dim3(grid_for(cnt, kBlock * 4)), dim3(kBlock), 0, s, a, u0, len);
  }
}

#define NWQ_LAUNCH_NT(KERNEL, P, units, s, a, ...)                                                          \
  do {                                                                                                      \
    const unsigned long long per_ = kMaxItems * P;                                                          \
    for (unsigned long long u0_ = 0; u0_ < (units); u0_ += per_) {                                          \
      const unsigned long long cnt_ = (units) - u0_ < per_ ? (units) - u0_ : per_;                          \
      if (cfg.nt)                                                                                           \
        hipLaunchKernelGGL((KERNEL<P, true>), dim3(grid_for(cnt_, kBlock * P)), dim3(kBlock), 0, s, a, u0_, \
                           __VA_ARGS__);                                                                    \
      else                                                                                                  \
        hipLaunchKernelGGL((KERNEL<P, false>), dim3(grid_for(cnt_, kBlock * P)), dim3(kBlock), 0, s, a, u0_, \
                           __VA_ARGS__);                                                                    \
    }                                                                                                       \
  } while (0)

#define NWQ_PPT_SWITCH(KERNEL, units, ...)                               \
  switch (cfg.ppt) {                                                     \
    case 1: NWQ_LAUNCH_NT(KERNEL, 1, units, __VA_ARGS__); break;         \
    case 2: NWQ_LAUNCH_NT(KERNEL, 2, units, __VA_ARGS__); break;         \
    case 8: NWQ_LAUNCH_NT(KERNEL, 8, units, __VA_ARGS__); break;         \
    default: NWQ_LAUNCH_NT(KERNEL, 4, units, __VA_ARGS__); break;        \
  }

// Kernels with at most two streams per group also take 16 groups per thread.
#define NWQ_PPT_SWITCH16(KERNEL, units, ...)                             \
  if (cfg.ppt == 16) NWQ_LAUNCH_NT(KERNEL, 16, units, __VA_ARGS__);      \
  else NWQ_PPT_SWITCH(KERNEL, units, __VA_ARGS__)

void launch_sv_1q(hipStream_t s, double2* a, int nbits, int q, const Mat2& m, const LaunchCfg& cfg) {
  const unsigned long long np = 1ull << (nbits - 1);
  NWQ_PPT_SWITCH16(k_sv_1q, np, s, a, np, q, m);
}

void launch_sv_diag(hipStream_t s, double2* a, int nbits, int q0, int q1, const Diag4& d, const LaunchCfg& cfg) {
  const unsigned long long len = 1ull << nbits;
  NWQ_PPT_SWITCH16(k_sv_diag, len, s, a, len, q0, q1, d);
}

void launch_sv_swap1(hipStream_t s, double2* a, int nbits, int q, const LaunchCfg& cfg) {
  const unsigned long long np = 1ull << (nbits - 1);
  NWQ_PPT_SWITCH16(k_sv_swap1, np, s, a, np, q);
}

void launch_sv_swap2(hipStream_t s, double2* a, int nbits, int qa, int qb, unsigned long long offA,
                     unsigned long long offB, const LaunchCfg& cfg) {
  const unsigned long long nq = 1ull << (nbits - 2);
  const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
  NWQ_PPT_SWITCH16(k_sv_swap2, nq, s, a, nq, lo, hi, offA, offB);
}

void launch_sv_2q(hipStream_t s, double2* a, int nbits, int q0, int q1, const Mat4& m, const LaunchCfg& cfg) {
  const unsigned long long nq = 1ull << (nbits - 2);
  const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
  NWQ_PPT_SWITCH(k_sv_2q, nq, s, a, nq, lo, hi, 1ull << q0, 1ull << q1, m);
}

void launch_sv_kq(hipStream_t s, double2* a, int nbits, int k, const int* qubits, const double2* dev_matrix,
                  const LaunchCfg& cfg) {
  QSet qs{};
  int sorted[4];
  for (int j = 0; j < k; ++j) {
    sorted[j] = qubits[j];
    qs.off[j] = 1ull << qubits[j];
  }
  for (int i = 1; i < k; ++i)
    for (int j = i; j > 0 && sorted[j - 1] > sorted[j]; --j) {
      const int t = sorted[j];
      sorted[j] = sorted[j - 1];
      sorted[j - 1] = t;
    }
  for (int j = 0; j < k; ++j) qs.sorted[j] = sorted[j];
  const unsigned long long ng = 1ull << (nbits - k);
  // one group per thread (16 loads in flight at k = 4); only the hint is tunable
  const dim3 grid(grid_for(ng, kBlock));
  if (k == 3) {
    if (cfg.nt) hipLaunchKernelGGL((k_sv_kq<3, true>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
    else hipLaunchKernelGGL((k_sv_kq<3, false>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
  } else {
    if (cfg.nt) hipLaunchKernelGGL((k_sv_kq<4, true>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
    else hipLaunchKernelGGL((k_sv_kq<4, false>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
  }
}

}  // namespace nwq

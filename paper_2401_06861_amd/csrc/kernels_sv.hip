// Streaming gate kernels for gfx950: one pass over the amplitude vector per
// gate.  The vector holds 2^nbits interleaved complex128 entries (nbits = n
// for a state vector, 2n for the row-major vec of a density matrix, whose
// superoperators are applied by the same kernels on (column, row) bit sets).
//
// Every kernel is HBM-bound (<= 4 flop/byte against a ~9.8 flop/byte FP64
// ridge), so the design goals are: 16-byte (dwordx4) loads of whole
// amplitudes, several independent groups per thread for bytes in flight,
// wave-contiguous addressing for targets q >= 6 and cache-line-local
// addressing below, and 64-bit byte offsets only in address arithmetic.
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

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * b + c
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}

// |0...0> (entry 0 = 1, rest 0) written with plain stores (no memset node,
// so the kernel is safe inside captured graphs).
template <int EPT>
__global__ __launch_bounds__(kBlock) void k_fill_basis0(double2* __restrict__ a, unsigned long long len) {
  const unsigned long long start = (unsigned long long)blockIdx.x * (kBlock * EPT) + threadIdx.x;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const unsigned long long i = start + (unsigned long long)j * kBlock;
    if (i < len) a[i] = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
  }
}

// 1-qubit dense gate: for each pair p, i0 = insert0(p, q), i1 = i0 | 2^q,
// (a_i0, a_i1) <- M (a_i0, a_i1).
template <int PPT>
__global__ __launch_bounds__(kBlock) void k_sv_1q(double2* __restrict__ a, unsigned long long npairs,
                                                  int q, Mat2 m) {
  const unsigned long long start = (unsigned long long)blockIdx.x * (kBlock * PPT) + threadIdx.x;
  const unsigned long long off = 1ull << q;
  if (start + (unsigned long long)(PPT - 1) * kBlock < npairs) {
    double2 x0[PPT], x1[PPT];
    unsigned long long i0[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      i0[j] = insert0(start + (unsigned long long)j * kBlock, q);
      x0[j] = a[i0[j]];
      x1[j] = a[i0[j] + off];
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      a[i0[j]] = cfma(m.m[0], x0[j], cmul(m.m[1], x1[j]));
      a[i0[j] + off] = cfma(m.m[2], x0[j], cmul(m.m[3], x1[j]));
    }
  } else {
    for (int j = 0; j < PPT; ++j) {
      const unsigned long long p = start + (unsigned long long)j * kBlock;
      if (p >= npairs) break;
      const unsigned long long i = insert0(p, q);
      const double2 v0 = a[i], v1 = a[i + off];
      a[i] = cfma(m.m[0], v0, cmul(m.m[1], v1));
      a[i + off] = cfma(m.m[2], v0, cmul(m.m[3], v1));
    }
  }
}

__device__ __forceinline__ double2 pick4(const Diag4& d, unsigned u) {
  const double2 lo = (u & 1u) ? d.d[1] : d.d[0];
  const double2 hi = (u & 1u) ? d.d[3] : d.d[2];
  return (u & 2u) ? hi : lo;
}

// Diagonal gate on one or two qubits: a_i <- d[u(i)] a_i, u = bit q0 + 2 bit q1.
template <int EPT>
__global__ __launch_bounds__(kBlock) void k_sv_diag(double2* __restrict__ a, unsigned long long len,
                                                    int q0, int q1, Diag4 d) {
  const unsigned long long start = (unsigned long long)blockIdx.x * (kBlock * EPT) + threadIdx.x;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const unsigned long long i = start + (unsigned long long)j * kBlock;
    if (i < len) {
      unsigned u = (unsigned)((i >> q0) & 1ull);
      if (q1 >= 0) u |= (unsigned)((i >> q1) & 1ull) << 1;
      a[i] = cmul(pick4(d, u), a[i]);
    }
  }
}

// X gate: swap the two members of each pair (no arithmetic).
template <int PPT>
__global__ __launch_bounds__(kBlock) void k_sv_swap1(double2* __restrict__ a, unsigned long long npairs, int q) {
  const unsigned long long start = (unsigned long long)blockIdx.x * (kBlock * PPT) + threadIdx.x;
  const unsigned long long off = 1ull << q;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const unsigned long long p = start + (unsigned long long)j * kBlock;
    if (p < npairs) {
      const unsigned long long i = insert0(p, q);
      const double2 v0 = a[i], v1 = a[i + off];
      a[i] = v1;
      a[i + off] = v0;
    }
  }
}

// Two-qubit permutation that exchanges two members of each quad (CX: the
// control=1 pair; SWAP: |01> <-> |10>).  Only the moved half of the vector
// is read and written.
template <int PPT>
__global__ __launch_bounds__(kBlock) void k_sv_swap2(double2* __restrict__ a2, unsigned long long nquads,
                                                     int qlo, int qhi, unsigned long long offA,
                                                     unsigned long long offB) {
  vd2* __restrict__ a = reinterpret_cast<vd2*>(a2);
  const unsigned long long start = (unsigned long long)blockIdx.x * (kBlock * PPT) + threadIdx.x;
  if (start + (unsigned long long)(PPT - 1) * kBlock < nquads) {
    vd2 va[PPT], vb[PPT];
    unsigned long long b[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      b[j] = insert0(insert0(start + (unsigned long long)j * kBlock, qlo), qhi);
      va[j] = a[b[j] + offA];
      vb[j] = a[b[j] + offB];
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      a[b[j] + offA] = vb[j];
      a[b[j] + offB] = va[j];
    }
  } else {
    for (int j = 0; j < PPT; ++j) {
      const unsigned long long p = start + (unsigned long long)j * kBlock;
      if (p >= nquads) break;
      const unsigned long long base = insert0(insert0(p, qlo), qhi);
      const vd2 x = a[base + offA], y = a[base + offB];
      a[base + offA] = y;
      a[base + offB] = x;
    }
  }
}

// Two-qubit dense gate: quads over the sorted bit pair; member u sits at
// base + bit0(u) 2^{q0} + bit1(u) 2^{q1} (operator order); out = M v.
template <int PPT>
__global__ __launch_bounds__(kBlock) void k_sv_2q(double2* __restrict__ a, unsigned long long nquads,
                                                  int qlo, int qhi, unsigned long long o0,
                                                  unsigned long long o1, Mat4 m) {
  const unsigned long long start = (unsigned long long)blockIdx.x * (kBlock * PPT) + threadIdx.x;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const unsigned long long p = start + (unsigned long long)j * kBlock;
    if (p < nquads) {
      const unsigned long long base = insert0(insert0(p, qlo), qhi);
      const unsigned long long idx[4] = {base, base + o0, base + o1, base + o0 + o1};
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = a[idx[u]];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double2 acc = cmul(m.m[4 * r], v[0]);
#pragma unroll
        for (int c = 1; c < 4; ++c) acc = cfma(m.m[4 * r + c], v[c], acc);
        a[idx[r]] = acc;
      }
    }
  }
}

// k-qubit dense operator (k = 3 or 4; the 16 x 16 case is the fused
// two-qubit gate + channel superoperator of the density matrix).  The
// matrix lives in device memory and is read with wave-uniform addresses.
template <int K>
__global__ __launch_bounds__(kBlock) void k_sv_kq(double2* __restrict__ a, unsigned long long ngroups,
                                                  QSet qs, const double2* __restrict__ M) {
  constexpr int D = 1 << K;
  const unsigned long long g = (unsigned long long)blockIdx.x * kBlock + threadIdx.x;
  if (g >= ngroups) return;
  unsigned long long base = g;
#pragma unroll
  for (int j = 0; j < K; ++j) base = insert0(base, qs.sorted[j]);
  unsigned long long idx[D];
  double2 v[D];
#pragma unroll
  for (int u = 0; u < D; ++u) {
    unsigned long long o = 0;
#pragma unroll
    for (int j = 0; j < K; ++j)
      if ((u >> j) & 1) o += qs.off[j];
    idx[u] = base + o;
    v[u] = a[idx[u]];
  }
#pragma unroll
  for (int r = 0; r < D; ++r) {
    double2 acc = cmul(M[r * D], v[0]);
#pragma unroll
    for (int c = 1; c < D; ++c) acc = cfma(M[r * D + c], v[c], acc);
    a[idx[r]] = acc;
  }
}

inline unsigned grid_for(unsigned long long units, int per_block) {
  return (unsigned)((units + per_block - 1) / per_block);
}

}  // namespace

void launch_fill_basis0(hipStream_t s, double2* a, unsigned long long len) {
  hipLaunchKernelGGL(k_fill_basis0<4>, dim3(grid_for(len, kBlock * 4)), dim3(kBlock), 0, s, a, len);
}

#define NWQ_PPT_SWITCH(ppt, KERNEL, units, ...)                                                  \
  switch (ppt) {                                                                                 \
    case 1: hipLaunchKernelGGL(KERNEL<1>, dim3(grid_for(units, kBlock)), dim3(kBlock), 0, __VA_ARGS__); break;     \
    case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(grid_for(units, kBlock * 2)), dim3(kBlock), 0, __VA_ARGS__); break; \
    case 8: hipLaunchKernelGGL(KERNEL<8>, dim3(grid_for(units, kBlock * 8)), dim3(kBlock), 0, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL(KERNEL<4>, dim3(grid_for(units, kBlock * 4)), dim3(kBlock), 0, __VA_ARGS__); break; \
  }

void launch_sv_1q(hipStream_t s, double2* a, int nbits, int q, const Mat2& m, int ppt) {
  const unsigned long long np = 1ull << (nbits - 1);
  NWQ_PPT_SWITCH(ppt, k_sv_1q, np, s, a, np, q, m);
}

void launch_sv_diag(hipStream_t s, double2* a, int nbits, int q0, int q1, const Diag4& d, int ppt) {
  const unsigned long long len = 1ull << nbits;
  NWQ_PPT_SWITCH(ppt, k_sv_diag, len, s, a, len, q0, q1, d);
}

void launch_sv_swap1(hipStream_t s, double2* a, int nbits, int q, int ppt) {
  const unsigned long long np = 1ull << (nbits - 1);
  NWQ_PPT_SWITCH(ppt, k_sv_swap1, np, s, a, np, q);
}

void launch_sv_swap2(hipStream_t s, double2* a, int nbits, int qa, int qb,
                     unsigned long long offA, unsigned long long offB, int ppt) {
  const unsigned long long nq = 1ull << (nbits - 2);
  const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
  NWQ_PPT_SWITCH(ppt, k_sv_swap2, nq, s, a, nq, lo, hi, offA, offB);
}

void launch_sv_2q(hipStream_t s, double2* a, int nbits, int q0, int q1, const Mat4& m, int ppt) {
  const unsigned long long nq = 1ull << (nbits - 2);
  const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
  NWQ_PPT_SWITCH(ppt, k_sv_2q, nq, s, a, nq, lo, hi, 1ull << q0, 1ull << q1, m);
}

void launch_sv_kq(hipStream_t s, double2* a, int nbits, int k, const int* qubits, const double2* dev_matrix) {
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
  if (k == 3)
    hipLaunchKernelGGL(k_sv_kq<3>, dim3(grid_for(ng, kBlock)), dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
  else
    hipLaunchKernelGGL(k_sv_kq<4>, dim3(grid_for(ng, kBlock)), dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
}

}  // namespace nwq

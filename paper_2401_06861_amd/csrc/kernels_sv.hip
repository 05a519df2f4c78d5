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
#include <type_traits>

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

// Workgroup order of the exchange kernels.  The dispatcher hands consecutive
// workgroups to the chip's 8 XCDs in turn (each XCD with its own L2).  With
// ORD, workgroup i takes block (i mod 8) G/8 + floor(i / 8) of the launch's G
// blocks (G a multiple of 8; the launchers check), so each XCD streams one
// contiguous eighth of the launch instead of every eighth block.
template <bool ORD>
__device__ __forceinline__ unsigned long long wg_block() {
  if constexpr (ORD) return (unsigned long long)((blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3));
  else return blockIdx.x;
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
  if constexpr (PPT == 1) {
    // one path only: when the two paths below coincide the compiler merges their
    // stores and the merged store loses its non-temporal hint
    if (start < npairs) {
      const unsigned long long i = insert0(start, q);
      const vd2 v0 = gld<NTM>(a + i), v1 = gld<NTM>(a + i + off);
      gst<NTM>(a + i, cfma(m0, v0, cmul(m1, v1)));
      gst<NTM>(a + i + off, cfma(m2, v0, cmul(m3, v1)));
    }
    return;
  }
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

// ---------------------------------------------------------------------------
// Lane-exchange kernels for gates whose partner amplitudes sit in the same
// 128-byte line (target bits below 3).  Pair-per-thread addressing there has
// each load instruction touch every line of its span twice (the two members
// of a pair in separate instructions) and runs at about 5.5 TB/s; here every
// load and store is one fully coalesced 1 KiB access per wave (lane l holds
// entry 64 m + l) and the pair partner comes from lane l ^ X through DPP row
// permutations (X = 1, 2, 4, 8) or ds_bpermute (other X).  Valid when the
// length is a multiple of 64 and the gate's bits are lane bits (below 6).
// ---------------------------------------------------------------------------
template <int X>
__device__ __forceinline__ int lane_xor32(int v) {
  // DPP controls: quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E, [3,2,1,0] = 0x1B;
  // row_half_mirror (lane ^ 7 within 8) = 0x141; row_mirror (lane ^ 15 within 16) = 0x140
  if constexpr (X == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
  else if constexpr (X == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
  else if constexpr (X == 4)   // (l ^ 7) ^ 3
    return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true), 0x1B, 0xF, 0xF, true);
  else   // X == 8: (l ^ 15) ^ 7
    return __builtin_amdgcn_mov_dpp(__builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true), 0x141, 0xF, 0xF, true);
}
template <int X>
__device__ __forceinline__ double lane_xor(double d, int src_byte) {
  const long long b = __double_as_longlong(d);
  int lo = (int)(unsigned)(b & 0xffffffffll), hi = (int)(b >> 32);
  if constexpr (X == 0) {   // run-time pattern: src_byte = 4 * (l ^ X)
    lo = __builtin_amdgcn_ds_bpermute(src_byte, lo);
    hi = __builtin_amdgcn_ds_bpermute(src_byte, hi);
  } else {
    lo = lane_xor32<X>(lo);
    hi = lane_xor32<X>(hi);
  }
  return __longlong_as_double(((long long)hi << 32) | (unsigned long long)(unsigned)lo);
}
template <int X>
__device__ __forceinline__ vd2 lane_xor_v(vd2 v, int src_byte) {
  return mk(lane_xor<X>(v.x, src_byte), lane_xor<X>(v.y, src_byte));
}

// 1-qubit dense gate on target q < log2(NB): each thread owns one entry of a
// workgroup's NB contiguous entries (one coalesced load and store per lane)
// and reads its pair partner, entry ^ 2^q, from the workgroup's copy in LDS.
// The thread holding member b of its pair (b = bit q of its index) writes
// M[b][b] own + M[b][1-b] partner.  At n=30 this runs at 6.7-6.8 TB/s on
// targets 0-7 (256 threads) and 6.5 TB/s on target 8 (512 threads), against
// 5.9 TB/s for one pair per thread.
template <int NB, bool NTM, bool ORD>
__global__ __launch_bounds__(NB) void k_sv_1q_xlds(double2* __restrict__ a, unsigned long long u0, int q, Mat2 m) {
  __shared__ vd2 t[NB];
  const unsigned tid = threadIdx.x;
  const unsigned long long i = u0 + wg_block<ORD>() * NB + tid;
  const vd2 v = gld<NTM>(a + i);
  t[tid] = v;
  __syncthreads();
  const vd2 p = t[tid ^ (1u << q)];
  const bool up = (tid >> q) & 1u;
  const vd2 cs = up ? tov(m.m[3]) : tov(m.m[0]), cp = up ? tov(m.m[2]) : tov(m.m[1]);
  gst<NTM>(a + i, cfma(cs, v, cmul(cp, p)));
}

// 1-qubit dense gate on a high target q: a workgroup of NB threads takes H =
// NB / 2 consecutive pairs; its first H threads hold their lower members and
// the other H their upper members (2^q further on), one coalesced entry per
// thread, and each reads its partner from the workgroup's copy in LDS.  With
// the pair-per-thread kernel each thread keeps two streams in flight; here
// each wave streams one run.  At n=30: 6.5-6.7 TB/s on most targets from 9
// up (the best NB varies by target), against 5.8-6.2 for pairs per thread.
template <int NB, bool NTM, bool ORD>
__global__ __launch_bounds__(NB) void k_sv_1q_x2(double2* __restrict__ a, unsigned long long u0, int q, Mat2 m) {
  constexpr unsigned H = NB / 2;
  __shared__ vd2 t[NB];
  const unsigned tid = threadIdx.x;
  const unsigned up = tid / H;
  const unsigned long long p = u0 + wg_block<ORD>() * H + (tid % H);
  const unsigned long long i = insert0(p, q) + ((unsigned long long)up << q);
  const vd2 v = gld<NTM>(a + i);
  t[tid] = v;
  __syncthreads();
  const vd2 w = t[tid ^ H];
  const vd2 cs = up ? tov(m.m[3]) : tov(m.m[0]), cp = up ? tov(m.m[2]) : tov(m.m[1]);
  gst<NTM>(a + i, cfma(cs, v, cmul(cp, w)));
}

// Permutation of lane-bit members (X, CX and SWAP with both bits below 6 and
// the lower below 3): lane l with (l & Q) in {oa, ob} takes lane l ^ X
// (X = oa ^ ob), the others keep their entry.  MASKED: only moving lanes
// store; used when the moved runs are at least 4 entries (64 bytes) long,
// since shorter partial-line writes cost more than writing the lines whole.
template <int X, int EPT, bool NTM, bool MASKED, bool ORD>
__global__ __launch_bounds__(kBlock) void k_sv_perm_lane(double2* __restrict__ a, unsigned long long u0,
                                                         unsigned long long len, int xr, int Q, int oa, int ob) {
  const unsigned long long start = u0 + wg_block<ORD>() * (kBlock * EPT) + threadIdx.x;
  const int l = threadIdx.x & 63;
  const bool mv = (l & Q) == oa || (l & Q) == ob;
  const int src = (l ^ xr) << 2;
  if constexpr (EPT == 1) {   // one path only (see k_sv_1q)
    if (start < len) {
      const vd2 v = gld<NTM>(a + start);
      const vd2 p = lane_xor_v<X>(v, src);
      if constexpr (MASKED) {
        if (mv) gst<NTM>(a + start, p);
      } else {
        gst<NTM>(a + start, mv ? p : v);
      }
    }
    return;
  }
  if (start + (unsigned long long)(EPT - 1) * kBlock < len) {
    vd2 v[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) v[j] = gld<NTM>(a + start + (unsigned long long)j * kBlock);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const vd2 p = lane_xor_v<X>(v[j], src);
      if constexpr (MASKED) {
        if (mv) gst<NTM>(a + start + (unsigned long long)j * kBlock, p);
      } else {
        gst<NTM>(a + start + (unsigned long long)j * kBlock, mv ? p : v[j]);
      }
    }
  } else {
    for (int j = 0; j < EPT; ++j) {
      const unsigned long long i = start + (unsigned long long)j * kBlock;
      if (i >= len) break;
      const vd2 v = gld<NTM>(a + i);
      const vd2 p = lane_xor_v<X>(v, src);
      if constexpr (MASKED) {
        if (mv) gst<NTM>(a + i, p);
      } else {
        gst<NTM>(a + i, mv ? p : v);
      }
    }
  }
}

// Dense 4x4 with one bit L < 3 (a lane bit) and the other H >= 6 (DM
// superoperator of a 1q gate on a low qubit: bits q and q + n).  A lane holds
// the two entries of its index with bit H = 0 and 1 (two coalesced streams);
// the other two members of each quad sit in lane l ^ 2^L.  Member u of a quad
// has bit0(u) on q0 and bit1(u) on q1 (operator order); LOW_IS_Q0 says which
// of them is L.  Each lane writes its own two entries, rows u(bl, h), from
// eight coefficients chosen once per thread by its bit bl.
template <int L, bool LOW_IS_Q0, int EPT, bool NTM>
__global__ __launch_bounds__(kBlock) void k_sv_2q_lane(double2* __restrict__ a, unsigned long long u0,
                                                       unsigned long long nhalf, int H, Mat4 m) {
  const unsigned long long start = u0 + (unsigned long long)blockIdx.x * (kBlock * EPT) + threadIdx.x;
  const unsigned long long off = 1ull << H;
  const int bl = (threadIdx.x >> L) & 1;
  auto u = [&](int b, int h) { return LOW_IS_Q0 ? (b + 2 * h) : (h + 2 * b); };
  // c[h][h2][0]: coefficient of own entry h2, c[h][h2][1]: of the partner's entry h2, for output h
  vd2 c[2][2][2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      c[h][h2][0] = bl ? tov(m.m[4 * u(1, h) + u(1, h2)]) : tov(m.m[4 * u(0, h) + u(0, h2)]);
      c[h][h2][1] = bl ? tov(m.m[4 * u(1, h) + u(0, h2)]) : tov(m.m[4 * u(0, h) + u(1, h2)]);
    }
  auto out = [&](int h, vd2 e0, vd2 e1, vd2 p0, vd2 p1) {
    return cfma(c[h][0][0], e0, cfma(c[h][1][0], e1, cfma(c[h][0][1], p0, cmul(c[h][1][1], p1))));
  };
  if constexpr (EPT == 1) {   // one path only (see k_sv_1q)
    if (start < nhalf) {
      const unsigned long long i = insert0(start, H);
      const vd2 e0 = gld<NTM>(a + i), e1 = gld<NTM>(a + i + off);
      const vd2 p0 = lane_xor_v<(1 << L)>(e0, 0), p1 = lane_xor_v<(1 << L)>(e1, 0);
      gst<NTM>(a + i, out(0, e0, e1, p0, p1));
      gst<NTM>(a + i + off, out(1, e0, e1, p0, p1));
    }
    return;
  }
  if (start + (unsigned long long)(EPT - 1) * kBlock < nhalf) {
    vd2 e0[EPT], e1[EPT];
    unsigned long long i0[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      i0[j] = insert0(start + (unsigned long long)j * kBlock, H);
      e0[j] = gld<NTM>(a + i0[j]);
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) e1[j] = gld<NTM>(a + i0[j] + off);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const vd2 p0 = lane_xor_v<(1 << L)>(e0[j], 0), p1 = lane_xor_v<(1 << L)>(e1[j], 0);
      gst<NTM>(a + i0[j], out(0, e0[j], e1[j], p0, p1));
      gst<NTM>(a + i0[j] + off, out(1, e0[j], e1[j], p0, p1));
    }
  } else {
    // nhalf is a multiple of 64: a wave is either wholly inside or wholly past the end
    for (int j = 0; j < EPT; ++j) {
      const unsigned long long p = start + (unsigned long long)j * kBlock;
      if (p >= nhalf) break;
      const unsigned long long i = insert0(p, H);
      const vd2 e0 = gld<NTM>(a + i), e1 = gld<NTM>(a + i + off);
      const vd2 p0 = lane_xor_v<(1 << L)>(e0, 0), p1 = lane_xor_v<(1 << L)>(e1, 0);
      gst<NTM>(a + i, out(0, e0, e1, p0, p1));
      gst<NTM>(a + i + off, out(1, e0, e1, p0, p1));
    }
  }
}

// Diagonal gate on one or two qubits: a_i <- d[u(i)] a_i, u = bit q0 + 2 bit q1
// (q1 < 0: one qubit).  Entries are chosen with selects, not an indexed load.
template <int EPT, bool NTM, bool ORD = false>
__global__ __launch_bounds__(kBlock) void k_sv_diag(double2* __restrict__ a, unsigned long long u0, unsigned long long len,
                                                    int q0, int q1, Diag4 d) {
  const unsigned long long start = u0 + wg_block<ORD>() * (kBlock * EPT) + threadIdx.x;
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

// Permutations (X, CX, SWAP) in the split-workgroup layout: the first half
// of a workgroup reads the member at offA of each of NB/2 consecutive groups,
// the second half the member at offB; once every member has been read (the
// barrier) each thread writes its value to its partner's place.  One-qubit
// groups (X) pass qhi = -1.
template <int NB, bool NTM, bool ORD>
__global__ __launch_bounds__(NB) void k_sv_swap_x2(double2* __restrict__ a, unsigned long long u0, int qlo, int qhi,
                                                   unsigned long long offA, unsigned long long offB) {
  constexpr unsigned H = NB / 2;
  const unsigned tid = threadIdx.x;
  const bool up = tid >= H;
  const unsigned long long p = u0 + wg_block<ORD>() * H + (tid % H);
  unsigned long long b = insert0(p, qlo);
  if (qhi >= 0) b = insert0(b, qhi);
  const vd2 v = gld<NTM>(a + b + (up ? offB : offA));
  __syncthreads();
  gst<NTM>(a + b + (up ? offA : offB), v);
}

// Dense 4x4 on bits (q0, q1) in the split-workgroup layout: a workgroup of
// NB threads takes H = NB / 4 consecutive quads, quarter u of its threads
// holding member u (bit0(u) on q0, bit1(u) on q1) of each, one coalesced
// entry per thread.  After one barrier each thread forms row u of M times its
// quad, read from the workgroup's copy in LDS.  H is a multiple of 64, so a
// wave lies in one quarter and its row of M is uniform.
template <int NB, bool NTM, bool ORD>
__global__ __launch_bounds__(NB) void k_sv_2q_x4(double2* __restrict__ a, unsigned long long u0, int lo, int hi,
                                                 unsigned long long o0, unsigned long long o1, Mat4 m) {
  constexpr unsigned H = NB / 4;
  static_assert(H % 64 == 0, "a wave must lie in one quarter");
  __shared__ vd2 t[NB];
  const unsigned tid = threadIdx.x, r = tid % H;
  const unsigned u = __builtin_amdgcn_readfirstlane(tid / H);
  const unsigned long long p = u0 + wg_block<ORD>() * H + r;
  const unsigned long long i = insert0(insert0(p, lo), hi) + ((u & 1u) ? o0 : 0ull) + ((u & 2u) ? o1 : 0ull);
  const vd2 v = gld<NTM>(a + i);
  t[tid] = v;
  __syncthreads();
  // row u picked by value (a pointer into the argument would copy it to scratch)
  auto coef = [&](int c) {
    return tov(u == 0 ? m.m[c] : (u == 1 ? m.m[4 + c] : (u == 2 ? m.m[8 + c] : m.m[12 + c])));
  };
  vd2 acc = cmul(coef(0), t[r]);
  acc = cfma(coef(1), t[H + r], acc);
  acc = cfma(coef(2), t[2 * H + r], acc);
  acc = cfma(coef(3), t[3 * H + r], acc);
  gst<NTM>(a + i, acc);
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

// Row r of a 16 x 16 with the pattern of a Pauli channel after a diagonal
// two-qubit gate, on the DM entries (q0, q1, q0 + n, q1 + n) of one group
// (operator index u = c0 + 2 c1 + 4 r0 + 8 r1): an entry whose row and column
// bits differ on either qubit (a coherence) is only scaled, by M[u]; the four
// populations u = 0, 5, 10, 15 mix through the 4 x 4 M[16 + 4 i + j] (rows
// and columns 5i, 5j).  x is the group (a register array or an LDS view).
template <typename X>
__device__ __forceinline__ vd2 kq_pauli_row(const double2* __restrict__ M, int r, const X& x) {
  if (r % 5 != 0) return cmul(tov(M[r]), x[r]);
  const int i = r / 5;
  vd2 acc = cmul(tov(M[16 + 4 * i]), x[0]);
#pragma unroll
  for (int j = 1; j < 4; ++j) acc = cfma(tov(M[16 + 4 * i + j]), x[5 * j], acc);
  return acc;
}

// k-qubit dense operator (k = 3 or 4; the 16 x 16 case is the fused
// two-qubit gate + channel superoperator of the density matrix).  The
// matrix lives in device memory and is read with wave-uniform addresses.
template <int K, bool NTM, bool PAULI = false>
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
  if constexpr (PAULI) {
#pragma unroll
    for (int r = 0; r < D; ++r) gst<NTM>(a + idx[r], kq_pauli_row(M, r, v));
    return;
  }
#pragma unroll
  for (int r = 0; r < D; ++r) {
    vd2 acc = cmul(tov(M[r * D]), v[0]);
#pragma unroll
    for (int c = 1; c < D; ++c) acc = cfma(tov(M[r * D + c]), v[c], acc);
    gst<NTM>(a + idx[r], acc);
  }
}

// 16 x 16 operator in the split-workgroup layout: a workgroup takes 64
// consecutive groups; member u (operator order) of each sits in the run of 64
// entries that wave u mod W loads (W = 16 / MPT waves, MPT members per
// thread), one coalesced entry per load.  After one barrier each thread forms
// rows u of M (uniform per wave: scalar loads) times its group, read from the
// workgroup's copy in LDS; with MPT = 2 each LDS read serves two rows.
template <int MPT, bool NTM, bool ORD, bool PAULI = false>
__global__ __launch_bounds__(1024 / MPT) void k_sv_kq4_x16(double2* __restrict__ a, unsigned long long g0, QSet qs,
                                                           const double2* __restrict__ M) {
  constexpr unsigned W = 16 / MPT;
  __shared__ vd2 t[1024];
  const unsigned tid = threadIdx.x, r = tid & 63u;
  const unsigned w = __builtin_amdgcn_readfirstlane(tid >> 6);
  unsigned long long base = g0 + wg_block<ORD>() * 64 + r;
#pragma unroll
  for (int j = 0; j < 4; ++j) base = insert0(base, qs.sorted[j]);
  unsigned long long i[MPT];
  vd2 acc[MPT];
#pragma unroll
  for (int mi = 0; mi < MPT; ++mi) {
    const unsigned u = w + mi * W;
    unsigned long long o = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if ((u >> j) & 1u) o += qs.off[j];
    i[mi] = base + o;
    acc[mi] = gld<NTM>(a + i[mi]);
  }
#pragma unroll
  for (int mi = 0; mi < MPT; ++mi) t[(w + mi * W) * 64 + r] = acc[mi];
  __syncthreads();
  if constexpr (PAULI) {
    // a coherence row needs only its own entry; a population row reads the
    // other three populations of its group from LDS
    struct View {
      const vd2* t;
      unsigned r;
      __device__ vd2 operator[](int u) const { return t[64 * u + r]; }
    } view{t, r};
#pragma unroll
    for (int mi = 0; mi < MPT; ++mi) {
      const unsigned u = w + mi * W;
      acc[mi] = u % 5u != 0u ? cmul(tov(M[u]), acc[mi]) : kq_pauli_row(M, (int)u, view);
    }
#pragma unroll
    for (int mi = 0; mi < MPT; ++mi) gst<NTM>(a + i[mi], acc[mi]);
    return;
  }
  const vd2 x0 = t[r];
#pragma unroll
  for (int mi = 0; mi < MPT; ++mi) acc[mi] = cmul(tov(M[16 * (w + mi * W)]), x0);
#pragma unroll
  for (int c = 1; c < 16; ++c) {
    const vd2 x = t[64 * c + r];
#pragma unroll
    for (int mi = 0; mi < MPT; ++mi) acc[mi] = cfma(tov(M[16 * (w + mi * W) + c]), x, acc[mi]);
  }
#pragma unroll
  for (int mi = 0; mi < MPT; ++mi) gst<NTM>(a + i[mi], acc[mi]);
}

// 16 x 16 operator whose two lower bits s0 < s1 lie inside a 256-entry run
// (s0 < 3, s1 < 8) and whose two upper bits s2 < s3 (>= 8) select runs: the
// noisy two-qubit DM superoperator on low qubits.  One-group-per-thread
// addressing there reads 16- to 64-byte pieces of every line in separate
// instructions (4.3 TB/s at qubits (0, 1)).  Here a workgroup stages 16 whole
// runs (4 run quads x the 4 combinations of s2, s3; 64 KiB) through LDS with
// coalesced 4 KiB loads and stores; each thread then applies the operator to
// one group read from LDS.  LDS entry e is stored at e ^ (((e >> swa) ^
// (e >> swb)) & 7) (swb = 0: no second term), an XOR swizzle within aligned
// 8-entry groups picked per (s0, s1) so that every 8 lanes of a group read hit
// distinct 16-byte bank groups.
struct KqStaged {
  int h0, h1;           // s2 - 8, s3 - 8
  int s0, s1;           // the lower bits
  int swa, swb;         // swizzle shifts
  int idx_off[16];      // member u (operator order): 256 * (run bits of u) + (bits of u at s0, s1)
};
__device__ __forceinline__ unsigned kq_swz(unsigned e, int a, int b) {
  return e ^ (((e >> a) ^ (b ? (e >> b) : 0u)) & 7u);
}
template <bool NTM, bool PAULI = false>
__global__ __launch_bounds__(kBlock) void k_sv_kq4_staged(double2* __restrict__ a, KqStaged ks,
                                                          const double2* __restrict__ M) {
  __shared__ vd2 t[16 * 256];
  const unsigned tid = threadIdx.x;
  // run of staged slab i = 4 rq + hc: run quad 4 blockIdx + rq, combination hc of (s2, s3)
  auto run_of = [&](int i) {
    unsigned long long q = (unsigned long long)blockIdx.x * 4 + (unsigned)(i >> 2);
    q = insert0(insert0(q, ks.h0), ks.h1);
    return q | ((unsigned long long)(i & 1) << ks.h0) | ((unsigned long long)((i >> 1) & 1) << ks.h1);
  };
  {
    vd2 r[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) r[i] = gld<NTM>(a + (run_of(i) << 8) + tid);
#pragma unroll
    for (int i = 0; i < 16; ++i) t[kq_swz((unsigned)i * 256u + tid, ks.swa, ks.swb)] = r[i];
  }
  __syncthreads();
  {
    const unsigned rq = tid >> 6, lam = tid & 63u;
    const unsigned base = rq * 1024u + (unsigned)insert0(insert0(lam, ks.s0), ks.s1);
    vd2 v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = t[kq_swz(base + (unsigned)ks.idx_off[u], ks.swa, ks.swb)];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      vd2 acc;
      if constexpr (PAULI) {
        acc = kq_pauli_row(M, r, v);
      } else {
        acc = cmul(tov(M[r * 16]), v[0]);
#pragma unroll
        for (int c = 1; c < 16; ++c) acc = cfma(tov(M[r * 16 + c]), v[c], acc);
      }
      t[kq_swz(base + (unsigned)ks.idx_off[r], ks.swa, ks.swb)] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) gst<NTM>(a + (run_of(i) << 8) + tid, t[kq_swz((unsigned)i * 256u + tid, ks.swa, ks.swb)]);
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
      if (cfg.nt & 1)                                                                                       \
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

// Lane-exchange launches: units are entries; the entries per thread (1, 2 or
// 4) come from the tuned groups per thread (8 and 16 map to 4).
namespace {
inline int lane_ept(const LaunchCfg& cfg) {
  if (cfg.ppt >= 32) return 1;   // split-workgroup shapes: one entry per thread
  return cfg.ppt >= 4 ? 4 : (cfg.ppt == 2 ? 2 : 1);
}

// Calls f(NT, ORD) with the hint and the workgroup order as compile-time
// booleans (std::true_type / std::false_type).
template <class F>
void with_hint_order(bool nt, bool ord, F&& f) {
  if (nt) {
    if (ord) f(std::true_type{}, std::true_type{});
    else f(std::true_type{}, std::false_type{});
  } else {
    if (ord) f(std::false_type{}, std::true_type{});
    else f(std::false_type{}, std::false_type{});
  }
}
// XCD-contiguous order when the flags ask for it and the grid splits into 8 equal parts
inline bool use_order(int flags, const dim3& grid) { return (flags & 2) && grid.x % 8u == 0; }

template <int NB>
void launch_1q_xlds(hipStream_t s, double2* a, unsigned long long len, int q, const Mat2& m, int flags) {
  for (unsigned long long u0 = 0; u0 < len; u0 += kMaxItems) {
    const unsigned long long cnt = len - u0 < kMaxItems ? len - u0 : kMaxItems;   // whole workgroups
    const dim3 grid((unsigned)(cnt / NB));
    with_hint_order(flags & 1, use_order(flags, grid), [&](auto nt, auto ord) {
      hipLaunchKernelGGL((k_sv_1q_xlds<NB, decltype(nt)::value, decltype(ord)::value>), grid, dim3(NB), 0, s, a, u0,
                         q, m);
    });
  }
}

template <int NB>
void launch_1q_x2(hipStream_t s, double2* a, unsigned long long npairs, int q, const Mat2& m, int flags) {
  const unsigned long long per = kMaxItems / 2;   // pairs per launch (two threads each)
  for (unsigned long long u0 = 0; u0 < npairs; u0 += per) {
    const unsigned long long cnt = npairs - u0 < per ? npairs - u0 : per;   // whole workgroups
    const dim3 grid((unsigned)(cnt / (NB / 2)));
    with_hint_order(flags & 1, use_order(flags, grid), [&](auto nt, auto ord) {
      hipLaunchKernelGGL((k_sv_1q_x2<NB, decltype(nt)::value, decltype(ord)::value>), grid, dim3(NB), 0, s, a, u0, q,
                         m);
    });
  }
}

template <int NB>
void launch_swap_x2(hipStream_t s, double2* a, unsigned long long ngroups, int qlo, int qhi, unsigned long long offA,
                    unsigned long long offB, int flags) {
  const unsigned long long per = kMaxItems / 2;   // groups per launch (two threads each)
  for (unsigned long long u0 = 0; u0 < ngroups; u0 += per) {
    const unsigned long long cnt = ngroups - u0 < per ? ngroups - u0 : per;   // whole workgroups
    const dim3 grid((unsigned)(cnt / (NB / 2)));
    with_hint_order(flags & 1, use_order(flags, grid), [&](auto nt, auto ord) {
      hipLaunchKernelGGL((k_sv_swap_x2<NB, decltype(nt)::value, decltype(ord)::value>), grid, dim3(NB), 0, s, a, u0,
                         qlo, qhi, offA, offB);
    });
  }
}
// shapes 32 / 64 / 128 of the permutation class: split workgroups of 256 / 512 / 1024 threads
void launch_swap_x2_cfg(hipStream_t s, double2* a, unsigned long long ngroups, int qlo, int qhi,
                        unsigned long long offA, unsigned long long offB, const LaunchCfg& cfg) {
  if (cfg.ppt == 32) launch_swap_x2<256>(s, a, ngroups, qlo, qhi, offA, offB, cfg.nt);
  else if (cfg.ppt == 64) launch_swap_x2<512>(s, a, ngroups, qlo, qhi, offA, offB, cfg.nt);
  else launch_swap_x2<1024>(s, a, ngroups, qlo, qhi, offA, offB, cfg.nt);
}

template <int NB>
void launch_2q_x4(hipStream_t s, double2* a, unsigned long long nquads, int lo, int hi, unsigned long long o0,
                  unsigned long long o1, const Mat4& m, int flags) {
  const unsigned long long per = kMaxItems / 4;   // quads per launch (four threads each)
  for (unsigned long long u0 = 0; u0 < nquads; u0 += per) {
    const unsigned long long cnt = nquads - u0 < per ? nquads - u0 : per;   // whole workgroups
    const dim3 grid((unsigned)(cnt / (NB / 4)));
    with_hint_order(flags & 1, use_order(flags, grid), [&](auto nt, auto ord) {
      hipLaunchKernelGGL((k_sv_2q_x4<NB, decltype(nt)::value, decltype(ord)::value>), grid, dim3(NB), 0, s, a, u0, lo,
                         hi, o0, o1, m);
    });
  }
}

template <int X, int E, bool MASKED>
void launch_perm_lane_e(hipStream_t s, double2* a, unsigned long long len, int xr, int Q, int oa, int ob, int flags) {
  const unsigned long long per = kMaxItems * E;
  for (unsigned long long u0 = 0; u0 < len; u0 += per) {
    const unsigned long long cnt = len - u0 < per ? len - u0 : per;
    const dim3 grid(grid_for(cnt, kBlock * E));
    // the ordered variant exists for one entry per thread (the split-workgroup shapes)
    const bool ord = E == 1 && use_order(flags, grid);
    with_hint_order(flags & 1, ord, [&](auto nt, auto o) {
      constexpr bool O = decltype(o)::value && E == 1;
      hipLaunchKernelGGL((k_sv_perm_lane<X, E, decltype(nt)::value, MASKED, O>), grid, dim3(kBlock), 0, s, a, u0, len,
                         xr, Q, oa, ob);
    });
  }
}
template <int X, bool MASKED>
void launch_perm_lane_x(hipStream_t s, double2* a, unsigned long long len, int xr, int Q, int oa, int ob,
                        const LaunchCfg& cfg) {
  switch (lane_ept(cfg)) {
    case 1: launch_perm_lane_e<X, 1, MASKED>(s, a, len, xr, Q, oa, ob, cfg.nt); break;
    case 2: launch_perm_lane_e<X, 2, MASKED>(s, a, len, xr, Q, oa, ob, cfg.nt); break;
    default: launch_perm_lane_e<X, 4, MASKED>(s, a, len, xr, Q, oa, ob, cfg.nt); break;
  }
}
// lane l with (l & Q) in {oa, ob} takes lane l ^ (oa ^ ob); every bit involved is below 6
template <bool MASKED>
void launch_perm_lane_m(hipStream_t s, double2* a, unsigned long long len, int Q, int oa, int ob, const LaunchCfg& cfg) {
  const int x = oa ^ ob;
  switch (x) {
    case 1: launch_perm_lane_x<1, MASKED>(s, a, len, x, Q, oa, ob, cfg); break;
    case 2: launch_perm_lane_x<2, MASKED>(s, a, len, x, Q, oa, ob, cfg); break;
    case 4: launch_perm_lane_x<4, MASKED>(s, a, len, x, Q, oa, ob, cfg); break;
    case 8: launch_perm_lane_x<8, MASKED>(s, a, len, x, Q, oa, ob, cfg); break;
    default: launch_perm_lane_x<0, MASKED>(s, a, len, x, Q, oa, ob, cfg); break;
  }
}
void launch_perm_lane(hipStream_t s, double2* a, unsigned long long len, int Q, int oa, int ob, const LaunchCfg& cfg) {
  // moving lanes come in runs of 2^b, b the lowest lane bit that changes whether a lane moves
  int b = 6;
  for (int l = 0; l < 64; ++l)
    for (int t = 0; t < b; ++t) {
      const int k = l ^ (1 << t);
      const bool ml = (l & Q) == oa || (l & Q) == ob, mk = (k & Q) == oa || (k & Q) == ob;
      if (ml != mk) b = t;
    }
  if (b >= 2) launch_perm_lane_m<true>(s, a, len, Q, oa, ob, cfg);
  else launch_perm_lane_m<false>(s, a, len, Q, oa, ob, cfg);
}
// the lane kernels need whole 256-entry blocks (lane bits = index bits 0..5)
constexpr int kLaneMinBits = 8;
}  // namespace

void launch_sv_1q(hipStream_t s, double2* a, int nbits, int q, const Mat2& m, const LaunchCfg& cfg) {
  // targets 0-8: LDS partner exchange (only the hint of the tuned shape applies)
  if (q < 8 && nbits >= 8) {
    launch_1q_xlds<256>(s, a, 1ull << nbits, q, m, cfg.nt);
    return;
  }
  if (q == 8 && nbits >= 9) {
    launch_1q_xlds<512>(s, a, 1ull << nbits, q, m, cfg.nt);
    return;
  }
  // shapes 32 / 64 / 128: split-workgroup exchange with 256 / 512 / 1024 threads
  if (cfg.ppt >= 32 && nbits >= 10) {
    const unsigned long long np = 1ull << (nbits - 1);
    if (cfg.ppt == 32) launch_1q_x2<256>(s, a, np, q, m, cfg.nt);
    else if (cfg.ppt == 64) launch_1q_x2<512>(s, a, np, q, m, cfg.nt);
    else launch_1q_x2<1024>(s, a, np, q, m, cfg.nt);
    return;
  }
  const unsigned long long np = 1ull << (nbits - 1);
  NWQ_PPT_SWITCH16(k_sv_1q, np, s, a, np, q, m);
}

void launch_sv_diag(hipStream_t s, double2* a, int nbits, int q0, int q1, const Diag4& d, const LaunchCfg& cfg) {
  const unsigned long long len = 1ull << nbits;
  if (cfg.ppt == 1 && (cfg.nt & 2)) {   // one entry per thread in XCD-contiguous order
    for (unsigned long long u0 = 0; u0 < len; u0 += kMaxItems) {
      const unsigned long long cnt = len - u0 < kMaxItems ? len - u0 : kMaxItems;
      const dim3 grid(grid_for(cnt, kBlock));
      with_hint_order(cfg.nt & 1, use_order(cfg.nt, grid), [&](auto nt, auto ord) {
        hipLaunchKernelGGL((k_sv_diag<1, decltype(nt)::value, decltype(ord)::value>), grid, dim3(kBlock), 0, s, a, u0,
                           len, q0, q1, d);
      });
    }
    return;
  }
  NWQ_PPT_SWITCH16(k_sv_diag, len, s, a, len, q0, q1, d);
}

void launch_sv_swap1(hipStream_t s, double2* a, int nbits, int q, const LaunchCfg& cfg) {
  if (q < 3 && nbits >= kLaneMinBits) {   // every lane takes lane ^ 2^q
    launch_perm_lane(s, a, 1ull << nbits, 1 << q, 0, 1 << q, cfg);
    return;
  }
  const unsigned long long np = 1ull << (nbits - 1);
  if (cfg.ppt >= 32 && nbits >= 10) {   // 512 pairs fill the largest split workgroup
    launch_swap_x2_cfg(s, a, np, q, -1, 0, 1ull << q, cfg);
    return;
  }
  NWQ_PPT_SWITCH16(k_sv_swap1, np, s, a, np, q);
}

void launch_sv_swap2(hipStream_t s, double2* a, int nbits, int qa, int qb, unsigned long long offA,
                     unsigned long long offB, const LaunchCfg& cfg) {
  const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
  if (lo < 3 && hi < 6 && nbits >= kLaneMinBits) {
    launch_perm_lane(s, a, 1ull << nbits, (1 << qa) | (1 << qb), (int)offA, (int)offB, cfg);
    return;
  }
  const unsigned long long nq = 1ull << (nbits - 2);
  if (cfg.ppt >= 32 && nbits >= 11) {   // 512 quads fill the largest split workgroup
    launch_swap_x2_cfg(s, a, nq, lo, hi, offA, offB, cfg);
    return;
  }
  NWQ_PPT_SWITCH16(k_sv_swap2, nq, s, a, nq, lo, hi, offA, offB);
}

namespace {
template <int L, bool LQ0, int E>
void launch_2q_lane_e(hipStream_t s, double2* a, unsigned long long nhalf, int H, const Mat4& m, bool nt) {
  const unsigned long long per = kMaxItems * E;
  for (unsigned long long u0 = 0; u0 < nhalf; u0 += per) {
    const unsigned long long cnt = nhalf - u0 < per ? nhalf - u0 : per;
    const dim3 grid(grid_for(cnt, kBlock * E));
    if (nt) hipLaunchKernelGGL((k_sv_2q_lane<L, LQ0, E, true>), grid, dim3(kBlock), 0, s, a, u0, nhalf, H, m);
    else hipLaunchKernelGGL((k_sv_2q_lane<L, LQ0, E, false>), grid, dim3(kBlock), 0, s, a, u0, nhalf, H, m);
  }
}
template <int L, bool LQ0>
void launch_2q_lane_l(hipStream_t s, double2* a, unsigned long long nhalf, int H, const Mat4& m, const LaunchCfg& cfg) {
  switch (lane_ept(cfg)) {
    case 1: launch_2q_lane_e<L, LQ0, 1>(s, a, nhalf, H, m, (cfg.nt & 1) != 0); break;
    case 2: launch_2q_lane_e<L, LQ0, 2>(s, a, nhalf, H, m, (cfg.nt & 1) != 0); break;
    default: launch_2q_lane_e<L, LQ0, 4>(s, a, nhalf, H, m, (cfg.nt & 1) != 0); break;
  }
}
template <bool LQ0>
void launch_2q_lane(hipStream_t s, double2* a, unsigned long long nhalf, int L, int H, const Mat4& m,
                    const LaunchCfg& cfg) {
  if (L == 0) launch_2q_lane_l<0, LQ0>(s, a, nhalf, H, m, cfg);
  else if (L == 1) launch_2q_lane_l<1, LQ0>(s, a, nhalf, H, m, cfg);
  else launch_2q_lane_l<2, LQ0>(s, a, nhalf, H, m, cfg);
}
}  // namespace

void launch_sv_2q(hipStream_t s, double2* a, int nbits, int q0, int q1, const Mat4& m, const LaunchCfg& cfg) {
  const unsigned long long nq = 1ull << (nbits - 2);
  const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
  if (lo < 3 && hi >= 6 && nbits >= kLaneMinBits) {   // lane bit lo, stream bit hi
    const unsigned long long nhalf = 1ull << (nbits - 1);
    if (q0 == lo) launch_2q_lane<true>(s, a, nhalf, lo, hi, m, cfg);
    else launch_2q_lane<false>(s, a, nhalf, lo, hi, m, cfg);
    return;
  }
  // shapes 32 / 64 / 128: split workgroups of 256 / 512 / 1024 threads (256 quads fill the largest)
  if (cfg.ppt >= 32 && nbits >= 10) {
    if (cfg.ppt == 32) launch_2q_x4<256>(s, a, nq, lo, hi, 1ull << q0, 1ull << q1, m, cfg.nt);
    else if (cfg.ppt == 64) launch_2q_x4<512>(s, a, nq, lo, hi, 1ull << q0, 1ull << q1, m, cfg.nt);
    else launch_2q_x4<1024>(s, a, nq, lo, hi, 1ull << q0, 1ull << q1, m, cfg.nt);
    return;
  }
  NWQ_PPT_SWITCH(k_sv_2q, nq, s, a, nq, lo, hi, 1ull << q0, 1ull << q1, m);
}

namespace {
// Swizzle shifts (a in 1..7, b in 0..7, b = 0: none) under which the reads of
// every 8 consecutive lanes of the staged 16 x 16 kernel hit distinct 16-byte
// slots of a 128-byte LDS row (checked for each member pattern of the lower
// bits); the first conflict-free pair is taken, else the one with the fewest
// conflicts.
void kq_pick_swizzle(KqStaged& ks) {
  auto ins = [](unsigned p, int q) { return ((p >> q) << (q + 1)) | (p & ((1u << q) - 1u)); };
  int best = 1 << 30;
  for (int sa = 1; sa < 8; ++sa)
    for (int sb = 0; sb < 8; ++sb) {
      int cost = 0;
      for (unsigned g0 = 0; g0 < 64; g0 += 8)
        for (unsigned low = 0; low < 4; ++low) {
          int cnt[8] = {0};
          for (unsigned l = g0; l < g0 + 8; ++l) {
            const unsigned e = ins(ins(l, ks.s0), ks.s1) | ((low & 1u) << ks.s0) | ((low >> 1) << ks.s1);
            const unsigned f = e ^ (((e >> sa) ^ (sb ? (e >> sb) : 0u)) & 7u);
            ++cnt[f & 7u];
          }
          for (int x = 0; x < 8; ++x) cost += cnt[x] > 1 ? cnt[x] - 1 : 0;
        }
      if (cost < best) {
        best = cost;
        ks.swa = sa;
        ks.swb = sb;
      }
      if (best == 0) return;
    }
}
}  // namespace

void launch_sv_kq(hipStream_t s, double2* a, int nbits, int k, const int* qubits, const double2* dev_matrix,
                  const LaunchCfg& cfg, bool pauli) {
  pauli = pauli && k == 4;
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
  // two lower bits in a 256-entry run (the lowest below 3): the LDS-staged
  // kernel, unless the shape picks a split-workgroup kernel (64, 128), which
  // the tuner compares with it bit by bit
  if (k == 4 && sorted[0] < 3 && sorted[1] < 8 && sorted[2] >= 8 && nbits >= 12 && cfg.ppt != 64 && cfg.ppt != 128) {
    KqStaged ks{};
    ks.h0 = sorted[2] - 8;
    ks.h1 = sorted[3] - 8;
    ks.s0 = sorted[0];
    ks.s1 = sorted[1];
    for (int u = 0; u < 16; ++u) {
      int o = 0;
      for (int j = 0; j < 4; ++j) {
        if (!((u >> j) & 1)) continue;
        if (qubits[j] < 8) o |= 1 << qubits[j];
        else o |= (qubits[j] == sorted[2] ? 1 : 2) << 8;
      }
      ks.idx_off[u] = o;
    }
    kq_pick_swizzle(ks);
    const dim3 grid((unsigned)(1ull << (nbits - 12)));   // 16 runs of 256 entries per workgroup
    if (pauli) {
      if (cfg.nt & 1) hipLaunchKernelGGL((k_sv_kq4_staged<true, true>), grid, dim3(kBlock), 0, s, a, ks, dev_matrix);
      else hipLaunchKernelGGL((k_sv_kq4_staged<false, true>), grid, dim3(kBlock), 0, s, a, ks, dev_matrix);
    } else {
      if (cfg.nt & 1) hipLaunchKernelGGL((k_sv_kq4_staged<true, false>), grid, dim3(kBlock), 0, s, a, ks, dev_matrix);
      else hipLaunchKernelGGL((k_sv_kq4_staged<false, false>), grid, dim3(kBlock), 0, s, a, ks, dev_matrix);
    }
    return;
  }
  // shapes 128 / 64: split workgroups of 1024 threads (one member each) or 512
  // threads (two members each), 64 groups per workgroup
  if (k == 4 && (cfg.ppt == 128 || cfg.ppt == 64) && nbits >= 10) {
    const unsigned long long per = kMaxItems / 16;   // groups per launch (at most sixteen threads each)
    for (unsigned long long g0 = 0; g0 < ng; g0 += per) {
      const unsigned long long cnt = ng - g0 < per ? ng - g0 : per;   // whole workgroups
      const dim3 grid((unsigned)(cnt / 64));
      with_hint_order(cfg.nt & 1, use_order(cfg.nt, grid), [&](auto nt, auto ord) {
        constexpr bool NT = decltype(nt)::value, ORD = decltype(ord)::value;
        if (cfg.ppt == 128) {
          if (pauli) hipLaunchKernelGGL((k_sv_kq4_x16<1, NT, ORD, true>), grid, dim3(1024), 0, s, a, g0, qs, dev_matrix);
          else hipLaunchKernelGGL((k_sv_kq4_x16<1, NT, ORD, false>), grid, dim3(1024), 0, s, a, g0, qs, dev_matrix);
        } else {
          if (pauli) hipLaunchKernelGGL((k_sv_kq4_x16<2, NT, ORD, true>), grid, dim3(512), 0, s, a, g0, qs, dev_matrix);
          else hipLaunchKernelGGL((k_sv_kq4_x16<2, NT, ORD, false>), grid, dim3(512), 0, s, a, g0, qs, dev_matrix);
        }
      });
    }
    return;
  }
  // one group per thread (16 loads in flight at k = 4); only the hint is tunable
  const dim3 grid(grid_for(ng, kBlock));
  if (k == 3) {
    if (cfg.nt & 1) hipLaunchKernelGGL((k_sv_kq<3, true>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
    else hipLaunchKernelGGL((k_sv_kq<3, false>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
  } else if (pauli) {
    if (cfg.nt & 1) hipLaunchKernelGGL((k_sv_kq<4, true, true>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
    else hipLaunchKernelGGL((k_sv_kq<4, false, true>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
  } else {
    if (cfg.nt & 1) hipLaunchKernelGGL((k_sv_kq<4, true>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
    else hipLaunchKernelGGL((k_sv_kq<4, false>), grid, dim3(kBlock), 0, s, a, ng, qs, dev_matrix);
  }
}

}  // namespace nwq

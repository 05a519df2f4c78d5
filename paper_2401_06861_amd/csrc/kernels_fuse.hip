// Fused k-qubit blocks: a run of gates whose qubits all lie in one tile set
// T = {0..c-1} u {hi_0..hi_{m-1}} is applied to each tile of 2^(c+m)
// amplitudes staged in LDS, so the block costs one read and one write of the
// vector instead of one per gate.  The low c bits give 2^m contiguous chunks
// of 2^c amplitudes (c >= 6: 1 KiB wave-contiguous loads and stores); the
// high bits pick which chunks form a tile.  Inside LDS each gate is a pass
// over the tile with a barrier between gates.
#include "nwq_internal.h"

namespace nwq {
namespace {

constexpr int kFuseBlock = 256;

__device__ __forceinline__ unsigned ins0(unsigned p, int q) { return ((p >> q) << (q + 1)) | (p & ((1u << q) - 1u)); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}

// Global index of tile entry l: low c bits in place, bit c + i of l on
// qubit hi[i].
template <class Blk>
__device__ __forceinline__ unsigned long long tile_index(unsigned long long base, unsigned l, unsigned cmask, int c,
                                                         int m, const Blk& blk) {
  unsigned long long g = base | (l & cmask);
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (i < m && ((l >> (c + i)) & 1u)) g |= 1ull << blk.hi[i];
  return g;
}

// Clang vector of two doubles: stays in registers where copies of HIP's
// double2 struct can go through scratch.
typedef double vd2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ vd2 ldv(const double2* p) { return *reinterpret_cast<const vd2*>(p); }
__device__ __forceinline__ void stv(double2* p, vd2 v) { *reinterpret_cast<vd2*>(p) = v; }

// Tile staging in chunks of kStage entries per thread: all loads of a chunk
// are issued before the first LDS write (and all LDS reads before the first
// global store), so each thread keeps kStage requests in flight instead of
// one.  Tiles of at least kStage * kFuseBlock entries take whole chunks.
constexpr int kStage = 8;

__global__ __launch_bounds__(kFuseBlock) void k_fused(double2* __restrict__ a, int nbits, FusedBlockDev blk,
                                                      const FusedOp* __restrict__ ops,
                                                      const double2* __restrict__ mats) {
  extern __shared__ double2 t[];
  const int c = blk.c, m = blk.m, k = c + m;
  const unsigned len = 1u << k;
  const unsigned long long ntiles = 1ull << (nbits - k);
  const unsigned cmask = (1u << c) - 1u;
  for (unsigned long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    unsigned long long base = tile << c;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < m) {
        const int q = blk.hi[i];
        base = ((base >> q) << (q + 1)) | (base & ((1ull << q) - 1ull));
      }
    }
    __syncthreads();
    if (len >= kStage * kFuseBlock) {
      for (unsigned l0 = threadIdx.x; l0 < len; l0 += kStage * kFuseBlock) {
        vd2 r[kStage];
#pragma unroll
        for (int j = 0; j < kStage; ++j) r[j] = ldv(a + tile_index(base, l0 + j * kFuseBlock, cmask, c, m, blk));
#pragma unroll
        for (int j = 0; j < kStage; ++j) stv(t + l0 + j * kFuseBlock, r[j]);
      }
    } else {
      for (unsigned l = threadIdx.x; l < len; l += kFuseBlock) t[l] = a[tile_index(base, l, cmask, c, m, blk)];
    }
    for (int oi = 0; oi < blk.op_count; ++oi) {
      const FusedOp op = ops[blk.op_begin + oi];
      const double2* M = mats + op.mat;
      __syncthreads();
      switch (op.kind) {
        case 0: {   // 1q dense on local bit lo
          const double2 m0 = M[0], m1 = M[1], m2 = M[2], m3 = M[3];
          const unsigned off = 1u << op.lo;
          for (unsigned p = threadIdx.x; p < (len >> 1); p += kFuseBlock) {
            const unsigned i0 = ins0(p, op.lo);
            const double2 v0 = t[i0], v1 = t[i0 + off];
            t[i0] = cfma(m0, v0, cmul(m1, v1));
            t[i0 + off] = cfma(m2, v0, cmul(m3, v1));
          }
          break;
        }
        case 1: {   // 1q diagonal
          const double2 d0 = M[0], d1 = M[1];
          for (unsigned l = threadIdx.x; l < len; l += kFuseBlock) t[l] = cmul(((l >> op.lo) & 1u) ? d1 : d0, t[l]);
          break;
        }
        case 2: {   // 2q dense, operator order offsets o0, o1
          const unsigned o0 = (unsigned)op.o0, o1 = (unsigned)op.o1;
          for (unsigned p = threadIdx.x; p < (len >> 2); p += kFuseBlock) {
            const unsigned b = ins0(ins0(p, op.lo), op.hi);
            const unsigned idx[4] = {b, b + o0, b + o1, b + o0 + o1};
            double2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = t[idx[u]];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              double2 acc = cmul(M[4 * r], v[0]);
#pragma unroll
              for (int cc = 1; cc < 4; ++cc) acc = cfma(M[4 * r + cc], v[cc], acc);
              t[idx[r]] = acc;
            }
          }
          break;
        }
        case 3: {   // exchange two members of each quad (CX, SWAP)
          const unsigned oa = (unsigned)op.o0, ob = (unsigned)op.o1;
          for (unsigned p = threadIdx.x; p < (len >> 2); p += kFuseBlock) {
            const unsigned b = ins0(ins0(p, op.lo), op.hi);
            const double2 x = t[b + oa], y = t[b + ob];
            t[b + oa] = y;
            t[b + ob] = x;
          }
          break;
        }
        default: {  // 2q diagonal, bits o0 (u bit 0) and o1 (u bit 1)
          const double2 d0 = M[0], d1 = M[1], d2 = M[2], d3 = M[3];
          for (unsigned l = threadIdx.x; l < len; l += kFuseBlock) {
            const unsigned u = ((l >> op.o0) & 1u) | (((l >> op.o1) & 1u) << 1);
            const double2 d = (u & 2u) ? ((u & 1u) ? d3 : d2) : ((u & 1u) ? d1 : d0);
            t[l] = cmul(d, t[l]);
          }
          break;
        }
      }
    }
    __syncthreads();
    if (len >= kStage * kFuseBlock) {
      for (unsigned l0 = threadIdx.x; l0 < len; l0 += kStage * kFuseBlock) {
        vd2 r[kStage];
#pragma unroll
        for (int j = 0; j < kStage; ++j) r[j] = ldv(t + l0 + j * kFuseBlock);
#pragma unroll
        for (int j = 0; j < kStage; ++j) stv(a + tile_index(base, l0 + j * kFuseBlock, cmask, c, m, blk), r[j]);
      }
    } else {
      for (unsigned l = threadIdx.x; l < len; l += kFuseBlock) a[tile_index(base, l, cmask, c, m, blk)] = t[l];
    }
  }
}

}  // namespace

void launch_fused_block(hipStream_t s, double2* a, int nbits, const FusedBlockDev& blk, const FusedOp* ops,
                        const double2* mats, int /*lds_k*/) {
  const int k = blk.c + blk.m;
  const unsigned long long ntiles = 1ull << (nbits - k);
  const unsigned long long cap = 1ull << 20;
  const unsigned grid = (unsigned)(ntiles < cap ? ntiles : cap);
  const size_t lds = sizeof(double2) << k;
  if (lds > 65536) (void)enable_dynamic_lds((const void*)k_fused);
  hipLaunchKernelGGL(k_fused, dim3(grid), dim3(kFuseBlock), lds, s, a, nbits, blk, ops, mats);
}

}  // namespace nwq

// ===========================================================================
// Register-blocked variant.  Each of the 2^(k-R) threads of a tile holds 2^R
// amplitudes that differ on R tile bits (the phase's register bits, R = 3 or
// 4); every gate of the phase acts on those bits only and runs in registers.
// Between phases the tile is exchanged through LDS (one write, one barrier,
// one read), so LDS traffic is one tile pass per phase instead of one per
// gate.  LDS rows are padded by one entry every 16 so that lanes whose local
// indices differ by multiples of 16 land in different banks.
//
// R trades registers for phases: R = 4 applies more gates per exchange but
// needs 256 VGPRs (2 waves per SIMD); R = 3 fits 128 VGPRs and halves the LDS
// per wave, so 4 waves per SIMD hide the LDS and HBM latency of each other.
// ===========================================================================
namespace nwq {
namespace {

__device__ __forceinline__ vd2 mkv(double a, double b) { vd2 r; r.x = a; r.y = b; return r; }
__device__ __forceinline__ vd2 vmul(vd2 a, vd2 b) { return mkv(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)); }
__device__ __forceinline__ vd2 vfma(vd2 a, vd2 b, vd2 c) {
  return mkv(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ unsigned padl(unsigned l) { return l + (l >> 4); }

// Every gate helper reads the register set x and writes all of y; x and y may be
// the same array.  With 4 register bits the op loop alternates two register
// sets, so each gate's results land directly in the registers the next gate
// reads (an in-place update ends every op with a copy of all 16 amplitudes
// back into the loop-carried registers).  With 3 register bits the second set
// would push the kernel past 128 VGPRs, so it updates in place.
// R00: M[0][0] is real (U3, RX), its imaginary part is not read and the
// first output of a pair takes two FMAs fewer.  REAL: all of M is real (RY,
// H): four FP64 operations per output instead of eight.
template <int NV, int B, bool R00 = false, bool REAL = false>
__device__ __forceinline__ void rb_dense1(const vd2 (&x)[NV], vd2 (&y)[NV], const double2* __restrict__ M) {
  const vd2 m0 = ldv(M), m1 = ldv(M + 1), m2 = ldv(M + 2), m3 = ldv(M + 3);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (j & (1 << B)) continue;
    const vd2 a = x[j], b = x[j | (1 << B)];
    if constexpr (REAL) {
      y[j] = mkv(fma(m0.x, a.x, m1.x * b.x), fma(m0.x, a.y, m1.x * b.y));
      y[j | (1 << B)] = mkv(fma(m2.x, a.x, m3.x * b.x), fma(m2.x, a.y, m3.x * b.y));
      continue;
    }
    if constexpr (R00) {
      const vd2 c = vmul(m1, b);
      y[j] = mkv(fma(m0.x, a.x, c.x), fma(m0.x, a.y, c.y));
    } else {
      y[j] = vfma(m0, a, vmul(m1, b));
    }
    y[j | (1 << B)] = vfma(m2, a, vmul(m3, b));
  }
}

// Dense 4x4 with operator index u = bit B0 + 2 bit B1.
template <int NV, int B0, int B1>
__device__ __forceinline__ void rb_dense2(const vd2 (&x)[NV], vd2 (&y)[NV], const double2* __restrict__ M) {
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (j & ((1 << B0) | (1 << B1))) continue;
    const int idx[4] = {j, j | (1 << B0), j | (1 << B1), j | (1 << B0) | (1 << B1)};
    vd2 in[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) in[u] = x[idx[u]];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      vd2 acc = vmul(ldv(M + 4 * r), in[0]);
#pragma unroll
      for (int c = 1; c < 4; ++c) acc = vfma(ldv(M + 4 * r + c), in[c], acc);
      y[idx[r]] = acc;
    }
  }
}

// Dense 16x16 over all four register bits, the matrix in register order:
// y[r] = sum_c M[16 r + c] x[c] (4-register-bit kernel only).
template <int NV>
__device__ __forceinline__ void rb_dense16(const vd2 (&x)[NV], vd2 (&y)[NV], const double2* __restrict__ M) {
  if constexpr (NV == 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      vd2 acc = vmul(ldv(M + 16 * r), x[0]);
#pragma unroll
      for (int c = 1; c < 16; ++c) acc = vfma(ldv(M + 16 * r + c), x[c], acc);
      y[r] = acc;
    }
  }
}

// A 16x16 with the pattern of a Pauli channel after a diagonal gate, in
// register order: M[u] is the diagonal entry of register u, M[16 + 4 i + j]
// the 4x4 among registers 5i and 5j (4-register-bit kernel only).
template <int NV>
__device__ __forceinline__ void rb_pauli16(const vd2 (&x)[NV], vd2 (&y)[NV], const double2* __restrict__ M) {
  if constexpr (NV == 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (u % 5 != 0) y[u] = vmul(ldv(M + u), x[u]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      vd2 acc = vmul(ldv(M + 16 + 4 * i), x[0]);
#pragma unroll
      for (int j = 1; j < 4; ++j) acc = vfma(ldv(M + 16 + 4 * i + j), x[5 * j], acc);
      y[5 * i] = acc;
    }
  }
}

// Exchange of members (base | OA) and (base | OB) of each quad over bits B0, B1.
template <int NV, int B0, int B1, int OA, int OB>
__device__ __forceinline__ void rb_swap2(const vd2 (&x)[NV], vd2 (&y)[NV]) {
  constexpr int Q = (1 << B0) | (1 << B1);
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (j & Q) continue;
    const vd2 a = x[j | OA], b = x[j | OB];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int m = ((u & 1) ? (1 << B0) : 0) | ((u & 2) ? (1 << B1) : 0);
      if (m != OA && m != OB) y[j | m] = x[j | m];
    }
    y[j | OA] = b;
    y[j | OB] = a;
  }
}

// 1q diagonal on register bit B: entries d0 (bit 0), d1 (bit 1).
template <int NV, int B>
__device__ __forceinline__ void rb_diag1(const vd2 (&x)[NV], vd2 (&y)[NV], vd2 d0, vd2 d1) {
#pragma unroll
  for (int j = 0; j < NV; ++j) y[j] = vmul(((j >> B) & 1) ? d1 : d0, x[j]);
}

// 2q diagonal on register bits B0 (u bit 0), B1 (u bit 1): entries M[u].
template <int NV, int B0, int B1>
__device__ __forceinline__ void rb_diag2(const vd2 (&x)[NV], vd2 (&y)[NV], const double2* __restrict__ M) {
  const vd2 d[4] = {ldv(M), ldv(M + 1), ldv(M + 2), ldv(M + 3)};
#pragma unroll
  for (int j = 0; j < NV; ++j) y[j] = vmul(d[((j >> B0) & 1) + 2 * ((j >> B1) & 1)], x[j]);
}

// The case bodies of rb_apply; bit positions at or above R never occur for
// that R (the guard keeps their templates from being instantiated).
template <int R, int B>
__device__ __forceinline__ void rb_c1(int sel, const vd2 (&x)[1 << R], vd2 (&y)[1 << R], const double2* M) {
  if constexpr (B < R) {
    if (sel == 0) rb_dense1<(1 << R), B>(x, y, M);
    else if (sel == 3) rb_dense1<(1 << R), B, true>(x, y, M);
    else if (sel == 4) rb_dense1<(1 << R), B, false, true>(x, y, M);
    else rb_diag1<(1 << R), B>(x, y, ldv(M), ldv(M + (sel == 1 ? 1 : 3)));
  }
}
template <int R, int B0, int B1>
__device__ __forceinline__ void rb_c2(int sel, const vd2 (&x)[1 << R], vd2 (&y)[1 << R], const double2* M) {
  constexpr int NV = 1 << R;
  if constexpr (B0 < R && B1 < R) {
    if (sel == 0) rb_dense2<NV, B0, B1>(x, y, M);
    else if (sel == 1) rb_swap2<NV, B0, B1, (1 << B0), (1 << B0) | (1 << B1)>(x, y);   // CX: control B0, target B1
    else if (sel == 2) rb_swap2<NV, B0, B1, (1 << B0), (1 << B1)>(x, y);                 // SWAP
    else rb_diag2<NV, B0, B1>(x, y, M);
  }
}

// One gate: a single switch over the op's code (rb_op_code); every case is
// specialised on its register bits, so diagonals select their entries at
// compile time.
template <int R>
__device__ __forceinline__ void rb_apply(int code, const double2* __restrict__ M, const vd2 (&x)[1 << R],
                                         vd2 (&y)[1 << R]) {
  constexpr int NV = 1 << R;
#define NWQ_RB1(BASE, SEL) \
  case BASE + 0: rb_c1<R, 0>(SEL, x, y, M); break; \
  case BASE + 1: rb_c1<R, 1>(SEL, x, y, M); break; \
  case BASE + 2: rb_c1<R, 2>(SEL, x, y, M); break; \
  case BASE + 3: rb_c1<R, 3>(SEL, x, y, M); break;
#define NWQ_RB2(BASE, SEL) \
  case BASE + 1: rb_c2<R, 0, 1>(SEL, x, y, M); break; \
  case BASE + 2: rb_c2<R, 0, 2>(SEL, x, y, M); break; \
  case BASE + 3: rb_c2<R, 0, 3>(SEL, x, y, M); break; \
  case BASE + 4: rb_c2<R, 1, 0>(SEL, x, y, M); break; \
  case BASE + 6: rb_c2<R, 1, 2>(SEL, x, y, M); break; \
  case BASE + 7: rb_c2<R, 1, 3>(SEL, x, y, M); break; \
  case BASE + 8: rb_c2<R, 2, 0>(SEL, x, y, M); break; \
  case BASE + 9: rb_c2<R, 2, 1>(SEL, x, y, M); break; \
  case BASE + 11: rb_c2<R, 2, 3>(SEL, x, y, M); break; \
  case BASE + 12: rb_c2<R, 3, 0>(SEL, x, y, M); break; \
  case BASE + 13: rb_c2<R, 3, 1>(SEL, x, y, M); break; \
  case BASE + 14: rb_c2<R, 3, 2>(SEL, x, y, M); break;
  switch (code) {
    NWQ_RB1(0, 0)
    NWQ_RB1(4, 1)
    NWQ_RB1(8, 2)
    NWQ_RB1(84, 3)
    NWQ_RB1(88, 4)
    NWQ_RB2(16, 0)
    NWQ_RB2(32, 1)
    NWQ_RB2(48, 2)
    NWQ_RB2(64, 3)
    case kRbCodeDense16:
      rb_dense16<NV>(x, y, M);
      break;
    case kRbCodePauli16:
      rb_pauli16<NV>(x, y, M);
      break;
    default:   // kRbCodeCopy
#pragma unroll
      for (int j = 0; j < NV; ++j) y[j] = x[j];
      break;
  }
#undef NWQ_RB1
#undef NWQ_RB2
}

// Writes the 2^R registers of a phase back to their LDS entries.
template <int R>
__device__ __forceinline__ void rb_store_phase(double2* __restrict__ tl, const FusedPhase& ph, const vd2 (&v)[1 << R]) {
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) stv(tl + ph.st_off[j], v[j]);
}

// Global loads and stores of tile entries; NT: non-temporal (each entry is
// read and written once per block, so nothing is worth keeping in cache).
template <bool NT>
__device__ __forceinline__ vd2 gld(const double2* p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const vd2*>(p));
  else return ldv(p);
}
template <bool NT>
__device__ __forceinline__ void gst(double2* p, vd2 v) {
  if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<vd2*>(p));
  else stv(p, v);
}

// Kernel-side view of a register-blocked block: tile shape, phase range and
// the global offsets of the registers a tile is loaded into (lo) and stored
// from (so): the first / last phase's register layout when that phase moves
// straight between HBM and registers (direct bits 0 / 1), else tile entry
// j * 2^(k - R).
struct RbBlockArgs {
  int c, m;
  int hi[8];
  int op_begin, op_count;
  int direct;
  int sparse;                  // tiles t = 0, 1, ... are tile indices pdep(t, tmask)
  unsigned long long tmask;
  unsigned long long lo[16], so[16];
};

// The bits of v deposited, lowest first, at the set bits of mask.
__device__ __forceinline__ unsigned long long pdep64(unsigned long long v, unsigned long long mask) {
  unsigned long long r = 0;
  for (; mask; mask &= mask - 1, v >>= 1)
    if (v & 1ull) r |= mask & (~mask + 1ull);
  return r;
}

template <int R, bool NT>
__global__ __launch_bounds__(R == 4 ? 512 : 1024) void k_fused_rb(double2* __restrict__ a0, int nbits,
                                                                  RbBlockArgs blk,
                                                                  const FusedPhase* __restrict__ phases,
                                                                  const FusedOp* __restrict__ ops,
                                                                  const double2* __restrict__ mats0,
                                                                  unsigned long long state_stride, int mat_stride,
                                                                  unsigned long long ntiles) {
  constexpr int NV = 1 << R;
  extern __shared__ double2 t[];
  // batch element blockIdx.y: its own state and its own matrix table
  double2* __restrict__ a = a0 + (size_t)blockIdx.y * state_stride;
  const double2* __restrict__ mats = mats0 + (size_t)blockIdx.y * mat_stride;
  const int c = blk.c, m = blk.m, k = c + m;
  const unsigned len = 1u << k;
  const unsigned nt = len >> R;
  const unsigned cmask = (1u << c) - 1u;
  const unsigned tid = threadIdx.x;
  const int P = blk.op_count;
  const bool ldd = (blk.direct & 1) != 0, sdd = (blk.direct & 2) != 0;
  // thread bits -> the tile bits outside a phase's register bits: insert a
  // zero at each (ascending) register position
  auto spread = [&](const FusedPhase& ph) {
    unsigned dep = tid;
#pragma unroll
    for (int r = 0; r < R; ++r) dep = ((dep >> ph.reg[r]) << (ph.reg[r] + 1)) | (dep & ((1u << ph.reg[r]) - 1u));
    return dep;
  };
  // thread part of the entry indices of the load and store layouts
  const unsigned long long gl_ld = tile_index(0ull, ldd ? spread(phases[blk.op_begin]) : tid, cmask, c, m, blk);
  const unsigned long long gl_st = tile_index(0ull, sdd ? spread(phases[blk.op_begin + P - 1]) : tid, cmask, c, m, blk);
  auto tile_base = [&](unsigned long long t) {
    unsigned long long base = (blk.sparse ? pdep64(t, blk.tmask) : t) << c;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < m) {
        const int q = blk.hi[i];
        base = ((base >> q) << (q + 1)) | (base & ((1ull << q) - 1ull));
      }
    }
    return base;
  };
  // A tile's NV entries per thread are loaded one tile ahead: the loads of
  // the next tile are in flight while this one runs its phases (tiles are
  // disjoint, so the early read is safe).  A tile's results go to HBM after
  // its last phase and before the next tile's loaded registers are used; the
  // vector memory counter retires in issue order, so the wait for those loads
  // (issued before the stores) leaves the stores in flight.  The loaded
  // registers are taken up at the bottom of the loop, behind the stores on
  // every path into it: at the loop head the paths from the first tile and
  // from the back edge differ, and the compiler's wait counts, merged there,
  // would wait for the stores too.  With direct I/O the first phase runs on
  // the loaded registers and the last phase's registers are the results, so
  // a block of one such phase never touches LDS.
  if (blockIdx.x >= ntiles) return;
  vd2 pf[NV], v[NV];
  // first phase input: the registers themselves, or the tile in LDS (every
  // wave must be done reading the previous tile before it is overwritten)
  auto take_loaded = [&]() {
    if (ldd) {
#pragma unroll
      for (int j = 0; j < NV; ++j) v[j] = pf[j];
    } else {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NV; ++j) stv(t + padl(tid + j * nt), pf[j]);
    }
  };
  auto load_tile = [&](unsigned long long tl) {
    const double2* __restrict__ p = a + tile_base(tl) + gl_ld;
#pragma unroll
    for (int j = 0; j < NV; ++j) pf[j] = gld<NT>(p + blk.lo[j]);
  };
  unsigned long long tile = blockIdx.x;
  load_tile(tile);
  take_loaded();
  if (tile + gridDim.x < ntiles) load_tile(tile + gridDim.x);
  for (;;) {
    for (int pi = 0; pi < P; ++pi) {
      const FusedPhase ph = phases[blk.op_begin + pi];
      // padl(dep | off) = padl(dep) + padl(off) for disjoint bit sets
      double2* __restrict__ tl = t + padl(spread(ph));
      if (pi > 0 || !ldd) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = ldv(tl + ph.ld_off[j]);
      }
      const FusedOp* __restrict__ po = ops + ph.op_begin;
      if constexpr (R == 4) {
        // two gates per trip, v -> w -> v; an odd count ends with a copy
        vd2 w[NV];
        for (int oi = 0; oi < ph.op_count; oi += 2) {
          rb_apply<R>(po[oi].code, mats + po[oi].mat, v, w);
          int c2 = kRbCodeCopy, m2 = 0;
          if (oi + 1 < ph.op_count) {
            c2 = po[oi + 1].code;
            m2 = po[oi + 1].mat;
          }
          rb_apply<R>(c2, mats + m2, w, v);
        }
      } else {
        for (int oi = 0; oi < ph.op_count; ++oi) rb_apply<R>(po[oi].code, mats + po[oi].mat, v, v);
      }
      if (pi < P - 1 || !sdd) {   // else the results stay in v
        // the tile's first LDS write when the first phase came from HBM:
        // every wave must be done reading the previous tile
        if (pi == 0 && ldd) __syncthreads();
        rb_store_phase<R>(tl, ph, v);
      }
    }
    if (!sdd) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NV; ++j) v[j] = ldv(t + padl(tid + j * nt));
    }
    double2* __restrict__ out = a + tile_base(tile) + gl_st;
#pragma unroll
    for (int j = 0; j < NV; ++j) gst<NT>(out + blk.so[j], v[j]);
    tile += gridDim.x;
    if (tile >= ntiles) break;
    take_loaded();
    if (tile + gridDim.x < ntiles) load_tile(tile + gridDim.x);
  }
}

}  // namespace

size_t fused_rb_lds_bytes(int k) { return sizeof(double2) * ((1u << k) + (1u << k) / 16); }

int fused_rb_enable_lds() {
  int rc = NWQ_OK;
  for (const void* f : {(const void*)k_fused_rb<3, false>, (const void*)k_fused_rb<3, true>,
                        (const void*)k_fused_rb<4, false>, (const void*)k_fused_rb<4, true>})
    if (!rc) rc = enable_dynamic_lds(f);
  return rc;
}

void launch_fused_rb(hipStream_t s, double2* a, int nbits, const FusedBlockDev& blk, const FusedPhase* phases,
                     const FusedOp* ops, const double2* mats, int rbits, int batch, int mat_stride, int max_grid,
                     int flags, unsigned long long max_tiles, unsigned long long tile_mask) {
  const int k = blk.c + blk.m;
  unsigned long long ntiles = 1ull << (nbits - k);
  if (max_tiles > 0 && max_tiles < ntiles) ntiles = max_tiles;
  const bool sparse = tile_mask != ~0ull && __builtin_popcountll(tile_mask) < nbits - k;
  if (sparse) ntiles = 1ull << __builtin_popcountll(tile_mask);
  // about four tiles per workgroup (so that the next tile's loads overlap
  // this one's phases), at least 2048 workgroups
  const unsigned long long cap = max_grid > 0 ? (unsigned long long)max_grid
                                              : (ntiles / 4 > 2048 ? ntiles / 4 : 2048);
  const unsigned grid = (unsigned)(ntiles < cap ? ntiles : cap);
  const size_t lds = fused_rb_lds_bytes(k);
  const unsigned long long stride = batch > 1 ? (1ull << nbits) : 0ull;
  RbBlockArgs b{};
  b.c = blk.c;
  b.m = blk.m;
  for (int i = 0; i < 8; ++i) b.hi[i] = blk.hi[i];
  b.op_begin = blk.op_begin;
  b.op_count = blk.op_count;
  b.direct = (flags & kFusedDirect) ? blk.direct : 0;
  b.sparse = sparse ? 1 : 0;
  b.tmask = sparse ? tile_mask : 0ull;
  for (int j = 0; j < 16; ++j) {
    b.lo[j] = (b.direct & 1) ? blk.jdir[j] : blk.joff[j];
    b.so[j] = (b.direct & 2) ? blk.sdir[j] : blk.joff[j];
  }
  auto go = [&](auto kern, int rb) {
    if (lds > 65536) (void)enable_dynamic_lds((const void*)kern);
    hipLaunchKernelGGL(kern, dim3(grid, batch), dim3(1u << (k - rb)), lds, s, a, nbits, b, phases, ops, mats,
                       stride, mat_stride, ntiles);
  };
  const bool nt = (flags & kFusedNonTemporal) != 0;
  if (rbits == 3) {
    if (nt) go(k_fused_rb<3, true>, 3);
    else go(k_fused_rb<3, false>, 3);
  } else {
    if (nt) go(k_fused_rb<4, true>, 4);
    else go(k_fused_rb<4, false>, 4);
  }
}

}  // namespace nwq

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
    for (unsigned l = threadIdx.x; l < len; l += kFuseBlock) {
      unsigned long long g = base | (l & cmask);
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < m && ((l >> (c + i)) & 1u)) g |= 1ull << blk.hi[i];
      t[l] = a[g];
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
    for (unsigned l = threadIdx.x; l < len; l += kFuseBlock) {
      unsigned long long g = base | (l & cmask);
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < m && ((l >> (c + i)) & 1u)) g |= 1ull << blk.hi[i];
      a[g] = t[l];
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
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)k_fused, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_fused, dim3(grid), dim3(kFuseBlock), lds, s, a, nbits, blk, ops, mats);
}

}  // namespace nwq

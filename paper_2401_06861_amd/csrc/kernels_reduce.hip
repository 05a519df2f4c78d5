// Deterministic reductions: Pauli-term expectation values of a state vector,
// Tr(rho P) of a density matrix, and sums of squared moduli.
//
// Every reduction has a fixed order: per-lane partials, a wave64 xor-shuffle
// tree, per-wave slots in LDS combined in wave order, per-block partials in
// global memory, and a second stage that sums each row of block partials in
// a fixed order.  No atomics, so results are bitwise reproducible for a given
// input size and launch shape, whatever else runs on the device.
//
// Pauli term P = i^{|x&z|} X^x Z^z acts as P|j> = i^y (-1)^{|j&z|} |j^x>, so
//   <P> = sum_j i^y (-1)^{|j&z|} conj(a_{j^x}) a_j .
// For x != 0 the contributions of j and j^x are complex conjugates, so the
// sum over j with bit h(x) clear of 2 Re(...) gives <P> with no imaginary
// residue; for x = 0 the summand (-1)^{|j&z|} |a_j|^2 is real.
//
// Tiling: a workgroup stages a tile of 2^(c+m) amplitudes in LDS -- 2^m
// contiguous chunks of 2^c amplitudes (c >= 6 gives 1 KiB wave-contiguous
// loads) whose high bits sit at m chosen positions -- so every term whose
// flipped bits x lie inside the tile finds its partner in LDS.  The host
// groups terms into passes of tiles that cover their x bits.
#include "nwq_internal.h"

namespace nwq {
namespace {

constexpr int kRedBlock = 256;
constexpr int kRedWaves = kRedBlock / kWave;
constexpr int kMaxTermsPerPass = 16;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Tile-local index l -> global index (without the tile base): low c bits
// pass through; bit c+i of l goes to position hi[i].
__device__ __forceinline__ unsigned long long scatter_local(unsigned l, int c, int m, const TileShape& t) {
  unsigned long long g = l & ((1u << c) - 1u);
#pragma unroll 8
  for (int i = 0; i < 8; ++i)
    if (i < m && ((l >> (c + i)) & 1u)) g |= 1ull << t.hi[i];
  return g;
}

// Per-term sums over tiles: each thread keeps one register accumulator per
// term (up to TPL terms per launch) across all tiles it visits, so the wave
// and workgroup reductions happen once per launch, not once per tile.
template <int TPL>
__global__ __launch_bounds__(kRedBlock) void k_pauli_tile(const double2* __restrict__ a, int nbits, TileShape t,
                                                          const TermDev* __restrict__ terms, int count,
                                                          double* __restrict__ partials, int first_row) {
  extern __shared__ double2 lds_tile[];
  __shared__ unsigned s_xl[TPL], s_zl[TPL], s_hb[TPL];
  __shared__ int s_y[TPL];
  __shared__ unsigned long long s_zo[TPL];
  __shared__ double s_acc[TPL][kRedWaves];
  const int k = t.c + t.m;
  const unsigned tile_len = 1u << k;
  const unsigned long long ntiles = 1ull << (nbits - k);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if ((int)threadIdx.x < count) {
    const TermDev T = terms[threadIdx.x];
    s_xl[threadIdx.x] = (unsigned)T.xl;
    s_zl[threadIdx.x] = (unsigned)T.zl;
    s_hb[threadIdx.x] = (unsigned)(T.xl & (~T.xl + 1ull));   // lowest flipped bit
    s_y[threadIdx.x] = T.y & 3;
    s_zo[threadIdx.x] = T.zo;
  }
  double acc[TPL];
#pragma unroll
  for (int i = 0; i < TPL; ++i) acc[i] = 0.0;

  for (unsigned long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // base: tile index spread over the bits outside the tile (low c bits are inside)
    unsigned long long base = tile << t.c;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < t.m) {
        const int q = t.hi[i];
        base = ((base >> q) << (q + 1)) | (base & ((1ull << q) - 1ull));
      }
    }
    __syncthreads();   // previous tile's readers are done (and the term table is written)
    for (unsigned l = threadIdx.x; l < tile_len; l += kRedBlock) lds_tile[l] = a[base | scatter_local(l, t.c, t.m, t)];
    __syncthreads();
    unsigned outer = 0;
#pragma unroll
    for (int ti = 0; ti < TPL; ++ti)
      if (ti < count) outer |= (unsigned)(__popcll(base & s_zo[ti]) & 1) << ti;
    for (unsigned l = threadIdx.x; l < tile_len; l += kRedBlock) {
      const double2 v = lds_tile[l];
      const double nv = fma(v.x, v.x, v.y * v.y);
#pragma unroll
      for (int ti = 0; ti < TPL; ++ti) {
        if (ti < count) {
          const unsigned xl = s_xl[ti];
          double r = 0.0;
          if (xl == 0u) {
            r = nv;
          } else if ((l & s_hb[ti]) == 0u) {
            const double2 p = lds_tile[l ^ xl];
            const double wr = fma(p.x, v.x, p.y * v.y);    // w = conj(p) v
            const double wi = fma(p.x, v.y, -p.y * v.x);
            const int y = s_y[ti];                           // Re(i^y w)
            r = (y == 0) ? wr : (y == 1) ? -wi : (y == 2) ? -wr : wi;
            r *= 2.0;
          }
          const unsigned sg = ((unsigned)__popc(l & s_zl[ti]) ^ (outer >> ti)) & 1u;
          acc[ti] += sg ? -r : r;
        }
      }
    }
  }
#pragma unroll
  for (int ti = 0; ti < TPL; ++ti) {
    if (ti < count) {
      const double w = wave_sum(acc[ti]);
      if (lane == 0) s_acc[ti][wave] = w;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < count) {
    double s = 0.0;
    for (int w = 0; w < kRedWaves; ++w) s += s_acc[threadIdx.x][w];
    partials[(unsigned long long)(first_row + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
}

// Terms with no flipped bits: <Z^z> = sum_j (-1)^{|j & z|} |a_j|^2.  A
// workgroup visits chunks of 256 EPT consecutive entries (grid-stride);
// thread tid reads entries B + 256 e + tid (e < EPT), one coalesced load each.
// The sign of entry j splits as the parities of (j & z) over three disjoint
// bit fields: tid (fixed per thread), e (bits 8.., fixed per e) and the chunk
// base B (uniform per chunk, scalar work).  Per chunk each term's EPT signs
// are one bit mask, so a term costs a bit extract and an add per entry (|a|^2
// is never negative, so the sign bit is set by an OR).
// Loads are non-temporal, and with xcd_order (grid a multiple of 8)
// workgroup i starts at chunk (i mod 8) G/8 + floor(i / 8), so each of the 8
// XCDs (dealt workgroups in turn) reads contiguous chunks on every sweep.  The
// chunks each block visits, and so the rounding of the sums, are fixed by the
// grid size alone.
template <int TPL, int EPT>
__global__ __launch_bounds__(kRedBlock) void k_pauli_diag(const double2* __restrict__ a, unsigned long long len,
                                                          ZMasks zs, int count, double* __restrict__ partials,
                                                          int first_row, int xcd_order) {
  static_assert(kRedBlock == 256 && EPT <= 32, "entry e sits at bit 8 + log2 e");
  __shared__ double s_acc[TPL][kRedWaves];
  constexpr unsigned long long kChunk = (unsigned long long)kRedBlock * EPT;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const unsigned tid = threadIdx.x;
  // per-thread part of each term's sign masks: bit e = parity((tid + 256 e) & z)
  unsigned fixed[TPL];
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    fixed[t] = 0u;
    if (t < count) {
      const unsigned long long z = zs.z[t];
      const unsigned tp = (unsigned)__popc(tid & (unsigned)(z & 0xFFull)) & 1u;
      unsigned m = 0u;
#pragma unroll
      for (int e = 0; e < EPT; ++e) m |= (((unsigned)__popc((unsigned)e & (unsigned)(z >> 8)) & 1u) ^ tp) << e;
      fixed[t] = m;
    }
  }
  double acc[TPL];
#pragma unroll
  for (int t = 0; t < TPL; ++t) acc[t] = 0.0;
  const unsigned long long first =
      xcd_order ? (unsigned long long)((blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3)) : blockIdx.x;
  for (unsigned long long B = first * kChunk; B < len; B += (unsigned long long)gridDim.x * kChunk) {
    double p[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const unsigned long long i = B + (unsigned long long)e * kRedBlock + tid;
      typedef double vd2r __attribute__((ext_vector_type(2)));
      const vd2r v = i < len ? __builtin_nontemporal_load(reinterpret_cast<const vd2r*>(a + i)) : vd2r{0.0, 0.0};
      p[e] = fma(v.x, v.x, v.y * v.y);
    }
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
      if (t < count) {
        // chunk parity: bits of B at and above bit 8 + log2(EPT) (B has none below)
        const unsigned cb = (unsigned)__popcll(B & zs.z[t]) & 1u;
        const unsigned sm = fixed[t] ^ (cb ? 0xFFFFFFFFu : 0u);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int hi = __double2hiint(p[e]) | (int)(((sm >> e) & 1u) << 31);
          acc[t] += __hiloint2double(hi, __double2loint(p[e]));
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    if (t < count) {
      const double w = wave_sum(acc[t]);
      if (lane == 0) s_acc[t][wave] = w;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < count) {
    double s = 0.0;
    for (int w = 0; w < kRedWaves; ++w) s += s_acc[threadIdx.x][w];
    partials[(unsigned long long)(first_row + threadIdx.x) * gridDim.x + blockIdx.x] = s;
  }
}

// One term whose flipped bits do not fit a tile: pairs (j, j^x) over the
// j with bit h (the lowest bit of x) clear, read straight from global memory.
__global__ __launch_bounds__(kRedBlock) void k_pauli_pairs(const double2* __restrict__ a, int nbits,
                                                           unsigned long long x, unsigned long long z, int y,
                                                           double* __restrict__ partials) {
  __shared__ double accw[kRedWaves];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int h = __ffsll((long long)x) - 1;
  const unsigned long long npairs = 1ull << (nbits - 1);
  double s = 0.0;
  for (unsigned long long p = (unsigned long long)blockIdx.x * kRedBlock + threadIdx.x; p < npairs;
       p += (unsigned long long)gridDim.x * kRedBlock) {
    const unsigned long long j = ((p >> h) << (h + 1)) | (p & ((1ull << h) - 1ull));
    const double2 v = a[j];
    const double2 q = a[j ^ x];
    const double wr = fma(q.x, v.x, q.y * v.y);
    const double wi = fma(q.x, v.y, -q.y * v.x);
    double r;
    switch (y & 3) {
      case 0: r = wr; break;
      case 1: r = -wi; break;
      case 2: r = -wr; break;
      default: r = wi; break;
    }
    r *= 2.0;
    s += (__popcll(j & z) & 1) ? -r : r;
  }
  s = wave_sum(s);
  if (lane == 0) accw[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kRedWaves; ++w) r += accw[w];
    partials[blockIdx.x] = r;
  }
}

// Tr(rho P) = sum_r rho[r, r^x] i^y (-1)^{|r&z|} over the 2^n rows.
__global__ __launch_bounds__(kRedBlock) void k_dm_pauli(const double2* __restrict__ rho, int n,
                                                        const TermDev* __restrict__ terms, int count,
                                                        double* __restrict__ partials) {
  __shared__ double accr[kRedWaves], acci[kRedWaves];
  const unsigned long long dim = 1ull << n;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int ti = 0; ti < count; ++ti) {
    const TermDev T = terms[ti];    // for DM the masks are global: xl = x, zl = z
    double sr = 0.0, si = 0.0;
    for (unsigned long long r = (unsigned long long)blockIdx.x * kRedBlock + threadIdx.x; r < dim;
         r += (unsigned long long)gridDim.x * kRedBlock) {
      const double2 v = rho[r * dim + (r ^ T.xl)];
      double vr = v.x, vi = v.y;
      switch (T.y & 3) {   // multiply by i^y
        case 1: { const double t0 = vr; vr = -vi; vi = t0; break; }
        case 2: vr = -vr; vi = -vi; break;
        case 3: { const double t0 = vr; vr = vi; vi = -t0; break; }
        default: break;
      }
      if (__popcll(r & T.zl) & 1) { vr = -vr; vi = -vi; }
      sr += vr;
      si += vi;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) { accr[wave] = sr; acci[wave] = si; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a0 = 0.0, a1 = 0.0;
      for (int w = 0; w < kRedWaves; ++w) { a0 += accr[w]; a1 += acci[w]; }
      partials[(unsigned long long)(2 * ti) * gridDim.x + blockIdx.x] = a0;
      partials[(unsigned long long)(2 * ti + 1) * gridDim.x + blockIdx.x] = a1;
    }
    __syncthreads();
  }
}

template <int EPT>
__global__ __launch_bounds__(kRedBlock) void k_sumsq(const double2* __restrict__ a, unsigned long long len,
                                                     double* __restrict__ partials) {
  __shared__ double accw[kRedWaves];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  double s = 0.0;
  const unsigned long long stride = (unsigned long long)gridDim.x * kRedBlock * EPT;
  for (unsigned long long i0 = (unsigned long long)blockIdx.x * kRedBlock * EPT + threadIdx.x; i0 < len; i0 += stride) {
    double2 v[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const unsigned long long i = i0 + (unsigned long long)j * kRedBlock;
      v[j] = i < len ? a[i] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) s += fma(v[j].x, v[j].x, v[j].y * v[j].y);
  }
  s = wave_sum(s);
  if (lane == 0) accw[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kRedWaves; ++w) r += accw[w];
    partials[blockIdx.x] = r;
  }
}

// Second stage: one wave per row, lane-strided partial sums then the xor
// tree; optional coefficient-weighted total in row order by one lane.
__global__ __launch_bounds__(kRedBlock) void k_reduce_rows(const double* __restrict__ partials, int rows, int grid,
                                                           const double* __restrict__ coeffs, double* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int r = wave; r < rows; r += kRedWaves) {
    double s = 0.0;
    for (int b = lane; b < grid; b += kWave) s += partials[(unsigned long long)r * grid + b];
    s = wave_sum(s);
    if (lane == 0) out[r] = s;
  }
  if (coeffs != nullptr) {
    __syncthreads();
    __threadfence_block();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int r = 0; r < rows; ++r) t = fma(coeffs[r], out[r], t);
      out[rows] = t;
    }
  }
}

}  // namespace

int pauli_tile_grid(int nbits, const TileShape& t) {
  const unsigned long long ntiles = 1ull << (nbits - t.c - t.m);
  const unsigned long long cap = 2048;
  return (int)(ntiles < cap ? ntiles : cap);
}

void launch_pauli_tile(hipStream_t s, const double2* a, int nbits, const TileShape& t, const TermDev* terms,
                       int count, double* partials, int first_row, int grid) {
  const size_t lds = sizeof(double2) << (t.c + t.m);
  hipLaunchKernelGGL(k_pauli_tile<kMaxTermsPerPass>, dim3(grid), dim3(kRedBlock), lds, s, a, nbits, t, terms, count, partials,
                     first_row);
}

void launch_pauli_diag(hipStream_t s, const double2* a, int nbits, const ZMasks& zs, int count, double* partials,
                       int first_row, int grid) {
  hipLaunchKernelGGL((k_pauli_diag<kMaxTermsPerPass, 8>), dim3(grid), dim3(kRedBlock), 0, s, a, 1ull << nbits, zs,
                     count, partials, first_row, grid % 8 == 0 ? 1 : 0);
}

void launch_pauli_pairs(hipStream_t s, const double2* a, int nbits, unsigned long long x, unsigned long long z,
                        int y, double* partials, int grid) {
  hipLaunchKernelGGL(k_pauli_pairs, dim3(grid), dim3(kRedBlock), 0, s, a, nbits, x, z, y, partials);
}

int dm_pauli_grid(int n) {
  const unsigned long long dim = 1ull << n;
  const unsigned long long g = (dim + kRedBlock - 1) / kRedBlock;
  return (int)(g < 256 ? g : 256);
}

void launch_dm_pauli(hipStream_t s, const double2* rho, int n, const TermDev* terms, int count, double* partials,
                     int grid) {
  hipLaunchKernelGGL(k_dm_pauli, dim3(grid), dim3(kRedBlock), 0, s, rho, n, terms, count, partials);
}

int sumsq_grid(unsigned long long len) {
  const unsigned long long g = (len + kRedBlock * 4 - 1) / (kRedBlock * 4);
  return (int)(g < 2048 ? g : 2048);
}

void launch_sumsq(hipStream_t s, const double2* a, unsigned long long len, double* partials, int grid) {
  hipLaunchKernelGGL(k_sumsq<4>, dim3(grid), dim3(kRedBlock), 0, s, a, len, partials);
}

void launch_reduce_rows(hipStream_t s, const double* partials, int rows, int grid, const double* coeffs,
                        double* out) {
  hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(kRedBlock), 0, s, partials, rows, grid, coeffs, out);
}

}  // namespace nwq

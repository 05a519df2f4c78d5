// Measurement: outcome probabilities, readout (measurement) noise on the
// outcome distribution, and shot sampling.
//
// The paper's simulators sit behind providers that return sampled counts and
// list measurement noise in the device noise model (Sec. II front-ends,
// Sec. III noise model).  The three steps here are data-parallel passes over
// the 2^n outcome distribution:
//
//   * probabilities: p_j = |a_j|^2 (state vector) or Re rho_jj (density
//     matrix), one streaming pass;
//   * readout noise: per qubit a column-stochastic 2x2 confusion matrix
//     C[r][t] = P(read r | true t) applied on that qubit's bit of the outcome
//     index, up to five qubits per pass with the group's entries in
//     registers;
//   * sampling by inverse transform on an integer CDF: q_j = floor(p_j 2^61)
//     (exact power-of-two scaling), C_j = q_0 + ... + q_j in 64-bit integers
//     (a tiled scan: per-tile totals, one workgroup for the tile offsets, then
//     the tiles' inclusive scans), and for uniform u the outcome is the
//     smallest j with C_j > floor(floor(u 2^53) Q / 2^53), Q = C_{N-1}.
//     Integer sums are exact and associative, so the CDF is the same in any
//     order, monotone, and never selects a zero-probability outcome.
#include <cmath>
#include <mutex>

#include "engine.h"

namespace nwq {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;                          // entries per thread in a scan tile
constexpr int kScanTile = kScanThreads * kScanPer;    // 4096 entries
constexpr double kQuantScale = 2305843009213693952.0;  // 2^61

typedef double vd2m __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned long long quantize(double p) {
  // probabilities outside [0, 1] (rounding noise below 0, NaN) count as 0 / 1
  if (!(p > 0.0)) return 0ull;
  if (p >= 1.0) return 1ull << 61;
  return (unsigned long long)(p * kQuantScale);   // exact scaling, truncation = floor
}

// One streaming pass with non-temporal loads and stores (each entry is read
// and written once).  xcd_order (grid a multiple of 8): workgroup i takes
// block (i mod 8) G/8 + floor(i / 8) of each sweep of the grid, so that each
// of the 8 XCDs, dealt workgroups in turn, streams one contiguous eighth.
__global__ __launch_bounds__(kBlock) void k_probs_sv(const double2* __restrict__ a, unsigned long long N,
                                                     double* __restrict__ p, int xcd_order) {
  const unsigned long long b =
      xcd_order ? (unsigned long long)((blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3)) : blockIdx.x;
  for (unsigned long long j = b * kBlock + threadIdx.x; j < N; j += (unsigned long long)gridDim.x * kBlock) {
    const vd2m v = __builtin_nontemporal_load(reinterpret_cast<const vd2m*>(a + j));
    __builtin_nontemporal_store(v.x * v.x + v.y * v.y, p + j);
  }
}

// Diagonal of the row-major vec(rho): entry (j, j) sits at j 2^n + j.
__global__ __launch_bounds__(kBlock) void k_probs_dm(const double2* __restrict__ rho, int n,
                                                     double* __restrict__ p) {
  const unsigned long long dim = 1ull << n;
  for (unsigned long long j = (unsigned long long)blockIdx.x * kBlock + threadIdx.x; j < dim;
       j += (unsigned long long)gridDim.x * kBlock)
    p[j] = rho[(j << n) + j].x;
}

// Confusion matrices of up to five qubits applied to each group of 2^g
// outcomes that differ only on those bits.  cm holds 4 entries per qubit:
// C[0][0], C[0][1], C[1][0], C[1][1] (C[r][t] = P(read r | true t)).
constexpr int kReadoutMaxGroup = 5;   // qubits per readout pass (2^5 entries per thread; 6 would need 320 VGPRs)
struct ConfGroup {
  int g;                              // qubits in the group (1..kReadoutMaxGroup)
  int bit[kReadoutMaxGroup];          // outcome bits, ascending
  double cm[kReadoutMaxGroup][4];
};

__device__ __forceinline__ unsigned long long ins0m(unsigned long long p, int q) {
  return ((p >> q) << (q + 1)) | (p & ((1ull << q) - 1ull));
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_readout(double* __restrict__ p, unsigned long long ngroups,
                                                    ConfGroup cg) {
  constexpr int D = 1 << G;
  // the group's entry offsets are ORs of these (uniform) bits, formed again
  // for the stores rather than held in 2^G registers
  unsigned long long mb[G];
#pragma unroll
  for (int i = 0; i < G; ++i) mb[i] = 1ull << cg.bit[i];
  auto off = [&](int u) {
    unsigned long long o = 0;
#pragma unroll
    for (int i = 0; i < G; ++i)
      if ((u >> i) & 1) o |= mb[i];
    return o;
  };
  for (unsigned long long gi = (unsigned long long)blockIdx.x * kBlock + threadIdx.x; gi < ngroups;
       gi += (unsigned long long)gridDim.x * kBlock) {
    unsigned long long base = gi;
#pragma unroll
    for (int i = 0; i < G; ++i) base = ins0m(base, cg.bit[i]);
    double v[D];
#pragma unroll
    for (int u = 0; u < D; ++u) v[u] = p[base | off(u)];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const double c00 = cg.cm[i][0], c01 = cg.cm[i][1], c10 = cg.cm[i][2], c11 = cg.cm[i][3];
#pragma unroll
      for (int u = 0; u < D; ++u) {
        if ((u >> i) & 1) continue;
        const double t0 = v[u], t1 = v[u | (1 << i)];
        v[u] = c00 * t0 + c01 * t1;
        v[u | (1 << i)] = c10 * t0 + c11 * t1;
      }
    }
#pragma unroll
    for (int u = 0; u < D; ++u) p[base | off(u)] = v[u];
  }
}

// Tile totals of the quantised distribution (exact integer sums).
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(const double* __restrict__ p, unsigned long long N,
                                                              unsigned long long* __restrict__ totals) {
  __shared__ unsigned long long red[kScanThreads / kWave];
  const unsigned long long t0 = (unsigned long long)blockIdx.x * kScanTile;
  unsigned long long s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const unsigned long long j = t0 + (unsigned long long)i * kScanThreads + threadIdx.x;
    if (j < N) s += quantize(p[j]);
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += red[w];
    totals[blockIdx.x] = t;
  }
}

// Exclusive prefix of the tile totals (one workgroup; each thread takes a
// contiguous chunk).
__global__ __launch_bounds__(1024) void k_scan_offsets(const unsigned long long* __restrict__ totals, int ntiles,
                                                       unsigned long long* __restrict__ offsets) {
  __shared__ unsigned long long part[1024];
  const int per = (ntiles + 1023) / 1024;
  const int b0 = threadIdx.x * per, b1 = min(ntiles, b0 + per);
  unsigned long long s = 0;
  for (int b = b0; b < b1; ++b) s += totals[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int t = 0; t < 1024; ++t) {
      const unsigned long long v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  unsigned long long run = part[threadIdx.x];
  for (int b = b0; b < b1; ++b) {
    offsets[b] = run;
    run += totals[b];
  }
}

// Inclusive integer CDF of each tile: coalesced load into LDS, each thread
// scans 16 contiguous entries, the thread totals are scanned in the
// workgroup, and the tile's offset is added.
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const double* __restrict__ p, unsigned long long N,
                                                             const unsigned long long* __restrict__ offsets,
                                                             unsigned long long* __restrict__ cdf) {
  __shared__ unsigned long long s[kScanTile + kScanTile / 16];
  __shared__ unsigned long long wsum[kScanThreads / kWave];
  auto pad = [](unsigned i) { return i + (i >> 4); };
  const unsigned long long t0 = (unsigned long long)blockIdx.x * kScanTile;
  const unsigned tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const unsigned l = i * kScanThreads + tid;
    const unsigned long long j = t0 + l;
    s[pad(l)] = j < N ? quantize(p[j]) : 0ull;
  }
  __syncthreads();
  unsigned long long loc[kScanPer];
  unsigned long long run = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    run += s[pad(tid * kScanPer + i)];
    loc[i] = run;
  }
  // inclusive scan of the thread totals within the wave, then across waves
  const int lane = tid & (kWave - 1), wave = tid / kWave;
  unsigned long long incl = run;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned long long up = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += up;
  }
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  unsigned long long before = offsets[blockIdx.x] + (incl - run);
  for (int w = 0; w < wave; ++w) before += wsum[w];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) s[pad(tid * kScanPer + i)] = before + loc[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const unsigned l = i * kScanThreads + tid;
    const unsigned long long j = t0 + l;
    if (j < N) cdf[j] = s[pad(l)];
  }
}

// One shot per thread: binary search for the smallest j with cdf[j] > target.
__global__ __launch_bounds__(kBlock) void k_sample(const unsigned long long* __restrict__ cdf, unsigned long long N,
                                                   const double* __restrict__ u, long long shots,
                                                   long long* __restrict__ out) {
  const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (s >= shots) return;
  const unsigned long long Q = cdf[N - 1];
  if (Q == 0) {
    out[s] = -1;
    return;
  }
  const double us = u[s];
  double f = us * 9007199254740992.0;   // 2^53
  if (!(f >= 0.0)) f = 0.0;
  if (f > 9007199254740991.0) f = 9007199254740991.0;
  const unsigned long long u53 = (unsigned long long)f;
  const unsigned long long hi = __umul64hi(u53, Q), lo = u53 * Q;
  const unsigned long long target = (hi << 11) | (lo >> 53);   // floor(u53 Q / 2^53) < Q
  unsigned long long lo_i = 0, hi_i = N - 1;                  // cdf[N-1] = Q > target
  while (lo_i < hi_i) {
    const unsigned long long mid = lo_i + ((hi_i - lo_i) >> 1);
    if (cdf[mid] > target) hi_i = mid;
    else lo_i = mid + 1;
  }
  out[s] = (long long)lo_i;
}

// Device scratch of the allocation-free sampler: the CDF of up to
// 2^kNoAllocMaxN outcomes, then the tile totals and tile offsets.  Each GPU
// the library runs on holds its own copy (8 MiB) until the process ends.
constexpr int kNoAllocMaxN = 20;
constexpr unsigned long long kNoAllocTiles = ((1ull << kNoAllocMaxN) + kScanTile - 1) / kScanTile;
constexpr unsigned long long kNoAllocEntries = (1ull << kNoAllocMaxN) + 2 * kNoAllocTiles;
static __device__ __align__(256) unsigned long long scratch[kNoAllocEntries];

// The device address of `scratch` on each device, looked up once per device
// with that device current (the host-side name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(unsigned long long** out) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices) return set_error(NWQ_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
  }
  *out = g_scratch_ptr[dev];
  return NWQ_OK;
}

inline unsigned grid_n(unsigned long long units, unsigned long long per, unsigned cap) {
  const unsigned long long g = (units + per - 1) / per;
  return (unsigned)(g < cap ? g : cap);
}

}  // namespace
}  // namespace nwq

using namespace nwq;

extern "C" {

int nwq_probabilities(nwq_handle h, double* probs_dev) {
  if (!h) return set_error(NWQ_EINVAL, "NULL handle");
  if (!probs_dev) return set_error(NWQ_EINVAL, "NULL probability array");
  int rc = flush_all(h);
  if (rc) return rc;
  const unsigned long long dim = 1ull << h->n;
  if (h->kind == NWQ_KIND_SV) {
    // one entry per thread up to 2^30 entries (the largest grid a dispatch takes)
    const unsigned grid = grid_n(dim, kBlock, 1u << 22);
    hipLaunchKernelGGL(k_probs_sv, dim3(grid), dim3(kBlock), 0, h->stream, h->data, dim, probs_dev,
                       grid % 8u == 0 ? 1 : 0);
  } else
    hipLaunchKernelGGL(k_probs_dm, dim3(grid_n(dim, kBlock, 1u << 16)), dim3(kBlock), 0, h->stream, h->data, h->n,
                       probs_dev);
  return check_hip(hipGetLastError(), "probabilities");
}

int nwq_readout_noise(int n, double* probs_dev, const double* confusion, void* stream) {
  if (n < 1 || n > 34) return set_error(NWQ_ERANGE, "n outside [1, 34]");
  if (!probs_dev || !confusion) return set_error(NWQ_EINVAL, "NULL argument");
  for (int q = 0; q < n; ++q) {
    const double* c = confusion + 4 * q;
    for (int i = 0; i < 4; ++i)
      if (!(c[i] >= 0.0 && c[i] <= 1.0))
        return set_error(NWQ_EINVAL, "qubit " + std::to_string(q) + ": confusion entry outside [0, 1]");
    if (std::fabs(c[0] + c[2] - 1.0) > 1e-12 || std::fabs(c[1] + c[3] - 1.0) > 1e-12)
      return set_error(NWQ_EINVAL, "qubit " + std::to_string(q) + ": confusion columns must sum to 1");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // identity matrices are skipped; the rest go up to five qubits per pass
  std::vector<int> qs;
  for (int q = 0; q < n; ++q) {
    const double* c = confusion + 4 * q;
    if (!(c[0] == 1.0 && c[3] == 1.0)) qs.push_back(q);
  }
  // The per-qubit matrices act on different bits and commute, so any grouping
  // gives the same result up to rounding.  Pass k takes qubits k, k + P,
  // k + 2P, ... of the list (P passes): the low bits, whose groups would
  // otherwise be read as short per-thread runs, are spread over the passes.
  const size_t P = (qs.size() + kReadoutMaxGroup - 1) / kReadoutMaxGroup;
  for (size_t k = 0; k < P; ++k) {
    ConfGroup cg{};
    for (size_t j = k; j < qs.size() && cg.g < kReadoutMaxGroup; j += P) {
      cg.bit[cg.g] = qs[j];
      for (int e = 0; e < 4; ++e) cg.cm[cg.g][e] = confusion[4 * qs[j] + e];
      ++cg.g;
    }
    const unsigned long long ng = 1ull << (n - cg.g);
    const dim3 grid(grid_n(ng, kBlock, 1u << 20));
    switch (cg.g) {
      case 1: hipLaunchKernelGGL(k_readout<1>, grid, dim3(kBlock), 0, s, probs_dev, ng, cg); break;
      case 2: hipLaunchKernelGGL(k_readout<2>, grid, dim3(kBlock), 0, s, probs_dev, ng, cg); break;
      case 3: hipLaunchKernelGGL(k_readout<3>, grid, dim3(kBlock), 0, s, probs_dev, ng, cg); break;
      case 4: hipLaunchKernelGGL(k_readout<4>, grid, dim3(kBlock), 0, s, probs_dev, ng, cg); break;
      default: hipLaunchKernelGGL(k_readout<5>, grid, dim3(kBlock), 0, s, probs_dev, ng, cg); break;
    }
    const int rc = check_hip(hipGetLastError(), "readout noise");
    if (rc) return rc;
  }
  return NWQ_OK;
}

size_t nwq_sample_workspace_bytes(int n) {
  if (n < 1 || n > 34) return 0;
  const unsigned long long N = 1ull << n;
  const unsigned long long nt = (N + kScanTile - 1) / kScanTile;
  return (size_t)(N + 2 * nt) * sizeof(unsigned long long);
}

}  // extern "C"

namespace {

// The scan and the search, with the workspace (CDF of 2^n entries, then the
// tile totals and the tile offsets) at `work`; arguments already checked.
int sample_launch(int n, const double* probs_dev, const double* u_dev, long long shots, long long* out_dev,
                  unsigned long long* work, hipStream_t s) {
  const unsigned long long N = 1ull << n;
  const unsigned long long ntiles = (N + kScanTile - 1) / kScanTile;
  unsigned long long* cdf = work;
  unsigned long long* totals = cdf + N;
  unsigned long long* offsets = totals + ntiles;
  hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, probs_dev, N, totals);
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, s, totals, (int)ntiles, offsets);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, probs_dev, N, offsets, cdf);
  if (shots > 0)
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((shots + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, cdf, N, u_dev,
                       shots, out_dev);
  return check_hip(hipGetLastError(), "sample");
}

int sample_args(int n, const double* probs_dev, const double* u_dev, long long shots, long long* out_dev) {
  if (n < 1 || n > 34) return set_error(NWQ_ERANGE, "n outside [1, 34]");
  if (shots < 0 || shots >= (1ll << 31)) return set_error(NWQ_EINVAL, "shot count outside [0, 2^31)");
  if (!probs_dev || (shots > 0 && (!u_dev || !out_dev))) return set_error(NWQ_EINVAL, "NULL argument");
  return NWQ_OK;
}

}  // namespace

extern "C" {

int nwq_sample(int n, const double* probs_dev, const double* u_dev, long long shots, long long* out_dev,
               void* work_dev, size_t work_bytes, void* stream) {
  int rc = sample_args(n, probs_dev, u_dev, shots, out_dev);
  if (rc) return rc;
  if (!work_dev) return set_error(NWQ_EINVAL, "NULL argument");
  if (work_bytes < nwq_sample_workspace_bytes(n)) return set_error(NWQ_EINVAL, "workspace smaller than nwq_sample_workspace_bytes(n)");
  return sample_launch(n, probs_dev, u_dev, shots, out_dev, static_cast<unsigned long long*>(work_dev),
                       static_cast<hipStream_t>(stream));
}

int nwq_sample_noalloc(int n, const double* probs_dev, const double* u_dev, long long shots, long long* out_dev,
                       void* stream) {
  if (n > kNoAllocMaxN)
    return set_error(NWQ_ERANGE, "nwq_sample_noalloc takes n <= " + std::to_string(kNoAllocMaxN) +
                                     " (its device scratch holds 2^" + std::to_string(kNoAllocMaxN) + " CDF entries)");
  int rc = sample_args(n, probs_dev, u_dev, shots, out_dev);
  if (rc) return rc;
  unsigned long long* work = nullptr;
  rc = scratch_address(&work);
  if (rc) return rc;
  return sample_launch(n, probs_dev, u_dev, shots, out_dev, work, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// Streaming ceilings: the fastest plain passes over a buffer of complex128
// entries that this chip runs, as yardsticks for the gate kernels.  An
// in-place scale reads and writes every entry at its own address (the
// access pattern of a gate pass); a copy reads one buffer and writes
// another.  Both use the gate kernels' best layout: one 16-byte entry per
// thread, non-temporal loads and stores, and workgroups ordered so that each
// of the 8 XCDs streams one contiguous eighth of the buffer.
#include "nwq_internal.h"

namespace nwq {
namespace {

typedef double vd2c __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned long long xcd_block(unsigned b, unsigned g) {
  // g is a multiple of 8: block b of the grid takes slot (b mod 8) g/8 + b/8
  return (unsigned long long)((b & 7u) * (g >> 3) + (b >> 3));
}

__global__ __launch_bounds__(kBlock) void k_scale_inplace(double2* __restrict__ a, unsigned long long first,
                                                          unsigned long long len, double s, int xcd) {
  const unsigned long long b = xcd ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const unsigned long long j = first + b * kBlock + threadIdx.x;
  if (j >= len) return;
  vd2c v = __builtin_nontemporal_load(reinterpret_cast<const vd2c*>(a + j));
  v *= s;
  __builtin_nontemporal_store(v, reinterpret_cast<vd2c*>(a + j));
}

__global__ __launch_bounds__(kBlock) void k_copy(double2* __restrict__ dst, const double2* __restrict__ src,
                                                 unsigned long long first, unsigned long long len, int xcd) {
  const unsigned long long b = xcd ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const unsigned long long j = first + b * kBlock + threadIdx.x;
  if (j >= len) return;
  const vd2c v = __builtin_nontemporal_load(reinterpret_cast<const vd2c*>(src + j));
  __builtin_nontemporal_store(v, reinterpret_cast<vd2c*>(dst + j));
}

// Launches of at most 2^30 work-items each (a dispatch packet holds its grid
// size in work-items as a 32-bit value), each starting at its own first entry.
template <typename F>
int chunked(unsigned long long len, F&& launch) {
  constexpr unsigned long long kMaxItems = 1ull << 30;
  for (unsigned long long first = 0; first < len; first += kMaxItems) {
    const unsigned long long items = len - first < kMaxItems ? len - first : kMaxItems;
    const unsigned grid = (unsigned)((items + kBlock - 1) / kBlock);
    launch(first, grid, grid % 8u == 0 ? 1 : 0);
    const int rc = check_hip(hipGetLastError(), "streaming ceiling kernel");
    if (rc) return rc;
  }
  return NWQ_OK;
}

}  // namespace
}  // namespace nwq

using namespace nwq;

extern "C" {

int nwq_stream_scale(void* buf_dev, size_t n_entries, double s, void* stream) {
  if (!buf_dev) return set_error(NWQ_EINVAL, "NULL buffer");
  double2* a = static_cast<double2*>(buf_dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned long long len = n_entries;
  return chunked(len, [&](unsigned long long first, unsigned grid, int xcd) {
    hipLaunchKernelGGL(k_scale_inplace, dim3(grid), dim3(kBlock), 0, st, a, first, len, s, xcd);
  });
}

int nwq_stream_copy(void* dst_dev, const void* src_dev, size_t n_entries, void* stream) {
  if (!dst_dev || !src_dev) return set_error(NWQ_EINVAL, "NULL buffer");
  double2* d = static_cast<double2*>(dst_dev);
  const double2* sp = static_cast<const double2*>(src_dev);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned long long len = n_entries;
  return chunked(len, [&](unsigned long long first, unsigned grid, int xcd) {
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kBlock), 0, st, d, sp, first, len, xcd);
  });
}

}  // extern "C"

// row_stats.hip -- exact per-DM-row lower median and MAD on gfx950.
//
// The boxcar S/N is normalised by each dedispersed row's median and median
// absolute deviation (sigma = 1.4826 MAD).  Both are order statistics of
// integers no larger than 255 * nchan (< 2^24 for nchan <= 65536), so they
// are found exactly by a two-level radix selection: a 4096-bin histogram of
// the high bits locates the bin holding rank floor((n-1)/2), a second
// histogram of the low bits inside that bin gives the value.  The same two
// passes over |Y - med| give the MAD.  One workgroup of 1024 threads owns a
// row; histograms live in LDS; the row is streamed with 16-byte loads when
// its start is 16-byte aligned.
#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kThreads = 1024;
constexpr int kBins = 4096;
constexpr int kPerThread = kBins / kThreads;

// Exclusive scan of one value per thread across the workgroup.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *tmp /* >= 16 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) tmp[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    uint32_t s = lane < kThreads / 64 ? tmp[lane] : 0u;
    uint32_t si = s;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const uint32_t y = __shfl_up(si, o, 64);
      if (lane >= o) si += y;
    }
    if (lane < kThreads / 64) tmp[lane] = si - s;
  }
  __syncthreads();
  const uint32_t r = tmp[wave] + inc - v;
  __syncthreads();
  return r;
}

// Finds the bin b with cum(b) <= k < cum(b) + hist[b]; writes b and cum(b)
// to out[0], out[1] (LDS), visible to all threads on return.
__device__ void locate_rank(const uint32_t *hist, uint32_t k, uint32_t *tmp, uint32_t *out) {
  const int t = threadIdx.x;
  uint32_t part = 0;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) part += hist[t * kPerThread + i];
  uint32_t below = block_exclusive_scan(part, tmp);
  if (k >= below && k < below + part) {
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const uint32_t h = hist[t * kPerThread + i];
      if (k < below + h) {
        out[0] = (uint32_t)(t * kPerThread + i);
        out[1] = below;
        break;
      }
      below += h;
    }
  }
  __syncthreads();
}

template <typename F>
__device__ __forceinline__ void for_each_value(const uint32_t *row, int64_t n, bool vec, F f) {
  if (vec) {
    const uint4 *r4 = reinterpret_cast<const uint4 *>(row);
    const int64_t n4 = n >> 2;
    for (int64_t i = threadIdx.x; i < n4; i += kThreads) {
      const uint4 v = r4[i];
      f(v.x);
      f(v.y);
      f(v.z);
      f(v.w);
    }
    for (int64_t i = (n4 << 2) + threadIdx.x; i < n; i += kThreads) f(row[i]);
  } else {
    for (int64_t i = threadIdx.x; i < n; i += kThreads) f(row[i]);
  }
}

__global__ __launch_bounds__(kThreads) void row_stats_kernel(const uint32_t *__restrict__ Y,
                                                             int64_t nout, int shift,
                                                             int32_t *__restrict__ stats) {
  __shared__ uint32_t hist[kBins];
  __shared__ uint32_t tmp[16];
  __shared__ uint32_t sel[2];
  const int d = blockIdx.x;
  const uint32_t *row = Y + (int64_t)d * nout;
  const bool vec = ((reinterpret_cast<uintptr_t>(row) & 15) == 0);
  const uint32_t k = (uint32_t)((nout - 1) / 2);
  const uint32_t fmask = (1u << shift) - 1u;
  uint32_t result[2];

  uint32_t med = 0;
  for (int pass = 0; pass < 2; ++pass) {  // pass 0: median of Y; pass 1: of |Y - med|
    const uint32_t m = med;
    const bool dev = pass == 1;
    for (int i = threadIdx.x; i < kBins; i += kThreads) hist[i] = 0u;
    __syncthreads();
    for_each_value(row, nout, vec, [&](uint32_t v) {
      const uint32_t x = dev ? (v >= m ? v - m : m - v) : v;
      atomicAdd(&hist[min(x >> shift, (uint32_t)(kBins - 1))], 1u);
    });
    __syncthreads();
    locate_rank(hist, k, tmp, sel);
    const uint32_t hb = sel[0], rank_in = k - sel[1];
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += kThreads) hist[i] = 0u;
    __syncthreads();
    for_each_value(row, nout, vec, [&](uint32_t v) {
      const uint32_t x = dev ? (v >= m ? v - m : m - v) : v;
      if ((x >> shift) == hb) atomicAdd(&hist[x & fmask], 1u);
    });
    __syncthreads();
    locate_rank(hist, rank_in, tmp, sel);
    result[pass] = (hb << shift) | sel[0];
    med = result[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[2 * (int64_t)d] = (int32_t)result[0];
    stats[2 * (int64_t)d + 1] = (int32_t)result[1];
  }
}

}  // namespace

hipError_t launch_row_stats(const uint32_t *Y, int ndm, int64_t nout, uint32_t vmax,
                            int32_t *stats, hipStream_t stream) {
  int bits = 32 - __builtin_clz(vmax | 1u);
  if (bits > 24) return hipErrorInvalidValue;
  const int shift = bits > 12 ? bits - 12 : 0;
  hipLaunchKernelGGL(row_stats_kernel, dim3(ndm), dim3(kThreads), 0, stream, Y, nout, shift,
                     stats);
  return hipGetLastError();
}

}  // namespace sps

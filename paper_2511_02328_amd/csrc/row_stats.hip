// row_stats.hip -- exact per-DM-row lower median and MAD on gfx950.
//
// The boxcar S/N is normalised by each dedispersed row's median and median
// absolute deviation (sigma = 1.4826 MAD).  Both are order statistics of
// integers no larger than 255 * nchan (< 2^24 for nchan <= 65536), so they
// are found exactly from histograms.  One workgroup of 1024 threads owns a
// row; histograms live in LDS (LDS atomics); the row is streamed with
// 16-byte loads when its start is 16-byte aligned.
//
// One read of the row in the common case: a small sample of the row (8
// runs of 512 samples spread over it) places a window of 16384 consecutive
// values around its median; one pass then builds the exact histogram of the
// window and counts the values below it.  The window's counts decide
// exactly whether it holds the median and every deviation up to the MAD;
// when it does, both follow from the window alone.  A row that fails the
// test (a sample that misleads, a MAD too wide for the window) takes the
// two-read path: a 4096-bin histogram of the high bits locates the median's
// bin and bounds the MAD, and an exact histogram over the window of bins
// around it yields both; rows wider than that window take two more reads
// (radix selection of |Y - med|).
#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kThreads = 1024;
constexpr int kBins = 4096;             // coarse histogram
constexpr int kFine = 16384;            // exact window histogram (64 KiB of LDS)
constexpr int kPerThread = kBins / kThreads;
constexpr int kSampleRuns = 8;
constexpr int kSampleRun = 4 * kThreads / kSampleRuns;  // 512: one 16-byte load per thread

// Exclusive scan of one value per thread across a workgroup of NT threads.
template <int NT = kThreads>
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *tmp /* >= NT / 64 */) {
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
    uint32_t s = lane < NT / 64 ? tmp[lane] : 0u;
    uint32_t si = s;
#pragma unroll
    for (int o = 1; o < NT / 64; o <<= 1) {
      const uint32_t y = __shfl_up(si, o, 64);
      if (lane >= o) si += y;
    }
    if (lane < NT / 64) tmp[lane] = si - s;
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

// As locate_rank over hist[0, n) for any n <= kFine: each thread owns a
// contiguous run of ceil(n / kThreads) bins.
__device__ void locate_rank_n(const uint32_t *hist, int n, uint32_t k, uint32_t *tmp,
                              uint32_t *out) {
  const int per = (n + kThreads - 1) / kThreads;
  const int lo = threadIdx.x * per;
  const int hi = min(lo + per, n);
  uint32_t part = 0;
  for (int i = lo; i < hi; ++i) part += hist[i];
  uint32_t below = block_exclusive_scan(part, tmp);
  if (k >= below && k < below + part) {
    for (int i = lo; i < hi; ++i) {
      const uint32_t h = hist[i];
      if (k < below + h) {
        out[0] = (uint32_t)i;
        out[1] = below;
        break;
      }
      below += h;
    }
  }
  __syncthreads();
}

// f(v) for every value of the row, four 16-byte loads (or four words) per
// thread in flight at a time.
template <typename F>
__device__ __forceinline__ void for_each_value(const uint32_t *row_in, int64_t n, bool vec, F f) {
  const SPS_GLOBAL uint32_t *row = gmem(row_in);
  int64_t i = threadIdx.x;
  if (vec) {
    const SPS_GLOBAL u32x4 *r4 = (const SPS_GLOBAL u32x4 *)row;
    const int64_t n4 = n >> 2;
    for (; i + 3 * kThreads < n4; i += 4 * kThreads) {
      u32x4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = r4[i + u * kThreads];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        f(v[u].x);
        f(v[u].y);
        f(v[u].z);
        f(v[u].w);
      }
    }
    for (; i < n4; i += kThreads) {
      const u32x4 v = r4[i];
      f(v.x);
      f(v.y);
      f(v.z);
      f(v.w);
    }
    for (i = (n4 << 2) + threadIdx.x; i < n; i += kThreads) f(row[i]);
  } else {
    for (; i + 3 * kThreads < n; i += 4 * kThreads) {
      uint32_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = row[i + u * kThreads];
#pragma unroll
      for (int u = 0; u < 4; ++u) f(v[u]);
    }
    for (; i < n; i += kThreads) f(row[i]);
  }
}

// Workgroup sum of one value per thread, visible to all threads on return.
__device__ uint32_t block_sum(uint32_t v, uint32_t *acc /* LDS word */) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (threadIdx.x == 0) *acc = 0u;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) atomicAdd(acc, v);
  __syncthreads();
  const uint32_t r = *acc;
  __syncthreads();
  return r;
}

// The one-read path.  Returns false (every thread alike) when the window
// does not hold the median or the deviations up to the MAD; hist is then
// free for the caller.
__device__ bool row_stats_one_pass(const uint32_t *__restrict__ row, int64_t nout, int shift,
                                   bool vec, uint32_t *hist, uint32_t *tmp, uint32_t *sel,
                                   uint32_t &med, uint32_t &mad) {
  const uint32_t k = (uint32_t)((nout - 1) / 2);
  // Sample: kSampleRuns runs of kSampleRun consecutive values, run j starting
  // at j (nout - kSampleRun) / (kSampleRuns - 1) rounded down to a multiple
  // of 4 (the whole row when it is no longer than the sample).
  for (int i = threadIdx.x; i < kBins; i += kThreads) hist[i] = 0u;
  __syncthreads();
  const SPS_GLOBAL uint32_t *g = gmem(row);
  const int64_t nsample = nout < (int64_t)(kSampleRuns * kSampleRun) ? nout
                                                                      : kSampleRuns * kSampleRun;
  auto bin = [&](uint32_t v) { atomicAdd(&hist[min(v >> shift, (uint32_t)(kBins - 1))], 1u); };
  if (nsample < (int64_t)(kSampleRuns * kSampleRun)) {
    for (int64_t i = threadIdx.x; i < nout; i += kThreads) bin(g[i]);
  } else {
    const int j = threadIdx.x / (kSampleRun / 4);
    const int64_t start = ((int64_t)j * (nout - kSampleRun) / (kSampleRuns - 1)) & ~(int64_t)3;
    const int64_t i = start + 4 * (threadIdx.x % (kSampleRun / 4));
    if (vec) {
      const u32x4 v = *(const SPS_GLOBAL u32x4 *)(g + i);
      bin(v.x);
      bin(v.y);
      bin(v.z);
      bin(v.w);
    } else {
      bin(g[i]);
      bin(g[i + 1]);
      bin(g[i + 2]);
      bin(g[i + 3]);
    }
  }
  __syncthreads();
  locate_rank(hist, (uint32_t)((nsample - 1) / 2), tmp, sel);
  // window [lo, lo + kFine) centred on the sample median's bin
  const uint32_t centre = (sel[0] << shift) + ((1u << shift) >> 1);
  const uint32_t lo = centre > (uint32_t)(kFine / 2) ? centre - (uint32_t)(kFine / 2) : 0u;
  __syncthreads();

  for (int i = threadIdx.x; i < kFine; i += kThreads) hist[i] = 0u;
  __syncthreads();
  uint32_t below = 0, inside = 0;
  for_each_value(row, nout, vec, [&](uint32_t v) {
    const uint32_t x = v - lo;
    if (x < (uint32_t)kFine) {
      atomicAdd(&hist[x], 1u);
      ++inside;
    }
    below += v < lo ? 1u : 0u;
  });
  below = block_sum(below, &sel[2]);
  inside = block_sum(inside, &sel[2]);
  if (k < below || k - below >= inside) return false;
  locate_rank_n(hist, kFine, k - below, tmp, sel);
  const uint32_t mloc = sel[0];  // median - lo
  __syncthreads();
  // Deviations m < mspan have both med - m and med + m inside the window:
  // dev[m] = #(|v - med| == m) there, formed in place after the window
  // histogram is read into registers.
  const int mspan = (int)min(mloc + 1u, (uint32_t)kFine - mloc);
  uint32_t devc[kFine / kThreads];
  uint32_t part = 0;
#pragma unroll
  for (int q = 0; q < kFine / kThreads; ++q) {
    const int m = threadIdx.x + kThreads * q;
    uint32_t c = 0;
    if (m < mspan) {
      c = hist[mloc - m];
      if (m > 0) c += hist[mloc + m];
    }
    devc[q] = c;
    part += c;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kFine / kThreads; ++q) hist[threadIdx.x + kThreads * q] = devc[q];
  // #(|v - med| < mspan) must exceed k for the MAD to lie below mspan
  if (block_sum(part, &sel[2]) < k + 1) return false;
  locate_rank_n(hist, mspan, k, tmp, sel);
  med = lo + mloc;
  mad = sel[0];
  return true;
}

// The two-read path (and the wide-row fallback beyond it).
__device__ void row_stats_two_pass(const uint32_t *__restrict__ row, int64_t nout, int shift,
                                   bool vec, uint32_t *hist, uint32_t *tmp, uint32_t *sel,
                                   uint32_t &med, uint32_t &mad) {
  // Pass 1: histogram of the high bits (4096 bins of width 2^shift) gives the
  // bin b holding the median and, from the counts around b, a bound on the
  // MAD.  Pass 2: an exact histogram of the values in the window of coarse
  // bins [b - r - 1, b + r + 1] gives the median and then the MAD, whose
  // deviations all fall inside the window.  Rows whose window would not fit
  // in LDS fall back to two more passes over |Y - med|.
  __shared__ int radius;
  const uint32_t k = (uint32_t)((nout - 1) / 2);
  const uint32_t width = 1u << shift;

  for (int i = threadIdx.x; i < kBins; i += kThreads) hist[i] = 0u;
  __syncthreads();
  for_each_value(row, nout, vec, [&](uint32_t v) {
    atomicAdd(&hist[min(v >> shift, (uint32_t)(kBins - 1))], 1u);
  });
  __syncthreads();
  locate_rank(hist, k, tmp, sel);
  const int b = (int)sel[0];
  const uint32_t below_b = sel[1];
  // Smallest r with at least k + 1 values in bins [b - r, b + r]: then every
  // |v - med| up to the MAD is at most (r + 1) 2^shift - 1.
  if (threadIdx.x == 0) {
    uint32_t cnt = hist[b];
    int r = 0;
    while (cnt < k + 1) {
      ++r;
      if (b - r >= 0) cnt += hist[b - r];
      if (b + r < kBins) cnt += hist[b + r];
    }
    radius = r;
  }
  __syncthreads();
  const int r = radius;
  const int lo_bin = max(b - r - 1, 0);
  const int hi_bin = min(b + r + 1, kBins - 1);
  const int64_t nwin = (int64_t)(hi_bin - lo_bin + 1) << shift;
  uint32_t below_lo = 0;
  if (nwin <= kFine) {
    // values below the window, from the coarse histogram
    if (threadIdx.x == 0) {
      uint32_t c = below_b;
      for (int j = lo_bin; j < b; ++j) c -= hist[j];
      sel[0] = c;
    }
    __syncthreads();
    below_lo = sel[0];
  }
  __syncthreads();

  if (nwin <= kFine) {
    const uint32_t lo = (uint32_t)lo_bin << shift;
    for (int i = threadIdx.x; i < kFine; i += kThreads) hist[i] = 0u;
    __syncthreads();
    for_each_value(row, nout, vec, [&](uint32_t v) {
      const uint32_t x = v - lo;
      if (v >= lo && x < (uint32_t)nwin) atomicAdd(&hist[x], 1u);
    });
    __syncthreads();
    locate_rank_n(hist, (int)nwin, k - below_lo, tmp, sel);
    const uint32_t mloc = sel[0];  // median - lo
    med = lo + mloc;
    __syncthreads();
    // deviation histogram: dev[m] = #(|v - med| == m) for m < mspan, formed
    // in place after the window histogram is read into registers
    const int mspan = (int)((uint32_t)(r + 1) << shift);
    // count(|v - med| <= m) >= k + 1 first happens at m = MAD <= mspan - 1.
    uint32_t devc[kFine / kThreads];
#pragma unroll
    for (int q = 0; q < kFine / kThreads; ++q) {
      const int m = threadIdx.x + kThreads * q;
      uint32_t c = 0;
      if (m < mspan) {
        const int64_t a = (int64_t)mloc - m, z = (int64_t)mloc + m;
        if (a >= 0 && a < nwin) c += hist[a];
        if (m > 0 && z >= 0 && z < nwin) c += hist[z];
      }
      devc[q] = c;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kFine / kThreads; ++q) hist[threadIdx.x + kThreads * q] = devc[q];
    __syncthreads();
    locate_rank_n(hist, mspan, k, tmp, sel);
    mad = sel[0];
  } else {
    // Wide row: radix selection of the median's low bits, then of |Y - med|.
    const uint32_t fmask = width - 1u;
    for (int i = threadIdx.x; i < kBins; i += kThreads) hist[i] = 0u;
    __syncthreads();
    for_each_value(row, nout, vec, [&](uint32_t v) {
      if ((v >> shift) == (uint32_t)b) atomicAdd(&hist[v & fmask], 1u);
    });
    __syncthreads();
    locate_rank(hist, k - below_b, tmp, sel);
    med = ((uint32_t)b << shift) | sel[0];
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += kThreads) hist[i] = 0u;
    __syncthreads();
    const uint32_t m0 = med;
    for_each_value(row, nout, vec, [&](uint32_t v) {
      const uint32_t x = v >= m0 ? v - m0 : m0 - v;
      atomicAdd(&hist[min(x >> shift, (uint32_t)(kBins - 1))], 1u);
    });
    __syncthreads();
    locate_rank(hist, k, tmp, sel);
    const uint32_t hb = sel[0], rank_in = k - sel[1];
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += kThreads) hist[i] = 0u;
    __syncthreads();
    for_each_value(row, nout, vec, [&](uint32_t v) {
      const uint32_t x = v >= m0 ? v - m0 : m0 - v;
      if ((x >> shift) == hb) atomicAdd(&hist[x & fmask], 1u);
    });
    __syncthreads();
    locate_rank(hist, rank_in, tmp, sel);
    mad = (hb << shift) | sel[0];
  }
}

// Median and MAD of one row (the whole workgroup), written to out[0..1].
__device__ void row_stats_row(const uint32_t *__restrict__ row, int64_t nout, int shift,
                              int32_t *__restrict__ out) {
  __shared__ uint32_t hist[kFine];
  __shared__ uint32_t tmp[16];
  __shared__ uint32_t sel[3];
  const bool vec = ((reinterpret_cast<uintptr_t>(row) & 15) == 0);
  uint32_t med, mad;
  if (!row_stats_one_pass(row, nout, shift, vec, hist, tmp, sel, med, mad)) {
    __syncthreads();
    row_stats_two_pass(row, nout, shift, vec, hist, tmp, sel, med, mad);
  }
  if (threadIdx.x == 0) {
    out[0] = (int32_t)med;
    out[1] = (int32_t)mad;
  }
}

// ---------------------------------------------------------------------------
// Short rows (nout <= kShortMax): the fixed cost of the path above (clearing
// and scanning 4096- and 16384-bin histograms with 16 waves) outweighs a row
// of a few thousand values.  Here one workgroup of 4 waves owns a row, holds
// it in registers (16 values per thread, read once) and centres a window of
// kShortWin unit bins on the row's mean.  The same exact tests as the
// one-read path decide whether the window holds the median and every
// deviation up to the MAD; rows that fail them (a spread wider than the
// window) take an exact radix selection over the registers, 8 bits a pass.

constexpr int kShortThreads = 256;
constexpr int kShortPer = 16;                          // values per thread
constexpr int kShortMax = kShortThreads * kShortPer;   // 4096
constexpr int kShortWin = 4096;                        // window bins (16 KiB)
constexpr int kShortBinsPer = kShortWin / kShortThreads;
static_assert(kShortBinsPer % 4 == 0, "bins are read as 16-byte vectors");
static_assert(kShortThreads == 256, "one radix bin per thread");

// Value j of thread t is row element 1024 (j / 4) + 4 t + j % 4: one 16-byte
// load per group of four, coalesced across the workgroup.
__device__ __forceinline__ int short_index(int j) {
  return (j >> 2) * (4 * kShortThreads) + 4 * (int)threadIdx.x + (j & 3);
}

// The k-th smallest (from 0) of key(v) over the row's n values, keys < 2^24,
// by three 8-bit radix passes over a 256-bin histogram.  The rare path: it
// reads the row again rather than keep the values live in registers.
template <typename Key>
__device__ uint32_t short_select(const SPS_GLOBAL uint32_t *row, int n, uint32_t k, Key key,
                                 uint32_t *hist, uint32_t *tmp, uint32_t *sel) {
  uint32_t prefix = 0;
#pragma unroll 1
  for (int sh = 16; sh >= 0; sh -= 8) {
    hist[threadIdx.x] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kShortThreads) {
      const uint32_t x = key(row[i]);
      if ((x >> (sh + 8)) == (prefix >> (sh + 8))) atomicAdd(&hist[(x >> sh) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t c = hist[threadIdx.x];
    const uint32_t below = block_exclusive_scan<kShortThreads>(c, tmp);
    if (k >= below && k < below + c) {
      sel[0] = threadIdx.x;
      sel[1] = below;
    }
    __syncthreads();
    prefix |= sel[0] << sh;
    k -= sel[1];
    __syncthreads();
  }
  return prefix;
}

// Exact median and MAD by radix selection, packed as med | mad << 32 (kept
// out of line: the fast path's registers stay free of it).
__device__ __noinline__ uint64_t short_select_both(const SPS_GLOBAL uint32_t *row, int n,
                                                   uint32_t k, uint32_t *hist, uint32_t *tmp,
                                                   uint32_t *sel) {
  const uint32_t med = short_select(row, n, k, [](uint32_t x) { return x; }, hist, tmp, sel);
  const uint32_t mad = short_select(
      row, n, k, [med](uint32_t x) { return x >= med ? x - med : med - x; }, hist, tmp, sel);
  return (uint64_t)med | ((uint64_t)mad << 32);
}

// Wave-level sum and inclusive scan (64 lanes).
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_inclusive(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

// Each reduction below has LDS slots of its own (one word per wave), written
// once per row, so one barrier completes it and none has to guard reuse.
struct ShortSlots {
  uint32_t mean[4], count[4], hscan[4];
};

// Median and MAD of a row of 1 <= n <= kShortMax values (the whole
// workgroup), written to out[0..1].
__device__ void row_stats_short_row(const uint32_t *__restrict__ row_in, int n,
                                    int32_t *__restrict__ out) {
  __shared__ __align__(16) uint32_t hist[kShortWin];
  __shared__ uint32_t tmp[kShortThreads / 64];
  __shared__ uint32_t sel[2];
  __shared__ ShortSlots sl;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const SPS_GLOBAL uint32_t *row = gmem(row_in);
  const bool vec = ((reinterpret_cast<uintptr_t>(row_in) & 15) == 0);
  uint32_t v[kShortPer];
#pragma unroll
  for (int g = 0; g < kShortPer / 4; ++g) {
    const int i = short_index(4 * g);
    if (vec && i + 3 < n) {
      const u32x4 q = *(const SPS_GLOBAL u32x4 *)(row + i);
      v[4 * g] = q.x;
      v[4 * g + 1] = q.y;
      v[4 * g + 2] = q.z;
      v[4 * g + 3] = q.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[4 * g + e] = i + e < n ? row[i + e] : 0u;
    }
  }
  // the window is cleared under the same barrier as the mean's sum
#pragma unroll
  for (int q = 0; q < kShortBinsPer; ++q) hist[threadIdx.x + kShortThreads * q] = 0u;
  const uint32_t k = (uint32_t)(n - 1) / 2;
  // window [lo, lo + kShortWin) around the mean (from the values' top 16 of
  // 24 bits: 4096 of them sum below 2^28)
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kShortPer; ++j) s += v[j] >> 8;
  s = wave_sum(s);
  if (lane == 0) sl.mean[wave] = s;
  __syncthreads();
  s = sl.mean[0] + sl.mean[1] + sl.mean[2] + sl.mean[3];
  const uint32_t centre = (uint32_t)(((uint64_t)s << 8) / (uint32_t)n) + 128u;
  const uint32_t lo = centre > (uint32_t)(kShortWin / 2) ? centre - (uint32_t)(kShortWin / 2) : 0u;
  uint32_t below = 0, inside = 0;
#pragma unroll
  for (int j = 0; j < kShortPer; ++j) {
    if (short_index(j) < n) {
      const uint32_t x = v[j] - lo;
      if (x < (uint32_t)kShortWin) {
        atomicAdd(&hist[x], 1u);
        ++inside;
      }
      below += v[j] < lo ? 1u : 0u;
    }
  }
  // both counts are at most 4096: one sum carries the two; its barrier also
  // completes the histogram
  uint32_t bi = wave_sum(below | (inside << 16));
  if (lane == 0) sl.count[wave] = bi;
  __syncthreads();
  bi = sl.count[0] + sl.count[1] + sl.count[2] + sl.count[3];
  below = bi & 0xFFFFu;
  inside = bi >> 16;
  uint32_t med = 0, mad = 0;
  bool ok = k >= below && k - below < inside;  // the window holds the median
  if (ok) {
    // The window's counts become their inclusive prefix P in place: thread t
    // owns bins [t kShortBinsPer, (t + 1) kShortBinsPer).
    const int b0 = threadIdx.x * kShortBinsPer;
    uint32_t h[kShortBinsPer];
#pragma unroll
    for (int q = 0; q < kShortBinsPer / 4; ++q) {
      const uint4 w = *reinterpret_cast<const uint4 *>(&hist[b0 + 4 * q]);
      h[4 * q] = w.x;
      h[4 * q + 1] = w.y;
      h[4 * q + 2] = w.z;
      h[4 * q + 3] = w.w;
    }
#pragma unroll
    for (int q = 1; q < kShortBinsPer; ++q) h[q] += h[q - 1];
    const uint32_t part = h[kShortBinsPer - 1];
    const uint32_t inc = wave_inclusive(part);
    if (lane == 63) sl.hscan[wave] = inc;
    __syncthreads();
    uint32_t run = inc - part;
    for (int w = 0; w < wave; ++w) run += sl.hscan[w];
#pragma unroll
    for (int q = 0; q < kShortBinsPer / 4; ++q)
      *reinterpret_cast<uint4 *>(&hist[b0 + 4 * q]) =
          make_uint4(h[4 * q] + run, h[4 * q + 1] + run, h[4 * q + 2] + run, h[4 * q + 3] + run);
    // the median's bin: the first whose prefix exceeds its rank in the window
    const uint32_t kk = k - below;
    if (kk >= run && kk < run + part) {
      int q = 0;  // prefixes are non-decreasing: count those not above kk
#pragma unroll
      for (int j = 0; j < kShortBinsPer; ++j) q += run + h[j] <= kk ? 1 : 0;
      sel[0] = (uint32_t)(b0 + q);
    }
    __syncthreads();
    const int mloc = (int)sel[0];  // median - lo
    // #(|v - med| <= m) = P[mloc + m] - P[mloc - m - 1] for m < mspan, where
    // med +- m both lie in the window.  The MAD is the least m at which it
    // exceeds k: one wave finds it in two steps, m = 33 l + 32 over the lanes
    // l (33 is odd: the 64 reads fall in distinct banks, and 64 x 33 covers
    // the widest mspan, 2048), then the 33 values below the first hit.
    const int mspan = min(mloc + 1, kShortWin - mloc);
    if (wave == 0) {
      auto reaches = [&](int m) {
        m = min(m, mspan - 1);
        const uint32_t lo_p = m < mloc ? hist[mloc - m - 1] : 0u;
        return hist[mloc + m] - lo_p >= k + 1;
      };
      const uint64_t b1 = __ballot(reaches(33 * lane + 32));
      if (b1 == 0) {
        // fewer than k + 1 deviations below mspan: the MAD lies outside
        if (lane == 0) sel[1] = 0xFFFFFFFFu;
      } else {
        const int f = __ffsll((unsigned long long)b1) - 1;
        const uint64_t b2 = __ballot(lane < 33 && reaches(33 * f + lane));
        if (lane == 0) sel[1] = (uint32_t)(33 * f + __ffsll((unsigned long long)b2) - 1);
      }
    }
    __syncthreads();
    ok = sel[1] != 0xFFFFFFFFu;
    med = lo + (uint32_t)mloc;
    mad = sel[1];
  }
  if (!ok) {
    __syncthreads();
    const uint64_t r = short_select_both(row, n, k, hist, tmp, sel);
    med = (uint32_t)r;
    mad = (uint32_t)(r >> 32);
  }
  if (threadIdx.x == 0) {
    out[0] = (int32_t)med;
    out[1] = (int32_t)mad;
  }
}

__global__ __launch_bounds__(kShortThreads) void row_stats_short_kernel(
    const uint32_t *__restrict__ Y, int nout, int32_t *__restrict__ stats) {
  const int d = blockIdx.x;
  row_stats_short_row(Y + (int64_t)d * nout, nout, stats + 2 * (int64_t)d);
}

// One workgroup per (beam, DM row) of a batch whose beams are all short.
__global__ __launch_bounds__(kShortThreads) void row_stats_short_batch_kernel(
    const BeamWork *__restrict__ beams, int ndm) {
  const int b = blockIdx.x / ndm;
  const int d = blockIdx.x - b * ndm;
  const BeamWork &bw = beams[b];
  row_stats_short_row(bw.Y + (int64_t)d * bw.nout, (int)bw.nout, bw.stats + 2 * (int64_t)d);
}

__global__ __launch_bounds__(kThreads) void row_stats_kernel(const uint32_t *__restrict__ Y,
                                                             int64_t nout, int shift,
                                                             int32_t *__restrict__ stats) {
  const int d = blockIdx.x;
  row_stats_row(Y + (int64_t)d * nout, nout, shift, stats + 2 * (int64_t)d);
}

// One workgroup per (beam, DM row) of a batch.
__global__ __launch_bounds__(kThreads) void row_stats_batch_kernel(
    const BeamWork *__restrict__ beams, int ndm, int shift) {
  const int b = blockIdx.x / ndm;
  const int d = blockIdx.x - b * ndm;
  const BeamWork &bw = beams[b];
  row_stats_row(bw.Y + (int64_t)d * bw.nout, bw.nout, shift, bw.stats + 2 * (int64_t)d);
}

}  // namespace

static int stats_shift(uint32_t vmax) {
  const int bits = 32 - __builtin_clz(vmax | 1u);
  return bits > 24 ? -1 : (bits > 12 ? bits - 12 : 0);
}

hipError_t launch_row_stats_batch(const BeamWork *beams, int nbeams, int ndm, uint32_t vmax,
                                  int64_t max_nout, hipStream_t stream) {
  const int shift = stats_shift(vmax);
  if (shift < 0 || (int64_t)nbeams * ndm > 0x7FFFFFFF || max_nout < 1)
    return hipErrorInvalidValue;
  if (max_nout <= kShortMax)
    hipLaunchKernelGGL(row_stats_short_batch_kernel, dim3(nbeams * ndm), dim3(kShortThreads), 0,
                       stream, beams, ndm);
  else
    hipLaunchKernelGGL(row_stats_batch_kernel, dim3(nbeams * ndm), dim3(kThreads), 0, stream,
                       beams, ndm, shift);
  return hipGetLastError();
}

hipError_t launch_row_stats(const uint32_t *Y, int ndm, int64_t nout, uint32_t vmax,
                            int32_t *stats, hipStream_t stream) {
  const int shift = stats_shift(vmax);
  if (shift < 0 || nout < 1) return hipErrorInvalidValue;
  if (nout <= kShortMax)
    hipLaunchKernelGGL(row_stats_short_kernel, dim3(ndm), dim3(kShortThreads), 0, stream, Y,
                       (int)nout, stats);
  else
    hipLaunchKernelGGL(row_stats_kernel, dim3(ndm), dim3(kThreads), 0, stream, Y, nout, shift,
                       stats);
  return hipGetLastError();
}

}  // namespace sps

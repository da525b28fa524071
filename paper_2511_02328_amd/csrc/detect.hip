// detect.hip -- candidate detection on the boxcar S/N plane (gfx950).
//
// Stage 1 (tile_peaks_kernel): one workgroup per tile of tile_dm x tile_t
// finds the tile's largest S/N.  Ties are broken towards the smallest t, then
// the smallest d, by reducing a 64-bit key: the S/N's bits mapped to an
// order-preserving unsigned integer in the high word, the complement of the
// in-tile position t_local * tile_dm + d_local in the low word.
// Stage 2 (select_nms_kernel): one workgroup gathers the peaks at or above
// the threshold into LDS, sorts them (bitonic) by S/N descending, then t,
// then d, and accepts them greedily unless an accepted one lies within the
// suppression radius.  The candidate record carries DM, arrival time at the
// top of the band, width and S/N (ASTROFLOW Sec. 2).
#include <float.h>
#include <limits.h>

#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kTileThreads = 256;
constexpr int kNmsThreads = 1024;

__device__ __forceinline__ uint32_t ordered_bits(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ uint64_t max_u64(uint64_t a, uint64_t b) { return a > b ? a : b; }

__device__ __forceinline__ void tile_peak(const float *__restrict__ snr,
                                          const uint8_t *__restrict__ best, int ndm,
                                          int64_t nout, int tile_dm, int64_t tile_t, int64_t ntt,
                                          int64_t tile, TilePeak *__restrict__ out) {
  __shared__ uint64_t red[kTileThreads / 64];
  const int a = (int)(tile / ntt);
  const int64_t b = tile - (int64_t)a * ntt;
  const int d0 = a * tile_dm;
  const int d1 = min(d0 + tile_dm, ndm);
  const int64_t t0 = b * tile_t;
  const int64_t t1 = t0 + tile_t < nout ? t0 + tile_t : nout;

  uint64_t key = 0;
  // 16-byte loads when every row segment of the tile is 16-byte aligned:
  // four keys per load, four loads of a row in flight per thread
  const bool vec = ((reinterpret_cast<uintptr_t>(snr) & 15) == 0) && nout % 4 == 0 &&
                   tile_t % 4 == 0;
  const int64_t nq = vec ? (t1 - t0) / 4 : 0;
#pragma unroll 2
  for (int d = d0; d < d1; ++d) {
    const SPS_GLOBAL float *row = gmem(snr + (int64_t)d * nout);
    const uint32_t dl = (uint32_t)(d - d0);
    const SPS_GLOBAL f32x4 *rv = (const SPS_GLOBAL f32x4 *)(row + t0);
#pragma unroll 4
    for (int64_t q = threadIdx.x; q < nq; q += kTileThreads) {
      const f32x4 v = rv[q];
      const uint32_t p0 = (uint32_t)(4 * q) * (uint32_t)tile_dm + dl;
      key = max_u64(key, ((uint64_t)ordered_bits(v.x) << 32) | (uint64_t)(~p0));
      key = max_u64(key, ((uint64_t)ordered_bits(v.y) << 32) | (uint64_t)(~(p0 + tile_dm)));
      key = max_u64(key, ((uint64_t)ordered_bits(v.z) << 32) | (uint64_t)(~(p0 + 2 * tile_dm)));
      key = max_u64(key, ((uint64_t)ordered_bits(v.w) << 32) | (uint64_t)(~(p0 + 3 * tile_dm)));
    }
    for (int64_t t = t0 + 4 * nq + threadIdx.x; t < t1; t += kTileThreads) {
      const uint32_t pos = (uint32_t)((t - t0) * tile_dm + (d - d0));
      const uint64_t k = ((uint64_t)ordered_bits(row[t]) << 32) | (uint64_t)(~pos);
      key = max_u64(key, k);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)key, o, 64);
    const uint32_t hi = __shfl_xor((uint32_t)(key >> 32), o, 64);
    key = max_u64(key, ((uint64_t)hi << 32) | lo);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kTileThreads / 64; ++w) key = max_u64(key, red[w]);
    const uint32_t pos = ~(uint32_t)key;
    int64_t tl = pos / (uint32_t)tile_dm;
    int dl = (int)(pos - (uint32_t)tl * (uint32_t)tile_dm);
    if (key == 0 || t0 + tl >= t1 || d0 + dl >= d1) {  // only if every value was NaN
      tl = 0;
      dl = 0;
    }
    const int d = d0 + dl;
    const int64_t t = t0 + tl;
    TilePeak p;
    p.snr = gmem(snr)[(int64_t)d * nout + t];
    p.d = d;
    p.t = (int32_t)t;
    p.w = gmem(best)[(int64_t)d * nout + t];
    *out = p;
  }
}

__global__ __launch_bounds__(kTileThreads) void tile_peaks_kernel(
    const float *__restrict__ snr, const uint8_t *__restrict__ best, int ndm, int64_t nout,
    int tile_dm, int64_t tile_t, int64_t ntt, TilePeak *__restrict__ peaks) {
  tile_peak(snr, best, ndm, nout, tile_dm, tile_t, ntt, blockIdx.x, peaks + blockIdx.x);
}

__global__ __launch_bounds__(kTileThreads) void tile_peaks_batch_kernel(
    const BeamWork *__restrict__ beams, int nbeams, int ndm, int tile_dm, int64_t tile_t,
    TilePeak *__restrict__ peaks) {
  const int64_t blk = blockIdx.x;
  const BeamWork &bw = beams[find_beam<&BeamWork::tp_begin>(beams, nbeams, blk)];
  tile_peak(bw.snr, bw.best, ndm, bw.nout, tile_dm, tile_t, bw.ntt, blk - bw.tp_begin,
            peaks + blk);
}

// True if a comes before b: S/N descending, then t, then d.
__device__ __forceinline__ bool before(const TilePeak &a, const TilePeak &b) {
  if (a.snr != b.snr) return a.snr > b.snr;
  if (a.t != b.t) return a.t < b.t;
  return a.d < b.d;
}

__device__ __forceinline__ bool near(const TilePeak &a, const TilePeak &b, int nms_dm,
                                     int64_t nms_t) {
  const int64_t dd = (int64_t)a.d - b.d, dt = (int64_t)a.t - b.t;
  return (dd < 0 ? -dd : dd) <= nms_dm && (dt < 0 ? -dt : dt) <= nms_t;
}

// Selection and greedy suppression in one workgroup.  Offers (tile peaks at
// or above the threshold) are gathered into LDS and bitonic-sorted into
// "before" order.  Greedy acceptance in that order has a unique result; when
// the suppression radius spans few tiles it is computed in parallel rounds:
// an offer is rejected once an accepted, earlier, nearby offer exists, and
// accepted once every earlier nearby offer is rejected.  Each round decides
// at least the earliest undecided offer, and decisions are final, so reading
// neighbours' states while they change is safe.  Otherwise the offers are
// scanned one by one.
__device__ void select_nms(const TilePeak *__restrict__ peaks, int64_t npeaks, int ntd,
                           int64_t ntt, int tile_dm, int64_t tile_t, float threshold, int nms_dm,
                           int64_t nms_t, TilePeak *__restrict__ out,
                           int32_t *__restrict__ status) {
  __shared__ TilePeak offer[kMaxOffers];
  __shared__ int16_t aux[kMaxOffers];  // tile -> offer rank, or the accepted list
  __shared__ uint8_t state[kMaxOffers];  // 0 undecided, 1 accepted, 2 rejected
  __shared__ int count;
  __shared__ int naccept;
  __shared__ uint32_t tmp[kNmsThreads / 64];
  const int tid = threadIdx.x;
  if (tid == 0) {
    count = 0;
    naccept = 0;
  }
  __syncthreads();
  for (int64_t i = tid; i < npeaks; i += kNmsThreads) {
    const TilePeak p = peaks[i];
    if (p.snr >= threshold) {
      const int slot = atomicAdd(&count, 1);
      if (slot < kMaxOffers) offer[slot] = p;
    }
  }
  __syncthreads();
  const int n = count;
  if (n > kMaxOffers) {
    if (tid == 0) {
      status[0] = n;
      status[1] = 0;
      status[2] = 1;
    }
    return;
  }
  int npow = 1;
  while (npow < n) npow <<= 1;
  for (int i = n + tid; i < npow; i += kNmsThreads) {
    TilePeak s;
    s.snr = -FLT_MAX;
    s.d = INT_MAX;
    s.t = INT_MAX;
    s.w = 0xFF;
    offer[i] = s;
  }
  __syncthreads();
  for (int size = 2; size <= npow; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < npow / 2; i += kNmsThreads) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const TilePeak x = offer[lo], y = offer[hi];
        if (up ? before(y, x) : before(x, y)) {
          offer[lo] = y;
          offer[hi] = x;
        }
      }
      __syncthreads();
    }
  }

  const int span_d = (nms_dm + tile_dm - 1) / tile_dm;
  const int64_t span_t = (nms_t + tile_t - 1) / tile_t;
  const bool grid = npeaks <= kMaxOffers && (2 * span_d + 1) * (2 * span_t + 1) <= 49;
  if (grid) {
    for (int i = tid; i < (int)npeaks; i += kNmsThreads) aux[i] = -1;
    for (int i = tid; i < n; i += kNmsThreads) state[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += kNmsThreads) {
      const TilePeak c = offer[i];
      aux[(int64_t)(c.d / tile_dm) * ntt + c.t / tile_t] = (int16_t)i;
    }
    __syncthreads();
    int undecided = 1;
    while (undecided) {
      int mine = 0;
      for (int i = tid; i < n; i += kNmsThreads) {
        if (state[i] != 0) continue;
        const TilePeak c = offer[i];
        const int a = c.d / tile_dm;
        const int64_t b = c.t / tile_t;
        bool blocked = false, rejected = false;
        for (int da = -span_d; da <= span_d && !rejected; ++da) {
          const int aa = a + da;
          if (aa < 0 || aa >= ntd) continue;
          for (int64_t db = -span_t; db <= span_t; ++db) {
            const int64_t bb = b + db;
            if (bb < 0 || bb >= ntt) continue;
            const int j = aux[(int64_t)aa * ntt + bb];
            if (j < 0 || j >= i) continue;
            if (!near(c, offer[j], nms_dm, nms_t)) continue;
            const uint8_t sj = *(volatile uint8_t *)&state[j];
            if (sj == 1) {
              rejected = true;
              break;
            }
            if (sj == 0) blocked = true;
          }
        }
        if (rejected)
          state[i] = 2;
        else if (!blocked)
          state[i] = 1;
        else
          mine = 1;
      }
      undecided = __syncthreads_or(mine);
    }
    // Accepted offers in order: block-wide exclusive scan of per-thread counts
    // over contiguous runs.
    const int per = (n + kNmsThreads - 1) / kNmsThreads;
    const int lo = tid * per, hi = min(lo + per, n);
    uint32_t cnt = 0;
    for (int i = lo; i < hi; ++i) cnt += state[i] == 1;
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t inc = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) tmp[wave] = inc;
    __syncthreads();
    uint32_t pos = inc - cnt;
    for (int w = 0; w < wave; ++w) pos += tmp[w];
    for (int i = lo; i < hi; ++i)
      if (state[i] == 1) out[pos++] = offer[i];
    if (tid == kNmsThreads - 1) naccept = (int)pos;
    __syncthreads();
  } else {
    for (int i = 0; i < n; ++i) {
      const TilePeak c = offer[i];
      const int na = naccept;
      bool hit = false;
      for (int j = tid; j < na; j += kNmsThreads)
        if (near(c, offer[(uint16_t)aux[j]], nms_dm, nms_t)) hit = true;
      const int any = __syncthreads_or(hit);
      if (!any && tid == 0) {
        aux[na] = (int16_t)i;
        naccept = na + 1;
      }
      __syncthreads();
    }
    const int na = naccept;
    for (int j = tid; j < na; j += kNmsThreads) out[j] = offer[(uint16_t)aux[j]];
  }
  if (tid == 0) {
    status[0] = n;
    status[1] = naccept;
    status[2] = 0;
  }
}

__global__ __launch_bounds__(kNmsThreads) void select_nms_kernel(
    const TilePeak *__restrict__ peaks, int64_t npeaks, int ntd, int64_t ntt, int tile_dm,
    int64_t tile_t, float threshold, int nms_dm, int64_t nms_t, TilePeak *__restrict__ out,
    int32_t *__restrict__ status) {
  select_nms(peaks, npeaks, ntd, ntt, tile_dm, tile_t, threshold, nms_dm, nms_t, out, status);
}

// One workgroup per beam: accepted peaks of beam b go to out[b * kMaxOffers ...]
// and its status to status[4 b ...].
__global__ __launch_bounds__(kNmsThreads) void select_nms_batch_kernel(
    const BeamWork *__restrict__ beams, int ndm, int tile_dm, int64_t tile_t, float threshold,
    int nms_dm, int64_t nms_t, const TilePeak *__restrict__ peaks, TilePeak *__restrict__ out,
    int32_t *__restrict__ status) {
  const int b = blockIdx.x;
  const BeamWork &bw = beams[b];
  const int ntd = (ndm + tile_dm - 1) / tile_dm;
  select_nms(peaks + bw.tp_begin, (int64_t)ntd * bw.ntt, ntd, bw.ntt, tile_dm, tile_t, threshold,
             nms_dm, nms_t, out + (int64_t)b * kMaxOffers, status + 4 * (int64_t)b);
}

}  // namespace

hipError_t launch_tile_peaks(const float *snr, const uint8_t *best, int ndm, int64_t nout,
                             int tile_dm, int64_t tile_t, TilePeak *peaks,
                             hipStream_t stream) {
  const int64_t ntd = (ndm + tile_dm - 1) / tile_dm;
  const int64_t ntt = (nout + tile_t - 1) / tile_t;
  if (ntd * ntt > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tile_peaks_kernel, dim3((unsigned)(ntd * ntt)), dim3(kTileThreads), 0,
                     stream, snr, best, ndm, nout, tile_dm, tile_t, ntt, peaks);
  return hipGetLastError();
}

hipError_t launch_select_nms(const TilePeak *peaks, int ndm, int64_t nout, int tile_dm,
                             int64_t tile_t, float threshold, int nms_dm, int64_t nms_t,
                             TilePeak *out, int32_t *status, hipStream_t stream) {
  const int ntd = (ndm + tile_dm - 1) / tile_dm;
  const int64_t ntt = (nout + tile_t - 1) / tile_t;
  hipLaunchKernelGGL(select_nms_kernel, dim3(1), dim3(kNmsThreads), 0, stream, peaks,
                     (int64_t)ntd * ntt, ntd, ntt, tile_dm, tile_t, threshold, nms_dm, nms_t, out,
                     status);
  return hipGetLastError();
}

hipError_t launch_detect_batch(const BeamWork *beams, int nbeams, int ndm, int64_t total_tiles,
                               int tile_dm, int64_t tile_t, float threshold, int nms_dm,
                               int64_t nms_t, TilePeak *peaks, TilePeak *out, int32_t *status,
                               hipStream_t stream) {
  if (total_tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tile_peaks_batch_kernel, dim3((unsigned)total_tiles), dim3(kTileThreads), 0,
                     stream, beams, nbeams, ndm, tile_dm, tile_t, peaks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(select_nms_batch_kernel, dim3(nbeams), dim3(kNmsThreads), 0, stream, beams,
                     ndm, tile_dm, tile_t, threshold, nms_dm, nms_t, peaks, out, status);
  return hipGetLastError();
}

}  // namespace sps

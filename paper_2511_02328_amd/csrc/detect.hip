// detect.hip -- candidate detection on the boxcar S/N plane (gfx950).
//
// Stage 1 (tile_peaks_kernel): one workgroup per tile of tile_dm x tile_t
// finds the tile's largest S/N.  Ties are broken towards the smallest t, then
// the smallest d, by reducing a 64-bit key: the S/N's bits mapped to an
// order-preserving unsigned integer in the high word, the complement of the
// in-tile position t_local * tile_dm + d_local in the low word.
// Stage 2 (select_nms_kernel): one workgroup gathers the peaks at or above
// the threshold, sorts them (bitonic) by S/N descending, then t, then d, and
// accepts them greedily unless an accepted one lies within the suppression
// radius.  Offers that fit stay in LDS; any larger number goes through the
// global arrays of the plane's detection scratch.  The candidate record
// carries DM, arrival time at the top of the band, width and S/N (ASTROFLOW
// Sec. 2).
#include <float.h>
#include <limits.h>

#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kTileThreads = 256;
constexpr int kNmsThreads = 1024;

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
      key = max_u64(key, ((uint64_t)snr_key_bits(v.x) << 32) | (uint64_t)(~p0));
      key = max_u64(key, ((uint64_t)snr_key_bits(v.y) << 32) | (uint64_t)(~(p0 + tile_dm)));
      key = max_u64(key, ((uint64_t)snr_key_bits(v.z) << 32) | (uint64_t)(~(p0 + 2 * tile_dm)));
      key = max_u64(key, ((uint64_t)snr_key_bits(v.w) << 32) | (uint64_t)(~(p0 + 3 * tile_dm)));
    }
    for (int64_t t = t0 + 4 * nq + threadIdx.x; t < t1; t += kTileThreads) {
      const uint32_t pos = (uint32_t)((t - t0) * tile_dm + (d - d0));
      const uint64_t k = ((uint64_t)snr_key_bits(row[t]) << 32) | (uint64_t)(~pos);
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

__device__ __forceinline__ TilePeak sentinel() {
  TilePeak s;
  s.snr = -FLT_MAX;
  s.d = INT_MAX;
  s.t = INT_MAX;
  s.w = 0xFF;
  return s;
}

// One compare-exchange step (k, j) of a bitonic sorting network into
// "before" order over the pairs of a[0 .. n2 * 2); idx0: global index of
// a[0] (the direction of a pair depends on its global index).
__device__ __forceinline__ void bitonic_step(TilePeak *a, int64_t n2, int64_t idx0, int64_t k,
                                             int64_t j) {
  for (int64_t i = threadIdx.x; i < n2; i += kNmsThreads) {
    const int64_t lo = 2 * i - (i & (j - 1));
    const int64_t hi = lo + j;
    const bool up = ((idx0 + lo) & k) == 0;
    const TilePeak x = a[lo], y = a[hi];
    if (up ? before(y, x) : before(x, y)) {
      a[lo] = y;
      a[hi] = x;
    }
  }
}

// Sorts a[0 .. npow) (npow a power of two) into "before" order with one
// workgroup; lds: kMaxOffers records.  Up to kMaxOffers records the whole
// network runs in LDS.  Beyond, blocks of kMaxOffers are sorted in LDS
// (alternating directions, as the network's first log2(kMaxOffers) stages
// leave them), then every merge stage takes its strides >= kMaxOffers on the
// global array and its shorter strides block by block in LDS.
__device__ void sort_offers(TilePeak *a, int64_t npow, TilePeak *lds) {
  constexpr int64_t B = kMaxOffers;
  const int tid = threadIdx.x;
  if (npow <= B) {
    for (int64_t i = tid; i < npow; i += kNmsThreads) lds[i] = a[i];
    __syncthreads();
    for (int64_t k = 2; k <= npow; k <<= 1)
      for (int64_t j = k >> 1; j > 0; j >>= 1) {
        bitonic_step(lds, npow / 2, 0, k, j);
        __syncthreads();
      }
    for (int64_t i = tid; i < npow; i += kNmsThreads) a[i] = lds[i];
    __syncthreads();
    return;
  }
  // stages k <= B, block by block
  for (int64_t base = 0; base < npow; base += B) {
    for (int64_t i = tid; i < B; i += kNmsThreads) lds[i] = a[base + i];
    __syncthreads();
    for (int64_t k = 2; k <= B; k <<= 1)
      for (int64_t j = k >> 1; j > 0; j >>= 1) {
        bitonic_step(lds, B / 2, base, k, j);
        __syncthreads();
      }
    for (int64_t i = tid; i < B; i += kNmsThreads) a[base + i] = lds[i];
    __syncthreads();
  }
  for (int64_t k = 2 * B; k <= npow; k <<= 1) {
    for (int64_t j = k >> 1; j >= B; j >>= 1) {
      bitonic_step(a, npow / 2, 0, k, j);
      __syncthreads();
    }
    for (int64_t base = 0; base < npow; base += B) {
      for (int64_t i = tid; i < B; i += kNmsThreads) lds[i] = a[base + i];
      __syncthreads();
      for (int64_t j = B >> 1; j > 0; j >>= 1) {
        bitonic_step(lds, B / 2, base, k, j);
        __syncthreads();
      }
      for (int64_t i = tid; i < B; i += kNmsThreads) a[base + i] = lds[i];
      __syncthreads();
    }
  }
}

// Greedy suppression of the sorted offers offer[0 .. n): an offer is
// accepted unless an accepted, earlier offer lies within the radius.  The
// result of greedy acceptance in a fixed order is unique.  When the radius
// spans few tiles it is computed in parallel rounds over the tile grid (aux:
// tile -> rank): an offer is rejected once an accepted, earlier, nearby
// offer exists, and accepted once every earlier nearby offer is rejected.
// Each round decides at least the earliest undecided offer, and decisions
// are final, so reading neighbours' states while they change is safe.
// Otherwise the offers are scanned one by one against the accepted list
// (aux).  Writes the accepted offers in order to out; returns their number.
// AUX is int16_t (LDS, ntiles <= kMaxOffers) or int32_t (global).
template <typename AUX>
__device__ __forceinline__ int suppress(const TilePeak *offer, int n, int64_t ntiles, int ntd, int64_t ntt,
                        int tile_dm, int64_t tile_t, int nms_dm, int64_t nms_t, AUX *aux,
                        uint8_t *state, TilePeak *__restrict__ out, int *naccept,
                        uint32_t *tmp) {
  const int tid = threadIdx.x;
  // spans in tiles, from radii already clamped to the plane
  const int64_t span_d = ((int64_t)nms_dm + tile_dm - 1) / tile_dm;
  const int64_t span_t = (nms_t + tile_t - 1) / tile_t;
  const bool grid = (2 * span_d + 1) * (2 * span_t + 1) <= 49;
  if (tid == 0) *naccept = 0;
  __syncthreads();
  if (grid) {
    for (int64_t i = tid; i < ntiles; i += kNmsThreads) aux[i] = (AUX)-1;
    for (int i = tid; i < n; i += kNmsThreads) state[i] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += kNmsThreads) {
      const TilePeak c = offer[i];
      aux[(int64_t)(c.d / tile_dm) * ntt + c.t / tile_t] = (AUX)i;
    }
    __syncthreads();
    int undecided = 1;
    while (undecided) {
      int mine = 0;
      for (int i = tid; i < n; i += kNmsThreads) {
        if (state[i] != 0) continue;
        const TilePeak c = offer[i];
        const int64_t a = c.d / tile_dm;
        const int64_t b = c.t / tile_t;
        bool blocked = false, rejected = false;
        for (int64_t da = -span_d; da <= span_d && !rejected; ++da) {
          const int64_t aa = a + da;
          if (aa < 0 || aa >= ntd) continue;
          for (int64_t db = -span_t; db <= span_t; ++db) {
            const int64_t bb = b + db;
            if (bb < 0 || bb >= ntt) continue;
            const int j = (int)aux[aa * ntt + bb];
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
    __syncthreads();  // every state written (they may be in global memory)
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
    if (tid == kNmsThreads - 1) *naccept = (int)pos;
    __syncthreads();
  } else {
    for (int i = 0; i < n; ++i) {
      const TilePeak c = offer[i];
      const int na = *naccept;
      bool hit = false;
      for (int j = tid; j < na; j += kNmsThreads)
        if (near(c, offer[(int)aux[j]], nms_dm, nms_t)) hit = true;
      const int any = __syncthreads_or(hit);
      if (!any && tid == 0) {
        aux[na] = (AUX)i;
        *naccept = na + 1;
      }
      __syncthreads();
    }
    const int na = *naccept;
    for (int j = tid; j < na; j += kNmsThreads) out[j] = offer[(int)aux[j]];
  }
  __syncthreads();
  return *naccept;
}

// Selection and greedy suppression of one plane in one workgroup.  The
// offers (tile peaks at or above the threshold) are counted first.  When
// they and the tile grid fit in LDS, the offers are gathered, sorted and
// suppressed there.  Otherwise the global arrays of the scratch hold the
// offers (sorted with LDS blocks), the tile -> rank map and the states.
// Either way there is no limit on the number of offers.
__device__ void select_nms(uint8_t *__restrict__ scratch, int64_t ntiles, int ntd, int64_t ntt,
                           int tile_dm, int64_t tile_t, float threshold, int nms_dm,
                           int64_t nms_t) {
  __shared__ TilePeak offer[kMaxOffers];
  __shared__ int16_t aux[kMaxOffers];
  __shared__ uint8_t state[kMaxOffers];
  __shared__ int count;
  __shared__ int naccept;
  __shared__ uint32_t tmp[kNmsThreads / 64];
  const int tid = threadIdx.x;
  const DetectLayout L = detect_layout(ntiles);
  const TilePeak *peaks = reinterpret_cast<const TilePeak *>(scratch + L.peaks);
  TilePeak *out = reinterpret_cast<TilePeak *>(scratch + L.out);
  int32_t *status = reinterpret_cast<int32_t *>(scratch + L.status);
  if (tid == 0) count = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t i = tid; i < ntiles; i += kNmsThreads) mine += peaks[i].snr >= threshold;
  atomicAdd(&count, mine);
  __syncthreads();
  const int n = count;
  int na = 0;
  if (n == 0) {
    na = 0;
  } else if (ntiles <= kMaxOffers) {
    if (tid == 0) count = 0;
    __syncthreads();
    for (int64_t i = tid; i < ntiles; i += kNmsThreads) {
      const TilePeak p = peaks[i];
      if (p.snr >= threshold) offer[atomicAdd(&count, 1)] = p;
    }
    __syncthreads();
    int npow = 1;
    while (npow < n) npow <<= 1;
    for (int i = n + tid; i < npow; i += kNmsThreads) offer[i] = sentinel();
    __syncthreads();
    for (int k = 2; k <= npow; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        bitonic_step(offer, npow / 2, 0, k, j);
        __syncthreads();
      }
    na = suppress<int16_t>(offer, n, ntiles, ntd, ntt, tile_dm, tile_t, nms_dm, nms_t, aux,
                           state, out, &naccept, tmp);
  } else {
    TilePeak *g_offer = reinterpret_cast<TilePeak *>(scratch + L.offer);
    int32_t *g_aux = reinterpret_cast<int32_t *>(scratch + L.aux);
    uint8_t *g_state = scratch + L.state;
    if (tid == 0) count = 0;
    __syncthreads();
    for (int64_t i = tid; i < ntiles; i += kNmsThreads) {
      const TilePeak p = peaks[i];
      if (p.snr >= threshold) g_offer[atomicAdd(&count, 1)] = p;
    }
    int64_t npow = 1;
    while (npow < n) npow <<= 1;
    for (int64_t i = n + tid; i < npow; i += kNmsThreads) g_offer[i] = sentinel();
    __syncthreads();
    sort_offers(g_offer, npow, offer);
    na = suppress<int32_t>(g_offer, n, ntiles, ntd, ntt, tile_dm, tile_t, nms_dm, nms_t, g_aux,
                           g_state, out, &naccept, tmp);
  }
  if (tid == 0) {
    status[0] = n;
    status[1] = na;
    status[2] = 0;
    status[3] = 0;
  }
}

__global__ __launch_bounds__(kNmsThreads) void select_nms_kernel(
    uint8_t *__restrict__ scratch, int64_t ntiles, int ntd, int64_t ntt, int tile_dm,
    int64_t tile_t, float threshold, int nms_dm, int64_t nms_t) {
  select_nms(scratch, ntiles, ntd, ntt, tile_dm, tile_t, threshold, nms_dm, nms_t);
}

// One workgroup per beam, on the beam's own scratch.
__global__ __launch_bounds__(kNmsThreads) void select_nms_batch_kernel(
    const BeamWork *__restrict__ beams, int ndm, int tile_dm, int64_t tile_t, float threshold,
    int nms_dm, int64_t nms_t, uint8_t *__restrict__ scratch) {
  const BeamWork &bw = beams[blockIdx.x];
  const int ntd = (ndm + tile_dm - 1) / tile_dm;
  // radii clamped to this beam's plane (they are clamped to the largest on the host)
  const int64_t nt = nms_t < bw.nout ? nms_t : bw.nout;
  select_nms(scratch + bw.det_begin, (int64_t)ntd * bw.ntt, ntd, bw.ntt, tile_dm, tile_t,
             threshold, nms_dm, nt);
}

// Candidate read-back of a whole batch: workgroup b copies beam b's status
// words and its first min(k, ntiles) accepted-offer records into slot b of
// staging (kGatherHeader bytes of status, then k records).  Records past the
// accepted count are copied as they are and ignored by the reader.
__global__ __launch_bounds__(256) void gather_candidates_kernel(
    const BeamWork *__restrict__ beams, int ndm, int tile_dm, const uint8_t *__restrict__ scratch,
    int k, uint8_t *__restrict__ staging) {
  const BeamWork &bw = beams[blockIdx.x];
  const int64_t ntiles = (int64_t)((ndm + tile_dm - 1) / tile_dm) * bw.ntt;
  const DetectLayout L = detect_layout(ntiles);
  const uint8_t *src = scratch + bw.det_begin;
  uint8_t *dst = staging + (int64_t)blockIdx.x * (kGatherHeader + 16 * (int64_t)k);
  if (threadIdx.x < 4)
    reinterpret_cast<int32_t *>(dst)[threadIdx.x] =
        reinterpret_cast<const int32_t *>(src + L.status)[threadIdx.x];
  const int64_t n = ntiles < k ? ntiles : k;
  const uint4 *rec = reinterpret_cast<const uint4 *>(src + L.out);
  uint4 *out = reinterpret_cast<uint4 *>(dst + kGatherHeader);
  for (int64_t i = threadIdx.x; i < n; i += 256) out[i] = rec[i];
}

}  // namespace

hipError_t launch_gather_candidates(const BeamWork *beams, int nbeams, int ndm, int tile_dm,
                                    const uint8_t *scratch, int k, uint8_t *staging,
                                    hipStream_t stream) {
  if (nbeams < 1 || k < 0 || tile_dm < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gather_candidates_kernel, dim3(nbeams), dim3(256), 0, stream, beams, ndm,
                     tile_dm, scratch, k, staging);
  return hipGetLastError();
}

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

hipError_t launch_select_nms(uint8_t *scratch, int ndm, int64_t nout, int tile_dm, int64_t tile_t,
                             float threshold, int nms_dm, int64_t nms_t, hipStream_t stream) {
  const int ntd = (ndm + tile_dm - 1) / tile_dm;
  const int64_t ntt = (nout + tile_t - 1) / tile_t;
  hipLaunchKernelGGL(select_nms_kernel, dim3(1), dim3(kNmsThreads), 0, stream, scratch,
                     (int64_t)ntd * ntt, ntd, ntt, tile_dm, tile_t, threshold, nms_dm, nms_t);
  return hipGetLastError();
}

hipError_t launch_select_nms_batch(const BeamWork *beams, int nbeams, int ndm, int tile_dm,
                                   int64_t tile_t, float threshold, int nms_dm, int64_t nms_t,
                                   uint8_t *scratch, hipStream_t stream) {
  hipLaunchKernelGGL(select_nms_batch_kernel, dim3(nbeams), dim3(kNmsThreads), 0, stream, beams,
                     ndm, tile_dm, tile_t, threshold, nms_dm, nms_t, scratch);
  return hipGetLastError();
}

}  // namespace sps

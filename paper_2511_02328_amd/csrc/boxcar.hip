// boxcar.hip -- boxcar matched-filter S/N over the DM-time plane on gfx950.
//
// For every trial row and start sample t the window sums B_w(t) of all
// requested widths come from one prefix sum P of the row segment held in LDS:
// B_w(t) = P(t + w) - P(t).  P is kept in wrapping u32 arithmetic; every
// window sum is below 2^31 (checked on the host), so the differences are
// exact.  The S/N numerator B_w - w med is an exact integer (with power-of-two
// widths the staged samples have the median subtracted, so it is P'(t + w) -
// P'(t) of the prefix of Y - med); it is scaled by 1 / (1.4826 MAD sqrt(w)) in
// binary32, and the maximum over widths (ties to the smallest width) is
// written with the index of its width.
//
// One workgroup of 256 threads covers 4096 consecutive outputs of one row
// plus a halo of w_max - 1 samples.  Lanes run along time, so the plane reads
// and the S/N writes are fully coalesced and the LDS reads P[t + w] of a wave
// are consecutive words (conflict-free).  Traffic is one read of Y and one
// write of snr and best_w (9 B per output), which runs at the device's
// streaming rate with 7 widths; with 9 widths the vector work is close to
// the same time and the part runs at its power limit (lower clock), so each
// width's numerator is kept to one two-operand subtraction.
//
// The same pass can gather the tile maxima of the detection step (64-bit
// key of order-preserving S/N bits and in-tile position, atomicMax per
// tile), or write the detector's max-pooled bfloat16 tiles instead of the
// planes.
#include <math.h>

#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kThreads = 256;
constexpr int kSeg = 4096;
constexpr int kPer = kSeg / kThreads;

// Inclusive sum over the lanes of a wave up to this one, with DPP moves
// (registers only): Hillis-Steele steps of 1, 2, 4, 8 lanes inside each row
// of 16, then the row totals broadcast from lane 15 into rows 1 and 3 and
// from lane 31 into rows 2 and 3.  Lanes whose source lies outside the row,
// and rows left out by the row mask, add 0.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// One DPP step of a running maximum: lanes whose source lies outside the
// row, and rows left out by the row mask, take their own value.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_max_step(float x) {
  const int y = __builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), CTRL, ROWS, 0xf,
                                            false);
  return fmaxf(x, __int_as_float(y));
}

// Maximum over the wave (the same steps as wave_inclusive_scan; lane 63
// ends with the whole wave's maximum), in every lane.
__device__ __forceinline__ float wave_max(float x) {
  x = dpp_max_step<0x111, 0xf>(x);
  x = dpp_max_step<0x112, 0xf>(x);
  x = dpp_max_step<0x114, 0xf>(x);
  x = dpp_max_step<0x118, 0xf>(x);
  x = dpp_max_step<0x142, 0xa>(x);
  x = dpp_max_step<0x143, 0xc>(x);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ uint32_t block_exclusive_scan256(uint32_t v, uint32_t *tmp /* >= 4 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) tmp[wave] = inc;
  __syncthreads();
  uint32_t off = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) off += (w < wave) ? tmp[w] : 0u;
  __syncthreads();
  return off + inc - v;
}

// Running tile maximum of one thread's outputs of a segment (row d, first
// output t0).  TILES = 0: none.  TILES = 1: the segment lies in one tile
// column; each thread keeps only its largest S/N (one max per output), and
// finish() reduces the workgroup to its maximum, whose first output the
// threads holding it find again in the S/N row they wrote (one atomic per
// such thread; the key orders equal S/N by position).  TILES = 2: any tiling; a thread flushes its
// maximum with an atomic whenever its outputs enter the next tile column.
// TILES = 3: tile_t and the row length multiples of 64, so the 64
// consecutive outputs a wave handles at a time share one column, and its
// lanes change column, and leave the last segment's loop, together: a
// flush reduces the wave's keys and issues one atomic.
// PK: the key's low word.  0: complement of the position (the planes hold
// the width).  1 (no planes): packed position and width index, the width
// tracked with each maximum.  2 (no planes, TILES = 1): packed; a thread
// tracks S/N and position only, and finish() recomputes the width index of
// the one output it reports (width_at(t_local)).
template <int TILES, int PK = 0>
struct TileTrack {
  float s = -INFINITY;
  int tl = 0;
  int bi = 0;
  int64_t col = 0, col_end = 0;

  __device__ __forceinline__ void begin(const TileSink &k, int64_t t0) {
    if constexpr (TILES != 0) {
      col = t0 / k.tile_t;
      col_end = (col + 1) * k.tile_t;
    }
  }
  __device__ __forceinline__ unsigned long long key(const TileSink &k, int d, int64_t t0) const {
    const int64_t t = t0 + tl;
    const int a = d / k.tile_dm;
    const uint32_t pos =
        (uint32_t)((t - col * k.tile_t) * k.tile_dm + (int64_t)(d - a * k.tile_dm));
    uint32_t lo;
    if constexpr (PK == 0)
      lo = ~pos;
    else
      lo = (((uint32_t)(kKeyPosLimit - 1) - pos) << kKeyWidthBits) |
           ((uint32_t)bi & ((1u << kKeyWidthBits) - 1u));
    return ((unsigned long long)snr_key_bits(s) << 32) | (unsigned long long)lo;
  }
  __device__ __forceinline__ void flush(const TileSink &k, int d, int64_t t0) {
    if constexpr (TILES == 3) {
      unsigned long long v = s == -INFINITY ? 0ull : key(k, d, t0);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
        const unsigned long long u = ((unsigned long long)hi << 32) | lo;
        v = u > v ? u : v;
      }
      if ((threadIdx.x & 63) == 0 && v != 0ull)
        atomicMax(k.keys + (int64_t)(d / k.tile_dm) * k.ntt + col, v);
    } else {
      if (s != -INFINITY)
        atomicMax(k.keys + (int64_t)(d / k.tile_dm) * k.ntt + col, key(k, d, t0));
    }
  }
  __device__ __forceinline__ void add(const TileSink &k, int d, int64_t t0, float v, int t_local,
                                      int b) {
    if constexpr (TILES == 1 && PK == 0) {
      s = fmaxf(s, v);
      return;
    }
    if constexpr (TILES >= 2) {
      if (t0 + t_local >= col_end) {
        flush(k, d, t0);
        col = (t0 + t_local) / k.tile_t;
        col_end = (col + 1) * k.tile_t;
        s = -INFINITY;
      }
    }
    if constexpr (TILES != 0) {
      const bool gt = v > s;  // the first output of a run of equal maxima stays
      tl = gt ? t_local : tl;
      if constexpr (PK == 1) bi = gt ? b : bi;
      s = fmaxf(s, v);
    }
  }
  // Every thread of the workgroup calls this once, after its last add;
  // srow[0, len) are the S/N values this segment wrote (TILES = 1 with
  // PK = 0 reads back its own outputs).
  template <class W>
  __device__ __forceinline__ void finish(const TileSink &k, int d, int64_t t0,
                                         unsigned long long *red, const SPS_GLOBAL float *srow,
                                         int len, W &&width_at) {
    if constexpr (TILES == 1) {
      float m = wave_max(s);
      float *redf = reinterpret_cast<float *>(red);
      if ((threadIdx.x & 63) == 0) redf[threadIdx.x >> 6] = m;
      __syncthreads();
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) m = fmaxf(m, redf[w]);
      if (s == m && m != -INFINITY) {
        if constexpr (PK == 0) {
          // this thread's outputs are threadIdx.x + kThreads j, in order; all
          // of them are read at once, the first equal to m wins
          float v[kPer];
#pragma unroll
          for (int j = 0; j < kPer; ++j) {
            const int t = threadIdx.x + kThreads * j;
            v[j] = t < len ? srow[t] : -INFINITY;
          }
          int first = kPer - 1;
#pragma unroll
          for (int j = kPer - 2; j >= 0; --j) first = v[j] == m ? j : first;
          tl = threadIdx.x + kThreads * first;
        } else if constexpr (PK == 2) {
          bi = width_at(tl);
        }
        atomicMax(k.keys + (int64_t)(d / k.tile_dm) * k.ntt + col, key(k, d, t0));
      }
    } else if constexpr (TILES >= 2) {
      flush(k, d, t0);
    }
  }
};

// finish() argument of segments whose sink needs no recomputed width.
struct NoWidth {
  __device__ __forceinline__ int operator()(int) const { return 0; }
};

// Where a segment's outputs go.  PlaneSink: the S/N and width planes, and
// the tile maxima (TileTrack).  KeySink: the tile maxima alone, with the
// width index in the key (a search that writes no planes).  PoolSink: an
// LDS row of S/N values, for the max-pooled detector tiles (first row of a
// pair stored, second maxed in).
template <int TILES>
struct PlaneSink {
  SPS_GLOBAL float *srow;
  SPS_GLOBAL uint8_t *brow;
  const TileSink *tiles;
  unsigned long long *red;
  int d;
  int len;  // outputs of the segment
  int64_t t0;
  TileTrack<TILES> tr;
  __device__ __forceinline__ void put(int tl, float v, int bi) {
    srow[tl] = v;
    brow[tl] = (uint8_t)bi;
    tr.add(*tiles, d, t0, v, tl, bi);
  }
  template <class W>
  __device__ __forceinline__ void finish(W &&) {
    tr.finish(*tiles, d, t0, red, srow, len, NoWidth{});
  }
};

template <int TILES, int PK>
struct KeySink {
  static_assert(TILES != 0 && PK != 0, "a sink without planes gathers packed tile keys");
  const TileSink *tiles;
  unsigned long long *red;
  int d;
  int len;
  int64_t t0;
  TileTrack<TILES, PK> tr;
  __device__ __forceinline__ void put(int tl, float v, int bi) {
    tr.add(*tiles, d, t0, v, tl, bi);
  }
  template <class W>
  __device__ __forceinline__ void finish(W &&width_at) {
    tr.finish(*tiles, d, t0, red, nullptr, len, width_at);
  }
};

struct PoolSink {
  float *pv;
  bool first;
  __device__ __forceinline__ void put(int tl, float v, int) {
    pv[tl] = first ? v : fmaxf(pv[tl], v);
  }
  template <class W>
  __device__ __forceinline__ void finish(W &&) {}
};

// Widths 1, 2, 4, ..., 2^(NPOW-1): window offsets are immediates of the LDS
// reads and width indices are constants, and the window length kLen is a
// compile-time constant, so each thread issues all of its loads before the
// first wait and reads and writes its scan chunk at immediate LDS offsets
// (an odd chunk length puts the chunk starts of a wave in distinct banks).
// A segment is fetched into registers (pow2_fetch), staged into LDS
// (pow2_stage) and filtered (pow2_filter).
// TAIL: the row ends inside the window (n_left < kLen samples remain); the
// missing samples read as zero, widths that run past the row end are left
// out of the maximum (as -inf; width 1 always fits), and outputs past the
// row end are not written.
template <int NPOW>
struct Pow2 {
  static constexpr int kLen = kSeg + (1 << (NPOW - 1)) - 1;
  static constexpr int kLd = (kLen + kThreads - 1) / kThreads;
  static constexpr int kCh = kLd | 1;
  static constexpr int kWords = kThreads * kCh + 1;  // P, scan chunks padded
};

template <int NPOW, bool TAIL>
__device__ __forceinline__ void pow2_fetch(const SPS_GLOBAL uint32_t *src, int n_left,
                                           uint32_t (&v)[Pow2<NPOW>::kLd]) {
  constexpr int kLen = Pow2<NPOW>::kLen, kLd = Pow2<NPOW>::kLd;
#pragma unroll
  for (int k = 0; k < kLd; ++k) {
    const int i = threadIdx.x + kThreads * k;
    const bool in = TAIL ? i < n_left : (k + 1 < kLd || i < kLen);
    v[k] = in ? src[i] : 0u;
  }
}

// P[i + 1] = sample i of the window minus the median (wrapping), for i
// up to the padded scan extent, and 0 past the window or the row end (so
// the prefix stays flat where only widths left out of the maximum, or no
// output, read it); the caller has made sure that every reader of the
// previous segment's P is done.  The prefix of Y - med makes each numerator
// B_w - w med one subtraction.
template <int NPOW, bool TAIL>
__device__ __forceinline__ void pow2_stage(const uint32_t (&v)[Pow2<NPOW>::kLd], int n_left,
                                           int32_t med, uint32_t *P) {
  constexpr int kLen = Pow2<NPOW>::kLen, kLd = Pow2<NPOW>::kLd, kCh = Pow2<NPOW>::kCh;
#pragma unroll
  for (int k = 0; k < kCh; ++k) {
    const int i = threadIdx.x + kThreads * k;
    const bool in = k < kLd && (TAIL ? i < n_left : (k + 1 < kLd || i < kLen));
    P[i + 1] = in ? v[k] - (uint32_t)med : 0u;
  }
}

// Width scales 1 / (1.4826 MAD sqrt(w)) into LDS (0 when MAD = 0); read
// after the next barrier.
__device__ __forceinline__ void set_scales(const WidthList &widths, int32_t mad, float *scale) {
  if (threadIdx.x < widths.n) {
    const double w = (double)widths.w[threadIdx.x];
    scale[threadIdx.x] = mad > 0 ? (float)(1.0 / (1.4826 * (double)mad * sqrt(w))) : 0.0f;
  }
}

// True in every thread iff pred holds in every thread of the workgroup
// (one barrier; flags: kThreads / 64 words of LDS).
__device__ __forceinline__ bool block_all(bool pred, uint32_t *flags) {
  const bool w = __all(pred);
  if ((threadIdx.x & 63) == 0) flags[threadIdx.x >> 6] = w ? 1u : 0u;
  __syncthreads();
  bool r = true;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) r = r && flags[i] != 0u;
  return r;
}

// The outputs of one segment from its prefix P (FLT: stored as floats),
// then out.finish(width_at).
template <int NPOW, bool TAIL, bool FLT, class Sink>
__device__ __forceinline__ void pow2_rows(int n_left, int32_t mad, const float *scale,
                                          const uint32_t *P, Sink &out) {
  // The maximum first (three-input max), then the smallest width that
  // attains it: equal to the strict running comparison, since S/N values are
  // never NaN and never -0 (the numerator is an integer, the scale positive).
  const int seg_len = TAIL ? (n_left < kSeg ? n_left : kSeg) : kSeg;
  if (mad <= 0) {
    // MAD 0 (scales 0): every S/N is 0 and width index 0 attains it
#pragma unroll 4
    for (int m = 0; m < kPer; ++m) {
      const int tl = threadIdx.x + kThreads * m;
      if (TAIL && tl >= seg_len) break;
      out.put(tl, 0.0f, 0);
    }
    out.finish(NoWidth{});
    return;
  }
  float sc[NPOW];
#pragma unroll
  for (int i = 0; i < NPOW; ++i) sc[i] = scale[i];
  const float *Pf = reinterpret_cast<const float *>(P);
  // S/N of every width at output tl, and their maximum.  The numerator is
  // exact either way: with FLT, a float difference of two exact integers,
  // rounded to nearest as the conversion of the integer difference is.
  auto eval = [&](int tl, float (&s)[NPOW]) {
    if constexpr (FLT) {
      const float *pt = Pf + tl;
      const float p0 = pt[0];
#pragma unroll
      for (int i = 0; i < NPOW; ++i) s[i] = (pt[1 << i] - p0) * sc[i];
    } else {
      const uint32_t *pt = P + tl;
      const uint32_t p0 = pt[0];
#pragma unroll
      for (int i = 0; i < NPOW; ++i) s[i] = (float)(int32_t)(pt[1 << i] - p0) * sc[i];
    }
#pragma unroll
    for (int i = 0; i < NPOW; ++i)
      if (TAIL && tl + (1 << i) > n_left) s[i] = -INFINITY;
    float mx = s[0];
#pragma unroll
    for (int i = 1; i < NPOW; ++i) mx = fmaxf(mx, s[i]);
    return mx;
  };
  auto first_of = [](const float (&s)[NPOW], float mx) {
    int bi = NPOW - 1;
#pragma unroll
    for (int i = NPOW - 2; i >= 0; --i) bi = s[i] == mx ? i : bi;
    return bi;
  };
#pragma unroll 2
  for (int m = 0; m < kPer; ++m) {
    const int tl = threadIdx.x + kThreads * m;
    if (TAIL && tl >= seg_len) break;
    float s[NPOW];
    const float mx = eval(tl, s);
    out.put(tl, mx, first_of(s, mx));
  }
  // the same arithmetic again, for a sink that tracks no width
  out.finish([&](int tl) {
    float s[NPOW];
    const float mx = eval(tl, s);
    return first_of(s, mx);
  });
}

template <int NPOW, bool TAIL, class Sink>
__device__ __forceinline__ void pow2_filter(int n_left, int32_t med, int32_t mad,
                                            const float *scale, uint32_t *tmp, uint32_t *P,
                                            Sink &out) {
  constexpr int kCh = Pow2<NPOW>::kCh;
  __shared__ uint32_t flags[kThreads / 64];
  __syncthreads();

  // Exclusive prefix over the padded extent: thread chunks of kCh samples
  // (entries past the window are never read).
  const int lo = threadIdx.x * kCh;
  uint32_t c[kCh];
  uint32_t part = 0;
#pragma unroll
  for (int j = 0; j < kCh; ++j) {
    c[j] = P[lo + j + 1];
    part += c[j];
  }
  uint32_t run = block_exclusive_scan256(part, tmp);
  // Where every prefix value of the window has magnitude below 2^24 (the
  // usual case: the samples stay near the median) it is stored as a float,
  // exactly, and a width's numerator costs one float subtraction instead of
  // an integer subtraction and a conversion.  Steps |Y - med| < 2^24 keep a
  // walk that stays inside +-2^24 from wrapping the 32-bit prefix.
  // Widths up to 256 (chunks of at most 17 values, held twice in
  // registers); longer windows keep the integers.
  constexpr bool kFlt = kCh <= 17;
  float f[kCh];
  float amax = 0.0f;
#pragma unroll
  for (int j = 0; j < kCh; ++j) {
    run += c[j];
    c[j] = run;
    if constexpr (kFlt) {
      f[j] = (float)(int32_t)run;
      amax = fmaxf(amax, fabsf(f[j]));
    }
  }
  const bool flt = kFlt && block_all(amax < 0x1p24f, flags);
  if (flt) {
#pragma unroll
    for (int j = 0; j < kCh; ++j) P[lo + j + 1] = __float_as_uint(f[j]);
  } else {
#pragma unroll
    for (int j = 0; j < kCh; ++j) P[lo + j + 1] = c[j];
  }
  if (threadIdx.x == 0) P[0] = 0u;  // 0 and 0.0f
  __syncthreads();
  if constexpr (kFlt) {
    if (flt) {
      pow2_rows<NPOW, TAIL, true>(n_left, mad, scale, P, out);
      return;
    }
  }
  pow2_rows<NPOW, TAIL, false>(n_left, mad, scale, P, out);
}

template <int NPOW, bool TAIL, class Sink>
__device__ __forceinline__ void pow2_segment(const SPS_GLOBAL uint32_t *src, int n_left,
                                             int32_t med, int32_t mad, const WidthList &widths,
                                             float *scale, uint32_t *tmp, uint32_t *P,
                                             Sink &out) {
  uint32_t v[Pow2<NPOW>::kLd];
  pow2_fetch<NPOW, TAIL>(src, n_left, v);
  set_scales(widths, mad, scale);
  pow2_stage<NPOW, TAIL>(v, n_left, med, P);
  pow2_filter<NPOW, TAIL>(n_left, med, mad, scale, tmp, P, out);
}

// NPOW > 0: power-of-two widths (pow2_segment); NPOW = 0: any width list.
// One segment of row d: outputs [seg kSeg, seg kSeg + kSeg) go to `out`
// (out.put(t - seg kSeg, S/N, width index)), then out.finish(width_at).
template <int NPOW, class Sink>
__device__ __forceinline__ void boxcar_core(const uint32_t *__restrict__ Y, int64_t nout, int d,
                                            int seg, const int32_t *__restrict__ stats,
                                            const WidthList &widths, uint32_t *P, Sink &out) {
  __shared__ float scale[kMaxWidths];
  __shared__ uint32_t tmp[4];
  const int64_t t0 = (int64_t)seg * kSeg;
  const SPS_GLOBAL uint32_t *row = gmem(Y + (int64_t)d * nout);
  const int nw = widths.n;
  const int wmax = widths.w[nw - 1];
  const int32_t med = gmem(stats)[2 * (int64_t)d];
  const int32_t mad = gmem(stats)[2 * (int64_t)d + 1];

  // Samples this segment needs: [t0, t0 + len), len <= kSeg + wmax - 1.
  const int64_t avail = nout - t0;

  if constexpr (NPOW > 0) {
    constexpr int kLen = Pow2<NPOW>::kLen;
    if (avail >= (int64_t)kLen)
      pow2_segment<NPOW, false>(row + t0, kLen, med, mad, widths, scale, tmp, P, out);
    else
      pow2_segment<NPOW, true>(row + t0, (int)avail, med, mad, widths, scale, tmp, P, out);
    return;
  }

  set_scales(widths, mad, scale);
  const int len = (int)(avail < (int64_t)(kSeg + wmax - 1) ? avail : (int64_t)(kSeg + wmax - 1));
  for (int i = threadIdx.x; i < len; i += kThreads) P[i + 1] = row[t0 + i];
  __syncthreads();

  // Exclusive prefix: each thread owns a contiguous chunk of ch samples.
  const int ch = (len + kThreads - 1) / kThreads;
  const int lo = threadIdx.x * ch;
  const int hi = lo + ch < len ? lo + ch : len;
  uint32_t part = 0;
  for (int i = lo; i < hi; ++i) part += P[i + 1];
  uint32_t run = block_exclusive_scan256(part, tmp);
  for (int i = lo; i < hi; ++i) {
    run += P[i + 1];
    P[i + 1] = run;
  }
  if (threadIdx.x == 0) P[0] = 0u;
  __syncthreads();

  const int seg_len = avail < kSeg ? (int)avail : kSeg;
  const bool live = mad > 0;

  if (avail >= (int64_t)(kSeg + wmax - 1)) {
    // Every width fits at every output of this segment: no per-width guard.
    // Widths, w * med and the scales are wave-uniform (kernel argument and
    // LDS), so a width costs one v_add3 (numerator), cvt, mul, compare and
    // two selects.
#pragma unroll 2
    for (int m = 0; m < kPer; ++m) {
      const int tl = threadIdx.x + kThreads * m;
      const uint32_t neg_p0 = 0u - P[tl];
      float bs = -INFINITY;
      int bi = 0;
#pragma unroll
      for (int i = 0; i < kMaxWidths; ++i) {
        if (i >= nw) break;
        const int w = widths.w[i];
        const int32_t num = (int32_t)(P[tl + w] + neg_p0 - (uint32_t)(w * med));
        const float s = (float)num * scale[i];
        if (s > bs) {
          bs = s;
          bi = i;
        }
      }
      out.put(tl, live ? bs : 0.0f, bi);
    }
    out.finish(NoWidth{});
    return;
  }

#pragma unroll 4
  for (int m = 0; m < kPer; ++m) {
    const int tl = threadIdx.x + kThreads * m;
    if (tl >= seg_len) break;
    const uint32_t p0 = P[tl];
    const int64_t room = avail - tl;  // widths with w <= room fit
    float bs = 0.0f;
    int bi = 0xFF;
    for (int i = 0; i < nw; ++i) {
      const int w = widths.w[i];
      if (w > room) break;
      const int32_t num = (int32_t)(P[tl + w] - p0) - w * med;
      const float s = live ? (float)num * scale[i] : 0.0f;
      if (bi == 0xFF || s > bs) {
        bs = s;
        bi = i;
      }
    }
    out.put(tl, bi == 0xFF ? 0.0f : bs, bi);
  }
  out.finish(NoWidth{});
}

// One segment of row d into `out` (planes and tile maxima, or tile maxima
// alone); the power-of-two path issues the segment's loads first.
template <int NPOW, class Sink>
__device__ __forceinline__ void boxcar_sink_segment(const uint32_t *__restrict__ Y, int64_t nout,
                                                    int d, int seg,
                                                    const int32_t *__restrict__ stats,
                                                    const WidthList &widths, uint32_t *P,
                                                    Sink &out) {
  if constexpr (NPOW == 0) {
    boxcar_core<0>(Y, nout, d, seg, stats, widths, P, out);
  } else {
    __shared__ float scale[kMaxWidths];
    __shared__ uint32_t tmp[4];
    constexpr int kLen = Pow2<NPOW>::kLen;
    const int64_t t0 = (int64_t)seg * kSeg, avail = nout - t0;
    const SPS_GLOBAL uint32_t *src = gmem(Y + (int64_t)d * nout + t0);
    const int32_t med = gmem(stats)[2 * (int64_t)d];
    const int32_t mad = gmem(stats)[2 * (int64_t)d + 1];
    uint32_t v[Pow2<NPOW>::kLd];
    if (avail >= (int64_t)kLen) {
      pow2_fetch<NPOW, false>(src, kLen, v);
      set_scales(widths, mad, scale);
      pow2_stage<NPOW, false>(v, kLen, med, P);
      pow2_filter<NPOW, false>(kLen, med, mad, scale, tmp, P, out);
    } else {
      pow2_fetch<NPOW, true>(src, (int)avail, v);
      set_scales(widths, mad, scale);
      pow2_stage<NPOW, true>(v, (int)avail, med, P);
      pow2_filter<NPOW, true>((int)avail, med, mad, scale, tmp, P, out);
    }
  }
}

// One segment of row d: with PK = 0 into the S/N and width planes, with
// the tile maxima (TILES); with PK != 0 the packed tile maxima alone.
template <int NPOW, int TILES, int PK>
__device__ __forceinline__ void boxcar_plane_segment(const uint32_t *__restrict__ Y, int64_t nout,
                                                     int d, int seg,
                                                     const int32_t *__restrict__ stats,
                                                     const WidthList &widths,
                                                     float *__restrict__ snr,
                                                     uint8_t *__restrict__ best, uint32_t *P,
                                                     const TileSink &sink) {
  static_assert(PK != 2 || (TILES == 1 && NPOW > 0), "widths recomputed only on power-of-two rows");
  __shared__ unsigned long long red[kThreads / 64];
  const int64_t t0 = (int64_t)seg * kSeg, avail = nout - t0;
  const int len = (int)(avail < kSeg ? avail : kSeg);
  if constexpr (PK == 0) {
    PlaneSink<TILES> out{gmem(snr + (int64_t)d * nout + t0), gmem(best + (int64_t)d * nout + t0),
                         &sink, red, d, len, t0, TileTrack<TILES>{}};
    out.tr.begin(sink, t0);
    boxcar_sink_segment<NPOW>(Y, nout, d, seg, stats, widths, P, out);
  } else {
    KeySink<TILES, PK> out{&sink, red, d, len, t0, TileTrack<TILES, PK>{}};
    out.tr.begin(sink, t0);
    boxcar_sink_segment<NPOW>(Y, nout, d, seg, stats, widths, P, out);
  }
}

// Trials d, d + 1 of one segment pooled over 2 trials x 8 samples, scaled
// and rounded to bfloat16: pooled[t / 8] of the segment, 512 values (the
// same S/N values the planes would hold; pooling as the tile kernels do).
// Power-of-two widths: both trials' windows are fetched into registers before
// the first is filtered, so the second trial's loads overlap the first's
// work instead of following it.
template <int NPOW, bool TAIL>
__device__ __forceinline__ void pow2_pool_pair(const uint32_t *__restrict__ Y, int64_t nout,
                                               int d, int64_t t0, int n_left,
                                               const int32_t *__restrict__ stats,
                                               const WidthList &widths, uint32_t *P, float *pv) {
  __shared__ float scale[kMaxWidths];
  __shared__ uint32_t tmp[4];
  const SPS_GLOBAL uint32_t *ra = gmem(Y + (int64_t)d * nout + t0);
  const SPS_GLOBAL uint32_t *rb = gmem(Y + (int64_t)(d + 1) * nout + t0);
  uint32_t va[Pow2<NPOW>::kLd], vb[Pow2<NPOW>::kLd];
  pow2_fetch<NPOW, TAIL>(ra, n_left, va);
  pow2_fetch<NPOW, TAIL>(rb, n_left, vb);
  const int32_t med_a = gmem(stats)[2 * (int64_t)d], mad_a = gmem(stats)[2 * (int64_t)d + 1];
  const int32_t med_b = gmem(stats)[2 * (int64_t)d + 2], mad_b = gmem(stats)[2 * (int64_t)d + 3];
  PoolSink first{pv, true};
  set_scales(widths, mad_a, scale);
  pow2_stage<NPOW, TAIL>(va, n_left, med_a, P);
  pow2_filter<NPOW, TAIL>(n_left, med_a, mad_a, scale, tmp, P, first);
  __syncthreads();  // P and the scales are refilled for the second trial
  PoolSink second{pv, false};
  set_scales(widths, mad_b, scale);
  pow2_stage<NPOW, TAIL>(vb, n_left, med_b, P);
  pow2_filter<NPOW, TAIL>(n_left, med_b, mad_b, scale, tmp, P, second);
}

template <int NPOW>
__device__ __forceinline__ void boxcar_pool_pair(const uint32_t *__restrict__ Y, int64_t nout,
                                                 int d, int seg, const int32_t *__restrict__ stats,
                                                 const WidthList &widths, uint32_t *P, float *pv,
                                                 float scale, uint16_t *__restrict__ pooled) {
  if constexpr (NPOW > 0) {
    constexpr int kLen = Pow2<NPOW>::kLen;
    const int64_t t0 = (int64_t)seg * kSeg, avail = nout - t0;
    if (avail >= (int64_t)kLen)
      pow2_pool_pair<NPOW, false>(Y, nout, d, t0, kLen, stats, widths, P, pv);
    else
      pow2_pool_pair<NPOW, true>(Y, nout, d, t0, (int)avail, stats, widths, P, pv);
  } else {
    PoolSink first{pv, true};
    boxcar_core<NPOW>(Y, nout, d, seg, stats, widths, P, first);
    __syncthreads();  // P is refilled for the second trial
    PoolSink second{pv, false};
    boxcar_core<NPOW>(Y, nout, d + 1, seg, stats, widths, P, second);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kSeg / 8; j += kThreads) {
    float m = pv[8 * j];
#pragma unroll
    for (int b = 1; b < 8; ++b) m = fmaxf(m, pv[8 * j + b]);
    const uint32_t u = __float_as_uint(m * scale);
    pooled[j] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // nearest even
  }
}

// One workgroup per (DM row, segment).
template <int NPOW, int TILES, int PK>
__global__ __launch_bounds__(kThreads) void boxcar_kernel(
    const uint32_t *__restrict__ Y, int64_t nout, int nseg, const int32_t *__restrict__ stats,
    WidthList widths, float *__restrict__ snr, uint8_t *__restrict__ best, TileSink sink) {
  extern __shared__ uint32_t P[];  // boxcar_lds_bytes
  const int64_t blk = blockIdx.x;
  const int d = (int)(blk / nseg);
  const int seg = (int)(blk - (int64_t)d * nseg);
  boxcar_plane_segment<NPOW, TILES, PK>(Y, nout, d, seg, stats, widths, snr, best, P, sink);
}

// One workgroup per (beam, DM row, segment) of a batch.  With TILES, the
// beam's tile keys are the out array of its detection scratch; with PK, no
// beam has planes.
template <int NPOW, int TILES, int PK>
__global__ __launch_bounds__(kThreads) void boxcar_batch_kernel(
    const BeamWork *__restrict__ beams, int nbeams, WidthList widths, uint8_t *scratch, int ndm,
    int tile_dm, int64_t tile_t) {
  extern __shared__ uint32_t P[];
  const int64_t blk = blockIdx.x;
  const BeamWork &bw = beams[find_beam_wave<&BeamWork::bx_begin>(beams, nbeams, blk)];
  const int64_t local = blk - bw.bx_begin;
  const int d = (int)(local / bw.nseg);
  const int seg = (int)(local - (int64_t)d * bw.nseg);
  TileSink sink{};
  if constexpr (TILES != 0) {
    const int64_t ntd = (ndm + tile_dm - 1) / tile_dm;
    sink.keys = reinterpret_cast<unsigned long long *>(scratch + bw.det_begin +
                                                       detect_layout(ntd * bw.ntt).out);
    sink.tile_dm = tile_dm;
    sink.tile_t = tile_t;
    sink.ntt = bw.ntt;
    sink.packed = PK != 0;
  }
  boxcar_plane_segment<NPOW, TILES, PK>(bw.Y, bw.nout, d, seg, bw.stats, widths, bw.snr, bw.best,
                                        P, sink);
}

// Tile keys: zeroed (DECODE false) or turned into tile peak records.
__device__ __forceinline__ void tile_key(const TileSink &k, int ndm, int64_t nout,
                                         const uint8_t *best, TilePeak *peaks, int64_t i,
                                         bool decode) {
  if (!decode) {
    k.keys[i] = 0ull;
    return;
  }
  const unsigned long long v = k.keys[i];
  const int a = (int)(i / k.ntt);
  const int64_t b = i - (int64_t)a * k.ntt;
  const uint32_t lo = (uint32_t)v;
  const uint32_t pos =
      k.packed ? (uint32_t)(kKeyPosLimit - 1) - (lo >> kKeyWidthBits) : ~lo;
  int64_t tl = pos / (uint32_t)k.tile_dm;
  int dl = (int)(pos - (uint32_t)tl * (uint32_t)k.tile_dm);
  const int d0 = a * k.tile_dm;
  const int64_t t0 = b * k.tile_t;
  if (v == 0ull || d0 + dl >= ndm || t0 + tl >= nout) {  // no output reached the tile
    tl = 0;
    dl = 0;
  }
  TilePeak p;
  p.snr = v == 0ull ? 0.0f : snr_from_key_bits((uint32_t)(v >> 32));
  p.d = d0 + dl;
  p.t = (int32_t)(t0 + tl);
  if (k.packed)
    p.w = v == 0ull ? 0 : (int32_t)(lo & ((1u << kKeyWidthBits) - 1u));
  else
    p.w = gmem(best)[(int64_t)p.d * nout + p.t];
  peaks[i] = p;
}

__global__ __launch_bounds__(kThreads) void tile_keys_kernel(TileSink k, int64_t ntiles, int ndm,
                                                             int64_t nout,
                                                             const uint8_t *__restrict__ best,
                                                             TilePeak *__restrict__ peaks,
                                                             int decode) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < ntiles) tile_key(k, ndm, nout, best, peaks, i, decode != 0);
}

// One thread per (beam, tile) of a batch.
__global__ __launch_bounds__(kThreads) void tile_keys_batch_kernel(
    const BeamWork *__restrict__ beams, int nbeams, int ndm, int64_t total_tiles, int tile_dm,
    int64_t tile_t, uint8_t *scratch, int decode, int packed) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= total_tiles) return;
  const BeamWork &bw = beams[find_beam<&BeamWork::tp_begin>(beams, nbeams, i)];
  const int64_t ntd = (ndm + tile_dm - 1) / tile_dm;
  const DetectLayout L = detect_layout(ntd * bw.ntt);
  TileSink k{};
  k.keys = reinterpret_cast<unsigned long long *>(scratch + bw.det_begin + L.out);
  k.tile_dm = tile_dm;
  k.tile_t = tile_t;
  k.ntt = bw.ntt;
  k.packed = packed;
  tile_key(k, ndm, bw.nout, bw.best, reinterpret_cast<TilePeak *>(scratch + bw.det_begin + L.peaks),
           i - bw.tp_begin, decode != 0);
}

// Detector tiles straight from the boxcar: one workgroup per (trial pair,
// segment) of the whole tiles (512 trials x 4096 samples) of a plane; tile
// (ti, tj) is tiles[ti * ncols + tj], pooled row i of a tile from trials
// 512 ti + 2i, + 1.
template <int NPOW>
__global__ __launch_bounds__(kThreads) void boxcar_pool_kernel(
    const uint32_t *__restrict__ Y, int64_t nout, int ncols, const int32_t *__restrict__ stats,
    WidthList widths, float scale, uint16_t *__restrict__ tiles) {
  extern __shared__ uint32_t P[];  // [kSeg + w_max]
  __shared__ float pv[kSeg];
  const int64_t blk = blockIdx.x;
  const int pair = (int)(blk / ncols), tj = (int)(blk - (int64_t)pair * ncols);
  const int d = 2 * pair, ti = d / kPoolTileDm, i = (d % kPoolTileDm) / 2;
  uint16_t *pooled = tiles + (((int64_t)ti * ncols + tj) * (kPoolTileDm / 2) + i) * (kSeg / 8);
  boxcar_pool_pair<NPOW>(Y, nout, d, tj, stats, widths, P, pv, scale, pooled);
}

template <int NPOW>
__global__ __launch_bounds__(kThreads) void boxcar_pool_batch_kernel(
    const BeamWork *__restrict__ beams, int nbeams, WidthList widths, float scale,
    uint16_t *__restrict__ tiles) {
  extern __shared__ uint32_t P[];
  __shared__ float pv[kSeg];
  const int64_t blk = blockIdx.x;
  const BeamWork &bw = beams[find_beam_wave<&BeamWork::pl_begin>(beams, nbeams, blk)];
  const int64_t local = blk - bw.pl_begin;
  const int ncols = (int)bw.pcols;
  const int pair = (int)(local / ncols), tj = (int)(local - (int64_t)pair * ncols);
  const int d = 2 * pair, ti = d / kPoolTileDm, i = (d % kPoolTileDm) / 2;
  uint16_t *pooled = tiles + ((bw.tile_begin + (int64_t)ti * ncols + tj) * (kPoolTileDm / 2) + i) *
                                 (kSeg / 8);
  boxcar_pool_pair<NPOW>(bw.Y, bw.nout, d, tj, bw.stats, widths, P, pv, scale, pooled);
}

// Dynamic LDS of the boxcar kernels: the window's prefix (kSeg + w_max words)
// and, for power-of-two widths, the padded scan extent.
size_t boxcar_lds_bytes(const WidthList &widths) {
  const int wmax = widths.w[widths.n - 1];
  size_t words = (size_t)kSeg + wmax + 1;
  const int ld = (kSeg + wmax - 1 + kThreads - 1) / kThreads;
  const size_t padded = (size_t)kThreads * (ld | 1) + 1;
  return (words > padded ? words : padded) * sizeof(uint32_t);
}

// 0: no tile maxima; 1: every segment inside one tile column (tile_t a
// multiple of the segment length); 2: any tiling.
int tile_mode(const void *keys, int64_t tile_t, bool rows_of_64) {
  if (!keys) return 0;
  return tile_t % kSeg == 0 ? 1 : (tile_t % 64 == 0 && rows_of_64 ? 3 : 2);
}

// f.run<NPOW, TILES, PK>() for a launch: NPOW = number of widths when they
// are 1, 2, 4, ... (else 0), TILES = tile mode; without planes PK = 2 where
// widths can be recomputed (TILES = 1, power-of-two widths), else 1.
template <int N, class F>
void boxcar_dispatch_n(int tm, bool planes, F &f) {
  if (planes) {
    if (tm == 0) f.template run<N, 0, 0>();
    else if (tm == 1) f.template run<N, 1, 0>();
    else if (tm == 3) f.template run<N, 3, 0>();
    else f.template run<N, 2, 0>();
  } else {
    if (tm == 1) f.template run<N, 1, (N > 0 ? 2 : 1)>();
    else if (tm == 3) f.template run<N, 3, 1>();
    else f.template run<N, 2, 1>();
  }
}

template <class F>
void boxcar_dispatch(const WidthList &widths, int tm, bool planes, F &f) {
  bool pow2 = widths.n <= 13;
  for (int i = 0; i < widths.n && pow2; ++i) pow2 = widths.w[i] == (1 << i);
  switch (pow2 ? widths.n : 0) {
    case 1: boxcar_dispatch_n<1>(tm, planes, f); break;
    case 2: boxcar_dispatch_n<2>(tm, planes, f); break;
    case 3: boxcar_dispatch_n<3>(tm, planes, f); break;
    case 4: boxcar_dispatch_n<4>(tm, planes, f); break;
    case 5: boxcar_dispatch_n<5>(tm, planes, f); break;
    case 6: boxcar_dispatch_n<6>(tm, planes, f); break;
    case 7: boxcar_dispatch_n<7>(tm, planes, f); break;
    case 8: boxcar_dispatch_n<8>(tm, planes, f); break;
    case 9: boxcar_dispatch_n<9>(tm, planes, f); break;
    case 10: boxcar_dispatch_n<10>(tm, planes, f); break;
    case 11: boxcar_dispatch_n<11>(tm, planes, f); break;
    case 12: boxcar_dispatch_n<12>(tm, planes, f); break;
    case 13: boxcar_dispatch_n<13>(tm, planes, f); break;
    default: boxcar_dispatch_n<0>(tm, planes, f); break;
  }
}

struct BoxcarLaunch {
  dim3 grid;
  size_t lds;
  hipStream_t stream;
  const uint32_t *Y;
  int64_t nout;
  int nseg;
  const int32_t *stats;
  WidthList widths;
  float *snr;
  uint8_t *best;
  TileSink sink;
  template <int N, int T, int K>
  void run() {
    hipLaunchKernelGGL((boxcar_kernel<N, T, K>), grid, dim3(kThreads), lds, stream, Y, nout, nseg,
                       stats, widths, snr, best, sink);
  }
};

struct BoxcarBatchLaunch {
  dim3 grid;
  size_t lds;
  hipStream_t stream;
  const BeamWork *beams;
  int nbeams;
  WidthList widths;
  uint8_t *scratch;
  int ndm, tile_dm;
  int64_t tile_t;
  template <int N, int T, int K>
  void run() {
    hipLaunchKernelGGL((boxcar_batch_kernel<N, T, K>), grid, dim3(kThreads), lds, stream, beams,
                       nbeams, widths, scratch, ndm, tile_dm, tile_t);
  }
};

}  // namespace

hipError_t launch_boxcar(const uint32_t *Y, int ndm, int64_t nout, const int32_t *stats,
                         const WidthList &widths, float *snr, uint8_t *best, hipStream_t stream,
                         const TileSink &sink) {
  const int64_t nseg = (nout + kSeg - 1) / kSeg;
  const int64_t grid = nseg * ndm;
  if (grid > 0x7FFFFFFF || nseg > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (sink.keys && (sink.tile_dm < 1 || sink.tile_t < 1)) return hipErrorInvalidValue;
  const bool planes = snr != nullptr;
  if (planes != (best != nullptr) || planes == (sink.packed != 0)) return hipErrorInvalidValue;
  if (!planes && !sink.keys) return hipErrorInvalidValue;
  const int tm = tile_mode(sink.keys, sink.tile_t, nout % 64 == 0);
  BoxcarLaunch f{dim3((unsigned)grid), boxcar_lds_bytes(widths), stream, Y, nout, (int)nseg,
                 stats, widths, snr, best, sink};
  boxcar_dispatch(widths, tm, planes, f);
  return hipGetLastError();
}

hipError_t launch_boxcar_batch(const BeamWork *beams, int nbeams, int64_t total_blocks,
                               const WidthList &widths, hipStream_t stream, uint8_t *scratch,
                               int ndm, int tile_dm, int64_t tile_t, bool rows_of_64,
                               bool planes) {
  if (total_blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (scratch && (tile_dm < 1 || tile_t < 1 || ndm < 1)) return hipErrorInvalidValue;
  if (!planes && !scratch) return hipErrorInvalidValue;
  const int tm = tile_mode(scratch, tile_t, rows_of_64);
  BoxcarBatchLaunch f{dim3((unsigned)total_blocks), boxcar_lds_bytes(widths), stream, beams,
                      nbeams, widths, scratch, ndm, tile_dm, tile_t};
  boxcar_dispatch(widths, tm, planes, f);
  return hipGetLastError();
}

hipError_t launch_tile_keys(const TileSink &sink, int ndm, int64_t nout, const uint8_t *best,
                            TilePeak *peaks, bool decode, hipStream_t stream) {
  if (!sink.keys || sink.tile_dm < 1 || sink.tile_t < 1) return hipErrorInvalidValue;
  const int64_t ntiles = (int64_t)((ndm + sink.tile_dm - 1) / sink.tile_dm) * sink.ntt;
  const int64_t grid = (ntiles + kThreads - 1) / kThreads;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(tile_keys_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream, sink,
                     ntiles, ndm, nout, best, peaks, decode ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_tile_keys_batch(const BeamWork *beams, int nbeams, int ndm, int64_t total_tiles,
                                  int tile_dm, int64_t tile_t, uint8_t *scratch, bool decode,
                                  bool packed, hipStream_t stream) {
  const int64_t grid = (total_tiles + kThreads - 1) / kThreads;
  if (grid > 0x7FFFFFFF || tile_dm < 1 || tile_t < 1) return hipErrorInvalidValue;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(tile_keys_batch_kernel, dim3((unsigned)grid), dim3(kThreads), 0, stream,
                     beams, nbeams, ndm, total_tiles, tile_dm, tile_t, scratch, decode ? 1 : 0,
                     packed ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_boxcar_pool(const uint32_t *Y, int ndm, int64_t nout, const int32_t *stats,
                              const WidthList &widths, float scale, uint16_t *tiles,
                              hipStream_t stream) {
  const int64_t ncols = nout / kSeg, pairs = (int64_t)(ndm / kPoolTileDm) * (kPoolTileDm / 2);
  const int64_t grid = pairs * ncols;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (grid == 0) return hipSuccess;
  bool pow2 = widths.n <= 13;
  for (int i = 0; i < widths.n && pow2; ++i) pow2 = widths.w[i] == (1 << i);
  const size_t lds = boxcar_lds_bytes(widths);
#define SPS_POOL_CASE(n_)                                                                       \
  if (pow2 && widths.n == n_) {                                                                 \
    hipLaunchKernelGGL(boxcar_pool_kernel<n_>, dim3((unsigned)grid), dim3(kThreads), lds, stream, \
                       Y, nout, (int)ncols, stats, widths, scale, tiles);                       \
    return hipGetLastError();                                                                   \
  }
  SPS_POOL_CASE(1) SPS_POOL_CASE(2) SPS_POOL_CASE(3) SPS_POOL_CASE(4) SPS_POOL_CASE(5)
  SPS_POOL_CASE(6) SPS_POOL_CASE(7) SPS_POOL_CASE(8) SPS_POOL_CASE(9) SPS_POOL_CASE(10)
  SPS_POOL_CASE(11) SPS_POOL_CASE(12) SPS_POOL_CASE(13)
#undef SPS_POOL_CASE
  hipLaunchKernelGGL(boxcar_pool_kernel<0>, dim3((unsigned)grid), dim3(kThreads), lds, stream, Y,
                     nout, (int)ncols, stats, widths, scale, tiles);
  return hipGetLastError();
}

hipError_t launch_boxcar_pool_batch(const BeamWork *beams, int nbeams, int64_t total_blocks,
                                    const WidthList &widths, float scale, uint16_t *tiles,
                                    hipStream_t stream) {
  if (total_blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (total_blocks == 0) return hipSuccess;
  bool pow2 = widths.n <= 13;
  for (int i = 0; i < widths.n && pow2; ++i) pow2 = widths.w[i] == (1 << i);
  const size_t lds = boxcar_lds_bytes(widths);
#define SPS_POOL_BCASE(n_)                                                                    \
  if (pow2 && widths.n == n_) {                                                               \
    hipLaunchKernelGGL(boxcar_pool_batch_kernel<n_>, dim3((unsigned)total_blocks), dim3(kThreads), \
                       lds, stream, beams, nbeams, widths, scale, tiles);                     \
    return hipGetLastError();                                                                 \
  }
  SPS_POOL_BCASE(1) SPS_POOL_BCASE(2) SPS_POOL_BCASE(3) SPS_POOL_BCASE(4) SPS_POOL_BCASE(5)
  SPS_POOL_BCASE(6) SPS_POOL_BCASE(7) SPS_POOL_BCASE(8) SPS_POOL_BCASE(9) SPS_POOL_BCASE(10)
  SPS_POOL_BCASE(11) SPS_POOL_BCASE(12) SPS_POOL_BCASE(13)
#undef SPS_POOL_BCASE
  hipLaunchKernelGGL(boxcar_pool_batch_kernel<0>, dim3((unsigned)total_blocks), dim3(kThreads), lds,
                     stream, beams, nbeams, widths, scale, tiles);
  return hipGetLastError();
}

int64_t boxcar_segments(int64_t nout) { return (nout + kSeg - 1) / kSeg; }

}  // namespace sps

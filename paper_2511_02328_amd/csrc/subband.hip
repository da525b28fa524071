// subband.hip -- the paper's own dedispersion path on gfx950: stage 2 of the
// two-stage subband method, the zero-DM filter and square-law downsampling.
//
// Stage 1 (Eq. stage1: per coarse DM, shift and sum the channels of each
// subband) is brute-force dedispersion restricted to a subband's channels
// over the coarse DM grid, so it runs on the dedispersion kernel of
// dedisperse.hip, once per subband.  Stage 2 (Eq. stage2) sums the subband
// series of the coarse group j(m) = floor(m / n0) with the residual shifts
// R[m][s] of Eq. (residual).
#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kS2Threads = 256;
constexpr int kS2Out = 4;  // outputs per thread

// Stage 2, Y[m][t] = sum_s I[s][j(m)][t + R[m][s]], one workgroup per coarse
// group j and 1024 output samples.  The subband loop is outside and up to
// GM fine DMs of the group are accumulated together, so the GM overlapping
// windows of one subband row (a few KB) are read back to back and served
// from L1, and each word of I leaves L2 about once per tile.  Rt: the
// residual table transposed, [nsub][ndm], so the GM shifts of one subband
// are one scalar load.
//
// Whole groups of GM trials on whole tiles take a branch-free path: thread i
// owns outputs t0 + 4 i .. t0 + 4 i + 3 and reads each trial's window with
// one 16-byte load at its (dword-aligned) offset; all GM loads of a subband
// are issued before the first add, and two subbands are in flight.  Group
// and tile edges take the guarded loop, in which thread i owns outputs
// t0 + i + 256 b (b < 4).
template <int GM>
__global__ __launch_bounds__(kS2Threads) void subband_stage2_blocked_kernel(
    const uint32_t *__restrict__ I, int64_t len1, int ncoarse, int nsub,
    const int32_t *__restrict__ Rt, int ndm, int n0, uint32_t *__restrict__ Y, int64_t nout,
    int64_t nchunks) {
  const int64_t blk = blockIdx.x;
  const int j = (int)(blk / nchunks);
  const int64_t t0 = (blk - (int64_t)j * nchunks) * kS2Threads * kS2Out;
  const int64_t t = t0 + threadIdx.x;
  const bool full_tile = t0 + kS2Threads * kS2Out <= nout;
  const int mend = min((j + 1) * n0, ndm);
  const int64_t plane = (int64_t)ncoarse * len1;
  const uint32_t *base = I + (int64_t)j * len1 + t;
  for (int m0 = j * n0; m0 < mend; m0 += GM) {
    const int gm = min(GM, mend - m0);
    uint32_t acc[GM][kS2Out];
#pragma unroll
    for (int a = 0; a < GM; ++a)
#pragma unroll
      for (int b = 0; b < kS2Out; ++b) acc[a][b] = 0u;
    if (gm == GM && full_tile) {
      // Lane-consecutive outputs here: the thread owns t0 + 4 tid .. + 3 and
      // reads each trial's window with one 16-byte load at its dword offset
      // (four times fewer load instructions than one dword per output).
      static_assert(kS2Out == 4, "one 16-byte load per trial");
      const uint32_t *base4 = I + (int64_t)j * len1 + t0 + 4 * (int64_t)threadIdx.x;
#pragma unroll 2
      for (int sb = 0; sb < nsub; ++sb) {
        const uint32_t *row = base4 + (int64_t)sb * plane;
        const int32_t *Rs = Rt + (int64_t)sb * ndm + m0;
        u32x4_a4 v[GM];
#pragma unroll
        for (int a = 0; a < GM; ++a) v[a] = *(const SPS_GLOBAL u32x4_a4 *)gmem(row + Rs[a]);
#pragma unroll
        for (int a = 0; a < GM; ++a) {
          acc[a][0] += v[a].x;
          acc[a][1] += v[a].y;
          acc[a][2] += v[a].z;
          acc[a][3] += v[a].w;
        }
      }
      const bool vec = ((reinterpret_cast<uintptr_t>(Y) & 15) == 0) && (nout & 3) == 0;
#pragma unroll
      for (int a = 0; a < GM; ++a) {
        SPS_GLOBAL uint32_t *Ym = gmem(Y + (int64_t)(m0 + a) * nout + t0 + 4 * (int64_t)threadIdx.x);
        if (vec) {
          *(SPS_GLOBAL u32x4 *)Ym = u32x4{acc[a][0], acc[a][1], acc[a][2], acc[a][3]};
        } else {
#pragma unroll
          for (int b = 0; b < 4; ++b) Ym[b] = acc[a][b];
        }
      }
      continue;
    } else if (t < nout) {
      for (int sb = 0; sb < nsub; ++sb) {
        const uint32_t *row = base + (int64_t)sb * plane;
        for (int a = 0; a < gm; ++a) {
          const uint32_t *w = row + Rt[(int64_t)sb * ndm + m0 + a];
#pragma unroll
          for (int b = 0; b < kS2Out; ++b)
            if (t + b * kS2Threads < nout) acc[a][b] += w[b * kS2Threads];
        }
      }
    }
    if (t < nout) {
#pragma unroll
      for (int a = 0; a < GM; ++a) {
        if (a < gm) {
          uint32_t *Ym = Y + (int64_t)(m0 + a) * nout + t;
#pragma unroll
          for (int b = 0; b < kS2Out; ++b)
            if (t + b * kS2Threads < nout) Ym[b * kS2Threads] = acc[a][b];
        }
      }
    }
  }
}

// Zero-DM filter: X'[c][t] = clip(X[c][t] - m(t) + 128, 0, 255) with m(t) the
// channel mean rounded half up.  A thread owns 4 consecutive samples; the
// column is read twice (sum, then apply), row by row, coalesced across lanes.
__global__ __launch_bounds__(256) void zero_dm_kernel(const uint8_t *__restrict__ X, int64_t pitch,
                                                      int64_t nsamp, int nchan,
                                                      uint8_t *__restrict__ Xo,
                                                      int64_t pitch_out) {
  const int64_t t = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  if (t >= nsamp) return;
  const bool full = t + 4 <= nsamp;
  uint32_t sum[4] = {0u, 0u, 0u, 0u};
  for (int c = 0; c < nchan; ++c) {
    const uint8_t *row = X + (int64_t)c * pitch + t;
    if (full) {
      const uint32_t w = *reinterpret_cast<const uint32_t *>(row);
#pragma unroll
      for (int b = 0; b < 4; ++b) sum[b] += (w >> (8 * b)) & 0xFFu;
    } else {
      for (int b = 0; b < 4; ++b)
        if (t + b < nsamp) sum[b] += row[b];
    }
  }
  int32_t mean[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) mean[b] = (int32_t)((sum[b] + (uint32_t)(nchan / 2)) / (uint32_t)nchan);
  for (int c = 0; c < nchan; ++c) {
    const uint8_t *row = X + (int64_t)c * pitch + t;
    uint8_t *out = Xo + (int64_t)c * pitch_out + t;
    if (full) {
      const uint32_t w = *reinterpret_cast<const uint32_t *>(row);
      uint32_t o = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int32_t v = (int32_t)((w >> (8 * b)) & 0xFFu) - mean[b] + 128;
        o |= (uint32_t)(v < 0 ? 0 : (v > 255 ? 255 : v)) << (8 * b);
      }
      *reinterpret_cast<uint32_t *>(out) = o;
    } else {
      for (int b = 0; b < 4; ++b)
        if (t + b < nsamp) {
          const int32_t v = (int32_t)row[b] - mean[b] + 128;
          out[b] = (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
        }
    }
  }
}

// Square-law downsampling (Sec. 2.2): out = min(sqrt(255 S / N), 255), S the
// sum of a bin of N samples, rounded half up.  The float square root gives a
// first guess; the rounding is then settled exactly in 64-bit integers:
// (2r - 1)^2 N <= 4 * 255 S < (2r + 1)^2 N.
__global__ __launch_bounds__(256) void downsample_sqrt_kernel(
    const uint8_t *__restrict__ X, int64_t pitch, int factor, int64_t nout, int nchan,
    uint8_t *__restrict__ Xo, int64_t pitch_out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (t >= nout || c >= nchan) return;
  const uint8_t *row = X + (int64_t)c * pitch + t * factor;
  int64_t S = 0;
  for (int k = 0; k < factor; ++k) S += row[k];
  const int64_t V = 255, N = factor;
  int64_t r = (int64_t)(sqrtf((float)(V * S) / (float)N) + 0.5f);
  while ((2 * r + 1) * (2 * r + 1) * N <= 4 * V * S) ++r;
  while (r > 0 && (2 * r - 1) * (2 * r - 1) * N > 4 * V * S) --r;
  Xo[(int64_t)c * pitch_out + t] = (uint8_t)(r > V ? V : r);
}

}  // namespace

hipError_t launch_subband_stage2(const uint32_t *I, int64_t len1, int ncoarse, int nsub,
                                 const int32_t *Rt, int rmax, int ndm, int n0, uint32_t *Y,
                                 int64_t nout, hipStream_t stream) {
  const int64_t per_block = (int64_t)kS2Threads * kS2Out;
  const int64_t nchunks = (nout + per_block - 1) / per_block;
  const int64_t grid = nchunks * ncoarse;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  (void)rmax;
  hipLaunchKernelGGL(subband_stage2_blocked_kernel<8>, dim3((unsigned)grid), dim3(kS2Threads), 0,
                     stream, I, len1, ncoarse, nsub, Rt, ndm, n0, Y, nout, nchunks);
  return hipGetLastError();
}

hipError_t launch_zero_dm(const uint8_t *X, int64_t pitch, int64_t nsamp, int nchan, uint8_t *Xo,
                          int64_t pitch_out, hipStream_t stream) {
  const int64_t threads = (nsamp + 3) / 4;
  const int64_t grid = (threads + 255) / 256;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_dm_kernel, dim3((unsigned)grid), dim3(256), 0, stream, X, pitch, nsamp,
                     nchan, Xo, pitch_out);
  return hipGetLastError();
}

hipError_t launch_downsample_sqrt(const uint8_t *X, int64_t pitch, int64_t nsamp, int nchan,
                                  int factor, uint8_t *Xo, int64_t pitch_out,
                                  hipStream_t stream) {
  const int64_t nout = nsamp / factor;
  const int64_t gx = (nout + 255) / 256;
  if (gx > 0x7FFFFFFF || nchan > 65535) return hipErrorInvalidValue;
  if (gx == 0) return hipSuccess;
  hipLaunchKernelGGL(downsample_sqrt_kernel, dim3((unsigned)gx, (unsigned)nchan), dim3(256), 0,
                     stream, X, pitch, factor, nout, nchan, Xo, pitch_out);
  return hipGetLastError();
}

}  // namespace sps

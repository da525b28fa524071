// dedisperse.hip -- brute-force incoherent dedispersion on gfx950.
//
// Computes Y[d][t] = sum_c X[c][t + D[d][c]] (ASTROFLOW Sec. 2.3, the direct
// method of cost N_DM N_t N_f; samples at or past nsamp_in count as zero as in
// Eq. stage1) exactly in integers.
//
// Design (CDNA4, wave64):
//  * A workgroup owns a block of nd = nw * dpw consecutive trials and a time
//    tile of nt = 256 m outputs.  Channels are processed in slabs of cs rows;
//    for each channel the slab row holds the input window that every trial of
//    the block needs, [t0 + D[d_lo][c] & ~15, ... + lds_pitch), loaded with
//    coalesced, 16-byte-aligned vector reads (one wave per row) and
//    zero-filled past nsamp_in.
//  * Lanes run along time: lane i owns outputs t0 + 4(i m + j) + b, j < m,
//    b < 4.  For one (trial, channel) the delay is wave-uniform, so a lane
//    reads m + 1 consecutive dwords of the staged row at a uniform byte
//    offset.  Lane stride m is odd, so the 64 lanes hit distinct LDS banks.
//  * Bytes are summed as packed u16 pairs (SWAR): v_perm_b32 with a
//    wave-uniform selector both realigns the window and spreads bytes
//    (t, t+2) resp. (t+1, t+3) into the two 16-bit halves of a dword; two
//    channels are added per v_add3_u32.  A u16 half holds at most 256 bytes
//    (255 * 256 < 2^16), so every 256 channels the halves are folded into
//    u32 accumulators.  Cost: about 3 VALU ops per 8 sample-adds plus one
//    address add per (trial, channel), against 1 op per add for a plain
//    byte-extract-and-add loop.
//  * Workgroups are dealt to the 8 XCDs round-robin by the hardware; the
//    logical index is remapped so that each XCD walks a contiguous range with
//    the DM block fastest, so the workgroups resident on one XCD share most
//    of their input windows in that XCD's L2.
#include "sps_internal.h"

namespace sps {
namespace {

__device__ __forceinline__ uint32_t perm_bytes(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// Selector that takes bytes (r, r+2) of the 8-byte window {hi:lo} into the
// low bytes of the two u16 halves and zeroes the high bytes; +0x00010001
// gives bytes (r+1, r+3).
__device__ __forceinline__ uint32_t even_selector(int off) {
  const uint32_t r = (uint32_t)off & 3u;
  return 0x0C000C00u | r | ((r + 2u) << 16);
}

// Adds two channels' windows (byte offsets offa, offb into staged rows r and
// r + 1) into the packed accumulators of one trial.
template <int M>
__device__ __forceinline__ void add_pair(uint32_t (&ev)[M], uint32_t (&od)[M],
                                         const uint32_t *lds32, int row_dw, int lane, int r,
                                         int offa, int offb) {
  const uint32_t sea = even_selector(offa), soa = sea + 0x00010001u;
  const uint32_t seb = even_selector(offb), sob = seb + 0x00010001u;
  const uint32_t *pa = lds32 + r * row_dw + (offa >> 2) + lane * M;
  const uint32_t *pb = lds32 + (r + 1) * row_dw + (offb >> 2) + lane * M;
  uint32_t wa[M + 1], wb[M + 1];
#pragma unroll
  for (int j = 0; j <= M; ++j) {
    wa[j] = pa[j];
    wb[j] = pb[j];
  }
#pragma unroll
  for (int j = 0; j < M; ++j) {
    ev[j] += perm_bytes(wa[j + 1], wa[j], sea) + perm_bytes(wb[j + 1], wb[j], seb);
    od[j] += perm_bytes(wa[j + 1], wa[j], soa) + perm_bytes(wb[j + 1], wb[j], sob);
  }
}

template <int M>
__device__ __forceinline__ void add_one(uint32_t (&ev)[M], uint32_t (&od)[M],
                                        const uint32_t *lds32, int row_dw, int lane, int r,
                                        int offa) {
  const uint32_t sea = even_selector(offa), soa = sea + 0x00010001u;
  const uint32_t *pa = lds32 + r * row_dw + (offa >> 2) + lane * M;
  uint32_t wa[M + 1];
#pragma unroll
  for (int j = 0; j <= M; ++j) wa[j] = pa[j];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    ev[j] += perm_bytes(wa[j + 1], wa[j], sea);
    od[j] += perm_bytes(wa[j + 1], wa[j], soa);
  }
}

template <int M, int DPW, int NW, int CS>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void dedisperse_kernel(
    const uint8_t *__restrict__ X, int64_t pitch, int64_t nsamp_in,
    const int32_t *__restrict__ D, int nchan, int ndm, uint32_t *__restrict__ Y,
    int64_t nout, int lds_pitch, int ntiles, int ndmb, int per_xcd, int vec_store) {
  static_assert(M % 2 == 1, "lane stride must be odd for conflict-free LDS reads");
  static_assert(CS % 2 == 0 && 256 % CS == 0, "slab must be even and divide 256");
  constexpr int NT = 256 * M;
  constexpr int ND = NW * DPW;
  extern __shared__ uint4 smem[];

  const int blk = blockIdx.x;
  const int logical = (blk & 7) * per_xcd + (blk >> 3);
  if (logical >= ntiles * ndmb) return;
  const int dblk = logical % ndmb;
  const int tile = logical / ndmb;
  const int64_t t0 = (int64_t)tile * NT;
  const int d_lo = dblk * ND;

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int dw0 = d_lo + wave * DPW;
  const int vpr = lds_pitch >> 4;
  const int row_dw = lds_pitch >> 2;

  uint32_t acc[DPW][M][4];
  uint32_t ev[DPW][M], od[DPW][M];
#pragma unroll
  for (int k = 0; k < DPW; ++k)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      ev[k][j] = 0u;
      od[k][j] = 0u;
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[k][j][b] = 0u;
    }

  const int32_t *Dlo = D + (int64_t)d_lo * nchan;
  const uint32_t *lds32 = reinterpret_cast<const uint32_t *>(smem);

  for (int c0 = 0; c0 < nchan; c0 += CS) {
    const int ncs = min(CS, nchan - c0);
    __syncthreads();
    // Stage the slab: wave w loads rows w, w + NW, ...
    for (int r = wave; r < ncs; r += NW) {
      const int64_t base = t0 + (int64_t)(Dlo[c0 + r] & ~15);
      const uint8_t *rowp = X + (int64_t)(c0 + r) * pitch;
      uint4 *dst = smem + r * vpr;
      for (int k0 = 0; k0 < vpr; k0 += 256) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + lane + 64 * u;
          const int64_t s0 = base + 16 * (int64_t)k;
          v[u] = make_uint4(0u, 0u, 0u, 0u);
          if (k < vpr && s0 < nsamp_in) {
            v[u] = *reinterpret_cast<const uint4 *>(rowp + s0);
            const int64_t nv = nsamp_in - s0;
            if (nv < 16) {
              uint32_t w4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int64_t keep = nv - 4 * q;
                w4[q] = keep >= 4 ? w4[q] : (keep <= 0 ? 0u : (w4[q] & ((1u << (8 * keep)) - 1u)));
              }
              v[u] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + lane + 64 * u;
          if (k < vpr) dst[k] = v[u];
        }
      }
    }
    __syncthreads();

    if (ncs == CS) {
      // Full slab: delays of all CS channels are loaded to SGPRs up front and
      // the channel loop is unrolled.
#pragma unroll
      for (int k = 0; k < DPW; ++k) {
        const int d = dw0 + k;
        if (d < ndm) {
          const int32_t *Dd = D + (int64_t)d * nchan + c0;
#pragma unroll
          for (int r = 0; r < CS; r += 2)
            add_pair<M>(ev[k], od[k], lds32, row_dw, lane, r, Dd[r] - (Dlo[c0 + r] & ~15),
                        Dd[r + 1] - (Dlo[c0 + r + 1] & ~15));
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < DPW; ++k) {
        const int d = dw0 + k;
        if (d < ndm) {
          const int32_t *Dd = D + (int64_t)d * nchan + c0;
          int r = 0;
          for (; r + 1 < ncs; r += 2)
            add_pair<M>(ev[k], od[k], lds32, row_dw, lane, r, Dd[r] - (Dlo[c0 + r] & ~15),
                        Dd[r + 1] - (Dlo[c0 + r + 1] & ~15));
          if (r < ncs)
            add_one<M>(ev[k], od[k], lds32, row_dw, lane, r, Dd[r] - (Dlo[c0 + r] & ~15));
        }
      }
    }

    if (((c0 + CS) & 255) == 0 || c0 + CS >= nchan) {
#pragma unroll
      for (int k = 0; k < DPW; ++k)
#pragma unroll
        for (int j = 0; j < M; ++j) {
          acc[k][j][0] += ev[k][j] & 0xFFFFu;
          acc[k][j][2] += ev[k][j] >> 16;
          acc[k][j][1] += od[k][j] & 0xFFFFu;
          acc[k][j][3] += od[k][j] >> 16;
          ev[k][j] = 0u;
          od[k][j] = 0u;
        }
    }
  }

#pragma unroll
  for (int k = 0; k < DPW; ++k) {
    const int d = dw0 + k;
    if (d >= ndm) continue;
    uint32_t *Yd = Y + (int64_t)d * nout;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t t = t0 + 4 * (int64_t)(lane * M + j);
      if (vec_store && t + 4 <= nout) {
        *reinterpret_cast<uint4 *>(Yd + t) =
            make_uint4(acc[k][j][0], acc[k][j][1], acc[k][j][2], acc[k][j][3]);
      } else {
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (t + b < nout) Yd[t + b] = acc[k][j][b];
      }
    }
  }
}

// Plain fallback for delay spreads too wide to stage in LDS: one thread sums
// four consecutive outputs of one trial straight from global memory.
__global__ __launch_bounds__(256) void dedisperse_direct_kernel(
    const uint8_t *__restrict__ X, int64_t pitch, int64_t nsamp_in,
    const int32_t *__restrict__ D, int nchan, int ndm, uint32_t *__restrict__ Y, int64_t nout) {
  const int64_t t = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  if (t >= nout) return;
  for (int d = blockIdx.y; d < ndm; d += gridDim.y) {
    const int32_t *Dd = D + (int64_t)d * nchan;
    uint32_t acc[4] = {0u, 0u, 0u, 0u};
    for (int c = 0; c < nchan; ++c) {
      const uint8_t *row = X + (int64_t)c * pitch;
      const int64_t s = t + Dd[c];
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (s + b < nsamp_in) acc[b] += row[s + b];
    }
    uint32_t *Yd = Y + (int64_t)d * nout;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (t + b < nout) Yd[t + b] = acc[b];
  }
}

template <int M, int DPW, int NW, int CS>
hipError_t launch_cfg(int lds_pitch, const uint8_t *X, int64_t pitch, int64_t nsamp_in,
                      const int32_t *D, int nchan, int ndm, uint32_t *Y, int64_t nout,
                      hipStream_t stream) {
  constexpr int NT = 256 * M;
  constexpr int ND = NW * DPW;
  const int64_t ntiles64 = (nout + NT - 1) / NT;
  const int ndmb = (ndm + ND - 1) / ND;
  const int64_t total = ntiles64 * ndmb;
  if (total > (int64_t)0x7FFFFFFF - 8) return hipErrorInvalidValue;
  const int per_xcd = (int)((total + 7) / 8);
  const int grid = per_xcd * 8;
  const size_t lds = (size_t)CS * (size_t)lds_pitch;
  const int vec_store = (nout % 4 == 0) && ((reinterpret_cast<uintptr_t>(Y) & 15) == 0);
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&dedisperse_kernel<M, DPW, NW, CS>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((dedisperse_kernel<M, DPW, NW, CS>), dim3(grid), dim3(NW * 64), lds, stream,
                     X, pitch, nsamp_in, D, nchan, ndm, Y, nout, lds_pitch, (int)ntiles64, ndmb,
                     per_xcd, vec_store);
  return hipGetLastError();
}

}  // namespace

int64_t dedisp_lds_pitch(const DedispConfig &cfg, int spread) {
  // Largest byte a lane touches: (spread + 15) alignment slack + nt + 3.
  const int64_t need = (int64_t)spread + cfg.nt() + 19;
  return (need + 15) & ~(int64_t)15;
}

int dedisp_block_spread(const int32_t *Dh, int nchan, int ndm, int nd) {
  int spread = 0;
  for (int d0 = 0; d0 < ndm; d0 += nd) {
    const int d1 = (d0 + nd < ndm ? d0 + nd : ndm) - 1;
    const int32_t *lo = Dh + (int64_t)d0 * nchan;
    const int32_t *hi = Dh + (int64_t)d1 * nchan;
    for (int c = 0; c < nchan; ++c) {
      const int s = hi[c] - lo[c];
      if (s > spread) spread = s;
    }
  }
  return spread;
}

#define SPS_DEDISP_CONFIGS(X) \
  X(5, 2, 8, 16)              \
  X(3, 2, 8, 16)              \
  X(7, 2, 8, 16)              \
  X(5, 1, 8, 16)              \
  X(5, 2, 4, 16)              \
  X(3, 4, 4, 16)              \
  X(5, 2, 8, 32)              \
  X(3, 4, 8, 16)

bool dedisp_config_supported(const DedispConfig &c) {
#define SPS_MATCH(m_, dpw_, nw_, cs_) \
  if (c.m == m_ && c.dpw == dpw_ && c.nw == nw_ && c.cs == cs_) return true;
  SPS_DEDISP_CONFIGS(SPS_MATCH)
#undef SPS_MATCH
  return false;
}

hipError_t launch_dedisperse(const DedispConfig &c, int lds_pitch, const uint8_t *X,
                             int64_t pitch, int64_t nsamp_in, const int32_t *D, int nchan,
                             int ndm, uint32_t *Y, int64_t nout, hipStream_t stream) {
  if (c.m == 0) {
    const int64_t nthreads = (nout + 3) / 4;
    const int64_t gx = (nthreads + 255) / 256;
    if (gx > 0x7FFFFFFF) return hipErrorInvalidValue;
    const int gy = ndm < 65535 ? ndm : 65535;
    hipLaunchKernelGGL(dedisperse_direct_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0,
                       stream, X, pitch, nsamp_in, D, nchan, ndm, Y, nout);
    return hipGetLastError();
  }
#define SPS_LAUNCH(m_, dpw_, nw_, cs_)                                                    \
  if (c.m == m_ && c.dpw == dpw_ && c.nw == nw_ && c.cs == cs_)                           \
    return launch_cfg<m_, dpw_, nw_, cs_>(lds_pitch, X, pitch, nsamp_in, D, nchan, ndm, Y, \
                                          nout, stream);
  SPS_DEDISP_CONFIGS(SPS_LAUNCH)
#undef SPS_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace sps

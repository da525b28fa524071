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
//  * The delay table is read in a staged form built once per tiling
//    (stage_delays): per (trial, channel) the LDS dword offset of its window
//    inside a slab buffer and its perm selector, per (DM block, channel) the
//    16-aligned first staged sample.  A wave loads a slab's entries with
//    wide scalar loads and spends two scalar ops per channel on them, so the
//    scalar unit, which issues at the same rate as the vector unit, stays
//    well below it.
//  * Workgroups are dealt to the 8 XCDs round-robin by the hardware; the
//    logical index is remapped so that each XCD walks a contiguous range in
//    panels of a few DM blocks (DM block fastest inside a panel, then time),
//    so the workgroups resident on one XCD share their staged delay rows and
//    most of their input windows in that XCD's L2.
#include "sps_internal.h"

namespace sps {
namespace {

__device__ __forceinline__ uint32_t perm_bytes(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// Uniform LDS dword offset of a window: slab buffer base + staged offset,
// kept opaque so that the compiler forms each lane address with one add
// instead of holding a register per staged row.
__device__ __forceinline__ int uniform_offset(int buf_dw, int staged) {
  int s = buf_dw + staged;
  asm volatile("" : "+s"(s));
  return s;
}

// Adds two channels' windows into the packed accumulators of one trial.
// ea, eb: staged entries (LDS dword offset within the slab buffer, selector
// that takes bytes (r, r+2) of the 8-byte window {hi:lo} into the low bytes
// of the two u16 halves, r the delay mod 4); + 0x00010001 selects bytes
// (r+1, r+3).
template <int M>
__device__ __forceinline__ void add_pair(uint32_t (&ev)[M], uint32_t (&od)[M],
                                         const uint32_t *lds32, int lane_m, int bo, int2 ea,
                                         int2 eb) {
  const uint32_t sea = (uint32_t)ea.y, soa = sea + 0x00010001u;
  const uint32_t seb = (uint32_t)eb.y, sob = seb + 0x00010001u;
  const uint32_t *pa = lds32 + (lane_m + uniform_offset(bo, ea.x));
  const uint32_t *pb = lds32 + (lane_m + uniform_offset(bo, eb.x));
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

template <int CS, int NW, int KMAX>
struct SlabRegs {
  static constexpr int RPW = CS / NW;
  uint4 v[RPW][KMAX];
};

// Global -> registers for the slab starting at channel c0; Bb: first staged
// sample (16-aligned) of each channel's row for this DM block.  Rows whose
// whole window lies below nsamp_in take a guard-free path; the others
// zero-fill every byte at or past nsamp_in.  Rows >= ncs (past the last
// channel) are zero.  The registers are cleared first and loaded in place,
// so that the loads stay in flight while the current slab is summed.
template <int CS, int NW, int KMAX>
__device__ __forceinline__ void slab_load(SlabRegs<CS, NW, KMAX> &st, const uint8_t *__restrict__ X,
                                          int64_t pitch, int64_t nsamp_in,
                                          const int32_t *__restrict__ Bb, int c0, int ncs,
                                          int64_t t0, int vpr, int wave, int lane) {
#pragma unroll
  for (int i = 0; i < SlabRegs<CS, NW, KMAX>::RPW; ++i) {
    const int r = wave + NW * i;
#pragma unroll
    for (int u = 0; u < KMAX; ++u) st.v[i][u] = make_uint4(0u, 0u, 0u, 0u);
    if (r < ncs) {
      const int64_t base = t0 + (int64_t)Bb[c0 + r];
      const SPS_GLOBAL uint8_t *rowp = gmem(X + (int64_t)(c0 + r) * pitch);
      if (base + 16 * (int64_t)vpr <= nsamp_in) {
        const SPS_GLOBAL u32x4 *src = (const SPS_GLOBAL u32x4 *)(rowp + base);
#pragma unroll
        for (int u = 0; u < KMAX; ++u) {
          const int k = lane + 64 * u;
          if (k < vpr) {
            const u32x4 v = src[k];
            st.v[i][u] = make_uint4(v.x, v.y, v.z, v.w);
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < KMAX; ++u) {
          const int k = lane + 64 * u;
          const int64_t s0 = base + 16 * (int64_t)k;
          if (k < vpr && s0 < nsamp_in) {
            const u32x4 v = *(const SPS_GLOBAL u32x4 *)(rowp + s0);
            uint32_t w4[4] = {v.x, v.y, v.z, v.w};
            const int64_t nv = nsamp_in - s0;
            if (nv < 16) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int64_t keep = nv - 4 * q;
                w4[q] = keep >= 4 ? w4[q]
                                  : (keep <= 0 ? 0u : (w4[q] & ((1u << (8 * keep)) - 1u)));
              }
            }
            st.v[i][u] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
          }
        }
      }
    }
  }
}

// Interior form of slab_load, for workgroups whose every staged window lies
// below nsamp_in and whose slabs are all whole (nchan a multiple of CS): no
// guards and no clearing.  Every lane loads; lanes past the row repeat its
// last vector, which slab_store skips.
template <int CS, int NW, int KMAX>
__device__ __forceinline__ void slab_load_interior(SlabRegs<CS, NW, KMAX> &st,
                                                   const uint8_t *__restrict__ X, int64_t pitch,
                                                   const int32_t *__restrict__ Bb, int c0,
                                                   int64_t t0, int vpr, int wave, int lane) {
#pragma unroll
  for (int i = 0; i < SlabRegs<CS, NW, KMAX>::RPW; ++i) {
    const int c = c0 + wave + NW * i;
    // native 4-vector loads: a struct copy of uint4 becomes a memcpy that
    // the compiler keeps in scratch memory
    const SPS_GLOBAL u32x4 *src =
        (const SPS_GLOBAL u32x4 *)gmem(X + (int64_t)c * pitch + t0 + (int64_t)Bb[c]);
#pragma unroll
    for (int u = 0; u < KMAX; ++u) {
      const u32x4 v = src[min(lane + 64 * u, vpr - 1)];
      st.v[i][u] = make_uint4(v.x, v.y, v.z, v.w);
    }
  }
}

template <int CS, int NW, int KMAX>
__device__ __forceinline__ void slab_store(const SlabRegs<CS, NW, KMAX> &st, uint4 *buf, int vpr,
                                           int wave, int lane) {
#pragma unroll
  for (int i = 0; i < SlabRegs<CS, NW, KMAX>::RPW; ++i) {
    const int r = wave + NW * i;
#pragma unroll
    for (int u = 0; u < KMAX; ++u) {
      const int k = lane + 64 * u;
      if (k < vpr) buf[r * vpr + k] = st.v[i][u];
    }
  }
}

// Writes the accumulators of trials dw0 .. dw0 + DPW - 1 at outputs
// t0 + 4 (lane m + j) + b of plane Y.
template <int M, int DPW>
__device__ __forceinline__ void store_acc(const uint32_t (&acc)[DPW][M][4], uint32_t *__restrict__ Y,
                                          int64_t nout, int ndm, int dw0, int lane, int64_t t0,
                                          int vec_store) {
#pragma unroll
  for (int k = 0; k < DPW; ++k) {
    const int d = dw0 + k;
    if (d >= ndm) continue;
    SPS_GLOBAL uint32_t *Yd = gmem(Y + (int64_t)d * nout);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t t = t0 + 4 * (int64_t)(lane * M + j);
      if (vec_store && t + 4 <= nout) {
        *(SPS_GLOBAL u32x4 *)(Yd + t) = u32x4{acc[k][j][0], acc[k][j][1], acc[k][j][2], acc[k][j][3]};
      } else {
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (t + b < nout) Yd[t + b] = acc[k][j][b];
      }
    }
  }
}

// One workgroup's share: trials [d_lo, d_lo + nw dpw) of DM block dblk x
// outputs [t0, t0 + 256 m) of one filterbank.  P (pcols entries per trial,
// channels padded to a multiple of CS), B: the staged delay table of this
// tiling.  With seg > 0 (a multiple of CS) the channels form consecutive
// groups of seg and group g's partial sums go to plane Y + g seg_stride
// instead of one total (the first stage of subband dedispersion in one pass
// over all channels).  Ends with a barrier, so the caller may reuse the LDS
// buffers right away.
//
// The channel loop is two nested loops: slabs inside a fold group (at most
// 256 channels, ending at a segment end), the fold of the u16 halves after
// each group, so the slab loop carries the packed accumulators without
// branches.  Padded channels of a last partial slab point at zeroed rows.
template <int M, int DPW, int NW, int CS, int KMAX, bool SEG = false, bool INTERIOR = false>
__device__ __forceinline__ void dedisperse_block(
    const uint8_t *__restrict__ X, int64_t pitch, int64_t nsamp_in, const int2 *__restrict__ P,
    int pcols, const int32_t *__restrict__ B, int nchan, int ndm, uint32_t *__restrict__ Y,
    int64_t nout, int lds_pitch, int vec_store, int64_t t0, int dblk, uint4 *smem, int seg = 0,
    int64_t seg_stride = 0) {
  static_assert(M % 2 == 1, "lane stride must be odd for conflict-free LDS reads");
  static_assert(CS % 8 == 0 && 256 % CS == 0, "slab must be a multiple of 8 dividing 256");
  static_assert(CS % NW == 0, "every wave stages the same number of rows");
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int dw0 = dblk * (NW * DPW) + wave * DPW;
  const int vpr = lds_pitch >> 4;
  const int buf_dw = CS * (lds_pitch >> 2);
  const int lane_m = lane * M;

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

  // Trials past the last one (a partial DM block) repeat the last trial's
  // entries, so the channel loop has no per-trial branch; store_acc drops
  // them.
  const int2 *Pk[DPW];
#pragma unroll
  for (int k = 0; k < DPW; ++k) Pk[k] = P + (int64_t)min(dw0 + k, ndm - 1) * pcols;
  const int32_t *Bb = B + (int64_t)dblk * nchan;
  const uint32_t *lds32 = reinterpret_cast<const uint32_t *>(smem);
  SlabRegs<CS, NW, KMAX> st;

  if constexpr (INTERIOR)
    slab_load_interior(st, X, pitch, Bb, 0, t0, vpr, wave, lane);
  else
    slab_load(st, X, pitch, nsamp_in, Bb, 0, min(CS, nchan), t0, vpr, wave, lane);
  slab_store(st, smem, vpr, wave, lane);
  __syncthreads();

  int parity = 0;
#pragma unroll 1
  for (int g0 = 0; g0 < nchan;) {
    int g1 = min(nchan, (g0 + 256) & ~255);
    if constexpr (SEG) g1 = min(g1, (g0 / seg + 1) * seg);
#pragma unroll 1
    for (int c0 = g0; c0 < g1; c0 += CS) {
      const int c1 = c0 + CS;
      const bool more = c1 < nchan;
      if (more) {
        if constexpr (INTERIOR)
          slab_load_interior(st, X, pitch, Bb, c1, t0, vpr, wave, lane);
        else
          slab_load(st, X, pitch, nsamp_in, Bb, c1, min(CS, nchan - c1), t0, vpr, wave, lane);
      }
      const int bo = parity * buf_dw;
#pragma unroll
      for (int k = 0; k < DPW; ++k) {
        const int2 *Pc = Pk[k] + c0;
#pragma unroll
        for (int r0 = 0; r0 < CS; r0 += 8) {
          int2 e[8];
#pragma unroll
          for (int r = 0; r < 8; ++r) e[r] = Pc[r0 + r];
#pragma unroll
          for (int r = 0; r < 8; r += 2) {
            add_pair<M>(ev[k], od[k], lds32, lane_m, bo, e[r], e[r + 1]);
            // the sums stay a chain, one pair at a time: regrouped, they
            // would keep a slab's perms live at once
#pragma unroll
            for (int j = 0; j < M; ++j) asm volatile("" : "+v"(ev[k][j]), "+v"(od[k][j]));
          }
        }
      }
      if (more) slab_store(st, smem + (parity ^ 1) * (buf_dw >> 2), vpr, wave, lane);
      __syncthreads();
      parity ^= 1;
    }
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
    if constexpr (SEG) {
      if (g1 % seg == 0) {
        store_acc<M, DPW>(acc, Y + (int64_t)(g0 / seg) * seg_stride, nout, ndm, dw0, lane, t0,
                          vec_store);
#pragma unroll
        for (int k = 0; k < DPW; ++k)
#pragma unroll
          for (int j = 0; j < M; ++j)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[k][j][b] = 0u;
      }
    }
    g0 = g1;
  }

  if constexpr (!SEG) store_acc<M, DPW>(acc, Y, nout, ndm, dw0, lane, t0, vec_store);
}

// DM blocks per panel of the workgroup order.  The 64 workgroups resident on
// an XCD then cover about 8 DM blocks x 8 time tiles: the staged delay rows
// of 8 blocks (8 x 16 trials x nchan entries) stay in the XCD's L2 and the
// input windows of neighbouring blocks and tiles overlap.  Measured on the
// full-scale chunk: 3x less fetched from memory than the DM block running
// fastest over all blocks, and 4-6% faster; panels of 4 or 16 fall between.
constexpr int kPanel = 8;

template <int M, int DPW, int NW, int CS, int KMAX, int WPE, bool SEG>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void
dedisperse_kernel(const uint8_t *__restrict__ X, int64_t pitch, int64_t nsamp_in,
                  const int2 *__restrict__ P, int pcols, const int32_t *__restrict__ B, int nchan,
                  int ndm, uint32_t *__restrict__ Y, int64_t nout, int lds_pitch, int ntiles,
                  int ndmb, int per_xcd, int vec_store, int seg, int64_t seg_stride, int dmax) {
  extern __shared__ uint4 smem[];  // two slab buffers of CS rows x lds_pitch bytes
  const int blk = blockIdx.x;
  const int logical = (blk & 7) * per_xcd + (blk >> 3);
  if (logical >= ntiles * ndmb) return;
  // panels of kPanel DM blocks: DM block fastest inside a panel, then the
  // time tile, then the next panel
  const int panel = logical / (ntiles * kPanel);
  const int pd = min(kPanel, ndmb - panel * kPanel);
  const int rem = logical - panel * (ntiles * kPanel);
  const int tile = rem / pd;
  const int dblk = panel * kPanel + rem % pd;
  const int64_t t0 = (int64_t)tile * (256 * M);
  // every staged row starts at or below t0 + dmax and spans lds_pitch bytes
  if (nchan % CS == 0 && t0 + dmax + lds_pitch <= nsamp_in)
    dedisperse_block<M, DPW, NW, CS, KMAX, SEG, true>(X, pitch, nsamp_in, P, pcols, B, nchan, ndm,
                                                      Y, nout, lds_pitch, vec_store, t0, dblk,
                                                      smem, seg, seg_stride);
  else
    dedisperse_block<M, DPW, NW, CS, KMAX, SEG, false>(X, pitch, nsamp_in, P, pcols, B, nchan,
                                                       ndm, Y, nout, lds_pitch, vec_store, t0,
                                                       dblk, smem, seg, seg_stride);
}

// Many filterbanks that share a plan (beams of one receiver, chunks of
// different lengths): the work items (beam, time tile, DM block) form one
// flat range, DM block fastest, and each workgroup takes one item.  The item
// numbering gives each XCD a contiguous share, so the workgroups resident on
// an XCD cover neighbouring time tiles of all DM blocks of a beam.  One item
// per workgroup (rather than a persistent loop over items) keeps no state
// across items, so the tilings fit their register budget as in the
// single-filterbank kernel.
template <int M, int DPW, int NW, int CS, int KMAX, int WPE>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE))) void
dedisperse_batch_kernel(const BeamWork *__restrict__ beams, int nbeams, int64_t total_items,
                        int64_t per_xcd, const int2 *__restrict__ P, int pcols,
                        const int32_t *__restrict__ B, int nchan, int ndm, int lds_pitch,
                        int ndmb, int dmax) {
  extern __shared__ uint4 smem[];
  const int64_t item = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (item >= total_items) return;
  const BeamWork &bw = beams[find_beam<&BeamWork::dd_begin>(beams, nbeams, item)];
  const int64_t local = item - bw.dd_begin;
  const int dblk = (int)(local % ndmb);
  const int64_t tile = local / ndmb;
  const int64_t t0 = tile * (256 * M);
  if (nchan % CS == 0 && t0 + dmax + lds_pitch <= bw.nsamp_in)
    dedisperse_block<M, DPW, NW, CS, KMAX, false, true>(bw.X, bw.pitch, bw.nsamp_in, P, pcols, B,
                                                        nchan, ndm, bw.Y, bw.nout, lds_pitch,
                                                        bw.vec_store, t0, dblk, smem);
  else
    dedisperse_block<M, DPW, NW, CS, KMAX, false, false>(bw.X, bw.pitch, bw.nsamp_in, P, pcols,
                                                         B, nchan, ndm, bw.Y, bw.nout, lds_pitch,
                                                         bw.vec_store, t0, dblk, smem);
}

// Staged form of the delay table for blocks of nd trials, slabs of cs rows
// and rows of row_dw dwords (see StagedDelays).  One thread per (trial,
// column); columns past the last channel (up to pcols, a multiple of cs)
// point at the start of their zeroed slab row.  Delays are non-decreasing in
// the trial, so a trial's offset from its block's first staged sample is
// >= 0.
__global__ __launch_bounds__(256) void stage_delays_kernel(const int32_t *__restrict__ D,
                                                           int nchan, int ndm, int pcols, int nd,
                                                           int cs, int row_dw,
                                                           int2 *__restrict__ P,
                                                           int32_t *__restrict__ B) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)ndm * pcols) return;
  const int d = (int)(i / pcols);
  const int c = (int)(i - (int64_t)d * pcols);
  if (c >= nchan) {
    P[i] = make_int2((c % cs) * row_dw, 0x0C020C00);
    return;
  }
  const int dlo = d - d % nd;
  const int32_t base = D[(int64_t)dlo * nchan + c] & ~15;
  const int32_t v = D[(int64_t)d * nchan + c];
  P[i] = make_int2((c % cs) * row_dw + ((v - base) >> 2),
                   (int32_t)(0x0C020C00u + (uint32_t)(v & 3) * 0x00010001u));
  if (d == dlo) B[(int64_t)(d / nd) * nchan + c] = base;
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

template <int M, int DPW, int NW, int CS, int KMAX, int WPE, bool SEG>
hipError_t launch_cfg(int lds_pitch, const uint8_t *X, int64_t pitch, int64_t nsamp_in,
                      const StagedDelays &sd, int nchan, int ndm, uint32_t *Y, int64_t nout,
                      hipStream_t stream, int seg, int64_t seg_stride) {
  constexpr int NT = 256 * M;
  constexpr int ND = NW * DPW;
  if (lds_pitch > 16 * 64 * KMAX || lds_pitch % 16 != 0) return hipErrorInvalidValue;
  if (SEG != (seg > 0) || (SEG && (seg % CS != 0 || nchan % seg != 0)))
    return hipErrorInvalidValue;
  const int64_t ntiles64 = (nout + NT - 1) / NT;
  const int ndmb = (ndm + ND - 1) / ND;
  const int64_t total = ntiles64 * ndmb;
  if (total > (int64_t)0x7FFFFFFF - 8) return hipErrorInvalidValue;
  const int per_xcd = (int)((total + 7) / 8);
  const int grid = per_xcd * 8;
  const size_t lds = 2 * (size_t)CS * (size_t)lds_pitch;
  const int vec_store = (nout % 4 == 0) && ((reinterpret_cast<uintptr_t>(Y) & 15) == 0) &&
                        (seg == 0 || seg_stride % 4 == 0);
  auto kern = dedisperse_kernel<M, DPW, NW, CS, KMAX, WPE, SEG>;
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), lds, stream, X, pitch, nsamp_in, sd.P,
                     sd.pcols, sd.B, nchan, ndm, Y, nout, lds_pitch, (int)ntiles64, ndmb, per_xcd,
                     vec_store, seg, seg_stride, sd.dmax);
  return hipGetLastError();
}

template <int M, int DPW, int NW, int CS, int KMAX, int WPE>
hipError_t launch_batch_cfg(int lds_pitch, const BeamWork *beams, int nbeams, int64_t total,
                            const StagedDelays &sd, int nchan, int ndm, int grid,
                            hipStream_t stream) {
  constexpr int ND = NW * DPW;
  // one workgroup per item: grid = 8 ceil(total / 8)
  if (lds_pitch > 16 * 64 * KMAX || lds_pitch % 16 != 0 || grid % 8 != 0 ||
      (int64_t)grid < total)
    return hipErrorInvalidValue;
  const int ndmb = (ndm + ND - 1) / ND;
  const size_t lds = 2 * (size_t)CS * (size_t)lds_pitch;
  auto kern = dedisperse_batch_kernel<M, DPW, NW, CS, KMAX, WPE>;
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), lds, stream, beams, nbeams, total,
                     (int64_t)(grid / 8), sd.P, sd.pcols, sd.B, nchan, ndm, lds_pitch, ndmb,
                     sd.dmax);
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

// Compiled tilings: (m, dpw, nw, cs, kmax, waves per EU).  kmax bounds the
// staged row length (lds_pitch <= 1024 kmax bytes).
#define SPS_DEDISP_CONFIGS(X) \
  X(5, 1, 16, 16, 2, 8)       \
  X(5, 1, 16, 16, 2, 4)       \
  X(5, 1, 16, 16, 4, 4)       \
  X(3, 1, 16, 16, 2, 8)       \
  X(7, 1, 16, 16, 3, 4)       \
  X(5, 1, 8, 8, 5, 4)         \
  X(5, 1, 8, 8, 8, 4)

bool dedisp_config_supported(const DedispConfig &c) {
#define SPS_MATCH(m_, dpw_, nw_, cs_, kmax_, wpe_)                                      \
  if (c.m == m_ && c.dpw == dpw_ && c.nw == nw_ && c.cs == cs_ && c.kmax == kmax_ && \
      c.wpe == wpe_)                                                                  \
    return true;
  SPS_DEDISP_CONFIGS(SPS_MATCH)
#undef SPS_MATCH
  return false;
}

int64_t dedisp_batch_items(const DedispConfig &c, int ndm, int64_t nout) {
  const int64_t nt = 256 * c.m, nd = c.nw * c.dpw;
  return ((nout + nt - 1) / nt) * ((ndm + nd - 1) / nd);
}

hipError_t launch_dedisperse_batch(const DedispConfig &c, int lds_pitch, const BeamWork *beams,
                                   int nbeams, int64_t total_items, const StagedDelays &sd,
                                   int nchan, int ndm, int grid, hipStream_t stream) {
  if (!sd.matches(c, lds_pitch, nchan, ndm)) return hipErrorInvalidValue;
#define SPS_BLAUNCH(m_, dpw_, nw_, cs_, kmax_, wpe_)                                          \
  if (c.m == m_ && c.dpw == dpw_ && c.nw == nw_ && c.cs == cs_ && c.kmax == kmax_ &&         \
      c.wpe == wpe_)                                                                          \
    return launch_batch_cfg<m_, dpw_, nw_, cs_, kmax_, wpe_>(lds_pitch, beams, nbeams,        \
                                                             total_items, sd, nchan, ndm, grid, \
                                                             stream);
  SPS_DEDISP_CONFIGS(SPS_BLAUNCH)
#undef SPS_BLAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_dedisperse(const DedispConfig &c, int lds_pitch, const uint8_t *X,
                             int64_t pitch, int64_t nsamp_in, const int32_t *D,
                             const StagedDelays *sd, int nchan, int ndm, uint32_t *Y,
                             int64_t nout, hipStream_t stream, int seg, int64_t seg_stride) {
  if (c.m == 0) {
    if (seg != 0) return hipErrorInvalidValue;
    const int64_t nthreads = (nout + 3) / 4;
    const int64_t gx = (nthreads + 255) / 256;
    if (gx > 0x7FFFFFFF) return hipErrorInvalidValue;
    const int gy = ndm < 65535 ? ndm : 65535;
    hipLaunchKernelGGL(dedisperse_direct_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0,
                       stream, X, pitch, nsamp_in, D, nchan, ndm, Y, nout);
    return hipGetLastError();
  }
  if (!sd || !sd->matches(c, lds_pitch, nchan, ndm)) return hipErrorInvalidValue;
#define SPS_LAUNCH(m_, dpw_, nw_, cs_, kmax_, wpe_)                                      \
  if (c.m == m_ && c.dpw == dpw_ && c.nw == nw_ && c.cs == cs_ && c.kmax == kmax_ &&     \
      c.wpe == wpe_)                                                                      \
    return seg > 0 ? launch_cfg<m_, dpw_, nw_, cs_, kmax_, wpe_, true>(                  \
                         lds_pitch, X, pitch, nsamp_in, *sd, nchan, ndm, Y, nout, stream, seg, \
                         seg_stride)                                                         \
                   : launch_cfg<m_, dpw_, nw_, cs_, kmax_, wpe_, false>(                     \
                         lds_pitch, X, pitch, nsamp_in, *sd, nchan, ndm, Y, nout, stream, 0, 0);
  SPS_DEDISP_CONFIGS(SPS_LAUNCH)
#undef SPS_LAUNCH
  return hipErrorInvalidValue;
}

void free_staged(StagedDelays &sd) {
  if (sd.P) (void)hipFree(sd.P);
  if (sd.B) (void)hipFree(sd.B);
  sd = StagedDelays{};
}

hipError_t stage_delays(StagedDelays &sd, const DedispConfig &c, int lds_pitch, const int32_t *D,
                        int nchan, int ndm, int32_t dmax) {
  if (c.m == 0) {
    free_staged(sd);
    return hipSuccess;
  }
  if (sd.matches(c, lds_pitch, nchan, ndm) && sd.dmax == dmax) return hipSuccess;
  if (nchan < 1 || ndm < 1 || lds_pitch % 16 != 0 || c.nd() < 1 || c.cs < 1)
    return hipErrorInvalidValue;
  const int pcols = (nchan + c.cs - 1) / c.cs * c.cs;
  const int64_t n = (int64_t)ndm * pcols;
  const int64_t nb = (int64_t)((ndm + c.nd() - 1) / c.nd()) * nchan;
  if ((n + 255) / 256 > 0x7FFFFFFF) return hipErrorInvalidValue;
  free_staged(sd);
  hipError_t e = hipMalloc(&sd.P, sizeof(int2) * (size_t)n);
  if (e == hipSuccess) e = hipMalloc(&sd.B, sizeof(int32_t) * (size_t)nb);
  if (e != hipSuccess) {
    free_staged(sd);
    return e;
  }
  // null stream, waited for: callers may launch on any stream afterwards
  hipLaunchKernelGGL(stage_delays_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nullptr,
                     D, nchan, ndm, pcols, c.nd(), c.cs, lds_pitch / 4, sd.P, sd.B);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    free_staged(sd);
    return e;
  }
  sd.nchan = nchan;
  sd.dmax = dmax;
  sd.pcols = pcols;
  sd.ndm = ndm;
  sd.nd = c.nd();
  sd.cs = c.cs;
  sd.pitch = lds_pitch;
  return hipSuccess;
}

}  // namespace sps

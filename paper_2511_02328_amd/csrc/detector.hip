// detector.hip -- the learned candidate detector: a small convolutional
// network on max-pooled S/N tiles, trained and run with BF16 matrix-core
// (MFMA) products accumulating in FP32.
//
// Tiles: the boxcar S/N plane max-pooled over 2 trials x 8 samples, scaled
// and rounded to bfloat16 (nearest, ties to even), 256 x 512 per tile.
// Network: six 3x3 convolutions (zero padding 1; strides 2,2,2,2,2,1;
// channels 1->16->32->64->128->128->128), each with bias and ReLU, and a
// 1x1 head giving, per cell of the final 8 x 16 grid, an objectness logit and
// the pulse's DM and time offsets inside the cell.  Loss: per cell binary
// cross-entropy of the objectness (positives weighted, 32 by default)
// averaged over the cells, plus the squared offset errors at positive cells
// (weight 1 by default); mean over tiles.
// Optimiser: Adam with bias correction on FP32 master weights.
//
// Precision: 3x3 weights are used as bfloat16, activations are stored as
// bfloat16 after ReLU, the back-propagated signal is stored as bfloat16 at
// the output of every 3x3 layer (masked by the stored activation, a > 0);
// every product sums in FP32.  The head, loss, gradients of the head and
// Adam run in FP32.
//
// Layout on the device: activations NHWC ([tile][y][x][channel]) so that
// 8 consecutive channels are one 16-byte load; weights packed twice in
// bfloat16, [cout][tap * cin + ci] for the forward product and
// [ci][tap * cout + co] for the backward data product.
//
// MFMA v_mfma_f32_16x16x32_bf16 on a 64-lane wave: lane l supplies row l%16
// of A and column l%16 of B with the 8 K-values 8*(l/16) .. +7 (the same K
// order on both sides, so any internal K order of the unit gives the same
// sum), and receives D rows 4*(l/16) .. +3 of column l%16.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <type_traits>
#include <vector>

#include "sps.h"
#include "sps_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kTileDm = 256, kTileT = 512, kPoolDm = 2, kPoolT = 8;
constexpr int kGridDm = 8, kGridT = 16, kCells = kGridDm * kGridT, kHead = 3;
constexpr float kPosWeight = 32.0f, kLambdaBox = 1.0f;  // default loss weights
constexpr int kNumLayers = 6;

struct Layer {
  int cin, cout, stride, hin, win, hout, wout;
  constexpr int kpad() const { return (9 * cin + 31) / 32 * 32; }
  constexpr int64_t wcount() const { return (int64_t)cout * cin * 9; }
};
constexpr Layer kLayers[kNumLayers] = {
    {1, 16, 2, 256, 512, 128, 256},  {16, 32, 2, 128, 256, 64, 128},
    {32, 64, 2, 64, 128, 32, 64},    {64, 128, 2, 32, 64, 16, 32},
    {128, 128, 2, 16, 32, 8, 16},    {128, 128, 1, 8, 16, 8, 16}};
constexpr int kFeat = 128;  // channels of the last 3x3 layer

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ bool bf_positive(uint16_t b) { return b != 0 && !(b & 0x8000u); }

typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// bf16(lo) | bf16(hi) << 16, nearest even (one v_cvt_pk_bf16_f32); the same
// values as f2bf for every non-NaN input.
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(floatx2{lo, hi}, bf16x2));
}

__device__ __forceinline__ floatx4 mfma(u32x4 a, u32x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Tiles
// ---------------------------------------------------------------------------

// out[i][j] = bf16(scale * max over the 2 x 8 window at (2i, 8j)).
__global__ __launch_bounds__(256) void pool_tiles_kernel(const float *__restrict__ snr,
                                                         int64_t pitch, int64_t nd, int64_t nt,
                                                         float scale, uint16_t *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= nd * nt) return;
  const int64_t i = idx / nt, j = idx - i * nt;
  float m = -INFINITY;
  for (int a = 0; a < kPoolDm; ++a) {
    const float *row = snr + (i * kPoolDm + a) * pitch + j * kPoolT;
    for (int b = 0; b < kPoolT; ++b) m = fmaxf(m, row[b]);
  }
  out[idx] = f2bf(m * scale);
}

// A whole plane cut into tiles: tile (ti, tj) covers trials
// [512 ti, 512 ti + 512) and samples [4096 tj, 4096 tj + 4096); tiles are
// written back to back in row-major tile order.  Only whole tiles.
__global__ __launch_bounds__(256) void pool_tile_grid_kernel(const float *__restrict__ snr,
                                                             int64_t pitch, int ncols,
                                                             int64_t ntiles, float scale,
                                                             uint16_t *__restrict__ out) {
  constexpr int64_t kTilePix = (int64_t)kTileDm * kTileT;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= ntiles * kTilePix) return;
  const int64_t tile = idx / kTilePix;
  const int pix = (int)(idx - tile * kTilePix);
  const int i = pix / kTileT, j = pix % kTileT;
  const int64_t ti = tile / ncols, tj = tile - ti * ncols;
  const int64_t r0 = ti * (kTileDm * kPoolDm) + (int64_t)i * kPoolDm;
  const int64_t c0 = tj * (kTileT * kPoolT) + (int64_t)j * kPoolT;
  float m = -INFINITY;
  for (int a = 0; a < kPoolDm; ++a) {
    const float *row = snr + (r0 + a) * pitch + c0;
    for (int b = 0; b < kPoolT; ++b) m = fmaxf(m, row[b]);
  }
  out[idx] = f2bf(m * scale);
}

// Adds to *count the number of cells among n tiles whose objectness logit
// (head channel 0) is at least logit; one atomic per wave.
__global__ __launch_bounds__(256) void count_cells_kernel(const float *__restrict__ head, int32_t n,
                                                          float logit, int32_t *count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool hit = false;
  if (i < (int64_t)n * kCells) {
    const int64_t t = i / kCells;
    const int cell = (int)(i - t * kCells);
    hit = head[t * kHead * kCells + cell] >= logit;
  }
  const unsigned long long b = __ballot(hit);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (int32_t)__popcll(b));
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------

// Forward of layers 1..5 as an implicit GEMM with the input staged in LDS
// (M = COUT, N = output pixels, K = taps x CIN in tap-major order, the
// order of the packed weights).  A workgroup of 4 waves computes a BH x 16
// block (one row of 16 pixels per N block) of one tile for all COUT
// channels.  Its input region ((BH-1)S+3) x (15S+3), zero outside the
// image, is loaded once into LDS as S*S stride-parity planes with CIN+8
// bf16 per pixel: the 16 pixels of a block then read consecutive pixels of
// one plane, 16 bytes each at a stride of CIN+8 bf16.  Waves split the block
// into WM x WN (row blocks x channel blocks).  A lane ends with 4
// consecutive channels of one pixel: bias, ReLU and bfloat16 are one packed
// conversion pair and an 8-byte LDS store, and the block leaves through LDS
// with 16-byte stores.
// FUSE0 (layer 1 only): the staged region is layer 0's output, computed in
// the workgroup from the tile (one 16x16x32 product per 16 pixels, K = the
// 9 taps), so layer 0's activation never leaves the chip; STORE0 also
// writes the block's own layer-0 pixels (the training pass needs them).
// The fused kernel is persistent: each workgroup loops over blocks and
// issues the next block's tile loads before working on the current one.
// Weight fragments the forward kernel keeps in flight per wave (K steps
// ahead = this / fragments per step).
constexpr int kFwdPrefetch = 16;

template <int LI, int BH, int BW>
struct FwdGeom {
  static constexpr Layer L = kLayers[LI];
  static constexpr int CIN = L.cin, COUT = L.cout, S = L.stride;
  static constexpr int KPAD = (9 * CIN + 31) / 32 * 32;
  static constexpr int IH = (BH - 1) * S + 3, IW = (BW - 1) * S + 3;
  static constexpr int PH = (IH + S - 1) / S, PW = (IW + S - 1) / S;
  static constexpr int CP = CIN + 8;
  static constexpr int PLANE = PH * PW * CP;
  static constexpr int HALO = S * S * PLANE;
  static constexpr int OUTP = COUT + 8;
  static constexpr int OUT = BH * BW * OUTP;
  // Tile region of a fused layer 0: TH x TW values, staged from an even
  // column as pairs (dwords), TP of them holding data per row.  Layer 0
  // reads a pixel's taps as rows of dword pairs with JB blocks of 16 lanes
  // per region row, so staged rows are TPP dwords long and one zero row
  // follows the region: every read stays inside the staged tile.
  static constexpr int TH = 2 * IH + 1, TW = 2 * IW + 1;
  static constexpr int TP = (TW + 2) / 2, JB = (IW + 15) / 16;
  static constexpr int TPP = TP > 16 * JB + 2 ? TP : 16 * JB + 2;
  static constexpr int TROWS = TH + 1;
  static constexpr int TILE = 2 * TROWS * TPP;  // bf16
  // LDS (bf16 elements): the halo, or with FUSE0 the halo and the tile
  // region; the output staging reuses the same space
  static constexpr int lds(bool fuse0) {
    const int a = HALO + (fuse0 ? TILE : 0);
    return a > OUT ? a : OUT;
  }
  // LDS offset (bf16) of staged input pixel (hy, hx) of the region
  __device__ static constexpr int at(int hy, int hx) {
    return ((hy % S) * S + (hx % S)) * PLANE + ((hy / S) * PW + hx / S) * CP;
  }
};

template <int LI, int BH, int BW, int WM, int WN, bool FUSE0, bool STORE0>
__global__ __launch_bounds__(256) void conv_fwd_lds_kernel(
    const uint16_t *__restrict__ x, const uint16_t *__restrict__ wp,
    const float *__restrict__ bias, uint16_t *__restrict__ y, const float *__restrict__ w0f,
    const float *__restrict__ b0, uint16_t *__restrict__ y0, int n) {
  using G = FwdGeom<LI, BH, BW>;
  constexpr Layer L = G::L;
  constexpr Layer L0 = kLayers[0];
  constexpr int CIN = G::CIN, COUT = G::COUT, S = G::S, KPAD = G::KPAD;
  constexpr int IH = G::IH, IW = G::IW;
  constexpr int MBLK = BH * BW / 16, NBLK = COUT / 16;
  constexpr int MB = MBLK / WM, NB = NBLK / WN;
  static_assert(WM * WN == 4 && MBLK % WM == 0 && NBLK % WN == 0, "four waves, even split");
  static_assert(BW == 16 && L.hout % BH == 0 && L.wout % BW == 0, "whole blocks, 16 wide");
  static_assert(!FUSE0 || LI == 1, "layer 0 fuses into layer 1 only");
  extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
  constexpr int BX = L.wout / BW, BPT = (L.hout / BH) * BX;  // blocks per tile
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, px = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int total = n * BPT;

  // ---- staging: the next block's loads go to registers while the current
  // block is computed; every load is issued (outside pixels read a pixel of
  // the tile and are zeroed), so none waits behind a branch ----
  // fused layer 0: tile pixels (2 (iy0 + hy) + ky - 1, 2 (ix0 + hx) + kx - 1),
  // staged from column 2 ix0 - 2 (even) as pairs: a pair is wholly inside or
  // wholly outside the tile, whose width is even
  constexpr int TP = G::TP, TPP = G::TPP;
  constexpr int NSV = FUSE0 ? G::TROWS * TPP : IH * IW * (CIN / 8);  // staged items
  constexpr int PER = (NSV + 255) / 256;
  using Item = typename std::conditional<FUSE0, uint32_t, u32x4>::type;
  Item sv[PER];
  auto stage_load = [&](int blk) {
    const int64_t tile = blk / BPT;
    const int bi = blk - (int)tile * BPT;
    const int iy0 = (bi / BX) * BH * S - 1, ix0 = (bi % BX) * BW * S - 1;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int i = threadIdx.x + 256 * r;
      if constexpr (FUSE0) {
        const int row = i / TPP, pc = i - row * TPP;
        const int ty = 2 * iy0 - 1 + row, tx = 2 * ix0 - 2 + 2 * pc;
        const bool in = i < NSV && row < G::TH && pc < TP && ty >= 0 && ty < L0.hin && tx >= 0 &&
                        tx < L0.win;
        const int64_t o = in ? (tile * L0.hin + ty) * L0.win + tx : tile * L0.hin * L0.win;
        sv[r] = *reinterpret_cast<const uint32_t *>(x + o);
        if (!in) sv[r] = 0u;
      } else {
        constexpr int V = CIN / 8;  // 16-byte vectors per pixel
        const int pix = i / V, v = i - pix * V;
        const int hy = pix / IW, hx = pix - hy * IW;
        const int yy = iy0 + hy, xx = ix0 + hx;
        const bool in = i < NSV && yy >= 0 && yy < L.hin && xx >= 0 && xx < L.win;
        const int64_t o = in ? ((tile * L.hin + yy) * L.win + xx) * CIN + 8 * v
                             : tile * L.hin * L.win * CIN;
        sv[r] = *reinterpret_cast<const u32x4 *>(x + o);
        if (!in) sv[r] = u32x4{0u, 0u, 0u, 0u};
      }
    }
  };
  auto stage_store = [&]() {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int i = threadIdx.x + 256 * r;
      if (i < NSV) {
        if constexpr (FUSE0) {
          reinterpret_cast<uint32_t *>(lds + G::HALO)[i] = sv[r];
        } else {
          constexpr int V = CIN / 8;
          const int pix = i / V, v = i - pix * V;
          const int hy = pix / IW, hx = pix - hy * IW;
          *reinterpret_cast<u32x4 *>(lds + G::at(hy, hx) + 8 * v) = sv[r];
        }
      }
    }
  };

  // ---- fused layer 0 constants: per 16 region pixels one 16x16x32 product
  // with M = the 16 channels, N = the pixels, K = (tap row ky, staged column
  // c) as 4 ky + c for ky < 3, c < 4, where staged columns 2 hx .. 2 hx + 3
  // of a pixel are its taps kx = c - 1 (c = 0 has weight 0), so a pixel's K
  // values are two aligned dword pairs of the staged tile ----
  u32x4 wa = {0u, 0u, 0u, 0u};  // A: row px = channel, K values 8g .. 8g + 7
  float bch[4] = {0.f, 0.f, 0.f, 0.f};
  if constexpr (FUSE0) {
    float wvv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * g + j, ky = k >> 2, c = k & 3;
      const bool use = ky < 3 && c > 0;
      wvv[j] = w0f[px * 9 + (use ? ky * 3 + c - 1 : 0)];
      if (!use) wvv[j] = 0.0f;
    }
    uint32_t h[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) h[j] = (uint32_t)f2bf(wvv[j]);
    wa = u32x4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
#pragma unroll
    for (int j = 0; j < 4; ++j) bch[j] = b0[4 * g + j];
  }

  // ---- main product constants: M = output channels (weights), N = pixels,
  // so that a lane ends with 4 consecutive channels of one pixel ----
  const int wm = wave / WN, wn = wave % WN;
  const uint16_t *wrow = wp + (int64_t)(wn * NB * 16 + px) * KPAD + 8 * g;
  const uint16_t *abase = lds + G::at(S * (wm * MB), S * px) + 8 * g;
  constexpr int ROWSTEP = G::PW * G::CP;  // next output row: one plane row further
  auto tap_off = [](int t) {
    const int ky = t / 3, kx = t % 3;
    return ((ky % S) * S + (kx % S)) * G::PLANE + ((ky / S) * G::PW + kx / S) * G::CP;
  };
  constexpr int NSTEP = KPAD / 32;
  constexpr int PFW = kFwdPrefetch / NB > 1 ? kFwdPrefetch / NB : 1;
  constexpr int PF = NSTEP < PFW ? NSTEP : PFW;
  auto load_a = [&](int st, u32x4 (&a)[MB]) {
    const int k0 = 32 * st;
    int off;
    bool live = true;
    if constexpr (CIN >= 32) {
      off = tap_off(k0 / CIN) + k0 % CIN;  // one tap for the whole step
    } else {
      // CIN == 16: lanes g < 2 take tap k0 / 16, lanes g >= 2 the next one
      const int t0 = k0 / CIN, t1 = t0 + 1;
      live = g < 2 || t1 < 9;
      off = g < 2 ? tap_off(t0) : (t1 < 9 ? tap_off(t1) : 0) - 16;
    }
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      a[i] = *reinterpret_cast<const u32x4 *>(abase + off + i * ROWSTEP);
      if constexpr (CIN < 32) {
        if (!live) a[i] = u32x4{0u, 0u, 0u, 0u};
      }
    }
  };

  // one block: stage it (its loads were issued before), compute, write
  auto process = [&](int blk) {
    const int64_t tile = blk / BPT;
    const int bi = blk - (int)tile * BPT;
    const int oy0 = (bi / BX) * BH, ox0 = (bi % BX) * BW;
    const int iy0 = oy0 * S - 1, ix0 = ox0 * S - 1;  // input pixel of region (0, 0)
    stage_store();
    __syncthreads();
    // persistent (fused layer 0, whose staging is a few registers): the
    // next block's loads are in flight meanwhile
    if constexpr (FUSE0)
      if (blk + (int)gridDim.x < total) stage_load(blk + gridDim.x);

    if constexpr (FUSE0) {
      // Layer 0 on the matrix cores.  Region rows are dealt to the waves
      // (row hy is wave-uniform); a row's IW pixels are JB blocks of 16
      // lanes, the lanes past IW idle.  K positions without a tap (groups
      // 2, 3 and the upper half of group 1) meet zero weights; the values
      // read there are staged tile values (finite), so they add exact
      // zeros.  Lanes past the row read inside the staged row (TPP >= 16 JB
      // + 2 dwords) and their columns are not stored; group 1's second row,
      // 2 hy + 3, is at most the zero row.  Pixels outside layer 0's output
      // (the next layer's zero padding) are stored as zeros.
      constexpr int JB = G::JB;
      const uint32_t *t32 =
          reinterpret_cast<const uint32_t *>(lds + G::HALO) + 2 * (g & 1) * TPP + px;
      uint16_t *dcol = lds + (px & 1) * G::PLANE + (px >> 1) * G::CP + 4 * g;
      bool xin[JB], lane_on[JB];
#pragma unroll
      for (int j = 0; j < JB; ++j) {
        const int hx = 16 * j + px, xx = ix0 + hx;
        lane_on[j] = hx < IW;
        xin[j] = hx < IW && xx >= 0 && xx < L0.wout;
      }
      for (int hy = wv; hy < IH; hy += 4) {
        const int yy = iy0 + hy;
        const bool row_in = yy >= 0 && yy < L0.hout;
        const uint32_t *rrow = t32 + 2 * hy * TPP;  // staged rows 2 hy + 2 (g & 1), + 1
        u32x4 tb[JB];
#pragma unroll
        for (int j = 0; j < JB; ++j)
          tb[j] = u32x4{rrow[16 * j], rrow[16 * j + 1], rrow[TPP + 16 * j], rrow[TPP + 16 * j + 1]};
        floatx4 dl[JB];  // every product first, then the stores
#pragma unroll
        for (int j = 0; j < JB; ++j) dl[j] = mfma(wa, tb[j], floatx4{0.f, 0.f, 0.f, 0.f});
        uint16_t *drow = dcol + (hy & 1) * S * G::PLANE + (hy >> 1) * G::PW * G::CP;
#pragma unroll
        for (int j = 0; j < JB; ++j) {
          if (lane_on[j]) {
            const floatx4 d = dl[j];
            uint32_t pk[2] = {0u, 0u};
            if (row_in && xin[j]) {
              pk[0] = f2bf2(fmaxf(d[0] + bch[0], 0.0f), fmaxf(d[1] + bch[1], 0.0f));
              pk[1] = f2bf2(fmaxf(d[2] + bch[2], 0.0f), fmaxf(d[3] + bch[3], 0.0f));
            }
            uint32_t *dst = reinterpret_cast<uint32_t *>(drow + 8 * j * G::CP);
            dst[0] = pk[0];
            dst[1] = pk[1];
          }
        }
      }
      __syncthreads();
      if constexpr (STORE0) {
        // the block's own layer-0 pixels (the region without its first row
        // and column), copied out of the staged region with 16-byte stores
        constexpr int OWN = (IH - 1) * (IW - 1);
        for (int i = threadIdx.x; i < OWN * 2; i += 256) {
          const int pix = i >> 1, half = i & 1;
          const int hy = 1 + pix / (IW - 1), hx = 1 + pix % (IW - 1);
          const int yy = iy0 + hy, xx = ix0 + hx;
          if (yy < L0.hout && xx < L0.wout)
            reinterpret_cast<u32x4 *>(y0 + ((tile * L0.hout + yy) * L0.wout + xx) * 16)[half] =
                reinterpret_cast<const u32x4 *>(lds + G::at(hy, hx))[half];
        }
      }
    }

    // ---- the main product, fully unrolled (tap and channel of every K step
    // are constants; LDS reads take immediate offsets from one base per
    // lane), as a software pipeline pinned with scheduling barriers (left
    // alone, the compiler moves each load next to its use): weight fragments
    // PF K steps ahead in a ring of registers, A fragments one step ahead ----
    floatx4 acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[i][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    u32x4 ring[PF][NB];
#pragma unroll
    for (int u = 0; u < PF; ++u)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        ring[u][b] = *reinterpret_cast<const u32x4 *>(wrow + (int64_t)b * 16 * KPAD + 32 * u);
    u32x4 acur[MB];
    load_a(0, acur);
#pragma unroll
    for (int st = 0; st < NSTEP; ++st) {
      u32x4 bv[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = ring[st % PF][b];
      if (st + PF < NSTEP) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
          ring[st % PF][b] =
              *reinterpret_cast<const u32x4 *>(wrow + (int64_t)b * 16 * KPAD + 32 * (st + PF));
      }
      u32x4 anext[MB];
      if (st + 1 < NSTEP) load_a(st + 1, anext);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[i][b] = mfma(bv[b], acur[i], acc[i][b]);
      __builtin_amdgcn_sched_barrier(0);
      if (st + 1 < NSTEP) {
#pragma unroll
        for (int i = 0; i < MB; ++i) acur[i] = anext[i];
      }
    }

    // ---- bias, ReLU, bf16 (8 bytes per lane and block pair); staged in
    // LDS, written with 16-byte stores ----
    __syncthreads();  // every wave is done with the staged input
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int co = (wn * NB + b) * 16 + 4 * g;  // channels co .. co + 3
      const float b0v = bias[co], b1v = bias[co + 1], b2v = bias[co + 2], b3v = bias[co + 3];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        const int m = (wm * MB + i) * 16 + px;  // pixel of the block (row-major)
        const floatx4 a = acc[i][b];
        uint32_t *dst = reinterpret_cast<uint32_t *>(lds + m * G::OUTP + co);
        dst[0] = f2bf2(fmaxf(a[0] + b0v, 0.0f), fmaxf(a[1] + b1v, 0.0f));
        dst[1] = f2bf2(fmaxf(a[2] + b2v, 0.0f), fmaxf(a[3] + b3v, 0.0f));
      }
    }
    __syncthreads();
    constexpr int V = COUT / 8;
    for (int i = threadIdx.x; i < BH * BW * V; i += 256) {
      const int m = i / V, v = i % V;
      const int oy = oy0 + m / BW, ox = ox0 + m % BW;
      *reinterpret_cast<u32x4 *>(y + ((tile * L.hout + oy) * L.wout + ox) * COUT + 8 * v) =
          *reinterpret_cast<const u32x4 *>(lds + m * G::OUTP + 8 * v);
    }
    __syncthreads();  // the staging of the next block overwrites this space
  };

  if constexpr (FUSE0) {
    for (int blk = blockIdx.x; blk < total; blk += gridDim.x) {
      if (blk == (int)blockIdx.x) stage_load(blk);
      process(blk);
    }
  } else {
    if ((int)blockIdx.x < total) {
      stage_load(blockIdx.x);
      process(blockIdx.x);
    }
  }
}

// Blocks and wave splits of the LDS-staged forward, per layer:
// (BH, BW, WM, WN).
#define SPS_FWD_LDS_CONFIGS(X) \
  X(1, 16, 16, 4, 1)           \
  X(2, 8, 16, 4, 1)            \
  X(3, 4, 16, 1, 4)            \
  X(4, 2, 16, 1, 4)            \
  X(5, 4, 16, 1, 4)

// ---------------------------------------------------------------------------
// Head, loss and the signal entering the last 3x3 layer
// ---------------------------------------------------------------------------

// One thread per cell (128 cells per block).  a6: [cells][128] bf16.
// Writes the head outputs, dz6 = bf16((wh^T g) * (a6 > 0)), and per block the
// partial sums of the head gradients and of the loss.
__global__ __launch_bounds__(128) void head_loss_kernel(
    const uint16_t *__restrict__ a6, const float *__restrict__ wh, const float *__restrict__ bh,
    const float *__restrict__ labels, int64_t ncell, float inv_n, float *__restrict__ head,
    uint16_t *__restrict__ dz6, float *__restrict__ part_wh, float *__restrict__ part_bh,
    float *__restrict__ part_loss, int train, float pos_weight, float lambda_box) {
  __shared__ float w_s[kHead][kFeat];
  __shared__ float g_s[128][kHead];
  __shared__ uint16_t a_s[128][kFeat + 2];
  __shared__ float l_s[128];
  for (int i = threadIdx.x; i < kHead * kFeat; i += 128) w_s[i / kFeat][i % kFeat] = wh[i];
  const int64_t cell = (int64_t)blockIdx.x * 128 + threadIdx.x;
  const bool valid = cell < ncell;
  // stage this block's activations (coalesced: 16 bytes per thread per step)
  for (int v = threadIdx.x; v < 128 * kFeat / 8; v += 128) {
    const int c = v / (kFeat / 8), f8 = (v % (kFeat / 8)) * 8;
    const int64_t q = (int64_t)blockIdx.x * 128 + c;
    u32x4 d = {0u, 0u, 0u, 0u};
    if (q < ncell) d = *reinterpret_cast<const u32x4 *>(a6 + q * kFeat + f8);
    const uint16_t *h = reinterpret_cast<const uint16_t *>(&d);
#pragma unroll
    for (int i = 0; i < 8; ++i) a_s[c][f8 + i] = h[i];
  }
  __syncthreads();
  float h[kHead] = {bh[0], bh[1], bh[2]};
  for (int c = 0; c < kFeat; ++c) {
    const float a = bf2f(a_s[threadIdx.x][c]);
#pragma unroll
    for (int k = 0; k < kHead; ++k) h[k] += w_s[k][c] * a;
  }
  const int64_t tile = cell / kCells;
  const int64_t cidx = cell - tile * kCells;
  float gk[kHead] = {0.f, 0.f, 0.f};
  float lc = 0.f;
  if (valid) {
    if (head)
      for (int k = 0; k < kHead; ++k) head[(tile * kHead + k) * kCells + cidx] = h[k];
    if (train) {
      const float y0 = labels[(tile * kHead + 0) * kCells + cidx];
      const float y1 = labels[(tile * kHead + 1) * kCells + cidx];
      const float y2 = labels[(tile * kHead + 2) * kCells + cidx];
      const float o = h[0];
      const float wgt = y0 > 0.f ? pos_weight : 1.0f;
      const float bce = fmaxf(o, 0.f) - y0 * o + log1pf(expf(-fabsf(o)));
      const float e1 = h[1] - y1, e2 = h[2] - y2;
      lc = (wgt * bce / (float)kCells + lambda_box * y0 * (e1 * e1 + e2 * e2)) * inv_n;
      const float sig = 1.0f / (1.0f + expf(-o));
      gk[0] = wgt * (sig - y0) / (float)kCells * inv_n;
      gk[1] = 2.0f * lambda_box * e1 * y0 * inv_n;
      gk[2] = 2.0f * lambda_box * e2 * y0 * inv_n;
    }
  }
  if (!train) return;
  for (int k = 0; k < kHead; ++k) g_s[threadIdx.x][k] = gk[k];
  l_s[threadIdx.x] = lc;
  if (valid) {
    for (int c0 = 0; c0 < kFeat; c0 += 8) {
      uint32_t pk[4];
#pragma unroll
      for (int i = 0; i < 8; i += 2) {
        const int c = c0 + i;
        const float d0 = w_s[0][c] * gk[0] + w_s[1][c] * gk[1] + w_s[2][c] * gk[2];
        const float d1 = w_s[0][c + 1] * gk[0] + w_s[1][c + 1] * gk[1] + w_s[2][c + 1] * gk[2];
        const uint16_t b0 = bf_positive(a_s[threadIdx.x][c]) ? f2bf(d0) : (uint16_t)0;
        const uint16_t b1 = bf_positive(a_s[threadIdx.x][c + 1]) ? f2bf(d1) : (uint16_t)0;
        pk[i / 2] = (uint32_t)b0 | ((uint32_t)b1 << 16);
      }
      *reinterpret_cast<u32x4 *>(dz6 + cell * kFeat + c0) = u32x4{pk[0], pk[1], pk[2], pk[3]};
    }
  }
  __syncthreads();
  // thread c: partial head-weight gradients of feature c over the block's cells
  {
    const int c = threadIdx.x;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (int q = 0; q < 128; ++q) {
      const float a = bf2f(a_s[q][c]);
      s0 += g_s[q][0] * a;
      s1 += g_s[q][1] * a;
      s2 += g_s[q][2] * a;
    }
    part_wh[((int64_t)blockIdx.x * kHead + 0) * kFeat + c] = s0;
    part_wh[((int64_t)blockIdx.x * kHead + 1) * kFeat + c] = s1;
    part_wh[((int64_t)blockIdx.x * kHead + 2) * kFeat + c] = s2;
  }
  if (threadIdx.x < kHead + 1) {
    float s = 0.f;
    for (int q = 0; q < 128; ++q) s += threadIdx.x < kHead ? g_s[q][threadIdx.x] : l_s[q];
    if (threadIdx.x < kHead)
      part_bh[(int64_t)blockIdx.x * kHead + threadIdx.x] = s;
    else
      part_loss[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Backward: data
// ---------------------------------------------------------------------------

typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) i16x4 lds_i16x4;

// Two transposed LDS reads (4 pixels each) as one 8-value MFMA operand;
// p: this lane's address for the first 4 pixels, next: element offset of
// the second 4.
__device__ __forceinline__ u32x4 tr_pair(const uint16_t *p, int next) {
  const i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)p);
  const i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)(p + next));
  u32x4 r;
  r.x = (uint32_t)(uint16_t)lo[0] | ((uint32_t)(uint16_t)lo[1] << 16);
  r.y = (uint32_t)(uint16_t)lo[2] | ((uint32_t)(uint16_t)lo[3] << 16);
  r.z = (uint32_t)(uint16_t)hi[0] | ((uint32_t)(uint16_t)hi[1] << 16);
  r.w = (uint32_t)(uint16_t)hi[2] | ((uint32_t)(uint16_t)hi[3] << 16);
  return r;
}

// Backward data of layers 2..5 as an implicit GEMM with the signal staged
// in LDS: dx[p][ci] = bf16(mask(x[p][ci]) * sum_{tap, co} W[co][ci][tap]
// dz[q(p, tap)][co]).  A workgroup owns RPW x 16 class pixels of each parity
// class (stride 2: input pixels (Y0 + 2 cy + py, X0 + 2 cx + px); stride 1:
// one class, (Y0 + cy, X0 + cx)) and stages the signal region they read,
// zero outside the image.  Each class is a product with M = input channels
// (the transposed weights, [ci][tap * COUT + co], straight from L2), N = 16
// class pixels of a class row, K = the class's taps x COUT.  The 4 waves
// split the M blocks (WMG groups) and the class rows (4 / WMG groups), so a
// weight fragment serves every class row of the wave.  A lane ends with 4
// consecutive channels of one pixel: 8-byte mask loads and signal stores.
// The grid is the resident workgroup count; each workgroup takes blocks
// blockIdx.x, + gridDim.x, ... and loads the next block's signal region
// into registers while it works on the current one.
template <int LI, int WMG, int RPW>
__global__ __launch_bounds__(256) void bwd_data_lds_kernel(const uint16_t *__restrict__ dz,
                                                           const uint16_t *__restrict__ wt,
                                                           const uint16_t *__restrict__ x,
                                                           uint16_t *__restrict__ dx,
                                                           int nblocks) {
  constexpr Layer L = kLayers[LI];
  constexpr int CIN = L.cin, COUT = L.cout, S = L.stride;
  constexpr int WRG = 4 / WMG, CR = WRG * RPW;       // class rows of a block
  constexpr int MBW = CIN / 16 / WMG;                 // M blocks of a wave
  static_assert(CIN % (16 * WMG) == 0 && MBW >= 1, "M blocks split evenly");
  constexpr int BH = S * CR, BW = S * 16;             // input pixels of a block
  static_assert(L.hin % BH == 0 && L.win % BW == 0, "whole blocks");
  constexpr int NBY = L.hin / BH, NBX = L.win / BW;
  // staged signal region: stride 2 rows Y0/2 .. Y0/2 + CR, columns X0/2 ..
  // X0/2 + 16; stride 1 rows Y0 - 1 .. Y0 + CR, columns X0 - 1 .. X0 + 16
  constexpr int ZH = S == 2 ? CR + 1 : CR + 2, ZW = S == 2 ? 17 : 18, ZP = COUT + 8;
  constexpr int K = 9 * COUT;
  __shared__ __attribute__((aligned(16))) uint16_t zs[ZH * ZW * ZP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c16 = lane & 15;
  const int wm = wave % WMG, wr = wave / WMG;
  constexpr int ZCH = ZH * ZW * (COUT / 8), NZ = (ZCH + 255) / 256;
  u32x4 rz[NZ];
  auto origin = [&](int blk, int &nn, int &Y0, int &X0) {
    nn = blk / (NBY * NBX);
    const int rb = blk % (NBY * NBX);
    Y0 = (rb / NBX) * BH;
    X0 = (rb % NBX) * BW;
  };
  auto load = [&](int blk) {
    int nn, Y0, X0;
    origin(blk, nn, Y0, X0);
    const int zy0 = S == 2 ? Y0 / 2 : Y0 - 1, zx0 = S == 2 ? X0 / 2 : X0 - 1;
#pragma unroll
    for (int u = 0; u < NZ; ++u) {
      const int v = threadIdx.x + 256 * u;
      const int pix = v / (COUT / 8), c8 = (v % (COUT / 8)) * 8;
      const int oy = zy0 + pix / ZW, ox = zx0 + pix % ZW;
      rz[u] = u32x4{0u, 0u, 0u, 0u};
      if (v < ZCH && oy >= 0 && oy < L.hout && ox >= 0 && ox < L.wout)
        rz[u] = *reinterpret_cast<const u32x4 *>(dz + ((int64_t)(nn * L.hout + oy) * L.wout + ox) *
                                                          COUT + c8);
    }
  };
  if ((int)blockIdx.x < nblocks) load(blockIdx.x);
  for (int blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
  int nn, Y0, X0;
  origin(blk, nn, Y0, X0);
  __syncthreads();  // the previous block's readers are done
#pragma unroll
  for (int u = 0; u < NZ; ++u) {
    const int v = threadIdx.x + 256 * u;
    if (v < ZCH) *reinterpret_cast<u32x4 *>(&zs[(v / (COUT / 8)) * ZP + (v % (COUT / 8)) * 8]) = rz[u];
  }
  __syncthreads();
  if (blk + (int)gridDim.x < nblocks) load(blk + gridDim.x);
  // A fragments: row ci = (wm * MBW + m) * 16 + c16, K = channels 8g..8g+7
  // of a 32-channel step
  const uint16_t *wrow = wt + (int64_t)(wm * MBW * 16 + c16) * K + 8 * g;
#pragma unroll
  for (int cls = 0; cls < S * S; ++cls) {
    const int py = S == 2 ? cls >> 1 : 0, px = S == 2 ? cls & 1 : 0;
    // masks of the lane's pixels, loaded before the products
    uint2 am[RPW][MBW];
    int64_t o[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int cy = wr * RPW + r;
      const int iy = Y0 + S * cy + py, ix = X0 + S * c16 + px;
      o[r] = (((int64_t)nn * L.hin + iy) * L.win + ix) * CIN + wm * MBW * 16 + 4 * g;
#pragma unroll
      for (int m = 0; m < MBW; ++m) am[r][m] = *reinterpret_cast<const uint2 *>(x + o[r] + 16 * m);
    }
    floatx4 acc[RPW][MBW];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int m = 0; m < MBW; ++m) acc[r][m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      if (S == 2 && ((py + 1 - ky) & 1) != 0) continue;
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        if (S == 2 && ((px + 1 - kx) & 1) != 0) continue;
        const int tap = ky * 3 + kx;
        // staged signal pixel read by class pixel (cy, c16) through the tap
        const int dr = S == 2 ? (py + 1 - ky) / 2 : 2 - ky;
        const int dc = S == 2 ? (px + 1 - kx) / 2 : 2 - kx;
#pragma unroll 2
        for (int ks = 0; ks < COUT / 32; ++ks) {
          u32x4 a[MBW];
#pragma unroll
          for (int m = 0; m < MBW; ++m)
            a[m] = *reinterpret_cast<const u32x4 *>(wrow + (int64_t)m * 16 * K + tap * COUT +
                                                    32 * ks);
#pragma unroll
          for (int r = 0; r < RPW; ++r) {
            const int cy = wr * RPW + r;
            const u32x4 b = *reinterpret_cast<const u32x4 *>(
                &zs[((cy + dr) * ZW + c16 + dc) * ZP + 32 * ks + 8 * g]);
#pragma unroll
            for (int m = 0; m < MBW; ++m) acc[r][m] = mfma(a[m], b, acc[r][m]);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int m = 0; m < MBW; ++m) {
        const uint2 a = am[r][m];
        const uint16_t ah[4] = {(uint16_t)(a.x & 0xFFFFu), (uint16_t)(a.x >> 16),
                                (uint16_t)(a.y & 0xFFFFu), (uint16_t)(a.y >> 16)};
        uint16_t zq[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) zq[j] = bf_positive(ah[j]) ? f2bf(acc[r][m][j]) : (uint16_t)0;
        *reinterpret_cast<uint2 *>(dx + o[r] + 16 * m) =
            make_uint2((uint32_t)zq[0] | ((uint32_t)zq[1] << 16),
                       (uint32_t)zq[2] | ((uint32_t)zq[3] << 16));
      }
    __builtin_amdgcn_sched_barrier(0);
  }
  }
}

// (WMG, RPW) of the backward-data kernel of layers 2..5 (entries 0 and 1
// unused): M-block groups and class rows per wave.
#define SPS_BWD_LDS_CONFIGS X(2, 2, 2) X(3, 4, 4) X(4, 4, 4) X(5, 4, 4)

template <int LI, int WMG, int RPW>
int bwd_data_lds_blocks(int n) {
  constexpr Layer L = kLayers[LI];
  constexpr int CR = (4 / WMG) * RPW;
  return n * (L.hin / (L.stride * CR)) * (L.win / (L.stride * 16));
}

// Workgroups resident at once for a persistent kernel (256 threads, no
// dynamic LDS); 1024 if the query fails.
int resident_workgroups(const void *kern) {
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return e == hipSuccess ? (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1) : 1024;
}

template <int LI, int WMG, int RPW>
int bwd_data_lds_grid(int n) {
  static const int resident =
      resident_workgroups(reinterpret_cast<const void *>(bwd_data_lds_kernel<LI, WMG, RPW>));
  const int blocks = bwd_data_lds_blocks<LI, WMG, RPW>(n);
  return blocks < resident ? blocks : resident;
}

// Layer 1's backward (data, weight and bias products) fused with layer 0's
// weight and bias gradients.  A block is 8 x 32 layer-0 pixels of one tile
// (layer 1's input), owning the 4 x 16 layer-1 output pixels whose
// windows start in it.  Staged in LDS once per block: layer 1's signal over
// (4 + 1) x (16 + 1) pixels, layer 0's stored activation over the block
// with a one-pixel halo (9 x 33 pixels), and the tile region layer 0 read
// for the block (17 x 65 values); the transposed layer-1 weights once per
// workgroup.
//  - Layer 0's signal: each of the four parity classes of the block's
//    pixels is a product with M = 16 channels (the transposed weights),
//    N = 16 class pixels of one class row, K = the class's taps x 32 (one
//    16x16x32 product per tap); a wave takes one class row.  The lane's 4
//    channels of one pixel are masked by the staged activation, rounded to
//    bfloat16, stored if store0 (nothing else reads layer 0's signal), and
//    then, as FP32, multiply the pixel's 9 tile values into the lane's
//    layer-0 weight-gradient sums (and bias sums).
//  - Layer 1's weight gradient: M = 32 output channels, N = 16 input
//    channels per tap, K = the 64 owned output pixels; both operands come
//    from the staged signal and activation through transposed LDS reads,
//    and the waves split the 9 taps.  Its bias gradient sums the owned
//    pixels of the staged signal.
// The grid is the number of workgroups resident at once (at most
// kB01Grid), each taking blocks blockIdx.x, + gridDim.x, ..., and loading
// the next block's staging while it works on the current one; every
// workgroup's partial sums are in a fixed order: partial[wg][0, 4608) layer 1's weights [co][tap][ci], then its 32
// biases, layer 0's weights [co][tap] and its 16 biases.
constexpr int kB01Rows = 4, kB01Cols = 16;  // class rows / columns of a block
constexpr int kB01Grid = 1024;  // at most this many workgroups (partial rows)
constexpr int kB01W1 = 32 * 9 * 16, kB01B1 = kB01W1, kB01W0 = kB01B1 + 32, kB01B0 = kB01W0 + 144;
constexpr int kB01Part = kB01B0 + 16;               // partial sums per workgroup
constexpr int kB01ZW = kB01Cols + 1, kB01ZP = 48;   // staged signal: pixels per row, bf16 per pixel
constexpr int kB01XH = 2 * kB01Rows + 1, kB01XW = 2 * kB01Cols + 1;  // staged activation region
constexpr int kB01TH = 4 * kB01Rows + 1, kB01TW = 4 * kB01Cols + 8;  // staged tile region
constexpr int kB01WP = 9 * 32 + 8;  // staged transposed weights: bf16 per input channel

// Three waves per SIMD: up to 168 registers, which hold the next block's
// staging registers without spills.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void bwd01_kernel(const uint16_t *__restrict__ dz1,
                                                    const uint16_t *__restrict__ wt1,
                                                    const uint16_t *__restrict__ act0,
                                                    const uint16_t *__restrict__ tiles,
                                                    uint16_t *__restrict__ dz0,
                                                    float *__restrict__ partial, int nblocks,
                                                    int store0) {
  constexpr Layer L0 = kLayers[0], L1 = kLayers[1];
  static_assert(L1.cin == 16 && L1.cout == 32 && L1.stride == 2, "layer 1 shape");
  constexpr int BY = L0.hout / (2 * kB01Rows), BX = L0.wout / (2 * kB01Cols);
  static_assert(L0.hout % (2 * kB01Rows) == 0 && L0.wout % (2 * kB01Cols) == 0, "whole blocks");
  __shared__ __attribute__((aligned(16))) uint16_t zs[(kB01Rows + 1) * kB01ZW * kB01ZP];
  __shared__ __attribute__((aligned(16))) uint16_t xs[kB01XH * kB01XW * 16];
  __shared__ __attribute__((aligned(16))) uint16_t ts[kB01TH * kB01TW];
  __shared__ __attribute__((aligned(16))) uint16_t ws[16 * kB01WP];
  __shared__ float red[4][4][40];
  __shared__ float red1[8][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c16 = lane & 15;
  // transposed weights [ci][tap * 32 + co]; a lane's A fragment of a tap is
  // row ci = c16, K = channels 8g .. 8g+7 of layer 1's signal
  for (int v = threadIdx.x; v < 16 * 36; v += 256)
    *reinterpret_cast<u32x4 *>(&ws[(v / 36) * kB01WP + 8 * (v % 36)]) =
        *reinterpret_cast<const u32x4 *>(wt1 + 8 * v);
  float accw[4][9], accb[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    accb[j] = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) accw[j][t] = 0.f;
  }
  // layer 1's weight gradient: wave w takes taps w, w + 4 (and 8 for w = 0)
  floatx4 acc1[3][2];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m) acc1[t][m] = floatx4{0.f, 0.f, 0.f, 0.f};
  float accb1 = 0.f;  // layer 1's bias: channel threadIdx.x % 32
  // A block's staging in registers (this thread's 16-byte chunks of the
  // signal, activation and tile regions); the next block's are loaded while
  // the current one is worked on.
  constexpr int ZCH = (kB01Rows + 1) * kB01ZW * 4, XCH = kB01XH * kB01XW * 2;
  constexpr int TCH = kB01TH * (kB01TW / 8);
  constexpr int NZ = (ZCH + 255) / 256, NX = (XCH + 255) / 256, NT = (TCH + 255) / 256;
  u32x4 rz[NZ], rx[NX], rt[NT];
  auto load = [&](int blk) {
    const int nn = blk / (BY * BX), r = blk % (BY * BX);
    const int Y0 = (r / BX) * 2 * kB01Rows, X0 = (r % BX) * 2 * kB01Cols;
    // layer 1's signal at rows Y0/2 + i (i <= kB01Rows), columns X0/2 + j
    // (j <= kB01Cols), zero outside the image
#pragma unroll
    for (int u = 0; u < NZ; ++u) {
      const int v = threadIdx.x + 256 * u;
      const int pix = v >> 2, q = v & 3;
      const int oy = Y0 / 2 + pix / kB01ZW, ox = X0 / 2 + pix % kB01ZW;
      rz[u] = u32x4{0u, 0u, 0u, 0u};
      if (v < ZCH && oy < L1.hout && ox < L1.wout)
        rz[u] = *reinterpret_cast<const u32x4 *>(
            dz1 + ((int64_t)(nn * L1.hout + oy) * L1.wout + ox) * 32 + 8 * q);
    }
    // layer 0's activation at rows Y0 - 1 + i, columns X0 - 1 + j
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int v = threadIdx.x + 256 * u;
      const int pix = v >> 1, q = v & 1;
      const int iy = Y0 - 1 + pix / kB01XW, ix = X0 - 1 + pix % kB01XW;
      rx[u] = u32x4{0u, 0u, 0u, 0u};
      if (v < XCH && iy >= 0 && iy < L0.hout && ix >= 0 && ix < L0.wout)
        rx[u] = *reinterpret_cast<const u32x4 *>(
            act0 + ((int64_t)(nn * L0.hout + iy) * L0.wout + ix) * 16 + 8 * q);
    }
    // tile rows 2 Y0 - 1 + i, columns from 2 X0 - 8 (16-byte chunks)
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int v = threadIdx.x + 256 * u;
      const int i = v / (kB01TW / 8), k = v % (kB01TW / 8);
      const int ty = 2 * Y0 - 1 + i, tx = 2 * X0 - 8 + 8 * k;
      rt[u] = u32x4{0u, 0u, 0u, 0u};
      if (v < TCH && ty >= 0 && ty < L0.hin && tx >= 0 && tx < L0.win)
        rt[u] = *reinterpret_cast<const u32x4 *>(tiles + ((int64_t)nn * L0.hin + ty) * L0.win + tx);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < NZ; ++u) {
      const int v = threadIdx.x + 256 * u;
      if (v < ZCH) *reinterpret_cast<u32x4 *>(&zs[(v >> 2) * kB01ZP + 8 * (v & 3)]) = rz[u];
    }
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int v = threadIdx.x + 256 * u;
      if (v < XCH) *reinterpret_cast<u32x4 *>(&xs[(v >> 1) * 16 + 8 * (v & 1)]) = rx[u];
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int v = threadIdx.x + 256 * u;
      if (v < TCH)
        *reinterpret_cast<u32x4 *>(&ts[(v / (kB01TW / 8)) * kB01TW + 8 * (v % (kB01TW / 8))]) = rt[u];
    }
  };
  if ((int)blockIdx.x < nblocks) load(blockIdx.x);
  for (int blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int nn = blk / (BY * BX), r = blk % (BY * BX);
    const int Y0 = (r / BX) * 2 * kB01Rows, X0 = (r % BX) * 2 * kB01Cols;
    __syncthreads();  // the previous block's readers are done
    store();
    __syncthreads();
    if (blk + (int)gridDim.x < nblocks) load(blk + gridDim.x);
    // layer 1's bias: owned pixels p = m + 8k of the staged signal
    {
      const int co = threadIdx.x & 31, m = threadIdx.x >> 5;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int p = m + 8 * k;
        accb1 += bf2f(zs[((p >> 4) * kB01ZW + (p & 15)) * kB01ZP + co]);
      }
    }
    // layer 1's weight gradient over the 64 owned output pixels, K steps
    // of 32: pixel p = 32 ks + 8 g + (s >> 2) (+ 4) for lane s of group g,
    // at output (p >> 4, p & 15) of the block and input (2 (p >> 4) + ky,
    // 2 (p & 15) + kx) of the staged activation
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int s = c16, pr = 2 * ks + (g >> 1), pc = 8 * (g & 1) + (s >> 2);
      u32x4 a[2];
#pragma unroll
      for (int m = 0; m < 2; ++m)
        a[m] = tr_pair(&zs[(pr * kB01ZW + pc) * kB01ZP + 16 * m + 4 * (s & 3)], 4 * kB01ZP);
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int tap = wave + 4 * t;
        if (tap < 9) {
          const int ky = tap / 3, kx = tap % 3;
          const u32x4 b =
              tr_pair(&xs[((2 * pr + ky) * kB01XW + 2 * pc + kx) * 16 + 4 * (s & 3)], 8 * 16);
#pragma unroll
          for (int m = 0; m < 2; ++m) acc1[t][m] = mfma(a[m], b, acc1[t][m]);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    {
      const int cy = wave;
#pragma unroll 1
      for (int cls = 0; cls < 4; ++cls) {
        const int py = cls >> 1, px = cls & 1;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        // taps (ky, kx) whose parity matches the class: an input pixel of
        // parity p is read through ky = 1 (p = 0) or ky = 0, 2 (p = 1)
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
          if (((py + 1 - ky) & 1) != 0) continue;
#pragma unroll
          for (int kx = 0; kx < 3; ++kx) {
            if (((px + 1 - kx) & 1) != 0) continue;
            const int zr = cy + (py + 1 - ky) / 2, zc = c16 + (px + 1 - kx) / 2;
            const u32x4 b = *reinterpret_cast<const u32x4 *>(&zs[(zr * kB01ZW + zc) * kB01ZP + 8 * g]);
            const u32x4 a =
                *reinterpret_cast<const u32x4 *>(&ws[c16 * kB01WP + (ky * 3 + kx) * 32 + 8 * g]);
            acc = mfma(a, b, acc);
          }
        }
        const int iy = Y0 + 2 * cy + py, ix = X0 + 2 * c16 + px;
        const int64_t o = (((int64_t)nn * L0.hout + iy) * L0.wout + ix) * 16 + 4 * g;
        const uint2 a = *reinterpret_cast<const uint2 *>(
            &xs[((iy - Y0 + 1) * kB01XW + ix - X0 + 1) * 16 + 4 * g]);
        const uint16_t ah[4] = {(uint16_t)(a.x & 0xFFFFu), (uint16_t)(a.x >> 16),
                                (uint16_t)(a.y & 0xFFFFu), (uint16_t)(a.y >> 16)};
        uint16_t zq[4];
        float zf[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          zq[j] = bf_positive(ah[j]) ? f2bf(acc[j]) : (uint16_t)0;
          zf[j] = bf2f(zq[j]);
          accb[j] += zf[j];
        }
        if (store0)
          *reinterpret_cast<uint2 *>(dz0 + o) =
              make_uint2((uint32_t)zq[0] | ((uint32_t)zq[1] << 16),
                         (uint32_t)zq[2] | ((uint32_t)zq[3] << 16));
        // the tile values layer 0 read for this pixel: (2 iy + ky - 1,
        // 2 ix + kx - 1), staged at (2 (iy - Y0) + ky, 2 (ix - X0) + kx + 7)
        const uint16_t *tp = ts + (2 * (iy - Y0)) * kB01TW + 2 * (ix - X0) + 7;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
          for (int kx = 0; kx < 3; ++kx) {
            const float tv = bf2f(tp[ky * kB01TW + kx]);
#pragma unroll
            for (int j = 0; j < 4; ++j) accw[j][ky * 3 + kx] = fmaf(zf[j], tv, accw[j][ky * 3 + kx]);
          }
        // one class at a time: its loads are not hoisted into the previous
        // class's work (which would hold every class's temporaries live)
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  float *pw = partial + (int64_t)blockIdx.x * kB01Part;
  // layer 1's weights: the lane holds co = 16 m + 4 g + j, ci = c16 of tap
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int tap = wave + 4 * t;
    if (tap < 9) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          pw[((16 * m + 4 * g + j) * 9 + tap) * 16 + c16] = acc1[t][m][j];
    }
  }
  // workgroup sums, fixed order: the 16 lanes of a channel group
  // (butterfly), then the 4 waves; layer 1's bias over the 8 threads of a
  // channel
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      accb[j] += __shfl_xor(accb[j], o, 64);
#pragma unroll
      for (int t = 0; t < 9; ++t) accw[j][t] += __shfl_xor(accw[j][t], o, 64);
    }
  }
  if (c16 == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int t = 0; t < 9; ++t) red[wave][g][j * 9 + t] = accw[j][t];
      red[wave][g][36 + j] = accb[j];
    }
  }
  red1[threadIdx.x >> 5][threadIdx.x & 31] = accb1;
  __syncthreads();
  if (threadIdx.x < 160) {
    const int i = threadIdx.x;
    // layer 0: weights co = i / 9, tap = i % 9; bias co = i - 144
    const int co = i < 144 ? i / 9 : i - 144;
    const int slot = i < 144 ? (co % 4) * 9 + i % 9 : 36 + co % 4;
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) s += red[w][co / 4][slot];
    pw[kB01W0 + i] = s;
  } else if (threadIdx.x < 192) {
    const int co = threadIdx.x - 160;
    float s = 0.f;
#pragma unroll
    for (int m = 0; m < 8; ++m) s += red1[m][co];
    pw[kB01B1 + co] = s;
  }
}



// ---------------------------------------------------------------------------
// Backward: weights and biases
// ---------------------------------------------------------------------------

// Pixels per staged K step of a layer's weight gradient (a multiple of 32,
// the K of one product).  Larger steps put more products between the
// barriers and the prefetched loads, but their staging registers cost
// occupancy: measured per layer at batch 256, 128 pixels took layer 3 from
// 98 to 89 us, while layers 2, 4 and 5 were slower with 64 or 128 (one wave
// per SIMD).  Layer 2's steps lie in one output row.
constexpr int wg_kp(int li) { return li == 3 ? 128 : 32; }

// bf16 per staged pixel row for C channels: the 4 rows that one group of 16
// lanes reads in a transposed read then fall in disjoint LDS banks (row
// strides of 8, 24, 40 or 72 dwords).
constexpr int wg_row(int c) { return c >= 32 ? c + 16 : c; }

// An MFMA operand with K = 8 consecutive staged pixels: the lane's 16-lane
// group g reads pixels k0 + 8g .. + 7 of channel c0 + (lane % 16) from a
// [pixel][channel] array with rows of `row` bf16.  A transposed read
// (ds_read_b64_tr_b16) gives lane o of a 16-lane group, as its element k
// (k < 4), element o & 3 of the 8 bytes that lane (o >> 2) + 4k of the
// group addresses.  With lane s pointing at pixel k0 + 8g + (s >> 2) (+ 4
// for the second read), channels c0 + 4 (s & 3) .. + 3, lane o therefore
// receives channel c0 + o of 4 consecutive pixels.
__device__ __forceinline__ u32x4 tr_operand(const uint16_t *base, int row, int k0, int c0,
                                            int lane) {
  const int g = lane >> 4, s = lane & 15;
  return tr_pair(base + (k0 + 8 * g + (s >> 2)) * row + c0 + 4 * (s & 3), 4 * row);
}

// partial[split][co][tap][ci] = sum over the split's output pixels q of
// dz[q][co] * x[input of q through tap][ci], layers 2..5, and (workgroups
// of the first tap group) partial[split][W + co] = sum of dz[q][co], the
// bias gradient; rows of W + COUT floats, W = COUT * 9 * CIN.  M = COUT,
// N = CIN, K = pixels, staged 32 pixels at a time through LDS in their
// natural [pixel][channel] layout with 16-byte copies; each lane's 8
// K-values come from two transposed LDS reads.  A workgroup handles TAPS
// taps (grid (9 / TAPS, nsplit)): all 9 for the narrow layers, where the
// staged signal tile is then shared by every tap, one for the wide layers,
// whose accumulators would not fit nine times.  With all 9 taps (stride
// 2) the 32 pixels of a K step lie in one output row, and the input region
// they read (3 rows x 65 pixels) is staged once for all taps; each lane
// addresses its pixels' tap inputs inside it.
template <int LI, int TAPS, int KP = wg_kp(LI)>
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const uint16_t *__restrict__ dz,
                                                              const uint16_t *__restrict__ x,
                                                              float *__restrict__ partial,
                                                              int64_t npix_out, int64_t chunk) {
  constexpr Layer L = kLayers[LI];
  constexpr int CIN = L.cin, COUT = L.cout, S = L.stride;
  constexpr int MB = COUT / 16, NB = CIN / 16, NBLK = MB * NB * TAPS;
  constexpr int PER_WAVE = (NBLK + 3) / 4;
  constexpr int ZR = wg_row(COUT), XR = wg_row(CIN);
  constexpr bool REGION = TAPS == 9;
  static_assert(!REGION || (S == 2 && L.wout % KP == 0), "region staging: whole K steps per row");
  constexpr int RW = 2 * KP + 1;  // region pixels per input row
  __shared__ __attribute__((aligned(16))) uint16_t dzs[KP * ZR];
  __shared__ __attribute__((aligned(16))) uint16_t xs[REGION ? 1 : TAPS][(REGION ? 3 * RW : KP) * XR];
  const int tap0 = blockIdx.x * TAPS;
  const int64_t split = blockIdx.y;
  const int64_t pbeg = split * chunk;
  const int64_t pend = pbeg + chunk < npix_out ? pbeg + chunk : npix_out;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
  constexpr int64_t PW = (int64_t)COUT * 9 * CIN + COUT;  // partial row
  floatx4 acc[PER_WAVE];
#pragma unroll
  for (int b = 0; b < PER_WAVE; ++b) acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
  float accb = 0.f;  // bias: channel threadIdx.x (< COUT), tap group 0
  // One K step's staging in registers: the signal's and the input's 16-byte
  // chunks of this thread (fixed trip counts).  The next step's are loaded
  // while the current one's products run.
  constexpr int ZCH = KP * COUT / 8;
  constexpr int XCH = REGION ? 3 * RW * CIN / 8 : TAPS * KP * CIN / 8;
  constexpr int NZ = (ZCH + 255) / 256, NX = (XCH + 255) / 256;
  u32x4 rz[NZ], rx[NX];
  auto load = [&](int64_t p0) {
#pragma unroll
    for (int u = 0; u < NZ; ++u) {
      const int v = threadIdx.x + 256 * u;
      const int pix = v / (COUT / 8), c8 = (v % (COUT / 8)) * 8;
      const int64_t q = p0 + pix;
      rz[u] = u32x4{0u, 0u, 0u, 0u};
      if (v < ZCH && q < pend) rz[u] = *reinterpret_cast<const u32x4 *>(dz + q * COUT + c8);
    }
    if constexpr (REGION) {
      // input rows 2 oy - 1 .. + 2, columns 2 ox0 - 1 .. 2 ox0 + 2 KP - 1
      const int64_t n = p0 / (L.hout * L.wout);
      const int r0 = (int)(p0 - n * L.hout * L.wout);
      const int oy = r0 / L.wout, ox0 = r0 % L.wout;
#pragma unroll
      for (int u = 0; u < NX; ++u) {
        const int v = threadIdx.x + 256 * u;
        const int pix = v / (CIN / 8), c8 = (v % (CIN / 8)) * 8;
        const int iy = 2 * oy - 1 + pix / RW, ix = 2 * ox0 - 1 + pix % RW;
        rx[u] = u32x4{0u, 0u, 0u, 0u};
        if (v < XCH && iy >= 0 && iy < L.hin && ix >= 0 && ix < L.win)
          rx[u] = *reinterpret_cast<const u32x4 *>(x + ((n * L.hin + iy) * L.win + ix) * CIN + c8);
      }
    } else {
#pragma unroll
      for (int u = 0; u < NX; ++u) {
        const int v = threadIdx.x + 256 * u;
        const int tt = v / (KP * CIN / 8);
        const int rem = v - tt * (KP * CIN / 8);
        const int pix = rem / (CIN / 8), c8 = (rem % (CIN / 8)) * 8;
        const int tap = tap0 + tt;
        const int64_t q = p0 + pix;
        rx[u] = u32x4{0u, 0u, 0u, 0u};
        if (v < XCH && q < pend) {
          const int64_t n = q / (L.hout * L.wout);
          const int r = (int)(q - n * L.hout * L.wout);
          const int iy = S * (r / L.wout) + tap / 3 - 1, ix = S * (r % L.wout) + tap % 3 - 1;
          if (iy >= 0 && iy < L.hin && ix >= 0 && ix < L.win)
            rx[u] = *reinterpret_cast<const u32x4 *>(x + ((n * L.hin + iy) * L.win + ix) * CIN + c8);
        }
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int u = 0; u < NZ; ++u) {
      const int v = threadIdx.x + 256 * u;
      if (v < ZCH)
        *reinterpret_cast<u32x4 *>(&dzs[(v / (COUT / 8)) * ZR + (v % (COUT / 8)) * 8]) = rz[u];
    }
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int v = threadIdx.x + 256 * u;
      if (v < XCH) {
        if constexpr (REGION) {
          *reinterpret_cast<u32x4 *>(&xs[0][(v / (CIN / 8)) * XR + (v % (CIN / 8)) * 8]) = rx[u];
        } else {
          const int tt = v / (KP * CIN / 8);
          const int rem = v - tt * (KP * CIN / 8);
          *reinterpret_cast<u32x4 *>(&xs[tt][(rem / (CIN / 8)) * XR + (rem % (CIN / 8)) * 8]) =
              rx[u];
        }
      }
    }
  };
  if (pbeg < pend) load(pbeg);
  for (int64_t p0 = pbeg; p0 < pend; p0 += KP) {
    store();
    __syncthreads();
    if (p0 + KP < pend) load(p0 + KP);
    if (blockIdx.x == 0 && threadIdx.x < COUT) {
#pragma unroll 8
      for (int k = 0; k < KP; ++k) accb += bf2f(dzs[k * ZR + threadIdx.x]);
    }
#pragma unroll
    for (int b = 0; b < PER_WAVE; ++b) {
      const int blk = wave * PER_WAVE + b;
      if (blk < NBLK) {
        const int tt = blk / (MB * NB), rb = blk % (MB * NB);
        const int mb = rb / NB, nb = rb % NB;
#pragma unroll
        for (int ks = 0; ks < KP / 32; ++ks) {
          const u32x4 av = tr_operand(dzs, ZR, 32 * ks, mb * 16, lane);
          u32x4 bv;
          if constexpr (REGION) {
            // pixel k = 32 ks + 8g + (s >> 2) (+ 4) of the step reads region
            // pixel (ky, 2k + kx) through tap (ky, kx)
            const int tap = tap0 + tt, sl = lane & 15;
            const int k = 32 * ks + 8 * g + (sl >> 2);
            bv = tr_pair(&xs[0][((tap / 3) * RW + 2 * k + tap % 3) * XR + nb * 16 + 4 * (sl & 3)],
                         8 * XR);
          } else {
            bv = tr_operand(xs[tt], XR, 32 * ks, nb * 16, lane);
          }
          acc[b] = mfma(av, bv, acc[b]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < PER_WAVE; ++b) {
    const int blk = wave * PER_WAVE + b;
    if (blk < NBLK) {
      const int tt = blk / (MB * NB), rb = blk % (MB * NB);
      const int mb = rb / NB, nb = rb % NB;
      const int ci = nb * 16 + (lane & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int co = mb * 16 + 4 * g + j;
        partial[split * PW + ((int64_t)co * 9 + tap0 + tt) * CIN + ci] = acc[b][j];
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < COUT)
    partial[split * PW + (PW - COUT) + threadIdx.x] = accb;
}


// Two-level sum of the weight-gradient partials, in a fixed order.  Level
// one: tmp[g][i] = sum of partial[k][i] over the g-th of kWGroups contiguous
// ranges of splits (grid (ceil(W / 256), kWGroups)); threads walk the
// partials in their own layout so that the loads coalesce.  Level two:
// grads[co][ci][tap] = sum_g tmp[g][i] (tmp rows `stride` floats apart),
// and the cout biases that follow the weights in tmp's rows likewise.
constexpr int kWGroups = 32;

__global__ __launch_bounds__(256) void reduce_weight_partial_kernel(
    const float *__restrict__ partial, int nsplit, int64_t total, float *__restrict__ tmp) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int per = (nsplit + kWGroups - 1) / kWGroups;
  const int k0 = blockIdx.y * per;
  const int k1 = k0 + per < nsplit ? k0 + per : nsplit;
  float s = 0.f;
  for (int k = k0; k < k1; ++k) s += partial[(int64_t)k * total + i];
  tmp[(int64_t)blockIdx.y * total + i] = s;
}

__global__ __launch_bounds__(256) void reduce_weight_kernel(const float *__restrict__ tmp,
                                                            int64_t stride, int cout, int cin,
                                                            float *__restrict__ grad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)cout * cin * 9;
  if (i >= total + cout) return;
  if (i >= total) {  // bias
    float s = 0.f;
    for (int g = 0; g < kWGroups; ++g) s += tmp[(int64_t)g * stride + i];
    grad[i] = s;
    return;
  }
  const int co = (int)(i / (9 * cin));
  const int rem = (int)(i - (int64_t)co * 9 * cin);
  const int tap = rem / cin, ci = rem % cin;
  float s = 0.f;
  for (int g = 0; g < kWGroups; ++g) s += tmp[(int64_t)g * stride + i];
  grad[((int64_t)co * cin + ci) * 9 + tap] = s;
}

// out[i] = sum_s part[s][i], one workgroup per output i: thread t adds rows
// t, t + 256, ... and a fixed-order tree in LDS combines the 256 partial
// sums (the result does not depend on scheduling).
__global__ __launch_bounds__(256) void reduce_rows_kernel(const float *__restrict__ part,
                                                          int nrows, int count,
                                                          float *__restrict__ out) {
  __shared__ float red[256];
  const int i = blockIdx.x;
  float s = 0.f;
  for (int k = threadIdx.x; k < nrows; k += 256) s += part[(int64_t)k * count + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// ---------------------------------------------------------------------------
// Optimiser and weight packing
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p,
                                                   const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   int64_t count, float lr, float b1, float b2,
                                                   float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Weight packing of every layer in one launch, from the FP32 master
// weights w[co][ci][tap]: wp[co][tap * cin + ci] (zero in the padding) and,
// where the layer has one, wt[ci][tap * cout + co], both bfloat16; element e
// belongs to the layer whose [begin, begin + cout * kpad) range holds it.
// The 144 elements after the last layer write layer 0's weights rounded to
// bfloat16 and kept as FP32 (w0f [16][9], for the forward kernel's scalar
// loads).
struct PackAll {
  int64_t begin[kNumLayers + 1];  // element ranges; begin[kNumLayers] = total packed
  int64_t param[kNumLayers];      // offset of each layer's master weights
  uint16_t *wp[kNumLayers], *wt[kNumLayers];
};

__global__ __launch_bounds__(256) void pack_all_kernel(const float *__restrict__ params, PackAll a,
                                                       float *__restrict__ w0f) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.begin[kNumLayers]) {
    const int64_t i = e - a.begin[kNumLayers];
    if (i < 16 * 9) w0f[i] = bf2f(f2bf(params[a.param[0] + i]));
    return;
  }
  int li = 0;
#pragma unroll
  for (int k = 1; k < kNumLayers; ++k) li += e >= a.begin[k] ? 1 : 0;
  const Layer L = kLayers[li];
  const int kpad = L.kpad();
  const int64_t le = e - a.begin[li];
  const int co = (int)(le / kpad), k = (int)(le % kpad);
  const int tap = k / L.cin, ci = k % L.cin;
  if (tap >= 9) {
    a.wp[li][le] = 0;
    return;
  }
  const uint16_t b = f2bf(params[a.param[li] + ((int64_t)co * L.cin + ci) * 9 + tap]);
  a.wp[li][le] = b;
  if (a.wt[li]) a.wt[li][(int64_t)ci * 9 * L.cout + tap * L.cout + co] = b;
}

int64_t layer_param_offset(int li) {
  int64_t off = 0;
  for (int i = 0; i < li; ++i) off += kLayers[i].wcount() + kLayers[i].cout;
  return off;
}
constexpr int64_t head_param_offset() {
  int64_t off = 0;
  for (int i = 0; i < kNumLayers; ++i) off += kLayers[i].wcount() + kLayers[i].cout;
  return off;
}
constexpr int64_t kParams = head_param_offset() + kHead * kFeat + kHead;

int64_t npix_out(int li, int n) { return (int64_t)n * kLayers[li].hout * kLayers[li].wout; }
int64_t npix_in(int li, int n) { return (int64_t)n * kLayers[li].hin * kLayers[li].win; }
// Blocks and workgroups of the fused layer-1 / layer-0 backward kernel.
int b01_blocks(int n) {
  return n * (kLayers[0].hout / (2 * kB01Rows)) * (kLayers[0].wout / (2 * kB01Cols));
}
int b01_grid(int n) {
  static int resident = 0;
  if (resident == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(bwd01_kernel), 256, 0);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int r = e == hipSuccess ? (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1) : kB01Grid;
    resident = r < kB01Grid ? r : kB01Grid;
  }
  return b01_blocks(n) < resident ? b01_blocks(n) : resident;
}

// Workgroups of a layer's weight-gradient kernel along its other grid
// dimension (9 / taps per workgroup) for layers 2..5; layers 0 and 1 take
// their gradients from the fused kernel (entries unused).
int wgrad_groups(int li) {
  static const int g[kNumLayers] = {1, 1, 1, 9, 9, 9};
  return g[li];
}

// Pixel splits of the weight-gradient reduction: about 512 workgroups in
// total per layer (two per compute unit; each prefetches its next K step,
// so long pixel ranges cost little, and fewer splits mean fewer FP32
// partials to write and sum), chunks a multiple of the layer's K step.
int64_t split_chunk(int64_t npix, int li) {
  const int64_t target = 512 / wgrad_groups(li), kp = wg_kp(li);
  int64_t c = (npix + target - 1) / target;
  c = (c + kp - 1) / kp * kp;
  return c < kp ? kp : c;
}

}  // namespace

struct sps_cnn_s {
  int device = 0;
  int32_t max_batch = 0;
  int64_t step = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *wp[kNumLayers] = {}, *wt[kNumLayers] = {};
  uint16_t *act[kNumLayers] = {}, *dz[kNumLayers] = {};
  float *partial = nullptr;   // weight-gradient partials (largest layer)
  float *wtmp = nullptr;      // second level of the weight-gradient sum
  float *head_part = nullptr; // per head block: [3][128] + [3] + [1]
  float *loss = nullptr;      // device scalar of the last loss_grad
  float *head = nullptr;      // head outputs of the last forward
  float *w0f = nullptr;       // layer-0 weights rounded to bfloat16, as FP32 [16][9]
  float pos_weight = kPosWeight, lambda_box = kLambdaBox;
  int64_t partial_cap = 0;
};

namespace {

sps_status cnn_dev_fail(hipError_t e, const char *what) {
  char m[256];
  snprintf(m, sizeof m, "%s: %s", what, hipGetErrorString(e));
  return sps::set_error(SPS_ERR_DEVICE, m);
}

void cnn_free(sps_cnn c) {
  void *ptrs[] = {c->params, c->grads, c->m, c->v, c->partial, c->head_part, c->loss,
                  c->head, c->wtmp, c->w0f};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (int i = 0; i < kNumLayers; ++i) {
    if (c->wp[i]) (void)hipFree(c->wp[i]);
    if (c->wt[i]) (void)hipFree(c->wt[i]);
    if (c->act[i]) (void)hipFree(c->act[i]);
    if (c->dz[i]) (void)hipFree(c->dz[i]);
  }
}

hipError_t pack_all(sps_cnn c, hipStream_t s) {
  PackAll a{};
  int64_t total = 0;
  for (int i = 0; i < kNumLayers; ++i) {
    a.begin[i] = total;
    a.param[i] = layer_param_offset(i);
    a.wp[i] = c->wp[i];
    a.wt[i] = c->wt[i];
    total += (int64_t)kLayers[i].cout * kLayers[i].kpad();
  }
  a.begin[kNumLayers] = total;
  hipLaunchKernelGGL(pack_all_kernel, dim3((unsigned)((total + 16 * 9 + 255) / 256)), dim3(256), 0,
                     s, c->params, a, c->w0f);
  return hipGetLastError();
}

#define SPS_LAUNCH_CHECK(what)                     \
  do {                                             \
    hipError_t e_ = hipGetLastError();             \
    if (e_ != hipSuccess) return cnn_dev_fail(e_, what); \
  } while (0)

template <int LI, int BH, int BW, int WM, int WN, bool FUSE0, bool STORE0>
hipError_t launch_fwd_lds(const uint16_t *x, const uint16_t *wp, const float *bias, uint16_t *y,
                          const float *w0f, const float *b0, uint16_t *y0, int n, hipStream_t s) {
  using G = FwdGeom<LI, BH, BW>;
  const size_t lds = sizeof(uint16_t) * (size_t)G::lds(FUSE0);
  auto kern = conv_fwd_lds_kernel<LI, BH, BW, WM, WN, FUSE0, STORE0>;
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // fused layer 0: persistent, as many workgroups as are resident at once,
  // each looping over blocks (the next block's loads overlap the current
  // one's work); other layers: one block per workgroup
  static int resident = FUSE0 ? 0 : 0x7FFFFFFF;  // per kernel instance
  if (resident == 0) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(kern), 256, lds);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    resident = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  }
  const int64_t blocks = (int64_t)(G::L.hout / BH) * (G::L.wout / BW) * n;
  const int grid = (int)(blocks < resident ? blocks : resident);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, s, x, wp, bias, y, w0f, b0, y0, n);
  return hipGetLastError();
}

// Layers 0..5.  Layer 0 runs inside layer 1's workgroups; keep0: also
// store layer 0's activation (training and read-back need it).
sps_status run_forward(sps_cnn c, const uint16_t *tiles, int32_t n, hipStream_t s, bool keep0) {
  const float *w0f = c->w0f, *b0 = c->params + layer_param_offset(0) + kLayers[0].wcount();
  hipError_t e = hipSuccess;
#define SPS_FWD_LAUNCH(LI, BH, BW, WM, WN)                                                   \
  if (e == hipSuccess) {                                                                     \
    const float *bias = c->params + layer_param_offset(LI) + kLayers[LI].wcount();          \
    if (LI == 1 && keep0)                                                                    \
      e = launch_fwd_lds<LI, BH, BW, WM, WN, LI == 1, true>(tiles, c->wp[LI], bias,          \
                                                              c->act[LI], w0f, b0, c->act[0], n, s); \
    else                                                                                     \
      e = launch_fwd_lds<LI, BH, BW, WM, WN, LI == 1, false>(                                \
          LI == 1 ? tiles : c->act[LI - 1], c->wp[LI], bias, c->act[LI], w0f, b0, c->act[0], n, s); \
  }
  SPS_FWD_LDS_CONFIGS(SPS_FWD_LAUNCH)
#undef SPS_FWD_LAUNCH
  if (e != hipSuccess) return cnn_dev_fail(e, "forward launch");
  return SPS_OK;
}

sps_status run_head(sps_cnn c, const float *labels, int32_t n, bool train, hipStream_t s) {
  const int64_t ncell = (int64_t)n * kCells;
  const int nblk = (int)((ncell + 127) / 128);
  float *part_wh = c->head_part;
  float *part_bh = part_wh + (int64_t)nblk * kHead * kFeat;
  float *part_loss = part_bh + (int64_t)nblk * kHead;
  const int64_t hoff = head_param_offset();
  hipLaunchKernelGGL(head_loss_kernel, dim3((unsigned)nblk), dim3(128), 0, s, c->act[5],
                     c->params + hoff, c->params + hoff + kHead * kFeat, labels, ncell,
                     1.0f / (float)n, c->head, c->dz[5], part_wh, part_bh, part_loss, train ? 1 : 0,
                     c->pos_weight, c->lambda_box);
  if (train) {
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(kHead * kFeat), dim3(256), 0, s,
                       part_wh, nblk, kHead * kFeat, c->grads + hoff);
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(kHead), dim3(256), 0, s, part_bh, nblk, kHead,
                       c->grads + hoff + kHead * kFeat);
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(256), 0, s, part_loss, nblk, 1, c->loss);
  }
  SPS_LAUNCH_CHECK("head launch");
  return SPS_OK;
}

// keep0: store layer 0's signal (for sps_cnn_signals); no product reads it.
sps_status run_backward(sps_cnn c, const uint16_t *tiles, int32_t n, hipStream_t s, bool keep0) {
  for (int li = kNumLayers - 1; li >= 1; --li) {
    const Layer &L = kLayers[li];
    float *gw = c->grads + layer_param_offset(li);
    if (li == 1) {
      // layers 1 and 0: one fused kernel, then the two-level sums of its
      // partials (weights of both layers, then the biases)
      float *gw0 = c->grads + layer_param_offset(0);
      const int nwg = b01_grid(n);
      hipLaunchKernelGGL(bwd01_kernel, dim3((unsigned)nwg), dim3(256), 0, s, c->dz[1], c->wt[1],
                         c->act[0], tiles, c->dz[0], c->partial, b01_blocks(n), keep0 ? 1 : 0);
      hipLaunchKernelGGL(reduce_weight_partial_kernel,
                         dim3((unsigned)((kB01Part + 255) / 256), kWGroups), dim3(256), 0, s,
                         c->partial, nwg, (int64_t)kB01Part, c->wtmp);
      hipLaunchKernelGGL(reduce_weight_kernel, dim3((unsigned)((kB01W1 + 32 + 255) / 256)),
                         dim3(256), 0, s, c->wtmp, (int64_t)kB01Part, 32, 16, gw);
      hipLaunchKernelGGL(reduce_weight_kernel, dim3(1), dim3(256), 0, s, c->wtmp + kB01W0,
                         (int64_t)kB01Part, 16, 1, gw0);
      SPS_LAUNCH_CHECK("backward launch");
      break;
    }
    const int64_t np = npix_out(li, n);
    const int64_t chunk = split_chunk(np, li);
    const int64_t nsplit = (np + chunk - 1) / chunk;
    const uint16_t *xin = c->act[li - 1];
    switch (li) {
#define SPS_BWDW(LI, TAPS)                                                                   \
  case LI:                                                                                   \
    hipLaunchKernelGGL((conv_bwd_weight_kernel<LI, TAPS>), dim3(9 / TAPS, (unsigned)nsplit),  \
                       dim3(256), 0, s, c->dz[LI], xin, c->partial, np, chunk);              \
    break;
      SPS_BWDW(2, 9) SPS_BWDW(3, 1) SPS_BWDW(4, 1) SPS_BWDW(5, 1)
#undef SPS_BWDW
    }
    {
      const int64_t pw = L.wcount() + L.cout;  // partial row: weights, then biases
      hipLaunchKernelGGL(reduce_weight_partial_kernel, dim3((unsigned)((pw + 255) / 256), kWGroups),
                         dim3(256), 0, s, c->partial, (int)nsplit, pw, c->wtmp);
      hipLaunchKernelGGL(reduce_weight_kernel, dim3((unsigned)((pw + 255) / 256)), dim3(256), 0, s,
                         c->wtmp, pw, L.cout, L.cin, gw);
    }
    switch (li) {
#define X(LI, WMG, RPW)                                                                       \
  case LI:                                                                                    \
    hipLaunchKernelGGL((bwd_data_lds_kernel<LI, WMG, RPW>),                                   \
                       dim3((unsigned)bwd_data_lds_grid<LI, WMG, RPW>(n)), dim3(256), 0, s,   \
                       c->dz[LI], c->wt[LI], c->act[LI - 1], c->dz[LI - 1],                   \
                       bwd_data_lds_blocks<LI, WMG, RPW>(n));                                 \
    break;
      SPS_BWD_LDS_CONFIGS
#undef X
    }
    SPS_LAUNCH_CHECK("backward launch");
  }
  return SPS_OK;
}

sps_status check_batch(sps_cnn c, const void *tiles, int32_t n) {
  if (!c || !tiles) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL network or tiles");
  if (n < 1 || n > c->max_batch)
    return sps::set_error(SPS_ERR_INVALID_ARG, "batch size must be in [1, max_batch]");
  if ((uintptr_t)tiles % 16 != 0) return sps::set_error(SPS_ERR_INVALID_ARG, "tiles not 16-byte aligned");
  return SPS_OK;
}

}  // namespace

extern "C" {

int64_t sps_cnn_param_count(void) { return kParams; }

sps_status sps_cnn_create(int32_t max_batch, sps_cnn *out) {
  if (!out) return sps::set_error(SPS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > 4096)
    return sps::set_error(SPS_ERR_INVALID_ARG, "max_batch must be in [1, 4096]");
  sps_cnn c = new (std::nothrow) sps_cnn_s;
  if (!c) return sps::set_error(SPS_ERR_NOMEM, "host allocation failed");
  hipError_t e = hipGetDevice(&c->device);
  c->max_batch = max_batch;
  int64_t pmax = 0;
  for (int i = 0; i < kNumLayers; ++i) {
    const int64_t np = npix_out(i, max_batch);
    const int64_t ns = (np + split_chunk(np, i) - 1) / split_chunk(np, i);
    const int64_t row = kLayers[i].wcount() + kLayers[i].cout;
    pmax = ns * row > pmax ? ns * row : pmax;
  }
  pmax = (int64_t)kB01Grid * kB01Part > pmax ? (int64_t)kB01Grid * kB01Part : pmax;
  c->partial_cap = pmax;
  const int64_t nblk = ((int64_t)max_batch * kCells + 127) / 128;
  auto alloc = [&](void **p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  alloc((void **)&c->params, sizeof(float) * kParams);
  alloc((void **)&c->grads, sizeof(float) * kParams);
  alloc((void **)&c->m, sizeof(float) * kParams);
  alloc((void **)&c->v, sizeof(float) * kParams);
  alloc((void **)&c->partial, sizeof(float) * (size_t)pmax);
  alloc((void **)&c->wtmp,
        sizeof(float) * (size_t)kWGroups * (size_t)(kLayers[5].wcount() + kLayers[5].cout));
  alloc((void **)&c->head_part, sizeof(float) * (size_t)(nblk * (kHead * kFeat + kHead + 1)));
  alloc((void **)&c->loss, sizeof(float) * 4);
  alloc((void **)&c->head, sizeof(float) * (size_t)max_batch * kHead * kCells);
  alloc((void **)&c->w0f, sizeof(float) * 16 * 9);
  for (int i = 0; i < kNumLayers; ++i) {
    const Layer &L = kLayers[i];
    alloc((void **)&c->wp[i], sizeof(uint16_t) * (size_t)L.cout * L.kpad());
    if (i > 0) alloc((void **)&c->wt[i], sizeof(uint16_t) * (size_t)L.cin * 9 * L.cout);
    const size_t a = sizeof(uint16_t) * (size_t)npix_out(i, max_batch) * L.cout;
    alloc((void **)&c->act[i], a);
    alloc((void **)&c->dz[i], a);
  }
  if (e == hipSuccess) e = hipMemset(c->params, 0, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMemset(c->grads, 0, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMemset(c->m, 0, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMemset(c->v, 0, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMemset(c->loss, 0, sizeof(float) * 4);
  if (e == hipSuccess) {
    e = pack_all(c, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    cnn_free(c);
    delete c;
    return sps::set_error(SPS_ERR_NOMEM, "device allocation for the network failed");
  }
  *out = c;
  return SPS_OK;
}

sps_status sps_cnn_destroy(sps_cnn c) {
  if (!c) return SPS_OK;
  (void)hipDeviceSynchronize();
  cnn_free(c);
  delete c;
  return SPS_OK;
}

sps_status sps_cnn_set_params(sps_cnn c, const float *host) {
  if (!c || !host) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL argument");
  hipError_t e = hipMemcpy(c->params, host, sizeof(float) * kParams, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->m, 0, sizeof(float) * kParams);
  if (e == hipSuccess) e = hipMemset(c->v, 0, sizeof(float) * kParams);
  if (e == hipSuccess) e = pack_all(c, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return cnn_dev_fail(e, "setting parameters");
  c->step = 0;
  return SPS_OK;
}

sps_status sps_cnn_set_loss_weights(sps_cnn c, float pos_weight, float lambda_box) {
  if (!c) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL network");
  if (!(pos_weight > 0.0f) || !(lambda_box >= 0.0f) || !isfinite(pos_weight) || !isfinite(lambda_box))
    return sps::set_error(SPS_ERR_INVALID_ARG, "loss weights must be finite, pos_weight > 0");
  c->pos_weight = pos_weight;
  c->lambda_box = lambda_box;
  return SPS_OK;
}

sps_status sps_cnn_get_params(sps_cnn c, float *host) {
  if (!c || !host) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL argument");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host, c->params, sizeof(float) * kParams, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return cnn_dev_fail(e, "reading parameters");
  return SPS_OK;
}

sps_status sps_cnn_get_grads(sps_cnn c, float *host) {
  if (!c || !host) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL argument");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host, c->grads, sizeof(float) * kParams, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return cnn_dev_fail(e, "reading gradients");
  return SPS_OK;
}

sps_status sps_cnn_set_grads(sps_cnn c, const float *host) {
  if (!c || !host) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL argument");
  hipError_t e = hipMemcpy(c->grads, host, sizeof(float) * kParams, hipMemcpyHostToDevice);
  if (e != hipSuccess) return cnn_dev_fail(e, "setting gradients");
  return SPS_OK;
}

sps_status sps_cnn_activations(sps_cnn c, int32_t layer, int32_t n, uint16_t *host) {
  if (!c || !host || layer < 0 || layer >= kNumLayers || n < 1 || n > c->max_batch)
    return sps::set_error(SPS_ERR_INVALID_ARG, "bad network, layer, count or output");
  hipError_t e = hipDeviceSynchronize();
  const size_t bytes = sizeof(uint16_t) * (size_t)npix_out(layer, n) * kLayers[layer].cout;
  if (e == hipSuccess) e = hipMemcpy(host, c->act[layer], bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return cnn_dev_fail(e, "reading activations");
  return SPS_OK;
}

sps_status sps_cnn_signals(sps_cnn c, int32_t layer, int32_t n, uint16_t *host) {
  if (!c || !host || layer < 0 || layer >= kNumLayers || n < 1 || n > c->max_batch)
    return sps::set_error(SPS_ERR_INVALID_ARG, "bad network, layer, count or output");
  hipError_t e = hipDeviceSynchronize();
  const size_t bytes = sizeof(uint16_t) * (size_t)npix_out(layer, n) * kLayers[layer].cout;
  if (e == hipSuccess) e = hipMemcpy(host, c->dz[layer], bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return cnn_dev_fail(e, "reading back-propagated signals");
  return SPS_OK;
}

sps_status sps_cnn_pool_tiles(const float *snr, int64_t pitch, int32_t ndm, int64_t nout,
                              float scale, uint16_t *tiles, void *stream) {
  if (!snr || !tiles) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL plane or tiles");
  if (ndm < kPoolDm || nout < kPoolT || pitch < nout)
    return sps::set_error(SPS_ERR_INVALID_ARG, "plane smaller than one pooling window");
  const int64_t nd = ndm / kPoolDm, nt = nout / kPoolT;
  const int64_t total = nd * nt;
  if ((total + 255) / 256 > 0x7FFFFFFF) return sps::set_error(SPS_ERR_RANGE, "plane too large");
  hipLaunchKernelGGL(pool_tiles_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, snr, pitch, nd, nt, scale, tiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return cnn_dev_fail(e, "pooling launch");
  return SPS_OK;
}

sps_status sps_cnn_pool_tile_grid(const float *snr, int64_t pitch, int32_t ndm, int64_t nout,
                                  float scale, uint16_t *tiles, int64_t *ntiles, void *stream) {
  if (!snr || !ntiles) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL plane or count");
  if (ndm < 0 || nout < 0 || pitch < nout)
    return sps::set_error(SPS_ERR_INVALID_ARG, "bad plane shape");
  const int64_t nrows = ndm / (kTileDm * kPoolDm), ncols = nout / (kTileT * kPoolT);
  *ntiles = nrows * ncols;
  if (*ntiles == 0) return SPS_OK;
  if (!tiles) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL tiles");
  const int64_t total = *ntiles * kTileDm * kTileT;
  if ((total + 255) / 256 > 0x7FFFFFFF || ncols > 0x7FFFFFFF)
    return sps::set_error(SPS_ERR_RANGE, "plane too large");
  hipLaunchKernelGGL(pool_tile_grid_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, snr, pitch, (int)ncols, *ntiles, scale, tiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return cnn_dev_fail(e, "tile-grid pooling launch");
  return SPS_OK;
}

int32_t sps_cnn_max_batch(sps_cnn c) { return c ? c->max_batch : 0; }

sps_status sps_cnn_forward(sps_cnn c, const uint16_t *tiles, int32_t n, float *head,
                           void *stream) {
  sps_status r = check_batch(c, tiles, n);
  if (r != SPS_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  r = run_forward(c, tiles, n, s, true);
  if (r != SPS_OK) return r;
  r = run_head(c, nullptr, n, false, s);
  if (r != SPS_OK) return r;
  if (head) {
    hipError_t e = hipMemcpyAsync(head, c->head, sizeof(float) * (size_t)n * kHead * kCells,
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return cnn_dev_fail(e, "head copy");
  }
  return SPS_OK;
}

sps_status sps_cnn_infer(sps_cnn c, const uint16_t *tiles, int32_t n, float *head, void *stream) {
  sps_status r = check_batch(c, tiles, n);
  if (r != SPS_OK) return r;
  hipStream_t s = (hipStream_t)stream;
  r = run_forward(c, tiles, n, s, false);
  if (r != SPS_OK) return r;
  r = run_head(c, nullptr, n, false, s);
  if (r != SPS_OK) return r;
  if (head) {
    hipError_t e = hipMemcpyAsync(head, c->head, sizeof(float) * (size_t)n * kHead * kCells,
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return cnn_dev_fail(e, "head copy");
  }
  return SPS_OK;
}

namespace {
sps_status loss_grad(sps_cnn c, const uint16_t *tiles, const float *labels, int32_t n, float *loss,
                     void *stream, bool keep0) {
  sps_status r = check_batch(c, tiles, n);
  if (r != SPS_OK) return r;
  if (!labels) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL labels");
  hipStream_t s = (hipStream_t)stream;
  r = run_forward(c, tiles, n, s, true);
  if (r == SPS_OK) r = run_head(c, labels, n, true, s);
  if (r == SPS_OK) r = run_backward(c, tiles, n, s, keep0);
  if (r != SPS_OK) return r;
  if (loss) {
    hipError_t e = hipMemcpyAsync(loss, c->loss, sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return cnn_dev_fail(e, "loss copy");
  }
  return SPS_OK;
}
}  // namespace

sps_status sps_cnn_loss_grad(sps_cnn c, const uint16_t *tiles, const float *labels, int32_t n,
                             float *loss, void *stream) {
  return loss_grad(c, tiles, labels, n, loss, stream, true);
}

sps_status sps_cnn_adam(sps_cnn c, float lr, float beta1, float beta2, float eps, void *stream) {
  if (!c) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL network");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return sps::set_error(SPS_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  hipStream_t s = (hipStream_t)stream;
  c->step += 1;
  const double bc1 = 1.0 - pow((double)beta1, (double)c->step);
  const double bc2 = 1.0 - pow((double)beta2, (double)c->step);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, s,
                     c->params, c->grads, c->m, c->v, kParams, lr, beta1, beta2, eps, (float)bc1,
                     (float)bc2);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = pack_all(c, s);
  if (e != hipSuccess) return cnn_dev_fail(e, "Adam launch");
  return SPS_OK;
}

sps_status sps_cnn_train_step(sps_cnn c, const uint16_t *tiles, const float *labels, int32_t n,
                              float lr, float *loss, void *stream) {
  sps_status r = loss_grad(c, tiles, labels, n, loss, stream, false);
  if (r != SPS_OK) return r;
  return sps_cnn_adam(c, lr, 0.9f, 0.999f, 1e-8f, stream);
}

sps_status sps_cnn_detect(sps_cnn c, const uint16_t *tiles, int32_t n, float threshold,
                          sps_cnn_candidate *out, int32_t cap, int32_t *n_found, void *stream) {
  if (!n_found) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL n_found");
  *n_found = 0;
  if (cap < 0 || (cap > 0 && !out)) return sps::set_error(SPS_ERR_INVALID_ARG, "bad output array");
  if (!(threshold > 0.0f && threshold < 1.0f))
    return sps::set_error(SPS_ERR_INVALID_ARG, "threshold must be a probability in (0, 1)");
  sps_status r = sps_cnn_infer(c, tiles, n, nullptr, stream);
  if (r != SPS_OK) return r;
  std::vector<float> h((size_t)n * kHead * kCells);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(h.data(), c->head, sizeof(float) * h.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return cnn_dev_fail(e, "reading head outputs");
  const float logit = logf(threshold / (1.0f - threshold));
  int32_t found = 0;
  for (int32_t t = 0; t < n; ++t)
    for (int cell = 0; cell < kCells; ++cell) {
      const float o = h[((size_t)t * kHead + 0) * kCells + cell];
      if (!(o >= logit)) continue;
      if (found < cap) {
        const int gy = cell / kGridT, gx = cell % kGridT;
        sps_cnn_candidate &q = out[found];
        q.tile = t;
        q.cell_dm = gy;
        q.cell_t = gx;
        q.prob = 1.0f / (1.0f + expf(-o));
        q.row = (gy + h[((size_t)t * kHead + 1) * kCells + cell]) * (float)(kTileDm / kGridDm);
        q.col = (gx + h[((size_t)t * kHead + 2) * kCells + cell]) * (float)(kTileT / kGridT);
      }
      ++found;
    }
  *n_found = found;
  if (found > cap) return sps::set_error(SPS_ERR_TRUNCATED, "more cells above threshold than cap");
  return SPS_OK;
}

}  // extern "C"

namespace sps {

sps_status cnn_count_cells(sps_cnn c, const uint16_t *tiles, int32_t n, float threshold,
                           int32_t *count, hipStream_t s) {
  sps_status r = check_batch(c, tiles, n);
  if (r != SPS_OK) return r;
  if (!count) return set_error(SPS_ERR_INVALID_ARG, "NULL count");
  if (!(threshold > 0.0f && threshold < 1.0f))
    return set_error(SPS_ERR_INVALID_ARG, "threshold must be a probability in (0, 1)");
  r = run_forward(c, tiles, n, s, false);
  if (r != SPS_OK) return r;
  r = run_head(c, nullptr, n, false, s);
  if (r != SPS_OK) return r;
  // the same FP32 logit and comparison as sps_cnn_detect, so counts agree
  const float logit = logf(threshold / (1.0f - threshold));
  const int64_t cells = (int64_t)n * kCells;
  hipLaunchKernelGGL(count_cells_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s,
                     c->head, n, logit, count);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return cnn_dev_fail(e, "cell count launch");
  return SPS_OK;
}

}  // namespace sps

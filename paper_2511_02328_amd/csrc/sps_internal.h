// sps_internal.h -- declarations shared by the HIP sources of libsps (not part
// of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sps.h"

namespace sps {

// Tile configuration of the dedispersion kernel.
//   m    : output dwords per lane (odd, so lane-strided LDS reads hit distinct
//          banks); a wave covers 64 lanes x 4m samples = 256 m outputs.
//   dpw  : DM trials each wave accumulates at once.
//   nw   : waves per workgroup; a workgroup covers nw * dpw trials.
//   cs   : channels per LDS slab (even, divides 256, multiple of nw).
//   kmax : 16-byte vectors per lane per staged row (row <= 1024 kmax bytes).
//   wpe  : waves per SIMD the register budget is sized for.
// m == 0 selects the plain global-memory kernel.
struct DedispConfig {
  int m, dpw, nw, cs, kmax, wpe;
  int nt() const { return 256 * m; }
  int nd() const { return nw * dpw; }
  int64_t lds_bytes(int64_t pitch) const { return 2 * (int64_t)cs * pitch; }
};

// Bytes of one staged channel row for a config whose DM blocks span at most
// `spread` samples of delay in any channel.
int64_t dedisp_lds_pitch(const DedispConfig &cfg, int spread);

// Largest delay difference within any block of nd consecutive trials.
int dedisp_block_spread(const int32_t *delays_host, int nchan, int ndm, int nd);

// True if the config is one the library instantiates.
bool dedisp_config_supported(const DedispConfig &cfg);

// Every buffer the kernels touch is in device memory.  Pointers are cast to
// the global address space where they are dereferenced: a pointer that a
// kernel reads from memory (a BeamWork field) or receives in a non-inlined
// function is generic to the compiler, which then emits flat loads and
// stores, and flat operations also count against the LDS wait counter, so
// every LDS wait would wait for them too.
#define SPS_GLOBAL __attribute__((address_space(1)))
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// four dwords at any dword-aligned address (one 16-byte load on gfx950)
typedef unsigned int u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

template <typename T>
__device__ __forceinline__ const SPS_GLOBAL T *gmem(const T *p) {
  return (const SPS_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ SPS_GLOBAL T *gmem(T *p) {
  return (SPS_GLOBAL T *)p;
}

// Per-filterbank work description of a batched call (device memory).  The
// *_begin fields are exclusive prefix sums of each kernel's work items over
// the preceding beams.
struct BeamWork {
  const uint8_t *X;
  int64_t pitch;
  int64_t nsamp_in;
  uint32_t *Y;
  int64_t nout;
  float *snr;
  uint8_t *best;
  int32_t *stats;
  int64_t dd_begin;     // dedispersion items (time tile x DM block)
  int64_t bx_begin;     // boxcar workgroups (DM row x segment)
  int64_t tp_begin;     // detection tiles
  int64_t nseg;         // boxcar segments per row
  int64_t ntt;          // detection tiles along time
  int64_t det_begin;    // byte offset of the beam's detection scratch
  int64_t pl_begin;     // pooled-tile boxcar workgroups (trial pair x tile column)
  int64_t tile_begin;   // first detector tile of the beam
  int64_t pcols;        // whole tiles along time
  int32_t vec_store;
  int32_t pad;
};

// The beam whose work range holds `item`: the last b with beams[b].*F <=
// item (the ranges are exclusive prefix sums from 0, so an empty beam never
// wins over the beam after it).  Binary search: log2(nbeams) dependent
// scalar loads.
template <int64_t BeamWork::*F>
__device__ __forceinline__ int find_beam(const BeamWork *beams, int nbeams, int64_t item) {
  int lo = 0, hi = nbeams - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (beams[mid].*F <= item)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// As find_beam for an item that is the same in every lane of the wave (a
// workgroup's own index): each lane compares one beam's start, 64 beams per
// load, so the search costs one load latency instead of a chain of them.
// Every lane of the wave must call it.
template <int64_t BeamWork::*F>
__device__ __forceinline__ int find_beam_wave(const BeamWork *beams, int nbeams, int64_t item) {
  int count = 0;
  for (int base = 0; base < nbeams; base += 64) {
    const int b = base + (int)(threadIdx.x & 63);
    count += __popcll(__ballot(b < nbeams && beams[b].*F <= item));
  }
  return count - 1;
}

// The delay table D [ndm][nchan] in the form the staged kernels of one
// tiling read (blocks of nd = nw dpw trials, slabs of cs rows, staged rows of
// `pitch` bytes):
//   P[d][c] = {(c mod cs) pitch/4 + (D[d][c] - B[d/nd][c]) / 4,
//              perm selector of bytes (r, r+2), r = D[d][c] mod 4}
//     with pcols columns (nchan rounded up to a multiple of cs; the padding
//     columns point at the start of their zeroed slab row)
//   B[j][c] = D[j nd][c] rounded down to a multiple of 16 (first staged
//             sample of channel c's row for DM block j).
// Device memory owned by the struct's holder (free_staged).
struct StagedDelays {
  int2 *P = nullptr;
  int32_t *B = nullptr;
  int nchan = 0, pcols = 0, ndm = 0, nd = 0, cs = 0, pitch = 0;
  int32_t dmax = 0;  // largest delay of the table
  bool matches(const DedispConfig &c, int lds_pitch, int nc, int nd_trials) const {
    return P && nchan == nc && ndm == nd_trials && nd == c.nd() && cs == c.cs &&
           pitch == lds_pitch;
  }
};

// (Re)builds sd for tiling c from the device table D (largest entry dmax)
// unless it already matches; frees it for the plain kernel (m = 0).  Allocates, and waits for
// its own kernel, so it is never called inside a launch sequence that a
// caller may capture.
hipError_t stage_delays(StagedDelays &sd, const DedispConfig &c, int lds_pitch, const int32_t *D,
                        int nchan, int ndm, int32_t dmax);
void free_staged(StagedDelays &sd);

int64_t dedisp_batch_items(const DedispConfig &c, int ndm, int64_t nout);
hipError_t launch_dedisperse_batch(const DedispConfig &c, int lds_pitch, const BeamWork *beams,
                                   int nbeams, int64_t total_items, const StagedDelays &sd,
                                   int nchan, int ndm, int grid, hipStream_t stream);

// D: raw table (plain kernel, m = 0); sd: its staged form for tiling cfg
// (m > 0).  seg > 0: channel groups of seg (a multiple of the slab, dividing
// nchan) write their partial sums to planes Y + g seg_stride (m > 0 tilings
// only).
hipError_t launch_dedisperse(const DedispConfig &cfg, int lds_pitch, const uint8_t *X,
                             int64_t pitch, int64_t nsamp_in, const int32_t *D,
                             const StagedDelays *sd, int nchan, int ndm, uint32_t *Y,
                             int64_t nout, hipStream_t stream, int seg = 0,
                             int64_t seg_stride = 0);

hipError_t launch_row_stats(const uint32_t *Y, int ndm, int64_t nout, uint32_t vmax,
                            int32_t *stats, hipStream_t stream);

constexpr int kMaxWidths = 64;
constexpr int kMaxWidth = 8192;

struct WidthList {
  int32_t n;
  int32_t w[kMaxWidths];
};

// Order-preserving map of a binary32 S/N to an unsigned integer (a larger
// value maps to a larger integer, -0 just below +0), and its inverse.
__device__ __forceinline__ uint32_t snr_key_bits(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float snr_from_key_bits(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Tile maxima of a plane gathered by the boxcar pass itself.  Detection
// tiles are tile_dm trials x tile_t samples (ntt of them along time); each
// tile has one 64-bit key: snr_key_bits(S/N) in the high word, the
// complement of the in-tile position (t - t_tile) * tile_dm + (d - d_tile)
// in the low word, so the largest key is the tile's largest S/N at the
// smallest t, then the smallest d (the order the tile peak kernel uses).
// keys == nullptr: no tile maxima.  The keys must be zero before the pass.
// packed != 0 (a pass that writes no planes): the low word is instead
// (kKeyPosLimit - 1 - position) << kKeyWidthBits | width index, the same
// order (a position holds one width), with the width carried in the key;
// in-tile positions must stay below kKeyPosLimit.
constexpr int kKeyWidthBits = 6;  // width indices < kMaxWidths = 64
constexpr int64_t kKeyPosLimit = int64_t(1) << (32 - kKeyWidthBits);
static_assert(kMaxWidths <= (1 << kKeyWidthBits), "width index must fit the key");
struct TileSink {
  unsigned long long *keys;  // [ntd][ntt]
  int32_t tile_dm;
  int32_t packed;
  int64_t tile_t;
  int64_t ntt;
};

// snr and best both null: no planes, tile maxima alone (sink.keys set,
// sink.packed != 0); otherwise sink.packed must be 0.
hipError_t launch_boxcar(const uint32_t *Y, int ndm, int64_t nout, const int32_t *stats,
                         const WidthList &widths, float *snr, uint8_t *best,
                         hipStream_t stream, const TileSink &sink = TileSink{});

// Tile peak record written by the first detection kernel.
struct TilePeak {
  float snr;
  int32_t d;
  int32_t t;
  int32_t w;
};
static_assert(sizeof(TilePeak) == 16, "tile peak records are copied as 16-byte units");

// Offers that the selection kernel keeps in LDS; larger offer sets (and tile
// grids larger than this) use the global arrays of the detection scratch.
constexpr int kMaxOffers = 8192;

// Detection scratch of one plane of ntiles tiles, as byte offsets from one
// base (each a multiple of 256):
//   peaks  [ntiles] TilePeak  the tile maxima
//   out    [ntiles] TilePeak  accepted offers, in candidate order
//   status [4] int32          offers, accepted, 0, 0
// and, when ntiles > kMaxOffers (offers that may not fit in LDS):
//   offer  [npow] TilePeak    offers, sorted in place (npow = ntiles rounded
//                             up to a power of two)
//   aux    [ntiles] int32     tile -> offer rank, or the accepted list
//   state  [npow] uint8       per offer: undecided, accepted, rejected
struct DetectLayout {
  int64_t peaks, out, status, offer, aux, state, bytes, npow;
};

__host__ __device__ constexpr inline DetectLayout detect_layout(int64_t ntiles) {
  auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
  DetectLayout L{};
  int64_t npow = 1;
  while (npow < ntiles) npow <<= 1;
  L.npow = npow;
  L.peaks = 0;
  L.out = up(L.peaks + 16 * ntiles);
  L.status = up(L.out + 16 * ntiles);
  int64_t end = up(L.status + 16);
  if (ntiles > kMaxOffers) {
    L.offer = end;
    L.aux = up(L.offer + 16 * npow);
    L.state = up(L.aux + 4 * ntiles);
    end = up(L.state + npow);
  } else {
    L.offer = L.aux = L.state = -1;
  }
  L.bytes = end;
  return L;
}

hipError_t launch_tile_peaks(const float *snr, const uint8_t *best, int ndm, int64_t nout,
                             int tile_dm, int64_t tile_t, TilePeak *peaks,
                             hipStream_t stream);

// Selects the tile peaks of scratch (laid out by detect_layout for the
// plane's tile count) at or above the threshold, orders them (S/N
// descending, then t, then d) and applies greedy suppression; writes the
// accepted offers in that order to the scratch's out array and to its status
// the number of offers and the number accepted.  Any number of offers.
// nms_dm and nms_t must already be clamped to ndm and nout.
hipError_t launch_select_nms(uint8_t *scratch, int ndm, int64_t nout, int tile_dm, int64_t tile_t,
                             float threshold, int nms_dm, int64_t nms_t, hipStream_t stream);

// Rt: residual table transposed, [nsub][ndm].
hipError_t launch_subband_stage2(const uint32_t *I, int64_t len1, int ncoarse, int nsub,
                                 const int32_t *Rt, int rmax, int ndm, int n0, uint32_t *Y,
                                 int64_t nout, hipStream_t stream);
hipError_t launch_zero_dm(const uint8_t *X, int64_t pitch, int64_t nsamp, int nchan, uint8_t *Xo,
                          int64_t pitch_out, hipStream_t stream);
hipError_t launch_downsample_sqrt(const uint8_t *X, int64_t pitch, int64_t nsamp, int nchan,
                                  int factor, uint8_t *Xo, int64_t pitch_out,
                                  hipStream_t stream);

// Device bytes a plan holds now: delay table, staged tables, statistics
// scratch and whatever detection / subband scratch it has grown.
int64_t plan_device_bytes(sps_plan plan);

// Records msg as the calling thread's last error (sps_last_error) and
// returns s.
sps_status set_error(sps_status s, const char *msg);

// max_nout: the longest beam's nout (picks the short-row form when every
// beam has at most 4096 outputs).
hipError_t launch_row_stats_batch(const BeamWork *beams, int nbeams, int ndm, uint32_t vmax,
                                  int64_t max_nout, hipStream_t stream);
// scratch != nullptr: every beam's tile maxima go to the key array of its
// detection scratch (the out array of detect_layout, at scratch +
// det_begin), which must be zero.
// rows_of_64: every beam's nout is a multiple of 64.  planes == false: no
// beam has S/N or width planes (snr, best null) and the keys are packed
// (TileSink::packed); needs scratch.
hipError_t launch_boxcar_batch(const BeamWork *beams, int nbeams, int64_t total_blocks,
                               const WidthList &widths, hipStream_t stream,
                               uint8_t *scratch = nullptr, int ndm = 0, int tile_dm = 1,
                               int64_t tile_t = 1, bool rows_of_64 = false, bool planes = true);
int64_t boxcar_segments(int64_t nout);

// Detector tiles taken straight from the boxcar pass: the S/N of whole
// tiles of kPoolTileDm trials x 4096 samples max-pooled over 2 trials x 8
// samples, times scale, rounded to bfloat16 (nearest even) -- the values
// the tile pooling kernels make from the S/N plane -- with no S/N or width
// plane written.  Tiles in row-major tile order, [256][512] each.
constexpr int kPoolTileDm = 512;
hipError_t launch_boxcar_pool(const uint32_t *Y, int ndm, int64_t nout, const int32_t *stats,
                              const WidthList &widths, float scale, uint16_t *tiles,
                              hipStream_t stream);
hipError_t launch_boxcar_pool_batch(const BeamWork *beams, int nbeams, int64_t total_blocks,
                                    const WidthList &widths, float scale, uint16_t *tiles,
                                    hipStream_t stream);

// Tile keys of a plane (TileSink): decode == false zeroes them; decode ==
// true turns them into the tile peak records (S/N, d, t and the width index
// best[d][t], or the key's own with packed keys, best unused) that the
// selection kernel reads, as the tile peak kernel would have written them.
hipError_t launch_tile_keys(const TileSink &sink, int ndm, int64_t nout, const uint8_t *best,
                            TilePeak *peaks, bool decode, hipStream_t stream);
// The same over every beam of a batch: keys in the out array of each beam's
// detection scratch, peaks in its peaks array.
hipError_t launch_tile_keys_batch(const BeamWork *beams, int nbeams, int ndm, int64_t total_tiles,
                                  int tile_dm, int64_t tile_t, uint8_t *scratch, bool decode,
                                  bool packed, hipStream_t stream);
// Selection and suppression of every beam of a batch from its tile peaks.
hipError_t launch_select_nms_batch(const BeamWork *beams, int nbeams, int ndm, int tile_dm,
                                   int64_t tile_t, float threshold, int nms_dm, int64_t nms_t,
                                   uint8_t *scratch, hipStream_t stream);
// Every beam's detection status and first k accepted offers in one launch:
// slot b of staging holds beam b's 4 status words (kGatherHeader bytes) and
// then k TilePeak records (nbeams * (kGatherHeader + 16 k) bytes).
constexpr int kGatherHeader = 16;
hipError_t launch_gather_candidates(const BeamWork *beams, int nbeams, int ndm, int tile_dm,
                                    const uint8_t *scratch, int k, uint8_t *staging,
                                    hipStream_t stream);

// Forward pass of n tiles (device) through net; adds to *count (device int32)
// the number of cells whose objectness probability is >= threshold, decided
// exactly as sps_cnn_detect decides it.  Asynchronous on s.
sps_status cnn_count_cells(sps_cnn net, const uint16_t *tiles, int32_t n, float threshold,
                           int32_t *count, hipStream_t s);

// Device microbenchmarks (probe.hip): rates[0..2] = sustained lane-ops/s of
// v_add_u32, v_add3_u32 and v_perm_b32; rates[3], rates[4] = LDS read
// bytes/s with 16-byte and 4-byte reads.
// Synchronous on `stream`; allocates and frees 8 MB.
hipError_t probe_device_peaks(double *rates, hipStream_t stream);

}  // namespace sps

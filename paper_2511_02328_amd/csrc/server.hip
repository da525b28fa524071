// server.hip -- native streaming runtime: many real-time filterbank streams
// searched on one GPU.
//
// Each admitted stream keeps a device ring of nchan x (O + chunk) samples:
// the last O samples of the previous chunk (the dispersion overlap of the
// time blocking in Sec. 2.3, L1 = L + R_max, here with the full channel delay:
// O = D_max rounded up to a multiple of 16) followed by the new chunk.
// Consecutive chunks therefore dedisperse into one gap-free series without
// the host resending data: chunk k's outputs are the dedispersed series at
// absolute samples [k L - O, (k + 1) L - O), the ring's overlap being zero
// before the first chunk.  A chunk travels host -> contiguous staging buffer
// (one linear DMA copy) -> ring row by row (a copy kernel); the overlap moves
// to the front of the ring with the same kernel.  Admission is by device-memory budget: a stream is refused
// when its ring, the plans of a new observing set-up and any growth of the
// shared per-worker planes do not fit.
//
// sps_server_run replays chunk arrivals on a wall-clock schedule (which may
// be compressed): stream i's chunk k becomes available at
// phase_i + (k + 1) T_i / compression, T_i the chunk's duration.  Worker
// threads take released chunks in arrival order (a stream's chunks strictly
// in sequence), each on its own HIP stream with its own output planes and
// plans: host-to-device copy into its staging buffer, then, holding the
// server's compute lock, staging -> ring, dedispersion, statistics + boxcar
// S/N, the learned detector on the S/N plane (if one is attached), overlap
// moved to the front of the ring and detection.  A chunk's latency is its completion time
// minus its arrival time.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "sps.h"
#include "sps_internal.h"

namespace {

struct SetupKey {
  std::vector<double> freq, dm;
  double fref = 0, tsamp = 0;
  bool operator==(const SetupKey &o) const {
    return freq == o.freq && dm == o.dm && fref == o.fref && tsamp == o.tsamp;
  }
};

struct StreamState {
  int setup = 0;
  int nchan = 0, ndm = 0;
  int64_t chunk = 0, overlap = 0, pitch = 0;
  uint8_t *ring = nullptr;
  std::vector<int32_t> widths;
  sps_detect_params det{};
  double duration_s = 0;
  int64_t next_chunk = 0;  // chunks searched so far
  bool busy = false;
};

struct Worker {
  hipStream_t stream = nullptr;
  uint8_t *staging = nullptr;   // contiguous [nchan][chunk] upload target
  int64_t staging_cap = 0;      // bytes
  uint32_t *Y = nullptr;
  float *snr = nullptr;
  uint8_t *best = nullptr;
  int32_t *stats = nullptr;
  int64_t cap = 0;              // elements of each plane
  int64_t stats_cap = 0;        // rows of the statistics array
  int32_t *d_cnn = nullptr;     // device count of the detector's flagged cells
  int32_t *h_cnn = nullptr;     // pinned host copy of it
  std::vector<sps_plan> plans;  // one per observing set-up
};

int64_t plane_bytes(int64_t elems, int64_t rows) {
  return elems * (int64_t)(sizeof(uint32_t) + sizeof(float) + sizeof(uint8_t)) +
         rows * 2 * (int64_t)sizeof(int32_t);
}

// Device memory of one plan: delay table, statistics, detection scratch for
// the stream's tile grid.
// Device bytes of one worker's plan: its tables (as held now) plus the
// detection scratch that its first chunk will allocate.
int64_t plan_bytes(sps_plan plan, int ndm, int64_t chunk, const sps_detect_params &det) {
  const int64_t ntiles = ((ndm + det.tile_dm - 1) / det.tile_dm) *
                         ((chunk + det.tile_t - 1) / det.tile_t);
  return sps::plan_device_bytes(plan) + sps::detect_layout(ntiles).bytes;
}

void free_planes(Worker &w) {
  if (w.Y) (void)hipFree(w.Y);
  if (w.snr) (void)hipFree(w.snr);
  if (w.best) (void)hipFree(w.best);
  if (w.stats) (void)hipFree(w.stats);
  w.Y = nullptr;
  w.snr = nullptr;
  w.best = nullptr;
  w.stats = nullptr;
  w.cap = 0;
  w.stats_cap = 0;
}

// dst[c][dst_off + i] = src[c][src_off + i] for i < len, c < nchan.  Each
// thread moves 16 bytes: one vector load and store when every row start is
// 16-byte aligned (vec), byte by byte otherwise.  Rows may overlap between
// src and dst only if dst_off + len <= src_off or src_off + len <= dst_off
// within a row (the caller splits longer moves).
__global__ __launch_bounds__(256) void copy_rows_kernel(const uint8_t *__restrict__ src,
                                                        int64_t src_pitch, int64_t src_off,
                                                        uint8_t *__restrict__ dst,
                                                        int64_t dst_pitch, int64_t dst_off,
                                                        int64_t len, int vec) {
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
  if (i >= len) return;
  const uint8_t *s = src + (int64_t)blockIdx.y * src_pitch + src_off + i;
  uint8_t *d = dst + (int64_t)blockIdx.y * dst_pitch + dst_off + i;
  if (vec && i + 16 <= len) {
    *reinterpret_cast<uint4 *>(d) = *reinterpret_cast<const uint4 *>(s);
  } else {
    const int64_t n = len - i < 16 ? len - i : 16;
    for (int64_t k = 0; k < n; ++k) d[k] = s[k];
  }
}

hipError_t copy_rows(const uint8_t *src, int64_t src_pitch, int64_t src_off, uint8_t *dst,
                     int64_t dst_pitch, int64_t dst_off, int64_t len, int nchan, hipStream_t s) {
  if (len <= 0) return hipSuccess;
  const int64_t gx = (len + 256 * 16 - 1) / (256 * 16);
  if (gx > 0x7FFFFFFF || nchan > 65535) return hipErrorInvalidValue;
  const int vec = ((((uintptr_t)src + (uint64_t)src_off) | ((uintptr_t)dst + (uint64_t)dst_off) |
                    (uint64_t)src_pitch | (uint64_t)dst_pitch) & 15u) == 0;
  hipLaunchKernelGGL(copy_rows_kernel, dim3((unsigned)gx, (unsigned)nchan), dim3(256), 0, s, src,
                     src_pitch, src_off, dst, dst_pitch, dst_off, len, vec);
  return hipGetLastError();
}

sps_status dev_fail(hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return sps::set_error(SPS_ERR_DEVICE, m.c_str());
}

}  // namespace

struct sps_server_s {
  int device = 0;
  int64_t budget = 0, used = 0;
  // One chunk's kernels at a time: the dedispersion kernel relies on the
  // workgroups resident on an XCD sharing input windows in its L2, which
  // concurrent launches from several workers would interleave away.  Uploads
  // run outside the lock, so one worker's copy overlaps another's search.
  std::mutex compute;
  // optional learned detector run on every chunk's S/N plane (under the
  // compute lock, so one network and one tile buffer serve every worker)
  sps_cnn detector = nullptr;
  float det_threshold = 0.9f, det_scale = 0.125f;
  uint16_t *tiles = nullptr;
  int64_t tiles_cap = 0;  // tiles
  std::vector<SetupKey> setups;
  std::vector<int64_t> setup_delay;  // D_max per set-up
  std::vector<StreamState> streams;
  std::vector<Worker> workers;
};

namespace {

// Grows every worker's staging buffer to hold bytes.
sps_status grow_staging(sps_server s, int64_t bytes) {
  for (Worker &w : s->workers) {
    if (w.staging_cap >= bytes) continue;
    if (w.staging) (void)hipFree(w.staging);
    w.staging = nullptr;
    w.staging_cap = 0;
    if (hipMalloc(&w.staging, (size_t)bytes) != hipSuccess) {
      (void)hipGetLastError();
      return sps::set_error(SPS_ERR_NOMEM, "device allocation of a staging buffer failed");
    }
    w.staging_cap = bytes;
  }
  return SPS_OK;
}

// Grows every worker's planes to hold elems samples and rows statistics.
sps_status grow_planes(sps_server s, int64_t elems, int64_t rows) {
  for (Worker &w : s->workers) {
    if (w.cap >= elems && w.stats_cap >= rows) continue;
    const int64_t ne = std::max(w.cap, elems), nr = std::max(w.stats_cap, rows);
    free_planes(w);
    hipError_t e = hipMalloc(&w.Y, sizeof(uint32_t) * (size_t)ne);
    if (e == hipSuccess) e = hipMalloc(&w.snr, sizeof(float) * (size_t)ne);
    if (e == hipSuccess) e = hipMalloc(&w.best, (size_t)ne);
    if (e == hipSuccess) e = hipMalloc(&w.stats, sizeof(int32_t) * 2 * (size_t)nr);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      free_planes(w);
      return sps::set_error(SPS_ERR_NOMEM, "device allocation of worker planes failed");
    }
    w.cap = ne;
    w.stats_cap = nr;
  }
  return SPS_OK;
}

constexpr int64_t kTileBytes = 256 * 512 * 2;  // one bfloat16 detector tile

int64_t grid_tiles(int ndm, int64_t chunk) { return (int64_t)(ndm / 512) * (chunk / 4096); }

// Grows the shared detector tile buffer to hold n tiles.
sps_status grow_tiles(sps_server s, int64_t n) {
  if (s->tiles_cap >= n) return SPS_OK;
  if (s->tiles) (void)hipFree(s->tiles);
  s->tiles = nullptr;
  s->tiles_cap = 0;
  if (hipMalloc(&s->tiles, (size_t)(n * kTileBytes)) != hipSuccess) {
    (void)hipGetLastError();
    return sps::set_error(SPS_ERR_NOMEM, "device allocation of detector tiles failed");
  }
  s->tiles_cap = n;
  return SPS_OK;
}

// Runs the attached detector on the S/N plane of worker w: the plane cut
// into whole tiles, the network over them in batches, the cells at or above
// the threshold counted on the device and the count copied to w.h_cnn.
// Asynchronous on the worker's stream: no host round trip per batch.
sps_status run_detector(sps_server s, Worker &w, const StreamState &st) {
  hipError_t e = hipMemsetAsync(w.d_cnn, 0, sizeof(int32_t), w.stream);
  if (e != hipSuccess) return dev_fail(e, "detector count reset");
  int64_t nt = 0;
  sps_status r = sps_cnn_pool_tile_grid(w.snr, st.chunk, st.ndm, st.chunk, s->det_scale, s->tiles,
                                        &nt, w.stream);
  if (r != SPS_OK) return r;
  const int32_t mb = sps_cnn_max_batch(s->detector);
  for (int64_t b0 = 0; b0 < nt; b0 += mb) {
    const int32_t nb = (int32_t)(nt - b0 < mb ? nt - b0 : mb);
    r = sps::cnn_count_cells(s->detector, s->tiles + b0 * (kTileBytes / 2), nb, s->det_threshold,
                             w.d_cnn, w.stream);
    if (r != SPS_OK) return r;
  }
  e = hipMemcpyAsync(w.h_cnn, w.d_cnn, sizeof(int32_t), hipMemcpyDeviceToHost, w.stream);
  if (e != hipSuccess) return dev_fail(e, "detector count copy");
  return SPS_OK;
}

// Searches the next chunk of stream sid on worker w.  src: host
// [nchan][src_pitch].  Y_copy (optional, device [ndm][chunk]) receives the
// dedispersed plane; out/cap/n_found as in sps_detect; n_cnn receives the
// attached detector's count (0 without one).  Synchronises the worker's
// stream.
// Wall-clock marks of one chunk's phases (seconds on the caller's clock).
struct Marks {
  std::chrono::steady_clock::time_point uploaded, locked;
};

sps_status process_chunk(sps_server s, Worker &w, int sid, const uint8_t *src, int64_t src_pitch,
                         uint32_t *Y_copy, sps_candidate *out, int32_t cap, int32_t *n_found,
                         int32_t *n_cnn, Marks *marks = nullptr) {
  StreamState &st = s->streams[(size_t)sid];
  sps_plan plan = w.plans[(size_t)st.setup];
  hipStream_t hs = w.stream;
  *n_found = 0;
  *n_cnn = 0;
  const int64_t bytes = st.chunk * (int64_t)st.nchan;
  if (bytes > w.staging_cap) return sps::set_error(SPS_ERR_RANGE, "chunk exceeds the staging buffer");
  // Upload to the contiguous staging buffer: one linear copy (a DMA engine,
  // no compute units) when the host rows are back to back.
  hipError_t e = src_pitch == st.chunk
                     ? hipMemcpyAsync(w.staging, src, (size_t)bytes, hipMemcpyHostToDevice, hs)
                     : hipMemcpy2DAsync(w.staging, (size_t)st.chunk, src, (size_t)src_pitch,
                                        (size_t)st.chunk, (size_t)st.nchan,
                                        hipMemcpyHostToDevice, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) return dev_fail(e, "chunk upload");
  if (marks) marks->uploaded = std::chrono::steady_clock::now();
  std::lock_guard<std::mutex> lk(s->compute);
  if (marks) marks->locked = std::chrono::steady_clock::now();
  e = copy_rows(w.staging, st.chunk, 0, st.ring, st.pitch, st.overlap, st.chunk, st.nchan, hs);
  if (e != hipSuccess) return dev_fail(e, "ring fill");
  sps_status r =
      sps_dedisperse(plan, st.ring, st.pitch, st.overlap + st.chunk, w.Y, st.chunk, 0, hs);
  if (r != SPS_OK) return r;
  if (Y_copy) {
    e = hipMemcpyAsync(Y_copy, w.Y, sizeof(uint32_t) * (size_t)st.ndm * (size_t)st.chunk,
                       hipMemcpyDeviceToDevice, hs);
    if (e != hipSuccess) return dev_fail(e, "plane copy");
  }
  // The last D_max samples move to the front of the ring, in pieces no
  // longer than the chunk, so that no piece's source overlaps its
  // destination; in stream order every piece reads its source before a
  // later piece overwrites it.  The search below reads only the plane.
  for (int64_t off = 0; off < st.overlap; off += st.chunk) {
    const int64_t len = std::min(st.chunk, st.overlap - off);
    e = copy_rows(st.ring, st.pitch, st.chunk + off, st.ring, st.pitch, off, len, st.nchan, hs);
    if (e != hipSuccess) return dev_fail(e, "overlap move");
  }
  // Statistics, boxcar and detection in one call, the tile maxima gathered
  // by the boxcar pass.  Without the learned detector (which reads the S/N
  // plane) no plane is written, where the tiles fit the packed keys.
  const bool learned = s->detector != nullptr;
  const int64_t tdm = std::min<int64_t>(st.det.tile_dm, st.ndm);
  const int64_t tt = std::min<int64_t>(st.det.tile_t, st.chunk);
  const bool planes = learned || tdm * tt > sps::kKeyPosLimit;
  r = sps_search(plan, w.Y, st.chunk, st.widths.data(), (int32_t)st.widths.size(),
                 planes ? w.snr : nullptr, planes ? w.best : nullptr, w.stats, &st.det, out, cap,
                 n_found, hs);
  if (learned && (r == SPS_OK || r == SPS_ERR_TRUNCATED)) {
    const sps_status rd = run_detector(s, w, st);
    if (rd != SPS_OK) return rd;
    e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return dev_fail(e, "detector count");
    *n_cnn = *w.h_cnn;
  }
  return r;
}

}  // namespace

extern "C" {

sps_status sps_server_create(int64_t hbm_budget, int32_t nworkers, sps_server *out) {
  if (!out) return sps::set_error(SPS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (hbm_budget <= 0 || nworkers < 1 || nworkers > 16)
    return sps::set_error(SPS_ERR_INVALID_ARG, "need hbm_budget > 0 and 1 <= nworkers <= 16");
  sps_server s = new (std::nothrow) sps_server_s;
  if (!s) return sps::set_error(SPS_ERR_NOMEM, "host allocation failed");
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) {
    delete s;
    return dev_fail(e, "hipGetDevice");
  }
  s->budget = hbm_budget;
  s->workers.resize((size_t)nworkers);
  for (Worker &w : s->workers) {
    e = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&w.d_cnn, sizeof(int32_t));
    if (e == hipSuccess) e = hipHostMalloc(&w.h_cnn, sizeof(int32_t), hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)sps_server_destroy(s);
      return dev_fail(e, "worker set-up");
    }
  }
  *out = s;
  return SPS_OK;
}

sps_status sps_server_destroy(sps_server s) {
  if (!s) return SPS_OK;
  for (Worker &w : s->workers)
    if (w.stream) (void)hipStreamSynchronize(w.stream);
  for (Worker &w : s->workers) {
    for (sps_plan p : w.plans) sps_plan_destroy(p);
    free_planes(w);
    if (w.staging) (void)hipFree(w.staging);
    if (w.d_cnn) (void)hipFree(w.d_cnn);
    if (w.h_cnn) (void)hipHostFree(w.h_cnn);
    if (w.stream) (void)hipStreamDestroy(w.stream);
  }
  for (StreamState &st : s->streams)
    if (st.ring) (void)hipFree(st.ring);
  if (s->tiles) (void)hipFree(s->tiles);
  delete s;
  return SPS_OK;
}

sps_status sps_server_set_detector(sps_server s, sps_cnn net, float threshold, float scale) {
  if (!s) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL server");
  if (net && (!(threshold > 0.0f && threshold < 1.0f) || !(scale > 0.0f)))
    return sps::set_error(SPS_ERR_INVALID_ARG, "need 0 < threshold < 1 and scale > 0");
  if (net) {
    int64_t need = 0;
    for (const StreamState &st : s->streams) need = std::max(need, grid_tiles(st.ndm, st.chunk));
    const int64_t grow = std::max<int64_t>(0, need - s->tiles_cap) * kTileBytes;
    if (s->used + grow > s->budget)
      return sps::set_error(SPS_ERR_NOMEM, "refused: detector tiles do not fit the budget");
    const sps_status r = grow_tiles(s, need);
    if (r != SPS_OK) return r;
    s->used += grow;
  }
  s->detector = net;
  s->det_threshold = threshold;
  s->det_scale = scale;
  return SPS_OK;
}

sps_status sps_server_add_stream(sps_server s, const sps_obs_desc *desc, const int32_t *widths,
                                 int32_t nw, const sps_detect_params *det, int64_t chunk_len,
                                 int32_t *stream_id) {
  if (!s || !desc || !widths || !det || !stream_id)
    return sps::set_error(SPS_ERR_INVALID_ARG, "NULL argument");
  *stream_id = -1;
  // Everything the chunk's boxcar and detection calls would check, so that
  // an admitted stream never fails on its first chunk for its parameters.
  if (nw < 1 || nw > sps::kMaxWidths)
    return sps::set_error(SPS_ERR_INVALID_ARG, "bad width count");
  for (int i = 0; i < nw; ++i)
    if (widths[i] < 1 || (i > 0 && widths[i] <= widths[i - 1]))
      return sps::set_error(SPS_ERR_INVALID_ARG, "widths must be >= 1 and strictly ascending");
  if (widths[nw - 1] > sps::kMaxWidth)
    return sps::set_error(SPS_ERR_RANGE, "largest width above the supported maximum");
  if (chunk_len < widths[nw - 1] || chunk_len > 0x7FFFFFFF)
    return sps::set_error(SPS_ERR_INVALID_ARG, "chunk length must be in [largest width, 2^31-1]");
  if (!(det->threshold > 0.0f) || !isfinite(det->threshold) || det->tile_dm < 1 ||
      det->tile_t < 1 || det->nms_dm < 0 || det->nms_t < 0)
    return sps::set_error(SPS_ERR_INVALID_ARG, "bad detection parameters");
  if ((uint64_t)det->tile_dm * (uint64_t)det->tile_t >= (1ull << 32))
    return sps::set_error(SPS_ERR_RANGE, "tile_dm * tile_t must be below 2^32");
  if (!desc->freq_mhz || !desc->dm || desc->nchan < 1 || desc->ndm < 1)
    return sps::set_error(SPS_ERR_INVALID_ARG, "bad observing description");
  if ((uint64_t)widths[nw - 1] * 255u * (uint64_t)desc->nchan >= (1ull << 31))
    return sps::set_error(SPS_ERR_OVERFLOW, "largest width x 255 x nchan reaches 2^31");
  if (((int64_t)desc->ndm + det->tile_dm - 1) / det->tile_dm *
          ((chunk_len + det->tile_t - 1) / det->tile_t) > 0x7FFFFFFF)
    return sps::set_error(SPS_ERR_RANGE, "too many detection tiles");
  SetupKey key;
  key.freq.assign(desc->freq_mhz, desc->freq_mhz + desc->nchan);
  key.dm.assign(desc->dm, desc->dm + desc->ndm);
  key.fref = desc->fref_mhz;
  key.tsamp = desc->tsamp_s;
  int setup = -1;
  for (size_t i = 0; i < s->setups.size(); ++i)
    if (s->setups[i] == key) setup = (int)i;
  const bool new_setup = setup < 0;
  // Plans of a new set-up (one per worker) validate the description and
  // give D_max.
  int64_t dmax = 0;
  std::vector<sps_plan> new_plans;
  auto drop = [&]() {
    for (sps_plan q : new_plans) sps_plan_destroy(q);
    new_plans.clear();
  };
  if (new_setup) {
    for (size_t wi = 0; wi < s->workers.size(); ++wi) {
      sps_plan p = nullptr;
      const sps_status r = sps_plan_create(desc, &p);
      if (r != SPS_OK) {
        drop();
        return r;  // sps_plan_create recorded the message
      }
      new_plans.push_back(p);
    }
    int32_t mx = 0;
    sps_plan_delays(new_plans[0], nullptr, &mx);
    dmax = mx;
  } else {
    dmax = s->setup_delay[(size_t)setup];
  }
  // The overlap keeps D_max samples rounded up to 16, so that the chunk's
  // region of every ring row starts 16-byte aligned.
  const int64_t overlap = (dmax + 15) / 16 * 16;
  const int64_t pitch = (overlap + chunk_len + 255) / 256 * 256;
  const int64_t ring = pitch * desc->nchan;
  const int64_t elems = (int64_t)desc->ndm * chunk_len;
  const int64_t stage = chunk_len * (int64_t)desc->nchan;
  int64_t grow = 0;
  for (const Worker &w : s->workers)
    grow += plane_bytes(std::max(w.cap, elems), std::max<int64_t>(w.stats_cap, desc->ndm)) -
            plane_bytes(w.cap, w.stats_cap) + std::max<int64_t>(0, stage - w.staging_cap);
  int64_t plans = 0;
  for (sps_plan q : new_plans) plans += plan_bytes(q, desc->ndm, chunk_len, *det);
  const int64_t tile_grow =
      s->detector ? std::max<int64_t>(0, grid_tiles(desc->ndm, chunk_len) - s->tiles_cap) * kTileBytes
                  : 0;
  const int64_t need = ring + grow + plans + tile_grow;
  if (s->used + need > s->budget) {
    drop();
    char m[192];
    snprintf(m, sizeof m, "refused: the stream needs %lld bytes, %lld of %lld are in use",
             (long long)need, (long long)s->used, (long long)s->budget);
    return sps::set_error(SPS_ERR_NOMEM, m);
  }
  sps_status r = grow_planes(s, elems, desc->ndm);
  if (r == SPS_OK) r = grow_staging(s, stage);
  if (r == SPS_OK && s->detector) r = grow_tiles(s, grid_tiles(desc->ndm, chunk_len));
  if (r != SPS_OK) {
    drop();
    return r;
  }
  StreamState st;
  hipError_t e = hipMalloc(&st.ring, (size_t)ring);
  if (e == hipSuccess) e = hipMemset(st.ring, 0, (size_t)ring);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (st.ring) (void)hipFree(st.ring);
    drop();
    return sps::set_error(SPS_ERR_NOMEM, "device allocation of the stream ring failed");
  }
  if (new_setup) {
    setup = (int)s->setups.size();
    s->setups.push_back(key);
    s->setup_delay.push_back(dmax);
    for (size_t wi = 0; wi < s->workers.size(); ++wi)
      s->workers[wi].plans.push_back(new_plans[wi]);
  }
  st.setup = setup;
  st.nchan = desc->nchan;
  st.ndm = desc->ndm;
  st.chunk = chunk_len;
  st.overlap = overlap;
  st.pitch = pitch;
  st.widths.assign(widths, widths + nw);
  st.det = *det;
  st.duration_s = (double)chunk_len * desc->tsamp_s;
  s->used += need;
  s->streams.push_back(std::move(st));
  *stream_id = (int32_t)s->streams.size() - 1;
  return SPS_OK;
}

sps_status sps_server_memory(sps_server s, int64_t *used, int64_t *budget) {
  if (!s) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL server");
  if (used) *used = s->used;
  if (budget) *budget = s->budget;
  return SPS_OK;
}

sps_status sps_server_stream_info(sps_server s, int32_t stream_id, int64_t *chunk_len,
                                  int64_t *overlap, double *duration_s) {
  if (!s || stream_id < 0 || stream_id >= (int32_t)s->streams.size())
    return sps::set_error(SPS_ERR_INVALID_ARG, "bad server or stream id");
  const StreamState &st = s->streams[(size_t)stream_id];
  if (chunk_len) *chunk_len = st.chunk;
  if (overlap) *overlap = st.overlap;
  if (duration_s) *duration_s = st.duration_s;
  return SPS_OK;
}

sps_status sps_server_push(sps_server s, int32_t stream_id, const uint8_t *host, int64_t src_pitch,
                           uint32_t *Y_copy, sps_candidate *out, int32_t cap, int32_t *n_found,
                           int32_t *n_cnn) {
  if (!s || !host || !n_found) return sps::set_error(SPS_ERR_INVALID_ARG, "NULL argument");
  if (stream_id < 0 || stream_id >= (int32_t)s->streams.size())
    return sps::set_error(SPS_ERR_INVALID_ARG, "bad stream id");
  StreamState &st = s->streams[(size_t)stream_id];
  if (src_pitch < st.chunk) return sps::set_error(SPS_ERR_INVALID_ARG, "src_pitch < chunk length");
  if (cap < 0 || (cap > 0 && !out)) return sps::set_error(SPS_ERR_INVALID_ARG, "bad output array");
  hipError_t e = hipSetDevice(s->device);
  if (e != hipSuccess) return dev_fail(e, "hipSetDevice");
  int32_t ncnn = 0;
  const sps_status r = process_chunk(s, s->workers[0], stream_id, host, src_pitch, Y_copy, out,
                                     cap, n_found, &ncnn);
  if (n_cnn) *n_cnn = ncnn;
  if (r == SPS_OK || r == SPS_ERR_TRUNCATED) st.next_chunk += 1;
  return r;
}

sps_status sps_server_run(sps_server s, const sps_feed *feeds, double run_s, double compression,
                          sps_chunk_record *records, int32_t cap, int32_t *n_records) {
  if (!s || !feeds || !n_records || cap < 0 || (cap > 0 && !records))
    return sps::set_error(SPS_ERR_INVALID_ARG, "NULL argument or bad record array");
  *n_records = 0;
  if (!(run_s > 0) || !(compression > 0))
    return sps::set_error(SPS_ERR_INVALID_ARG, "run time and compression must be positive");
  const int ns = (int)s->streams.size();
  if (ns == 0) return sps::set_error(SPS_ERR_INVALID_ARG, "no streams admitted");
  for (int i = 0; i < ns; ++i)
    if (!feeds[i].host || feeds[i].nsrc < 1 || feeds[i].first < 0 ||
        feeds[i].src_pitch < s->streams[(size_t)i].chunk)
      return sps::set_error(SPS_ERR_INVALID_ARG, "bad feed");
  hipError_t he = hipSetDevice(s->device);
  if (he != hipSuccess) return dev_fail(he, "hipSetDevice");

  // Arrival schedule: stream i's chunk k is complete at phase_i + (k + 1) T_i.
  struct Arrival {
    double t;
    int stream;
    int64_t index;
  };
  std::vector<Arrival> sched;
  for (int i = 0; i < ns; ++i) {
    const double T = s->streams[(size_t)i].duration_s / compression;
    const double phase = T * (double)i / (double)ns;
    for (int64_t k = 0;; ++k) {
      const double t = phase + (double)(k + 1) * T;
      if (t > run_s) break;
      sched.push_back({t, i, k});
    }
  }
  std::sort(sched.begin(), sched.end(), [](const Arrival &a, const Arrival &b) {
    return a.t < b.t || (a.t == b.t && a.stream < b.stream);
  });
  std::vector<int64_t> base((size_t)ns);
  for (int i = 0; i < ns; ++i) base[(size_t)i] = s->streams[(size_t)i].next_chunk;

  std::mutex mu;
  std::condition_variable cv;
  std::deque<Arrival> queue;
  bool done_releasing = false;
  sps_status err = SPS_OK;
  std::string err_msg;
  std::vector<sps_chunk_record> recs;
  recs.reserve(sched.size());
  const auto t0 = std::chrono::steady_clock::now();
  auto now_s = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };

  auto worker_fn = [&](int wi) {
    (void)hipSetDevice(s->device);
    Worker &w = s->workers[(size_t)wi];
    for (;;) {
      Arrival job{};
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (err != SPS_OK) return;
          auto it = std::find_if(queue.begin(), queue.end(), [&](const Arrival &a) {
            const StreamState &st = s->streams[(size_t)a.stream];
            return !st.busy && st.next_chunk == base[(size_t)a.stream] + a.index;
          });
          if (it != queue.end()) {
            job = *it;
            queue.erase(it);
            s->streams[(size_t)job.stream].busy = true;
            break;
          }
          if (done_releasing && queue.empty()) return;
          cv.wait(lk);
        }
      }
      const double start = now_s();
      const sps_feed &f = feeds[job.stream];
      const StreamState &st = s->streams[(size_t)job.stream];
      const int64_t src_idx = (f.first + job.index) % f.nsrc;
      const uint8_t *src = f.host + (size_t)src_idx * (size_t)st.nchan * (size_t)f.src_pitch;
      int32_t nc = 0, ncnn = 0;
      Marks mk;
      mk.uploaded = mk.locked = std::chrono::steady_clock::now();
      sps_status r = process_chunk(s, w, job.stream, src, f.src_pitch, nullptr, nullptr, 0, &nc,
                                   &ncnn, &mk);
      if (r == SPS_ERR_TRUNCATED) r = SPS_OK;  // only the count is kept
      const double end = now_s();
      const double up = std::chrono::duration<double>(mk.uploaded - t0).count();
      const double lk_s = std::chrono::duration<double>(mk.locked - t0).count();
      {
        std::lock_guard<std::mutex> lk(mu);
        StreamState &sm = s->streams[(size_t)job.stream];
        sm.busy = false;
        sm.next_chunk += 1;
        // a device or memory failure stops the run; any other failure stays
        // in the chunk's record and the run goes on
        if ((r == SPS_ERR_DEVICE || r == SPS_ERR_NOMEM) && err == SPS_OK) {
          err = r;
          err_msg = sps_last_error();
        }
        recs.push_back({job.stream, wi, job.index, job.t, start, up, lk_s, end, nc, (int32_t)r,
                        ncnn, 0});
      }
      cv.notify_all();
    }
  };

  std::vector<std::thread> threads;
  for (size_t wi = 0; wi < s->workers.size(); ++wi) threads.emplace_back(worker_fn, (int)wi);
  for (const Arrival &a : sched) {
    const double wait = a.t - now_s();
    if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
    std::lock_guard<std::mutex> lk(mu);
    if (err != SPS_OK) break;
    queue.push_back(a);
    cv.notify_all();
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    done_releasing = true;
  }
  cv.notify_all();
  for (std::thread &t : threads) t.join();
  std::sort(recs.begin(), recs.end(), [](const sps_chunk_record &a, const sps_chunk_record &b) {
    return a.arrival_s < b.arrival_s || (a.arrival_s == b.arrival_s && a.stream < b.stream);
  });
  const size_t n = std::min(recs.size(), (size_t)cap);
  if (n > 0) memcpy(records, recs.data(), sizeof(sps_chunk_record) * n);
  *n_records = (int32_t)recs.size();
  if (err != SPS_OK) return sps::set_error(err, err_msg.c_str());
  if (recs.size() > (size_t)cap) return sps::set_error(SPS_ERR_TRUNCATED, "record array too small");
  return SPS_OK;
}

}  // extern "C"

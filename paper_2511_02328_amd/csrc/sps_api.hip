// sps_api.hip -- the C ABI (include/sps.h): plans, argument checks, launches.
//
// Host-side work is limited to what the ABI promises: the integer delay table
// of Eq. (KDM) / Eq. (coarse_delay) (ASTROFLOW Sec. 2.3), computed once per
// plan in IEEE double and uploaded, argument validation before anything is
// enqueued, and turning the detection kernels' output into candidate
// records.  Every step of the search itself runs in the HIP kernels.
#include <algorithm>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sps.h"
#include "sps_internal.h"

namespace {

thread_local std::string g_error;

sps_status fail(sps_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
sps_status fail(sps_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

sps_status hip_fail(hipError_t e, const char *what) {
  return fail(SPS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Dispersion constant of Eq. (KDM) in s MHz^2 pc^-1 cm^3 (the printed unit,
// ms, would make delays a thousand times too small).
constexpr double kKdm = 4.148808e3;

// Makes the plan's device current for the duration of a call.
struct DeviceScope {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

namespace sps {
sps_status set_error(sps_status s, const char *msg) { return fail(s, "%s", msg); }
}  // namespace sps

struct sps_plan_s {
  int device = 0;
  int nchan = 0, ndm = 0;
  double fref_mhz = 0, tsamp_s = 0;
  std::vector<double> freq, dm;
  std::vector<int32_t> delays;
  int32_t max_delay = 0;
  int32_t *d_delays = nullptr;
  int32_t *d_stats = nullptr;  // [ndm][2] used when the caller passes none
  sps::DedispConfig cfg{5, 1, 16, 16, 2, 8};
  int lds_pitch = 0;
  sps::StagedDelays staged;  // d_delays in the form the tiling cfg reads
  // subband method (sps_subband_plan_create)
  bool subband = false;
  int n0 = 0, nsub = 0, ncoarse = 0;
  std::vector<int32_t> sub;            // [nsub + 1] channel boundaries
  std::vector<double> fsub;            // representative frequencies
  std::vector<int32_t> coarse_delays;  // [ncoarse][nchan]
  std::vector<int32_t> residuals;      // [ndm][nsub]
  int32_t rmax = 0, eff_max_delay = 0;
  std::vector<int32_t *> d_coarse_sub;  // per subband: [ncoarse][channels of s]
  std::vector<sps::DedispConfig> sub_cfg;
  std::vector<int> sub_pitch;
  std::vector<sps::StagedDelays> sub_staged;
  // stage 1 in one launch over all channels (equal subbands that are a
  // multiple of the tiling's slab): the whole coarse table and its tiling
  bool fused = false;      // the one-launch form exists
  bool use_fused = true;   // and is used (sps_plan_autotune may switch it off)
  sps::DedispConfig fused_cfg{0, 0, 0, 0, 0, 0};
  int fused_pitch = 0;
  int32_t *d_coarse_full = nullptr;
  sps::StagedDelays fused_staged;
  int32_t *d_resid = nullptr;  // residuals transposed, [nsub][ndm]
  uint32_t *d_I = nullptr;
  size_t I_bytes = 0;
  // detection scratch (sps::detect_layout of the last plane's tile count)
  uint8_t *d_det = nullptr;
  int64_t det_bytes = 0;
};

namespace {

void free_plan(sps_plan p) {
  if (!p) return;
  if (p->d_delays) (void)hipFree(p->d_delays);
  if (p->d_stats) (void)hipFree(p->d_stats);
  if (p->d_det) (void)hipFree(p->d_det);
  for (int32_t *q : p->d_coarse_sub)
    if (q) (void)hipFree(q);
  if (p->d_resid) (void)hipFree(p->d_resid);
  if (p->d_I) (void)hipFree(p->d_I);
  if (p->d_coarse_full) (void)hipFree(p->d_coarse_full);
  sps::free_staged(p->staged);
  for (sps::StagedDelays &q : p->sub_staged) sps::free_staged(q);
  sps::free_staged(p->fused_staged);
  delete p;
}

// Compiled tilings in order of preference (see dedisperse.hip).
const sps::DedispConfig kPrefs[] = {
    {5, 1, 16, 16, 2, 8}, {5, 1, 16, 16, 2, 4}, {5, 1, 16, 16, 4, 4}, {3, 1, 16, 16, 2, 8},
    {7, 1, 16, 16, 3, 4}, {5, 1, 8, 8, 5, 4},   {5, 1, 8, 8, 8, 4}};

// Staged-row bytes of config c for a delay table, or -1 if it does not fit.
int64_t fitted_pitch(const int32_t *D, int nchan, int ndm, const sps::DedispConfig &c,
                     int64_t lds_budget) {
  const int spread = sps::dedisp_block_spread(D, nchan, ndm, c.nd());
  const int64_t pitch = sps::dedisp_lds_pitch(c, spread);
  if (pitch > 1024 * (int64_t)c.kmax || c.lds_bytes(pitch) > lds_budget) return -1;
  return pitch;
}

int64_t fitted_pitch(sps_plan p, const sps::DedispConfig &c, int64_t lds_budget) {
  return fitted_pitch(p->delays.data(), p->nchan, p->ndm, c, lds_budget);
}

// Picks the first preferred tiling whose double-buffered slab fits the LDS
// budget (64 KiB keeps two workgroups per CU; up to 160 KiB is allowed
// next); otherwise the plain global-memory kernel (m = 0) is used.
// seg > 0 restricts the choice to slabs that divide seg (segmented output)
// and to the 4-waves-per-SIMD tilings, whose register budget holds the
// segment stores without spilling.
void pick_tiling(const int32_t *D, int nchan, int ndm, sps::DedispConfig *cfg, int *pitch,
                 int seg = 0) {
  for (int64_t budget : {(int64_t)64 * 1024, (int64_t)160 * 1024}) {
    for (const auto &c : kPrefs) {
      if (seg > 0 && (seg % c.cs != 0 || c.wpe != 4)) continue;
      const int64_t pp = fitted_pitch(D, nchan, ndm, c, budget);
      if (pp > 0) {
        *cfg = c;
        *pitch = (int)pp;
        return;
      }
    }
  }
  *cfg = sps::DedispConfig{0, 0, 0, 0, 0, 0};
  *pitch = 0;
}

sps_status choose_tiling(sps_plan p) {
  pick_tiling(p->delays.data(), p->nchan, p->ndm, &p->cfg, &p->lds_pitch);
  return SPS_OK;
}

// Rebuilds the staged delay table for the plan's current tiling.
sps_status restage(sps_plan p) {
  DeviceScope scope(p->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  const hipError_t e =
      sps::stage_delays(p->staged, p->cfg, p->lds_pitch, p->d_delays, p->nchan, p->ndm,
                        p->max_delay);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    return fail(SPS_ERR_NOMEM, "device allocation of the staged delay table failed");
  }
  if (e != hipSuccess) return hip_fail(e, "staging the delay table");
  return SPS_OK;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// A tile peak record as a candidate (Sec. 2): DM, TOA at the top of the band
// (the window's centre), width and S/N.
sps_candidate to_candidate(const sps::TilePeak &q, const int32_t *widths, int nw,
                           const double *dm, int ndm, double tsamp_s) {
  sps_candidate c;
  c.dm_idx = q.d;
  c.t_idx = q.t;
  c.width = (q.w >= 0 && q.w < nw) ? widths[q.w] : 0;
  c.snr = q.snr;
  c.reserved = 0.0f;
  c.dm = (q.d >= 0 && q.d < ndm) ? dm[q.d] : 0.0;
  c.toa_s = ((double)q.t + 0.5 * (double)c.width) * tsamp_s;
  return c;
}

// Reads the result of the selection kernel from a plane's detection scratch
// (d_scratch, laid out by sps::detect_layout(ntiles)) and converts the first
// min(n, cap) accepted offers into candidate records (Sec. 2: DM, TOA at the
// top of the band, width, S/N).  Synchronises the stream.  Allocates nothing:
// the records pass through a fixed host buffer.
sps_status read_candidates(const uint8_t *d_scratch, int64_t ntiles, const int32_t *widths,
                           int nw, const double *dm, int ndm, double tsamp_s, sps_candidate *out,
                           int32_t cap, int32_t *n_found, hipStream_t s) {
  const sps::DetectLayout L = sps::detect_layout(ntiles);
  int32_t status[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(status, d_scratch + L.status, sizeof status, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading detection status");
  const int32_t na = status[1];
  if (na < 0 || (int64_t)na > ntiles || status[0] < na) {
    *n_found = 0;
    return fail(SPS_ERR_DEVICE, "detection status is inconsistent (%d offers, %d accepted, %lld tiles)",
                status[0], na, (long long)ntiles);
  }
  const int32_t ncopy = na < cap ? na : cap;
  constexpr int kChunk = 256;
  sps::TilePeak buf[kChunk];
  const sps::TilePeak *src = reinterpret_cast<const sps::TilePeak *>(d_scratch + L.out);
  for (int32_t i0 = 0; i0 < ncopy; i0 += kChunk) {
    const int32_t m = ncopy - i0 < kChunk ? ncopy - i0 : kChunk;
    e = hipMemcpyAsync(buf, src + i0, sizeof(sps::TilePeak) * (size_t)m, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading candidates");
    for (int32_t k = 0; k < m; ++k)
      out[i0 + k] = to_candidate(buf[k], widths, nw, dm, ndm, tsamp_s);
  }
  *n_found = na;
  if (na > cap) return fail(SPS_ERR_TRUNCATED, "%d candidates found, %d returned", na, cap);
  return SPS_OK;
}

// Fixed detection scratch of sps_detect_noalloc: one copy on every device
// the library runs on, held until the process ends.  Host code never uses
// the array's name as an address: on each device, with that device current,
// the first call looks up the device address of that device's copy once and
// keeps it in g_fixed_scratch.  Calls that overlap on one device share the
// copy and race.  Every byte a call reads is first written by its own
// kernels (tile peaks, status, and the tile map and states the selection
// kernel clears), so nothing carries over between calls.
constexpr int64_t kFixedScratchBytes = 4ll << 20;
constexpr int64_t kFixedScratchTiles = 65536;
static_assert(sps::detect_layout(kFixedScratchTiles).bytes <= kFixedScratchBytes,
              "the fixed detection scratch must hold the stated tile count");
static __device__ __align__(256) uint8_t scratch[kFixedScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
uint8_t *g_fixed_scratch[kMaxDevices] = {};

// Device address of the current device's copy of the fixed scratch.
sps_status fixed_scratch(int device, uint8_t **ptr) {
  if (device < 0 || device >= kMaxDevices)
    return fail(SPS_ERR_DEVICE, "device %d is beyond the %d the fixed scratch serves", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_fixed_mu);
  if (!g_fixed_scratch[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "looking up the fixed detection scratch");
    g_fixed_scratch[device] = static_cast<uint8_t *>(p);
  }
  *ptr = g_fixed_scratch[device];
  return SPS_OK;
}

// Checks shared by the calls that detect candidates; fills the tile count,
// the scratch layout and the suppression radii clamped to the plane.
struct DetectArgs {
  int64_t ntiles = 0, ntt = 0;
  int32_t nms_dm = 0;
  int64_t nms_t = 0;
  sps::DetectLayout L{};
};

sps_status check_detect(sps_plan plan, int64_t nout, int32_t nw, const sps_detect_params *prm,
                        sps_candidate *out, int32_t cap, const int32_t *n_found, DetectArgs *a) {
  if (!prm || !n_found) return fail(SPS_ERR_INVALID_ARG, "NULL parameter or count");
  if (cap < 0 || (cap > 0 && !out)) return fail(SPS_ERR_INVALID_ARG, "bad output array");
  if (nout < 1 || nout > 0x7FFFFFFF) return fail(SPS_ERR_RANGE, "nout must be in [1, 2^31-1]");
  if (nw < 1 || nw > sps::kMaxWidths) return fail(SPS_ERR_INVALID_ARG, "bad width count");
  if (!(prm->threshold > 0.0f) || !isfinite(prm->threshold))
    return fail(SPS_ERR_INVALID_ARG, "threshold must be positive");
  if (prm->tile_dm < 1 || prm->tile_t < 1 || prm->nms_dm < 0 || prm->nms_t < 0)
    return fail(SPS_ERR_INVALID_ARG, "bad tile or suppression sizes");
  if ((uint64_t)prm->tile_dm * (uint64_t)prm->tile_t >= (1ull << 32))
    return fail(SPS_ERR_RANGE, "tile_dm * tile_t must be below 2^32");
  const int64_t ntd = (plan->ndm + prm->tile_dm - 1) / prm->tile_dm;
  a->ntt = (nout + prm->tile_t - 1) / prm->tile_t;
  a->ntiles = ntd * a->ntt;
  if (a->ntiles > 0x7FFFFFFF) return fail(SPS_ERR_RANGE, "too many tiles");
  a->L = sps::detect_layout(a->ntiles);
  // radii past the plane's extent suppress the same offers as the extent
  a->nms_dm = prm->nms_dm < plan->ndm ? prm->nms_dm : plan->ndm;
  a->nms_t = prm->nms_t < nout ? prm->nms_t : nout;
  return SPS_OK;
}

// The plan's detection scratch, grown with hipMalloc to at least `bytes`.
sps_status plan_scratch(sps_plan plan, int64_t bytes, uint8_t **det) {
  if (plan->det_bytes < bytes) {
    if (plan->d_det) (void)hipFree(plan->d_det);
    plan->d_det = nullptr;
    plan->det_bytes = 0;
    const hipError_t e = hipMalloc(&plan->d_det, (size_t)bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SPS_ERR_NOMEM, "device allocation of detection scratch failed");
    }
    plan->det_bytes = bytes;
  }
  *det = plan->d_det;
  return SPS_OK;
}

// Checks of the boxcar calls; fills the width list and 255 nchan.
sps_status check_boxcar(sps_plan plan, int64_t nout, const int32_t *widths, int32_t nw,
                        sps::WidthList *wl, uint32_t *vmax) {
  if (nout < 1 || nout > 0x7FFFFFFF) return fail(SPS_ERR_RANGE, "nout must be in [1, 2^31-1]");
  if (nw < 1 || nw > sps::kMaxWidths)
    return fail(SPS_ERR_INVALID_ARG, "nw must be in [1, %d]", sps::kMaxWidths);
  wl->n = nw;
  for (int i = 0; i < nw; ++i) {
    wl->w[i] = widths[i];
    if (widths[i] < 1) return fail(SPS_ERR_INVALID_ARG, "widths must be >= 1");
    if (i > 0 && widths[i] <= widths[i - 1])
      return fail(SPS_ERR_INVALID_ARG, "widths must be strictly ascending");
  }
  for (int i = nw; i < sps::kMaxWidths; ++i) wl->w[i] = 0;
  const int64_t wmax = widths[nw - 1];
  if (wmax > nout || wmax > sps::kMaxWidth)
    return fail(SPS_ERR_RANGE, "largest width %lld exceeds nout or %d", (long long)wmax,
                sps::kMaxWidth);
  *vmax = 255u * (uint32_t)plan->nchan;
  if ((uint64_t)wmax * *vmax >= (1ull << 31))
    return fail(SPS_ERR_OVERFLOW, "width %lld x 255 x nchan reaches 2^31", (long long)wmax);
  return SPS_OK;
}

// A search without planes carries the in-tile position and the width index
// in one 32-bit key word: a tile (clipped to the plane) may hold at most
// kKeyPosLimit outputs.
bool packed_keys_fit(int ndm, int64_t nout, const sps_detect_params *prm) {
  const int64_t td = prm->tile_dm < ndm ? prm->tile_dm : ndm;
  const int64_t tt = prm->tile_t < nout ? prm->tile_t : nout;
  return td * tt <= sps::kKeyPosLimit;
}

// sps_detect and sps_detect_noalloc: the same checks and kernels; the
// scratch is the plan's (grown with hipMalloc on demand) or the fixed one.
sps_status run_detect(sps_plan plan, const float *snr, const uint8_t *best_w, int64_t nout,
                      const int32_t *widths, int32_t nw, const sps_detect_params *prm,
                      sps_candidate *out, int32_t cap, int32_t *n_found, void *stream,
                      bool fixed) {
  g_error.clear();
  if (!plan || !snr || !best_w || !widths)
    return fail(SPS_ERR_INVALID_ARG, "NULL plan, buffer or parameter");
  DetectArgs a;
  sps_status st = check_detect(plan, nout, nw, prm, out, cap, n_found, &a);
  if (st != SPS_OK) return st;
  if (fixed && a.L.bytes > kFixedScratchBytes)
    return fail(SPS_ERR_RANGE,
                "%lld tiles need %lld bytes of detection scratch; the fixed scratch holds %lld "
                "(at least %lld tiles)",
                (long long)a.ntiles, (long long)a.L.bytes, (long long)kFixedScratchBytes,
                (long long)kFixedScratchTiles);
  DeviceScope scope(plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  uint8_t *det = nullptr;
  st = fixed ? fixed_scratch(plan->device, &det) : plan_scratch(plan, a.L.bytes, &det);
  if (st != SPS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = sps::launch_tile_peaks(snr, best_w, plan->ndm, nout, prm->tile_dm, prm->tile_t,
                                        reinterpret_cast<sps::TilePeak *>(det + a.L.peaks), s);
  if (e != hipSuccess) return hip_fail(e, "tile peak launch");
  e = sps::launch_select_nms(det, plan->ndm, nout, prm->tile_dm, prm->tile_t, prm->threshold,
                             a.nms_dm, a.nms_t, s);
  if (e != hipSuccess) return hip_fail(e, "selection launch");
  return read_candidates(det, a.ntiles, widths, nw, plan->dm.data(), plan->ndm, plan->tsamp_s,
                         out, cap, n_found, s);
}

}  // namespace

namespace sps {

int64_t plan_device_bytes(sps_plan p) {
  if (!p) return 0;
  auto staged = [](const sps::StagedDelays &sd) -> int64_t {
    if (!sd.P) return 0;
    const int64_t nb = (int64_t)((sd.ndm + sd.nd - 1) / sd.nd) * sd.nchan;
    return (int64_t)sd.ndm * sd.pcols * (int64_t)sizeof(int2) + nb * (int64_t)sizeof(int32_t);
  };
  int64_t b = 0;
  if (p->d_delays) b += (int64_t)p->delays.size() * (int64_t)sizeof(int32_t);
  if (p->d_stats) b += (int64_t)p->ndm * 2 * (int64_t)sizeof(int32_t);
  b += staged(p->staged) + staged(p->fused_staged);
  for (const sps::StagedDelays &q : p->sub_staged) b += staged(q);
  if (p->d_det) b += p->det_bytes;
  if (p->d_coarse_full) b += (int64_t)p->coarse_delays.size() * (int64_t)sizeof(int32_t);
  for (size_t s = 0; s < p->d_coarse_sub.size(); ++s)
    if (p->d_coarse_sub[s])
      b += (int64_t)p->ncoarse * (p->sub[s + 1] - p->sub[s]) * (int64_t)sizeof(int32_t);
  if (p->d_resid) b += (int64_t)p->residuals.size() * (int64_t)sizeof(int32_t);
  b += (int64_t)p->I_bytes;
  return b;
}

}  // namespace sps

extern "C" {

const char *sps_last_error(void) { return g_error.c_str(); }

sps_status sps_plan_create(const sps_obs_desc *desc, sps_plan *out) {
  g_error.clear();
  if (!out) return fail(SPS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!desc || !desc->freq_mhz || !desc->dm) return fail(SPS_ERR_INVALID_ARG, "NULL descriptor");
  if (desc->nchan < 1 || desc->ndm < 1) return fail(SPS_ERR_INVALID_ARG, "nchan and ndm must be >= 1");
  if (desc->nchan > 65536) return fail(SPS_ERR_RANGE, "nchan must be <= 65536");
  if (!(desc->tsamp_s > 0) || !(desc->fref_mhz > 0) || !isfinite(desc->tsamp_s) ||
      !isfinite(desc->fref_mhz))
    return fail(SPS_ERR_INVALID_ARG, "tsamp_s and fref_mhz must be positive and finite");
  for (int c = 0; c < desc->nchan; ++c) {
    const double f = desc->freq_mhz[c];
    if (!(f > 0) || f > desc->fref_mhz)
      return fail(SPS_ERR_INVALID_ARG, "channel %d at %g MHz is not in (0, fref]", c, f);
  }
  for (int d = 0; d < desc->ndm; ++d) {
    if (!(desc->dm[d] >= 0) || !isfinite(desc->dm[d]))
      return fail(SPS_ERR_INVALID_ARG, "trial DM %d is negative or not finite", d);
    if (d > 0 && desc->dm[d] < desc->dm[d - 1])
      return fail(SPS_ERR_INVALID_ARG, "trial DMs must be non-decreasing");
  }
  sps_plan p = new (std::nothrow) sps_plan_s;
  if (!p) return fail(SPS_ERR_NOMEM, "host allocation failed");
  p->nchan = desc->nchan;
  p->ndm = desc->ndm;
  p->fref_mhz = desc->fref_mhz;
  p->tsamp_s = desc->tsamp_s;
  try {
    p->freq.assign(desc->freq_mhz, desc->freq_mhz + desc->nchan);
    p->dm.assign(desc->dm, desc->dm + desc->ndm);
    p->delays.resize((size_t)p->ndm * p->nchan);
  } catch (...) {
    free_plan(p);
    return fail(SPS_ERR_NOMEM, "host allocation failed");
  }
  // Eq. (coarse_delay): D = round((K DM / t_samp) (1/f^2 - 1/f_ref^2)),
  // rounding half up; x >= 0 since f <= f_ref.
  const double inv_ref2 = 1.0 / (p->fref_mhz * p->fref_mhz);
  int32_t dmax = 0;
  for (int d = 0; d < p->ndm; ++d) {
    const double a = kKdm * p->dm[d] / p->tsamp_s;
    for (int c = 0; c < p->nchan; ++c) {
      const double f = p->freq[c];
      const double k = 1.0 / (f * f) - inv_ref2;
      const double x = floor(a * k + 0.5);
      if (x > 2147483647.0) {
        free_plan(p);
        return fail(SPS_ERR_OVERFLOW, "delay of trial %d channel %d exceeds 2^31-1 samples", d, c);
      }
      const int32_t v = (int32_t)x;
      p->delays[(size_t)d * p->nchan + c] = v;
      if (v > dmax) dmax = v;
    }
  }
  p->max_delay = dmax;
  sps_status st = choose_tiling(p);
  if (st != SPS_OK) {
    free_plan(p);
    return st;
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "hipGetDevice");
  }
  const size_t tbytes = p->delays.size() * sizeof(int32_t);
  e = hipMalloc(&p->d_delays, tbytes);
  if (e == hipSuccess) e = hipMalloc(&p->d_stats, (size_t)p->ndm * 2 * sizeof(int32_t));
  if (e != hipSuccess) {
    free_plan(p);
    (void)hipGetLastError();
    return fail(SPS_ERR_NOMEM, "device allocation of the delay table failed");
  }
  e = hipMemcpy(p->d_delays, p->delays.data(), tbytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "uploading the delay table");
  }
  st = restage(p);
  if (st != SPS_OK) {
    free_plan(p);
    return st;
  }
  *out = p;
  return SPS_OK;
}

sps_status sps_plan_destroy(sps_plan plan) {
  g_error.clear();
  if (!plan) return SPS_OK;
  DeviceScope scope(plan->device);
  free_plan(plan);
  return SPS_OK;
}

sps_status sps_plan_delays(sps_plan plan, int32_t *host_out, int32_t *max_delay) {
  g_error.clear();
  if (!plan) return fail(SPS_ERR_INVALID_ARG, "plan is NULL");
  if (host_out) memcpy(host_out, plan->delays.data(), plan->delays.size() * sizeof(int32_t));
  if (max_delay) *max_delay = plan->max_delay;
  return SPS_OK;
}

sps_status sps_plan_set_tiling(sps_plan plan, int32_t m, int32_t dpw, int32_t nw, int32_t cs,
                               int32_t waves_per_eu) {
  g_error.clear();
  if (!plan) return fail(SPS_ERR_INVALID_ARG, "plan is NULL");
  if (m == 0) {
    plan->cfg = sps::DedispConfig{0, 0, 0, 0, 0, 0};
    plan->lds_pitch = 0;
    return restage(plan);
  }
  bool known = false;
  for (const auto &c : kPrefs) {
    if (c.m != m || c.dpw != dpw || c.nw != nw || c.cs != cs) continue;
    if (waves_per_eu != 0 && c.wpe != waves_per_eu) continue;
    known = true;
    const int64_t pitch = fitted_pitch(plan, c, 160 * 1024);
    if (pitch > 0) {
      const sps::DedispConfig old_cfg = plan->cfg;
      const int old_pitch = plan->lds_pitch;
      plan->cfg = c;
      plan->lds_pitch = (int)pitch;
      const sps_status r = restage(plan);
      if (r != SPS_OK) {  // keep the previous tiling usable
        plan->cfg = old_cfg;
        plan->lds_pitch = old_pitch;
        (void)restage(plan);
      }
      return r;
    }
  }
  if (!known)
    return fail(SPS_ERR_INVALID_ARG, "tiling (%d, %d, %d, %d, %d) is not compiled in", m, dpw, nw,
                cs, waves_per_eu);
  return fail(SPS_ERR_RANGE, "tiling (%d, %d, %d, %d) does not fit this plan's delay spread", m,
              dpw, nw, cs);
}

sps_status sps_plan_get_tiling(sps_plan plan, int32_t *m, int32_t *dpw, int32_t *nw, int32_t *cs,
                               int32_t *waves_per_eu, int32_t *lds_bytes) {
  g_error.clear();
  if (!plan) return fail(SPS_ERR_INVALID_ARG, "plan is NULL");
  if (m) *m = plan->cfg.m;
  if (dpw) *dpw = plan->cfg.dpw;
  if (nw) *nw = plan->cfg.nw;
  if (cs) *cs = plan->cfg.cs;
  if (waves_per_eu) *waves_per_eu = plan->cfg.wpe;
  if (lds_bytes) *lds_bytes = (int32_t)plan->cfg.lds_bytes(plan->lds_pitch);
  return SPS_OK;
}

sps_status sps_dedisperse(sps_plan plan, const uint8_t *X, int64_t pitch, int64_t nsamp_in,
                          uint32_t *Y, int64_t nout, uint32_t flags, void *stream) {
  g_error.clear();
  if (!plan || !X || !Y) return fail(SPS_ERR_INVALID_ARG, "NULL plan or buffer");
  if (flags & ~SPS_ZERO_PAD) return fail(SPS_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if (!aligned16(X) || pitch % 16 != 0)
    return fail(SPS_ERR_INVALID_ARG, "X must be 16-byte aligned with a pitch multiple of 16");
  if (nsamp_in < 0 || pitch < nsamp_in)
    return fail(SPS_ERR_RANGE, "need 0 <= nsamp_in <= pitch (nsamp_in %lld, pitch %lld)",
                (long long)nsamp_in, (long long)pitch);
  if (nout < 1 || nout > 0x7FFFFFFF) return fail(SPS_ERR_RANGE, "nout must be in [1, 2^31-1]");
  if (!(flags & SPS_ZERO_PAD) && nsamp_in < nout + plan->max_delay)
    return fail(SPS_ERR_RANGE, "nsamp_in %lld < nout %lld + max delay %d (pass SPS_ZERO_PAD to allow)",
                (long long)nsamp_in, (long long)nout, plan->max_delay);
  DeviceScope scope(plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  hipError_t e = sps::launch_dedisperse(plan->cfg, plan->lds_pitch, X, pitch, nsamp_in,
                                        plan->d_delays, &plan->staged, plan->nchan, plan->ndm, Y,
                                        nout, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "dedispersion launch");
  return SPS_OK;
}

sps_status sps_boxcar_snr(sps_plan plan, const uint32_t *Y, int64_t nout, const int32_t *widths,
                          int32_t nw, float *snr, uint8_t *best_w, int32_t *stats,
                          void *stream) {
  g_error.clear();
  if (!plan || !Y || !widths || !snr || !best_w)
    return fail(SPS_ERR_INVALID_ARG, "NULL plan or buffer");
  sps::WidthList wl;
  uint32_t vmax = 0;
  const sps_status st = check_boxcar(plan, nout, widths, nw, &wl, &vmax);
  if (st != SPS_OK) return st;
  DeviceScope scope(plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  int32_t *sts = stats ? stats : plan->d_stats;
  hipError_t e = sps::launch_row_stats(Y, plan->ndm, nout, vmax, sts, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "row statistics launch");
  e = sps::launch_boxcar(Y, plan->ndm, nout, sts, wl, snr, best_w, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "boxcar launch");
  return SPS_OK;
}

sps_status sps_search(sps_plan plan, const uint32_t *Y, int64_t nout, const int32_t *widths,
                      int32_t nw, float *snr, uint8_t *best_w, int32_t *stats,
                      const sps_detect_params *prm, sps_candidate *out, int32_t cap,
                      int32_t *n_found, void *stream) {
  g_error.clear();
  if (!plan || !Y || !widths || (!snr) != (!best_w))
    return fail(SPS_ERR_INVALID_ARG, "NULL plan or buffer (snr and best_w are NULL together)");
  sps::WidthList wl;
  uint32_t vmax = 0;
  sps_status st = check_boxcar(plan, nout, widths, nw, &wl, &vmax);
  if (st != SPS_OK) return st;
  DetectArgs a;
  st = check_detect(plan, nout, nw, prm, out, cap, n_found, &a);
  if (st != SPS_OK) return st;
  const bool planes = snr != nullptr;
  if (!planes && !packed_keys_fit(plan->ndm, nout, prm))
    return fail(SPS_ERR_RANGE, "without planes a tile may hold at most %lld outputs",
                (long long)sps::kKeyPosLimit);
  DeviceScope scope(plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  uint8_t *det = nullptr;
  st = plan_scratch(plan, a.L.bytes, &det);
  if (st != SPS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // tile keys in the out array of the scratch (16 bytes per tile), zeroed
  sps::TileSink sink{};
  sink.keys = reinterpret_cast<unsigned long long *>(det + a.L.out);
  sink.tile_dm = prm->tile_dm;
  sink.tile_t = prm->tile_t;
  sink.ntt = a.ntt;
  sink.packed = planes ? 0 : 1;
  sps::TilePeak *peaks = reinterpret_cast<sps::TilePeak *>(det + a.L.peaks);
  hipError_t e = sps::launch_tile_keys(sink, plan->ndm, nout, best_w, peaks, false, s);
  if (e != hipSuccess) return hip_fail(e, "tile key clearing launch");
  int32_t *sts = stats ? stats : plan->d_stats;
  e = sps::launch_row_stats(Y, plan->ndm, nout, vmax, sts, s);
  if (e != hipSuccess) return hip_fail(e, "row statistics launch");
  e = sps::launch_boxcar(Y, plan->ndm, nout, sts, wl, snr, best_w, s, sink);
  if (e != hipSuccess) return hip_fail(e, "boxcar launch");
  e = sps::launch_tile_keys(sink, plan->ndm, nout, best_w, peaks, true, s);
  if (e != hipSuccess) return hip_fail(e, "tile key decoding launch");
  e = sps::launch_select_nms(det, plan->ndm, nout, prm->tile_dm, prm->tile_t, prm->threshold,
                             a.nms_dm, a.nms_t, s);
  if (e != hipSuccess) return hip_fail(e, "selection launch");
  return read_candidates(det, a.ntiles, widths, nw, plan->dm.data(), plan->ndm, plan->tsamp_s,
                         out, cap, n_found, s);
}

sps_status sps_boxcar_pool(sps_plan plan, const uint32_t *Y, int64_t nout, const int32_t *widths,
                           int32_t nw, int32_t *stats, float scale, uint16_t *tiles,
                           int64_t *ntiles, void *stream) {
  g_error.clear();
  if (!plan || !Y || !widths || !tiles) return fail(SPS_ERR_INVALID_ARG, "NULL plan or buffer");
  if (!(scale > 0.0f) || !isfinite(scale))
    return fail(SPS_ERR_INVALID_ARG, "scale must be positive and finite");
  sps::WidthList wl;
  uint32_t vmax = 0;
  const sps_status st = check_boxcar(plan, nout, widths, nw, &wl, &vmax);
  if (st != SPS_OK) return st;
  if (ntiles) *ntiles = (int64_t)(plan->ndm / sps::kPoolTileDm) * (nout / 4096);
  DeviceScope scope(plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  int32_t *sts = stats ? stats : plan->d_stats;
  hipError_t e = sps::launch_row_stats(Y, plan->ndm, nout, vmax, sts, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "row statistics launch");
  e = sps::launch_boxcar_pool(Y, plan->ndm, nout, sts, wl, scale, tiles, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pooled boxcar launch");
  return SPS_OK;
}

sps_status sps_detect(sps_plan plan, const float *snr, const uint8_t *best_w, int64_t nout,
                      const int32_t *widths, int32_t nw, const sps_detect_params *prm,
                      sps_candidate *out, int32_t cap, int32_t *n_found, void *stream) {
  return run_detect(plan, snr, best_w, nout, widths, nw, prm, out, cap, n_found, stream, false);
}

sps_status sps_detect_noalloc(sps_plan plan, const float *snr, const uint8_t *best_w,
                              int64_t nout, const int32_t *widths, int32_t nw,
                              const sps_detect_params *prm, sps_candidate *out, int32_t cap,
                              int32_t *n_found, void *stream) {
  return run_detect(plan, snr, best_w, nout, widths, nw, prm, out, cap, n_found, stream, true);
}

sps_status sps_subband_plan_create(const sps_subband_desc *desc, sps_plan *out) {
  g_error.clear();
  if (!out) return fail(SPS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!desc || !desc->freq_mhz) return fail(SPS_ERR_INVALID_ARG, "NULL descriptor");
  if (desc->ndm < 1 || desc->n0 < 1 || desc->nsub < 1 || desc->nsub > desc->nchan)
    return fail(SPS_ERR_INVALID_ARG, "need ndm >= 1, n0 >= 1 and 1 <= nsub <= nchan");
  if (!(desc->dm_lo >= 0) || !(desc->dm_step >= 0) || !isfinite(desc->dm_lo) ||
      !isfinite(desc->dm_step))
    return fail(SPS_ERR_INVALID_ARG, "dm_lo and dm_step must be finite and >= 0");
  std::vector<double> dm;
  try {
    dm.resize((size_t)desc->ndm);
  } catch (...) {
    return fail(SPS_ERR_NOMEM, "host allocation failed");
  }
  for (int m = 0; m < desc->ndm; ++m) dm[(size_t)m] = desc->dm_lo + (double)m * desc->dm_step;
  sps_obs_desc base{desc->nchan, desc->freq_mhz, desc->fref_mhz, desc->tsamp_s, desc->ndm,
                    dm.data()};
  sps_plan p = nullptr;
  sps_status st = sps_plan_create(&base, &p);
  if (st != SPS_OK) return st;
  DeviceScope scope(p->device);
  p->subband = true;
  p->n0 = desc->n0;
  p->nsub = desc->nsub;
  p->ncoarse = (p->ndm + p->n0 - 1) / p->n0;
  const int nchan = p->nchan, nsub = p->nsub, ncoarse = p->ncoarse, ndm = p->ndm;
  try {
    p->sub.resize((size_t)nsub + 1);
    p->fsub.resize((size_t)nsub);
    p->coarse_delays.resize((size_t)ncoarse * nchan);
    p->residuals.resize((size_t)ndm * nsub);
    p->d_coarse_sub.assign((size_t)nsub, nullptr);
    p->sub_cfg.resize((size_t)nsub);
    p->sub_staged.resize((size_t)nsub);
    p->sub_pitch.resize((size_t)nsub);
  } catch (...) {
    free_plan(p);
    return fail(SPS_ERR_NOMEM, "host allocation failed");
  }
  for (int s = 0; s <= nsub; ++s) p->sub[(size_t)s] = (int32_t)(((int64_t)s * nchan) / nsub);
  const double inv_ref2 = 1.0 / (p->fref_mhz * p->fref_mhz);
  // Eq. (coarse_delay) on the coarse grid DM_j = dm_lo + j n0 dDM.
  for (int j = 0; j < ncoarse; ++j) {
    const double dmj = desc->dm_lo + (double)j * (double)p->n0 * desc->dm_step;
    const double a = kKdm * dmj / p->tsamp_s;
    for (int c = 0; c < nchan; ++c) {
      const double f = p->freq[(size_t)c];
      const double x = floor(a * (1.0 / (f * f) - inv_ref2) + 0.5);
      if (x > 2147483647.0) {
        free_plan(p);
        return fail(SPS_ERR_OVERFLOW, "coarse delay exceeds 2^31-1 samples");
      }
      p->coarse_delays[(size_t)j * nchan + c] = (int32_t)x;
    }
  }
  // Eq. (residual): subband s represented by F_s with 1/F_s^2 the mean of
  // 1/f^2 over its channels; dDM_m = DM_m - DM_j(m).
  int32_t rmax = 0;
  for (int s = 0; s < nsub; ++s) {
    double acc = 0.0;
    for (int c = p->sub[(size_t)s]; c < p->sub[(size_t)s + 1]; ++c) {
      const double f = p->freq[(size_t)c];
      acc += 1.0 / (f * f);
    }
    const double inv_f2 = acc / (double)(p->sub[(size_t)s + 1] - p->sub[(size_t)s]);
    p->fsub[(size_t)s] = 1.0 / sqrt(inv_f2);
    const double k = inv_f2 - inv_ref2;
    for (int m = 0; m < ndm; ++m) {
      const double dm_m = desc->dm_lo + (double)m * desc->dm_step;
      const double dm_j = desc->dm_lo + (double)((m / p->n0) * p->n0) * desc->dm_step;
      const double x = floor((kKdm * (dm_m - dm_j) / p->tsamp_s) * k + 0.5);
      if (x > 2147483647.0 || x < 0) {
        free_plan(p);
        return fail(SPS_ERR_OVERFLOW, "residual shift out of range");
      }
      p->residuals[(size_t)m * nsub + s] = (int32_t)x;
      if ((int32_t)x > rmax) rmax = (int32_t)x;
    }
  }
  p->rmax = rmax;
  int32_t eff = 0;
  for (int m = 0; m < ndm; ++m)
    for (int s = 0; s < nsub; ++s)
      for (int c = p->sub[(size_t)s]; c < p->sub[(size_t)s + 1]; ++c) {
        const int64_t v = (int64_t)p->coarse_delays[(size_t)(m / p->n0) * nchan + c] +
                          p->residuals[(size_t)m * nsub + s];
        if (v > 2147483647) {
          free_plan(p);
          return fail(SPS_ERR_OVERFLOW, "effective delay exceeds 2^31-1 samples");
        }
        if (v > eff) eff = (int32_t)v;
      }
  p->eff_max_delay = eff;
  // Per-subband coarse tables and stage-1 tilings.
  std::vector<int32_t> tab;
  for (int s = 0; s < nsub; ++s) {
    const int c0 = p->sub[(size_t)s], ns = p->sub[(size_t)s + 1] - c0;
    tab.resize((size_t)ncoarse * ns);
    for (int j = 0; j < ncoarse; ++j)
      for (int c = 0; c < ns; ++c)
        tab[(size_t)j * ns + c] = p->coarse_delays[(size_t)j * nchan + c0 + c];
    pick_tiling(tab.data(), ns, ncoarse, &p->sub_cfg[(size_t)s], &p->sub_pitch[(size_t)s]);
    hipError_t e = hipMalloc(&p->d_coarse_sub[(size_t)s], tab.size() * sizeof(int32_t));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_coarse_sub[(size_t)s], tab.data(), tab.size() * sizeof(int32_t),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = sps::stage_delays(p->sub_staged[(size_t)s], p->sub_cfg[(size_t)s],
                            p->sub_pitch[(size_t)s], p->d_coarse_sub[(size_t)s], ns, ncoarse,
                            *std::max_element(tab.begin(), tab.end()));
    if (e != hipSuccess) {
      free_plan(p);
      (void)hipGetLastError();
      return fail(SPS_ERR_NOMEM, "device allocation of subband tables failed");
    }
  }
  // One stage-1 launch over all channels when the subbands are equal.
  if (nchan % nsub == 0) {
    const int seg = nchan / nsub;
    pick_tiling(p->coarse_delays.data(), nchan, ncoarse, &p->fused_cfg, &p->fused_pitch, seg);
    if (p->fused_cfg.m != 0) {
      hipError_t e = hipMalloc(&p->d_coarse_full, p->coarse_delays.size() * sizeof(int32_t));
      if (e == hipSuccess)
        e = hipMemcpy(p->d_coarse_full, p->coarse_delays.data(),
                      p->coarse_delays.size() * sizeof(int32_t), hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = sps::stage_delays(p->fused_staged, p->fused_cfg, p->fused_pitch, p->d_coarse_full,
                              nchan, ncoarse,
                              *std::max_element(p->coarse_delays.begin(), p->coarse_delays.end()));
      if (e != hipSuccess) {
        free_plan(p);
        (void)hipGetLastError();
        return fail(SPS_ERR_NOMEM, "device allocation of the coarse table failed");
      }
      p->fused = true;
    }
  }
  // stage 2 reads the residuals transposed, [nsub][ndm]
  std::vector<int32_t> rt(p->residuals.size());
  for (int m = 0; m < ndm; ++m)
    for (int s = 0; s < nsub; ++s)
      rt[(size_t)s * ndm + m] = p->residuals[(size_t)m * nsub + s];
  hipError_t e = hipMalloc(&p->d_resid, rt.size() * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_resid, rt.data(), rt.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(p);
    (void)hipGetLastError();
    return fail(SPS_ERR_NOMEM, "device allocation of the residual table failed");
  }
  *out = p;
  return SPS_OK;
}

sps_status sps_subband_tables(sps_plan plan, int32_t *coarse_delays, int32_t *residuals,
                              double *fsub, int32_t *max_delay) {
  g_error.clear();
  if (!plan || !plan->subband) return fail(SPS_ERR_INVALID_ARG, "not a subband plan");
  if (coarse_delays)
    memcpy(coarse_delays, plan->coarse_delays.data(),
           plan->coarse_delays.size() * sizeof(int32_t));
  if (residuals)
    memcpy(residuals, plan->residuals.data(), plan->residuals.size() * sizeof(int32_t));
  if (fsub) memcpy(fsub, plan->fsub.data(), plan->fsub.size() * sizeof(double));
  if (max_delay) *max_delay = plan->eff_max_delay;
  return SPS_OK;
}

sps_status sps_dedisperse_subband(sps_plan plan, const uint8_t *X, int64_t pitch,
                                  int64_t nsamp_in, uint32_t *Y, int64_t nout, uint32_t flags,
                                  void *stream) {
  g_error.clear();
  if (!plan || !X || !Y) return fail(SPS_ERR_INVALID_ARG, "NULL plan or buffer");
  if (!plan->subband) return fail(SPS_ERR_INVALID_ARG, "plan was not made by sps_subband_plan_create");
  if (flags & ~SPS_ZERO_PAD) return fail(SPS_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if (!aligned16(X) || pitch % 16 != 0)
    return fail(SPS_ERR_INVALID_ARG, "X must be 16-byte aligned with a pitch multiple of 16");
  if (nsamp_in < 0 || pitch < nsamp_in) return fail(SPS_ERR_RANGE, "need 0 <= nsamp_in <= pitch");
  if (nout < 1 || nout > 0x7FFFFFFF - plan->rmax)
    return fail(SPS_ERR_RANGE, "nout must be in [1, 2^31-1 - max residual]");
  if (!(flags & SPS_ZERO_PAD) && nsamp_in < nout + plan->eff_max_delay)
    return fail(SPS_ERR_RANGE, "nsamp_in %lld < nout %lld + effective max delay %d",
                (long long)nsamp_in, (long long)nout, plan->eff_max_delay);
  DeviceScope scope(plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  // Subband series rows: nout + R_max samples, padded to a multiple of 4 so
  // that stage 1 stores 16-byte vectors.
  const int64_t len1 = (nout + plan->rmax + 3) / 4 * 4;
  const size_t need = (size_t)plan->nsub * plan->ncoarse * (size_t)len1 * sizeof(uint32_t);
  if (plan->I_bytes < need) {
    if (plan->d_I) (void)hipFree(plan->d_I);
    plan->d_I = nullptr;
    plan->I_bytes = 0;
    hipError_t e = hipMalloc(&plan->d_I, need);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SPS_ERR_NOMEM, "device allocation of %zu bytes of subband series failed", need);
    }
    plan->I_bytes = need;
  }
  hipStream_t s = (hipStream_t)stream;
  if (plan->fused && plan->use_fused) {
    hipError_t e = sps::launch_dedisperse(plan->fused_cfg, plan->fused_pitch, X, pitch, nsamp_in,
                                          plan->d_coarse_full, &plan->fused_staged, plan->nchan,
                                          plan->ncoarse, plan->d_I, len1, s,
                                          plan->nchan / plan->nsub, (int64_t)plan->ncoarse * len1);
    if (e != hipSuccess) return hip_fail(e, "subband stage 1 launch");
  } else {
    for (int b = 0; b < plan->nsub; ++b) {
      const int c0 = plan->sub[(size_t)b], ns = plan->sub[(size_t)b + 1] - c0;
      hipError_t e = sps::launch_dedisperse(
          plan->sub_cfg[(size_t)b], plan->sub_pitch[(size_t)b], X + (int64_t)c0 * pitch, pitch,
          nsamp_in, plan->d_coarse_sub[(size_t)b], &plan->sub_staged[(size_t)b], ns,
          plan->ncoarse, plan->d_I + (size_t)b * plan->ncoarse * (size_t)len1, len1, s);
      if (e != hipSuccess) return hip_fail(e, "subband stage 1 launch");
    }
  }
  hipError_t e = sps::launch_subband_stage2(plan->d_I, len1, plan->ncoarse, plan->nsub,
                                            plan->d_resid, plan->rmax, plan->ndm, plan->n0, Y,
                                            nout, s);
  if (e != hipSuccess) return hip_fail(e, "subband stage 2 launch");
  return SPS_OK;
}

sps_status sps_zero_dm(const uint8_t *X, int64_t pitch, int64_t nsamp, int32_t nchan, uint8_t *Xo,
                       int64_t pitch_out, void *stream) {
  g_error.clear();
  if (!X || !Xo) return fail(SPS_ERR_INVALID_ARG, "NULL buffer");
  if (nchan < 1) return fail(SPS_ERR_INVALID_ARG, "nchan must be >= 1");
  if (!aligned16(X) || !aligned16(Xo) || pitch % 16 != 0 || pitch_out % 16 != 0)
    return fail(SPS_ERR_INVALID_ARG, "buffers must be 16-byte aligned with pitches multiple of 16");
  if (nsamp < 0 || pitch < nsamp || pitch_out < nsamp)
    return fail(SPS_ERR_RANGE, "need 0 <= nsamp <= pitch, pitch_out");
  if ((int64_t)nchan * 255 >= (1ll << 31)) return fail(SPS_ERR_OVERFLOW, "too many channels");
  hipError_t e = sps::launch_zero_dm(X, pitch, nsamp, nchan, Xo, pitch_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "zero-DM launch");
  return SPS_OK;
}

sps_status sps_downsample_sqrt(const uint8_t *X, int64_t pitch, int64_t nsamp, int32_t nchan,
                               int32_t factor, uint8_t *Xo, int64_t pitch_out, void *stream) {
  g_error.clear();
  if (!X || !Xo) return fail(SPS_ERR_INVALID_ARG, "NULL buffer");
  if (nchan < 1 || nchan > 65535 || factor < 1 || factor > (1 << 20))
    return fail(SPS_ERR_INVALID_ARG, "need 1 <= nchan <= 65535 and 1 <= factor <= 2^20");
  if (nsamp < 0 || pitch < nsamp || pitch_out < nsamp / factor)
    return fail(SPS_ERR_RANGE, "need 0 <= nsamp <= pitch and pitch_out >= nsamp / factor");
  hipError_t e = sps::launch_downsample_sqrt(X, pitch, nsamp, nchan, factor, Xo, pitch_out,
                                             (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "downsampling launch");
  return SPS_OK;
}

/* ---------------- batches of filterbanks sharing one plan ---------------- */

}  // extern "C"

// Accepted offers per beam that sps_batch_candidates_all brings back in its
// one copy; a beam with more reads the rest through its own copies.
constexpr int kGatherRecords = 512;
constexpr size_t kGatherSlot = sps::kGatherHeader + sizeof(sps::TilePeak) * kGatherRecords;

struct sps_batch_s {
  sps_plan plan = nullptr;
  int nbeams = 0;
  std::vector<sps::BeamWork> beams;
  std::vector<int64_t> nout;
  sps::BeamWork *d_beams = nullptr;
  int64_t dd_items = 0, bx_blocks = 0, tp_tiles = 0;
  sps::WidthList widths{};
  std::vector<int32_t> widths_host;
  sps_detect_params prm{};
  sps::DedispConfig cfg{};
  int lds_pitch = 0;
  sps::StagedDelays staged;  // the plan's table for cfg, owned by the batch
  int grid_dd = 0;
  uint8_t *d_det = nullptr;  // detection scratch of every beam (BeamWork::det_begin)
  uint8_t *d_gather = nullptr;  // sps_batch_candidates_all: device slots of every beam
  uint8_t *h_gather = nullptr;  // and their pinned host copy
  int64_t det_bytes = 0;
  int64_t pl_blocks = 0, pool_tiles = 0;  // pooled-tile boxcar workgroups, detector tiles
  uint16_t *tiles = nullptr;              // tile mode (sps_batch_set_tiles): destination
  float tile_scale = 0.0f;
  bool planes = true;  // false: no beam has S/N or width planes (packed tile keys)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t graph_stream = nullptr;
};

namespace {

void free_batch(sps_batch b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_beams) (void)hipFree(b->d_beams);
  if (b->d_det) (void)hipFree(b->d_det);
  if (b->d_gather) (void)hipFree(b->d_gather);
  if (b->h_gather) (void)hipHostFree(b->h_gather);
  sps::free_staged(b->staged);
  delete b;
}

// Dedispersion item ranges of the beams (and the grid: one workgroup per
// item, rounded up to whole XCD shares) for tiling c; host side only.
// False (and nothing changed) if the grid would pass 2^31 - 1 workgroups.
bool layout_dedisp(sps_batch b, const sps::DedispConfig &c) {
  int64_t items = 0;
  for (int i = 0; i < b->nbeams; ++i)
    items += sps::dedisp_batch_items(c, b->plan->ndm, b->nout[(size_t)i]);
  if (items > 0x7FFFFFF8) return false;
  items = 0;
  for (int i = 0; i < b->nbeams; ++i) {
    b->beams[(size_t)i].dd_begin = items;
    items += sps::dedisp_batch_items(c, b->plan->ndm, b->nout[(size_t)i]);
  }
  b->dd_items = items;
  b->grid_dd = (int)(((items + 7) / 8) * 8);
  return true;
}

sps_status batch_enqueue(sps_batch b, hipStream_t s) {
  sps_plan p = b->plan;
  hipError_t e = sps::launch_dedisperse_batch(b->cfg, b->lds_pitch, b->d_beams, b->nbeams,
                                              b->dd_items, b->staged, p->nchan, p->ndm,
                                              b->grid_dd, s);
  if (e != hipSuccess) return hip_fail(e, "batched dedispersion launch");
  e = sps::launch_row_stats_batch(b->d_beams, b->nbeams, p->ndm, 255u * (uint32_t)p->nchan,
                                  *std::max_element(b->nout.begin(), b->nout.end()), s);
  if (e != hipSuccess) return hip_fail(e, "batched statistics launch");
  if (b->tiles) {
    // tile mode: detector tiles straight from the boxcar pass, no planes
    e = sps::launch_boxcar_pool_batch(b->d_beams, b->nbeams, b->pl_blocks, b->widths,
                                      b->tile_scale, b->tiles, s);
    if (e != hipSuccess) return hip_fail(e, "batched pooled boxcar launch");
    return SPS_OK;
  }
  // tile maxima taken inside the boxcar pass: keys zeroed, gathered, decoded
  e = sps::launch_tile_keys_batch(b->d_beams, b->nbeams, p->ndm, b->tp_tiles, b->prm.tile_dm,
                                  b->prm.tile_t, b->d_det, false, !b->planes, s);
  if (e != hipSuccess) return hip_fail(e, "batched tile key clearing launch");
  bool rows_of_64 = true;
  for (int64_t n : b->nout) rows_of_64 = rows_of_64 && n % 64 == 0;
  e = sps::launch_boxcar_batch(b->d_beams, b->nbeams, b->bx_blocks, b->widths, s, b->d_det,
                               p->ndm, b->prm.tile_dm, b->prm.tile_t, rows_of_64, b->planes);
  if (e != hipSuccess) return hip_fail(e, "batched boxcar launch");
  e = sps::launch_tile_keys_batch(b->d_beams, b->nbeams, p->ndm, b->tp_tiles, b->prm.tile_dm,
                                  b->prm.tile_t, b->d_det, true, !b->planes, s);
  if (e != hipSuccess) return hip_fail(e, "batched tile key decoding launch");
  e = sps::launch_select_nms_batch(b->d_beams, b->nbeams, p->ndm, b->prm.tile_dm, b->prm.tile_t,
                                   b->prm.threshold, b->prm.nms_dm, b->prm.nms_t, b->d_det, s);
  if (e != hipSuccess) return hip_fail(e, "batched selection launch");
  return SPS_OK;
}

}  // namespace

extern "C" {

sps_status sps_batch_create(sps_plan plan, int32_t nbeams, const sps_beam *beams,
                            const int32_t *widths, int32_t nw, const sps_detect_params *prm,
                            uint32_t flags, sps_batch *out) {
  g_error.clear();
  if (!out) return fail(SPS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!plan || !beams || !widths || !prm) return fail(SPS_ERR_INVALID_ARG, "NULL argument");
  if (nbeams < 1 || nbeams > 4096) return fail(SPS_ERR_INVALID_ARG, "nbeams must be in [1, 4096]");
  if (flags & ~SPS_ZERO_PAD) return fail(SPS_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
  if (plan->cfg.m == 0)
    return fail(SPS_ERR_RANGE, "the plan's delay spread needs the plain kernel, which has no batched form");
  if (nw < 1 || nw > sps::kMaxWidths) return fail(SPS_ERR_INVALID_ARG, "bad width count");
  for (int i = 0; i < nw; ++i)
    if (widths[i] < 1 || (i > 0 && widths[i] <= widths[i - 1]))
      return fail(SPS_ERR_INVALID_ARG, "widths must be >= 1 and strictly ascending");
  if (widths[nw - 1] > sps::kMaxWidth) return fail(SPS_ERR_RANGE, "largest width above %d", sps::kMaxWidth);
  const uint32_t vmax = 255u * (uint32_t)plan->nchan;
  if ((uint64_t)widths[nw - 1] * vmax >= (1ull << 31))
    return fail(SPS_ERR_OVERFLOW, "width x 255 x nchan reaches 2^31");
  if (!(prm->threshold > 0.0f) || prm->tile_dm < 1 || prm->tile_t < 1 || prm->nms_dm < 0 ||
      prm->nms_t < 0 || (uint64_t)prm->tile_dm * (uint64_t)prm->tile_t >= (1ull << 32))
    return fail(SPS_ERR_INVALID_ARG, "bad detection parameters");
  sps_batch b = new (std::nothrow) sps_batch_s;
  if (!b) return fail(SPS_ERR_NOMEM, "host allocation failed");
  b->plan = plan;
  b->nbeams = nbeams;
  b->prm = *prm;
  // radii past the plane's extent suppress the same offers as the extent
  // (the kernel clamps nms_t to each beam's length)
  if (b->prm.nms_dm > plan->ndm) b->prm.nms_dm = plan->ndm;
  if (b->prm.nms_t > 0x7FFFFFFF) b->prm.nms_t = 0x7FFFFFFF;
  b->cfg = plan->cfg;
  b->lds_pitch = plan->lds_pitch;
  b->widths.n = nw;
  for (int i = 0; i < sps::kMaxWidths; ++i) b->widths.w[i] = i < nw ? widths[i] : 0;
  b->widths_host.assign(widths, widths + nw);
  b->beams.resize((size_t)nbeams);
  b->nout.resize((size_t)nbeams);
  const int64_t ntd = (plan->ndm + prm->tile_dm - 1) / prm->tile_dm;
  for (int i = 0; i < nbeams; ++i) {
    const sps_beam &q = beams[i];
    if (i == 0) b->planes = q.snr != nullptr;
    if (!q.X || !q.Y || !q.stats || (!q.snr) != (!q.best_w) || (q.snr != nullptr) != b->planes) {
      free_batch(b);
      return fail(SPS_ERR_INVALID_ARG,
                  "beam %d has a NULL buffer (snr and best_w may be NULL together, in every beam)",
                  i);
    }
    if (!b->planes && !packed_keys_fit(plan->ndm, q.nout, prm)) {
      free_batch(b);
      return fail(SPS_ERR_RANGE, "without planes a tile may hold at most %lld outputs",
                  (long long)sps::kKeyPosLimit);
    }
    if (!aligned16(q.X) || q.pitch % 16 != 0) {
      free_batch(b);
      return fail(SPS_ERR_INVALID_ARG, "beam %d: X must be 16-byte aligned, pitch a multiple of 16", i);
    }
    if (q.nout < widths[nw - 1] || q.nout > 0x7FFFFFFF || q.nsamp_in < 0 || q.pitch < q.nsamp_in) {
      free_batch(b);
      return fail(SPS_ERR_RANGE, "beam %d: bad nout / nsamp_in / pitch", i);
    }
    if (!(flags & SPS_ZERO_PAD) && q.nsamp_in < q.nout + plan->max_delay) {
      free_batch(b);
      return fail(SPS_ERR_RANGE, "beam %d: nsamp_in < nout + max delay", i);
    }
    sps::BeamWork &w = b->beams[(size_t)i];
    w.X = q.X;
    w.pitch = q.pitch;
    w.nsamp_in = q.nsamp_in;
    w.Y = q.Y;
    w.nout = q.nout;
    w.snr = q.snr;
    w.best = q.best_w;
    w.stats = q.stats;
    w.bx_begin = b->bx_blocks;
    w.tp_begin = b->tp_tiles;
    w.nseg = sps::boxcar_segments(q.nout);
    w.ntt = (q.nout + prm->tile_t - 1) / prm->tile_t;
    w.vec_store = (q.nout % 4 == 0) && aligned16(q.Y);
    w.pad = 0;
    w.det_begin = b->det_bytes;
    // whole detector tiles of the beam's plane (tile mode)
    w.pcols = q.nout / 4096;
    w.pl_begin = b->pl_blocks;
    w.tile_begin = b->pool_tiles;
    b->pl_blocks += (int64_t)(plan->ndm / sps::kPoolTileDm) * (sps::kPoolTileDm / 2) * w.pcols;
    b->pool_tiles += (int64_t)(plan->ndm / sps::kPoolTileDm) * w.pcols;
    b->bx_blocks += w.nseg * plan->ndm;
    b->tp_tiles += w.ntt * ntd;
    b->det_bytes += sps::detect_layout(w.ntt * ntd).bytes;
    b->nout[(size_t)i] = q.nout;
  }
  if (b->bx_blocks > 0x7FFFFFFF || b->tp_tiles > 0x7FFFFFFF || b->pl_blocks > 0x7FFFFFFF ||
      !layout_dedisp(b, b->cfg)) {
    free_batch(b);
    return fail(SPS_ERR_RANGE, "batch too large");
  }
  DeviceScope scope(plan->device);
  hipError_t e = hipMalloc(&b->d_beams, sizeof(sps::BeamWork) * (size_t)nbeams);
  if (e == hipSuccess) e = hipMalloc(&b->d_det, (size_t)b->det_bytes);
  // zero statuses: candidates read before the first run are none
  if (e == hipSuccess) e = hipMemset(b->d_det, 0, (size_t)b->det_bytes);
  const size_t gather_bytes = (size_t)nbeams * kGatherSlot;
  if (e == hipSuccess) e = hipMalloc(&b->d_gather, gather_bytes);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&b->h_gather), gather_bytes);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_beams, b->beams.data(), sizeof(sps::BeamWork) * (size_t)nbeams,
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = sps::stage_delays(b->staged, b->cfg, b->lds_pitch, plan->d_delays, plan->nchan,
                          plan->ndm, plan->max_delay);
  if (e != hipSuccess) {
    free_batch(b);
    (void)hipGetLastError();
    return fail(SPS_ERR_NOMEM, "device allocation for the batch failed");
  }
  *out = b;
  return SPS_OK;
}

sps_status sps_batch_destroy(sps_batch batch) {
  g_error.clear();
  if (!batch) return SPS_OK;
  DeviceScope scope(batch->plan->device);
  free_batch(batch);
  return SPS_OK;
}

sps_status sps_batch_enqueue(sps_batch batch, void *stream) {
  g_error.clear();
  if (!batch) return fail(SPS_ERR_INVALID_ARG, "batch is NULL");
  DeviceScope scope(batch->plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  return batch_enqueue(batch, (hipStream_t)stream);
}

sps_status sps_batch_launch_graph(sps_batch batch, void *stream) {
  g_error.clear();
  if (!batch) return fail(SPS_ERR_INVALID_ARG, "batch is NULL");
  if (!stream) return fail(SPS_ERR_INVALID_ARG, "graph replay needs a non-null stream");
  DeviceScope scope(batch->plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  hipStream_t s = (hipStream_t)stream;
  if (!batch->exec || batch->graph_stream != s) {
    if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
    if (batch->graph) (void)hipGraphDestroy(batch->graph);
    batch->exec = nullptr;
    batch->graph = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "beginning stream capture");
    sps_status st = batch_enqueue(batch, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (st != SPS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "ending stream capture");
    e = hipGraphInstantiate(&batch->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e, "instantiating the graph");
    }
    batch->graph = g;
    batch->graph_stream = s;
  }
  hipError_t e = hipGraphLaunch(batch->exec, s);
  if (e != hipSuccess) return hip_fail(e, "launching the graph");
  return SPS_OK;
}

sps_status sps_batch_autotune(sps_batch batch, int32_t iters, void *stream, float *ms_out,
                              int32_t *n_tried) {
  g_error.clear();
  if (!batch) return fail(SPS_ERR_INVALID_ARG, "batch is NULL");
  if (iters < 1 || iters > 100) return fail(SPS_ERR_INVALID_ARG, "need 1 <= iters <= 100");
  sps_plan p = batch->plan;
  DeviceScope scope(p->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipError_t e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  float best_ms = 1e30f;
  int best = -1;
  int64_t best_pitch = 0;
  int tried = 0;
  const int nprefs = (int)(sizeof(kPrefs) / sizeof(kPrefs[0]));
  for (int i = 0; i < nprefs && e == hipSuccess; ++i) {
    const sps::DedispConfig &c = kPrefs[i];
    if (ms_out) ms_out[i] = -1.0f;
    const int64_t lp = fitted_pitch(p, c, 160 * 1024);
    if (lp <= 0 || !layout_dedisp(batch, c)) continue;
    e = hipMemcpy(batch->d_beams, batch->beams.data(),
                  sizeof(sps::BeamWork) * (size_t)batch->nbeams, hipMemcpyHostToDevice);
    sps::StagedDelays sd;
    if (e == hipSuccess)
      e = sps::stage_delays(sd, c, (int)lp, p->d_delays, p->nchan, p->ndm, p->max_delay);
    if (e == hipSuccess)  // warm-up
      e = sps::launch_dedisperse_batch(c, (int)lp, batch->d_beams, batch->nbeams,
                                       batch->dd_items, sd, p->nchan, p->ndm, batch->grid_dd, s);
    if (e == hipSuccess) e = hipEventRecord(ev0, s);
    for (int it = 0; it < iters && e == hipSuccess; ++it)
      e = sps::launch_dedisperse_batch(c, (int)lp, batch->d_beams, batch->nbeams,
                                       batch->dd_items, sd, p->nchan, p->ndm, batch->grid_dd, s);
    if (e == hipSuccess) e = hipEventRecord(ev1, s);
    if (e == hipSuccess) e = hipEventSynchronize(ev1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // before its table is freed
    sps::free_staged(sd);
    if (e != hipSuccess) break;
    ms /= (float)iters;
    if (ms_out) ms_out[i] = ms;
    ++tried;
    if (ms < best_ms) {
      best_ms = ms;
      best = i;
      best_pitch = lp;
    }
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (n_tried) *n_tried = tried;
  // keep the fastest (or restore the batch's tiling after a failure)
  const sps::DedispConfig keep = best >= 0 && e == hipSuccess ? kPrefs[best] : batch->cfg;
  const int keep_pitch = best >= 0 && e == hipSuccess ? (int)best_pitch : batch->lds_pitch;
  (void)layout_dedisp(batch, keep);  // laid out before, so it fits
  hipError_t e2 = hipMemcpy(batch->d_beams, batch->beams.data(),
                            sizeof(sps::BeamWork) * (size_t)batch->nbeams, hipMemcpyHostToDevice);
  if (e2 == hipSuccess)
    e2 = sps::stage_delays(batch->staged, keep, keep_pitch, p->d_delays, p->nchan, p->ndm,
                           p->max_delay);
  batch->cfg = keep;
  batch->lds_pitch = keep_pitch;
  // the captured graph holds the old tiling's launch
  if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
  if (batch->graph) (void)hipGraphDestroy(batch->graph);
  batch->exec = nullptr;
  batch->graph = nullptr;
  if (e != hipSuccess) return hip_fail(e, "batch autotuning");
  if (e2 != hipSuccess) return hip_fail(e2, "restaging the batch");
  if (tried == 0) return fail(SPS_ERR_RANGE, "no compiled tiling fits this plan");
  return SPS_OK;
}

sps_status sps_batch_set_tiles(sps_batch batch, uint16_t *tiles, float scale, int64_t *ntiles) {
  g_error.clear();
  if (!batch) return fail(SPS_ERR_INVALID_ARG, "batch is NULL");
  if (tiles && (!(scale > 0.0f) || !isfinite(scale)))
    return fail(SPS_ERR_INVALID_ARG, "scale must be positive and finite");
  if (ntiles) *ntiles = batch->pool_tiles;
  if (tiles != batch->tiles || scale != batch->tile_scale) {
    // the captured graph holds the other mode's launches
    DeviceScope scope(batch->plan->device);
    if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
    if (batch->graph) (void)hipGraphDestroy(batch->graph);
    batch->exec = nullptr;
    batch->graph = nullptr;
  }
  batch->tiles = tiles;
  batch->tile_scale = tiles ? scale : 0.0f;
  return SPS_OK;
}

sps_status sps_batch_candidates(sps_batch batch, int32_t beam, sps_candidate *out, int32_t cap,
                                int32_t *n_found, void *stream) {
  g_error.clear();
  if (!batch || !n_found) return fail(SPS_ERR_INVALID_ARG, "NULL argument");
  if (batch->tiles)
    return fail(SPS_ERR_INVALID_ARG, "the batch is in tile mode: it searches for no candidates");
  if (beam < 0 || beam >= batch->nbeams) return fail(SPS_ERR_RANGE, "beam out of range");
  if (cap < 0 || (cap > 0 && !out)) return fail(SPS_ERR_INVALID_ARG, "bad output array");
  DeviceScope scope(batch->plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  const sps::BeamWork &w = batch->beams[(size_t)beam];
  const int64_t ntd = (batch->plan->ndm + batch->prm.tile_dm - 1) / batch->prm.tile_dm;
  return read_candidates(batch->d_det + w.det_begin, ntd * w.ntt, batch->widths_host.data(),
                         (int)batch->widths_host.size(), batch->plan->dm.data(),
                         batch->plan->ndm, batch->plan->tsamp_s, out, cap, n_found,
                         (hipStream_t)stream);
}

sps_status sps_batch_candidates_all(sps_batch batch, sps_candidate *out, int32_t cap,
                                    int32_t *n_found, void *stream) {
  g_error.clear();
  if (!batch || !n_found) return fail(SPS_ERR_INVALID_ARG, "NULL argument");
  if (batch->tiles)
    return fail(SPS_ERR_INVALID_ARG, "the batch is in tile mode: it searches for no candidates");
  if (cap < 0 || (cap > 0 && !out)) return fail(SPS_ERR_INVALID_ARG, "bad output array");
  DeviceScope scope(batch->plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = sps::launch_gather_candidates(batch->d_beams, batch->nbeams, batch->plan->ndm,
                                               batch->prm.tile_dm, batch->d_det, kGatherRecords,
                                               batch->d_gather, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(batch->h_gather, batch->d_gather, (size_t)batch->nbeams * kGatherSlot,
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading the batch's candidates");
  const int32_t *widths = batch->widths_host.data();
  const int nw = (int)batch->widths_host.size();
  const int64_t ntd = (batch->plan->ndm + batch->prm.tile_dm - 1) / batch->prm.tile_dm;
  bool truncated = false;
  for (int bi = 0; bi < batch->nbeams; ++bi) {
    const sps::BeamWork &w = batch->beams[(size_t)bi];
    const int64_t ntiles = ntd * w.ntt;
    const uint8_t *slot = batch->h_gather + (size_t)bi * kGatherSlot;
    int32_t status[4];
    memcpy(status, slot, sizeof status);
    const int32_t na = status[1];
    if (na < 0 || (int64_t)na > ntiles || status[0] < na) {
      n_found[bi] = 0;
      return fail(SPS_ERR_DEVICE, "beam %d: detection status is inconsistent", bi);
    }
    const int32_t ncopy = na < cap ? na : cap;
    const int64_t held = ntiles < kGatherRecords ? ntiles : kGatherRecords;
    sps_candidate *dst = out ? out + (int64_t)bi * cap : nullptr;
    if (ncopy <= held) {
      const sps::TilePeak *rec = reinterpret_cast<const sps::TilePeak *>(slot + sps::kGatherHeader);
      for (int32_t k = 0; k < ncopy; ++k)
        dst[k] = to_candidate(rec[k], widths, nw, batch->plan->dm.data(), batch->plan->ndm,
                              batch->plan->tsamp_s);
      n_found[bi] = na;
    } else {
      // more accepted offers than the slot holds: this beam's own copies
      const sps_status st =
          read_candidates(batch->d_det + w.det_begin, ntiles, widths, nw, batch->plan->dm.data(),
                          batch->plan->ndm, batch->plan->tsamp_s, dst, cap, &n_found[bi], s);
      if (st != SPS_OK && st != SPS_ERR_TRUNCATED) return st;
      g_error.clear();
    }
    truncated = truncated || na > cap;
  }
  if (truncated) return fail(SPS_ERR_TRUNCATED, "a beam found more than %d candidates", cap);
  return SPS_OK;
}


sps_status sps_plan_autotune(sps_plan plan, int64_t nout_probe, int32_t iters, void *stream,
                             float *ms_out, int32_t *n_tried) {
  g_error.clear();
  if (!plan) return fail(SPS_ERR_INVALID_ARG, "plan is NULL");
  if (nout_probe < 1 || nout_probe > (1 << 26) || iters < 1 || iters > 100)
    return fail(SPS_ERR_INVALID_ARG, "need 1 <= nout_probe <= 2^26 and 1 <= iters <= 100");
  DeviceScope scope(plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nsamp = nout_probe + std::max(plan->max_delay, plan->eff_max_delay);
  const int64_t pitch = (nsamp + 255) / 256 * 256;
  uint8_t *X = nullptr;
  uint32_t *Y = nullptr;
  hipError_t e = hipMalloc(&X, (size_t)pitch * plan->nchan);
  if (e == hipSuccess) e = hipMalloc(&Y, sizeof(uint32_t) * (size_t)plan->ndm * nout_probe);
  if (e == hipSuccess) e = hipMemsetAsync(X, 0x5A, (size_t)pitch * plan->nchan, s);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&ev0);
  if (e == hipSuccess) e = hipEventCreate(&ev1);
  float best_ms = 1e30f;
  sps::DedispConfig best_cfg = plan->cfg;
  int best_pitch = plan->lds_pitch;
  int tried = 0;
  const int nprefs = (int)(sizeof(kPrefs) / sizeof(kPrefs[0]));
  for (int i = 0; i < nprefs && e == hipSuccess; ++i) {
    const sps::DedispConfig &c = kPrefs[i];
    const int64_t lp = fitted_pitch(plan, c, 160 * 1024);
    if (ms_out) ms_out[i] = -1.0f;
    if (lp <= 0) continue;
    sps::StagedDelays sd;
    e = sps::stage_delays(sd, c, (int)lp, plan->d_delays, plan->nchan, plan->ndm,
                          plan->max_delay);
    if (e == hipSuccess)
      e = sps::launch_dedisperse(c, (int)lp, X, pitch, nsamp, plan->d_delays, &sd, plan->nchan,
                                 plan->ndm, Y, nout_probe, s);  // warm-up
    float total = 0.0f;
    for (int it = 0; it < iters && e == hipSuccess; ++it) {
      e = hipEventRecord(ev0, s);
      if (e == hipSuccess)
        e = sps::launch_dedisperse(c, (int)lp, X, pitch, nsamp, plan->d_delays, &sd, plan->nchan,
                                   plan->ndm, Y, nout_probe, s);
      if (e == hipSuccess) e = hipEventRecord(ev1, s);
      if (e == hipSuccess) e = hipEventSynchronize(ev1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
      total += ms;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // before its table is freed
    sps::free_staged(sd);
    if (e != hipSuccess) break;
    const float mean = total / (float)iters;
    if (ms_out) ms_out[i] = mean;
    ++tried;
    if (mean < best_ms) {
      best_ms = mean;
      best_cfg = c;
      best_pitch = (int)lp;
    }
  }
  // Subband plans: stage 1 in one segmented launch against one launch per
  // subband (each with its own tiling), on the same probe; the faster stays.
  sps_status sub_st = SPS_OK;
  if (e == hipSuccess && plan->subband && plan->fused) {
    float t_form[2] = {0.0f, 0.0f};
    for (int f = 0; f < 2 && e == hipSuccess && sub_st == SPS_OK; ++f) {
      plan->use_fused = f == 0;
      sub_st = sps_dedisperse_subband(plan, X, pitch, nsamp, Y, nout_probe, 0, stream);  // warm-up
      if (sub_st == SPS_OK) e = hipEventRecord(ev0, s);
      for (int it = 0; it < iters && e == hipSuccess && sub_st == SPS_OK; ++it)
        sub_st = sps_dedisperse_subband(plan, X, pitch, nsamp, Y, nout_probe, 0, stream);
      if (e == hipSuccess && sub_st == SPS_OK) e = hipEventRecord(ev1, s);
      if (e == hipSuccess && sub_st == SPS_OK) e = hipEventSynchronize(ev1);
      if (e == hipSuccess && sub_st == SPS_OK) e = hipEventElapsedTime(&t_form[f], ev0, ev1);
    }
    plan->use_fused = !(e == hipSuccess && sub_st == SPS_OK) || t_form[0] <= t_form[1];
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (X) (void)hipFree(X);
  if (Y) (void)hipFree(Y);
  if (n_tried) *n_tried = tried;
  if (e != hipSuccess) return hip_fail(e, "autotuning");
  if (sub_st != SPS_OK) return sub_st;  // the subband call recorded its message
  if (tried == 0) return fail(SPS_ERR_RANGE, "no compiled tiling fits this plan");
  plan->cfg = best_cfg;
  plan->lds_pitch = best_pitch;
  return restage(plan);
}

int32_t sps_tiling_count(void) { return (int32_t)(sizeof(kPrefs) / sizeof(kPrefs[0])); }

sps_status sps_tiling_describe(int32_t index, int32_t *m, int32_t *dpw, int32_t *nw, int32_t *cs,
                               int32_t *waves_per_eu) {
  g_error.clear();
  if (index < 0 || index >= sps_tiling_count()) return fail(SPS_ERR_RANGE, "index out of range");
  const sps::DedispConfig &c = kPrefs[index];
  if (m) *m = c.m;
  if (dpw) *dpw = c.dpw;
  if (nw) *nw = c.nw;
  if (cs) *cs = c.cs;
  if (waves_per_eu) *waves_per_eu = c.wpe;
  return SPS_OK;
}

sps_status sps_probe_peaks(int32_t device, double *rates, int32_t n) {
  g_error.clear();
  if (!rates) return fail(SPS_ERR_INVALID_ARG, "rates is NULL");
  if (n < SPS_PROBE_COUNT) return fail(SPS_ERR_INVALID_ARG, "rates needs %d entries", SPS_PROBE_COUNT);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "counting devices");
  if (device < 0 || device >= ndev) return fail(SPS_ERR_INVALID_ARG, "no device %d", device);
  DeviceScope scope(device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the device");
  hipStream_t s = nullptr;
  e = hipStreamCreate(&s);
  if (e == hipSuccess) e = sps::probe_device_peaks(rates, s);
  if (s) (void)hipStreamDestroy(s);
  if (e != hipSuccess) return hip_fail(e, "device probes");
  return SPS_OK;
}

}  // extern "C"

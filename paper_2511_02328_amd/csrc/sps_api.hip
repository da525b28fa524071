// sps_api.hip -- the C ABI (include/sps.h): plans, argument checks, launches.
//
// Host-side work is limited to what the ABI promises: the integer delay table
// of Eq. (KDM) / Eq. (coarse_delay) (ASTROFLOW Sec. 2.3), computed once per
// plan in IEEE double and uploaded, argument validation before anything is
// enqueued, and turning the detection kernels' output into candidate
// records.  Every step of the search itself runs in the HIP kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

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
  // detection scratch
  sps::TilePeak *d_peaks = nullptr;
  int64_t peaks_cap = 0;
  sps::TilePeak *d_accepted = nullptr;
  int32_t *d_status = nullptr;
};

namespace {

void free_plan(sps_plan p) {
  if (!p) return;
  if (p->d_delays) (void)hipFree(p->d_delays);
  if (p->d_stats) (void)hipFree(p->d_stats);
  if (p->d_peaks) (void)hipFree(p->d_peaks);
  if (p->d_accepted) (void)hipFree(p->d_accepted);
  if (p->d_status) (void)hipFree(p->d_status);
  delete p;
}

// Compiled tilings in order of preference (see dedisperse.hip).
const sps::DedispConfig kPrefs[] = {
    {5, 1, 16, 16, 2, 8}, {5, 2, 8, 16, 2, 4}, {5, 1, 16, 16, 2, 4}, {5, 2, 16, 16, 2, 4},
    {5, 2, 8, 16, 4, 4}, {5, 1, 16, 16, 4, 4}, {3, 2, 8, 16, 2, 4}, {3, 1, 16, 16, 2, 8},
    {7, 1, 16, 16, 3, 4}};

// Staged-row bytes of config c for this plan, or -1 if it does not fit.
int64_t fitted_pitch(sps_plan p, const sps::DedispConfig &c, int64_t lds_budget) {
  const int spread = sps::dedisp_block_spread(p->delays.data(), p->nchan, p->ndm, c.nd());
  const int64_t pitch = sps::dedisp_lds_pitch(c, spread);
  if (pitch > 1024 * (int64_t)c.kmax || c.lds_bytes(pitch) > lds_budget) return -1;
  return pitch;
}

// Picks the first preferred tiling whose double-buffered slab fits the LDS
// budget (64 KiB keeps two workgroups per CU; up to 160 KiB is allowed
// next); otherwise the plain global-memory kernel is used.
sps_status choose_tiling(sps_plan p) {
  for (int64_t budget : {(int64_t)64 * 1024, (int64_t)160 * 1024}) {
    for (const auto &c : kPrefs) {
      const int64_t pitch = fitted_pitch(p, c, budget);
      if (pitch > 0) {
        p->cfg = c;
        p->lds_pitch = (int)pitch;
        return SPS_OK;
      }
    }
  }
  p->cfg = sps::DedispConfig{0, 0, 0, 0, 0, 0};
  p->lds_pitch = 0;
  return SPS_OK;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

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
    return SPS_OK;
  }
  bool known = false;
  for (const auto &c : kPrefs) {
    if (c.m != m || c.dpw != dpw || c.nw != nw || c.cs != cs) continue;
    if (waves_per_eu != 0 && c.wpe != waves_per_eu) continue;
    known = true;
    const int64_t pitch = fitted_pitch(plan, c, 160 * 1024);
    if (pitch > 0) {
      plan->cfg = c;
      plan->lds_pitch = (int)pitch;
      return SPS_OK;
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
                                        plan->d_delays, plan->nchan, plan->ndm, Y, nout,
                                        (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "dedispersion launch");
  return SPS_OK;
}

sps_status sps_boxcar_snr(sps_plan plan, const uint32_t *Y, int64_t nout, const int32_t *widths,
                          int32_t nw, float *snr, uint8_t *best_w, int32_t *stats,
                          void *stream) {
  g_error.clear();
  if (!plan || !Y || !widths || !snr || !best_w)
    return fail(SPS_ERR_INVALID_ARG, "NULL plan or buffer");
  if (nout < 1 || nout > 0x7FFFFFFF) return fail(SPS_ERR_RANGE, "nout must be in [1, 2^31-1]");
  if (nw < 1 || nw > sps::kMaxWidths)
    return fail(SPS_ERR_INVALID_ARG, "nw must be in [1, %d]", sps::kMaxWidths);
  sps::WidthList wl;
  wl.n = nw;
  for (int i = 0; i < nw; ++i) {
    wl.w[i] = widths[i];
    if (widths[i] < 1) return fail(SPS_ERR_INVALID_ARG, "widths must be >= 1");
    if (i > 0 && widths[i] <= widths[i - 1])
      return fail(SPS_ERR_INVALID_ARG, "widths must be strictly ascending");
  }
  for (int i = nw; i < sps::kMaxWidths; ++i) wl.w[i] = 0;
  const int64_t wmax = widths[nw - 1];
  if (wmax > nout || wmax > sps::kMaxWidth)
    return fail(SPS_ERR_RANGE, "largest width %lld exceeds nout or %d", (long long)wmax,
                sps::kMaxWidth);
  const uint32_t vmax = 255u * (uint32_t)plan->nchan;
  if ((uint64_t)wmax * vmax >= (1ull << 31))
    return fail(SPS_ERR_OVERFLOW, "width %lld x 255 x nchan reaches 2^31", (long long)wmax);
  DeviceScope scope(plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  int32_t *st = stats ? stats : plan->d_stats;
  hipError_t e = sps::launch_row_stats(Y, plan->ndm, nout, vmax, st, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "row statistics launch");
  e = sps::launch_boxcar(Y, plan->ndm, nout, st, wl, snr, best_w, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "boxcar launch");
  return SPS_OK;
}

sps_status sps_detect(sps_plan plan, const float *snr, const uint8_t *best_w, int64_t nout,
                      const int32_t *widths, int32_t nw, const sps_detect_params *prm,
                      sps_candidate *out, int32_t cap, int32_t *n_found, void *stream) {
  g_error.clear();
  if (!plan || !snr || !best_w || !widths || !prm || !n_found)
    return fail(SPS_ERR_INVALID_ARG, "NULL plan, buffer or parameter");
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
  const int64_t ntt = (nout + prm->tile_t - 1) / prm->tile_t;
  const int64_t ntiles = ntd * ntt;
  if (ntiles > 0x7FFFFFFF) return fail(SPS_ERR_RANGE, "too many tiles");
  DeviceScope scope(plan->device);
  if (scope.err != hipSuccess) return hip_fail(scope.err, "selecting the plan's device");
  hipError_t e = hipSuccess;
  if (!plan->d_accepted) {
    e = hipMalloc(&plan->d_accepted, sizeof(sps::TilePeak) * sps::kMaxOffers);
    if (e == hipSuccess) e = hipMalloc(&plan->d_status, 4 * sizeof(int32_t));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SPS_ERR_NOMEM, "device allocation of detection scratch failed");
    }
  }
  if (plan->peaks_cap < ntiles) {
    if (plan->d_peaks) (void)hipFree(plan->d_peaks);
    plan->d_peaks = nullptr;
    plan->peaks_cap = 0;
    e = hipMalloc(&plan->d_peaks, sizeof(sps::TilePeak) * (size_t)ntiles);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SPS_ERR_NOMEM, "device allocation of tile peaks failed");
    }
    plan->peaks_cap = ntiles;
  }
  hipStream_t s = (hipStream_t)stream;
  e = sps::launch_tile_peaks(snr, best_w, plan->ndm, nout, prm->tile_dm, prm->tile_t,
                             plan->d_peaks, s);
  if (e != hipSuccess) return hip_fail(e, "tile peak launch");
  e = sps::launch_select_nms(plan->d_peaks, plan->ndm, nout, prm->tile_dm, prm->tile_t,
                             prm->threshold, prm->nms_dm, prm->nms_t, plan->d_accepted,
                             plan->d_status, s);
  if (e != hipSuccess) return hip_fail(e, "selection launch");
  int32_t status[4] = {0, 0, 0, 0};
  e = hipMemcpyAsync(status, plan->d_status, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading detection status");
  if (status[2]) {
    *n_found = 0;
    return fail(SPS_ERR_RANGE, "%d tiles reach the threshold; at most %d are supported", status[0],
                sps::kMaxOffers);
  }
  const int32_t na = status[1];
  const int32_t ncopy = na < cap ? na : cap;
  std::vector<sps::TilePeak> acc((size_t)ncopy);
  if (ncopy > 0) {
    e = hipMemcpyAsync(acc.data(), plan->d_accepted, sizeof(sps::TilePeak) * (size_t)ncopy,
                       hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading candidates");
  }
  for (int32_t i = 0; i < ncopy; ++i) {
    const sps::TilePeak &q = acc[(size_t)i];
    sps_candidate c;
    c.dm_idx = q.d;
    c.t_idx = q.t;
    c.width = (q.w >= 0 && q.w < nw) ? widths[q.w] : 0;
    c.snr = q.snr;
    c.reserved = 0.0f;
    c.dm = (q.d >= 0 && q.d < plan->ndm) ? plan->dm[(size_t)q.d] : 0.0;
    c.toa_s = ((double)q.t + 0.5 * (double)c.width) * plan->tsamp_s;
    out[i] = c;
  }
  *n_found = na;
  if (na > cap) return fail(SPS_ERR_TRUNCATED, "%d candidates found, %d returned", na, cap);
  return SPS_OK;
}

}  // extern "C"

/*
 * sps_oracle.c -- plain CPU oracle for the single-pulse search hot path.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library.  It shares
 * no source, header, table or helper with the GPU library; the two meet only
 * through seeded inputs.
 *
 * Everything here is the plain definition of each step written out with
 * obvious loops, in double precision wherever floating point appears:
 *
 *   delays      Sec. 2.3, Eq. (KDM) and Eq. (coarse_delay): integer sample
 *               delay per (trial DM, channel).
 *   dedisperse  Sec. 2.3, the brute-force method (cost N_DM N_t N_f), with the
 *               "zero outside bounds" convention of Eq. (stage1).
 *   stats       per-DM-row lower median and median absolute deviation (the
 *               paper gives no S/N definition; the reading is stated below).
 *   boxcar      Sec. 1, step (iii) of the standard workflow: matched filtering
 *               of every dedispersed series with boxcars of several widths,
 *               by direct summation of each window.
 *   detect      tile maxima above a threshold, greedy suppression of
 *               neighbours; the candidate record carries DM, arrival time at
 *               the top of the band (Sec. 2, candidate record), width, S/N.
 *   checksums   sum over time of each dedispersed row, from per-channel
 *               prefix sums: a property that holds at any size.
 *
 * Readings of points the paper leaves open (each one also listed in the
 * design notes):
 *   - K_DM is printed as 4.148808e3 "ms MHz^2"; with f in MHz that gives
 *     millisecond-scale delays for a 500 MHz band at DM 1000, which is
 *     physically wrong by 10^3.  Taken as 4.148808e3 s MHz^2 pc^-1 cm^3.
 *   - "round" is taken as round-half-up, floor(x + 1/2); x >= 0 always
 *     because every channel lies at or below f_ref.
 *   - x is evaluated as (K DM / t_samp) * (1/f^2 - 1/f_ref^2), in the order
 *     Eq. (coarse_delay) is written, in IEEE double without contraction.
 *   - S/N of width w at start t: (B_w(t) - w*med) / (1.4826 * MAD * sqrt(w)),
 *     med the lower median (rank floor((n-1)/2)) of the row, MAD the lower
 *     median of |Y - med|; only full windows t + w <= nout are formed; the
 *     best width is the smallest one attaining the maximum, the comparison
 *     taken on values rounded to binary32 (the precision the S/N is
 *     delivered in); a row with MAD = 0 has S/N 0 everywhere.
 *   - where no width fits (t + widths[0] > nout) S/N is 0 and the width
 *     index is 0xFF.
 *
 * Build: gcc -O2 -std=c99 -fopenmp -ffp-contract=off -fPIC -shared -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)
#define ORACLE_EOVERFLOW (-3)

/* Dispersion constant in s MHz^2 pc^-1 cm^3 (reading of Eq. KDM's unit). */
static const double ORACLE_K_DM = 4.148808e3;
/* Scale from MAD to the standard deviation of a normal distribution. */
static const double ORACLE_MAD_TO_SIGMA = 1.4826;

/* Sec. 2.3, Eq. (KDM) / Eq. (coarse_delay). D is [ndm][nchan], row-major. */
int sps_oracle_delays(int32_t nchan, const double *freq_mhz, double fref_mhz,
                      double tsamp_s, int32_t ndm, const double *dm,
                      int32_t *D) {
  if (nchan <= 0 || ndm <= 0 || !freq_mhz || !dm || !D) return ORACLE_EINVAL;
  if (!(tsamp_s > 0.0) || !(fref_mhz > 0.0)) return ORACLE_EINVAL;
  for (int32_t c = 0; c < nchan; ++c)
    if (!(freq_mhz[c] > 0.0) || freq_mhz[c] > fref_mhz) return ORACLE_EINVAL;
  for (int32_t d = 0; d < ndm; ++d)
    if (!(dm[d] >= 0.0)) return ORACLE_EINVAL;

  for (int32_t d = 0; d < ndm; ++d) {
    for (int32_t c = 0; c < nchan; ++c) {
      double f = freq_mhz[c];
      double k = 1.0 / (f * f) - 1.0 / (fref_mhz * fref_mhz);
      double x = (ORACLE_K_DM * dm[d] / tsamp_s) * k;
      double r = floor(x + 0.5);
      if (r > 2147483647.0) return ORACLE_EOVERFLOW;
      D[(int64_t)d * nchan + c] = (int32_t)r;
    }
  }
  return ORACLE_OK;
}

/*
 * Sec. 2.3 brute force: Y[d][t] = sum_c X[c][t + D[d][c]] for t in [0, nout);
 * an index at or past nsamp_in contributes zero.  X is [nchan][pitch] uint8,
 * Y is [ndm][nout] uint32.  Sums are formed in 64 bits and must fit 32.
 */
int sps_oracle_dedisperse(int32_t nchan, const uint8_t *X, int64_t pitch,
                          int64_t nsamp_in, int32_t ndm, const int32_t *D,
                          int64_t nout, uint32_t *Y) {
  if (nchan <= 0 || ndm <= 0 || nout < 0 || nsamp_in < 0 || pitch < nsamp_in)
    return ORACLE_EINVAL;
  if (!X || !D || !Y) return ORACLE_EINVAL;
  int err = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t d = 0; d < ndm; ++d) {
    uint64_t *acc = (uint64_t *)calloc((size_t)(nout > 0 ? nout : 1), sizeof(uint64_t));
    if (!acc) {
#pragma omp atomic write
      err = ORACLE_ENOMEM;
      continue;
    }
    for (int32_t c = 0; c < nchan; ++c) {
      const uint8_t *row = X + (int64_t)c * pitch;
      int64_t shift = D[(int64_t)d * nchan + c];
      for (int64_t t = 0; t < nout; ++t) {
        int64_t idx = t + shift;
        if (idx < nsamp_in) acc[t] += row[idx];
      }
    }
    for (int64_t t = 0; t < nout; ++t) {
      if (acc[t] > 0xFFFFFFFFull) {
#pragma omp atomic write
        err = ORACLE_EOVERFLOW;
      }
      Y[(int64_t)d * nout + t] = (uint32_t)acc[t];
    }
    free(acc);
  }
  return err;
}

static int cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return (x > y) - (x < y);
}

/*
 * Per-row lower median and MAD. stats is [ndm][2] int64: (median, MAD).
 * Median = element of rank floor((n-1)/2) of the sorted row; MAD = the same
 * rank of the sorted absolute deviations from that median.
 */
int sps_oracle_stats(int32_t ndm, int64_t nout, const uint32_t *Y,
                     int64_t *stats) {
  if (ndm <= 0 || nout <= 0 || !Y || !stats) return ORACLE_EINVAL;
  int err = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t d = 0; d < ndm; ++d) {
    uint32_t *tmp = (uint32_t *)malloc((size_t)nout * sizeof(uint32_t));
    if (!tmp) {
#pragma omp atomic write
      err = ORACLE_ENOMEM;
      continue;
    }
    const uint32_t *row = Y + (int64_t)d * nout;
    int64_t k = (nout - 1) / 2;
    memcpy(tmp, row, (size_t)nout * sizeof(uint32_t));
    qsort(tmp, (size_t)nout, sizeof(uint32_t), cmp_u32);
    uint32_t med = tmp[k];
    for (int64_t t = 0; t < nout; ++t)
      tmp[t] = row[t] >= med ? row[t] - med : med - row[t];
    qsort(tmp, (size_t)nout, sizeof(uint32_t), cmp_u32);
    stats[2 * (int64_t)d] = med;
    stats[2 * (int64_t)d + 1] = tmp[k];
    free(tmp);
  }
  return err;
}

/*
 * Boxcar matched filter (Sec. 1, step iii) with median/MAD normalisation.
 * widths: nw strictly ascending, >= 1.  For each (d, t) the S/N of every
 * width w with t + w <= nout is formed from the directly summed window;
 * snr[d][t] is the largest (as binary32), best[d][t] the index of the
 * smallest width attaining it.  snr64 (optional) receives the same maximum
 * before rounding.
 */
int sps_oracle_boxcar(int32_t ndm, int64_t nout, const uint32_t *Y,
                      const int64_t *stats, int32_t nw, const int32_t *widths,
                      float *snr, uint8_t *best, double *snr64) {
  if (ndm <= 0 || nout <= 0 || nw <= 0 || nw > 255 || !Y || !stats ||
      !widths || !snr || !best)
    return ORACLE_EINVAL;
  for (int32_t i = 0; i < nw; ++i) {
    if (widths[i] < 1) return ORACLE_EINVAL;
    if (i > 0 && widths[i] <= widths[i - 1]) return ORACLE_EINVAL;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t d = 0; d < ndm; ++d) {
    const uint32_t *row = Y + (int64_t)d * nout;
    double med = (double)stats[2 * (int64_t)d];
    double mad = (double)stats[2 * (int64_t)d + 1];
    double sigma = ORACLE_MAD_TO_SIGMA * mad;
    for (int64_t t = 0; t < nout; ++t) {
      float best_f = 0.0f;
      double best_d = 0.0;
      int best_i = 0xFF;
      for (int32_t i = 0; i < nw; ++i) {
        int64_t w = widths[i];
        if (t + w > nout) break;
        int64_t B = 0;
        for (int64_t k = 0; k < w; ++k) B += row[t + k];
        double s = 0.0;
        if (mad > 0.0) s = ((double)B - (double)w * med) / (sigma * sqrt((double)w));
        float f = (float)s;
        if (best_i == 0xFF || f > best_f) {
          best_f = f;
          best_d = s;
          best_i = i;
        }
      }
      snr[(int64_t)d * nout + t] = best_f;
      best[(int64_t)d * nout + t] = (uint8_t)best_i;
      if (snr64) snr64[(int64_t)d * nout + t] = best_d;
    }
  }
  return ORACLE_OK;
}

typedef struct {
  float snr;
  int64_t t;
  int32_t d;
} oracle_peak;

/* Order: S/N descending, then t ascending, then d ascending. */
static int cmp_peak(const void *a, const void *b) {
  const oracle_peak *p = (const oracle_peak *)a, *q = (const oracle_peak *)b;
  if (p->snr != q->snr) return p->snr > q->snr ? -1 : 1;
  if (p->t != q->t) return p->t < q->t ? -1 : 1;
  return (p->d > q->d) - (p->d < q->d);
}

/*
 * Candidate detection.  The plane is cut into tiles of tile_dm rows by
 * tile_t samples (the last ones ragged).  Each tile contributes its largest
 * S/N (ties: smallest t, then smallest d) when it reaches the threshold.
 * These peaks, taken in the order above, are accepted greedily unless an
 * already accepted one lies within |dd| <= nms_dm and |dt| <= nms_t.
 * Outputs (first min(count, cap) accepted, in acceptance order): DM index,
 * time index, width index, S/N.  *n_found = number accepted.
 */
int sps_oracle_detect(int32_t ndm, int64_t nout, const float *snr,
                      const uint8_t *best, float threshold, int32_t tile_dm,
                      int64_t tile_t, int32_t nms_dm, int64_t nms_t,
                      int32_t cap, int32_t *out_d, int64_t *out_t,
                      int32_t *out_w, float *out_snr, int64_t *n_found) {
  if (ndm <= 0 || nout <= 0 || !snr || !best || tile_dm <= 0 || tile_t <= 0 ||
      nms_dm < 0 || nms_t < 0 || cap < 0 || !n_found)
    return ORACLE_EINVAL;
  int64_t ntd = (ndm + tile_dm - 1) / tile_dm;
  int64_t ntt = (nout + tile_t - 1) / tile_t;
  oracle_peak *peaks = (oracle_peak *)malloc((size_t)(ntd * ntt) * sizeof(oracle_peak));
  oracle_peak *acc = (oracle_peak *)malloc((size_t)(ntd * ntt) * sizeof(oracle_peak));
  if (!peaks || !acc) {
    free(peaks);
    free(acc);
    return ORACLE_ENOMEM;
  }
  int64_t np = 0;
  for (int64_t a = 0; a < ntd; ++a) {
    for (int64_t b = 0; b < ntt; ++b) {
      int32_t d0 = (int32_t)(a * tile_dm);
      int32_t d1 = d0 + tile_dm < ndm ? d0 + tile_dm : ndm;
      int64_t t0 = b * tile_t;
      int64_t t1 = t0 + tile_t < nout ? t0 + tile_t : nout;
      oracle_peak best_p = {0.0f, -1, -1};
      /* scan t outer, d inner, strict '>': the first maximum found has the
         smallest t, then the smallest d */
      for (int64_t t = t0; t < t1; ++t) {
        for (int32_t d = d0; d < d1; ++d) {
          float v = snr[(int64_t)d * nout + t];
          if (best_p.t < 0 || v > best_p.snr) {
            best_p.snr = v;
            best_p.t = t;
            best_p.d = d;
          }
        }
      }
      if (best_p.snr >= threshold) peaks[np++] = best_p;
    }
  }
  qsort(peaks, (size_t)np, sizeof(oracle_peak), cmp_peak);
  int64_t na = 0;
  for (int64_t i = 0; i < np; ++i) {
    int keep = 1;
    for (int64_t j = 0; j < na && keep; ++j) {
      int64_t dd = peaks[i].d - acc[j].d;
      int64_t dt = peaks[i].t - acc[j].t;
      if (dd < 0) dd = -dd;
      if (dt < 0) dt = -dt;
      if (dd <= nms_dm && dt <= nms_t) keep = 0;
    }
    if (keep) acc[na++] = peaks[i];
  }
  for (int64_t j = 0; j < na && j < cap; ++j) {
    if (out_d) out_d[j] = acc[j].d;
    if (out_t) out_t[j] = acc[j].t;
    if (out_w) out_w[j] = best[(int64_t)acc[j].d * nout + acc[j].t];
    if (out_snr) out_snr[j] = acc[j].snr;
  }
  *n_found = na;
  free(peaks);
  free(acc);
  return ORACLE_OK;
}

/*
 * Row sums of the dedispersed plane without forming it:
 *   sum_t Y[d][t] = sum_c (S_c[min(D+nout, n)] - S_c[min(D, n)]),
 * S_c the prefix sums of channel c over its first n = nsamp_in samples.
 */
int sps_oracle_row_checksums(int32_t nchan, const uint8_t *X, int64_t pitch,
                             int64_t nsamp_in, int32_t ndm, const int32_t *D,
                             int64_t nout, uint64_t *sums) {
  if (nchan <= 0 || ndm <= 0 || nout < 0 || nsamp_in < 0 || pitch < nsamp_in ||
      !X || !D || !sums)
    return ORACLE_EINVAL;
  int err = ORACLE_OK;
  for (int32_t d = 0; d < ndm; ++d) sums[d] = 0;
#pragma omp parallel
  {
    uint64_t *Sc = (uint64_t *)malloc((size_t)(nsamp_in + 1) * sizeof(uint64_t));
    uint64_t *part = (uint64_t *)calloc((size_t)ndm, sizeof(uint64_t));
    if (!Sc || !part) {
#pragma omp atomic write
      err = ORACLE_ENOMEM;
    }
#pragma omp for schedule(dynamic, 1)
    for (int32_t c = 0; c < nchan; ++c) {
      if (!Sc || !part) continue;
      const uint8_t *row = X + (int64_t)c * pitch;
      Sc[0] = 0;
      for (int64_t i = 0; i < nsamp_in; ++i) Sc[i + 1] = Sc[i] + row[i];
      for (int32_t d = 0; d < ndm; ++d) {
        int64_t lo = D[(int64_t)d * nchan + c];
        int64_t hi = lo + nout;
        if (lo > nsamp_in) lo = nsamp_in;
        if (hi > nsamp_in) hi = nsamp_in;
        part[d] += Sc[hi] - Sc[lo];
      }
    }
#pragma omp critical
    {
      if (part)
        for (int32_t d = 0; d < ndm; ++d) sums[d] += part[d];
    }
    free(Sc);
    free(part);
  }
  return err;
}

/* Number of threads a parallel region here uses (1 without OpenMP). */
int sps_oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * The paper's own dedispersion (Sec. 2.3): two-stage subband method, and the
 * pre-dedispersion steps of Sec. 2.1 / Sec. 2.2.
 * ------------------------------------------------------------------------- */

/*
 * Residual shift table of Eq. (residual).  Fine grid DM_m = dm_lo + m*ddm,
 * coarse grid DM_j = dm_lo + j*n0*ddm, j(m) = floor(m / n0), and
 * dDM_m = DM_m - DM_j(m).  Subband s holds channels [sub[s], sub[s+1]) and is
 * represented by F_s with 1/F_s^2 = mean of 1/f_c^2 over its channels (the
 * "1/f^2-weighted centre").  R[m][s] = floor(K dDM_m / t_samp (1/F_s^2 -
 * 1/f_ref^2) + 1/2).  F (optional) receives F_s.  Coarse DMs are returned in
 * dm_coarse[ceil(ndm / n0)] (optional).
 */
int sps_oracle_subband_residuals(int32_t nchan, const double *freq_mhz, double fref_mhz,
                                 double tsamp_s, int32_t nsub, const int32_t *sub,
                                 int32_t ndm, double dm_lo, double ddm, int32_t n0,
                                 int32_t *R, double *F, double *dm_coarse) {
  if (nchan <= 0 || nsub <= 0 || ndm <= 0 || n0 <= 0 || !freq_mhz || !sub || !R)
    return ORACLE_EINVAL;
  if (!(tsamp_s > 0.0) || !(ddm >= 0.0) || !(dm_lo >= 0.0)) return ORACLE_EINVAL;
  if (sub[0] != 0 || sub[nsub] != nchan) return ORACLE_EINVAL;
  for (int32_t s = 0; s < nsub; ++s)
    if (sub[s + 1] <= sub[s]) return ORACLE_EINVAL;
  for (int32_t c = 0; c < nchan; ++c)
    if (!(freq_mhz[c] > 0.0) || freq_mhz[c] > fref_mhz) return ORACLE_EINVAL;
  int32_t ncoarse = (ndm + n0 - 1) / n0;
  if (dm_coarse)
    for (int32_t j = 0; j < ncoarse; ++j) dm_coarse[j] = dm_lo + (double)j * (double)n0 * ddm;
  for (int32_t s = 0; s < nsub; ++s) {
    double acc = 0.0;
    for (int32_t c = sub[s]; c < sub[s + 1]; ++c) acc += 1.0 / (freq_mhz[c] * freq_mhz[c]);
    double inv_f2 = acc / (double)(sub[s + 1] - sub[s]);
    if (F) F[s] = 1.0 / sqrt(inv_f2);
    double k = inv_f2 - 1.0 / (fref_mhz * fref_mhz);
    for (int32_t m = 0; m < ndm; ++m) {
      double dm_m = dm_lo + (double)m * ddm;
      double dm_j = dm_lo + (double)((m / n0) * n0) * ddm;
      double x = (ORACLE_K_DM * (dm_m - dm_j) / tsamp_s) * k;
      double r = floor(x + 0.5);
      if (r > 2147483647.0 || r < 0.0) return ORACLE_EOVERFLOW;
      R[(int64_t)m * nsub + s] = (int32_t)r;
    }
  }
  return ORACLE_OK;
}

/*
 * Two-stage subband dedispersion, Eq. (stage1) and Eq. (stage2), without
 * time blocking (blocking with the overlap of Eq. L1 gives the same values).
 *   Stage 1: I[j][s][u] = sum_{c in s} X[c][u + Dc[j][c]], zero past nsamp_in,
 *            for u in [0, nout + max R).
 *   Stage 2: Y[m][t] = sum_s I[j(m)][s][t + R[m][s]].
 * Dc is the coarse-grid delay table [ncoarse][nchan] (from
 * sps_oracle_delays on the coarse DMs).
 */
int sps_oracle_subband_dedisperse(int32_t nchan, const uint8_t *X, int64_t pitch,
                                  int64_t nsamp_in, int32_t ncoarse, const int32_t *Dc,
                                  int32_t nsub, const int32_t *sub, int32_t ndm, int32_t n0,
                                  const int32_t *R, int64_t nout, uint32_t *Y) {
  if (nchan <= 0 || ncoarse <= 0 || nsub <= 0 || ndm <= 0 || n0 <= 0 || nout < 0 ||
      !X || !Dc || !sub || !R || !Y || pitch < nsamp_in || (ndm + n0 - 1) / n0 > ncoarse)
    return ORACLE_EINVAL;
  int32_t rmax = 0;
  for (int64_t i = 0; i < (int64_t)ndm * nsub; ++i)
    if (R[i] > rmax) rmax = R[i];
  int64_t len = nout + rmax;
  uint64_t *I = (uint64_t *)calloc((size_t)ncoarse * nsub * (size_t)(len > 0 ? len : 1), sizeof(uint64_t));
  if (!I) return ORACLE_ENOMEM;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t j = 0; j < ncoarse; ++j) {
    for (int32_t s = 0; s < nsub; ++s) {
      uint64_t *row = I + ((int64_t)j * nsub + s) * len;
      for (int32_t c = sub[s]; c < sub[s + 1]; ++c) {
        const uint8_t *x = X + (int64_t)c * pitch;
        int64_t shift = Dc[(int64_t)j * nchan + c];
        for (int64_t u = 0; u < len; ++u)
          if (u + shift < nsamp_in) row[u] += x[u + shift];
      }
    }
  }
  int err = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t m = 0; m < ndm; ++m) {
    int32_t j = m / n0;
    for (int64_t t = 0; t < nout; ++t) {
      uint64_t acc = 0;
      for (int32_t s = 0; s < nsub; ++s)
        acc += I[((int64_t)j * nsub + s) * len + t + R[(int64_t)m * nsub + s]];
      if (acc > 0xFFFFFFFFull) {
#pragma omp atomic write
        err = ORACLE_EOVERFLOW;
      }
      Y[(int64_t)m * nout + t] = (uint32_t)acc;
    }
  }
  free(I);
  return err;
}

/*
 * Zero-DM filter (cited in Sec. 2.1; the paper gives no formula): subtract
 * from every channel the DM = 0 series, the channel mean at each sample,
 * m(t) = floor((sum_c X[c][t] + nchan/2) / nchan), and restore the 8-bit
 * mid-level: X'[c][t] = clip(X[c][t] - m(t) + 128, 0, 255).
 */
int sps_oracle_zero_dm(int32_t nchan, const uint8_t *X, int64_t pitch, int64_t nsamp,
                       uint8_t *Xo, int64_t pitch_out) {
  if (nchan <= 0 || nsamp < 0 || !X || !Xo || pitch < nsamp || pitch_out < nsamp)
    return ORACLE_EINVAL;
  for (int64_t t = 0; t < nsamp; ++t) {
    int64_t sum = 0;
    for (int32_t c = 0; c < nchan; ++c) sum += X[(int64_t)c * pitch + t];
    int64_t m = (sum + nchan / 2) / nchan;
    for (int32_t c = 0; c < nchan; ++c) {
      int64_t v = (int64_t)X[(int64_t)c * pitch + t] - m + 128;
      Xo[(int64_t)c * pitch_out + t] = (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
    }
  }
  return ORACLE_OK;
}

/*
 * Square-law downsampling, Sec. 2.2:
 *   out = min{ V sqrt(S) / sqrt(N V), V } = min{ sqrt(V S / N), V },
 * S the sum of the N samples of a bin, V = 255, rounded half up to an
 * integer.  Bins are the full ones, t in [0, floor(nsamp / N)).  The rounding
 * is settled exactly in integers: r is the value with
 * (2r - 1)^2 N <= 4 V S < (2r + 1)^2 N.
 */
int sps_oracle_downsample_sqrt(int32_t nchan, const uint8_t *X, int64_t pitch, int64_t nsamp,
                               int32_t factor, uint8_t *Xo, int64_t pitch_out) {
  if (nchan <= 0 || nsamp < 0 || factor <= 0 || !X || !Xo || pitch < nsamp)
    return ORACLE_EINVAL;
  const int64_t V = 255;
  int64_t nout = nsamp / factor;
  if (pitch_out < nout) return ORACLE_EINVAL;
  for (int32_t c = 0; c < nchan; ++c) {
    for (int64_t t = 0; t < nout; ++t) {
      int64_t S = 0;
      for (int32_t k = 0; k < factor; ++k) S += X[(int64_t)c * pitch + t * factor + k];
      int64_t r = (int64_t)floor(sqrt((double)V * (double)S / (double)factor) + 0.5);
      while ((2 * r + 1) * (2 * r + 1) * (int64_t)factor <= 4 * V * S) ++r;
      while (r > 0 && (2 * r - 1) * (2 * r - 1) * (int64_t)factor > 4 * V * S) --r;
      if (r > V) r = V;
      Xo[(int64_t)c * pitch_out + t] = (uint8_t)r;
    }
  }
  return ORACLE_OK;
}
